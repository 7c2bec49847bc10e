"""Reference bank on 16-bit MFMA with hi+lo correction: every eligible
reference's planes against the oracle (and the FP32 plain path)."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

# relative L2 error per plane against the FP64 oracle
TOL = {"fp32": 1e-5, "fp16": 1e-5, "bf16": 1e-4}


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0607001_amd as S
    S._lib.lib()
    return torch, S


def bank_refs(seed=7, count=6):
    return W.reference_set(seed, count=count, m_lo=24, m_hi=400)


@pytest.mark.parametrize("precision", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("filt", ["cdf97", "d4"])
def test_bank_matches_oracle(dev, filt, precision):
    torch, S = dev
    refs = bank_refs()
    rng = np.random.default_rng(3)
    Jmax = 10
    print(f"[case] bank {filt} {precision} m={[len(r) for r in refs]}", flush=True)
    with S.Bank(filt, Jmax, refs, precision) as bank:
        ns = [200, 700, 3000, 16000]
        Js = [W.levels_for(n) for n in ns]
        ys = [W.echoes(n, refs[-1] if len(refs[-1]) <= n else refs[0], rng) for n in ns]
        rx = [torch.from_numpy(y.astype(np.complex64)).cuda() for y in ys]
        out = bank.correlate(rx, Js)
        torch.cuda.synchronize()
        worst = 0.0
        for y, J, o in zip(ys, Js, out):
            E = bank.eligible(len(y))
            assert o.shape[0] == E == sum(len(r) <= len(y) for r in refs)
            g = o.cpu().numpy().astype(np.complex128)
            N = O.transform_length(len(y), J)
            for e in range(E):
                if N <= 1024:
                    want = O.correlate_direct(filt, J, refs[e], y)
                    lags = np.arange(N)
                else:
                    lags = np.concatenate([[0, N - 1], rng.integers(0, N, 30)])
                    want = np.stack([O.correlate_at(filt, J, refs[e], y, j, lags)
                                     for j in range(J)])
                for j in range(J):
                    err = np.linalg.norm(g[e, j, lags] - want[j]) / np.linalg.norm(want[j])
                    worst = max(worst, err)
                    assert err <= TOL[precision], (len(y), e, j, err)
        print(f"[case] worst rel L2 {worst:.2e}", flush=True)


@pytest.mark.parametrize("precision", ["fp16", "bf16"])
def test_bank_with_only_shallow_levels(dev, precision):
    """Jmax = 3: every item runs on the general kernel and the deep levels'
    launch is empty; whole planes against the oracle."""
    torch, S = dev
    refs = W.reference_set(11, count=3, m_lo=20, m_hi=60)
    rng = np.random.default_rng(5)
    print(f"[case] shallow bank {precision}", flush=True)
    with S.Bank("cdf97", 3, refs, precision) as bank:
        ns, Js = [130, 400, 64], [3, 3, 2]
        ys = [W.echoes(n, refs[0], rng) for n in ns]
        rx = [torch.from_numpy(y.astype(np.complex64)).cuda() for y in ys]
        out = bank.correlate(rx, Js)
        torch.cuda.synchronize()
        for y, J, o in zip(ys, Js, out):
            E = bank.eligible(len(y))
            assert E > 0 and o.shape[0] == E
            g = o.cpu().numpy().astype(np.complex128)
            for e in range(E):
                want = O.correlate_direct("cdf97", J, refs[e], y)
                for j in range(J):
                    err = np.linalg.norm(g[e, j] - want[j]) / np.linalg.norm(want[j])
                    assert err <= TOL[precision], (len(y), e, j, err)


def test_split_launch_equals_single_requests_bit_for_bit(dev):
    """A call large enough to be split (levels 1-3 on the general kernel,
    deeper levels on the deep instance) gives the same bits as each request
    alone (one launch of the general kernel): both accumulate every tile in
    the same order.  Two requests of the large call are also checked against
    the oracle on sampled lags."""
    torch, S = dev
    refs = W.reference_set(13, count=16, m_lo=40, m_hi=900)
    rng = np.random.default_rng(17)
    n, J, count = 16384, 10, 64
    ys = [W.echoes(n, refs[k % 16], rng) for k in range(count)]
    rx = [torch.from_numpy(y.astype(np.complex64)).cuda() for y in ys]
    print(f"[case] split bank call: {count} x {n}, J={J}", flush=True)
    with S.Bank("cdf97", J, refs, "fp16") as bank:
        big = bank.correlate(rx, [J] * count)
        torch.cuda.synchronize()
        for i in (0, 17, 63):
            one = bank.correlate([rx[i]], [J])[0]
            torch.cuda.synchronize()
            assert torch.equal(one, big[i]), i
        N = O.transform_length(n, J)
        for i in (5, 40):
            g = big[i].cpu().numpy().astype(np.complex128)
            for e in (0, 7, 15):
                lags = np.concatenate([[0, N - 1], rng.integers(0, N, 20)])
                for j in (0, 3, 6, 9):
                    want = O.correlate_at("cdf97", J, refs[e], ys[i], j, lags)
                    err = np.linalg.norm(g[e, j, lags] - want) / np.linalg.norm(want)
                    assert err <= TOL["fp16"], (i, e, j, err)


def test_bank_with_the_longest_reference_a_plan_accepts(dev):
    """Plans take references of up to 8192 samples (longer ones are refused
    with SIDWT_E_SIZE before anything is launched); at 8192 the bank's
    level-1 window is about 4100 lags, its largest LDS footprint (one
    workgroup per CU), checked against the oracle on sampled lags."""
    torch, S = dev
    rng = np.random.default_rng(23)
    too_long = W.reference_set(29, count=1, m_lo=8193, m_hi=8194)[0]
    assert len(too_long) == 8193
    with pytest.raises(S.SidwtError) as e:
        S.Bank("cdf97", 4, [too_long], "fp16")
    assert e.value.code == -2
    ref = W.reference_set(31, count=1, m_lo=8192, m_hi=8193)[0]
    assert len(ref) == 8192
    n, J = 16384, 4
    y = W.echoes(n, ref, rng)
    print(f"[case] bank with a {len(ref)}-sample reference", flush=True)
    with S.Bank("cdf97", J, [ref], "fp16") as bank:
        out = bank.correlate([torch.from_numpy(y.astype(np.complex64)).cuda()], [J])[0]
        torch.cuda.synchronize()
        g = out.cpu().numpy().astype(np.complex128)
    N = O.transform_length(n, J)
    lags = np.concatenate([[0, N - 1], rng.integers(0, N, 10)])
    for j in range(J):
        want = O.correlate_at("cdf97", J, ref, y, j, lags)
        err = np.linalg.norm(g[0, j, lags] - want) / np.linalg.norm(want)
        assert err <= TOL["fp16"], (j, err)


def test_bank_equals_fp32_path_within_tolerance(dev):
    torch, S = dev
    refs = bank_refs(seed=9, count=4)
    rng = np.random.default_rng(4)
    with S.Bank("cdf97", 8, refs, "fp16") as bank:
        n = 2048
        J = 7
        y = W.echoes(n, refs[1], rng)
        x = torch.from_numpy(y.astype(np.complex64)).cuda()
        out = bank.correlate([x], [J])[0]
        torch.cuda.synchronize()
        for e in range(bank.eligible(n)):
            p = bank.plan(e)
            # the bank plan has Jmax levels; the FP32 path with J levels uses
            # the same phases of levels 1..J
            ref32 = S.correlate(S.plan_create("cdf97", J, refs[e]), x)
            torch.cuda.synchronize()
            a = out[e].cpu().numpy()
            b = ref32.cpu().numpy()
            for j in range(J):
                err = np.linalg.norm(a[j] - b[j]) / np.linalg.norm(b[j])
                assert err <= 1e-5, (e, j, err)
            p.free()


def test_bank_argument_checks(dev):
    torch, S = dev
    refs = bank_refs(count=3)
    with pytest.raises(S.SidwtError):
        S.Bank("cdf97", 6, refs[::-1])          # not ascending
    with pytest.raises(S.SidwtError):
        S.Bank("legall53_int", 6, refs)         # integer filter
    with S.Bank("d4", 6, refs) as bank:
        assert bank.eligible(1) == 0
        assert bank.eligible(10 ** 6) == 3
        with pytest.raises(S.SidwtError):
            bank.correlate([torch.zeros(64, dtype=torch.complex64, device="cuda")], [7])  # J > Jmax


def test_workspace_kernel_timing(dev):
    torch, S = dev
    refs = bank_refs(seed=11, count=3)
    rng = np.random.default_rng(6)
    with S.Bank("cdf97", 6, refs, "bf16") as bank:
        ws = bank.workspace()
        with pytest.raises(S.SidwtError):
            ws.times()                           # nothing timed yet
        ws.timing(True)
        x = torch.from_numpy(W.echoes(1500, refs[0], rng).astype(np.complex64)).cuda()
        a = bank.correlate([x], [6], workspace=ws)[0]
        lift_ms, gemm_ms = ws.times()
        assert lift_ms > 0 and gemm_ms > 0
        ws.timing(False)
        b = bank.correlate([x], [6], workspace=ws)[0]
        torch.cuda.synchronize()
        assert torch.equal(a, b)                 # timing changes nothing in the results
        ws.free()


def test_fp32_bank_equals_split_bank(dev):
    """The FP32 bank (one-shot batch of every request-reference pair) and the
    FP16 hi+lo bank agree within the FP16 split's tolerance on one request
    mix, including a request with no eligible reference."""
    torch, S = dev
    refs = bank_refs(seed=10, count=5)
    rng = np.random.default_rng(8)
    ns = [20, 900, 5000]          # 20 < every reference: no eligible one
    Js = [1, W.levels_for(900), W.levels_for(5000)]
    ys = [W.echoes(n, refs[0], rng) if n >= len(refs[0]) else rng.standard_normal(n) + 0j
          for n in ns]
    rx = [torch.from_numpy(y.astype(np.complex64)).cuda() for y in ys]
    with S.Bank("cdf97", 10, refs, "fp32") as b32, S.Bank("cdf97", 10, refs, "fp16") as b16:
        o32 = b32.correlate(rx, Js)
        o16 = b16.correlate(rx, Js)
        torch.cuda.synchronize()
        assert o32[0].shape[0] == 0 and o16[0].shape[0] == 0
        for n, a, c in zip(ns, o32, o16):
            assert a.shape == c.shape
            if a.numel() == 0:
                continue
            for e in range(a.shape[0]):
                for j in range(a.shape[1]):
                    x, y = a[e, j].cpu().numpy(), c[e, j].cpu().numpy()
                    err = np.linalg.norm(x - y) / np.linalg.norm(x)
                    assert err <= 1e-5, (n, e, j, err)
