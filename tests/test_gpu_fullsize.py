"""Parity at the full workload sizes, in the launch configuration the
benchmark times (one launch over the whole batch), checked on sampled
pulses and lags that the oracle computes one by one."""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0607001_amd as S
    S._lib.lib()
    return torch, S


def test_single_chirp_many_seeds(dev):
    torch, S = dev
    for seed in range(1, 21):
        w = W.single_chirp(seed=seed)
        with S.plan_create(w.filter, w.J, w.ref) as plan:
            out = S.correlate(plan, torch.from_numpy(w.rx.astype(np.complex64)).cuda())
            torch.cuda.synchronize()
            got = out.cpu().numpy().astype(np.complex128)
        want = O.correlate_direct(w.filter, w.J, w.ref, w.rx)
        for j in range(w.J):
            e = np.linalg.norm(got[j] - want[j]) / np.linalg.norm(want[j])
            assert e <= 1e-5, (seed, j, e)
        assert int(np.argmax(np.abs(got[0]))) == w.delay


def test_batched_uniform_full_size_sampled(dev):
    torch, S = dev
    count, n, J = 4096, 8192, 5
    print("[case] batched uniform 4096 x 8192 cdf97 J=5", flush=True)
    b = W.batched_uniform(seed=2, count=count, n=n, m=512, J=J)
    with S.plan_create(b.filter, J, b.ref) as plan:
        out = S.correlate_many(plan, torch.from_numpy(b.rx).cuda())
        torch.cuda.synchronize()
        rng = np.random.default_rng(0)
        for i in (0, 1, 2047, 4095):
            lags = np.concatenate([[0, 1, 2, n - 1], rng.integers(0, n, 60)])
            got = out[i][:, lags].cpu().numpy().astype(np.complex128)
            for j in range(J):
                want = O.correlate_at(b.filter, J, b.ref, b.rx[i].astype(np.complex128), j, lags)
                e = np.linalg.norm(got[j] - want) / np.linalg.norm(want)
                assert e <= 1e-5, (i, j, e)
        # the whole batch is finite and every pulse's plane 0 peaks at an echo
        assert torch.isfinite(torch.view_as_real(out)).all().item()


def test_integer_full_size_sampled(dev):
    torch, S = dev
    count, n, J = 16384, 4096, 6
    print("[case] integer 16384 x 4096 int16 J=6", flush=True)
    ib = W.integer_batch(seed=3, count=count, n=n, m=512, J=J)
    with S.plan_create("legall53_int", J, ib.ref_iq) as plan:
        out = S.correlate_many(plan, torch.from_numpy(ib.rx_iq).cuda())
        torch.cuda.synchronize()
        rng = np.random.default_rng(1)
        for i in (0, 777, 16383):
            lags = np.concatenate([[0, 1, n - 1], rng.integers(0, n, 40)])
            got = out[i][:, lags].cpu().numpy()
            for j in range(J):
                want = O.correlate_int_at(J, ib.ref_iq, ib.rx_iq[i], j, lags)
                assert np.array_equal(got[j], want), (i, j)


def _sampled_lags(rng, N, k=8):
    return np.unique(np.concatenate([[0, 1, N - 1], rng.integers(0, N, k)]))


def test_uneven_full_size_sampled(dev):
    """10^4 pulses of log-uniform length in [512, 65536], 16 references, D4
    and 9/7, autotuned split and one graph-replayed run, as in the uneven
    benchmark; sampled pulses (first, last, middle, longest, shortest)."""
    torch, S = dev
    refs, reqs = W.uneven_batch(seed=4, count=10000)
    print("[case] uneven 10000 pulses, autotuned", flush=True)
    plans, cache = [], {}
    for r in reqs:
        key = (r.ref_index, r.filter, r.J)
        if key not in cache:
            cache[key] = S.plan_create(r.filter, r.J, refs[r.ref_index])
        plans.append(cache[key])
    ns = [r.n for r in reqs]
    rx = [torch.from_numpy(r.rx.astype(np.complex64)).cuda() for r in reqs]
    out = S.batch_outputs(plans, ns, rx[0].device)
    with S.Batch(plans, ns) as b:
        info = b.tune(rx, out)
        print(f"[case] tuned {info}", flush=True)
        b.run(rx, out)
        torch.cuda.synchronize()
    rng = np.random.default_rng(11)
    picks = {0, len(reqs) // 2, len(reqs) - 1, int(np.argmax(ns)), int(np.argmin(ns))}
    for i in sorted(picks):
        r = reqs[i]
        N = O.transform_length(r.n, r.J)
        lags = _sampled_lags(rng, N)
        got = out[i][:, lags].cpu().numpy().astype(np.complex128)
        for j in range(r.J):
            want = O.correlate_at(r.filter, r.J, refs[r.ref_index],
                                  r.rx.astype(np.complex128), j, lags)
            e = np.linalg.norm(got[j] - want) / np.linalg.norm(want)
            assert e <= 1e-5, (i, r.n, j, e)
    del out, rx
    for p in cache.values():
        p.free()
    torch.cuda.empty_cache()


def test_bank_full_size_sampled(dev):
    """256 requests of the serving mix against the 64-reference 9/7 bank
    (FP16 hi+lo), one call as in the bank benchmark; sampled requests and
    references (first, middle and last eligible)."""
    torch, S = dev
    refs = W.reference_set(5, count=64)
    rng = np.random.default_rng([5, 1])     # the benchmark's request stream
    reqs = []
    for _ in range(256):
        n = W.uneven_length(rng)
        elig = [k for k, r in enumerate(refs) if len(r) <= n // 2] or [0]
        k = elig[int(rng.integers(0, len(elig)))]
        reqs.append((n, W.levels_for(n), W.echoes(n, refs[k], rng).astype(np.complex64)))
    print("[case] bank 256 requests x 64 references", flush=True)
    with S.Bank("cdf97", 12, refs, "fp16") as bank:
        rx = [torch.from_numpy(y).cuda() for _, _, y in reqs]
        outs = bank.correlate(rx, [J for _, J, _ in reqs])
        torch.cuda.synchronize()
        srng = np.random.default_rng(12)
        ns = [n for n, _, _ in reqs]
        Es = [bank.eligible(n) for n in ns]
        # also the shortest request and one whose eligible references end
        # mid-bank (their tiles are a prefix of each level's tiles)
        picks = {0, 255, 128, int(np.argmax(ns)), int(np.argmin(ns)),
                 int(np.argmin([abs(e - 33) for e in Es]))}
        for i in sorted(picks):
            n, J, y = reqs[i]
            E = bank.eligible(n)
            N = O.transform_length(n, J)
            lags = _sampled_lags(srng, N, k=6)
            for e in sorted({0, E // 2, E - 1}):
                got = outs[i][e][:, lags].cpu().numpy().astype(np.complex128)
                for j in range(J):
                    want = O.correlate_at("cdf97", J, refs[e], y.astype(np.complex128), j, lags)
                    err = np.linalg.norm(got[j] - want) / np.linalg.norm(want)
                    assert err <= 1e-5, (i, n, e, j, err)
        del outs, rx
    torch.cuda.empty_cache()
