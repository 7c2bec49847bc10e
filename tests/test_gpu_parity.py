"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Float filters: relative L2 error per plane <= 1e-5 (FP32 lifting and FP32
MFMA accumulation against the FP64 definition).  Integer filter: bit-exact.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0607001_amd as S
    S._lib.lib()  # loud failure if the library is missing
    return torch, S


def crandn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def run_float(dev, filt, J, ref, rx):
    torch, S = dev
    print(f"[case] filter={filt} J={J} m={len(ref)} n={len(rx)}", flush=True)
    with S.plan_create(filt, J, ref) as plan:
        x = torch.from_numpy(np.asarray(rx, np.complex64)).cuda()
        out = S.correlate(plan, x)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def assert_planes_close(got, want, tol=TOL):
    assert got.shape == want.shape
    for j in range(want.shape[0]):
        e = rel_l2(got[j].astype(np.complex128), want[j])
        assert e <= tol, f"plane {j}: rel L2 {e:.3e}"


# ---------------------------------------------------------------------------
# Single pulses, every float filter, ragged lengths, several tiles
# ---------------------------------------------------------------------------

def test_single_chirp_legall53_j3(dev):
    w = W.single_chirp(seed=1)
    got = run_float(dev, w.filter, w.J, w.ref, w.rx)
    want = O.correlate_direct(w.filter, w.J, w.ref, w.rx)
    assert_planes_close(got, want)
    assert int(np.argmax(np.abs(got[0]))) == w.delay


@pytest.mark.parametrize("filt,J,m,n", [
    ("legall53", 3, 37, 200),     # N = 200 (ragged, 25 * 8)
    ("legall53", 5, 120, 1000),   # N = 1024
    ("cdf97", 5, 100, 640),
    ("cdf97", 4, 300, 1500),      # N = 1504
    ("cdf97", 2, 16, 40),
    ("d4", 4, 50, 300),           # N = 304
    ("d4", 6, 64, 1024),
    ("d4", 1, 5, 9),              # N = 10
])
def test_float_filters_random(dev, filt, J, m, n):
    rng = np.random.default_rng(hash((filt, J, m, n)) & 0xffff)
    ref, rx = crandn(rng, m), crandn(rng, n)
    got = run_float(dev, filt, J, ref, rx)
    want = O.correlate_direct(filt, J, ref, rx)
    assert_planes_close(got, want)


def test_reference_as_long_as_the_transform(dev):
    rng = np.random.default_rng(5)
    ref, rx = crandn(rng, 64), crandn(rng, 64)
    got = run_float(dev, "cdf97", 3, ref, rx)
    assert_planes_close(got, O.correlate_direct("cdf97", 3, ref, rx))


def test_dc_and_delta_special_cases(dev):
    rng = np.random.default_rng(6)
    x = crandn(rng, 21)
    got = run_float(dev, "cdf97", 4, x, np.ones(128))
    assert np.abs(got - np.conj(x.sum())).max() < 1e-5 * abs(x.sum())
    y = crandn(rng, 96)
    got = run_float(dev, "d4", 3, np.array([1.0 + 0j]), y)
    assert np.abs(got[0] - y).max() < 1e-5 * np.abs(y).max()


# ---------------------------------------------------------------------------
# Reference phase pyramid (plan) against the oracle's directly computed phases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", ["legall53", "cdf97", "d4", "legall53_int"])
def test_plan_phases_match_direct_computation(dev, filt):
    torch, S = dev
    rng = np.random.default_rng(7)
    J, m, N = 4, 23, 512
    if filt == "legall53_int":
        ref = rng.integers(-2047, 2048, size=(m, 2)).astype(np.int16)
    else:
        ref = crandn(rng, m).astype(np.complex64)
    with S.plan_create(filt, J, ref) as plan:
        for lvl in range(1, J + 1):
            L = N >> lvl
            for r in range(1 << lvl):
                want = O.reference_phase(filt, ref, N, lvl, r)
                for b in (0, 1):
                    lo, c = S.plan_phase(plan, lvl, b, r)
                    if filt == "legall53_int":
                        c = c[:, 0] + 1j * c[:, 1]
                    circ = np.zeros(L, complex)
                    np.add.at(circ, (lo + np.arange(len(c))) % L, c)
                    tol = 0 if filt == "legall53_int" else 1e-5 * np.abs(want[b]).max()
                    assert np.abs(circ - want[b]).max() <= tol, (lvl, r, b)


# ---------------------------------------------------------------------------
# Lifting-only kernel against the oracle's lifting
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt,J,n", [("legall53", 3, 1000), ("cdf97", 5, 8192), ("d4", 4, 300)])
def test_lift_many_float(dev, filt, J, n):
    torch, S = dev
    rng = np.random.default_rng(8)
    count = 3
    rx = np.stack([crandn(rng, n) for _ in range(count)])
    pyr = S.lift_many(filt, J, torch.from_numpy(rx.astype(np.complex64)).cuda())
    torch.cuda.synchronize()
    pyr = pyr.cpu().numpy()
    N = O.transform_length(n, J)
    _, _, ylo, yhi = O.TAPS[filt]
    for i in range(count):
        c = O.zero_pad(rx[i], N)
        parts = []
        for _ in range(J):
            c, d = O.analyze(c, ylo), O.analyze(c, yhi)
            parts.append(d)
        want = np.concatenate(parts + [c])
        assert rel_l2(pyr[i].astype(complex), want) < 1e-6


def test_lift_many_integer(dev):
    torch, S = dev
    J, n, count = 6, 4096, 2
    rx = np.stack([W.int_pulse(3, i, n=n) for i in range(count)])
    pyr = S.lift_many("legall53_int", J, torch.from_numpy(rx).cuda())
    torch.cuda.synchronize()
    pyr = pyr.cpu().numpy().astype(np.int64)
    for i in range(count):
        re, im = rx[i, :, 0].astype(np.int64), rx[i, :, 1].astype(np.int64)
        parts = []
        for _ in range(J):
            (re, dre), (im, dim) = O.i2i_lift_y(re), O.i2i_lift_y(im)
            parts.append(np.stack([dre, dim], -1))
        want = np.concatenate(parts + [np.stack([re, im], -1)])
        assert np.array_equal(pyr[i], want)


@pytest.mark.parametrize("filt,J,n,count", [("cdf97", 5, 8192, 2000), ("d4", 5, 8192, 1100),
                                              ("cdf97", 4, 16384, 300),
                                              ("legall53_int", 6, 4096, 4000)])
def test_lift_many_more_pulses_than_workgroups(dev, filt, J, n, count):
    """Each workgroup lifts several pulses in turn (with the next pulse's
    level-1 input prefetched when it fits, directly otherwise); sampled
    pulses, including the first and the last, against the oracle."""
    torch, S = dev
    rng = np.random.default_rng(count)
    print(f"[case] lift {filt} J={J} n={n} count={count}", flush=True)
    if filt == "legall53_int":
        rx = rng.integers(-2048, 2048, size=(count, n, 2)).astype(np.int16)
    else:
        rx = (rng.standard_normal((count, n)) + 1j * rng.standard_normal((count, n))).astype(
            np.complex64)
    pyr = S.lift_many(filt, J, torch.from_numpy(rx).cuda())
    torch.cuda.synchronize()
    N = O.transform_length(n, J)
    for i in sorted({0, 1, count // 3, count // 2, count - 2, count - 1}):
        g = pyr[i].cpu().numpy()
        parts = []
        if filt == "legall53_int":
            re, im = rx[i, :, 0].astype(np.int64), rx[i, :, 1].astype(np.int64)
            for _ in range(J):
                (re, dre), (im, dim) = O.i2i_lift_y(re), O.i2i_lift_y(im)
                parts.append(np.stack([dre, dim], -1))
            want = np.concatenate(parts + [np.stack([re, im], -1)])
            assert np.array_equal(g.astype(np.int64), want), i
        else:
            _, _, ylo, yhi = O.TAPS[filt]
            c = O.zero_pad(rx[i].astype(np.complex128), N)
            for _ in range(J):
                c, d = O.analyze(c, ylo), O.analyze(c, yhi)
                parts.append(d)
            want = np.concatenate(parts + [c])
            assert rel_l2(g.astype(complex), want) < 1e-6, i


# ---------------------------------------------------------------------------
# Integer path: bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("J,m,n", [(3, 40, 200), (6, 64, 1024), (4, 31, 230)])
def test_integer_path_bit_exact(dev, J, m, n):
    torch, S = dev
    rng = np.random.default_rng(J * 1000 + m)
    ref = rng.integers(-2047, 2048, size=(m, 2)).astype(np.int16)
    rx = rng.integers(-2048, 2048, size=(n, 2)).astype(np.int16)
    print(f"[case] int J={J} m={m} n={n}", flush=True)
    with S.plan_create("legall53_int", J, ref) as plan:
        out = S.correlate(plan, torch.from_numpy(rx).cuda())
        torch.cuda.synchronize()
    want = O.correlate_int(J, ref, rx)
    assert np.array_equal(out.cpu().numpy(), want)


def test_integer_full_scale_bit_exact(dev):
    """Pulse and reference at the int16 extremes (random signs of 32767 and
    -32768): the largest products the integer path can meet at J = 8."""
    torch, S = dev
    rng = np.random.default_rng(77)
    ref = np.where(rng.random((200, 2)) < 0.5, 32767, -32768).astype(np.int16)
    rx = np.where(rng.random((4096, 2)) < 0.5, 32767, -32768).astype(np.int16)
    print("[case] int full scale J=8 m=200 n=4096", flush=True)
    with S.plan_create("legall53_int", 8, ref) as plan:
        out = S.correlate(plan, torch.from_numpy(rx).cuda())
        torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), O.correlate_int(8, ref, rx))


def test_integer_plans_take_the_int8_path_where_it_applies(dev):
    """Plans up to J = 7 run on int8 matrix cores with as many weight digits
    as their phases need; deeper plans keep the FP64 form."""
    torch, S = dev
    rng = np.random.default_rng(5)
    quiet = rng.integers(-100, 101, (40, 2)).astype(np.int16)
    adc = rng.integers(-2047, 2048, (512, 2)).astype(np.int16)
    loud = np.where(rng.random((60, 2)) < 0.5, 32767, -32768).astype(np.int16)
    for ref, J, digits in ((quiet, 2, 2), (adc, 6, 2), (loud, 3, 3), (loud, 7, 3), (adc, 8, 0)):
        with S.plan_create("legall53_int", J, ref) as plan:
            info = plan.info()
            assert info["i8_weight_digits"] == digits, (J, info)
            assert (info["i8_panel_bytes"] > 0) == (digits > 0)


@pytest.mark.parametrize("value", [32767, -32768])
def test_integer_int8_path_at_the_digit_limits(dev, value):
    """J = 7, the deepest plan on int8 matrix cores: a full-scale DC pulse
    drives the level-7 coefficients to the top of the three data digits,
    a full-scale reference needs three weight digits; plus random
    full-scale signs, through one launch of several pulses."""
    torch, S = dev
    rng = np.random.default_rng(abs(value))
    ref = np.where(rng.random((90, 2)) < 0.5, 32767, -32768).astype(np.int16)
    n = 2048
    rx = np.stack([np.full((n, 2), value), np.where(rng.random((n, 2)) < 0.5, 32767, -32768),
                   rng.integers(-32768, 32768, (n, 2))]).astype(np.int16)
    print(f"[case] int8 limits J=7 m=90 n={n} value={value}", flush=True)
    with S.plan_create("legall53_int", 7, ref) as plan:
        assert plan.info()["i8_weight_digits"] == 3
        out = S.correlate_many(plan, torch.from_numpy(rx).cuda())
        torch.cuda.synchronize()
    got = out.cpu().numpy()
    for i in range(rx.shape[0]):
        assert np.array_equal(got[i], O.correlate_int(7, ref, rx[i])), i


@pytest.mark.parametrize("n,J,count", [(65536, 6, 2), (20000, 7, 1)])
def test_integer_pulses_beyond_one_workgroup(dev, n, J, count):
    """Integer pulses too long for one workgroup's LDS: lifted into an HBM
    pyramid and correlated in blocks of lag rows on int8 matrix cores;
    bit-exact on sampled lags (block edges, both ends) of every plane."""
    torch, S = dev
    rng = np.random.default_rng(n + J)
    ref = rng.integers(-2047, 2048, (512, 2)).astype(np.int16)
    rx = rng.integers(-32768, 32768, (count, n, 2)).astype(np.int16)
    print(f"[case] int long pulse n={n} J={J} count={count}", flush=True)
    with S.plan_create("legall53_int", J, ref) as plan:
        out = S.correlate_many(plan, torch.from_numpy(rx).cuda())
        torch.cuda.synchronize()
    N = O.transform_length(n, J)
    got = out.cpu().numpy()
    lags = np.unique(np.concatenate([[0, 1, 2, N // 2, N - 2, N - 1],
                                     rng.integers(0, N, 24),
                                     # lags around the row blocks of level 1 (992 rows of 16 lags)
                                     [992 * 16 - 1, 992 * 16, 992 * 16 + 1]]))
    lags = lags[lags < N]
    for i in range(count):
        for j in range(J):
            want = O.correlate_int_at(J, ref, rx[i], j, lags)
            assert np.array_equal(got[i, j, lags], want), (i, j)


def test_integer_support_wrap_is_rejected(dev):
    torch, S = dev
    ref = np.ones((60, 2), np.int16)
    with S.plan_create("legall53_int", 3, ref) as plan:
        rx = torch.zeros((64, 2), dtype=torch.int16, device="cuda")
        with pytest.raises(S.SidwtError) as e:
            S.correlate(plan, rx)
        assert e.value.code == -2


# ---------------------------------------------------------------------------
# Error paths through the ABI with a real plan
# ---------------------------------------------------------------------------

def test_size_errors(dev):
    torch, S = dev
    rng = np.random.default_rng(9)
    with S.plan_create("cdf97", 3, crandn(rng, 40)) as plan:
        with pytest.raises(S.SidwtError) as e:      # m > N
            S.correlate(plan, torch.zeros(32, dtype=torch.complex64, device="cuda"))
        assert e.value.code == -2
        with pytest.raises(S.SidwtError) as e:      # N / 2^J < 2
            S.correlate(plan, torch.zeros(8, dtype=torch.complex64, device="cuda"))
        assert e.value.code == -1


# ---------------------------------------------------------------------------
# Uniform batch in one launch: every pulse equals its own single launch and
# the oracle (small batch, full planes)
# ---------------------------------------------------------------------------

def test_correlate_many_matches_oracle(dev):
    torch, S = dev
    b = W.batched_uniform(seed=21, count=5, n=1024, m=128, J=4)
    with S.plan_create(b.filter, b.J, b.ref) as plan:
        out = S.correlate_many(plan, torch.from_numpy(b.rx).cuda())
        torch.cuda.synchronize()
        out = out.cpu().numpy()
    for i in range(5):
        assert_planes_close(out[i], O.correlate_direct(b.filter, b.J, b.ref, b.rx[i]))


# ---------------------------------------------------------------------------
# Empty batches: sizes are checked, nothing is launched
# ---------------------------------------------------------------------------

def test_empty_batches(dev):
    torch, S = dev
    rng = np.random.default_rng(12)
    with S.plan_create("cdf97", 3, crandn(rng, 20)) as plan:
        out = S.correlate_many(plan, torch.empty((0, 100), dtype=torch.complex64, device="cuda"))
        assert tuple(out.shape) == (0, 3, 104)
    pyr = S.lift_many("d4", 4, torch.empty((0, 64), dtype=torch.complex64, device="cuda"))
    assert tuple(pyr.shape) == (0, 64)
    with S.plan_create("legall53_int", 2, np.ones((8, 2), np.int16)) as plan:
        out = S.correlate_many(plan, torch.empty((0, 64, 2), dtype=torch.int16, device="cuda"))
        assert tuple(out.shape) == (0, 2, 64, 2)
    with S.Bank("cdf97", 3, [crandn(rng, 16), crandn(rng, 32)]) as bank:
        assert bank.correlate([], []) == []
    torch.cuda.synchronize()


@pytest.mark.parametrize("n", [2048, 4096])
def test_uniform_batch_of_short_pulses(dev, n):
    """More pulses than CUs of a length whose levels leave most waves idle:
    the balanced whole-pulse instance with its partial-sum slots after the
    layout (two workgroups per CU)."""
    torch, S = dev
    count, J = 300, 5
    b = W.batched_uniform(seed=31, count=count, n=n, m=256, J=J)
    print(f"[case] uniform {count} x {n}, 9/7 J=5", flush=True)
    with S.plan_create(b.filter, J, b.ref) as plan:
        out = S.correlate_many(plan, torch.from_numpy(b.rx).cuda())
        torch.cuda.synchronize()
        rng = np.random.default_rng(2)
        for i in (0, 151, count - 1):
            lags = np.unique(np.concatenate([[0, 1, n - 1], rng.integers(0, n, 40)]))
            got = out[i][:, lags].cpu().numpy().astype(np.complex128)
            for j in range(J):
                want = O.correlate_at(b.filter, J, b.ref, b.rx[i].astype(np.complex128), j, lags)
                e = np.linalg.norm(got[j] - want) / np.linalg.norm(want)
                assert e <= 1e-5, (n, i, j, e)


@pytest.mark.parametrize("filt,planes", [("cdf97", [4]), ("cdf97", [3, 4]), ("d4", [0, 2]),
                                         ("legall53_int", [5])])
def test_plane_mask_computes_only_the_chosen_planes(dev, filt, planes):
    """Scale mask (coarse scales on their own): the chosen planes equal the
    full correlation's, the others keep what out held."""
    torch, S = dev
    rng = np.random.default_rng(len(planes) * 7 + len(filt))
    count = 3
    print(f"[case] plane mask {filt} {planes}", flush=True)
    if filt == "legall53_int":
        J, n, m = 6, 1024, 40
        ref = rng.integers(-2047, 2048, size=(m, 2)).astype(np.int16)
        rx = torch.from_numpy(rng.integers(-2048, 2048, size=(count, n, 2)).astype(np.int16))
    else:
        J, n, m = 5, 1000, 60
        ref = crandn(rng, m)
        rx = torch.from_numpy(np.stack([crandn(rng, n) for _ in range(count)]).astype(np.complex64))
    with S.plan_create(filt, J, ref) as plan:
        rx = rx.cuda()
        full = S.correlate_many(plan, rx)
        part = torch.full_like(full, 7)
        S.correlate_many(plan, rx, out=part, planes=planes)
        torch.cuda.synchronize()
        for j in range(J):
            if j in planes:
                assert torch.equal(part[:, j], full[:, j]), j
            else:
                assert bool((part[:, j] == 7).all()), j


@pytest.mark.parametrize("filt", ["cdf97", "legall53_int"])
def test_few_pulses_one_workgroup_per_plane_match_the_batch(dev, filt):
    """A launch of a few pulses runs one workgroup per (pulse, plane); the
    same pulses inside a batch too large for that run one workgroup per
    pulse.  Both give the same planes bit for bit, and the oracle's."""
    torch, S = dev
    rng = np.random.default_rng(91)
    J, n, m = 5, 1500, 80
    count = 64   # 64 x 5 planes: more than one workgroup per plane allows
    if filt == "legall53_int":
        ref = rng.integers(-2047, 2048, size=(m, 2)).astype(np.int16)
        rx = torch.from_numpy(rng.integers(-2048, 2048, size=(count, n, 2)).astype(np.int16))
    else:
        ref = crandn(rng, m)
        rx = torch.from_numpy(np.stack([crandn(rng, n) for _ in range(count)]).astype(np.complex64))
    print(f"[case] per-plane workgroups {filt}", flush=True)
    with S.plan_create(filt, J, ref) as plan:
        rx = rx.cuda()
        big = S.correlate_many(plan, rx)
        few = S.correlate_many(plan, rx[:3].contiguous())
        one = S.correlate(plan, rx[5].contiguous())
        torch.cuda.synchronize()
        assert torch.equal(few, big[:3])
        assert torch.equal(one, big[5])
        got = one.cpu().numpy()
        if filt == "legall53_int":
            assert np.array_equal(got, O.correlate_int(J, ref, rx[5].cpu().numpy()))
        else:
            want = O.correlate_direct(filt, J, ref, rx[5].cpu().numpy())
            for j in range(J):
                assert np.linalg.norm(got[j] - want[j]) <= 1e-5 * np.linalg.norm(want[j]), j
