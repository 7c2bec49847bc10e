"""Generic lifting (steps from the host factorizer, taken at run time) on
the GPU against the oracle's convolve-and-downsample analysis with the same
taps, for the paper's pairs on both sides, the irrational CDF 9/7 member of
the Case II family, D4 (a factorization with shifts), Haar, a three-step
pair, and predictors of four taps and of six taps (every one of the
kernel's instances runs);
ragged and tiny lengths; the benchmark size on sampled pulses."""
import math

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_cs_0607001_amd as S
    S._lib.lib()
    return torch, S


def taps_of(lift, consts):
    N = 64
    lo, hi = {}, {}
    for i in range(-12, 13):
        u = np.zeros(N)
        u[i % N] = 1.0
        A, B = lift(u, consts)
        if abs(A[0]) > 1e-15:
            lo[i] = A[0]
        if abs(B[0]) > 1e-15:
            hi[i] = B[0]
    return lo, hi


def pairs():
    s = 1 / math.sqrt(2)
    out = {}
    for name in ("legall53", "cdf97", "d4"):
        xl, xh, yl, yh = O.TAPS[name]
        out[name + "_x"] = (xl, xh)
        out[name + "_y"] = (yl, yh)
    out["cdf97_irrational"] = taps_of(lambda u, c: O.lift_x("cdf97", u, c),
                                      O.cdf97_constants_from_t(1.230174104914001))
    out["haar"] = ({0: s, 1: s}, {0: -s, 1: s})
    # a six-tap predictor on the lazy split (one step longer than four taps:
    # the kernel's general, non-unrolled instance)
    p = [0.6, -0.25, 0.1, -0.05, 0.02, 0.01]
    out["wide_predict"] = ({0: 1.0}, {1: 1.0, 0: -p[0], 2: -p[1], -2: -p[2], 4: -p[3], -4: -p[4],
                                      6: -p[5]})
    # three alternating two-tap steps (predict, update, predict) and a scaling
    def three_steps(u, _):
        e, o = u[0::2].copy(), u[1::2].copy()
        o = o - 0.7 * (e + np.roll(e, -1))
        e = e + 0.3 * (o + np.roll(o, 1))
        o = o - 0.2 * (e + np.roll(e, -1))
        return 1.3 * e, o / 1.3
    out["three_steps"] = taps_of(three_steps, None)
    # a four-tap predictor reaching two lanes
    q = [0.55, -0.12, 0.07, -0.03]
    out["four_tap_predict"] = ({0: 1.0}, {1: 1.0, 0: -q[0], 2: -q[1], -2: -q[2], 4: -q[3]})
    return out


PAIRS = pairs()


def oracle_pyramid(lo, hi, J, u):
    c, parts = u, []
    for _ in range(J):
        parts.append(O.analyze(c, hi))
        c = O.analyze(c, lo)
    return parts, c


def rel_l2(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name", sorted(PAIRS))
@pytest.mark.parametrize("J,n", [(3, 1000), (5, 4096), (2, 8), (6, 300)])
def test_generic_lifting_matches_the_taps(dev, name, J, n):
    torch, S = dev
    lo, hi = PAIRS[name]
    rng = np.random.default_rng(n + J)
    rx = (rng.standard_normal((3, n)) + 1j * rng.standard_normal((3, n))).astype(np.complex64)
    N = O.transform_length(n, J)
    print(f"[case] generic {name} J={J} n={n}", flush=True)
    with S.Lifting(lo, hi) as f:
        pyr = S.lift_generic(f, J, torch.from_numpy(rx).cuda()).cpu().numpy().astype(np.complex128)
    for i in range(3):
        d, cJ = oracle_pyramid(lo, hi, J, O.zero_pad(rx[i].astype(np.complex128), N))
        for l in range(1, J + 1):
            off, L = N - (N >> (l - 1)), N >> l
            assert rel_l2(pyr[i, off:off + L], d[l - 1]) <= 1e-5, (i, l)
        assert rel_l2(pyr[i, N - (N >> J):], cJ) <= 1e-5, i


def test_generic_with_the_papers_dual_steps_equals_lift_many(dev):
    torch, S = dev
    rng = np.random.default_rng(12)
    rx = torch.from_numpy((rng.standard_normal((4, 2048)) + 1j * rng.standard_normal((4, 2048)))
                          .astype(np.complex64)).cuda()
    for name in ("legall53", "cdf97"):
        with S.Lifting(*O.TAPS[name][2:]) as f:
            a = S.lift_generic(f, 4, rx).cpu().numpy().astype(np.complex128)
        b = S.lift_many(name, 4, rx).cpu().numpy().astype(np.complex128)
        assert rel_l2(a, b) <= 1e-6, name


def test_generic_full_size_sampled(dev):
    torch, S = dev
    import workloads as W
    count, n, J = 4096, 8192, 5
    print("[case] generic irrational 9/7 on 4096 x 8192", flush=True)
    b = W.batched_uniform(seed=2, count=count, n=n, m=512, J=J)
    lo, hi = PAIRS["cdf97_irrational"]
    with S.Lifting(lo, hi) as f:
        pyr = S.lift_generic(f, J, torch.from_numpy(b.rx).cuda())
        torch.cuda.synchronize()
    for i in (0, 2047, 4095):
        got = pyr[i].cpu().numpy().astype(np.complex128)
        d, cJ = oracle_pyramid(lo, hi, J, b.rx[i].astype(np.complex128))
        want = np.concatenate(d + [cJ])
        assert rel_l2(got, want) <= 1e-5, i
