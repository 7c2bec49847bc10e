"""The library's lifting factorizer (eq. (16), host code) against what the
paper and mathematics fix: from the printed taps it recovers the paper's
lifting steps (Sec. III-C Case I and Table I), the steps reproduce the
taps for every pair tried (including the 9/7 family of Sec. III-C Case II
and the irrational CDF 9/7 at t = 1.2301741..., whose multipliers are the
published -1.586134342, -0.052980118, 0.882911075, 0.443506852), and pairs
without perfect reconstruction are refused."""
import math
import os

import numpy as np
import pytest

import oracle as O

LIB = os.path.join(os.path.dirname(__file__), "..", "paper_cs_0607001_amd", "libsidwt.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsidwt.so not built")


@pytest.fixture(scope="module")
def S():
    import paper_cs_0607001_amd as S
    return S


def apply_steps(f, u):
    """The step semantics stated in the C header, on one real sequence."""
    e, o = u[0::2].astype(float), u[1::2].astype(float)
    for kind, first, coef in f.steps:
        src = e if kind == 0 else o
        acc = sum(c * np.roll(src, -(first + t)) for t, c in enumerate(coef))
        if kind == 0:
            o = o + acc
        else:
            e = e + acc
    ke, se, ko, so = f.scaling
    return ke * np.roll(e, -se), ko * np.roll(o, -so)


def taps_of(lift, consts):
    """Impulse responses of a lifting (lowpass, highpass tap dicts)."""
    N = 64
    lo, hi = {}, {}
    for i in range(-12, 13):
        u = np.zeros(N)
        u[i % N] = 1.0
        A, B = lift(u, consts)
        # out[k] = sum_i c_i u[2k + i]: the impulse at position p = i mod N
        # shows up in output k = 0 with offset i (k = 0 rows only)
        if abs(A[0]) > 1e-15:
            lo[i] = A[0]
        if abs(B[0]) > 1e-15:
            hi[i] = B[0]
    return lo, hi


def test_recovers_the_papers_lifting_steps(S):
    xl, xh, yl, yh = O.TAPS["legall53"]
    f = S.Lifting(xl, xh)
    assert [(k, fi) for k, fi, _ in f.steps] == [(0, 0), (1, -1)]
    assert np.allclose(f.steps[0][2], [-0.5, -0.5]) and np.allclose(f.steps[1][2], [0.25, 0.25])
    assert np.allclose(f.scaling, (1.0, 0, 0.5, 0))
    c = O.CDF97_TABLE_I
    f = S.Lifting(*O.TAPS["cdf97"][:2])
    got = [coef[0] for _, _, coef in f.steps]
    assert np.allclose(got, [c["a"], c["b"], c["g"], c["d"]], atol=1e-12, rtol=0)
    assert all(len(coef) == 2 and abs(coef[0] - coef[1]) < 1e-12 for _, _, coef in f.steps)
    assert np.allclose(f.scaling, (c["x"], 0, 1 / c["x"], 0))
    f = S.Lifting(*O.TAPS["cdf97"][2:])     # dual side: the same multipliers, negated, dual order
    got = [coef[0] for _, _, coef in f.steps]
    assert np.allclose(got, [-c["a"], -c["b"], -c["g"], -c["d"]], atol=1e-12, rtol=0)


def _pairs():
    out = [(name, side) for name in ("legall53", "cdf97", "d4") for side in ("x", "y")]
    return out


@pytest.mark.parametrize("name,side", _pairs())
def test_steps_reproduce_the_taps(S, name, side):
    xl, xh, yl, yh = O.TAPS[name]
    lo, hi = (xl, xh) if side == "x" else (yl, yh)
    f = S.Lifting(lo, hi)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(64)
    A, B = apply_steps(f, u)
    assert np.abs(A - O.analyze(u, lo)).max() < 1e-12
    assert np.abs(B - O.analyze(u, hi)).max() < 1e-12


@pytest.mark.parametrize("t", [0.9, 1.1, 1.25, 1.6, 1.230174104914001])
def test_the_97_family_round_trips(S, t):
    consts = O.cdf97_constants_from_t(t)
    lo, hi = taps_of(lambda u, c: O.lift_x("cdf97", u, c), consts)
    f = S.Lifting(lo, hi)
    got = [coef[0] for _, _, coef in f.steps]
    assert np.allclose(got, [consts["a"], consts["b"], consts["g"], consts["d"]], atol=1e-10)
    rng = np.random.default_rng(4)
    u = rng.standard_normal(64)
    A, B = apply_steps(f, u)
    assert np.abs(A - O.analyze(u, lo)).max() < 1e-12
    assert np.abs(B - O.analyze(u, hi)).max() < 1e-12


def test_irrational_cdf97_multipliers(S):
    # the irrational CDF 9/7 is the member t = 1.2301741049... of the family
    t = 1.230174104914001
    c = O.cdf97_constants_from_t(t)
    published = [-1.586134342059924, -0.052980118572961, 0.882911075530934, 0.443506852043971]
    assert np.allclose([c["a"], c["b"], c["g"], c["d"]], published, atol=1e-9)
    lo, hi = taps_of(lambda u, k: O.lift_x("cdf97", u, k), c)
    f = S.Lifting(lo, hi)
    assert np.allclose([coef[0] for _, _, coef in f.steps], published, atol=1e-9)
    # against Table I's rational multipliers: the same structure, different values
    r = O.CDF97_TABLE_I
    assert abs(r["a"] - published[0]) > 0.05 and abs(r["g"] - published[2]) > 0.05


def test_haar_and_refusals(S):
    s = 1 / math.sqrt(2)
    f = S.Lifting({0: s, 1: s}, {0: -s, 1: s})
    u = np.random.default_rng(5).standard_normal(16)
    A, B = apply_steps(f, u)
    assert np.abs(A - O.analyze(u, {0: s, 1: s})).max() < 1e-14
    assert np.abs(B - O.analyze(u, {0: -s, 1: s})).max() < 1e-14
    with pytest.raises(S.SidwtError):            # no perfect reconstruction
        S.Lifting({0: 1.0, 1: 1.0}, {0: 1.0, 1: 1.0})
    with pytest.raises(S.SidwtError):
        S.Lifting({0: 1.0, 1: 2.0, 2: 1.0}, {0: 1.0, 2: 1.0})


def test_lift_generic_arguments_are_checked_on_the_host(S):
    import ctypes
    L = S._lib.lib()
    vp = ctypes.c_void_p
    with S.Lifting(*O.TAPS["cdf97"][:2]) as f:
        h = f.handle
        assert L.sidwt_lift_generic(h, 3, None, 64, 0, 64, None, None) == 0      # nothing to do
        assert L.sidwt_lift_generic(h, 0, vp(16), 64, 1, 64, vp(16), None) == -1  # J
        assert L.sidwt_lift_generic(h, 3, vp(16), 64, 1, 63, vp(16), None) == -1  # stride < n
        assert L.sidwt_lift_generic(h, 6, vp(16), 64, 1, 64, vp(16), None) == -1  # N / 2^J < 2
        assert L.sidwt_lift_generic(h, 3, None, 64, 1, 64, vp(16), None) == -1    # no input
        assert L.sidwt_lift_generic(h, 3, vp(16), 1 << 20, 1, 1 << 20, vp(16), None) == -5  # LDS
    assert L.sidwt_lift_generic(None, 3, vp(16), 64, 1, 64, vp(16), None) == -1
    assert L.sidwt_lifting_count(None) == -1
    assert L.sidwt_lifting_step(None, 0, None, None, None, None) == -1
