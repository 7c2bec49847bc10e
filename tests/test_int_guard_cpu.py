"""CPU checks of the integer plan's exactness guard (host planning code):
the per-level bounds it uses for the pulse and reference coefficients, and
the partial-sum bound it compares with 2^53, must hold for what the oracle's
integer lifting actually produces -- full-scale DC pulses (the pulse side's
worst case: the y-side lowpass (1/2, 1, 1/2) has only positive taps, so its
l1 norm 2 per level is reached), inputs carrying the sign pattern of a
composite filter, and brute-force sums of |terms| of tiny correlations --
and against the composite l1 norms of the x-side filters up to 16 levels."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from oracle import sidwt_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bounds_exe(tmp_path_factory):
    cxx = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not cxx:
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("ibc") / "int_bound_check"
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "cpp", "int_bound_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    return str(exe)


def guard(exe, J, m, peak):
    """{level: (xp_{l-1}, xr_{l-1}, len0, len1, sum_bound)}, accepted."""
    r = subprocess.run([exe, str(J), str(m), str(peak)], capture_output=True, text=True, check=True)
    rows, ok = {}, None
    for line in r.stdout.splitlines():
        f = line.split()
        if f[0] == "exact":
            ok = f[1] == "1"
        else:
            rows[int(f[0])] = (float(f[1]), float(f[2]), int(f[3]), int(f[4]), float(f[5]))
    return rows, ok


def approx_bound(rows, level):
    """Bound on the level-`level` approximation (pulse, reference) implied
    by the guard's recursion."""
    xp, xr = rows[1][0], rows[1][1]
    for _ in range(level):
        xp, xr = 2 * xp + 1, 1.5 * xr + 2
    return xp, xr


def composite(taps_first: dict, taps_next: dict, levels: int):
    """Impulse response of `levels` levels of convolve-and-downsample: the
    first level with taps_first, the earlier ones with taps_next (the
    approximation filter), as a dict offset -> coefficient on the input."""
    resp = dict(taps_first)
    for _ in range(levels - 1):
        nxt = {}
        # out[k] = sum_i c_i a[2k + i], a[q] = sum_t h_t u[2q + t]
        for i, c in resp.items():
            for t, h in taps_next.items():
                nxt[2 * i + t] = nxt.get(2 * i + t, 0.0) + c * h
        resp = nxt
    return resp


@pytest.mark.parametrize("value", [-32768, 32767])
def test_pulse_bound_covers_a_full_scale_dc_pulse(bounds_exe, value):
    J = 10
    rows, _ = guard(bounds_exe, J, 64, 2047)
    u = np.full(1 << (J + 2), value, np.int64)
    c = u
    for lvl in range(1, J + 1):
        xp_prev = approx_bound(rows, lvl - 1)[0]
        c, d = O.i2i_lift_y(c)
        assert np.abs(c).max() <= 2 * xp_prev + 1
        assert np.abs(d).max() <= 2 * xp_prev + 1
        # the DC pulse nearly reaches the bound: growth 2 per level
        assert np.abs(c).max() >= (2 * xp_prev + 1) * 0.99
        assert abs(int(c[0])) == abs(value) * 2 ** lvl or value > 0


def test_pulse_detail_bound_covers_its_sign_pattern(bounds_exe):
    J = 8
    rows, _ = guard(bounds_exe, J, 64, 2047)
    for lvl in range(1, J + 1):
        hi = composite(O.LEGALL53_Y_HI, O.LEGALL53_Y_LO, lvl)
        N = 1 << (lvl + 4)
        u = np.zeros(N, np.int64)
        for off, c in hi.items():   # output 4 of level lvl reads u[2^lvl * 4 + off]
            u[((4 << lvl) + off) % N] = 32767 if c > 0 else -32768
        a = u
        for _ in range(lvl):
            a, d = O.i2i_lift_y(a)
        xp_prev = approx_bound(rows, lvl - 1)[0]
        assert np.abs(d).max() <= 2 * xp_prev + 1
        assert np.abs(a).max() <= 2 * xp_prev + 1


@pytest.mark.parametrize("peak", [2047, 32767])
def test_reference_bound_covers_composite_l1_norms(bounds_exe, peak):
    J = 16
    rows, _ = guard(bounds_exe, J, 64, peak)
    for lvl in range(1, J + 1):
        xr_prev = approx_bound(rows, lvl - 1)[1]
        lo = composite(O.LEGALL53_X_LO, O.LEGALL53_X_LO, lvl)
        hi = composite(O.LEGALL53_X_HI, O.LEGALL53_X_LO, lvl)
        # the detail scaling 1/2 is dropped by the integer lifting: its
        # highpass is 2 g~
        assert 2 * xr_prev + 1 >= peak * sum(abs(c) for c in lo.values())
        assert 2 * xr_prev + 1 >= peak * 2 * sum(abs(c) for c in hi.values())


def test_reference_bound_covers_its_sign_patterns(bounds_exe):
    J, peak = 7, 32767
    rows, _ = guard(bounds_exe, J, 64, peak)
    for lvl in range(1, J + 1):
        for taps in (composite(O.LEGALL53_X_LO, O.LEGALL53_X_LO, lvl),
                     composite(O.LEGALL53_X_HI, O.LEGALL53_X_LO, lvl)):
            N = 1 << (lvl + 5)
            u = np.zeros(N, np.int64)
            for off, c in taps.items():
                u[((4 << lvl) + off) % N] = peak if c > 0 else -peak
            a = u
            for _ in range(lvl):
                a, b = O.i2i_lift_x(a)
            xr_prev = approx_bound(rows, lvl - 1)[1]
            assert np.abs(a).max() <= 2 * xr_prev + 1
            assert np.abs(b).max() <= 2 * xr_prev + 1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_partial_sums_stay_within_the_guard_bound(bounds_exe, seed):
    """Brute force: for every lag of a tiny correlation, the sum of |terms|
    (which bounds every partial sum in any order) stays below the guard's
    level bound; inputs are full-scale random signs and DC."""
    rng = np.random.default_rng(seed)
    J, m, n = 3, 24, 64
    ref = rng.choice([-32768, 32767], size=(m, 2)).astype(np.int64)
    peak = int(np.abs(ref).max())
    rows, ok = guard(bounds_exe, J, m, peak)
    assert ok
    for rx in (rng.choice([-32768, 32767], size=(n, 2)), np.full((n, 2), -32768)):
        rx = np.asarray(rx, np.int64)
        N = O.transform_length(n, J)
        for j in range(J):
            lvl = j + 1
            (c_re, c_im), (d_re, d_im) = O.i2i_bands_y(O.zero_pad(rx[:, 0], N),
                                                       O.zero_pad(rx[:, 1], N), lvl)
            X_re = np.stack([np.roll(O.zero_pad(ref[:, 0], N), s) for s in range(N)])
            X_im = np.stack([np.roll(O.zero_pad(ref[:, 1], N), s) for s in range(N)])
            (a_re, a_im), (b_re, b_im) = O.i2i_bands_x(X_re, X_im, lvl)
            absum = (np.abs(a_re) @ np.abs(c_re) + np.abs(a_im) @ np.abs(c_im)
                     + np.abs(b_re) @ np.abs(d_re) + np.abs(b_im) @ np.abs(d_im))
            assert absum.max() <= rows[lvl][4]
            # nonzero reference terms per lag fit the stored supports
            nz = (np.count_nonzero(a_re | a_im, axis=1) + np.count_nonzero(b_re | b_im, axis=1))
            assert nz.max() <= rows[lvl][2] + rows[lvl][3]


def test_guard_refuses_where_the_true_growth_passes_2_to_53(bounds_exe):
    """J = 12 with a full-scale reference: the pulse's level-11
    approximation reaches 2^11 * 32768 for a DC pulse, so the level-12 sums
    can exceed 2^53; the guard refuses the plan.  Quiet references keep deep
    plans."""
    rows, ok = guard(bounds_exe, 12, 64, 32767)
    assert not ok
    _, ok = guard(bounds_exe, 16, 64, 100)
    assert ok
    _, ok = guard(bounds_exe, 6, 512, 2047)  # the 16384 x 4096 integer workload
    assert ok
