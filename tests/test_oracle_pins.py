"""Pins of the CPU oracle against what the paper and mathematics fix.

Every check here is independent of the oracle's own formulas: printed taps
and Table I (golden fixtures), lifting impulse responses, the dual-analysis
identity, FFT correlation, closed-form special cases (DC, delta),
shift-circulance, perfect reconstruction / reversibility, textbook D4
properties, and brute force in scalar Python on tiny inputs.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O

SCALES = {"1": 1.0, "sqrt2": math.sqrt(2), "1/(10sqrt2)": 1 / (10 * math.sqrt(2)),
          "1/(4sqrt2)": 1 / (4 * math.sqrt(2))}
FLOATS = ["legall53", "cdf97", "d4"]


def load_taps(golden_dir):
    out = {}
    with open(os.path.join(golden_dir, "printed_taps.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, first, scale, vals = [p.strip() for p in line.split("|")]
            vals = [float(Fraction(v)) * SCALES[scale] for v in vals.split()]
            out[name] = {int(first) + k: v for k, v in enumerate(vals)}
    return out


def load_table1(golden_dir):
    out = {}
    with open(os.path.join(golden_dir, "table1.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = [p.strip() for p in line.split("|")]
            out[k] = float(Fraction(v))
    return out


def taps_equal(a, b, tol=1e-15):
    keys = set(a) | set(b)
    return all(abs(a.get(k, 0.0) - b.get(k, 0.0)) <= tol for k in keys)


def impulse_response(fn, N=32, band=0):
    """Taps of a one-level operator: column responses to unit impulses,
    read back as offsets relative to 2k for output k = N/4."""
    k = N // 4
    taps = {}
    for n in range(N):
        u = np.zeros(N)
        u[n] = 1.0
        v = fn(u)[band][k]
        if abs(v) > 1e-14:
            taps[n - 2 * k] = float(v)
    return taps


def crandn(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


# ---------------------------------------------------------------------------
# P1: printed taps, Table I, lifting impulse responses
# ---------------------------------------------------------------------------

def test_oracle_taps_are_the_printed_ones(golden_dir):
    g = load_taps(golden_dir)
    assert taps_equal(O.LEGALL53_X_LO, g["legall53.x_lo"])
    assert taps_equal(O.LEGALL53_X_HI, g["legall53.x_hi"])
    assert taps_equal(O.LEGALL53_Y_LO, g["legall53.y_lo"])
    assert taps_equal(O.LEGALL53_Y_HI, g["legall53.y_hi"])
    assert taps_equal(O.CDF97_X_LO, g["cdf97.x_lo"])
    assert taps_equal(O.CDF97_Y_LO, g["cdf97.y_lo"])


def test_table1_from_free_variable(golden_dir):
    t1 = load_table1(golden_dir)
    c = O.cdf97_constants_from_t(t1["t"])
    for k in "abgd":
        assert abs(c[k] - t1[k]) < 1e-15
        assert abs(O.CDF97_TABLE_I[k] - t1[k]) < 1e-15
    assert abs(c["x"] - t1["x_over_sqrt2"] * math.sqrt(2)) < 1e-15
    assert abs(O.CDF97_TABLE_I["x"] - t1["x_over_sqrt2"] * math.sqrt(2)) < 1e-15


@pytest.mark.parametrize("filt", FLOATS)
def test_lifting_impulse_response_equals_taps(filt, golden_dir):
    g = load_taps(golden_dir)
    xlo, xhi, ylo, yhi = O.TAPS[filt]
    got = {
        "x_lo": impulse_response(lambda u: O.lift_x(filt, u), band=0),
        "x_hi": impulse_response(lambda u: O.lift_x(filt, u), band=1),
        "y_lo": impulse_response(lambda u: O.lift_y(filt, u), band=0),
        "y_hi": impulse_response(lambda u: O.lift_y(filt, u), band=1),
    }
    for key, want in zip(["x_lo", "x_hi", "y_lo", "y_hi"], [xlo, xhi, ylo, yhi]):
        assert taps_equal(got[key], want, 1e-14), (filt, key, got[key], want)
        printed = g.get(f"{filt}.{key}")
        if printed is not None:
            assert taps_equal(got[key], printed, 1e-14), (filt, key)


def test_cdf97_highpass_matches_eq7_from_the_lifting():
    # The lifting highpass responses must be the eq. (7) highpasses built from
    # the *printed* lowpass filters (not from the oracle's own tables).
    xh = impulse_response(lambda u: O.lift_x("cdf97", u), band=1)
    yh = impulse_response(lambda u: O.lift_y("cdf97", u), band=1)
    h = O.CDF97_Y_LO
    ht = O.CDF97_X_LO
    want_xh = {q: (-1) ** (q + 1) * h[q - 1] for q in range(-2, 5)}
    want_yh = {q: (-1) ** (q + 1) * ht[q - 1] for q in range(-3, 6)}
    assert taps_equal(xh, want_xh, 1e-14)
    assert taps_equal(yh, want_yh, 1e-14)


def test_d4_textbook_properties_and_eq17_polyphase():
    h = np.array(O.D4_H)
    assert abs(h.sum() - math.sqrt(2)) < 1e-15           # lowpass normalisation
    assert abs((h * h).sum() - 1) < 1e-15                # unit energy
    assert abs(h[0] * h[2] + h[1] * h[3]) < 1e-15        # orthogonal to even shifts
    k = np.arange(4)
    assert abs(((-1) ** k * h).sum()) < 1e-15            # two vanishing moments
    assert abs(((-1) ** k * k * h).sum()) < 1e-15
    # eq. (17) multiplied out must give the polyphase matrix P~'(z^-1):
    # rows [h0 + h2 z^-1, h1 + h3 z^-1 ; -h3 - h1 z^-1, h2 + h0 z^-1] on
    # pairs (e[k], o[k]) = (u[2k], u[2k-1]).
    lo = impulse_response(lambda u: O.lift_x("d4", u), band=0)
    hi = impulse_response(lambda u: O.lift_x("d4", u), band=1)
    assert taps_equal(lo, {0: h[0], -1: h[1], -2: h[2], -3: h[3]}, 1e-14)
    assert taps_equal(hi, {0: -h[3], -1: h[2], -2: -h[1], -3: h[0]}, 1e-14)


# ---------------------------------------------------------------------------
# P2: dual-analysis identity and the two-band form of the planes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", FLOATS)
def test_dual_analysis_identity(filt):
    rng = np.random.default_rng(7)
    N = 32
    # matrix form: A_x^T A_y + B_x^T B_y = I  (eq. (13))
    I = np.eye(N)
    Ax = np.stack([O.lift_x(filt, I[n])[0] for n in range(N)])
    Bx = np.stack([O.lift_x(filt, I[n])[1] for n in range(N)])
    Cy = np.stack([O.lift_y(filt, I[n])[0] for n in range(N)])
    Dy = np.stack([O.lift_y(filt, I[n])[1] for n in range(N)])
    assert np.abs(Ax @ Cy.T + Bx @ Dy.T - I).max() < 1e-14
    # inner-product form, complex, conjugate on the reference (eq. (4), (15))
    u, v = crandn(rng, N), crandn(rng, N)
    A, B = O.lift_x(filt, u)
    C, D = O.lift_y(filt, v)
    lhs = np.vdot(u, v)
    assert abs(np.vdot(A, C) + np.vdot(B, D) - lhs) < 1e-13 * abs(lhs) + 1e-13


@pytest.mark.parametrize("filt", FLOATS)
def test_two_band_form_equals_direct_form(filt):
    rng = np.random.default_rng(11)
    x, y = crandn(rng, 21), crandn(rng, 128)
    a = O.correlate_direct(filt, 4, x, y)
    b = O.correlate_dwt(filt, 4, x, y)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


# ---------------------------------------------------------------------------
# P3: plane 0 is the plain circular cross-correlation (FFT, textbook)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", FLOATS)
def test_plane0_is_fft_cross_correlation(filt):
    rng = np.random.default_rng(3)
    x, y = crandn(rng, 37), crandn(rng, 100)    # ragged n -> N = 104
    J = 3
    N = O.transform_length(100, J)
    assert N == 104
    r = O.correlate_direct(filt, J, x, y)
    X = np.zeros(N, complex)
    X[:37] = x
    Y = np.zeros(N, complex)
    Y[:100] = y
    want = np.fft.ifft(np.conj(np.fft.fft(X)) * np.fft.fft(Y))
    assert np.abs(r[0] - want).max() < 1e-12 * np.abs(want).max()


# ---------------------------------------------------------------------------
# P4: perfect reconstruction / reversibility
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", FLOATS)
def test_perfect_reconstruction(filt):
    rng = np.random.default_rng(5)
    u = crandn(rng, 16)
    A, B = O.lift_x(filt, u)
    assert np.abs(O.unlift_x(filt, A, B) - u).max() < 1e-14


def test_integer_lifting_is_reversible():
    rng = np.random.default_rng(6)
    u = rng.integers(-2048, 2048, size=(20, 64))
    A, B = O.i2i_lift_x(u)
    assert np.array_equal(O.i2i_unlift_x(A, B), u)
    C, D = O.i2i_lift_y(u)
    assert np.array_equal(O.i2i_unlift_y(C, D), u)


@pytest.mark.parametrize("filt", ["legall53", "cdf97", "d4"])
def test_y_side_synthesis_inverts_y_side_analysis(filt):
    """The coarse-to-fine step (eq. (21)): the y-side steps undone in reverse
    order return the finer approximation, one level and across J levels
    (synthesize_y from c_J and the details gives back c_to, c_0 = the pulse)."""
    rng = np.random.default_rng(15)
    u = crandn(rng, 64)
    C, D = O.lift_y(filt, u)
    assert np.abs(O.unlift_y(filt, C, D) - u).max() < 1e-13
    J, c, details, approx = 4, u, [], [u]
    for _ in range(J):
        c, d = O.lift_y(filt, c)
        details.append(d)
        approx.append(c)
    for to in range(J):
        got = O.synthesize_y(filt, details, approx[J], to)
        assert np.abs(got - approx[to]).max() < 1e-12 * np.abs(approx[to]).max()


def test_integer_synthesis_is_exact():
    rng = np.random.default_rng(16)
    u = rng.integers(-2048, 2048, size=(3, 64))
    J, c, details, approx = 5, u, [], [u]
    for _ in range(J):
        c, d = O.i2i_lift_y(c)
        details.append(d)
        approx.append(c)
    for to in range(J):
        assert np.array_equal(O.synthesize_y("legall53_int", details, approx[J], to), approx[to])


def test_53_synthesis_matrix_inverts_analysis():
    # Sec. III-C Case I: P~(z^-1) P(z) = I/2, so the synthesis P(z) as printed
    # (scaled by 2) applied to (A, B) returns 2x... the oracle's unlift uses
    # the scaled form, whose product with the analysis is the identity.
    rng = np.random.default_rng(8)
    u = rng.standard_normal(32)
    A, B = O.lift_x("legall53", u)
    assert np.abs(O.unlift_x("legall53", A, B) - u).max() < 1e-14


# ---------------------------------------------------------------------------
# P5: energy equivalence for the orthogonal D4 bank
# ---------------------------------------------------------------------------

def test_d4_energy_equivalence():
    rng = np.random.default_rng(9)
    u = crandn(rng, 64)
    e = 0.0
    a = u
    for _ in range(4):
        a, b = O.lift_x("d4", a)
        e += np.vdot(b, b).real
    e += np.vdot(a, a).real
    assert abs(e - np.vdot(u, u).real) < 1e-12 * np.vdot(u, u).real


# ---------------------------------------------------------------------------
# P6: shift-circulance of the reference coefficients
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", FLOATS + ["legall53_int"])
def test_shift_circulance(filt):
    rng = np.random.default_rng(12)
    N, m = 64, 13
    if filt == "legall53_int":
        ref = rng.integers(-2047, 2048, size=(m, 2))
    else:
        ref = crandn(rng, m)
    for lvl in (1, 2, 3):
        P = 1 << lvl
        for s in range(0, N, 5):
            A, B = O.reference_phase(filt, ref, N, lvl, s)
            A0, B0 = O.reference_phase(filt, ref, N, lvl, s % P)
            assert np.abs(A - np.roll(A0, s // P)).max() < 1e-12
            assert np.abs(B - np.roll(B0, s // P)).max() < 1e-12


# ---------------------------------------------------------------------------
# P7: shift-equivariance, in exactly the forms that hold
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", FLOATS)
def test_shift_equivariance_float(filt):
    rng = np.random.default_rng(13)
    J, n, m = 3, 64, 11
    x, y = crandn(rng, m), crandn(rng, n)
    R = O.correlate_direct(filt, J, x, y)
    # (i) delaying the reference by any t: R'[s] = R[s + t]
    t = 5
    xd = np.concatenate([np.zeros(t), x])
    Rx = O.correlate_direct(filt, J, xd, y)
    assert np.abs(Rx - np.roll(R, -t, axis=1)).max() < 1e-12 * np.abs(R).max()
    # (ii) delaying rx by a multiple of 2^J: R'[s] = R[s - t] on every plane
    t = 8
    Ry = O.correlate_direct(filt, J, x, np.roll(y, t))
    assert np.abs(Ry - np.roll(R, t, axis=1)).max() < 1e-12 * np.abs(R).max()
    # (iii) plane 0 for any delay
    t = 3
    Ry = O.correlate_direct(filt, J, x, np.roll(y, t))
    assert np.abs(Ry[0] - np.roll(R[0], t)).max() < 1e-12 * np.abs(R).max()


def test_shift_equivariance_integer_reference_delay():
    rng = np.random.default_rng(14)
    J = 3
    x = rng.integers(-2047, 2048, size=(9, 2))
    y = rng.integers(-2048, 2048, size=(64, 2))
    R = O.correlate_int(J, x, y)
    t = 7
    xd = np.concatenate([np.zeros((t, 2), np.int64), x])
    Rd = O.correlate_int(J, xd, y)
    assert np.array_equal(Rd, np.roll(R, -t, axis=1))


# ---------------------------------------------------------------------------
# P8: planted peak (noise-free chirp)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", FLOATS)
def test_planted_peak(filt):
    from workloads import lfm_chirp
    m, n, J = 32, 256, 3
    x = lfm_chirp(m, 16)
    for d in (0, 37, 100, 224):
        y = np.zeros(n, complex)
        y[d:d + m] = x
        R = O.correlate_direct(filt, J, x, y)
        assert int(np.argmax(np.abs(R[0]))) == d
        for j in range(1, J):
            assert abs(int(np.argmax(np.abs(R[j]))) - d) < (1 << j)


# ---------------------------------------------------------------------------
# P9 / P10: DC and delta special cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", FLOATS)
def test_dc_input_gives_conj_sum_on_every_plane(filt):
    rng = np.random.default_rng(15)
    x = crandn(rng, 19)
    y = np.ones(64, complex)
    R = O.correlate_direct(filt, 4, x, y)
    assert np.abs(R - np.conj(x.sum())).max() < 1e-12 * abs(x.sum()) + 1e-12


@pytest.mark.parametrize("filt", FLOATS)
def test_delta_reference_plane0_is_rx(filt):
    rng = np.random.default_rng(16)
    y = crandn(rng, 48)
    R = O.correlate_direct(filt, 3, np.array([1.0 + 0j]), y)
    assert np.abs(R[0] - y).max() < 1e-14


# ---------------------------------------------------------------------------
# P11: integer path close to the float 5/3 path, bounded bit growth
# ---------------------------------------------------------------------------

def test_integer_planes_track_float_53_planes():
    from workloads import int_reference, int_pulse
    J = 3
    ref = int_reference(64).astype(np.int64)
    rx = int_pulse(99, 0, n=256, m=64).astype(np.int64)
    Ri = O.correlate_int(J, ref, rx)
    Rf = O.correlate_direct("legall53", J, ref[:, 0] + 1j * ref[:, 1], rx[:, 0] + 1j * rx[:, 1])
    Ric = Ri[..., 0] + 1j * Ri[..., 1]
    for j in range(J):
        rel = np.linalg.norm(Ric[j] - Rf[j]) / np.linalg.norm(Rf[j])
        assert rel < 2e-2, (j, rel)


def test_integer_bit_growth():
    rng = np.random.default_rng(17)
    u = rng.integers(-2048, 2048, size=(4, 4096))
    c = u
    for lvl in range(1, 7):
        c, d = O.i2i_lift_y(c)
        assert np.abs(c).max() <= 2 ** (11 + lvl)
        assert np.abs(d).max() <= 2 ** (11 + lvl)


# ---------------------------------------------------------------------------
# P12: brute force in scalar Python on tiny inputs
# ---------------------------------------------------------------------------

def _scalar_analyze(u, taps):
    L = len(u)
    return [sum(c * u[(2 * k + i) % L] for i, c in taps.items()) for k in range(L // 2)]


@pytest.mark.parametrize("filt", FLOATS)
def test_brute_force_tiny(filt):
    rng = np.random.default_rng(18)
    J, n, m = 3, 24, 7          # N = 24: ragged (not a power of two)
    x, y = crandn(rng, m), crandn(rng, n)
    R = O.correlate_direct(filt, J, x, y)
    xlo, _, ylo, _ = O.TAPS[filt]
    N = 24
    xs = list(x) + [0] * (N - m)
    for j in range(J):
        c = list(y)
        for _ in range(j):
            c = _scalar_analyze(c, ylo)
        for s in range(N):
            a = [xs[(t - s) % N] for t in range(N)]
            for _ in range(j):
                a = _scalar_analyze(a, xlo)
            want = sum(complex(ai).conjugate() * ci for ai, ci in zip(a, c))
            assert abs(R[j, s] - want) < 1e-12


def _scalar_i2i_x(u):
    L = len(u) // 2
    e = [u[2 * k] for k in range(L)]
    o = [u[2 * k + 1] for k in range(L)]
    o = [o[k] - (e[k] + e[(k + 1) % L]) // 2 for k in range(L)]
    e = [e[k] + (o[k - 1] + o[k] + 2) // 4 for k in range(L)]
    return e, o


def _scalar_i2i_y(u):
    L = len(u) // 2
    e = [u[2 * k] for k in range(L)]
    o = [u[2 * k + 1] for k in range(L)]
    e = [e[k] + (o[k - 1] + o[k] + 1) // 2 for k in range(L)]
    o = [o[k] - (e[k] + e[(k + 1) % L] + 2) // 4 for k in range(L)]
    return e, o


def test_brute_force_integer_tiny():
    rng = np.random.default_rng(19)
    J, n, m = 2, 16, 5
    x = rng.integers(-2047, 2048, size=(m, 2))
    y = rng.integers(-2048, 2048, size=(n, 2))
    R = O.correlate_int(J, x, y)
    N = 16
    for j in range(J):
        cy = [[int(v) for v in y[:, 0]], [int(v) for v in y[:, 1]]]
        for _ in range(j):
            cy = [_scalar_i2i_y(cy[0])[0], _scalar_i2i_y(cy[1])[0]]
        Cr, Dr = _scalar_i2i_y(cy[0])
        Ci, Di = _scalar_i2i_y(cy[1])
        for s in range(N):
            xr = [int(x[(t - s) % N, 0]) if (t - s) % N < m else 0 for t in range(N)]
            xi = [int(x[(t - s) % N, 1]) if (t - s) % N < m else 0 for t in range(N)]
            for _ in range(j):
                xr, xi = _scalar_i2i_x(xr)[0], _scalar_i2i_x(xi)[0]
            Ar, Br = _scalar_i2i_x(xr)
            Ai, Bi = _scalar_i2i_x(xi)
            re = sum(a * c for a, c in zip(Ar, Cr)) + sum(a * c for a, c in zip(Ai, Ci)) \
                + sum(a * c for a, c in zip(Br, Dr)) + sum(a * c for a, c in zip(Bi, Di))
            im = sum(a * c for a, c in zip(Ar, Ci)) - sum(a * c for a, c in zip(Ai, Cr)) \
                + sum(a * c for a, c in zip(Br, Di)) - sum(a * c for a, c in zip(Bi, Dr))
            assert R[j, s, 0] == re and R[j, s, 1] == im


def test_correlate_at_matches_full_planes():
    rng = np.random.default_rng(20)
    x, y = crandn(rng, 30), crandn(rng, 96)
    R = O.correlate_direct("cdf97", 3, x, y)
    lags = [0, 5, 47, 95]
    for j in range(3):
        assert np.abs(O.correlate_at("cdf97", 3, x, y, j, lags) - R[j, lags]).max() < 1e-13


# ---------------------------------------------------------------------------
# P13: roles exchanged (redundant analysis on the received signal, critical
# on the reference): plane 0 is the FFT cross-correlation, a shift of the
# received signal shifts every plane by exactly that many lags, plane j
# agrees with the direct form at lags that are multiples of 2^j (where both
# sides see the same phase), for the orthogonal D4 bank the exchange is the
# conjugate of the direct form with the signals' roles swapped, and scalar
# brute force on a tiny input.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("filt", FLOATS)
def test_swapped_plane0_is_fft_cross_correlation(filt):
    rng = np.random.default_rng(31)
    x, y = crandn(rng, 29), crandn(rng, 90)     # N = 96
    r = O.correlate_swapped(filt, 3, x, y)
    X = np.zeros(96, complex)
    X[:29] = x
    Y = np.zeros(96, complex)
    Y[:90] = y
    want = np.fft.ifft(np.conj(np.fft.fft(X)) * np.fft.fft(Y))
    assert np.abs(r[0] - want).max() < 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("filt", FLOATS)
def test_swapped_is_exactly_covariant_in_the_received_shift(filt):
    rng = np.random.default_rng(32)
    J, N = 4, 128
    x, y = crandn(rng, 19), crandn(rng, N)
    r = O.correlate_swapped(filt, J, x, y)
    for t in (1, 3, 8):
        rt = O.correlate_swapped(filt, J, x, np.roll(y, t))
        assert np.abs(rt - np.roll(r, t, axis=1)).max() < 1e-12 * np.abs(r).max()
    # the direct form is not (its redundant analysis sits on the reference)
    d = O.correlate_direct(filt, J, x, y)
    d1 = O.correlate_direct(filt, J, x, np.roll(y, 1))
    assert np.abs(d1[1:] - np.roll(d[1:], 1, axis=1)).max() > 1e-3 * np.abs(d).max()


@pytest.mark.parametrize("filt", FLOATS)
def test_swapped_equals_direct_on_the_common_phase(filt):
    rng = np.random.default_rng(33)
    J, N = 4, 96
    x, y = crandn(rng, 23), crandn(rng, N)
    r = O.correlate_swapped(filt, J, x, y)
    d = O.correlate_direct(filt, J, x, y)
    for j in range(J):
        s = np.arange(0, N, 1 << j)
        assert np.abs(r[j, s] - d[j, s]).max() < 1e-12 * np.abs(d).max()
        if j:   # other lags: a different polyphase component, not equal
            o = np.arange(1, N, 1 << j)
            assert np.abs(r[j, o] - d[j, o]).max() > 1e-3 * np.abs(d).max()


def test_swapped_d4_is_the_conjugate_of_the_direct_form_with_roles_swapped():
    rng = np.random.default_rng(34)
    J, N = 3, 64
    x, y = crandn(rng, N), crandn(rng, N)
    r = O.correlate_swapped("d4", J, x, y)
    d = O.correlate_direct("d4", J, y, x)
    neg = (-np.arange(N)) % N
    assert np.abs(r - np.conj(d[:, neg])).max() < 1e-12 * np.abs(r).max()


@pytest.mark.parametrize("filt", FLOATS)
def test_swapped_brute_force_tiny(filt):
    rng = np.random.default_rng(35)
    J, n, m = 3, 24, 6
    x, y = crandn(rng, m), crandn(rng, n)
    R = O.correlate_swapped(filt, J, x, y)
    xlo, _, ylo, _ = O.TAPS[filt]
    N = 24
    xs = list(x) + [0] * (N - m)
    for j in range(J):
        a = list(xs)
        for _ in range(j):
            a = _scalar_analyze(a, xlo)
        for s in range(N):
            c = [y[(t + s) % N] for t in range(N)]
            for _ in range(j):
                c = _scalar_analyze(c, ylo)
            want = sum(complex(ai).conjugate() * ci for ai, ci in zip(a, c))
            assert abs(R[j, s] - want) < 1e-12


def test_swapped_sampled_lags_equal_the_full_planes():
    rng = np.random.default_rng(36)
    x, y = crandn(rng, 17), crandn(rng, 80)
    r = O.correlate_swapped("cdf97", 4, x, y)
    lags = [0, 3, 17, 79]
    for j in range(4):
        assert np.abs(O.correlate_swapped_at("cdf97", 4, x, y, j, lags) - r[j, lags]).max() < 1e-13


# ---------------------------------------------------------------------------
# P14: target declaration (local power maxima above a level relative to the
# plane's peak): closed-form cases and scalar brute force.
# ---------------------------------------------------------------------------

def _plane(N, pts):
    z = np.zeros(N, np.complex64)
    for i, v in pts.items():
        z[i] = v
    return z


def test_detect_closed_forms():
    rel = np.float32(0.1)
    (l, d), = O.detect_peaks(_plane(64, {7: 3 - 4j}), rel, 8)
    assert list(l) == [7] and abs(d[0]) < 1e-12                       # a delta
    bumps = _plane(64, {9: 0.5, 10: 1.0, 11: 0.5, 39: 0.3j, 40: np.sqrt(0.5) * 1j, 41: 0.3j})
    (l, d), = O.detect_peaks(bumps, rel, 8)
    assert list(l) == [10, 40] and abs(d[1] - 10 * np.log10(0.5)) < 1e-6
    (l, _), = O.detect_peaks(bumps, np.float32(0.6), 8)               # level above the second
    assert list(l) == [10]
    (l, _), = O.detect_peaks(_plane(32, {20: 1.0, 21: 1.0}), rel, 8)  # flat top: first sample
    assert list(l) == [20]
    (l, _), = O.detect_peaks(_plane(32, {0: 1.0, 31: 0.5, 1: 0.5}), rel, 8)   # circular
    assert list(l) == [0]
    (l, _), = O.detect_peaks(_plane(32, {31: 1.0, 30: 0.5, 0: 0.5}), rel, 8)
    assert list(l) == [31]
    (l, _), = O.detect_peaks(np.zeros(16, np.complex64), rel, 8)      # nothing there
    assert len(l) == 0
    (l, _), = O.detect_peaks(np.full(16, 1 + 1j, np.complex64), rel, 8)  # constant: no rise
    assert len(l) == 0


def test_detect_brute_force_tiny():
    rng = np.random.default_rng(37)
    f32 = np.float32
    for trial in range(20):
        N = int(rng.integers(3, 40))
        z = (rng.standard_normal(N) + 1j * rng.standard_normal(N)).astype(np.complex64)
        if trial % 3 == 0:   # some exact ties
            z[int(rng.integers(0, N))] = z[0]
        rel = f32(rng.choice([0.0, 0.05, 0.3, 0.9]))
        (l, _), = O.detect_peaks(z, rel, 64)
        p = [f32(f32(f32(c.real) * f32(c.real)) + f32(f32(c.imag) * f32(c.imag))) for c in z]
        M = max(p)
        thr = f32(rel * M)
        want = [s for s in range(N)
                if p[s] > p[(s - 1) % N] and p[s] >= p[(s + 1) % N] and p[s] >= thr]
        assert list(l) == want, trial
