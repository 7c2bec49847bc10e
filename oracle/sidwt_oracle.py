"""Plain CPU oracle for multiresolution SIDWT correlation of complex signals.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code, constants or tables with the HIP
library: every tap below is typed in from the paper, and every routine is a
slow, literal rendering of the definitions.

Paper: C. Bhattacharya and P.R. Mahapatra, "A Novel Application of Lifting
Scheme for Multiresolution Correlation of Complex Radar Signals".

What is computed (float filters, FP64):

* Sec. II, eq. (2): the level-j approximation of a vector is j-fold
  convolve-and-downsample (Mallat) with the lowpass analysis filter.  The
  reference x is analysed with the x-side lowpass, the received y with the
  y-side (dual analysis) lowpass, Sec. III-A eq. (13).
* Sec. II, eq. (5)/(6) and Sec. IV, eq. (20)/(20a): the correlation at scale
  2^j for shift s is the inner product of the level-j approximation of the
  reference delayed by s with the level-j approximation of the received
  signal.  The oracle computes exactly that, for every shift, with no
  shift-circulant shortcut ("direct form").
* Conjugation sits on the reference (matched filter): plane 0 is
  sum_n conj(x[n - s]) y[n].
* Circular indexing on N = 2^J * ceil(n / 2^J) samples, both inputs
  zero-padded to N.

Integer path: the integer-to-integer (reversible) 5/3 lifting is nonlinear,
so the definition is the algorithm itself: the oracle runs the lifting steps
on every shifted reference and on the received signal, then takes the
level-(j+1) two-band inner product of eq. (15) in int64.

Each routine cites the section / equation it follows.  Every routine here is
pinned by tests against facts the paper or mathematics fix (printed taps,
Table I, the dual-analysis identity, FFT correlation, DC/delta special cases,
shift-circulance, brute force on tiny inputs).
"""
from __future__ import annotations

import math

import numpy as np

FLOAT_FILTERS = ("legall53", "cdf97", "d4")
INT_FILTERS = ("legall53_int",)
ALL_FILTERS = FLOAT_FILTERS + INT_FILTERS

SQRT2 = math.sqrt(2.0)
SQRT3 = math.sqrt(3.0)


# ---------------------------------------------------------------------------
# Filter taps, typed in from the paper.  A tap table maps an offset i to a
# coefficient c_i and is used as  out[k] = sum_i c_i * u[(2k + i) mod len(u)].
# ---------------------------------------------------------------------------

# Sec. III-C, Case I: LeGall 5/3.  x-side lowpass h~(z^-1) and highpass
# g~(z^-1), where the coefficient of z^i multiplies u[2k + i].
LEGALL53_X_LO = {-2: -1 / 8, -1: 1 / 4, 0: 3 / 4, 1: 1 / 4, 2: -1 / 8}
LEGALL53_X_HI = {0: -1 / 4, 1: 1 / 2, 2: -1 / 4}
# Synthesis pair h(z), g(z), coefficient of z^-n multiplies u[2k + n]; the
# product of analysis and synthesis matrices is I/2, so the synthesis matrix
# (and therefore the dual analysis filters) is scaled by 2.
_LEGALL53_H = {-1: 1 / 4, 0: 1 / 2, 1: 1 / 4}
_LEGALL53_G = {-1: -1 / 8, 0: -1 / 4, 1: 3 / 4, 2: -1 / 4, 3: -1 / 8}
LEGALL53_Y_LO = {i: 2 * c for i, c in _LEGALL53_H.items()}
LEGALL53_Y_HI = {i: 2 * c for i, c in _LEGALL53_G.items()}

# Sec. III-C, Case II: CDF 9/7 finite-precision lowpass pair (t = 5/4).
# The printed half-filters list outer tap first, centre tap last; both
# filters are symmetric about offset 0.
_H97_X_HALF = [9 / 16, -6 / 16, -24 / 16, 86 / 16, 190 / 16]  # times 1/(10 sqrt2)
_H97_Y_HALF = [-3 / 64, -1 / 32, 19 / 64, 18 / 32]  # times sqrt2


def _symmetric(half, scale):
    c = len(half) - 1
    taps = {}
    for k, v in enumerate(half):
        taps[k - c] = v * scale
        taps[c - k] = v * scale
    return taps


CDF97_X_LO = _symmetric(_H97_X_HALF, 1 / (10 * SQRT2))
CDF97_Y_LO = _symmetric(_H97_Y_HALF, SQRT2)


def highpass_from_eq7(lowpass):
    """Eq. (7): g~(z) = z^-1 h(-z^-1) and g(z) = z^-1 h~(-z^-1).

    With filters written as f(z) = sum_n f[n] z^-n this reads
    g[q] = (-1)^(q+1) * h[1 - q]; for the symmetric lowpass filters used
    here h[1 - q] = h[q - 1]."""
    return {1 - n: (-1) ** (1 - n + 1) * c for n, c in lowpass.items()}


CDF97_X_HI = highpass_from_eq7(CDF97_Y_LO)  # built from the synthesis lowpass h
CDF97_Y_HI = highpass_from_eq7(CDF97_X_LO)  # built from the analysis lowpass h~

# Table I: rational lifting constants of the 9/7 pair.
CDF97_TABLE_I = {"a": -3 / 2, "b": -1 / 16, "g": 4 / 5, "d": 15 / 32,
                 "x": 4 * SQRT2 / 5}


def cdf97_constants_from_t(t):
    """Sec. III-C, Case II: lifting multipliers as functions of the free
    variable t (valid for 0.780 < t < 1.852)."""
    return {"a": (-2 * t + 1) / (4 * (t - 1)), "b": -(t - 1) ** 2,
            "g": 1 / (4 * t * (t - 1)), "d": t ** 3 - 7 / 4 * t ** 2 + t,
            "x": SQRT2 / t}


# Sec. III-B: Daubechies-4 orthogonal pair in causal form.  The lowpass is
# h~(z^-1) = h0 + h1 z^-1 + h2 z^-2 + h3 z^-3 and the delayed highpass is
# g~'(z^-1) = -h3 + h2 z^-1 - h1 z^-2 + h0 z^-3; here the coefficient of
# z^-i multiplies u[2k - i].  The taps themselves are the textbook D4 values.
D4_H = [(1 + SQRT3) / (4 * SQRT2), (3 + SQRT3) / (4 * SQRT2),
        (3 - SQRT3) / (4 * SQRT2), (1 - SQRT3) / (4 * SQRT2)]
D4_LO = {-i: D4_H[i] for i in range(4)}
D4_HI = {0: -D4_H[3], -1: D4_H[2], -2: -D4_H[1], -3: D4_H[0]}

TAPS = {
    # filter: (x-side lowpass, x-side highpass, y-side lowpass, y-side highpass)
    "legall53": (LEGALL53_X_LO, LEGALL53_X_HI, LEGALL53_Y_LO, LEGALL53_Y_HI),
    "cdf97": (CDF97_X_LO, CDF97_X_HI, CDF97_Y_LO, CDF97_Y_HI),
    # Sec. III-B: for an orthogonal bank both sides use the same matrix.
    "d4": (D4_LO, D4_HI, D4_LO, D4_HI),
}


# ---------------------------------------------------------------------------
# Sizes
# ---------------------------------------------------------------------------

def transform_length(n: int, J: int) -> int:
    """Circular length: n rounded up to a multiple of 2^J."""
    q = 1 << J
    return q * ((n + q - 1) // q)


def zero_pad(v, N):
    v = np.asarray(v)
    out = np.zeros(N, dtype=v.dtype)
    out[: len(v)] = v
    return out


# ---------------------------------------------------------------------------
# Mallat analysis (Sec. II; eq. (2) and the convolve-and-downsample form
# used for the shift-circulant vectors)
# ---------------------------------------------------------------------------

def analyze(u: np.ndarray, taps: dict) -> np.ndarray:
    """One level of circular convolve-and-downsample along the last axis:
    out[..., k] = sum_i taps[i] * u[..., (2k + i) mod L]."""
    L = u.shape[-1]
    assert L % 2 == 0
    lo, hi = min(taps), max(taps)
    pl, ph = max(0, -lo), max(0, hi)
    # circular extension so that every u[(2k + i) mod L] is a strided slice
    reps = [u[..., (np.arange(-pl, 0)) % L], u, u[..., np.arange(ph) % L]]
    ext = np.concatenate(reps, axis=-1)
    out = np.zeros(u.shape[:-1] + (L // 2,), dtype=np.result_type(u, 1.0))
    for i, c in taps.items():
        out += c * ext[..., pl + i: pl + i + L: 2]
    return out


def approximation(u: np.ndarray, taps: dict, level: int) -> np.ndarray:
    """Level-`level` approximation: `level` iterations of the lowpass."""
    for _ in range(level):
        u = analyze(u, taps)
    return u


# ---------------------------------------------------------------------------
# Float correlation, direct form (Sec. II eq. (5)-(6), Sec. IV eq. (20)-(20a))
# ---------------------------------------------------------------------------

def _check_float(filt):
    if filt not in FLOAT_FILTERS:
        raise ValueError(f"not a float filter: {filt}")


def correlate_at(filt: str, J: int, ref, rx, plane: int, lags) -> np.ndarray:
    """R_plane[s] for the listed lags s, computed one shift at a time:
    approximation at level `plane` of the reference delayed by s, inner
    product (conjugate on the reference) with the approximation of rx."""
    _check_float(filt)
    ref = np.asarray(ref, dtype=np.complex128)
    rx = np.asarray(rx, dtype=np.complex128)
    N = transform_length(len(rx), J)
    if len(ref) > N:
        raise ValueError("reference longer than the transform length")
    x = zero_pad(ref, N)
    y = zero_pad(rx, N)
    xlo, _, ylo, _ = TAPS[filt]
    Cj = approximation(y, ylo, plane)
    lags = np.asarray(lags, dtype=np.int64)
    shifted = np.stack([np.roll(x, int(s)) for s in lags]) if len(lags) else \
        np.zeros((0, N), np.complex128)
    Aj = approximation(shifted, xlo, plane)
    return np.conj(Aj) @ Cj


def correlate_direct(filt: str, J: int, ref, rx, chunk: int = 256) -> np.ndarray:
    """All J planes at all N circular lags; returns complex128 [J, N].
    For each block of shifts the delayed references are analysed level by
    level; plane j takes the level-j approximations."""
    _check_float(filt)
    ref = np.asarray(ref, dtype=np.complex128)
    rx = np.asarray(rx, dtype=np.complex128)
    N = transform_length(len(rx), J)
    if len(ref) > N:
        raise ValueError("reference longer than the transform length")
    x = zero_pad(ref, N)
    y = zero_pad(rx, N)
    xlo, _, ylo, _ = TAPS[filt]
    C = [y]
    for _ in range(J - 1):
        C.append(analyze(C[-1], ylo))
    out = np.zeros((J, N), dtype=np.complex128)
    for s0 in range(0, N, chunk):
        lags = np.arange(s0, min(N, s0 + chunk))
        a = np.stack([np.roll(x, int(s)) for s in lags])
        for j in range(J):
            out[j, lags] = np.conj(a) @ C[j]
            if j + 1 < J:
                a = analyze(a, xlo)
    return out


# ---------------------------------------------------------------------------
# Lifting steps (Sec. III-B eq. (17); Sec. III-C Case I and Case II).  These
# are used to pin the printed taps (lifting impulse responses must equal
# them) and to state the DWT-domain (two-band) form of eq. (15).
# Polyphase split: e[k] = u[2k], o[k] = u[2k+1]; for the causal D4 form the
# pairs are (u[2k-1], u[2k]), i.e. o[k] = u[2k-1].
# A factor matrix acting on [e; o] is applied right-most first; z e[k] is
# e[k+1] and z^-1 o[k] is o[k-1].
# ---------------------------------------------------------------------------

def _adv(v):  # z v : v[k+1]
    return np.roll(v, -1, axis=-1)


def _dly(v):  # z^-1 v : v[k-1]
    return np.roll(v, 1, axis=-1)


def lift_x(filt: str, u: np.ndarray, consts=None):
    """x-side (analysis matrix P~(z^-1)) one level; returns (A, B)."""
    u = np.asarray(u)
    if filt == "legall53":
        e, o = u[..., 0::2] * 1.0, u[..., 1::2] * 1.0
        o = o - 0.5 * (e + _adv(e))            # [1 0; -(1+z)/2 1]
        e = e + 0.25 * (o + _dly(o))           # [1 (1+z^-1)/4; 0 1]
        return e, 0.5 * o                      # diag(1, 1/2)
    if filt == "cdf97":
        c = CDF97_TABLE_I if consts is None else consts
        e, o = u[..., 0::2] * 1.0, u[..., 1::2] * 1.0
        o = o + c["a"] * (e + _adv(e))
        e = e + c["b"] * (o + _dly(o))
        o = o + c["g"] * (e + _adv(e))
        e = e + c["d"] * (o + _dly(o))
        return c["x"] * e, o / c["x"]
    if filt == "d4":
        e = u[..., 0::2] * 1.0
        o = np.roll(u, 1, axis=-1)[..., 0::2] * 1.0  # o[k] = u[2k-1]
        o = o - SQRT3 * e                                       # [1 0; -sqrt3 1]
        e = e + (SQRT3 / 4) * o + ((SQRT3 - 2) / 4) * _dly(o)   # update
        o = e + _dly(o)                                         # [1 0; 1 z^-1]
        return ((SQRT3 + 1) / SQRT2) * e, ((SQRT3 - 1) / SQRT2) * o
    raise ValueError(filt)


def lift_y(filt: str, u: np.ndarray, consts=None):
    """y-side (dual analysis matrix P^T(z^-1)) one level; returns (C, D)."""
    u = np.asarray(u)
    if filt == "legall53":
        e, o = u[..., 0::2] * 1.0, u[..., 1::2] * 1.0
        e = e + 0.5 * (o + _dly(o))            # [1 (1+z^-1)/2; 0 1]
        o = o - 0.25 * (e + _adv(e))           # [1 0; -(1+z)/4 1]
        return e, 2.0 * o                      # diag(1, 2)
    if filt == "cdf97":
        c = CDF97_TABLE_I if consts is None else consts
        e, o = u[..., 0::2] * 1.0, u[..., 1::2] * 1.0
        e = e - c["a"] * (o + _dly(o))
        o = o - c["b"] * (e + _adv(e))
        e = e - c["g"] * (o + _dly(o))
        o = o - c["d"] * (e + _adv(e))
        return e / c["x"], c["x"] * o
    if filt == "d4":
        return lift_x("d4", u)
    raise ValueError(filt)


def unlift_x(filt: str, A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Inverse of lift_x: the synthesis matrix P(z) (for 5/3 the matrix
    scaled by 2, Sec. III-C Case I; for D4 the causal synthesis of
    Sec. III-B, whose output is delayed by one pair)."""
    if filt == "legall53":
        e, o = A * 1.0, 2.0 * B
        e = e - 0.25 * (o + _dly(o))
        o = o + 0.5 * (e + _adv(e))
    elif filt == "cdf97":
        c = CDF97_TABLE_I
        e, o = A / c["x"], B * c["x"]
        e = e - c["d"] * (o + _dly(o))
        o = o - c["g"] * (e + _adv(e))
        e = e - c["b"] * (o + _dly(o))
        o = o - c["a"] * (e + _adv(e))
    elif filt == "d4":
        e1 = A * SQRT2 / (SQRT3 + 1)
        o2 = B * SQRT2 / (SQRT3 - 1)
        o1 = _adv(o2 - e1)          # undo [1 0; 1 z^-1]: o2[k] = e1[k] + o1[k-1]
        e = e1 - (SQRT3 / 4) * o1 - ((SQRT3 - 2) / 4) * _dly(o1)
        o = o1 + SQRT3 * e
        u = np.zeros(A.shape[:-1] + (2 * A.shape[-1],), dtype=np.result_type(e, o))
        u[..., 0::2] = e
        u[..., 1::2] = _adv(o)      # o[k] = u[2k-1]
        return u
    else:
        raise ValueError(filt)
    u = np.zeros(A.shape[:-1] + (2 * A.shape[-1],), dtype=np.result_type(e, o))
    u[..., 0::2] = e
    u[..., 1::2] = o
    return u


def unlift_y(filt: str, C: np.ndarray, D: np.ndarray) -> np.ndarray:
    """Inverse of lift_y (synthesis of one finer approximation from the
    y-side approximation and detail, the coarse-to-fine step of eq. (21)):
    the y-side steps undone in reverse order."""
    if filt == "legall53":
        e, o = C * 1.0, 0.5 * D
        o = o + 0.25 * (e + _adv(e))
        e = e - 0.5 * (o + _dly(o))
    elif filt == "cdf97":
        c = CDF97_TABLE_I
        e, o = C * c["x"], D / c["x"]
        o = o + c["d"] * (e + _adv(e))
        e = e + c["g"] * (o + _dly(o))
        o = o + c["b"] * (e + _adv(e))
        e = e + c["a"] * (o + _dly(o))
    elif filt == "d4":
        return unlift_x("d4", C, D)     # one matrix serves both sides (Sec. III-B)
    else:
        raise ValueError(filt)
    u = np.zeros(C.shape[:-1] + (2 * C.shape[-1],), dtype=np.result_type(e, o))
    u[..., 0::2] = e
    u[..., 1::2] = o
    return u


def synthesize_y(filt: str, details, cJ, to: int):
    """Coarse-to-fine formation (eq. (21) applied level by level): from the
    coarsest approximation c_J and the details d_J, ..., d_{to+1} (details[l-1]
    = d_l), the approximation c_to of the received pulse (c_0 = the zero
    padded pulse).  Integer filter: the reversible steps."""
    c = cJ
    for l in range(len(details), to, -1):
        if filt == "legall53_int":
            c = i2i_unlift_y(c, details[l - 1])
        else:
            c = unlift_y(filt, c, details[l - 1])
    return c


# ---------------------------------------------------------------------------
# DWT-domain (two-band, level j+1) form of eq. (15), float filters
# ---------------------------------------------------------------------------

def correlate_dwt(filt: str, J: int, ref, rx, chunk: int = 256) -> np.ndarray:
    """Plane j from level-(j+1) approximation and detail bands (eq. (15),
    eq. (20)), every shift computed separately.  Equal to correlate_direct
    in exact arithmetic; used as a cross-check."""
    _check_float(filt)
    ref = np.asarray(ref, dtype=np.complex128)
    rx = np.asarray(rx, dtype=np.complex128)
    N = transform_length(len(rx), J)
    x = zero_pad(ref, N)
    y = zero_pad(rx, N)
    xlo, xhi, ylo, yhi = TAPS[filt]
    out = np.zeros((J, N), dtype=np.complex128)
    for j in range(J):
        Cj = approximation(y, ylo, j)
        C1, D1 = analyze(Cj, ylo), analyze(Cj, yhi)
        for s0 in range(0, N, chunk):
            lags = np.arange(s0, min(N, s0 + chunk))
            X = np.stack([np.roll(x, int(s)) for s in lags])
            Aj = approximation(X, xlo, j)
            A1, B1 = analyze(Aj, xlo), analyze(Aj, xhi)
            out[j, lags] = np.conj(A1) @ C1 + np.conj(B1) @ D1
    return out


def correlate_swapped(filt: str, J: int, ref, rx, chunk: int = 256) -> np.ndarray:
    """Roles exchanged (Sec. I: the redundant transform may sit on either
    signal; eq. (20a) approximation form): the received signal gets the
    all-shift (redundant) y-side analysis and the reference only its critical
    x-side one.  Plane j, lag s: inner product (conjugate on the reference)
    of the level-j approximation of the reference with the level-j
    approximation of the received signal advanced by s, i.e. of
    roll(y, -s).  Plane 0 is the circular cross-correlation, as for
    correlate_direct; a shift of rx by t shifts every plane by exactly t;
    at lags that are multiples of 2^j plane j equals correlate_direct's.
    Returns complex128 [J, N]."""
    _check_float(filt)
    ref = np.asarray(ref, dtype=np.complex128)
    rx = np.asarray(rx, dtype=np.complex128)
    N = transform_length(len(rx), J)
    if len(ref) > N:
        raise ValueError("reference longer than the transform length")
    x = zero_pad(ref, N)
    y = zero_pad(rx, N)
    xlo, _, ylo, _ = TAPS[filt]
    out = np.zeros((J, N), dtype=np.complex128)
    for j in range(J):
        a = approximation(x, xlo, j)
        for s0 in range(0, N, chunk):
            lags = np.arange(s0, min(N, s0 + chunk))
            Y = np.stack([np.roll(y, -int(s)) for s in lags])
            out[j, lags] = approximation(Y, ylo, j) @ np.conj(a)
    return out


def correlate_swapped_at(filt: str, J: int, ref, rx, plane: int, lags) -> np.ndarray:
    """correlate_swapped's plane `plane` at the listed lags only (for
    sampled checks at sizes where every lag would be too slow)."""
    _check_float(filt)
    ref = np.asarray(ref, dtype=np.complex128)
    rx = np.asarray(rx, dtype=np.complex128)
    N = transform_length(len(rx), J)
    x = zero_pad(ref, N)
    y = zero_pad(rx, N)
    xlo, _, ylo, _ = TAPS[filt]
    a = approximation(x, xlo, plane)
    lags = np.asarray(lags, dtype=np.int64)
    Y = np.stack([np.roll(y, -int(s)) for s in lags]) if len(lags) else \
        np.zeros((0, N), np.complex128)
    return approximation(Y, ylo, plane) @ np.conj(a)


def detect_peaks(planes, rel: float, max_peaks: int):
    """Target declaration on the correlation magnitude (Sec. V-A, Fig. 6:
    |R| in dB at each scale, targets read off as peaks above a level): on
    each plane (last axis, circular lags) a lag s is a peak when its power
    p[s] = Re^2 + Im^2 exceeds p[s-1], is not below p[s+1] (the first
    sample of a flat top) and is not below rel * max(p).  The decisions use
    single precision with one rounding per operation (each square, the sum,
    rel times the maximum), the precision the planes are delivered in.
    Returns, per plane, (lags in increasing order, all of them; dB of each
    relative to the plane's maximum, float64)."""
    planes = np.asarray(planes)
    assert planes.dtype == np.complex64
    re = planes.real.astype(np.float32)
    im = planes.imag.astype(np.float32)
    p = re * re + im * im
    p2 = p.reshape(-1, p.shape[-1])
    out = []
    for row in p2:
        M = row.max()
        thr = np.float32(rel) * M
        peak = (row > np.roll(row, 1)) & (row >= np.roll(row, -1)) & (row >= thr)
        lags = np.nonzero(peak)[0]
        db = 10.0 * np.log10(row[lags].astype(np.float64) / np.float64(M)) if len(lags) else \
            np.zeros(0)
        out.append((lags, db))
    return out


# ---------------------------------------------------------------------------
# Integer-to-integer 5/3 (reversible lifting with floor shifts).
# The paper cites reversible integer lifting but prints no rounding rule;
# the reading used here:
#   x-side:  o -= (e[k] + e[k+1]) >> 1 ;  e += (o[k-1] + o[k] + 2) >> 2
#   y-side:  e += (o[k-1] + o[k] + 1) >> 1 ;  o -= (e[k] + e[k+1] + 2) >> 2
# (">>" is an arithmetic shift, i.e. floor division by a power of two).
# The detail scalings 1/2 (x-side) and 2 (y-side) cancel in the product
# B*D and are dropped.  I and Q are lifted independently (Sec. IV).
# ---------------------------------------------------------------------------

def i2i_lift_x(u: np.ndarray):
    u = np.asarray(u, dtype=np.int64)
    e, o = u[..., 0::2].copy(), u[..., 1::2].copy()
    o = o - ((e + _adv(e)) >> 1)
    e = e + ((_dly(o) + o + 2) >> 2)
    return e, o


def i2i_lift_y(u: np.ndarray):
    u = np.asarray(u, dtype=np.int64)
    e, o = u[..., 0::2].copy(), u[..., 1::2].copy()
    e = e + ((_dly(o) + o + 1) >> 1)
    o = o - ((e + _adv(e) + 2) >> 2)
    return e, o


def i2i_unlift_x(A, B):
    """Exact inverse of i2i_lift_x (reversibility)."""
    e, o = np.asarray(A, np.int64).copy(), np.asarray(B, np.int64).copy()
    e = e - ((_dly(o) + o + 2) >> 2)
    o = o + ((e + _adv(e)) >> 1)
    u = np.zeros(e.shape[:-1] + (2 * e.shape[-1],), np.int64)
    u[..., 0::2] = e
    u[..., 1::2] = o
    return u


def i2i_unlift_y(C, D):
    e, o = np.asarray(C, np.int64).copy(), np.asarray(D, np.int64).copy()
    o = o + ((e + _adv(e) + 2) >> 2)
    e = e - ((_dly(o) + o + 1) >> 1)
    u = np.zeros(e.shape[:-1] + (2 * e.shape[-1],), np.int64)
    u[..., 0::2] = e
    u[..., 1::2] = o
    return u


def _i2i_complex(lift, re, im):
    a_re, b_re = lift(re)
    a_im, b_im = lift(im)
    return (a_re, a_im), (b_re, b_im)


def i2i_bands_y(rx_re, rx_im, level):
    """Received-signal bands (C_level, D_level) as (re, im) int64 pairs."""
    c_re, c_im = np.asarray(rx_re, np.int64), np.asarray(rx_im, np.int64)
    for _ in range(level - 1):
        (c_re, c_im), _ = _i2i_complex(i2i_lift_y, c_re, c_im)
    return _i2i_complex(i2i_lift_y, c_re, c_im)


def i2i_bands_x(x_re, x_im, level):
    a_re, a_im = np.asarray(x_re, np.int64), np.asarray(x_im, np.int64)
    for _ in range(level - 1):
        (a_re, a_im), _ = _i2i_complex(i2i_lift_x, a_re, a_im)
    return _i2i_complex(i2i_lift_x, a_re, a_im)


def _conj_dot_int(a, c):
    """sum conj(a) * c for int64 (re, im) pairs; rows of `a` against `c`."""
    a_re, a_im = a
    c_re, c_im = c
    re = a_re @ c_re + a_im @ c_im
    im = a_re @ c_im - a_im @ c_re
    return re, im


def correlate_int_at(J: int, ref_iq, rx_iq, plane: int, lags) -> np.ndarray:
    """Integer plane values at the listed lags; ref_iq, rx_iq are int arrays
    of shape [len, 2] (I, Q).  Returns int64 [len(lags), 2]."""
    ref_iq = np.asarray(ref_iq, np.int64)
    rx_iq = np.asarray(rx_iq, np.int64)
    N = transform_length(rx_iq.shape[0], J)
    if ref_iq.shape[0] > N:
        raise ValueError("reference longer than the transform length")
    x_re, x_im = zero_pad(ref_iq[:, 0], N), zero_pad(ref_iq[:, 1], N)
    y_re, y_im = zero_pad(rx_iq[:, 0], N), zero_pad(rx_iq[:, 1], N)
    lvl = plane + 1
    C, D = i2i_bands_y(y_re, y_im, lvl)
    lags = np.asarray(lags, np.int64)
    X_re = np.stack([np.roll(x_re, int(s)) for s in lags])
    X_im = np.stack([np.roll(x_im, int(s)) for s in lags])
    A, B = i2i_bands_x(X_re, X_im, lvl)
    re1, im1 = _conj_dot_int(A, C)
    re2, im2 = _conj_dot_int(B, D)
    return np.stack([re1 + re2, im1 + im2], axis=-1)


def correlate_int(J: int, ref_iq, rx_iq, chunk: int = 256) -> np.ndarray:
    """All planes, all lags; int64 [J, N, 2]."""
    N = transform_length(np.asarray(rx_iq).shape[0], J)
    out = np.zeros((J, N, 2), np.int64)
    for j in range(J):
        for s0 in range(0, N, chunk):
            lags = np.arange(s0, min(N, s0 + chunk))
            out[j, lags] = correlate_int_at(J, ref_iq, rx_iq, j, lags)
    return out


# ---------------------------------------------------------------------------
# Reference phase coefficients (used to check the plan's stored pyramid).
# A_l^(r) is the level-l x-side approximation of the reference delayed by r
# (Sec. II: shift-circulant vectors; Sec. IV Fig. 5: the even/odd tree).
# ---------------------------------------------------------------------------

def reference_phase(filt: str, ref, N: int, level: int, r: int):
    """(A_level^(r), B_level^(r)) of the zero-padded reference delayed by r,
    each of length N / 2^level, computed directly (no tree)."""
    if filt in FLOAT_FILTERS:
        xlo, xhi, _, _ = TAPS[filt]
        x = np.roll(zero_pad(np.asarray(ref, np.complex128), N), r)
        a = approximation(x, xlo, level - 1)
        return analyze(a, xlo), analyze(a, xhi)
    ref = np.asarray(ref, np.int64)
    x_re = np.roll(zero_pad(ref[:, 0], N), r)
    x_im = np.roll(zero_pad(ref[:, 1], N), r)
    (a_re, a_im), (b_re, b_im) = i2i_bands_x(x_re, x_im, level)
    return a_re + 1j * a_im, b_re + 1j * b_im


def correlate(filt: str, J: int, ref, rx):
    """Dispatch: float filters -> complex128 [J, N]; the integer filter ->
    int64 [J, N, 2] (ref and rx as int [len, 2] I/Q arrays)."""
    if filt in FLOAT_FILTERS:
        return correlate_direct(filt, J, ref, rx)
    if filt in INT_FILTERS:
        return correlate_int(J, ref, rx)
    raise ValueError(filt)
