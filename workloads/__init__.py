"""Seeded synthetic radar workloads (inputs only; none of the method's
arithmetic lives here).

Both the HIP library's tests/benchmark and the CPU oracle draw their inputs
from this module.  Every pulse is generated from its own generator seeded by
(seed, pulse index), so one pulse of a large batch can be rebuilt alone.

Waveforms follow the paper's radar model: the LFM chirp of eq. (18) sampled
at its bandwidth over the pulse, and target backscatter as a sum of delayed,
complex-scaled copies of the transmitted pulse (Sec. V-A), plus circular
complex Gaussian noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

BARKER13 = np.array([1, 1, 1, 1, 1, -1, -1, 1, 1, -1, 1, -1, 1], dtype=np.float64)

FILTER_IDS = {"legall53": 1, "cdf97": 2, "d4": 3, "legall53_int": 4}


def lfm_chirp(m: int, tbp: float) -> np.ndarray:
    """exp(i pi K t^2) over |t| <= Tp/2, sampled at the bandwidth B = K Tp:
    with t = (n - (m-1)/2) / B and K = B / Tp the phase is
    pi * tbp * ((n - (m-1)/2) / m)^2 for m samples."""
    n = np.arange(m, dtype=np.float64)
    return np.exp(1j * math.pi * tbp * ((n - (m - 1) / 2) / m) ** 2)


def barker13_code(m: int) -> np.ndarray:
    """Barker-13 phase code, each chip held c = max(1, m // 52) samples, the
    13c block repeated to m samples."""
    c = max(1, m // 52)
    block = np.repeat(BARKER13, c)
    reps = -(-m // len(block))
    return np.tile(block, reps)[:m].astype(np.complex128)


def polyphase_code(m: int, rng: np.random.Generator) -> np.ndarray:
    """Random unit-modulus polyphase code."""
    return np.exp(2j * math.pi * rng.random(m))


def noise(n: int, sigma2: float, rng: np.random.Generator) -> np.ndarray:
    s = math.sqrt(sigma2 / 2.0)
    return s * (rng.standard_normal(n) + 1j * rng.standard_normal(n))


def echoes(n: int, ref: np.ndarray, rng: np.random.Generator, k_max: int = 3,
           snr_db_range=(-5.0, 20.0)) -> np.ndarray:
    """1..k_max copies of `ref` at uniform delays inside the pulse, complex
    amplitude |a| ~ U[0.5, 1], arg a ~ U[0, 2 pi), plus noise at an SNR
    (per sample, relative to a unit echo) ~ U[snr_db_range]."""
    m = len(ref)
    y = np.zeros(n, np.complex128)
    k = int(rng.integers(1, k_max + 1))
    for _ in range(k):
        d = int(rng.integers(0, max(1, n - m + 1)))
        a = rng.uniform(0.5, 1.0) * np.exp(2j * math.pi * rng.random())
        seg = min(m, n - d)
        y[d:d + seg] += a * ref[:seg]
    snr = rng.uniform(*snr_db_range)
    y += noise(n, 10.0 ** (-snr / 10.0), rng)
    return y


def _rng(seed: int, i: int) -> np.random.Generator:
    return np.random.default_rng([seed, i])


# ---------------------------------------------------------------------------
# Workload 1: one correlation, 5/3, J = 3
# ---------------------------------------------------------------------------

@dataclass
class Single:
    filter: str
    J: int
    ref: np.ndarray
    rx: np.ndarray
    delay: int


def single_chirp(seed: int = 1, n: int = 1024, m: int = 256, tbp: float = 64.0,
                 snr_db: float = 10.0, J: int = 3) -> Single:
    """1024-sample pulse holding a 256-sample chirp (time-bandwidth 64) at a
    seed-chosen delay, complex Gaussian noise at 10 dB SNR; LeGall 5/3, J=3."""
    rng = _rng(seed, 0)
    ref = lfm_chirp(m, tbp)
    d = int(rng.integers(0, n - m + 1))
    y = np.zeros(n, np.complex128)
    y[d:d + m] = ref
    y += noise(n, 10.0 ** (-snr_db / 10.0), rng)
    return Single("legall53", J, ref, y, d)


# ---------------------------------------------------------------------------
# Workload 2: batched uniform, CDF 9/7, J = 5
# ---------------------------------------------------------------------------

@dataclass
class Batch:
    filter: str
    J: int
    ref: np.ndarray
    rx: np.ndarray  # [count, n]
    n: int


def batched_uniform_pulse(seed: int, i: int, n: int = 8192, m: int = 512) -> np.ndarray:
    ref = lfm_chirp(m, m / 4)
    return echoes(n, ref, _rng(seed, i))


def batched_uniform(seed: int = 2, count: int = 4096, n: int = 8192, m: int = 512,
                    J: int = 5, dtype=np.complex64) -> Batch:
    """count x n pulses, each 1-3 echoes of a 512-sample chirp (TBP = m/4)."""
    ref = lfm_chirp(m, m / 4)
    rx = np.empty((count, n), dtype)
    for i in range(count):
        rx[i] = echoes(n, ref, _rng(seed, i))
    return Batch("cdf97", J, ref, rx, n)


# ---------------------------------------------------------------------------
# Multi-target scene (Sec. V-A, Fig. 6 analogue): P point targets, CDF 9/7
# ---------------------------------------------------------------------------

@dataclass
class Scene:
    filter: str
    J: int
    ref: np.ndarray
    rx: np.ndarray      # [count, n]
    delays: np.ndarray  # [count, P]
    refl: np.ndarray    # [count, P] complex reflectivities


def multi_target(seed: int = 5, count: int = 1, n: int = 1024, m: int = 160, P: int = 5,
                 J: int = 3, snr_db: float = 20.0, dtype=np.complex64) -> Scene:
    """Backscatter of P point targets: y[n] = sum_k s_k x[n - d_k] plus noise,
    x a chirp of time-bandwidth product 160 sampled at its bandwidth (m =
    160 samples).  Four targets sit close together (gaps of 3..12 samples)
    and one about 60..100 samples earlier, as in the paper's scene; |s_k| ~
    U[0.5, 1], arg s_k ~ U[0, 2 pi); SNR per sample relative to a unit
    echo."""
    ref = lfm_chirp(m, float(m))
    rx = np.empty((count, n), dtype)
    delays = np.empty((count, P), np.int64)
    refl = np.empty((count, P), np.complex128)
    for i in range(count):
        rng = _rng(seed, i)
        base = int(rng.integers(n // 4, n - m - 60))
        d = [base]
        for _ in range(P - 2):
            d.append(d[-1] + int(rng.integers(3, 13)))
        d.insert(0, base - int(rng.integers(60, 101)))
        y = np.zeros(n, np.complex128)
        s = rng.uniform(0.5, 1.0, P) * np.exp(2j * math.pi * rng.random(P))
        for dk, sk in zip(d, s):
            seg = min(m, n - dk)
            y[dk:dk + seg] += sk * ref[:seg]
        y += noise(n, 10.0 ** (-snr_db / 10.0), rng)
        rx[i] = y
        delays[i] = d
        refl[i] = s
    return Scene("cdf97", J, ref, rx, delays, refl)


# ---------------------------------------------------------------------------
# Workload 3: integer path, int16 I/Q, reversible 5/3, J = 6
# ---------------------------------------------------------------------------

@dataclass
class IntBatch:
    J: int
    ref_iq: np.ndarray  # int16 [m, 2]
    rx_iq: np.ndarray   # int16 [count, n, 2]
    n: int


def adc12(v: np.ndarray, gain: float) -> np.ndarray:
    """12-bit ADC: rint(v * gain) clipped to [-2048, 2047], I and Q."""
    iq = np.stack([np.rint(v.real * gain), np.rint(v.imag * gain)], axis=-1)
    return np.clip(iq, -2048, 2047).astype(np.int16)


def int_reference(m: int = 512) -> np.ndarray:
    return adc12(lfm_chirp(m, m / 4), 2047.0)


def int_pulse(seed: int, i: int, n: int = 4096, m: int = 512) -> np.ndarray:
    return adc12(echoes(n, lfm_chirp(m, m / 4), _rng(seed, i)), 512.0)


def integer_batch(seed: int = 3, count: int = 16384, n: int = 4096, m: int = 512,
                  J: int = 6) -> IntBatch:
    rx = np.empty((count, n, 2), np.int16)
    for i in range(count):
        rx[i] = int_pulse(seed, i, n, m)
    return IntBatch(J, int_reference(m), rx, n)


# ---------------------------------------------------------------------------
# Workloads 4/5: uneven lengths, 16 mixed references (or a bank of 64)
# ---------------------------------------------------------------------------

def reference_set(seed: int, count: int = 16, m_lo: int = 64, m_hi: int = 2048):
    """References with log-uniform lengths: in proportion 6:5:5 LFM chirps
    (TBP = m/4), Barker-13 repeated phase codes, random polyphase codes.
    Returned sorted by length."""
    rng = _rng(seed, 10 ** 6)
    n_lfm = round(count * 6 / 16)
    n_bar = round(count * 5 / 16)
    kinds = ["lfm"] * n_lfm + ["barker"] * n_bar + ["poly"] * (count - n_lfm - n_bar)
    refs = []
    for kind in kinds:
        m = int(math.floor(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        if kind == "lfm":
            refs.append(lfm_chirp(m, m / 4))
        elif kind == "barker":
            refs.append(barker13_code(m))
        else:
            refs.append(polyphase_code(m, rng))
    refs.sort(key=len)
    return refs


def uneven_length(rng: np.random.Generator, n_lo: int = 512, n_hi: int = 65536) -> int:
    return int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))


def levels_for(n: int) -> int:
    """J = floor(log2(n / 16))."""
    return int(math.floor(math.log2(n / 16)))


@dataclass
class UnevenRequest:
    n: int
    J: int
    filter: str
    ref_index: int
    rx: np.ndarray = field(repr=False)


def uneven_request(seed: int, i: int, refs) -> UnevenRequest:
    rng = _rng(seed, i)
    n = uneven_length(rng)
    J = levels_for(n)
    filt = "d4" if rng.random() < 0.5 else "cdf97"
    eligible = [k for k, r in enumerate(refs) if len(r) <= n // 2]
    k = eligible[int(rng.integers(0, len(eligible)))]
    rx = echoes(n, refs[k], rng)
    return UnevenRequest(n, J, filt, k, rx)


def uneven_batch(seed: int = 4, count: int = 10000, n_refs: int = 16):
    refs = reference_set(seed, n_refs)
    reqs = [uneven_request(seed, i, refs) for i in range(count)]
    return refs, reqs


def poisson_arrivals(seed: int, rate_hz: float, count: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process."""
    rng = _rng(seed, 2 * 10 ** 6)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=count))
