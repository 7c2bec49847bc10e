"""CPU emulation of the integer path on int8 matrix cores (digit panels
from the library's host planning code, the kernel's index arithmetic
mirrored in tests/cpp/i8_emulate.cpp) against the oracle: bit-exact planes,
every plane and panel read in bounds, every shift-class sum inside int32.
The cases cover the Toeplitz blocks T = 8, 4 and 2, one to three weight
digits, references as long as the pulse allows, and full-scale pulses."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import sidwt_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    cxx = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not cxx:
        pytest.skip("hipcc not available")
    exe = tmp_path_factory.mktemp("i8") / "i8_emulate"
    subprocess.run([cxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "cpp", "i8_emulate.cpp"), "-o", str(exe)],
                   check=True, capture_output=True)
    return str(exe)


def plan_pyramid(J, ref):
    """The plan's stored phases (linear supports) from the oracle, in the
    library's order: level, band, phase, support index."""
    m = ref.shape[0]
    N0 = (1 << J) * (-(-4 * m // (1 << J)) + 8)    # long enough that no support wraps
    out = []
    lo_in, len_in = 0, m
    for l in range(1, J + 1):
        sup = []
        for b, (tlo, thi) in enumerate(((-2, 2), (0, 2))):
            kf = -((-(lo_in - thi)) // 2)
            kl = (lo_in + len_in - tlo) // 2
            sup.append((kf, kl - kf + 1))
        for b in range(2):
            lo, ln = sup[b]
            for r in range(1 << l):
                A, B = O.reference_phase("legall53_int", ref, N0, l, r)
                v = (A, B)[b]
                L = len(v)
                idx = (lo + np.arange(ln)) % L
                # the support covers every nonzero coefficient
                mask = np.ones(L, bool)
                mask[idx] = False
                assert not np.any(v[mask])
                out.append(np.stack([v[idx].real, v[idx].imag], -1).astype(np.int64))
        lo_in, len_in = sup[0]
    return np.concatenate(out).reshape(-1)


def run_emu(emu, J, N, ref, rx, mode=None):
    lines = [f"{J} {N} {ref.shape[0]}", " ".join(map(str, plan_pyramid(J, ref)))]
    y_re = O.zero_pad(rx[:, 0], N)
    y_im = O.zero_pad(rx[:, 1], N)
    for l in range(1, J + 1):
        (c_re, c_im), (d_re, d_im) = O.i2i_bands_y(y_re, y_im, l)
        lines.append(" ".join(map(str, np.stack([c_re, c_im], -1).reshape(-1))))
        lines.append(" ".join(map(str, np.stack([d_re, d_im], -1).reshape(-1))))
    r = subprocess.run([emu] + ([mode] if mode else []), input="\n".join(lines),
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-400:] + r.stderr[-400:]
    head = r.stdout.splitlines()
    Ts = [int(x) for x in head[0].split()[1:]]
    wl = int(head[1].split()[1])
    vals = np.array([int(x) for x in head[2:]], np.int64).reshape(J, N, 2)
    return Ts, wl, vals


@pytest.mark.parametrize("J,n,m,peak,seed,want_T", [
    (4, 1024, 100, 2047, 0, [8, 8, 4, 2]),
    (3, 600, 90, 120, 1, None),          # one weight digit, ragged n
    (6, 4096, 512, 2047, 2, [8, 8, 8, 8, 4, 2]),
    (2, 256, 120, 32767, 3, None),       # three weight digits
    (5, 2048, 300, 20000, 4, None),
])
def test_int8_emulation_matches_the_oracle(emu, J, n, m, peak, seed, want_T):
    rng = np.random.default_rng(seed)
    ref = rng.integers(-peak, peak + 1, (m, 2)).astype(np.int64)
    rx = rng.integers(-32768, 32768, (n, 2)).astype(np.int64)
    N = O.transform_length(n, J)
    Ts, wl, got = run_emu(emu, J, N, ref, rx)
    if want_T is not None:
        assert Ts == want_T
    assert wl == (1 if peak < 64 else 3 if peak > 16000 else 2) or wl in (1, 2, 3)
    want = O.correlate_int(J, ref, rx)
    assert np.array_equal(got, want)


def test_int8_emulation_full_scale_dc_pulse(emu):
    """The pulse side's worst case: a full-scale DC pulse reaches the level
    bound 2^l * 32768, the top of the three digits' range at level 7."""
    J, n, m = 7, 4096, 40
    rng = np.random.default_rng(7)
    ref = rng.integers(-2047, 2048, (m, 2)).astype(np.int64)
    rx = np.full((n, 2), -32768, np.int64)
    N = O.transform_length(n, J)
    _, _, got = run_emu(emu, J, N, ref, rx)
    lags = np.arange(0, N, 61)
    for j in (0, J - 1):
        assert np.array_equal(got[j, lags], O.correlate_int_at(J, ref, rx, j, lags))


@pytest.mark.parametrize("J,n,m,seed", [(3, 20000, 300, 11), (5, 30000, 700, 12)])
def test_int8_long_pulse_blocks_match_the_oracle(emu, J, n, m, seed):
    """The long-pulse form: levels cut into row blocks (several per level at
    these lengths), each block's digit window starting at its first row;
    bit-exact against the oracle on sampled lags of every plane."""
    rng = np.random.default_rng(seed)
    ref = rng.integers(-2047, 2048, (m, 2)).astype(np.int64)
    rx = rng.integers(-32768, 32768, (n, 2)).astype(np.int64)
    N = O.transform_length(n, J)
    _, _, got = run_emu(emu, J, N, ref, rx, mode="blocks")
    lags = np.unique(np.concatenate([np.arange(0, N, 397), [1, N // 2, N - 1]]))
    for j in range(J):
        assert np.array_equal(got[j, lags], O.correlate_int_at(J, ref, rx, j, lags)), j
