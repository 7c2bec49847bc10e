"""CPU check of the uneven batch's multi-level lifting blocks (the
library's own geometry code): for every pass of a sweep of transform
lengths, scale counts and depths, the blocks' own outputs tile every level
exactly once; every input pair an owned output's lifting window reads lies
inside the block's range of the level above (with the filters' actual reach,
also measured here on the oracle's lifting); the levels kept in LDS fit the
two buffers the pass is given; and the kernel's clamped circular read index
equals the true one for every needed sample."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import sidwt_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILTERS = ("legall53", "cdf97", "d4")


@pytest.fixture(scope="module")
def geometry():
    cxx = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not cxx:
        pytest.skip("hipcc not available")
    exe = os.path.join(str(pytest.importorskip("tempfile").mkdtemp()), "lift_blocks")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "cpp", "lift_blocks.cpp"), "-o", exe],
                   check=True, capture_output=True)
    cases = []
    for J in (5, 6, 8, 10, 12):
        for k in (1, 2, 3, 5, 17, 64):
            N = (1 << J) * k
            if N < 512 or N > (1 << 17):
                continue
            for D in (1, 2, 3, 4, 6):
                cases.append((N, J, D))
    cases += [(65536, 12, 4), (40960, 11, 3), (8704, 9, 4), (4352, 8, 4)]
    inp = "\n".join(f"{N} {J} {D}" for N, J, D in cases)
    r = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
    lines = r.stdout.splitlines()
    v = [int(x) for x in lines[0].split()[1:]]
    reach = {"legall53": tuple(v[0:3]), "cdf97": tuple(v[3:6]), "d4": tuple(v[6:9])}
    passes = []
    for ln in lines[1:]:
        f = ln.split()
        if f[0] == "pass":
            N, l0, l1, nb, lds, whole = map(int, f[1:])
            passes.append({"N": N, "l0": l0, "l1": l1, "nb": nb, "lds": lds, "whole": whole,
                           "blocks": []})
        else:
            vals = list(map(int, f[2:]))
            rng = {}
            p = passes[-1]
            for i, l in enumerate(range(p["l0"] - 1, p["l1"] + 1)):
                rng[l] = tuple(vals[4 * i:4 * i + 4])
            p["blocks"].append(rng)
    return reach, passes


def measured_reach(filt):
    """(pairs before, pairs after) that output pair k of one level of the
    oracle's y-side lifting depends on."""
    N = 64
    lo, hi = 0, 0
    base = np.zeros(N)
    c0, d0 = O.lift_y(filt, base.astype(complex))
    for q in range(N):
        u = base.copy()
        u[q] = 1.0
        c, d = O.lift_y(filt, u.astype(complex))
        k = 10
        if abs(c[k] - c0[k]) > 0 or abs(d[k] - d0[k]) > 0:
            pair = q // 2
            lo = max(lo, k - pair)
            hi = max(hi, pair - k)
    return lo, hi


@pytest.mark.parametrize("filt", FILTERS)
def test_library_reach_covers_the_lifting(geometry, filt):
    reach, _ = geometry
    HL, HR, _ob = reach[filt]
    lo, hi = measured_reach(filt)
    assert lo <= HL + (1 if _ob else 0) and hi <= HR


@pytest.mark.parametrize("filt", FILTERS)
def test_blocks_tile_levels_and_read_inside_their_ranges(geometry, filt):
    reach, passes = geometry
    HL, HR, OB = reach[filt]
    OWN = 64 - HL - HR
    assert passes
    for p in passes:
        N, l0, l1 = p["N"], p["l0"], p["l1"]
        buf0, buf1 = None, None
        for l in range(l0, l1 + 1):
            covered = np.zeros(N >> l, np.int64)
            for rng in p["blocks"]:
                os_, oe = rng[l][2], rng[l][3]
                covered[os_:oe] += 1
            assert np.all(covered == 1), (p["N"], l0, l1, l)
        for rng in p["blocks"]:
            # level l0 is lifted from global memory; levels l0 .. l1 - 1
            # are kept in LDS, level l in buffer (l - l0) & 1, whose sizes
            # are those of levels l0 and l0 + 1
            if l1 > l0:
                R0 = rng[l0][1] - rng[l0][0]
                R1 = rng[l0 + 1][1] - rng[l0 + 1][0]
                assert R0 + R1 <= p["lds"]
            else:
                assert p["lds"] == 0
            for l in range(l0, l1 + 1):
                s, e, os_, oe = rng[l]
                S, E = rng[l - 1][0], rng[l - 1][1]
                R, Nin = E - S, N >> (l - 1)
                if l < l1:
                    assert e - s <= (R0 if (l - l0) % 2 == 0 else R1)
                assert s <= os_ and oe <= e
                # every output of [s, e) reads pairs k - HL .. k + HR
                ks = np.arange(s, e)
                pairs = (ks[:, None] + np.arange(-HL, HR + 1)[None, :]).ravel()
                q = np.concatenate([2 * pairs, 2 * pairs - 1 if OB else 2 * pairs + 1])
                if p["whole"]:
                    # the whole circular level is in LDS: reads wrap
                    assert S == 0 and R == Nin
                else:
                    assert q.min() >= S and q.max() < E, (N, l0, l1, l, q.min(), q.max(), S, E)
                # the kernel's clamped circular index equals the position of q
                idx = np.minimum(np.mod(q - S, Nin), R - 1)
                assert np.all(np.mod(S + idx, Nin) == np.mod(q, Nin))
