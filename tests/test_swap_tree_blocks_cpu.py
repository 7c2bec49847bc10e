"""CPU check of the roles-exchanged tree's block order (the library's own
mapping): every (pulse, child phase) of a level is taken by exactly one
block, and in every whole group of 16 blocks, blocks x and x + 8 (which the
hardware hands to the same XCD one after the other) are the two children of
one parent phase of one pulse."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mapping():
    cxx = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else shutil.which("hipcc")
    if not cxx:
        pytest.skip("hipcc not available")
    exe = os.path.join(tempfile.mkdtemp(), "swap_tree_blocks")
    subprocess.run([cxx, "-O1", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "cpp", "swap_tree_blocks.cpp"), "-o", exe],
                   check=True, capture_output=True)
    cases = [(c, j) for c in (1, 2, 3, 5, 8, 13, 64) for j in range(1, 7)]
    inp = "\n".join(f"{c} {j}" for c, j in cases)
    r = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
    grids = {}
    for ln in r.stdout.splitlines():
        f = ln.split()
        if f[0] == "grid":
            cur = grids.setdefault((int(f[1]), int(f[2])), [])
        else:
            cur.append(tuple(map(int, f)))
    assert set(grids) == set(cases)
    return grids


def test_every_child_phase_once(mapping):
    for (count, j), rows in mapping.items():
        got = sorted((pulse, p) for _, pulse, p in rows)
        assert got == [(q, p) for q in range(count) for p in range(1 << j)], (count, j)


def test_same_xcd_blocks_share_a_parent(mapping):
    for (count, j), rows in mapping.items():
        G = count << j
        half = 1 << (j - 1)
        for x in range(0, G - G % 16, 16):
            for i in range(8):
                _, pa, a = rows[x + i]
                _, pb, b = rows[x + i + 8]
                assert pa == pb and a % half == b % half and a // half == 0 and b // half == 1, \
                    (count, j, x + i)
