"""Build libsidwt.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libsidwt.so")
SOURCES = ["sidwt_kernels.hip", "sidwt_bank.hip", "sidwt_synth.hip", "sidwt_swap.hip", "sidwt_detect.hip",
           "sidwt_generic.hip", "sidwt_int8.hip", "sidwt_noalloc.hip", "sidwt_api.cpp", "sidwt_factor.cpp",
           "sidwt_batch.cpp", "sidwt_bank.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # packed FP32 VALU forms are kept out of the generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function",
    ]


def build(verbose: bool = False, jobs: int = 0) -> str:
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(os.path.join(PKG, "_build"), exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(PKG, "_build", src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        cmds.append([hipcc()] + flags() + lang + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    jobs = jobs or max(1, min(len(cmds), len(os.sched_getaffinity(0)), 8))
    with ThreadPoolExecutor(jobs) as pool:
        for r in pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds):
            err = "\n".join(l for l in r.stderr.splitlines()
                            if "packed-fp32-ops" not in l)
            if err.strip():
                print(err, file=sys.stderr, flush=True)
            if r.returncode != 0:
                raise subprocess.CalledProcessError(r.returncode, r.args)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
