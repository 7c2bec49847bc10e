#!/usr/bin/env python
"""Benchmark: complex samples/s through the J-scale SIDWT correlate.

Default workload (one "step" = one pass of the whole path over one batch):
4096 pulses x 8192 complex64 samples, each holding 1-3 echoes of a
512-sample LFM chirp (time-bandwidth 128) at random delays and complex
amplitudes, noise SNR uniform in [-5, 20] dB; CDF 9/7 lifting, J = 5 scales;
one fused launch (lifting + per-scale correlation against the stored
shift-circulant phases) per step.  Inputs are resident in HBM before timing.

Prints one JSON line.  Also reported: the roofline of the dominant kernel
(FP32 MFMA contraction), the lifting-only kernel's HBM roofline, and the CPU
oracle timed on the host's cores over a bounded sample of pulses.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MATRIX_TFLOPS = 157.3   # MI355X dense FP32 matrix
PEAK_HBM_GBS = 8000.0             # MI355X HBM3E


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, as it stands, one pulse per worker process.
# ---------------------------------------------------------------------------

def _oracle_pulse(args):
    filt, J, ref, rx = args
    import oracle
    t0 = time.perf_counter()
    oracle.correlate_direct(filt, J, ref, rx)
    return time.perf_counter() - t0


def _warm(_):
    import oracle  # noqa: F401
    return os.getpid()


def cpu_baseline(filt, J, ref, pulses, max_workers=32):
    import multiprocessing as mp
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, max_workers, len(pulses)))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_warm, range(workers))
        t0 = time.perf_counter()
        pool.map(_oracle_pulse, [(filt, J, ref, p) for p in pulses[:workers]])
        wall = time.perf_counter() - t0
    n = pulses.shape[1]
    return {"value": workers * n / wall, "unit": "complex samples/s", "cores": workers,
            "kind": "oracle",
            "sample": f"{workers} pulses x {n} samples of the same batch, one pulse per process "
                      f"(FP64 NumPy, OMP_NUM_THREADS=1), wall {wall:.1f} s; host has {cores} cores"}


# ---------------------------------------------------------------------------

def algorithmic_flops_per_pulse(S, plan, N):
    """8 real flops per complex MAC of the block-circulant products
    (eq. (20)/(20a)): every lag of plane j = l-1 takes the stored support of
    its phase in both bands of level l."""
    total = 0
    for lvl in range(1, plan.J + 1):
        for band in (0, 1):
            import ctypes
            lo, ln = ctypes.c_int32(), ctypes.c_int32()
            S._lib.check(S._lib.lib().sidwt_plan_phase(plan.handle, lvl, band, 0, ctypes.byref(lo),
                                                       ctypes.byref(ln), None))
            total += 8 * N * ln.value
    return total


PROFILE = os.path.join(ROOT, "profiles", "fused_correlate_cdf97_4096x8192_J5.md")
KERNEL_SOURCES = ["sidwt_kernels.hip", "sidwt_device.hpp", "sidwt_host.hpp"]


def profiled_traffic():
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    counter summary, or None if the kernel sources changed since."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_cs_0607001_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    if h.hexdigest()[:16] not in text:
        return None
    for line in text.splitlines():
        if line.startswith("traffic_bytes_per_launch:"):
            return int(line.split(":")[1])
    return None


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--cpu-baseline", dest="cpu", action="store_true", default=True)
    ap.add_argument("--no-cpu-baseline", dest="cpu", action="store_false")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run an elementwise kernel that reads and writes 256 MiB "
                         "(calibrates the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(pulses are independent; see DESIGN.md for how the work would shard).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_cs_0607001_amd as S
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    J, m = 5, 512
    log(f"generating {args.count} x {args.n} pulses")
    b = W.batched_uniform(seed=2, count=args.count, n=args.n, m=m, J=J)
    N = S.transform_length(args.n, J)
    rx = torch.from_numpy(b.rx).to(dev)
    plan = S.plan_create(b.filter, J, b.ref)
    out = torch.empty((args.count, J, N), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()

    # Sanity check of one pulse on sampled lags before timing anything.
    S.correlate_many(plan, rx, out=out)
    torch.cuda.synchronize()
    import oracle
    probe = np.array([0, 1, 7, 511, 4097, N - 1])
    for j in range(J):
        want = oracle.correlate_at(b.filter, J, b.ref, b.rx[3].astype(np.complex128), j, probe)
        got = out[3, j, probe].cpu().numpy()
        err = np.abs(got - want).max() / max(np.abs(want).max(), 1e-30)
        assert err < 1e-4, f"bench sanity check failed: plane {j} err {err}"
    log("sanity check vs oracle ok")

    for _ in range(args.warmup):
        S.correlate_many(plan, rx, out=out)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        S.correlate_many(plan, rx, out=out)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    samples = args.count * args.n
    value = samples / (ms_step * 1e-3)
    flops = algorithmic_flops_per_pulse(S, plan, N) * args.count
    achieved_tflops = flops / (ms_step * 1e-3) / 1e12
    log(f"fused: {ms_step:.3f} ms/step, {value / 1e9:.2f} G samples/s, "
        f"{achieved_tflops:.1f} TFLOP/s (wall {wall:.2f} s)")

    # Lifting-only kernel (a1 + a2), HBM roofline: 8 B in + 8 B out per sample.
    pyr = torch.empty((args.count, N), dtype=torch.complex64, device=dev)
    for _ in range(3):
        S.lift_many(b.filter, J, rx, pyr=pyr)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lift_reps = 20
    for _ in range(lift_reps):
        S.lift_many(b.filter, J, rx, pyr=pyr)
    e1.record(stream)
    torch.cuda.synchronize()
    lift_ms = e0.elapsed_time(e1) / lift_reps
    lift_bytes = args.count * (args.n * 8 + N * 8)
    lift_gbs = lift_bytes / (lift_ms * 1e-3) / 1e9
    log(f"lifting only: {lift_ms * 1e3:.1f} us, {lift_gbs:.0f} GB/s")

    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log("copy probe: 3 x elementwise kernels reading and writing 256 MiB each")
        del src, dst

    cpu = None
    if args.cpu:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(b.filter, J, b.ref, b.rx[: 64].astype(np.complex128))

    rec = {
        "metric": "complex samples/sec through J-scale SIDWT correlate",
        "value": value,
        "unit": "complex samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched uniform: {args.count} pulses x {args.n} complex64, "
                               f"512-sample LFM chirp echoes, CDF 9/7 lifting, J={J}, one fused "
                               f"launch per step",
                   "pulses": args.count, "n": args.n, "ref_len": m, "filter": "cdf97", "J": J},
        "roofline": {"bound": "mfma", "achieved": achieved_tflops,
                     "peak": PEAK_FP32_MATRIX_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved_tflops / PEAK_FP32_MATRIX_TFLOPS,
                     "traffic": profiled_traffic() if (args.count, args.n) == (4096, 8192) else None,
                     "kernel": "fused_correlate<CDF97>"},
        "lifting_roofline": {"bound": "hbm", "achieved": lift_gbs, "peak": PEAK_HBM_GBS,
                             "unit": "GB/s", "frac": lift_gbs / PEAK_HBM_GBS,
                             "us_per_launch": lift_ms * 1e3, "kernel": "lift_many<CDF97>"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)
    plan.free()


if __name__ == "__main__":
    main()
