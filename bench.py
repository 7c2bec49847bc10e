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
PEAK_INT8_TOPS = 5000.0           # MI355X dense INT8 matrix


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# CPU baseline: the oracle, as it stands, one pulse per worker process.
# ---------------------------------------------------------------------------

def _oracle_pulse(args):
    filt, J, ref, rx = args
    import oracle
    t0 = time.perf_counter()
    R = oracle.correlate_direct(filt, J, ref, rx)
    return time.perf_counter() - t0, R


def _warm(_):
    import oracle  # noqa: F401
    return os.getpid()


def cpu_baseline(filt, J, ref, pulses, max_workers=32):
    """The oracle on whole pulses, one per worker process; returns the
    baseline record and the oracle's planes of each pulse timed."""
    res, wall, workers, cores = _pool_map(_oracle_pulse, [(filt, J, ref, p) for p in pulses],
                                          max_workers)
    n = pulses.shape[1]
    k = len(res)
    return ({"value": k * n / wall, "unit": "complex samples/s", "cores": workers,
             "kind": "oracle",
             "sample": f"{k} pulses x {n} samples of the same batch, one pulse per process "
                       f"(FP64 NumPy, OMP_NUM_THREADS=1), wall {wall:.1f} s; host has {cores} "
                       f"cores"},
            [r[1] for r in res])


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
KERNEL_SOURCES = ["sidwt_kernels.hip", "sidwt_lift.hpp", "sidwt_device.hpp", "sidwt_host.hpp"]


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
    ap.add_argument("--no-per-pulse", dest="per_pulse", action="store_false", default=True,
                    help="skip the plain per-pulse comparison (keeps profiles to the batch)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run an elementwise kernel that reads and writes 256 MiB "
                         "(calibrates the HBM byte counters)")
    ap.add_argument("--workload", default="batched_uniform",
                    choices=["batched_uniform", "uneven", "integer", "single", "serving", "bank",
                             "swapped", "detect", "generic"])
    ap.add_argument("--headline-only", action="store_true",
                    help="default workload without the single / integer / uneven / serving "
                         "sub-records")
    ap.add_argument("--uneven-config", default=None, metavar="FMAX,WINDOW,DEPTH",
                    help="uneven batch: this split, tile window and lifting depth instead of "
                         "the autotuner (e.g. 0,4096,4)")
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="requests per arrival rate in the serving runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path in this library "
              "(pulses are independent; a multi-GPU run would shard the pulse list).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    fn = {"batched_uniform": bench_batched_uniform, "uneven": bench_uneven,
          "integer": bench_integer, "single": bench_single,
          "serving": bench_serving, "bank": bench_bank,
          "swapped": bench_swapped, "detect": bench_detect,
          "generic": bench_generic}[args.workload]
    rec = fn(args)
    if args.workload == "batched_uniform" and not args.headline_only:
        # The other configurations of the metric, each timed and checked the
        # same way, as sub-records of the one JSON line.
        import torch
        for key, sub in (("single", bench_single), ("integer", bench_integer),
                         ("uneven", bench_uneven), ("serving", bench_serving)):
            torch.cuda.empty_cache()
            log(f"---- sub-record: {key}")
            r = sub(args)
            rec[key] = {k: v for k, v in r.items()
                        if k not in ("n_gpus", "scaling", "data", "higher_is_better")}
    print(json.dumps(rec), flush=True)


def plain_per_pulse(S, plans, rx, out):
    """The plain per-pulse GPU path: one sidwt_correlate call (one launch)
    per pulse, issued back to back on the current stream.  Returns the ms of
    one pass over all pulses (after one untimed pass)."""
    import torch
    stream = torch.cuda.current_stream()

    def one_pass():
        for p, x, o in zip(plans, rx, out):
            S.correlate(p, x, out=o)
    one_pass()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    one_pass()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def lifting_roofline(S, filt, J, rx, kernel, reps=20):
    """The lifting-only kernel over the same batch: HBM roofline from the bytes
    it must move (pulses in, pyramid out), timed with HIP events on the launch
    stream."""
    import torch
    stream = torch.cuda.current_stream()
    pyr = S.lift_many(filt, J, rx)
    for _ in range(3):
        S.lift_many(filt, J, rx, pyr=pyr)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        S.lift_many(filt, J, rx, pyr=pyr)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = rx.numel() * rx.element_size() + pyr.numel() * pyr.element_size()
    gbs = nbytes / (ms * 1e-3) / 1e9
    del pyr
    return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS, "us_per_launch": ms * 1e3, "bytes": nbytes,
            "kernel": kernel}


def synthesis_roofline(S, filt, J, rx, kernel, reps=20):
    """Coarse-to-fine formation over the same batch: from its pyramid back to
    the zero-padded pulses (c_0), HBM roofline from the bytes it must move
    (pyramid in, pulses out), timed with HIP events on the launch stream."""
    import torch
    stream = torch.cuda.current_stream()
    pyr = S.lift_many(filt, J, rx)
    out = S.synth_many(filt, J, pyr, to=0)
    for _ in range(3):
        S.synth_many(filt, J, pyr, to=0, out=out)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        S.synth_many(filt, J, pyr, to=0, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = pyr.numel() * pyr.element_size() + out.numel() * out.element_size()
    gbs = nbytes / (ms * 1e-3) / 1e9
    del pyr, out
    return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS, "us_per_launch": ms * 1e3, "bytes": nbytes,
            "kernel": kernel}


def bench_batched_uniform(args):
    import numpy as np
    import torch

    import paper_cs_0607001_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    J, m = 5, 512
    log(f"generating {args.count} x {args.n} pulses")
    b = W.batched_uniform(seed=2, count=args.count, n=args.n, m=m, J=J)
    N = S.transform_length(args.n, J)
    rx = torch.from_numpy(b.rx).to(dev)
    plan = S.plan_create(b.filter, J, b.ref)
    out = torch.empty((args.count, J, N), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()

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

    # The plain per-pulse path over the same batch (one launch per pulse).
    pp_ms = None
    if args.per_pulse:
        pp_ms = plain_per_pulse(S, [plan] * args.count, list(rx), list(out))
        log(f"plain per-pulse path: {pp_ms:.2f} ms per batch ({pp_ms / ms_step:.1f}x the fused "
            f"batch's time)")

    # Lifting-only kernel (a1 + a2), HBM roofline: 8 B in + 8 B out per sample.
    lift = lifting_roofline(S, b.filter, J, rx, "lift_many<CDF97>")
    log(f"lifting only: {lift['us_per_launch']:.1f} us, {lift['achieved']:.0f} GB/s")
    synth = synthesis_roofline(S, b.filter, J, rx, "synth_many<CDF97>")
    log(f"coarse-to-fine synthesis: {synth['us_per_launch']:.1f} us, {synth['achieved']:.0f} GB/s")

    # Scale mask: the two coarsest planes only (every level still lifted).
    coarse = [J - 2, J - 1]
    for _ in range(3):
        S.correlate_many(plan, rx, out=out, planes=coarse)
    ev0.record(stream)
    for _ in range(args.steps):
        S.correlate_many(plan, rx, out=out, planes=coarse)
    ev1.record(stream)
    torch.cuda.synchronize()
    coarse_ms = ev0.elapsed_time(ev1) / args.steps
    log(f"coarse planes {coarse} only: {coarse_ms:.3f} ms/step ({ms_step / coarse_ms:.1f}x faster "
        f"than all {J})")

    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        log("copy probe: 3 x elementwise kernels reading and writing 256 MiB each")
        del src, dst

    cpu, parity = None, None
    if args.cpu:
        log("timing the CPU oracle on a bounded sample")
        k = min(args.count, max(1, min(32, len(os.sched_getaffinity(0)))))
        cpu, planes = cpu_baseline(b.filter, J, b.ref, b.rx[:k].astype(np.complex128))
        S.correlate_many(plan, rx, out=out)
        got = out[:k].cpu().numpy()
        worst = max(float(np.linalg.norm(got[i, j] - R[j]) / np.linalg.norm(R[j]))
                    for i, R in enumerate(planes) for j in range(J))
        parity = {"pulses": k, "planes": "all lags", "worst_rel_l2": worst, "tolerance": 1e-5,
                  "ok": worst <= 1e-5}
        log(f"oracle parity on the {k} timed pulses: worst rel L2 {worst:.2e}")
        assert worst <= 1e-5, f"parity failed: {worst}"

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
        "lifting_roofline": lift,
        "synthesis_roofline": synth,
        "coarse_planes_only": {"planes": coarse, "ms_per_step": coarse_ms,
                               "samples_per_s": samples / (coarse_ms * 1e-3)},
        "planes_out": {"bytes": out.numel() * 8, "gb_per_s": out.numel() * 8 / (ms_step * 1e-3) / 1e9},
        "plain_per_pulse": None if pp_ms is None else {
            "ms_per_batch": pp_ms, "samples_per_s": args.count * args.n / (pp_ms * 1e-3),
            "batched_speedup": pp_ms / ms_step},
        "parity": parity,
        "cpu_baseline": cpu,
    }
    plan.free()
    return rec


# ---------------------------------------------------------------------------
# Other workloads (not the default line)
# ---------------------------------------------------------------------------

def _time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _oracle_lag_sample(args):
    """CPU time of the oracle on `k` lags per plane of one pulse, scaled to
    all N lags (the direct form costs the same per lag), and the values at
    those lags (plane-major) for a parity check of the GPU planes."""
    filt, J, ref, rx, k = args
    import numpy as np
    import oracle
    N = oracle.transform_length(len(rx), J)
    lags = np.unique(np.linspace(0, N - 1, k).astype(np.int64))
    t0 = time.perf_counter()
    vals = [oracle.correlate_at(filt, J, ref, rx, j, lags) for j in range(J)]
    return (time.perf_counter() - t0) * N / len(lags), lags, vals


def _pool_map(fn, items, max_workers=32):
    """The oracle over `items`, one item per worker process (spawned, one
    BLAS thread each).  Returns (results, wall seconds, workers, host cores)."""
    import multiprocessing as mp
    os.environ["OMP_NUM_THREADS"] = "1"
    os.environ["OPENBLAS_NUM_THREADS"] = "1"
    os.environ["MKL_NUM_THREADS"] = "1"
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, max_workers, len(items)))
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_warm, range(workers))
        t0 = time.perf_counter()
        res = pool.map(fn, items, chunksize=1)
        wall = time.perf_counter() - t0
    return res, wall, workers, cores


def cpu_baseline_lags(items, k=64, max_workers=32):
    """items: list of (filter, J, ref, rx).  Returns (samples/s of the pool,
    workers, host cores, per-item (lags, values))."""
    res, _, workers, cores = _pool_map(_oracle_lag_sample, [it + (k,) for it in items],
                                       max_workers)
    samples = sum(len(it[3]) for it in items)
    secs = sum(r[0] for r in res)
    # work spread over `workers` processes
    return samples / (secs / workers), workers, cores, [(r[1], r[2]) for r in res]


def sampled_parity(got_planes, lags, want, tol=1e-5):
    """Relative L2 error per plane of GPU planes (J, N) at `lags` against
    the oracle's values there; returns the worst plane's error."""
    import numpy as np
    worst = 0.0
    for j, w in enumerate(want):
        g = got_planes[j, lags].astype(np.complex128)
        e = float(np.linalg.norm(g - w) / max(np.linalg.norm(w), 1e-300))
        worst = max(worst, e)
    return worst


def pulse_flops(plan_desc_lens, N):
    return 8 * N * sum(plan_desc_lens)


def plan_lens(S, plan):
    import ctypes
    lens = []
    for lvl in range(1, plan.J + 1):
        for band in (0, 1):
            lo, ln = ctypes.c_int32(), ctypes.c_int32()
            S._lib.check(S._lib.lib().sidwt_plan_phase(plan.handle, lvl, band, 0, ctypes.byref(lo),
                                                       ctypes.byref(ln), None))
            lens.append(ln.value)
    return lens


def bench_uneven(args):
    """10^4 pulses, lengths log-uniform in [512, 65536], 16 references
    (LFM / Barker-13 / polyphase, 64..2048 samples), D4 and 9/7 mixed,
    J = floor(log2(n/16)); one persistent launch per step from a HIP graph,
    split chosen by the autotuner."""
    import numpy as np
    import torch

    import paper_cs_0607001_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    count = 10000 if args.count == 4096 else args.count
    log(f"generating {count} uneven pulses")
    refs, reqs = W.uneven_batch(seed=4, count=count)
    ns = [r.n for r in reqs]
    total = sum(ns)
    flat = np.empty(total, np.complex64)
    offs = np.cumsum([0] + ns)
    for r, o in zip(reqs, offs):
        flat[o:o + r.n] = r.rx
    rx_all = torch.from_numpy(flat).to(dev)
    rx = [rx_all[o:o + n] for o, n in zip(offs, ns)]
    plans, cache, flops = [], {}, 0
    for r in reqs:
        key = (r.ref_index, r.filter, r.J)
        if key not in cache:
            p = S.plan_create(r.filter, r.J, refs[r.ref_index])
            cache[key] = (p, plan_lens(S, p))
        plans.append(cache[key][0])
        flops += pulse_flops(cache[key][1], S.transform_length(r.n, r.J))
    out_sizes = [p.J * S.transform_length(n, p.J) for p, n in zip(plans, ns)]
    out_all = torch.empty(sum(out_sizes), dtype=torch.complex64, device=dev)
    oo = np.cumsum([0] + out_sizes)
    out = [out_all[o:o + sz].view(p.J, -1) for o, sz, p in zip(oo, out_sizes, plans)]
    log(f"{count} pulses, {total / 1e6:.1f} M samples, {len(cache)} plans, "
        f"{out_all.numel() * 8 / 1e9:.1f} GB of planes")
    stream = torch.cuda.current_stream()
    b = S.Batch(plans, ns)
    if args.uneven_config:
        fmax, win, depth = (int(v) for v in args.uneven_config.split(","))
        b.config(fmax, win, depth)
        info = b.info()
        log(f"configured: {info}")
    else:
        info = b.tune(rx, out)
        log(f"autotuned: {info}")
    # the buffers are bound once (pointer arrays kept), as a serving loop over
    # fixed buffers would: per-call marshalling of 2 x 10^4 tensor pointers in
    # Python takes longer than the GPU step
    b.bind(rx, out)
    ms = _time_steps(lambda: b.run_bound(), args.steps, args.warmup, stream)
    ms_unbound = _time_steps(lambda: b.run(rx, out), min(args.steps, 5), 1, stream)
    log(f"uneven with the pointers marshalled on every call (run): {ms_unbound:.3f} ms/step")
    value = total / (ms * 1e-3)
    tflops = flops / (ms * 1e-3) / 1e12
    log(f"uneven: {ms:.3f} ms/step, {value / 1e9:.2f} G samples/s, {tflops:.1f} TFLOP/s")
    pp_ms = plain_per_pulse(S, plans, rx, out) if args.per_pulse else None
    if pp_ms is not None:
        log(f"plain per-pulse path: {pp_ms:.2f} ms per batch ({pp_ms / ms:.1f}x the batched time)")
    cpu, parity = None, None
    if args.cpu:
        idx = np.argsort(ns)[np.linspace(0, count - 1, 100).astype(int)]
        items = [(reqs[i].filter, reqs[i].J, refs[reqs[i].ref_index], reqs[i].rx) for i in idx]
        v, workers, cores, vals = cpu_baseline_lags(items)
        cpu = {"value": v, "unit": "complex samples/s", "cores": workers, "kind": "oracle",
               "sample": f"100 pulses stratified by length (every 100th by n), 64 lags per "
                         f"plane each, oracle time scaled to all N lags; host has {cores} cores"}
        worst = max(sampled_parity(out[i].cpu().numpy(), lags, want)
                    for i, (lags, want) in zip(idx, vals))
        parity = {"pulses": len(idx), "lags_per_plane": 64, "worst_rel_l2": worst,
                  "tolerance": 1e-5, "ok": worst <= 1e-5}
        log(f"oracle parity on the 100 sampled pulses: worst rel L2 {worst:.2e}")
        assert worst <= 1e-5, f"uneven batch parity failed: {worst}"
    b.free()
    return {
        "metric": "complex samples/sec through J-scale SIDWT correlate",
        "value": value, "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"uneven batch: {count} pulses, n log-uniform in [512, 65536], "
                               f"16 references 64..2048, D4 / CDF 9/7, J=floor(log2(n/16)), "
                               f"one persistent graph-replayed launch, pulse and output buffers "
                               f"bound once", "samples": total,
                   "batch": info},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_FP32_MATRIX_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / PEAK_FP32_MATRIX_TFLOPS, "traffic": None,
                     "kernel": "one graph replay: batch_lift_blocks passes + batch_persistent classes",
                     "flops_per_step": flops},
        "planes_out": {"bytes": out_all.numel() * 8,
                       "gb_per_s": out_all.numel() * 8 / (ms * 1e-3) / 1e9},
        "ms_per_step_marshalling_each_call": ms_unbound,
        "plain_per_pulse": None if pp_ms is None else {
            "ms_per_batch": pp_ms, "samples_per_s": total / (pp_ms * 1e-3),
            "batched_speedup": pp_ms / ms},
        "parity": parity,
        "cpu_baseline": cpu,
    }


def bench_integer(args):
    """16384 x 4096 int16 I/Q pulses, reversible 5/3, J = 6, exact int64
    planes (balanced base-256 digits on int8 matrix cores, int32 sums per
    shift class, combined in int64)."""
    import numpy as np
    import torch

    import paper_cs_0607001_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    count = 16384 if args.count == 4096 else args.count
    n, J = 4096, 6
    log(f"generating {count} x {n} int16 pulses")
    ib = W.integer_batch(seed=3, count=count, n=n, m=512, J=J)
    rx = torch.from_numpy(ib.rx_iq).to(dev)
    plan = S.plan_create("legall53_int", J, ib.ref_iq)
    out = torch.empty((count, J, n, 2), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream()
    ms = _time_steps(lambda: S.correlate_many(plan, rx, out=out), args.steps, args.warmup, stream)
    flops = pulse_flops(plan_lens(S, plan), n) * count
    value = count * n / (ms * 1e-3)
    tflops = flops / (ms * 1e-3) / 1e12
    info = plan.info()
    wl = info["i8_weight_digits"]
    # int8 path: every algorithmic op becomes 3 x wl digit products; its
    # floor is the larger of those on the INT8 peak and the bytes on HBM
    nbytes = rx.numel() * rx.element_size() + out.numel() * out.element_size()
    digit_ops = flops * 3 * wl
    t_mfma = digit_ops / (PEAK_INT8_TOPS * 1e12) if wl else flops / 78.6e12
    t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
    bound = "hbm" if t_hbm >= t_mfma else "mfma"
    log(f"integer: {ms:.3f} ms/step, {value / 1e9:.2f} G samples/s, {tflops:.1f} T algorithmic "
        f"ops/s ({'int8 matrix cores, ' + str(wl) + ' weight digits' if wl else 'FP64 MFMA'}); "
        f"floor {max(t_mfma, t_hbm) * 1e3:.3f} ms ({bound})")
    lift = lifting_roofline(S, "legall53_int", J, rx, "lift_many<LEGALL53_INT>")
    log(f"lifting only: {lift['us_per_launch']:.1f} us, {lift['achieved']:.0f} GB/s")
    synth = synthesis_roofline(S, "legall53_int", J, rx, "synth_many<LEGALL53_INT>")
    log(f"coarse-to-fine synthesis: {synth['us_per_launch']:.1f} us, {synth['achieved']:.0f} GB/s")
    cpu, parity = None, None
    if args.cpu:
        idx = np.linspace(0, count - 1, 16).astype(int)
        items = [("legall53_int", J, ib.ref_iq, ib.rx_iq[i]) for i in idx]
        v, workers, cores, vals = cpu_baseline_lags_int(items)
        cpu = {"value": v, "unit": "complex samples/s", "cores": workers, "kind": "oracle",
               "sample": f"16 pulses spread over the batch, 64 lags per plane each, int64 oracle "
                         f"time scaled to all N lags; host has {cores} cores"}
        S.correlate_many(plan, rx, out=out)
        torch.cuda.synchronize()
        bad = 0
        for i, (lags, want) in zip(idx, vals):
            got = out[i].cpu().numpy()
            for j in range(J):
                bad += int(not np.array_equal(got[j, lags], want[j]))
        parity = {"pulses": len(idx), "lags_per_plane": 64, "planes_differing": bad,
                  "bit_exact": bad == 0}
        log(f"oracle parity on 16 sampled pulses: {'bit-exact' if bad == 0 else f'{bad} planes differ'}")
        assert bad == 0, "integer parity failed"
    plan.free()
    return {
        "metric": "complex samples/sec through J-scale SIDWT correlate",
        "value": value, "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32 lifting; int8 digits, int32 class sums, int64 planes",
        "data": "synthetic",
        "config": {"workload": f"integer: {count} x {n} int16 I/Q, reversible 5/3, J={J}, "
                               f"bit-exact int64 planes", "weight_digits": wl},
        "roofline": {"bound": bound,
                     "achieved": nbytes / (ms * 1e-3) / 1e9 if bound == "hbm"
                     else digit_ops / (ms * 1e-3) / 1e12,
                     "peak": PEAK_HBM_GBS if bound == "hbm" else PEAK_INT8_TOPS,
                     "unit": "GB/s" if bound == "hbm" else "TOP/s",
                     "frac": max(t_mfma, t_hbm) / (ms * 1e-3), "traffic": None,
                     "kernel": "fused_correlate_i8" if wl else "fused_correlate<INT53>",
                     "bytes": nbytes, "algorithmic_ops": flops, "digit_ops": digit_ops,
                     "int8_frac": digit_ops / (ms * 1e-3) / (PEAK_INT8_TOPS * 1e12),
                     "hbm_frac": t_hbm / (ms * 1e-3)},
        "lifting_roofline": lift,
        "synthesis_roofline": synth,
        "parity": parity,
        "cpu_baseline": cpu,
    }


def bench_swapped(args):
    """Roles exchanged on the uniform batch (4096 x 8192 complex64, 512-sample
    chirp echoes, CDF 9/7, J = 5): redundant y-side tree of every received
    pulse (J - 1 tree launches into a workspace), then one correlation launch
    over (pulse, plane).  The forward path on the same batch is timed beside
    it."""
    import ctypes

    import torch

    import paper_cs_0607001_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    J, m = 5, 512
    log(f"generating {args.count} x {args.n} pulses")
    b = W.batched_uniform(seed=2, count=args.count, n=args.n, m=m, J=J)
    N = S.transform_length(args.n, J)
    rx = torch.from_numpy(b.rx).to(dev)
    plan = S.plan_create(b.filter, J, b.ref)
    out = torch.empty((args.count, J, N), dtype=torch.complex64, device=dev)
    ws = torch.empty(S._lib.lib().sidwt_swap_workspace_bytes(plan.handle, args.n, args.count),
                     dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ms = _time_steps(lambda: S.correlate_swapped(plan, rx, out=out, workspace=ws), args.steps,
                     args.warmup, stream)
    # 8 real flops per complex MAC: every lag of plane j takes the support of
    # the reference's level-j approximation (plane 0: the reference itself)
    flops = 8 * N * m
    for j in range(1, J):
        lo, ln = ctypes.c_int32(), ctypes.c_int32()
        S._lib.check(S._lib.lib().sidwt_plan_phase(plan.handle, j, 0, 0, ctypes.byref(lo),
                                                   ctypes.byref(ln), None))
        flops += 8 * N * ln.value
    flops *= args.count
    value = args.count * args.n / (ms * 1e-3)
    tflops = flops / (ms * 1e-3) / 1e12
    log(f"swapped: {ms:.3f} ms/step, {value / 1e9:.2f} G samples/s, {tflops:.1f} TFLOP/s "
        f"(tree + correlation)")
    fwd = _time_steps(lambda: S.correlate_many(plan, rx, out=out), args.steps, args.warmup, stream)
    log(f"forward path on the same batch: {fwd:.3f} ms/step")
    plan.free()
    return {
        "metric": "complex samples/sec through J-scale SIDWT correlate",
        "value": value, "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"roles exchanged: {args.count} pulses x {args.n} complex64, "
                               f"{m}-sample LFM chirp echoes, CDF 9/7, J={J}; redundant tree on "
                               f"each pulse, critical reference"},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_FP32_MATRIX_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / PEAK_FP32_MATRIX_TFLOPS, "traffic": None,
                     "kernel": "swap_tree_level + swap_correlate (whole call)"},
        "forward_ms_per_step": fwd,
        "cpu_baseline": None,
    }


def bench_detect(args):
    """Target declaration after the correlation: the uniform batch's planes
    (4096 x 5 x 8192 complex64) scanned for peaks at -10 dB, timed alone (HBM
    roofline: the planes are read once) and as correlation + declaration; the
    five-target scene (CDF 9/7, J = 3) reports its peaks per plane."""
    import numpy as np
    import torch

    import paper_cs_0607001_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    J, m = 5, 512
    log(f"generating {args.count} x {args.n} pulses")
    b = W.batched_uniform(seed=2, count=args.count, n=args.n, m=m, J=J)
    N = S.transform_length(args.n, J)
    rx = torch.from_numpy(b.rx).to(dev)
    plan = S.plan_create(b.filter, J, b.ref)
    planes = S.correlate_many(plan, rx)
    stream = torch.cuda.current_stream()
    ms_det = _time_steps(lambda: S.detect_peaks(planes, -10.0, 64), args.steps, args.warmup,
                         stream)
    ms_all = _time_steps(lambda: (S.correlate_many(plan, rx, out=planes),
                                  S.detect_peaks(planes, -10.0, 64)), args.steps, args.warmup,
                         stream)
    nbytes = planes.numel() * planes.element_size()
    gbs = nbytes / (ms_det * 1e-3) / 1e9
    value = args.count * args.n / (ms_all * 1e-3)
    _, _, found = S.detect_peaks(planes, -10.0, 64)
    mean_found = found.float().mean(dim=0).cpu().numpy()
    log(f"declaration: {ms_det * 1e3:.1f} us ({gbs:.0f} GB/s of planes); correlation + "
        f"declaration {ms_all:.3f} ms/step; mean peaks per plane {np.round(mean_found, 2)}")
    plan.free()
    sc = W.multi_target(seed=5, count=8)
    with S.plan_create(sc.filter, sc.J, sc.ref) as sp:
        sl, sd, sf = S.detect_peaks(S.correlate_many(sp, torch.from_numpy(sc.rx).to(dev)), -10.0, 32)
    sf = sf.cpu().numpy()
    log(f"five-target scene, peaks at -10 dB per plane (8 pulses): {sf.tolist()}")
    return {
        "metric": "complex samples/sec through J-scale SIDWT correlate",
        "value": value, "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_all, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"correlation + target declaration at -10 dB: {args.count} pulses "
                               f"x {args.n} complex64, {m}-sample chirp echoes, CDF 9/7, J={J}"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gbs / PEAK_HBM_GBS, "traffic": None, "kernel": "detect_peaks",
                     "us_per_launch": ms_det * 1e3, "bytes": nbytes},
        "scene_peaks_per_plane": sf.tolist(),
        "cpu_baseline": None,
    }


def _impulse_taps(lift):
    """Lowpass and highpass tap dicts of a one-level lifting, from its
    impulse responses (out[k] = sum_i c_i u[2k + i])."""
    import numpy as np
    lo, hi = {}, {}
    for i in range(-12, 13):
        u = np.zeros(64)
        u[i % 64] = 1.0
        A, B = lift(u)
        if abs(A[0]) > 1e-15:
            lo[i] = float(A[0])
        if abs(B[0]) > 1e-15:
            hi[i] = float(B[0])
    return lo, hi


def _cdf97_x_lift(t):
    """x-side 9/7 lifting of the Case II family at parameter t (Sec. III-C),
    written out here so that the benchmark needs no test code."""
    import numpy as np
    a = (-2 * t + 1) / (4 * (t - 1))
    b = -(t - 1) ** 2
    g = 1 / (4 * t * (t - 1))
    d = t ** 3 - 7 / 4 * t ** 2 + t
    x = np.sqrt(2) / t

    def lift(u):
        e, o = u[0::2].copy(), u[1::2].copy()
        o = o + a * (e + np.roll(e, -1))
        e = e + b * (o + np.roll(o, 1))
        o = o + g * (e + np.roll(e, -1))
        e = e + d * (o + np.roll(o, 1))
        return x * e, o / x
    return lift


def bench_generic(args):
    """Generic lifting (steps from the host factorizer at run time) with the
    irrational CDF 9/7 (t = 1.2301741...) on the uniform batch (4096 x 8192
    complex64, J = 5), against the compiled Table I lifting kernel."""
    import torch

    import paper_cs_0607001_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    J = 5
    log(f"generating {args.count} x {args.n} pulses")
    b = W.batched_uniform(seed=2, count=args.count, n=args.n, m=512, J=J)
    rx = torch.from_numpy(b.rx).to(dev)
    lo, hi = _impulse_taps(_cdf97_x_lift(1.230174104914001))
    f = S.Lifting(lo, hi)
    pyr = S.lift_generic(f, J, rx)
    stream = torch.cuda.current_stream()
    ms = _time_steps(lambda: S.lift_generic(f, J, rx, pyr=pyr), args.steps, args.warmup, stream)
    nbytes = rx.numel() * rx.element_size() + pyr.numel() * pyr.element_size()
    gbs = nbytes / (ms * 1e-3) / 1e9
    ms_c = _time_steps(lambda: S.lift_many("cdf97", J, rx, pyr=pyr), args.steps, args.warmup,
                       stream)
    log(f"generic lifting (irrational 9/7, {len(f.steps)} steps): {ms * 1e3:.1f} us, {gbs:.0f} GB/s; "
        f"compiled Table I lifting {ms_c * 1e3:.1f} us")
    f.free()
    value = args.count * args.n / (ms * 1e-3)
    return {
        "metric": "complex samples/sec through J-scale SIDWT lifting",
        "value": value, "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"generic lifting: {args.count} x {args.n} complex64, irrational "
                               f"CDF 9/7 factorized on the host, J={J}"},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": gbs / PEAK_HBM_GBS, "traffic": None, "kernel": "lift_generic",
                     "us_per_launch": ms * 1e3, "bytes": nbytes},
        "compiled_lift_many_us": ms_c * 1e3,
        "cpu_baseline": None,
    }


def _oracle_lag_sample_int(args):
    filt, J, ref, rx, k = args
    import numpy as np
    import oracle
    N = oracle.transform_length(len(rx), J)
    lags = np.unique(np.linspace(0, N - 1, k).astype(np.int64))
    t0 = time.perf_counter()
    vals = [oracle.correlate_int_at(J, ref, rx, j, lags) for j in range(J)]
    return (time.perf_counter() - t0) * N / len(lags), lags, vals


def cpu_baseline_lags_int(items, k=64, max_workers=32):
    res, _, workers, cores = _pool_map(_oracle_lag_sample_int, [it + (k,) for it in items],
                                       max_workers)
    samples = sum(len(it[3]) for it in items)
    secs = sum(r[0] for r in res)
    return samples / (secs / workers), workers, cores, [(r[1], r[2]) for r in res]


def _oracle_single(seed):
    """The oracle on one request of the single-correlation workload (all
    planes, all lags); returns (seconds, planes)."""
    import oracle
    import workloads as W
    w = W.single_chirp(seed=seed)
    t0 = time.perf_counter()
    R = oracle.correlate_direct(w.filter, w.J, w.ref, w.rx)
    return time.perf_counter() - t0, R


def bench_single(args):
    """One 1024-sample pulse per request (256-sample chirp, 10 dB, 5/3,
    J = 3), 1000 seeded requests one at a time: per-request latency (call to
    completion, host clock), kernel duration (HIP events on the launch
    stream), and the oracle over all 1000 requests with parity on each."""
    import numpy as np
    import torch

    import paper_cs_0607001_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    seeds = list(range(1, 1001))
    reqs = [W.single_chirp(seed=s) for s in seeds]
    rx = [torch.from_numpy(w.rx.astype(np.complex64)).to(dev) for w in reqs]
    plan = S.plan_create("legall53", 3, reqs[0].ref)
    N = 1024
    outs = torch.empty((len(reqs), 3, N), dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream()
    for x in rx[:50]:
        S.correlate(plan, x, out=outs[0])
    torch.cuda.synchronize()
    lat = []
    for i, x in enumerate(rx):
        t0 = time.perf_counter()
        S.correlate(plan, x, out=outs[i])
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    lat = np.array(lat)
    p50, p99 = np.percentile(lat, 50), np.percentile(lat, 99)
    # kernel durations: events around each launch, launches back to back
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in rx]
    for (a, b), x, i in zip(ev, rx, range(len(rx))):
        a.record(stream)
        S.correlate(plan, x, out=outs[i])
        b.record(stream)
    torch.cuda.synchronize()
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    flops = pulse_flops(plan_lens(S, plan), N)
    tflops = flops / (kern_ms * 1e-3) / 1e12
    log(f"single: p50 {p50 * 1e6:.1f} us, p99 {p99 * 1e6:.1f} us per request; kernel "
        f"{kern_ms * 1e3:.1f} us")
    cpu, parity = None, None
    if args.cpu:
        res, wall, workers, cores = _pool_map(_oracle_single, seeds)
        got = outs.cpu().numpy().astype(np.complex128)
        errs = np.array([[np.linalg.norm(got[i, j] - R[j]) / np.linalg.norm(R[j])
                          for j in range(3)] for i, (_, R) in enumerate(res)])
        peaks_ok = int(sum(int(np.argmax(np.abs(got[i, 0]))) == w.delay
                           for i, w in enumerate(reqs)))
        cpu = {"value": len(seeds) * N / wall, "unit": "complex samples/s", "cores": workers,
               "kind": "oracle",
               "sample": f"all {len(seeds)} seeded requests (FP64 NumPy, one request per process, "
                         f"OMP_NUM_THREADS=1), wall {wall:.1f} s; host has {cores} cores",
               "requests_per_s": len(seeds) / wall}
        parity = {"requests": len(seeds), "worst_rel_l2": float(errs.max()), "tolerance": 1e-5,
                  "ok": bool(errs.max() <= 1e-5), "peak_at_planted_delay": peaks_ok}
        log(f"oracle over all {len(seeds)} requests: {wall:.1f} s on {workers} processes; "
            f"parity worst rel L2 {errs.max():.2e}; peak at the planted delay in {peaks_ok}")
        assert errs.max() <= 1e-5, "single-request parity failed"
    plan.free()
    return {
        "metric": "complex samples/sec through J-scale SIDWT correlate; p50/p99 request latency",
        "value": N / p50, "unit": "complex samples/s", "n_gpus": 1, "steps": len(lat),
        "warmup": 50, "ms_per_step": p50 * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "single correlation: 1024-sample pulse, 256-sample chirp "
                               "(TBP 64), 10 dB, 5/3, J=3, one request at a time, 1000 requests",
                   "p50_us": p50 * 1e6, "p99_us": p99 * 1e6, "kernel_us": kern_ms * 1e3},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": PEAK_FP32_MATRIX_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / PEAK_FP32_MATRIX_TFLOPS,
                     "traffic": None, "kernel": "fused_correlate<LEGALL53> (one workgroup per plane)",
                     "flops_per_launch": flops,
                     "note": "one 1024-sample pulse per launch runs on three workgroups (one "
                             "per plane) of three CUs: bound by launch latency, not by the chip"},
        "parity": parity,
        "cpu_baseline": cpu,
    }


def _serving_requests(refs, count, seed=5):
    """Requests of the serving workload: n log-uniform in [512, 65536], J =
    floor(log2(n / 16)), an echo train of one bank reference (m <= n / 2)
    in noise."""
    import numpy as np

    import workloads as W
    rng = np.random.default_rng([seed, 1])
    out = []
    for _ in range(count):
        n = W.uneven_length(rng)
        elig = [k for k, r in enumerate(refs) if len(r) <= n // 2] or [0]
        k = elig[int(rng.integers(0, len(elig)))]
        out.append((n, W.levels_for(n), W.echoes(n, refs[k], rng).astype(np.complex64)))
    return out


def bench_bank(args):
    """One bank call per step: 256 requests of the serving mix against a bank
    of 64 references (64..2048 samples, CDF 9/7, FP16 hi+lo MFMA).  The GEMM
    kernel's duration comes from HIP events the library records around its
    launch on the call's stream."""
    import torch

    import paper_cs_0607001_amd as S
    import workloads as W

    dev = torch.device("cuda:0")
    count = 256 if args.count == 4096 else args.count
    refs = W.reference_set(5, count=64)
    bank = S.Bank("cdf97", 12, refs, "fp16")
    reqs = _serving_requests(refs, count)
    rx = [torch.from_numpy(y).to(dev) for _, _, y in reqs]
    Js = [J for _, J, _ in reqs]
    ws = bank.workspace()
    outs = bank.correlate(rx, Js, workspace=ws)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ms = _time_steps(lambda: bank.correlate(rx, Js, out=outs, workspace=ws),
                     args.steps, args.warmup, stream)
    ws.timing(True)
    lift, gemm = [], []
    for _ in range(args.steps):
        bank.correlate(rx, Js, out=outs, workspace=ws)
        a, b = ws.times()
        lift.append(a)
        gemm.append(b)
    ws.timing(False)
    lift_ms, gemm_ms = sum(lift) / len(lift), sum(gemm) / len(gemm)
    lens = [plan_lens(S, bank.plan(e)) for e in range(len(refs))]
    flops = 0
    samples = sum(n for n, _, _ in reqs)
    out_bytes = sum(o.numel() * 8 for o in outs)
    for n, J, _ in reqs:
        N = S.transform_length(n, J)
        for e in range(bank.eligible(n)):
            flops += 3 * pulse_flops(lens[e][:2 * J], N)   # hi*hi + hi*lo + lo*hi
    tflops = flops / (gemm_ms * 1e-3) / 1e12
    value = samples / (ms * 1e-3)
    log(f"bank: {ms:.3f} ms/step ({lift_ms:.3f} lifting + {gemm_ms:.3f} GEMM), "
        f"{value / 1e9:.3f} G samples/s, {tflops:.0f} TFLOP/s FP16, "
        f"planes {out_bytes / (gemm_ms * 1e-3) / 1e12:.2f} TB/s")
    ws.free()
    bank.free()
    return {
        "metric": "complex samples/sec through J-scale SIDWT correlate",
        "value": value, "unit": "complex samples/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp16 hi+lo MFMA, fp32 accumulate", "data": "synthetic",
        "config": {"workload": f"reference bank: {count} requests, n log-uniform in [512, 65536], "
                               f"64 references (64..2048), CDF 9/7, J=floor(log2(n/16)), "
                               f"all eligible references per request",
                   "samples": samples, "plane_bytes": out_bytes,
                   "lift_ms": lift_ms, "gemm_ms": gemm_ms},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": tflops / 2500.0, "traffic": None,
                     "kernel": "bank_items<FP16> (levels 1-3) + bank_items_deep<FP16> (levels 4+)",
                     "hbm_write_frac": out_bytes / (gemm_ms * 1e-3) / 8e12},
        "cpu_baseline": None,
    }


def _oracle_bank_sample(args):
    """The oracle on one serving request against a few of its eligible
    references, `k` lags per plane; returns (seconds scaled to all N lags,
    lags, values[ref][plane])."""
    J, refs, rx, k = args
    import numpy as np
    import oracle
    N = oracle.transform_length(len(rx), J)
    lags = np.unique(np.linspace(0, N - 1, k).astype(np.int64))
    y = rx.astype(np.complex128)
    t0 = time.perf_counter()
    vals = [[oracle.correlate_at("cdf97", J, r, y, j, lags) for j in range(J)] for r in refs]
    return (time.perf_counter() - t0) * N / len(lags), lags, vals


def _bank_flops_bytes(S, bank, lens, reqs):
    """Algorithmic work of bank requests (n, J, rx): complex MACs of the
    block-circulant products counted once (8 real flops each) over every
    eligible reference, and HBM bytes of pulses in and planes out."""
    flops, nbytes = 0, 0
    for n, J, _ in reqs:
        N = S.transform_length(n, J)
        E = bank.eligible(n)
        for e in range(E):
            flops += pulse_flops(lens[e][:2 * J], N)
        nbytes += n * 8 + E * J * N * 8
    return flops, nbytes


def bench_serving(args):
    """Serving with a bank of 64 references (ascending length, LFM /
    Barker-13 / polyphase, 64..2048 samples, CDF 9/7, FP16 hi+lo MFMA):
    requests sized as the uneven workload arrive as a Poisson process at
    rates relative to the measured saturation rate (0.5x and 0.9x; the whole
    sweep 0.1x..1.2x with --workload serving); p50/p99 latency and samples/s
    per rate, the roofline of the saturation run, the bank's per-scale error
    against the oracle and the oracle's own rate on a length-stratified
    sample.  With --workload serving also: the same requests through the FP32
    plain path (every (request, reference) pair as one pulse of an uneven
    batch, and one launch per pair)."""
    import numpy as np
    import torch

    import paper_cs_0607001_amd as S
    import workloads as W
    from paper_cs_0607001_amd import serving

    full = args.workload == "serving"
    dev = torch.device("cuda:0")
    count = args.serve_requests
    refs = W.reference_set(5, count=64)
    log("building the bank (64 references, Jmax 12)")
    bank = S.Bank("cdf97", 12, refs, "fp16")
    lens = [plan_lens(S, bank.plan(e)) for e in range(len(refs))]
    log(f"generating {count} requests")
    pulses = _serving_requests(refs, count)
    host = [torch.from_numpy(p[2]).pin_memory() for p in pulses]
    total_samples = sum(p[0] for p in pulses)

    def reqs(times, keep=False):
        return [serving.Request(i, float(times[i]), host[i], pulses[i][1], keep)
                for i in range(count)]

    budget = 64 << 30
    srv = serving.Server(bank, slots=4, budget_bytes=budget, max_group=32)
    srv.run(reqs(np.zeros(count))[:64])          # warm-up (workspaces grow)
    log(f"saturation run: {count} requests at t = 0")
    sat_recs = srv.run(reqs(np.zeros(count)))
    sat = serving.summarize(sat_recs)
    rate_sat = sat["requests_per_s"]
    ref_samples = sum(p[0] * bank.eligible(p[0]) for p in pulses)
    sat["reference_samples_per_s"] = sat["samples_per_s"] * ref_samples / total_samples
    log(f"saturation: {rate_sat:.0f} requests/s, {sat['samples_per_s'] / 1e9:.2f} G samples/s")
    span_s = count / rate_sat
    flops, nbytes = _bank_flops_bytes(S, bank, lens, pulses)
    mfma_floor = 3 * flops / 2.5e15              # hi*hi + hi*lo + lo*hi on FP16 matrix cores
    hbm_floor = nbytes / 8e12
    floor = max(mfma_floor, hbm_floor)
    bound = "mfma" if mfma_floor >= hbm_floor else "hbm"
    roof = {"bound": bound,
            "achieved": (3 * flops / span_s / 1e12) if bound == "mfma" else nbytes / span_s / 1e9,
            "peak": 2500.0 if bound == "mfma" else PEAK_HBM_GBS,
            "unit": "TFLOP/s" if bound == "mfma" else "GB/s",
            "frac": floor / span_s, "traffic": None,
            "kernel": "saturation run: lifting + bank_items per group, 4 streams",
            "floor_ms": floor * 1e3, "mfma_floor_ms": mfma_floor * 1e3,
            "hbm_floor_ms": hbm_floor * 1e3, "run_ms": span_s * 1e3,
            "flops_once": flops, "flops_split": 3 * flops, "bytes": nbytes,
            "note": "frac = max(split flops / FP16 peak, bytes / HBM peak) / measured time of "
                    "the saturation run (pulses copied from pinned host memory inside it)"}
    log(f"saturation roofline: floor {floor * 1e3:.1f} ms ({bound}) of {span_s * 1e3:.1f} ms "
        f"({roof['frac'] * 100:.1f} %)")
    sweep = []
    for f in ((0.1, 0.2, 0.4, 0.6, 0.8, 0.9, 1.0, 1.1, 1.2) if full else (0.5, 0.9)):
        rate = f * rate_sat
        t = W.poisson_arrivals(5 + int(f * 100), rate, count)
        rec = serving.summarize(srv.run(reqs(t - t[0])))
        rec["rate_fraction"] = f
        rec["offered_requests_per_s"] = rate
        sweep.append(rec)
        log(f"rate {f:.1f}x: p50 {rec['p50_ms']:.2f} ms, p99 {rec['p99_ms']:.2f} ms, "
            f"{rec['samples_per_s'] / 1e9:.2f} G samples/s")
    srv.close()

    # Oracle: 100 requests stratified by length, four eligible references
    # each (spread over the eligible prefix), 16 lags per plane; its time is
    # scaled to every eligible reference and every lag.  The bank's planes
    # at those lags give the per-scale error against the oracle.
    cpu, err = None, {}
    if args.cpu:
        order = np.argsort([p[0] for p in pulses])
        idx = order[np.linspace(0, count - 1, 100).astype(int)]
        picks = []
        for i in idx:
            E = bank.eligible(pulses[i][0])
            picks.append(sorted({int(e) for e in np.linspace(0, E - 1, 4).round()}))
        items = [(pulses[i][1], [refs[e] for e in pk], pulses[i][2], 16)
                 for i, pk in zip(idx, picks)]
        res, _, workers, cores = _pool_map(_oracle_bank_sample, items)
        secs = sum(r[0] * bank.eligible(pulses[i][0]) / len(pk)
                   for r, i, pk in zip(res, idx, picks))
        samples = sum(pulses[i][0] for i in idx)
        cpu = {"value": samples / (secs / workers), "unit": "complex samples/s",
               "cores": workers, "kind": "oracle",
               "sample": f"100 requests stratified by length, 4 of their eligible references "
                         f"each, 16 lags per plane; oracle time scaled to every eligible "
                         f"reference and all N lags; host has {cores} cores",
               "reference_samples_per_s": sum(pulses[i][0] * bank.eligible(pulses[i][0])
                                              for i in idx) / (secs / workers)}
        rx = [host[i].to(dev) for i in idx]
        outs = bank.correlate(rx, [pulses[i][1] for i in idx])
        torch.cuda.synchronize()
        for i, pk, (_, lags, vals), o in zip(idx, picks, res, outs):
            g = o.cpu().numpy()
            for e, want in zip(pk, vals):
                for j, w in enumerate(want):
                    r = float(np.linalg.norm(g[e, j, lags] - w) / np.linalg.norm(w))
                    err[j] = max(err.get(j, 0.0), r)
        log(f"bank vs oracle, worst rel L2 per scale: "
            f"{ {j: f'{v:.1e}' for j, v in sorted(err.items())} }")
        assert max(err.values()) <= 1e-5, "bank parity failed"

    rec = {
        "metric": "complex samples/sec through J-scale SIDWT correlate; p50/p99 request latency",
        "value": sat["samples_per_s"], "unit": "complex samples/s", "n_gpus": 1, "steps": count,
        "warmup": 64, "ms_per_step": 1e3 / rate_sat, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "fp16 hi+lo MFMA, fp32 accumulate", "data": "synthetic",
        "config": {"workload": f"serving: {count} requests per rate, n log-uniform in "
                               f"[512, 65536], bank of 64 references (64..2048), CDF 9/7, "
                               f"J=floor(log2(n/16)), 4 slots, {budget >> 30} GiB budget, "
                               f"Poisson arrivals",
                   "saturation": sat, "sweep": sweep,
                   "bank_rel_l2_per_scale_max": err},
        "p50_ms": {f"{r['rate_fraction']}x": r["p50_ms"] for r in sweep},
        "p99_ms": {f"{r['rate_fraction']}x": r["p99_ms"] for r in sweep},
        "roofline": roof, "cpu_baseline": cpu,
    }
    if full:
        rec["config"]["bank_vs_fp32"] = _bank_vs_fp32(S, bank, refs, pulses, host, dev)
    bank.free()
    return rec


def _bank_vs_fp32(S, bank, refs, pulses, host, dev):
    """Bank (FP16 hi+lo) against the FP32 plain path on the first 200
    requests: every (request, eligible reference) pair as one pulse of an
    uneven batch, and as one launch per pair."""
    import torch
    sub = list(range(min(len(pulses), 200)))
    rx = [host[i].to(dev) for i in sub]
    Js = [pulses[i][1] for i in sub]
    outs = bank.correlate(rx, Js)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ms_bank = _time_steps(lambda: bank.correlate(rx, Js, out=outs), 3, 1, stream)
    plan_cache, plans, prx, pouts = {}, [], [], []
    for i, x, J, o in zip(sub, rx, Js, outs):
        for e in range(bank.eligible(pulses[i][0])):
            key = (e, J)
            if key not in plan_cache:
                plan_cache[key] = S.plan_create("cdf97", J, refs[e])
            plans.append(plan_cache[key])
            prx.append(x)
            pouts.append(o[e])
    b32 = S.Batch(plans, [x.numel() for x in prx])
    b32.tune(prx, pouts)
    ms_fp32 = _time_steps(lambda: b32.run(prx, pouts), 3, 1, stream)
    ms_pp = plain_per_pulse(S, plans, prx, pouts)
    sub_samples = sum(pulses[i][0] for i in sub)
    log(f"bank FP16 hi+lo: {ms_bank:.2f} ms, FP32 uneven batch: {ms_fp32:.2f} ms, FP32 plain "
        f"per-pulse path: {ms_pp:.2f} ms for {len(sub)} requests ({len(plans)} reference "
        f"correlations)")
    b32.free()
    for p in plan_cache.values():
        p.free()
    return {"requests": len(sub), "samples": sub_samples, "bank_ms": ms_bank, "fp32_ms": ms_fp32,
            "fp32_per_pulse_ms": ms_pp,
            "bank_samples_per_s": sub_samples / (ms_bank * 1e-3),
            "fp32_samples_per_s": sub_samples / (ms_fp32 * 1e-3)}


if __name__ == "__main__":
    main()
