"""Benchmark: BLS trial-periods x points per second on one MI355X.

One step = the whole search of the uniform batch workload (4096 light curves
x N = 2000 epochs, 20000 shared log-spaced trial periods 0.2-10 d, 300 phase
bins, box duty cycles 0.01-0.10) with the inputs already in HBM: prep
(centring, t0, fixed-point encoding), fold + bin, box scan, per-period argmax
and per-curve best period, all in the HIP library, replayed as one HIP graph.

Prints ONE JSON line (rank 0) with the metric, the roofline of the dominant
kernel (the search kernel) and the FP64 CPU oracle timed on a bounded sample
of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU issue rate of gfx950: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# 32- or 64-bit add/mul/compare per lane per clock (= 78.6 TFLOP/s FP64 or
# non-packed FP32 when an FMA counts as two).
PEAK_VALU_OPS = 256 * 4 * 16 * 2.4e9
# Algorithmic operations: per trial-period x point the fold (multiply,
# floor, subtract, multiply, truncate) and one accumulation; per box
# evaluation two running sums, W - R, R (W - R), S^2 and one comparison.
OPS_PER_TRIAL_POINT = 6
OPS_PER_BOX_EVAL = 6


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_baseline(batch, budget_s: float):
    """FP64 oracle on the first curves of the batch until budget_s elapses."""
    import numpy as np

    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or \
        os.cpu_count()
    oracle.build(force=False)
    done_pp = 0.0
    t0 = time.perf_counter()
    ncur = 0
    for c in range(batch.ncurves):
        lc = batch.curve(c)
        oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                      lc.qmax, nthreads=threads)
        done_pp += float(lc.n) * lc.periods.size
        ncur += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    del np
    return {"value": done_pp / el, "unit": "trial-periods*points/s",
            "cores": threads, "kind": "oracle",
            "sample": "first %d of %d curves, all %d periods each, %.1f s"
                      % (ncur, batch.ncurves, batch.periods.size, el)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--curves", type=int, default=4096)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the search shards by curve with "
              "no collective, and this build measures the single-GPU kernel "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1112_1701_amd as bls
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(0)
    log("generating workload")
    b = synth.config2(args.curves)
    nres = b.ncurves * b.periods.size
    t = torch.tensor(b.t, device=dev)
    x = torch.tensor(b.x, device=dev)
    per = torch.tensor(b.periods, device=dev)
    sr = torch.empty(nres, device=dev, dtype=torch.float32)
    dp = torch.empty(nres, device=dev, dtype=torch.float32)
    js = torch.empty(nres, device=dev, dtype=torch.int32)
    ks = torch.empty(nres, device=dev, dtype=torch.int32)
    bi = torch.empty(b.ncurves, device=dev, dtype=torch.int64)
    nbins, qmin, qmax = int(b.nbins[0]), float(b.qmin[0]), float(b.qmax[0])
    cap = dict(max_curves=b.ncurves, max_points=b.total_points(),
               max_periods=nres)

    def call(plan):
        bls.bls_search_device(plan, b.n_off, t, x, None, per, None, nbins,
                              qmin, qmax, sr, dp, js, ks, bi)

    plan = bls.Plan(**cap)
    stream = torch.cuda.ExternalStream(bls.bls_get_stream(plan.handle))
    log("warmup", args.warmup)
    for _ in range(max(args.warmup, 1)):
        call(plan.handle)
        bls.bls_synchronize(plan.handle)
    st = bls.bls_last_stats(plan.handle)

    log("timed", args.steps)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(args.steps):
        call(plan.handle)
        evs[k + 1].record(stream)
    bls.bls_synchronize(plan.handle)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    dev_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    pp = st["trial_points"]
    evals = st["box_evals"]
    value = pp / (ms_step * 1e-3)

    # Dominant kernel alone: the same launch without a graph, bracketed by
    # HIP events on the plan's stream.
    log("kernel timing")
    kplan = bls.Plan(flags=bls.BLS_NO_GRAPH, **cap)
    kms = []
    for _ in range(max(args.steps, 3)):
        call(kplan.handle)
        bls.bls_synchronize(kplan.handle)
        kms.append(bls.bls_last_stats(kplan.handle)["search_ms"])
    kst = bls.bls_last_stats(kplan.handle)
    kplan.close()
    k_ms = float(np.mean(kms))
    ops = OPS_PER_TRIAL_POINT * pp + OPS_PER_BOX_EVAL * evals
    achieved = ops / (k_ms * 1e-3) / 1e12
    peak = PEAK_VALU_OPS / 1e12

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(b, args.cpu_budget)
    plan.close()

    out = {
        "metric": "BLS trial-periods*points/s on 1 MI355X",
        "value": value,
        "unit": "trial-periods*points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 phase, exact int64 bins, f32 scan",
        "data": "synthetic",
        "config": {"workload": "uniform batch: %d light curves x N=2000, "
                               "20000 log periods 0.2-10 d, nbins=300, "
                               "q 0.01-0.10, unit weights" % b.ncurves,
                   "curves": b.ncurves, "points": int(b.total_points()),
                   "periods": int(b.periods.size), "nbins": nbins,
                   "parallelism": "1 GPU"},
        "box_evals_per_s": evals / (ms_step * 1e-3),
        "device_ms_per_step": float(np.median(dev_ms)),
        "search_kernel_ms": k_ms,
        "launch": {"grid": kst["grid"], "block": kst["block"],
                   "lds_bytes": kst["lds_bytes"],
                   "work_items": kst["work_items"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": None},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
