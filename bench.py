"""Benchmark: BLS trial-periods x points per second on one MI355X.

Default run (the headline line): one step = the whole search of the uniform
batch workload (4096 light curves x N = 2000 epochs, 20000 shared
log-spaced trial periods 0.2-10 d, 300 phase bins, box duty cycles
0.01-0.10) with the inputs already in HBM: prep (centring, t0, fixed-point
encoding), fold + bin, box scan, per-period argmax and per-curve best period,
all in the HIP library, replayed as one HIP graph.  Prints ONE JSON line with
the metric, the roofline of the dominant kernel (the search kernel) and the
FP64 CPU oracle timed on a bounded sample of the same workload.

--suite: one JSON line per workload (plain, uniform, uneven, long baseline):
batched throughput, the plain per-curve GPU form for comparison, and the
oracle; then the serving workload swept over Poisson arrival rates with
p50/p99 latency.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
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
    return {"value": done_pp / el, "unit": "trial-periods*points/s",
            "cores": threads, "kind": "oracle",
            "sample": "first %d of %d curves, all their periods, %.1f s"
                      % (ncur, batch.ncurves, el)}


class DeviceBatch:
    """A batch resident in device memory with its result tensors."""

    def __init__(self, b):
        import torch
        dev = torch.device("cuda:0")
        self.b = b
        self.nres = int(b.p_off[-1]) if b.p_off is not None else \
            b.ncurves * b.periods.size
        self.t = torch.tensor(b.t, device=dev)
        self.x = torch.tensor(b.x, device=dev)
        self.w = None if b.w is None else torch.tensor(b.w, device=dev)
        self.per = torch.tensor(b.periods, device=dev)
        self.outs = [torch.empty(self.nres, device=dev, dtype=torch.float32),
                     torch.empty(self.nres, device=dev, dtype=torch.float32),
                     torch.empty(self.nres, device=dev, dtype=torch.int32),
                     torch.empty(self.nres, device=dev, dtype=torch.int32),
                     torch.empty(b.ncurves, device=dev, dtype=torch.int64)]
        self.cap = dict(max_curves=b.ncurves, max_points=b.total_points(),
                        max_periods=self.nres, max_nbins=int(max(b.nbins)))

    def call(self, bls, plan):
        b = self.b
        bls.bls_search_device(plan, b.n_off, self.t, self.x, self.w, self.per,
                              b.p_off, b.nbins, b.qmin, b.qmax, *self.outs)


def time_batched(bls, db, steps, warmup):
    """Graph-replayed steps; returns (ms/step, stats, per-step device ms)."""
    import torch
    plan = bls.Plan(**db.cap)
    stream = torch.cuda.ExternalStream(bls.bls_get_stream(plan.handle))
    for _ in range(max(warmup, 1)):
        db.call(bls, plan.handle)
        bls.bls_synchronize(plan.handle)
    st = bls.bls_last_stats(plan.handle)
    torch.cuda.synchronize()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    evs[0].record(stream)
    for k in range(steps):
        db.call(bls, plan.handle)
        evs[k + 1].record(stream)
    bls.bls_synchronize(plan.handle)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.close()
    dev_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(steps)]
    return (t1 - t0) * 1e3 / steps, st, dev_ms


def time_kernel(bls, db, reps):
    """The search kernel alone (non-graph launch bracketed by HIP events)."""
    kplan = bls.Plan(flags=bls.BLS_NO_GRAPH, **db.cap)
    kms = []
    for _ in range(max(reps, 3)):
        db.call(bls, kplan.handle)
        bls.bls_synchronize(kplan.handle)
        kms.append(bls.bls_last_stats(kplan.handle)["search_ms"])
    kst = bls.bls_last_stats(kplan.handle)
    kplan.close()
    return sum(kms) / len(kms), kst


def time_plain(bls, db, max_curves, budget_s=5.0):
    """Plain per-curve GPU form: one synchronous, non-graph call per curve."""
    import torch
    b = db.b
    plan = bls.Plan(flags=bls.BLS_NO_GRAPH, **db.cap)
    done_pp, ncur = 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(min(max_curves, b.ncurves)):
        a, e = int(b.n_off[c]), int(b.n_off[c + 1])
        if b.p_off is None:
            pa, pe = 0, b.periods.size
        else:
            pa, pe = int(b.p_off[c]), int(b.p_off[c + 1])
        ra = pa if b.p_off is not None else c * b.periods.size
        outs = [o[ra:ra + (pe - pa)] for o in db.outs[:4]] + \
            [db.outs[4][c:c + 1]]
        bls.bls_search_device(
            plan.handle, [0, e - a], db.t[a:e], db.x[a:e],
            None if db.w is None else db.w[a:e], db.per[pa:pe], None,
            int(b.nbins[c]), float(b.qmin[c]), float(b.qmax[c]), *outs)
        bls.bls_synchronize(plan.handle)
        done_pp += float(e - a) * (pe - pa)
        ncur += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    plan.close()
    return {"value": done_pp / el, "curves": ncur, "seconds": el}


def roofline(pp, evals, k_ms):
    ops = OPS_PER_TRIAL_POINT * pp + OPS_PER_BOX_EVAL * evals
    achieved = ops / (k_ms * 1e-3) / 1e12
    peak = PEAK_VALU_OPS / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": peak,
            "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None}


def headline(args):
    import numpy as np

    import paper_1112_1701_amd as bls
    import synth
    import torch
    torch.cuda.set_device(0)
    log("generating workload")
    b = synth.config2(args.curves)
    db = DeviceBatch(b)
    log("timed", args.steps)
    ms_step, st, dev_ms = time_batched(bls, db, args.steps, args.warmup)
    pp, evals = st["trial_points"], st["box_evals"]
    log("kernel timing")
    k_ms, kst = time_kernel(bls, db, args.steps)
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(b, args.cpu_budget)
    out = {
        "metric": "BLS trial-periods*points/s on 1 MI355X",
        "value": pp / (ms_step * 1e-3),
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
                   "periods": int(b.periods.size), "nbins": 300,
                   "parallelism": "1 GPU"},
        "box_evals_per_s": evals / (ms_step * 1e-3),
        "device_ms_per_step": float(np.median(dev_ms)),
        "search_kernel_ms": k_ms,
        "launch": {"grid": kst["grid"], "block": kst["block"],
                   "lds_bytes": kst["lds_bytes"],
                   "work_items": kst["work_items"]},
        "roofline": roofline(pp, evals, k_ms),
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def suite_batch(name, b, args, bls):
    log("suite", name)
    db = DeviceBatch(b)
    ms_step, st, _ = time_batched(bls, db, args.suite_steps, 1)
    k_ms, kst = time_kernel(bls, db, 2)
    plain = time_plain(bls, db, 64)
    pp, evals = st["trial_points"], st["box_evals"]
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(b, args.cpu_budget / 2)
    rec = {"workload": name, "curves": b.ncurves,
           "points": int(b.total_points()),
           "trial_points": pp, "box_evals": evals,
           "batched": {"ms_per_step": ms_step,
                       "trial_points_per_s": pp / (ms_step * 1e-3),
                       "box_evals_per_s": evals / (ms_step * 1e-3)},
           "plain_per_curve": plain,
           "search_kernel_ms": k_ms,
           "launch": {"grid": kst["grid"], "lds_bytes": kst["lds_bytes"],
                      "work_items": kst["work_items"]},
           "roofline": roofline(pp, evals, k_ms),
           "cpu_baseline": cpu}
    del db
    return rec


def suite_serving(bls, rates, pool_size, max_requests, seconds):
    """Open-loop Poisson client at each rate; requests drawn from a pool."""
    import numpy as np

    import synth
    log("serving pool")
    pool = [lc for _, lc in synth.serving_requests(pool_size, 1.0)]
    recs = []
    for rate in rates:
        nreq = int(min(max_requests, rate * seconds))
        rng = np.random.default_rng(int(rate))
        gaps = rng.exponential(1.0 / rate, nreq)
        srv = bls.bls_server_create(max_slots=512, arena_bytes=8 << 30)
        try:
            # warm the kernels once, then measure
            lc = pool[0]
            tk = bls.bls_server_submit(srv, lc.t, lc.x, lc.w, lc.periods,
                                       lc.nbins, lc.qmin, lc.qmax)
            bls.bls_server_wait(srv, tk, 60.0)
            bls.bls_server_release(srv, tk)
            bls.bls_server_reset_stats(srv)
            t0 = time.perf_counter()
            tarr = 0.0
            tickets = []
            for k in range(nreq):
                tarr += gaps[k]
                while time.perf_counter() - t0 < tarr:
                    pass
                lc = pool[k % len(pool)]
                tickets.append(bls.bls_server_submit(
                    srv, lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                    lc.qmax))
            offered_s = time.perf_counter() - t0
            bls.bls_server_drain(srv, 600.0)
            st = bls.bls_server_get_stats(srv)
        finally:
            bls.bls_server_destroy(srv)
        rec = {"rate_req_per_s": rate, "requests": nreq,
               "offered_seconds": offered_s,
               "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
               "mean_ms": st["mean_ms"], "max_ms": st["max_ms"],
               "trial_points_per_s": st["trial_points"] / st["wall_s"],
               "completed_per_s": st["completed"] / st["wall_s"],
               "device_busy_frac": st["busy_s"] / st["wall_s"],
               "ticks": st["ticks"],
               "device_bytes_peak": st["device_bytes_peak"]}
        log("serving", json.dumps(rec))
        recs.append(rec)
    return recs


def suite(args):
    import paper_1112_1701_amd as bls
    import synth
    import torch
    torch.cuda.set_device(0)
    names = args.workloads.split(",")
    gens = {"plain": lambda: _as_batch(synth.config1()),
            "uniform": synth.config2, "uneven": synth.config3,
            "long": synth.config4}
    for name in names:
        if name == "serving":
            recs = suite_serving(bls, [float(r) for r in
                                       args.rates.split(",")],
                                 args.pool, args.max_requests,
                                 args.seconds)
            print(json.dumps({"workload": "serving", "sweep": recs}),
                  flush=True)
            continue
        rec = suite_batch(name, gens[name](), args, bls)
        print(json.dumps(rec), flush=True)


def _as_batch(lc):
    import numpy as np

    import synth
    return synth.Batch(lc.t, lc.x, lc.w, np.array([0, lc.n], np.int64),
                       lc.periods, None, np.array([lc.nbins], np.int32),
                       np.array([lc.qmin]), np.array([lc.qmax]),
                       [lc.truth])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--curves", type=int, default=4096)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--suite", action="store_true")
    ap.add_argument("--workloads", default="plain,uniform,uneven,long,serving")
    ap.add_argument("--suite-steps", type=int, default=3)
    ap.add_argument("--rates", default="100,500,1000,2000,5000")
    ap.add_argument("--pool", type=int, default=300)
    ap.add_argument("--max-requests", type=int, default=1500)
    ap.add_argument("--seconds", type=float, default=3.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the search shards by curve with "
              "no collective, and this build measures the single-GPU kernel "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.suite:
        suite(args)
    else:
        headline(args)


if __name__ == "__main__":
    main()
