"""Benchmark: BLS trial-periods x points per second on one MI355X.

Default run (the headline line): one step = the whole search of the
high-cadence long-baseline workload (256 light curves x N = 50000 epochs on a
1-minute grid over 120 nights, 100000 shared log-spaced trial periods
0.1-20 d, 1000 phase bins, box duty cycles 0.005-0.05), the largest
single-GPU workload in trial-period x points, with the inputs already in HBM:
prep (centring, t0, fixed-point encoding), fold + bin, box scan, per-period
argmax and per-curve best period, all in the HIP library, replayed as HIP
graphs.  The search kernel's duration is read from the HIP events the library
records around it on its stream in every timed step.  Prints ONE JSON line
with the metric, the roofline of the dominant kernel (the search kernel,
per-unit operation counts against the published FP64/FP32 peaks), its LDS
traffic against the LDS peak, the FP64 CPU oracle timed on a bounded sample
of the same workload, and as extra keys: the uniform and uneven batch
workloads' throughput, the served form's p50/p99 latency at two arrival
rates, and the end-to-end time of the host-array call (PCIe included).

--workload picks another batch workload for the headline (uniform, uneven,
plain); --no-extras drops the extra keys (profiling runs).

--suite: one JSON line per workload (plain, uniform, uneven, long baseline):
batched throughput, the plain per-curve GPU form for comparison, and the
oracle; then the serving workload swept over Poisson arrival rates with
p50/p99 latency; then the eclipse-window, variability and unbinned
workloads, each with its kernel time, roofline and oracle.

--copy-calibration: three plain device copies of 1 GiB and nothing else,
the reference run that scales the HBM traffic counters (FETCH_SIZE,
WRITE_SIZE) to bytes.

--probes: micro-benchmarks of LDS atomic and read rates and VALU issue rates
(libbls_probes.so), the measured basis of the kernel design notes.
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

# Published MI355X peaks (dense, no sparsity).
FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# LDS: 128 bytes per clock per CU (32 banks of 4 bytes), 256 CUs, 2.4 GHz.
LDS_PEAK_TBS = 128 * 256 * 2.4e9 / 1e12
# Algorithmic work of the binned search, per unit:
#   per trial-period x point, the fold in FP64: multiply d f, floor,
#   subtract (the phase), multiply by nbins, truncate: 5 operations;
#   per box evaluation, FP32: the two window sums, theta R, S^2,
#   S^2 - theta R (W - R), the comparison and its selects: 10 operations.
# The low ends of the ranges in the design notes, so the fraction is not
# inflated.  FP64 operations count against the FP64 peak, FP32 ones against
# the FP32 peak; the roofline quotes FP32-equivalent TFLOP/s (an FP64
# operation counts as two, the ratio of the peaks).
FP64_OPS_PER_TRIAL_POINT = 5
FP32_OPS_PER_BOX_EVAL = 10
# LDS bytes per unit: one 8-byte atomic per trial-period x point (two for
# weighted curves), one 8-byte read per box evaluation.
LDS_BYTES_PER_TRIAL_POINT = 8
LDS_BYTES_PER_BOX_EVAL = 8
# The former issue-slot count (FP32 issue slots: 10 per trial-period x point,
# 6 per box evaluation, two FLOP per slot), kept as a separate figure.
SLOTS_PER_TRIAL_POINT = 10
SLOTS_PER_BOX_EVAL = 6
FP32_SLOTS_PER_S = 256 * 128 * 2.4e9
ALU_PEAK_TFLOPS = 2 * FP32_SLOTS_PER_S / 1e12


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(batch, budget_s: float):
    """FP64 oracle on whole curves of the batch, in order, until budget_s."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or \
        os.cpu_count()
    oracle.build(force=False)
    done_pp = done_ev = 0.0
    t0 = time.perf_counter()
    ncur = 0
    for c in range(batch.ncurves):
        lc = batch.curve(c)
        o = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                          lc.qmax, nthreads=threads)
        done_pp += float(lc.n) * lc.periods.size
        done_ev += float(lc.nbins) * (o.kmax - o.kmin + 1) * lc.periods.size
        ncur += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": done_pp / el, "unit": "trial-periods*points/s",
            "cores": threads, "kind": "oracle",
            "sample": "first %d of %d curves, all their periods, %.1f s"
                      % (ncur, batch.ncurves, el),
            "box_evals_per_s": done_ev / el, "cpu_model": cpu_model()}


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
    """Graph-replayed steps, bracketed by device synchronizations.

    Returns (ms per step, call statistics, search-kernel ms of each timed
    step from the events the library records around the kernel on its
    stream; the last 64 steps when there are more).
    """
    import torch
    plan = bls.Plan(**db.cap)
    for _ in range(max(warmup, 1)):
        db.call(bls, plan.handle)
        bls.bls_synchronize(plan.handle)
    st = bls.bls_last_stats(plan.handle)
    bls.bls_kernel_times_reset(plan.handle)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        db.call(bls, plan.handle)
    bls.bls_synchronize(plan.handle)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms = bls.bls_kernel_times(plan.handle, min(steps, 64))
    plan.close()
    return (t1 - t0) * 1e3 / steps, st, kms


def time_kernel(bls, db, reps):
    """The search kernel of non-graph calls (HIP events around the launch)."""
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


def time_host_arrays(bls, b, reps=2):
    """End to end from host arrays (bls_search_batch): uploads, the search,
    downloads and the widening to FP64 outputs; the last of reps calls."""
    with bls.Plan(max_curves=b.ncurves, max_points=b.total_points(),
                  max_periods=int(b.p_off[-1]) if b.p_off is not None
                  else b.ncurves * b.periods.size,
                  max_nbins=int(max(b.nbins))) as p:
        for _ in range(reps):
            t0 = time.perf_counter()
            bls.bls_search_batch(p.handle, b.n_off, b.t, b.x, b.w, b.periods,
                                 b.p_off, b.nbins, b.qmin, b.qmax)
            el = time.perf_counter() - t0
        st = bls.bls_last_stats(p.handle)
    return {"ms": el * 1e3, "device_ms": st["total_ms"],
            "search_kernel_ms": st["search_ms"],
            "trial_points_per_s": b.trial_points() / el}


KERNEL_SOURCE = os.path.join(ROOT, "paper_1112_1701_amd", "csrc", "bls_kernels.hip")
PROFILE_TAG = {"long": "long256", "uniform": "uniform4096",
               "uneven": "uneven10000", "plain": "plain1"}


def _profile_record(kind, workload):
    """key: value lines of profiles/search_kernel_<workload>_<kind>.txt, or
    None when missing or taken on another version of the kernel source (the
    file records the SHA-256 of the source its counters were taken on)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "search_kernel_%s_%s.txt"
                        % (PROFILE_TAG.get(workload, workload), kind))
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and not line.startswith((" ", "#")):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256") != src:
        return None
    return vals


def measured_traffic(workload):
    """HBM bytes per search-kernel launch from the committed counter runs."""
    vals = _profile_record("traffic", workload)
    try:
        return float(vals["hbm_bytes_per_launch"]) if vals else None
    except (KeyError, ValueError):
        return None


def roofline(pp, evals, k_ms, traffic=None):
    """The search kernel against the published FP64 and FP32 peaks: the
    algorithmic operations (FP64_OPS_PER_TRIAL_POINT, FP32_OPS_PER_BOX_EVAL)
    over the launch's duration, in FP32-equivalent TFLOP/s."""
    t = k_ms * 1e-3
    flop32 = 2 * FP64_OPS_PER_TRIAL_POINT * pp + FP32_OPS_PER_BOX_EVAL * evals
    achieved = flop32 / t / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP32_PEAK_TFLOPS,
            "traffic": traffic}


def issue_slot_fraction(pp, evals, k_ms):
    """The former figure: FP32 issue slots of the kernel's own instruction
    mix over the issue peak."""
    slots = SLOTS_PER_TRIAL_POINT * pp + SLOTS_PER_BOX_EVAL * evals
    return 2 * slots / (k_ms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS


def lds_roofline(pp, evals, k_ms, weighted, workload):
    """Algorithmic LDS bytes of the search kernel over the LDS peak, with
    the bank-conflict rate and LDS activity of the committed counter run."""
    nb = (2 if weighted else 1) * LDS_BYTES_PER_TRIAL_POINT * pp + \
        LDS_BYTES_PER_BOX_EVAL * evals
    achieved = nb / (k_ms * 1e-3) / 1e12
    out = {"achieved": achieved, "peak": LDS_PEAK_TBS, "unit": "TB/s",
           "frac": achieved / LDS_PEAK_TBS, "bytes": nb,
           "bank_conflict_frac": None, "lds_active_frac": None}
    vals = _profile_record("lds", workload)
    if vals:
        for k in ("bank_conflict_frac", "lds_active_frac"):
            try:
                out[k] = float(vals[k])
            except (KeyError, ValueError):
                pass
    return out


WORKLOADS = {
    "long": ("high-cadence long baseline: 256 light curves x N=50000 on a "
             "1-minute grid over 120 nights, 100000 log periods 0.1-20 d, "
             "nbins=1000, q 0.005-0.05, unit weights"),
    "uniform": ("uniform batch: 4096 light curves x N=2000, 20000 log periods "
                "0.2-10 d, nbins=300, q 0.01-0.10, unit weights"),
    "uneven": ("uneven batch: 10000 light curves, N log-uniform 200-10000, "
               "5000-40000 own log periods 0.2-10 d, nbins 200-500, "
               "q 0.01-0.10, weights 1/sigma^2"),
    "plain": ("plain: 1 light curve x N=1000, 5000 log periods 0.2-10 d, "
              "nbins=200, q 0.01-0.10"),
}


def _generate(name):
    import synth
    return {"plain": lambda: _as_batch(synth.config1()),
            "uniform": synth.config2, "uneven": synth.config3,
            "long": synth.config4}[name]()


def extra_batch(bls, name, steps):
    """Graph-replayed throughput of another batch workload."""
    b = _generate(name)
    db = DeviceBatch(b)
    ms_step, st, kms = time_batched(bls, db, steps, 1)
    pp, evals = st["trial_points"], st["box_evals"]
    k_ms = sum(kms) / len(kms)
    out = {"workload": WORKLOADS[name], "ms_per_step": ms_step,
           "trial_points_per_s": pp / (ms_step * 1e-3),
           "box_evals_per_s": evals / (ms_step * 1e-3),
           "search_kernel_ms": k_ms,
           "roofline_frac": roofline(pp, evals, k_ms)["frac"]}
    del db
    return out


def headline(args):
    import paper_1112_1701_amd as bls
    import torch
    torch.cuda.set_device(0)
    log("generating workload", args.workload)
    b = _generate(args.workload)
    weighted = b.w is not None
    db = DeviceBatch(b)
    log("timed", args.steps)
    ms_step, st, kms = time_batched(bls, db, args.steps, args.warmup)
    pp, evals = st["trial_points"], st["box_evals"]
    k_ms = sum(kms) / len(kms)
    extras = {}
    if not args.no_extras:
        log("end to end from host arrays")
        extras["end_to_end_host_arrays"] = time_host_arrays(bls, b)
        del db
        for name in ("uniform", "uneven"):
            if name != args.workload:
                log("extra", name)
                extras[name] = extra_batch(bls, name, 3)
        log("serving")
        recs = suite_serving(bls, [500.0, 1000.0], 300, 3000, 3.0)
        extras["served"] = {
            "workload": "Poisson arrivals; requests N log-U[500, 20000], "
                        "5000-100000 log periods 0.2-10 d, nbins 200-1000",
            "rates": [{k: r[k] for k in ("rate_req_per_s", "p50_ms",
                                         "p99_ms", "trial_points_per_s",
                                         "completed_per_s")}
                      for r in recs]}
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
        "config": {"workload": WORKLOADS[args.workload],
                   "curves": b.ncurves, "points": int(b.total_points()),
                   "trial_points": pp, "box_evals": evals,
                   "parallelism": "1 GPU"},
        "box_evals_per_s": evals / (ms_step * 1e-3),
        "search_kernel_ms": k_ms,
        "search_kernel_ms_per_step": kms,
        "launch": {"grid": st["grid"], "block": st["block"],
                   "lds_bytes": st["lds_bytes"],
                   "work_items": st["work_items"]},
        "roofline": roofline(pp, evals, k_ms, measured_traffic(args.workload)),
        "issue_slot_frac": issue_slot_fraction(pp, evals, k_ms),
        "lds_roofline": lds_roofline(pp, evals, k_ms, weighted,
                                     args.workload),
        "cpu_baseline": cpu,
    }
    out.update(extras)
    print(json.dumps(out), flush=True)


def suite_batch(name, b, args, bls):
    log("suite", name)
    db = DeviceBatch(b)
    ms_step, st, kms = time_batched(bls, db, args.suite_steps, 1)
    k_ms = sum(kms) / len(kms)
    _, kst = time_kernel(bls, db, 2)
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
           "issue_slot_frac": issue_slot_fraction(pp, evals, k_ms),
           "lds_roofline": lds_roofline(pp, evals, k_ms, b.w is not None,
                                        name),
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


# Algorithmic operations of the other workloads (per unit, stated in the
# design notes): eclipse window: per point x period the fold (multiply,
# floor, fract, multiply, truncate) and two LDS min/max updates, per
# (period, trial epoch) one window decision (min, max, compare, count);
# unbinned search: per point x period the fold and rank (10), per run step
# the two exact sums, span and gap distances, S^2, R (W - R), compare (8).
# FP32 issue slots of the other searches (their work is FP64 and integer,
# two slots per operation): the eclipse window's fold (multiply, fractional
# part, multiply, truncate, address) per point x period and four integer
# operations per epoch decision; the unbinned search's phase and counting
# sort (10 operations) per point x period and its 8 integer operations per
# run step.
SLOTS_WINDOW_PP, SLOTS_WINDOW_EPOCH = 10, 8
SLOTS_UNBINNED_PP, SLOTS_UNBINNED_STEP = 20, 16


def _alu_roofline(slots, k_ms):
    achieved = 2 * slots / (k_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / ALU_PEAK_TFLOPS,
            "traffic": None}


def _median(v):
    v = sorted(v)
    return v[len(v) // 2]


def suite_window(args, bls):
    """Eclipse detection efficiency of 64 field cadences x 100000 periods."""
    import numpy as np
    import torch

    import synth
    log("suite window")
    b = synth.cadence_batch()
    dev = torch.device("cuda:0")
    t = torch.tensor(b.t, device=dev)
    per = torch.tensor(b.periods, device=dev)
    obs = torch.empty(b.ncurves * b.periods.size, device=dev,
                      dtype=torch.int32)
    with bls.Plan(max_curves=b.ncurves, max_points=b.total_points(),
                  max_periods=obs.numel()) as p:
        kms, wall = [], []
        for r in range(args.suite_steps + 1):
            t0 = time.perf_counter()
            bls.bls_eclipse_window_device(p.handle, b.n_off, t, per, None,
                                          1000, 0.02, 2, obs)
            wall.append((time.perf_counter() - t0) * 1e3)
            kms.append(bls.bls_last_stats(p.handle)["search_ms"])
            st = bls.bls_last_stats(p.handle)
    k_ms, w_ms = _median(kms[1:]), _median(wall[1:])
    pp, dec = st["trial_points"], st["box_evals"]
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sub = b.periods[::50]
        t0 = time.perf_counter()
        done = 0.0
        for c in range(b.ncurves):
            tc = b.curve(c).t
            oracle.eclipse_window(tc, None, sub, 1000, 0.02, 2)
            done += float(tc.size) * sub.size
            if time.perf_counter() - t0 > args.cpu_budget / 3:
                break
        el = time.perf_counter() - t0
        cpu = {"value": done / el, "unit": "trial-periods*points/s",
               "cores": os.cpu_count(), "kind": "oracle",
               "sample": "%d cadences x every 50th period" % (c + 1)}
    return {"workload": "eclipse window: 64 field cadences x 100000 log "
                        "periods 0.1-10 d, 1000 epochs, 0.02 d eclipses, "
                        "two required",
            "points": int(b.total_points()), "trial_points": pp,
            "epoch_decisions": dec, "kernel_ms": k_ms, "call_ms": w_ms,
            "trial_points_per_s": pp / (k_ms * 1e-3),
            "launch": {"grid": st["grid"], "lds_bytes": st["lds_bytes"],
                       "work_items": st["work_items"]},
            "roofline": _alu_roofline(SLOTS_WINDOW_PP * pp +
                                      SLOTS_WINDOW_EPOCH * dec, k_ms),
            "cpu_baseline": cpu}


def suite_variability(args, bls):
    """High-variability pre-search of one 100000-star pointing."""
    import torch

    import synth
    log("suite variability")
    b, mag, chip_off, _ = synth.variability_field()
    dev = torch.device("cuda:0")
    nc, nk = b.ncurves, len(chip_off) - 1
    x = torch.tensor(b.x, device=dev)
    m = torch.tensor(mag, device=dev)
    f64, i32 = torch.float64, torch.int32
    out = dict(rms=torch.empty(nc, device=dev, dtype=f64),
               bin=torch.empty(nc, device=dev, dtype=i32),
               flag=torch.empty(nc, device=dev, dtype=i32),
               bin_mean=torch.empty(nk * 60, device=dev, dtype=f64),
               bin_std=torch.empty(nk * 60, device=dev, dtype=f64),
               bin_count=torch.empty(nk * 60, device=dev, dtype=i32))
    with bls.Plan(max_curves=nc, max_points=b.total_points(),
                  max_periods=16) as p:
        kms, wall = [], []
        for r in range(args.suite_steps + 3):
            t0 = time.perf_counter()
            bls.bls_variability_device(p.handle, b.n_off, x, None, m,
                                       chip_off, 60, out, origin=14.0)
            wall.append((time.perf_counter() - t0) * 1e3)
            kms.append(bls.bls_last_stats(p.handle)["search_ms"])
    k_ms, w_ms = _median(kms[1:]), _median(wall[1:])
    npts = int(b.total_points())
    nbytes = 8.0 * npts + 40.0 * nc
    achieved = nbytes / (k_ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        oracle.variability(b.x, None, b.n_off, mag, chip_off, 60,
                           origin=14.0)
        el = time.perf_counter() - t0
        cpu = {"value": npts / el, "unit": "points/s", "cores": 1,
               "kind": "oracle", "sample": "the whole pointing"}
    return {"workload": "variability pre-search: 100000 stars on 11 chips, "
                        "140-300 epochs, 60 bins of 0.1 mag",
            "points": npts, "stars": nc, "kernel_ms": k_ms, "call_ms": w_ms,
            "points_per_s": npts / (k_ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None},
            "cpu_baseline": cpu}


def suite_unbinned(args, bls):
    """Unbinned search: 8 noisy copies of the plain curve, 5000 periods."""
    import numpy as np
    import torch

    import synth
    log("suite unbinned")
    lc = synth.config1()
    ncur = 8
    rng = np.random.default_rng(3)
    xs = [lc.x + rng.normal(0, 0.001, lc.n) for _ in range(ncur)]
    n_off = np.arange(0, (ncur + 1) * lc.n, lc.n, dtype=np.int64)
    dev = torch.device("cuda:0")
    t = torch.tensor(np.tile(lc.t, ncur), device=dev)
    x = torch.tensor(np.concatenate(xs), device=dev)
    per = torch.tensor(lc.periods, device=dev)
    mres = ncur * lc.periods.size
    outs = [torch.empty(mres, device=dev, dtype=torch.float32),
            torch.empty(mres, device=dev, dtype=torch.float32),
            torch.empty(mres, device=dev, dtype=torch.int32),
            torch.empty(mres, device=dev, dtype=torch.int32),
            torch.empty(ncur, device=dev, dtype=torch.int64)]
    with bls.Plan(max_curves=ncur, max_points=int(n_off[-1]),
                  max_periods=mres) as p:
        kms = []
        for r in range(args.suite_steps + 1):
            bls.bls_search_unbinned_device(p.handle, n_off, t, x, None, per,
                                           None, lc.qmin, lc.qmax, *outs)
            bls.bls_synchronize(p.handle)
            kms.append(bls.bls_last_stats(p.handle)["search_ms"])
        st = bls.bls_last_stats(p.handle)
    k_ms = _median(kms[1:])
    pp, steps = st["trial_points"], st["box_evals"]
    long_rec = _unbinned_long_curves(args, bls)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        sub = lc.periods[::10]
        t0 = time.perf_counter()
        oracle.unbinned(lc.t, xs[0], None, sub, lc.qmin, lc.qmax)
        el = time.perf_counter() - t0
        cpu = {"value": lc.n * sub.size / el,
               "unit": "trial-periods*points/s", "cores": os.cpu_count(),
               "kind": "oracle", "sample": "1 curve x every 10th period"}
    return {"workload": "unbinned search: 8 x N=1000, 5000 log periods "
                        "0.2-10 d, q 0.01-0.10",
            "trial_points": pp, "run_steps_est": steps, "kernel_ms": k_ms,
            "trial_points_per_s": pp / (k_ms * 1e-3),
            "launch": {"grid": st["grid"], "lds_bytes": st["lds_bytes"],
                       "work_items": st["work_items"]},
            "roofline": _alu_roofline(SLOTS_UNBINNED_PP * pp +
                                      SLOTS_UNBINNED_STEP * steps, k_ms),
            "long_curves": long_rec,
            "cpu_baseline": cpu}


def _unbinned_long_curves(args, bls):
    """Unbinned search of curves too long for LDS (their per-point arrays in
    the device workspace): 4 curves of 20000 points, 2000 periods."""
    import numpy as np
    import torch

    import synth
    log("suite unbinned long curves")
    ncur, n = 4, 20000
    lcs = [synth.small_curve(7100 + k, n, nperiods=2000, nbins=64, qmin=0.01,
                             qmax=0.1) for k in range(ncur)]
    n_off = np.arange(0, (ncur + 1) * n, n, dtype=np.int64)
    dev = torch.device("cuda:0")
    t = torch.tensor(np.concatenate([lc.t for lc in lcs]), device=dev)
    x = torch.tensor(np.concatenate([lc.x for lc in lcs]), device=dev)
    per = torch.tensor(lcs[0].periods, device=dev)
    mres = ncur * lcs[0].periods.size
    outs = [torch.empty(mres, device=dev, dtype=torch.float32),
            torch.empty(mres, device=dev, dtype=torch.float32),
            torch.empty(mres, device=dev, dtype=torch.int32),
            torch.empty(mres, device=dev, dtype=torch.int32),
            torch.empty(ncur, device=dev, dtype=torch.int64)]
    with bls.Plan(max_curves=ncur, max_points=int(n_off[-1]),
                  max_periods=mres) as p:
        kms = []
        for r in range(args.suite_steps + 1):
            bls.bls_search_unbinned_device(p.handle, n_off, t, x, None, per,
                                           None, 0.01, 0.1, *outs)
            bls.bls_synchronize(p.handle)
            kms.append(bls.bls_last_stats(p.handle)["search_ms"])
        st = bls.bls_last_stats(p.handle)
    k_ms = _median(kms[1:])
    return {"workload": "4 x N=20000 (device-workspace path), 2000 log "
                        "periods, q 0.01-0.10",
            "kernel_ms": k_ms,
            "trial_points_per_s": st["trial_points"] / (k_ms * 1e-3),
            "run_steps_est": st["box_evals"],
            "launch": {"grid": st["grid"], "work_items": st["work_items"]}}


def suite_detect(args, bls):
    """Detection statistics of the uniform batch's 4096 periodograms."""
    import torch

    import synth
    log("suite detect")
    b = synth.config2(4096)
    db = DeviceBatch(b)
    with bls.Plan(**db.cap) as p:
        db.call(bls, p.handle)
        bls.bls_synchronize(p.handle)
        kms = []
        for r in range(args.suite_steps + 1):
            det = bls.bls_detect_device(p.handle, b.n_off, db.per, None, 300,
                                        0.01, 0.1, db.outs[0], max_peaks=8,
                                        window=0.01, sde_threshold=7.0)
            kms.append(bls.bls_last_stats(p.handle)["search_ms"])
    k_ms = _median(kms[1:])
    m = float(b.ncurves) * b.periods.size
    # algorithmic bytes: every SR value once, the shared period grid once and
    # one detection record per curve (the kernel reads a curve's SR values
    # once, plus a thread's slice again on a rare refill)
    import ctypes

    from paper_1112_1701_amd import _lib
    nbytes = (4.0 * m + 8.0 * b.periods.size +
              float(b.ncurves) * ctypes.sizeof(_lib.BlsDetection))
    achieved = nbytes / (k_ms * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        import numpy as np

        import oracle
        sr = db.outs[0].cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        ncur = 0
        for c in range(b.ncurves):
            oracle.detect(sr[c * b.periods.size:(c + 1) * b.periods.size],
                          b.periods, max_peaks=8, window=0.01, threshold=7.0)
            ncur += 1
            if time.perf_counter() - t0 > args.cpu_budget / 3:
                break
        el = time.perf_counter() - t0
        cpu = {"value": ncur * b.periods.size / el, "unit": "periods/s",
               "cores": 1, "kind": "oracle",
               "sample": "first %d periodograms" % ncur}
    return {"workload": "detection statistics: 4096 periodograms x 20000 "
                        "periods, 8 peaks, window 0.01",
            "periods": m, "kernel_ms": k_ms,
            "periods_per_s": m / (k_ms * 1e-3),
            "candidates": int(sum(d["candidate"] for d in det)),
            "roofline": {"bound": "hbm", "achieved": achieved,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": None},
            "cpu_baseline": cpu}


def suite_recovery(args, bls):
    """Injection-recovery: 4096 box eclipses injected into copies of one
    survey cadence, each copy searched over 20000 trial periods with its
    detection statistics, recovered fraction per injected-period decade."""
    import numpy as np
    import torch

    import synth
    log("suite recovery")
    s = synth.injection_set(4096)
    ninj, n = s.base.shape
    m = s.periods.size
    dev = torch.device("cuda:0")
    t = torch.tensor(s.t, device=dev)
    base = torch.tensor(s.base, device=dev)
    per = torch.tensor(s.periods, device=dev)
    thr, ptol = 7.0, 0.01
    with bls.Plan(max_curves=ninj, max_points=ninj * n,
                  max_periods=ninj * m) as p:
        kms, wall = [], []
        for r in range(args.suite_steps + 1):
            t0 = time.perf_counter()
            res = bls.bls_injection_recovery_device(
                p.handle, t, None, base, s.period, s.phase, s.q, s.depth,
                per, s.nbins, s.qmin, s.qmax, sde_threshold=thr, ptol=ptol)
            wall.append((time.perf_counter() - t0) * 1e3)
            kms.append(bls.bls_last_stats(p.handle)["search_ms"])
        st = bls.bls_last_stats(p.handle)
    k_ms, w_ms = _median(kms[1:]), _median(wall[1:])
    pp, evals = st["trial_points"], st["box_evals"]
    edges = [0.3, 1.0, 3.0, 10.0]
    frac = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (s.period >= lo) & (s.period < hi)
        frac.append({"period_d": [lo, hi], "injections": int(sel.sum()),
                     "recovered_frac": float(np.mean(res["recovered"][sel]
                                                     == 1))})
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < args.cpu_budget / 3 and k < ninj:
            oracle.recovery(s.t, None, s.base[k:k + 1], s.period[k],
                            s.phase[k], s.q[k], s.depth[k], s.periods,
                            s.nbins, s.qmin, s.qmax, sde_threshold=thr,
                            ptol=ptol)
            k += 1
        el = time.perf_counter() - t0
        cpu = {"value": k / el, "unit": "injections/s",
               "cores": os.cpu_count(), "kind": "oracle",
               "sample": "first %d injections, all periods" % k}
    return {"workload": "injection-recovery: 4096 box eclipses (P 0.3-10 d "
                        "log-uniform, q 0.01-0.05, depth 0.003-0.03, noise "
                        "0.01) in copies of one %d-epoch survey cadence, "
                        "20000 log periods 0.2-10 d, nbins=300, SDE >= 7, "
                        "period within 1%% (or half/double)" % n,
            "injections": ninj, "trial_points": pp, "box_evals": evals,
            "call_ms": w_ms, "search_kernel_ms": k_ms,
            "injections_per_s": ninj / (w_ms * 1e-3),
            "trial_points_per_s": pp / (w_ms * 1e-3),
            "recovered_frac": float(np.mean(res["recovered"] == 1)),
            "by_period": frac,
            "roofline": roofline(pp, evals, k_ms),
            "cpu_baseline": cpu}


def suite(args):
    import paper_1112_1701_amd as bls
    import synth
    import torch
    torch.cuda.set_device(0)
    names = args.workloads.split(",")
    extra = {"window": suite_window, "variability": suite_variability,
             "unbinned": suite_unbinned, "detect": suite_detect,
             "recovery": suite_recovery}
    for name in names:
        if name in extra:
            print(json.dumps(extra[name](args, bls)), flush=True)
            continue
        if name == "serving":
            recs = suite_serving(bls, [float(r) for r in
                                       args.rates.split(",")],
                                 args.pool, args.max_requests,
                                 args.seconds)
            print(json.dumps({"workload": "serving", "sweep": recs}),
                  flush=True)
            continue
        rec = suite_batch(name, _generate(name), args, bls)
        print(json.dumps(rec), flush=True)


def _as_batch(lc):
    import numpy as np

    import synth
    return synth.Batch(lc.t, lc.x, lc.w, np.array([0, lc.n], np.int64),
                       lc.periods, None, np.array([lc.nbins], np.int32),
                       np.array([lc.qmin]), np.array([lc.qmax]),
                       [lc.truth])


def probes():
    """Micro-benchmarks of the rates the search kernel's design rests on
    (libbls_probes.so): LDS atomics by width and type at random addresses,
    64-bit LDS reads by lane stride, VALU issue by instruction type.  One JSON
    line; rates per CU per clock at the device's reported peak clock."""
    import ctypes

    import torch
    torch.cuda.set_device(0)
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    clock_hz = 2.4e9
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1112_1701_amd",
                                   "libbls_probes.so"))
    for f in (lib.bls_probe_lds_atomic, lib.bls_probe_lds_read,
              lib.bls_probe_valu):
        f.restype = ctypes.c_int
    grid = cus * 8
    out = {"probe": "gfx950 rates", "cus": cus,
           "clock_hz_assumed": clock_hz, "grid": grid, "block": 256}
    ms = ctypes.c_double()

    def per_cu_clk(count, t_ms):
        return count / (t_ms * 1e-3) / cus / clock_hz

    atom = {}
    for name, kind in (("ds_add_u64", 0), ("ds_add_u32", 1),
                       ("ds_add_f32", 2)):
        for span in (1024, 4096):
            iters = 4096
            st = lib.bls_probe_lds_atomic(kind, span, iters, grid,
                                          ctypes.byref(ms))
            if st != 0:
                raise RuntimeError("probe %s failed: %d" % (name, st))
            n = grid * 256.0 * iters
            atom["%s_span%d" % (name, span)] = {
                "ms": ms.value, "per_s": n / (ms.value * 1e-3),
                "lanes_per_cu_clk": per_cu_clk(n, ms.value)}
    out["lds_atomics"] = atom
    rd = {}
    for stride in (1, 2, 8, 16, 17, 32):
        iters = 8192
        st = lib.bls_probe_lds_read(stride, iters, grid, ctypes.byref(ms))
        if st != 0:
            raise RuntimeError("probe read failed: %d" % st)
        n = grid * 256.0 * iters
        rd["lane_stride_%d" % stride] = {
            "ms": ms.value, "bytes_per_cu_clk": per_cu_clk(8 * n, ms.value)}
    out["lds_read_b64"] = rd
    va = {}
    for name, kind in (("v_fma_f32", 0), ("v_add_f32", 3), ("v_mul_f64", 1),
                       ("v_lshl_add_u32", 2)):
        iters = 16384
        st = lib.bls_probe_valu(kind, iters, grid, ctypes.byref(ms))
        if st != 0:
            raise RuntimeError("probe valu failed: %d" % st)
        waves = grid * 4.0 * 8 * iters
        va[name] = {"ms": ms.value,
                    "wave_instr_per_cu_clk": per_cu_clk(waves, ms.value)}
    out["valu"] = va
    print(json.dumps(out), flush=True)


def copy_calibration():
    """Three device copies of 2^28 float32 (1 GiB each), for the counters."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    log("copied 3 x 1 GiB")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="long",
                    choices=sorted(WORKLOADS))
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--suite", action="store_true")
    ap.add_argument("--workloads", default="plain,uniform,uneven,long,"
                    "serving,window,variability,unbinned,detect,recovery")
    ap.add_argument("--suite-steps", type=int, default=3)
    ap.add_argument("--rates", default="100,500,1000,2000,5000")
    ap.add_argument("--pool", type=int, default=300)
    ap.add_argument("--max-requests", type=int, default=1500)
    ap.add_argument("--seconds", type=float, default=3.0)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--probes", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the search shards by curve with "
              "no collective, and bench.py measures the single-GPU kernel "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
    elif args.probes:
        probes()
    elif args.suite:
        suite(args)
    else:
        headline(args)


if __name__ == "__main__":
    main()
