"""Full-size workloads on the GPU, in the launch configuration bench.py times
(device arrays, persistent launch, autotuned tiles), checked against the FP64
oracle on sampled outputs: a few whole curves, plus random (curve, period)
pairs that the oracle computes one period at a time.  Each test writes its
error statistics (the per-configuration precision report) to
gpurun_out/precision_<workload>.json.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.parity import REL_TOL, check_curve, oracle_box_sr

pytestmark = pytest.mark.gpu
OUT = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(
    __file__))), "gpurun_out")


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bls():
    import paper_1112_1701_amd as bls
    bls._lib.load()
    return bls


def _run_device(bls, b):
    """Whole batch through bls_search_device; returns device result tensors."""
    import torch
    dev = torch.device("cuda:0")
    nres = int(b.p_off[-1]) if b.p_off is not None else \
        b.ncurves * b.periods.size
    t = torch.tensor(b.t, device=dev)
    x = torch.tensor(b.x, device=dev)
    w = None if b.w is None else torch.tensor(b.w, device=dev)
    per = torch.tensor(b.periods, device=dev)
    outs = [torch.empty(nres, device=dev, dtype=torch.float32),
            torch.empty(nres, device=dev, dtype=torch.float32),
            torch.empty(nres, device=dev, dtype=torch.int32),
            torch.empty(nres, device=dev, dtype=torch.int32),
            torch.empty(b.ncurves, device=dev, dtype=torch.int64)]
    cap = dict(max_curves=b.ncurves, max_points=b.total_points(),
               max_periods=nres, max_nbins=int(max(b.nbins)))
    with bls.Plan(**cap) as p:
        bls.bls_search_device(p.handle, b.n_off, t, x, w, per, b.p_off,
                              b.nbins, b.qmin, b.qmax, *outs)
        bls.bls_synchronize(p.handle)
        st = bls.bls_last_stats(p.handle)
    del t, x, w, per
    return outs, st


def _r_off(b, c):
    return int(b.p_off[c]) if b.p_off is not None else c * b.periods.size


def _sampled_pairs(b, outs, rng, npairs, label):
    """Oracle one period at a time on random (curve, period) pairs."""
    import torch
    cs = rng.integers(0, b.ncurves, npairs)
    ps = np.array([rng.integers(0, b.nperiods(int(c))) for c in cs])
    idx = torch.tensor([_r_off(b, int(c)) + int(p) for c, p in zip(cs, ps)],
                       device=outs[0].device)
    sr, dp, js, ks = [o[idx].cpu().numpy() for o in outs[:4]]
    rels, mism = [], 0
    for i, (c, p) in enumerate(zip(cs, ps)):
        lc = b.curve(int(c))
        P = lc.periods[int(p)]
        o = oracle.search(lc.t, lc.x, lc.w, [P], lc.nbins, lc.qmin, lc.qmax)
        if o.kwidth[0] < 0:
            assert sr[i] == 0 and ks[i] < 0, (label, c, p)
            continue
        rel = abs(float(sr[i]) - o.sr[0]) / o.sr[0]
        assert rel <= REL_TOL, (label, int(c), int(p), rel)
        rels.append(rel)
        if (js[i], ks[i]) != (o.jstart[0], o.kwidth[0]):
            mism += 1
            alt = oracle_box_sr(lc, P, int(js[i]), int(ks[i]), lc.nbins)
            assert alt >= (1 - REL_TOL) * o.sr[0], (label, int(c), int(p))
    return rels, mism


def _full_curves(b, outs, curves, label):
    rels, mism = [], 0
    bi_all = outs[4].cpu().numpy()
    for c in curves:
        lc = b.curve(c)
        a = _r_off(b, c)
        e = a + lc.periods.size
        g = dict(sr=outs[0][a:e].cpu().numpy(),
                 depth=outs[1][a:e].cpu().numpy(),
                 jstart=outs[2][a:e].cpu().numpy(),
                 kwidth=outs[3][a:e].cpu().numpy(), best_index=bi_all[c])
        o = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                          lc.qmax)
        st = check_curve(lc, g, o, label="%s curve %d" % (label, c))
        some = o.kwidth >= 0
        rels.extend((np.abs(g["sr"][some] - o.sr[some]) / o.sr[some]).tolist())
        mism += st["box_mismatch"]
    return rels, mism


def _report(name, stats, rels, mism, npairs, curves):
    rels = np.asarray(rels)
    rep = dict(workload=name, checked_periods=int(rels.size),
               sampled_pairs=npairs, full_curves=list(map(int, curves)),
               max_rel_sr_error=float(rels.max()) if rels.size else 0.0,
               p99_rel_sr_error=float(np.percentile(rels, 99))
               if rels.size else 0.0,
               box_mismatches_within_tolerance=int(mism),
               trial_points=stats["trial_points"],
               box_evals=stats["box_evals"], search_ms=stats["search_ms"],
               lds_bytes=stats["lds_bytes"], grid=stats["grid"])
    _say("report", json.dumps(rep))
    os.makedirs(OUT, exist_ok=True)
    with open(os.path.join(OUT, "precision_%s.json" % name), "w") as f:
        json.dump(rep, f, indent=1)


def test_uniform_batch_full_size(bls):
    """4096 curves x N = 2000, 20000 shared periods, 300 bins."""
    b = synth.config2()
    _say("uniform batch full size")
    outs, st = _run_device(bls, b)
    curves = [0, 1, 2047, 4095]
    rels, mism = _full_curves(b, outs, curves, "uniform")
    r2, m2 = _sampled_pairs(b, outs, np.random.default_rng(1), 300, "uniform")
    _report("uniform", st, rels + r2, mism + m2, 300, curves)


def test_uneven_batch_full_size(bls):
    """10000 weighted curves, N log-uniform in [200, 10000], own grids."""
    b = synth.config3()
    _say("uneven batch full size", b.ncurves, b.periods.size)
    outs, st = _run_device(bls, b)
    ns = np.diff(b.n_off)
    nps = np.diff(b.p_off)
    small = np.flatnonzero((ns < 1500) & (nps < 12000))[:2].tolist()
    big = [int(np.argmax(ns))]
    curves = small + big
    rels, mism = _full_curves(b, outs, curves, "uneven")
    r2, m2 = _sampled_pairs(b, outs, np.random.default_rng(2), 300, "uneven")
    _report("uneven", st, rels + r2, mism + m2, 300, curves)


def test_long_baseline_full_size(bls):
    """256 curves x N = 50000 on a 1-minute grid, 100000 periods, 1000 bins:
    two whole periodograms (every period, the box rule and the best index)
    and 200 sampled (curve, period) pairs against the oracle."""
    b = synth.config4()
    _say("long baseline full size")
    outs, st = _run_device(bls, b)
    curves = [0, 255]
    rels, mism = _full_curves(b, outs, curves, "long")
    r2, m2 = _sampled_pairs(b, outs, np.random.default_rng(3), 200, "long")
    _report("long", st, rels + r2, mism + m2, 200, curves)
    # the injected period (or an alias) is found for most curves
    import torch
    bi = outs[4].cpu().numpy()
    hits = 0
    for c in range(b.ncurves):
        P = b.periods[bi[c]]
        Ptrue = b.truth[c]["period"]
        if any(abs(P * f - Ptrue) / Ptrue < 2e-3 for f in (1, 2, 0.5, 3, 1 / 3)):
            hits += 1
    _say("long recovery", hits, "of", b.ncurves)
    assert hits > 0.5 * b.ncurves
    del torch
