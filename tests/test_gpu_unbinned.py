"""Unbinned box search on the GPU against the FP64 oracle.

SR within the floating-point tolerance of the binned search (1e-5
relative); the GPU sums runs exactly in fixed point, so its SR differs from
the oracle's FP64 sums only by the fixed-point quantisation (about 1e-9).
The best box (first and last point) must be the oracle's, except where two
runs tie to within that tolerance: then the GPU's run must score, on the
CPU in FP64, within the tolerance of the oracle's best.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
REL_TOL = 1e-5


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bls():
    import paper_1112_1701_amd as bls
    bls._lib.load()
    return bls


@pytest.fixture(scope="module")
def plan(bls):
    p = bls.Plan(max_curves=64, max_points=1 << 20, max_periods=1 << 21)
    yield p.handle
    p.close()


def _gpu(bls, plan, curves, per_list, qmin, qmax, shared=True):
    import torch
    dev = torch.device("cuda:0")
    n_off = np.concatenate([[0], np.cumsum([c[0].size for c in curves])]).astype(np.int64)
    t = np.concatenate([c[0] for c in curves])
    x = np.concatenate([c[1] for c in curves])
    ws = [c[2] for c in curves]
    w = None if all(v is None for v in ws) else np.concatenate(
        [np.ones(c[0].size) if c[2] is None else c[2] for c in curves])
    if shared:
        per = per_list[0]
        p_off = None
        nres = len(curves) * per.size
    else:
        per = np.concatenate(per_list)
        p_off = np.concatenate([[0], np.cumsum([p.size for p in per_list])]).astype(np.int64)
        nres = int(p_off[-1])
    T = lambda a: torch.tensor(a, device=dev)
    sr = torch.empty(nres, device=dev, dtype=torch.float32)
    depth = torch.empty(nres, device=dev, dtype=torch.float32)
    first = torch.empty(nres, device=dev, dtype=torch.int32)
    last = torch.empty(nres, device=dev, dtype=torch.int32)
    best = torch.empty(len(curves), device=dev, dtype=torch.int64)
    bls.bls_search_unbinned_device(plan, n_off, T(t), T(x),
                                   None if w is None else T(w), T(per), p_off,
                                   qmin, qmax, sr, depth, first, last, best)
    bls.bls_synchronize(plan)
    return (sr.cpu().numpy(), depth.cpu().numpy(), first.cpu().numpy(),
            last.cpu().numpy(), best.cpu().numpy())


def _run_value(t, x, w, P, first, last):
    """FP64 statistic of the run first..last in the fold's phase order."""
    w = np.ones_like(x) if w is None else w
    keep = np.flatnonzero(w > 0)
    d = t[keep] - t[keep].min()
    c = d * (1.0 / P)
    ph = c - np.floor(c)
    order = keep[np.lexsort((keep, ph))]
    pos = {int(k): i for i, k in enumerate(order)}
    a, b = pos[int(first)], pos[int(last)]
    run = order[a:b + 1] if b >= a else np.concatenate([order[a:], order[:b + 1]])
    W = math.fsum(w[keep])
    xbar = math.fsum(w[keep] * x[keep]) / W
    R = math.fsum(w[run])
    S = math.fsum(w[run] * (x[run] - xbar))
    return math.sqrt(S * S / (R * (W - R)))


def _check(curve, per, g, o, tag):
    t, x, w = curve
    sr, depth, first, last = g
    osr = o["sr"]
    err = np.abs(sr - osr) / np.maximum(osr, 1e-30)
    assert np.all((osr == 0) == (sr == 0)), tag
    assert err.max() <= REL_TOL, (tag, err.max(), int(err.argmax()))
    mism = np.flatnonzero((first != o["first"]) | (last != o["last"]))
    for i in mism:   # near-ties only
        v = _run_value(t, x, w, per[i], first[i], last[i])
        assert abs(v - osr[i]) <= REL_TOL * osr[i], (tag, i, v, osr[i])
    ok = osr > 0
    de = np.abs(depth[ok] - o["depth"][ok]) / np.abs(o["depth"][ok])
    same = (first[ok] == o["first"][ok]) & (last[ok] == o["last"][ok])
    assert np.all(de[same] <= 1e-4), tag
    return len(mism)


@pytest.mark.parametrize("n,nper,qmin,qmax,weighted", [
    (37, 50, 0.05, 0.3, False),      # fewer points than a wave
    (257, 80, 0.01, 0.1, False),     # ragged against the block
    (1000, 120, 0.01, 0.1, True),
    (4096, 12, 0.005, 0.02, False),  # the largest curve held in LDS
    (4097, 6, 0.005, 0.02, True),    # the smallest in the workspace
    (10000, 6, 0.005, 0.03, False),  # workspace: uneven-batch sizes
    (20000, 4, 0.005, 0.02, True),
    (600, 60, 0.2, 0.5, True),       # wide boxes
])
def test_single_curves(bls, plan, n, nper, qmin, qmax, weighted):
    lc = synth.small_curve(3000 + n, n, nperiods=nper, nbins=64, qmin=qmin,
                           qmax=qmax, weighted=weighted)
    _say("unbinned", n, nper, qmin, qmax, weighted)
    g = _gpu(bls, plan, [(lc.t, lc.x, lc.w)], [lc.periods], qmin, qmax)
    o = oracle.unbinned(lc.t, lc.x, lc.w, lc.periods, qmin, qmax)
    nm = _check((lc.t, lc.x, lc.w), lc.periods, g[:4], o, "n%d" % n)
    _say("unbinned near-tie box differences", nm)
    assert g[4][0] == o["best_index"] or \
        abs(g[0][g[4][0]] - o["sr"].max()) <= REL_TOL * o["sr"].max()


def test_batch_per_curve_grids_zero_weights(bls, plan):
    rng = np.random.default_rng(21)
    curves, grids = [], []
    for k, n in enumerate([120, 900, 33, 2500, 700]):
        lc = synth.small_curve(4000 + k, n, nperiods=int(rng.integers(5, 40)),
                               nbins=64, qmin=0.02, qmax=0.15,
                               weighted=(k % 2 == 1))
        w = lc.w
        if w is not None:
            w = w.copy()
            w[::7] = 0.0
        curves.append((lc.t, lc.x, w))
        grids.append(lc.periods)
    _say("unbinned batch", [c[0].size for c in curves])
    sr, depth, first, last, best = _gpu(bls, plan, curves, grids, 0.02, 0.15,
                                        shared=False)
    off = np.concatenate([[0], np.cumsum([g.size for g in grids])])
    for k, (c, per) in enumerate(zip(curves, grids)):
        o = oracle.unbinned(c[0], c[1], c[2], per, 0.02, 0.15)
        sl = slice(off[k], off[k + 1])
        _check(c, per, (sr[sl], depth[sl], first[sl], last[sl]), o, "b%d" % k)


def test_degenerate_and_errors(bls, plan):
    # every point at one time: no box can separate them
    t = np.full(50, synth.T_START + 1.0)
    x = np.random.default_rng(1).normal(1, 0.01, 50)
    per = synth.log_period_grid(0.3, 3.0, 10)
    _say("unbinned one phase")
    sr, depth, first, last, best = _gpu(bls, plan, [(t, x, None)], [per],
                                        0.01, 0.2)
    assert np.all(sr == 0) and np.all(first == -1) and np.all(last == -1)
    n_big = (1 << 20) + 1
    t_big = synth.T_START + np.arange(n_big) / 1440.0
    _say("unbinned too long")
    with bls.Plan(max_points=n_big, max_periods=8) as pbig:
        with pytest.raises(bls.BlsError) as ei:
            _gpu(bls, pbig.handle, [(t_big, np.ones(n_big), None)], [per[:3]],
                 0.01, 0.1)
    assert ei.value.status == bls.BLS_ERR_CAPACITY
    lc = synth.small_curve(6, 300, nperiods=5, nbins=64, qmin=0.01, qmax=0.1)
    for qmin, qmax in ((0.0, 0.1), (0.2, 0.1), (0.1, 1.0)):
        _say("unbinned bad q", qmin, qmax)
        with pytest.raises(bls.BlsError) as ei:
            _gpu(bls, plan, [(lc.t, lc.x, None)], [lc.periods], qmin, qmax)
        assert ei.value.status == bls.BLS_ERR_INVALID_ARG
    bad = lc.x.copy()
    bad[3] = np.nan
    _say("unbinned bad data")
    with pytest.raises(bls.BlsError) as ei:
        _gpu(bls, plan, [(lc.t, bad, None)], [lc.periods], 0.01, 0.1)
    assert ei.value.status == bls.BLS_ERR_INVALID_ARG


def test_plain_workload_full(bls, plan):
    """The plain workload at full size: N = 1000, 5000 periods, q 0.01-0.1;
    the injected box is recovered."""
    lc = synth.config1()
    _say("unbinned plain full", lc.n, lc.periods.size)
    g = _gpu(bls, plan, [(lc.t, lc.x, lc.w)], [lc.periods], lc.qmin, lc.qmax)
    o = oracle.unbinned(lc.t, lc.x, lc.w, lc.periods, lc.qmin, lc.qmax)
    nm = _check((lc.t, lc.x, lc.w), lc.periods, g[:4], o, "plain")
    _say("unbinned plain near-tie box differences", nm)
    assert abs(lc.periods[g[4][0]] - 1.7) / 1.7 < 0.01
