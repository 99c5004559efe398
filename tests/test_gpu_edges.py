"""Edge regimes of the binned search on the GPU, against the FP64 oracle.

* boxes up to nearly every bin (nbins 4096, qmax 0.999), where a wide box's
  sums cancel and are taken through the complement;
* only wide boxes (q between 0.6 and 0.9);
* a large outlier and weights spread over four decades (the fixed-point
  encoding is relative to the curve's largest value and weight);
* one long curve among hundreds of tiny ones in one persistent launch;
* several device calls queued on one plan without synchronizing, each with
  its own batch;
* the kernel-time ring, and the allocation-failure hook;
* the host-array path with and without its pinned staging.

Every test prints the case it runs (flushed) before touching the GPU.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.parity import check_curve

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bls():
    import paper_1112_1701_amd as bls
    bls._lib.load()
    return bls


def _orc(lc, **kw):
    return oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                         lc.qmax, **kw)


def _host(bls, lc, **cfg):
    with bls.Plan(max_points=1 << 17, max_periods=1 << 12, **cfg) as p:
        return bls.bls_search(p.handle, lc.t, lc.x, lc.w, lc.periods,
                              lc.nbins, lc.qmin, lc.qmax)


def _curve(seed, n, nperiods, nbins, qmin, qmax, weights=None):
    rng = np.random.default_rng(seed)
    t = synth.nightly_times(rng, n)
    x = 1.0 + 0.01 * rng.standard_normal(n)
    x += synth.inject_box(t, 2.3, 0.04, 0.37, 0.01)
    w = None
    if weights == "spread":                   # weights over four decades
        w = 10.0 ** rng.uniform(-2.0, 2.0, n)
    elif weights == "mild":
        w = rng.uniform(0.5, 2.0, n)
    per = synth.log_period_grid(0.5, 6.0, nperiods)
    return synth.LightCurve(t, x, w, per, nbins, qmin, qmax)


@pytest.mark.parametrize("weighted,nbins", [(False, 4096), (True, 2048)])
def test_widest_boxes(bls, weighted, nbins):
    """kmin 1, kmax nearly nbins: every narrow box has a wide twin (its
    complement) with the same statistic up to rounding, and widths above
    nbins/2 are scanned through the complement."""
    lc = _curve(31 + weighted, 50000, 8, nbins, 1.0 / nbins, 0.999,
                "mild" if weighted else None)
    o = _orc(lc)
    assert o.kmin == 1 and o.kmax >= nbins - 5
    _say("widest boxes", nbins, o.kmax, "weighted" if weighted else "unit")
    g = _host(bls, lc)
    st = check_curve(lc, g, o, label="widest %d" % nbins)
    _say("widest stats", st)


@pytest.mark.parametrize("weighted,dip", [(False, False), (True, False),
                                          (False, True)])
def test_only_wide_boxes(bls, weighted, dip):
    """q in [0.6, 0.9]: no width is scanned directly."""
    lc = _curve(41 + weighted + 2 * dip, 3000, 40, 250, 0.6, 0.9,
                "mild" if weighted else None)
    _say("only wide boxes", weighted, dip)
    flags = bls.BLS_DIP_ONLY if dip else 0
    g = _host(bls, lc, flags=flags)
    check_curve(lc, g, _orc(lc, dip_only=dip), label="wide only")


@pytest.mark.parametrize("outlier,weights,dip", [
    (1e4, None, False), (1e4, None, True), (0.0, "spread", False),
    (1e2, "spread", True)])
def test_dynamic_range(bls, outlier, weights, dip):
    """One point far above the noise and/or weights spanning 1e-2..1e2: the
    fixed-point scales follow the largest value and weight."""
    lc = _curve(51, 5000, 60, 200, 0.01, 0.1, weights)
    x = lc.x.copy()
    x[1234] += outlier * 0.01
    lc = synth.LightCurve(lc.t, x, lc.w, lc.periods, lc.nbins, lc.qmin,
                          lc.qmax)
    _say("dynamic range", outlier, weights, dip)
    flags = bls.BLS_DIP_ONLY if dip else 0
    st = check_curve(lc, _host(bls, lc, flags=flags), _orc(lc, dip_only=dip),
                     label="range %g %s %d" % (outlier, weights, dip))
    _say("dynamic range stats", st)


def test_huge_among_tiny(bls):
    """One 50000-point curve among 500 curves of 60 points, one launch."""
    import torch
    rng = np.random.default_rng(61)
    nt = 500
    big = _curve(62, 50000, 1, 300, 0.01, 0.1)
    ts, xs = [big.t], [big.x]
    for c in range(nt):
        t = synth.nightly_times(rng, 60)
        ts.append(t)
        xs.append(1.0 + 0.01 * rng.standard_normal(60))
    ns = [a.size for a in ts]
    n_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    per = synth.log_period_grid(0.2, 10.0, 2000)
    nc = nt + 1
    b = synth.Batch(np.concatenate(ts), np.concatenate(xs), None, n_off, per,
                    None, np.full(nc, 300, np.int32), np.full(nc, 0.01),
                    np.full(nc, 0.1))
    dev = torch.device("cuda:0")
    m = nc * per.size
    outs = [torch.empty(m, device=dev, dtype=torch.float32),
            torch.empty(m, device=dev, dtype=torch.float32),
            torch.empty(m, device=dev, dtype=torch.int32),
            torch.empty(m, device=dev, dtype=torch.int32),
            torch.empty(nc, device=dev, dtype=torch.int64)]
    _say("huge among tiny", nc, b.total_points())
    with bls.Plan(max_curves=nc, max_points=b.total_points(),
                  max_periods=m) as p:
        bls.bls_search_device(p.handle, n_off, torch.tensor(b.t, device=dev),
                              torch.tensor(b.x, device=dev), None,
                              torch.tensor(per, device=dev), None, 300, 0.01,
                              0.1, *outs)
        bls.bls_synchronize(p.handle)
    sr, dp, js, ks, bi = [o.cpu().numpy() for o in outs]
    for c in [0, 1, 2, 250, nc - 1] + list(range(3, nc, 50)):
        lc = b.curve(c)
        a = c * per.size
        g = dict(sr=sr[a:a + per.size], depth=dp[a:a + per.size],
                 jstart=js[a:a + per.size], kwidth=ks[a:a + per.size],
                 best_index=bi[c])
        check_curve(lc, g, _orc(lc), label="huge/tiny curve %d" % c)


def _device_batch(b):
    import torch
    dev = torch.device("cuda:0")
    m = int(b.p_off[-1]) if b.p_off is not None else \
        b.ncurves * b.periods.size
    ins = dict(t=torch.tensor(b.t, device=dev), x=torch.tensor(b.x, device=dev),
               w=None if b.w is None else torch.tensor(b.w, device=dev),
               per=torch.tensor(b.periods, device=dev))
    outs = [torch.full((m,), -7.0, device=dev, dtype=torch.float32),
            torch.empty(m, device=dev, dtype=torch.float32),
            torch.empty(m, device=dev, dtype=torch.int32),
            torch.empty(m, device=dev, dtype=torch.int32),
            torch.empty(b.ncurves, device=dev, dtype=torch.int64)]
    return ins, outs


def _call(bls, plan, b, ins, outs):
    bls.bls_search_device(plan, b.n_off, ins["t"], ins["x"], ins["w"],
                          ins["per"], b.p_off, b.nbins, b.qmin, b.qmax, *outs)


@pytest.mark.parametrize("graph", [True, False])
def test_queued_calls_different_batches(bls, graph):
    """Four bls_search_device calls on one plan, three different batches,
    no synchronization in between: each result equals the same batch run
    alone (bit for bit) and the oracle.  The first batch keeps the device
    busy so that later calls' descriptor uploads queue behind it while the
    host plans the next call."""
    import torch
    batches = [synth.uniform_batch(512, 2000, 4000, 300, seed=71),
               synth.uniform_batch(7, 900, 300, 200, seed=72),
               synth.uneven_batch(5, 73, n_range=(100, 3000),
                                  np_range=(50, 400), nbins_range=(64, 400)),
               None]
    batches[3] = batches[1]
    flags = 0 if graph else bls.BLS_NO_GRAPH
    cap = dict(max_curves=512, max_points=1 << 21, max_periods=1 << 22,
               flags=flags)
    dev = [_device_batch(b) for b in batches]
    _say("queued calls", "graph" if graph else "no graph")
    with bls.Plan(**cap) as p:
        for b, (ins, outs) in zip(batches, dev):
            _call(bls, p.handle, b, ins, outs)
        bls.bls_synchronize(p.handle)
        got = [[o.cpu().numpy().copy() for o in outs] for _, outs in dev]
    with bls.Plan(**cap) as p:
        for k, b in enumerate(batches[:3]):
            ins, outs = _device_batch(b)
            _call(bls, p.handle, b, ins, outs)
            bls.bls_synchronize(p.handle)
            alone = [o.cpu().numpy() for o in outs]
            for g, a in zip(got[k], alone):
                assert np.array_equal(g, a), "call %d differs from alone" % k
    for g, a in zip(got[3], got[1]):
        assert np.array_equal(g, a)
    for k in (1, 2):
        b = batches[k]
        sr, dp, js, ks, bi = got[k]
        for c in range(b.ncurves):
            lc = b.curve(c)
            a = int(b.p_off[c]) if b.p_off is not None else c * b.periods.size
            e = a + lc.periods.size
            g = dict(sr=sr[a:e], depth=dp[a:e], jstart=js[a:e],
                     kwidth=ks[a:e], best_index=bi[c])
            check_curve(lc, g, _orc(lc), label="queued %d/%d" % (k, c))
    del torch


def test_kernel_time_ring(bls):
    """Every search call brackets its kernel with events, graph replays
    included; the durations agree with the call statistics."""
    b = synth.uniform_batch(64, 1500, 2000, 300, seed=74)
    ins, outs = _device_batch(b)
    _say("kernel time ring")
    with bls.Plan(max_curves=64, max_points=1 << 20, max_periods=1 << 20) as p:
        bls.bls_kernel_times_reset(p.handle)
        for _ in range(4):
            _call(bls, p.handle, b, ins, outs)
        ms = bls.bls_kernel_times(p.handle, 16)
        st = bls.bls_last_stats(p.handle)
        assert len(ms) == 4 and all(v > 0 for v in ms)
        assert st["graph_replayed"] == 1
        bls.bls_synchronize(p.handle)
        st = bls.bls_last_stats(p.handle)
        assert abs(st["search_ms"] - ms[-1]) <= 1e-3 * ms[-1] + 1e-3
        assert st["search_ms"] <= st["total_ms"] * 1.001 + 1e-3
        bls.bls_kernel_times_reset(p.handle)
        assert bls.bls_kernel_times(p.handle, 16) == []
        assert bls.bls_kernel_times(p.handle, 0) == []


def test_debug_fail_alloc_hook(bls, monkeypatch):
    """BLS_DEBUG_FAIL_ALLOC makes device allocations fail: plan creation and
    a lazily allocating call report NO_MEMORY; the plan stays usable."""
    lc = synth.small_curve(75, 700, nperiods=30, nbins=100)
    _say("fail alloc hook")
    monkeypatch.setenv("BLS_DEBUG_FAIL_ALLOC", "all")
    with pytest.raises(bls.BlsError) as ei:
        bls.Plan(max_points=1 << 12, max_periods=1 << 10)
    assert ei.value.status == bls.BLS_ERR_NO_MEMORY
    monkeypatch.delenv("BLS_DEBUG_FAIL_ALLOC")
    with bls.Plan(max_points=1 << 12, max_periods=1 << 10) as p:
        monkeypatch.setenv("BLS_DEBUG_FAIL_ALLOC", "all")
        # the host-array path allocates its staging buffers on first use
        with pytest.raises(bls.BlsError) as ei:
            bls.bls_search(p.handle, lc.t, lc.x, lc.w, lc.periods, lc.nbins,
                           lc.qmin, lc.qmax)
        assert ei.value.status == bls.BLS_ERR_NO_MEMORY
        monkeypatch.delenv("BLS_DEBUG_FAIL_ALLOC")
        g = bls.bls_search(p.handle, lc.t, lc.x, lc.w, lc.periods, lc.nbins,
                           lc.qmin, lc.qmax)
    check_curve(lc, g, _orc(lc), label="after failed allocation")
    assert "BLS_DEBUG_FAIL_ALLOC" not in os.environ


@pytest.mark.parametrize("weighted", [False, True])
def test_grouped_items_equal_tile_items(bls, monkeypatch, weighted):
    """Work items of 32 consecutive periods (results staged in LDS and written
    as whole lines, groups aligned to the result index) give the same results
    bit for bit as one tile per item, on curves whose result offsets are not
    multiples of 32 and whose period counts are not either; and the oracle's."""
    b = synth.uneven_batch(9, 81 + weighted, n_range=(150, 4000),
                           np_range=(37, 700), nbins_range=(64, 400),
                           weighted=weighted)
    assert any(int(o) % 32 for o in b.p_off[1:-1])
    got = {}
    for g in ("0", "32"):
        monkeypatch.setenv("BLS_ITEM_GROUP", g)
        ins, outs = _device_batch(b)
        _say("grouped items", g, "weighted" if weighted else "unit")
        with bls.Plan(max_curves=b.ncurves, max_points=b.total_points(),
                      max_periods=int(b.p_off[-1]),
                      flags=bls.BLS_NO_GRAPH | bls.BLS_NO_AUTOTUNE) as p:
            _call(bls, p.handle, b, ins, outs)
            bls.bls_synchronize(p.handle)
            st = bls.bls_last_stats(p.handle)
        got[g] = ([o.cpu().numpy() for o in outs], st["work_items"])
    (a, na), (c, nc) = got["0"], got["32"]
    assert nc < na
    for name, x, y in zip(("sr", "depth", "jstart", "kwidth", "best"), a, c):
        assert np.array_equal(x, y, equal_nan=True), name
    sr, dp, js, ks, bi = c
    for k in (0, 4, 8):
        lc = b.curve(k)
        lo, hi = int(b.p_off[k]), int(b.p_off[k + 1])
        check_curve(lc, dict(sr=sr[lo:hi], depth=dp[lo:hi], jstart=js[lo:hi],
                             kwidth=ks[lo:hi], best_index=bi[k]), _orc(lc),
                    label="grouped %d" % k)


def test_host_path_pageable_fallback(bls, monkeypatch):
    """The host-array path without pinned staging (BLS_DEBUG_FAIL_ALLOC=pinned
    refuses it) gives bit-identical results to the path with it, on a batch of
    curves of different lengths and period grids."""
    rng = np.random.default_rng(77)
    curves = [synth.small_curve(7700 + k, int(n), nperiods=int(m), nbins=120,
                                weighted=(k % 2 == 1))
              for k, (n, m) in enumerate(zip(rng.integers(200, 3000, 5),
                                             rng.integers(20, 200, 5)))]
    _say("host path pageable fallback", [lc.n for lc in curves])
    res = {}
    for mode in ("pinned", "pageable"):
        if mode == "pageable":
            monkeypatch.setenv("BLS_DEBUG_FAIL_ALLOC", "pinned")
        with bls.Plan(max_points=1 << 14, max_periods=1 << 12) as p:
            res[mode] = [bls.bls_search(p.handle, lc.t, lc.x, lc.w, lc.periods,
                                        lc.nbins, lc.qmin, lc.qmax)
                         for lc in curves]
        monkeypatch.delenv("BLS_DEBUG_FAIL_ALLOC", raising=False)
    for k, (a, b) in enumerate(zip(res["pinned"], res["pageable"])):
        for key in ("sr", "depth", "phase", "duration", "jstart", "kwidth"):
            assert np.array_equal(a[key], b[key], equal_nan=True), (k, key)
        assert a["best_index"] == b["best_index"], k
    check_curve(curves[0], res["pageable"][0], _orc(curves[0]),
                label="pageable host path")
    assert "BLS_DEBUG_FAIL_ALLOC" not in os.environ
