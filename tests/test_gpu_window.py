"""Eclipse detection efficiency on the GPU against the FP64 oracle.

The result is an integer count per (cadence, period): the GPU must equal the
oracle exactly.  Both fold with the same FP64 operations, so the bins and
cycle numbers, hence the counts, are identical.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


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
    p = bls.Plan(max_curves=128, max_points=1 << 20, max_periods=1 << 24)
    yield p.handle
    p.close()


def _gpu(bls, plan, t, n_off, per, p_off, nphase, dur, m, w=None):
    import torch
    dev = torch.device("cuda:0")
    nres = int(p_off[-1]) if p_off is not None else \
        (len(n_off) - 1) * per.shape[0]
    obs = torch.full((nres,), -7, device=dev, dtype=torch.int32)
    bls.bls_eclipse_window_device(
        plan, n_off, torch.tensor(t, device=dev), torch.tensor(per, device=dev),
        p_off, nphase, dur, m, obs,
        weights=None if w is None else torch.tensor(w, device=dev))
    return obs.cpu().numpy()


def _pack(ts):
    n_off = np.concatenate([[0], np.cumsum([x.size for x in ts])]).astype(np.int64)
    return np.concatenate(ts), n_off


def _cadences(seed, k):
    rng = np.random.default_rng(seed)
    ts = []
    for i in range(k):
        if i % 3 == 0:       # times on a binary grid, integer-day aliases
            d = np.repeat(np.arange(int(rng.integers(3, 20))), 12)
            ts.append(synth.T_START + d + rng.integers(0, 400, d.size) / 1024.0)
        else:
            ts.append(synth.survey_cadence(rng, nights=int(rng.integers(5, 60))))
    return ts


@pytest.mark.parametrize("nphase,dur,m", [(16, 0.05, 2), (64, 0.02, 1),
                                          (300, 0.02, 2), (1000, 0.01, 2),
                                          (1000, 0.3, 1), (1000, 0.3, 2),
                                          (333, 0.5, 2), (2048, 0.05, 2),
                                          (4096, 0.02, 2), (4096, 0.9, 2),
                                          (2, 0.05, 2), (127, 0.03, 1)])
def test_shared_grid_bit_exact(bls, plan, nphase, dur, m):
    ts = _cadences(200 + nphase, 10)
    t, n_off = _pack(ts)
    # includes P = 1 d and 0.5 d exactly (alias structure) and a ragged tail
    per = np.sort(np.concatenate([synth.log_period_grid(0.1, 10.0, 397),
                                  [0.5, 1.0, 2.0]]))
    _say("window shared", nphase, dur, m, per.size, n_off[-1])
    g = _gpu(bls, plan, t, n_off, per, None, nphase, dur, m)
    for c, tc in enumerate(ts):
        o = oracle.eclipse_window(tc, None, per, nphase, dur, m)
        gc = g[c * per.size:(c + 1) * per.size]
        assert np.array_equal(gc, o), (c, np.flatnonzero(gc != o)[:5])


@pytest.mark.parametrize("nphase,dur,m", [(1000, 0.02, 2), (1000, 0.02, 1),
                                          (250, 0.2, 2)])
def test_dense_and_sparse_cadences(bls, plan, nphase, dur, m):
    # continuous 1-minute sampling over 5 days (every bin filled, most
    # holding several cycles; more points than the register cache), three
    # exposures, and two on one night
    ts = [synth.T_START + np.arange(7200) / 1440.0,
          synth.T_START + np.array([0.1, 3.7, 9.2]),
          synth.T_START + np.array([0.2, 0.21])]
    t, n_off = _pack(ts)
    per = synth.log_period_grid(0.1, 10.0, 301)
    _say("window dense/sparse", nphase, dur, m)
    g = _gpu(bls, plan, t, n_off, per, None, nphase, dur, m)
    for c, tc in enumerate(ts):
        o = oracle.eclipse_window(tc, None, per, nphase, dur, m)
        gc = g[c * per.size:(c + 1) * per.size]
        assert np.array_equal(gc, o), (c, np.flatnonzero(gc != o)[:5])


@pytest.mark.parametrize("nphase,m", [(1000, 2), (1000, 1), (257, 2), (64, 2)])
def test_one_cycle_and_a_little(bls, plan, nphase, m):
    # a cadence just over one cycle at most trial periods: nearly every bin
    # holds one cycle number, the same one, so each window's decision hangs
    # on the few bins of the second cycle, far from most offsets (long runs
    # of single-valued entries across many lanes of the window pass)
    ts = [synth.T_START + np.linspace(0.0, 1.3, 500),
          synth.T_START + np.sort(np.random.default_rng(3).uniform(0, 2.05, 300))]
    t, n_off = _pack(ts)
    per = np.linspace(0.6, 2.2, 161)
    _say("window one cycle and a little", nphase, m)
    g = _gpu(bls, plan, t, n_off, per, None, nphase, 0.07, m)
    for c, tc in enumerate(ts):
        o = oracle.eclipse_window(tc, None, per, nphase, 0.07, m)
        gc = g[c * per.size:(c + 1) * per.size]
        assert np.array_equal(gc, o), (c, np.flatnonzero(gc != o)[:5])
    assert g.max() > 0 and g.min() < nphase


def test_per_cadence_grids_and_zero_weights(bls, plan):
    ts = _cadences(301, 7)
    t, n_off = _pack(ts)
    rng = np.random.default_rng(5)
    grids = [synth.log_period_grid(0.2, 5.0, int(rng.integers(1, 90)))
             for _ in ts]
    p_off = np.concatenate([[0], np.cumsum([x.size for x in grids])]).astype(np.int64)
    w = (rng.uniform(size=t.size) > 0.3).astype(np.float64) * 2.5
    for c in range(len(ts)):                      # keep >= 1 point each
        w[n_off[c]] = 1.0
    _say("window per-cadence grids", p_off[-1], n_off[-1])
    g = _gpu(bls, plan, t, n_off, np.concatenate(grids), p_off, 200, 0.03, 2,
             w=w)
    for c, tc in enumerate(ts):
        wc = w[n_off[c]:n_off[c + 1]]
        o = oracle.eclipse_window(tc, wc, grids[c], 200, 0.03, 2)
        assert np.array_equal(g[p_off[c]:p_off[c + 1]], o), c


def test_degenerate_cadences(bls, plan):
    # one point; all points in one exposure; nphase 1
    ts = [np.array([synth.T_START + 0.3]),
          np.full(5, synth.T_START + 1.25),
          synth.T_START + np.arange(0, 40) * 0.37]
    t, n_off = _pack(ts)
    per = synth.log_period_grid(0.3, 3.0, 50)
    for nphase, m in ((64, 1), (64, 2), (1, 2), (1, 1)):
        _say("window degenerate", nphase, m)
        g = _gpu(bls, plan, t, n_off, per, None, nphase, 0.05, m)
        for c, tc in enumerate(ts):
            o = oracle.eclipse_window(tc, None, per, nphase, 0.05, m)
            assert np.array_equal(g[c * 50:(c + 1) * 50], o), (nphase, m, c)
    assert np.all(g[:50] >= 0)


def test_errors(bls, plan):
    ts = _cadences(9, 2)
    t, n_off = _pack(ts)
    per = synth.log_period_grid(0.3, 3.0, 20)
    for kw in (dict(nphase=0), dict(nphase=4097), dict(m=3), dict(dur=0.0)):
        a = dict(nphase=64, dur=0.02, m=2)
        a.update(kw)
        _say("window bad argument", kw)
        with pytest.raises(bls.BlsError) as ei:
            _gpu(bls, plan, t, n_off, per, None, a["nphase"], a["dur"], a["m"])
        assert ei.value.status == bls.BLS_ERR_INVALID_ARG
    bad = per.copy()
    bad[7] = -1.0
    _say("window bad period on the device")
    with pytest.raises(bls.BlsError) as ei:
        _gpu(bls, plan, t, n_off, bad, None, 64, 0.02, 2)
    assert ei.value.status == bls.BLS_ERR_INVALID_ARG
    assert "period" in bls.bls_last_error(plan)
    tn = t.copy()
    tn[n_off[1] + 3] = np.nan
    _say("window non-finite time")
    with pytest.raises(bls.BlsError) as ei:
        _gpu(bls, plan, tn, n_off, per, None, 64, 0.02, 2)
    assert "cadence 1" in bls.bls_last_error(plan)
    # the plan still works afterwards
    g = _gpu(bls, plan, t, n_off, per, None, 64, 0.02, 2)
    assert np.array_equal(g[:20], oracle.eclipse_window(ts[0], None, per, 64,
                                                        0.02, 2))


def test_cycle_count_limit(bls, plan):
    # cycle numbers are held below 2^29: a cadence whose last kept time lies
    # more cycles than that after its first, at some trial period, is
    # refused; just below the limit it is counted as usual
    per = np.array([0.1, 1.0])
    lim = float(1 << 29)
    for span, ok in ((lim * 0.1 * 1.01, False), (lim * 1.0 * 0.99, True)):
        t = np.array([10.0, 10.5, 11.0 + span * 0.5, 10.0 + span])
        n_off = np.array([0, t.size], np.int64)
        _say("window cycle limit", span, ok)
        if ok:
            g = _gpu(bls, plan, t, n_off, per[1:], None, 64, 0.02, 1)
            assert np.array_equal(g, oracle.eclipse_window(t, None, per[1:],
                                                           64, 0.02, 1))
        else:
            with pytest.raises(bls.BlsError) as ei:
                _gpu(bls, plan, t, n_off, per, None, 64, 0.02, 1)
            assert ei.value.status == bls.BLS_ERR_CAPACITY
            assert "2^29" in bls.bls_last_error(plan)


def test_full_size_sampled(bls, plan):
    """The efficiency workload at full size: 64 fields x 100000 periods,
    1000 trial epochs; every cadence checked on a sample of periods."""
    b = synth.cadence_batch()
    m = b.periods.size
    _say("window full", b.ncurves, m, b.total_points())
    g = _gpu(bls, plan, b.t, b.n_off, b.periods, None, 1000, 0.02, 2)
    assert g.min() >= 0 and g.max() <= 1000
    idx = np.unique(np.concatenate([np.arange(0, m, 997), [m - 1]]))
    for c in range(b.ncurves):
        o = oracle.eclipse_window(b.curve(c).t, None, b.periods[idx], 1000,
                                  0.02, 2)
        assert np.array_equal(g[c * m + idx], o), c
    eff = g.reshape(b.ncurves, m) / 1000.0
    # short periods are seen almost always; the 1-day alias dips
    assert eff[:, b.periods < 0.3].mean() > 0.9
    near1 = np.abs(b.periods - 1.0) < 0.002
    assert eff[:, near1].mean() < eff[:, (b.periods > 0.7) &
                                      (b.periods < 0.9)].mean()
