"""GPU (gfx950) results against the FP64 oracle, through the C ABI.

Every test prints the case it runs (flushed) before touching the GPU.
"""
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


@pytest.fixture(scope="module")
def plan(bls):
    p = bls.Plan(max_curves=64, max_points=1 << 22, max_periods=1 << 22)
    yield p.handle
    p.close()


def _orc(lc, **kw):
    return oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                         lc.qmax, **kw)


def _run(bls, plan, lc):
    return bls.bls_search(plan, lc.t, lc.x, lc.w, lc.periods, lc.nbins,
                          lc.qmin, lc.qmax)


def test_config1_full(bls, plan):
    """Plain single curve at its full size: N=1000, 5000 periods, 200 bins."""
    lc = synth.config1()
    _say("config1 full", lc.n, lc.periods.size, lc.nbins)
    g = _run(bls, plan, lc)
    o = _orc(lc)
    stats = check_curve(lc, g, o, label="config1")
    _say("config1 stats", stats)
    assert abs(lc.periods[g["best_index"]] - 1.7) / 1.7 < 0.01


@pytest.mark.parametrize("n,nper,nbins,weighted", [
    (37, 19, 40, False),      # fewer points than a wave
    (257, 33, 64, False),     # ragged: not a multiple of the block
    (3000, 70, 300, False),   # several point chunks and tiles
    (500, 45, 120, True),     # weighted
    (2049, 100, 500, True),   # weighted, ragged chunk
])
def test_small_curves(bls, plan, n, nper, nbins, weighted):
    lc = synth.small_curve(1000 + n, n, nperiods=nper, nbins=nbins,
                           qmin=0.01, qmax=0.12, weighted=weighted)
    _say("small", n, nper, nbins, weighted)
    check_curve(lc, _run(bls, plan, lc), _orc(lc), label="small%d" % n)


@pytest.mark.parametrize("n,nbins,dip", [(30, 400, False), (60, 200, False),
                                         (45, 300, True)])
def test_sparse_bins_empty_boxes(bls, plan, n, nbins, dip):
    """Far fewer points than bins: most narrow boxes hold no point, so their
    statistic is 0/0 and they must never be taken, neither on their own nor
    on a tie with another box of equal (zero) products."""
    lc = synth.small_curve(7000 + n, n, nperiods=40, nbins=nbins, qmin=0.005,
                           qmax=0.05)
    _say("sparse bins", n, nbins, dip)
    flags = bls.BLS_DIP_ONLY if dip else 0
    with bls.Plan(max_curves=4, max_points=1 << 12, max_periods=1 << 10,
                  max_nbins=nbins, flags=flags) as p:
        g = _run(bls, p.handle, lc)
    assert np.all(np.isfinite(g["sr"])), "non-finite SR"
    check_curve(lc, g, _orc(lc, dip_only=dip), label="sparse%d" % n)


@pytest.mark.parametrize("weighted", [False, True])
def test_dense_cadence_lane_gap(bls, plan, weighted):
    """A 1-minute cadence with long trial periods: the fold spaces its lanes
    2 and 4 runs of points apart in full chunks of 1024 points (the lane gap
    follows the curve's cadence), which must not change any bin sum."""
    rng = np.random.default_rng(91)
    n = 5000
    t = synth.minute_grid_times(n)
    x = 1.0 + rng.normal(0.0, 0.003, n)
    x -= 0.01 * (((t - t[0]) % 7.3) < 0.15)        # a box at 7.3 d
    w = rng.uniform(0.5, 2.0, n) if weighted else None
    per = synth.log_period_grid(2.0, 20.0, 48)
    lc = synth.LightCurve(t, x, w, per, 1000, 0.005, 0.05)
    _say("dense cadence lane gap", n, weighted)
    check_curve(lc, _run(bls, plan, lc), _orc(lc), label="dense%d" % weighted)


def test_single_period_and_widest_boxes(bls, plan):
    lc = synth.small_curve(5, 400, nperiods=1, nbins=50, qmin=0.01,
                           qmax=0.999)
    _say("nperiods=1, kmax=nbins-1")
    o = _orc(lc)
    assert o.kmax == 49
    check_curve(lc, _run(bls, plan, lc), o, label="kmax")


def test_max_nbins(bls, plan):
    lc = synth.small_curve(6, 5000, nperiods=20, nbins=4096, qmin=0.001,
                           qmax=0.02)
    _say("nbins=4096")
    check_curve(lc, _run(bls, plan, lc), _orc(lc), label="nbins4096")


def test_all_points_in_one_bin(bls, plan):
    """Times on an exact multiple of the period: every point in bin 0, so no
    box holds between 1 and n-1 points: SR 0, no box."""
    t = synth.T_START + np.arange(50) * 2.0
    x = 1.0 + 0.01 * np.random.default_rng(1).standard_normal(50)
    periods = np.array([1.0, 0.5, 2.0])
    _say("commensurate")
    g = bls.bls_search(plan, t, x, None, periods, 100, 0.01, 0.1)
    o = oracle.search(t, x, None, periods, 100, 0.01, 0.1)
    assert np.all(o.kwidth < 0)
    assert np.all(g["sr"] == 0) and np.all(g["kwidth"] < 0)
    assert np.all(np.isnan(g["phase"]))


def test_zero_weights_dropped(bls, plan):
    lc = synth.small_curve(7, 600, nperiods=40, nbins=100, weighted=True)
    w = lc.w.copy()
    w[::7] = 0.0
    x = lc.x.copy()
    x[::7] = np.nan          # dropped points may hold anything
    t = lc.t.copy()
    t[0] = np.nan if w[0] == 0 else t[0]
    lc2 = synth.LightCurve(t, x, w, lc.periods, lc.nbins, lc.qmin, lc.qmax)
    _say("zero weights")
    check_curve(lc2, _run(bls, plan, lc2), _orc(lc2), label="zerow")


def test_long_baseline_short_period(bls, plan):
    """120 nights of 1-minute cadence folded at P ~ 0.1 d: 1200 cycles, the
    case that needs the FP64 phase."""
    t = synth.minute_grid_times(6000, nights=120, per_night=50)
    rng = np.random.default_rng(2)
    x = 1.0 + 0.003 * rng.standard_normal(t.size)
    x += synth.inject_box(t, 0.1037, 0.02, 0.3, 0.01)
    periods = synth.log_period_grid(0.1, 0.11, 300)
    lc = synth.LightCurve(t, x, None, periods, 1000, 0.005, 0.05)
    _say("long baseline")
    check_curve(lc, _run(bls, plan, lc), _orc(lc), label="longbase")


def test_dip_only_and_min_points(bls):
    lc = synth.small_curve(8, 800, nperiods=60, nbins=150)
    for flags, mip in ((bls.BLS_DIP_ONLY, 1), (0, 3), (bls.BLS_DIP_ONLY, 5)):
        _say("flags", flags, "mip", mip)
        with bls.Plan(max_points=1 << 16, max_periods=1 << 16, flags=flags,
                      min_in_points=mip) as p:
            g = _run(bls, p.handle, lc)
        o = _orc(lc, dip_only=bool(flags), min_in_points=mip)
        check_curve(lc, g, o, label="flags%d mip%d" % (flags, mip))


def test_batch_matches_alone_and_oracle(bls, plan):
    """Uneven weighted batch: each curve's results are bit-identical alone and
    in the batch, and match the oracle."""
    b = synth.uneven_batch(9, 4242, n_range=(60, 4000), np_range=(50, 400),
                           nbins_range=(100, 400), weighted=True)
    _say("uneven batch", b.ncurves)
    g = bls.bls_search_batch(plan, b.n_off, b.t, b.x, b.w, b.periods,
                             b.p_off, b.nbins, b.qmin, b.qmax)
    for c in range(b.ncurves):
        lc = b.curve(c)
        a, e = int(b.p_off[c]), int(b.p_off[c + 1])
        gc = {k: g[k][a:e] for k in ("sr", "jstart", "kwidth", "depth")}
        gc["best_index"] = g["best_index"][c]
        check_curve(lc, gc, _orc(lc), label="batch curve %d" % c)
        alone = _run(bls, plan, lc)
        assert np.array_equal(alone["sr"], gc["sr"])
        assert np.array_equal(alone["jstart"], gc["jstart"])
        assert alone["best_index"] == gc["best_index"]


def test_shared_grid_batch(bls, plan):
    b = synth.uniform_batch(12, 700, 250, 200, seed=77)
    _say("uniform batch", b.ncurves)
    g = bls.bls_search_batch(plan, b.n_off, b.t, b.x, b.w, b.periods, None,
                             200, 0.01, 0.1)
    m = b.periods.size
    for c in range(b.ncurves):
        lc = b.curve(c)
        gc = {k: g[k][c * m:(c + 1) * m] for k in ("sr", "jstart", "kwidth",
                                                  "depth")}
        gc["best_index"] = g["best_index"][c]
        check_curve(lc, gc, _orc(lc), label="uniform %d" % c)


def test_device_api_graph_replay_and_determinism(bls):
    import torch
    b = synth.uniform_batch(6, 1500, 300, 300, seed=78)
    dev = torch.device("cuda:0")
    _say("device api")
    t = torch.tensor(b.t, device=dev)
    x = torch.tensor(b.x, device=dev)
    per = torch.tensor(b.periods, device=dev)
    m = b.periods.size * b.ncurves
    outs = []
    with bls.Plan(max_curves=8, max_points=1 << 16, max_periods=1 << 16) as p:
        for rep in range(3):
            sr = torch.full((m,), -1.0, device=dev, dtype=torch.float32)
            dp = torch.empty(m, device=dev, dtype=torch.float32)
            js = torch.empty(m, device=dev, dtype=torch.int32)
            ks = torch.empty(m, device=dev, dtype=torch.int32)
            bi = torch.empty(b.ncurves, device=dev, dtype=torch.int64)
            if rep > 0:
                sr, dp, js, ks, bi = keep
            bls.bls_search_device(p.handle, b.n_off, t, x, None, per, None,
                                  300, 0.01, 0.1, sr, dp, js, ks, bi)
            bls.bls_synchronize(p.handle)
            st = bls.bls_last_stats(p.handle)
            assert st["graph_replayed"] == (1 if rep > 0 else 0)
            keep = (sr, dp, js, ks, bi)
            outs.append([a.cpu().numpy().copy() for a in keep])
    for o in outs[1:]:
        for a0, a1 in zip(outs[0], o):
            assert np.array_equal(a0, a1)
    sr, dp, js, ks, bi = outs[0]
    mm = b.periods.size
    for c in range(b.ncurves):
        lc = b.curve(c)
        gc = dict(sr=sr[c * mm:(c + 1) * mm], depth=dp[c * mm:(c + 1) * mm],
                  jstart=js[c * mm:(c + 1) * mm],
                  kwidth=ks[c * mm:(c + 1) * mm], best_index=bi[c])
        check_curve(lc, gc, _orc(lc), label="device %d" % c)


def test_device_api_reports_bad_data(bls):
    import torch
    b = synth.uniform_batch(3, 300, 50, 100, seed=79)
    x = b.x.copy()
    x[310] = np.inf                       # curve 1
    dev = torch.device("cuda:0")
    _say("device bad data")
    m = b.periods.size * 3
    with bls.Plan(max_curves=4, max_points=4096, max_periods=4096,
                  flags=bls.BLS_NO_GRAPH) as p:
        args = [torch.tensor(a, device=dev) for a in (b.t, x, b.periods)]
        outs = [torch.empty(m, device=dev, dtype=torch.float32),
                torch.empty(m, device=dev, dtype=torch.float32),
                torch.empty(m, device=dev, dtype=torch.int32),
                torch.empty(m, device=dev, dtype=torch.int32),
                torch.empty(3, device=dev, dtype=torch.int64)]
        bls.bls_search_device(p.handle, b.n_off, args[0], args[1], None,
                              args[2], None, 100, 0.01, 0.1, *outs)
        with pytest.raises(bls.BlsError) as ei:
            bls.bls_synchronize(p.handle)
        assert "curve 1" in str(ei.value)
        sr = outs[0].cpu().numpy()
        assert np.all(np.isnan(sr[50:100]))
        assert np.all(np.isfinite(sr[:50]))


def test_host_errors_leave_outputs_untouched(bls, plan):
    lc = synth.small_curve(3, 100, nperiods=10, nbins=50)
    _say("errors")
    x = lc.x.copy()
    x[5] = np.nan
    with pytest.raises(bls.BlsError) as ei:
        _run(bls, plan, synth.LightCurve(lc.t, x, None, lc.periods, 50,
                                         lc.qmin, lc.qmax))
    assert ei.value.status == bls.BLS_ERR_INVALID_ARG
    with pytest.raises(bls.BlsError) as ei:
        bls.bls_search(plan, lc.t, lc.x, None, lc.periods, 50, 0.3, 0.2)
    assert ei.value.status == bls.BLS_ERR_INVALID_ARG
    with pytest.raises(bls.BlsError) as ei:
        bls.bls_search(plan, lc.t, lc.x, None, lc.periods, 5000, 0.01, 0.1)
    assert ei.value.status == bls.BLS_ERR_CAPACITY
    # the plan is still usable
    check_curve(lc, _run(bls, plan, lc), _orc(lc), label="after errors")


@pytest.mark.parametrize("cadence", ["nightly", "minute_grid"])
def test_phase_bins_bit_exact(bls, plan, cadence):
    """Where FP64 rounding decides an integer (the bin), both sides decide in
    FP64 with the same operation order: bins must be identical."""
    rng = np.random.default_rng(12)
    if cadence == "nightly":
        t = synth.nightly_times(rng, 20000, nights=60)
    else:
        t = synth.minute_grid_times(50000)
    periods = np.concatenate([
        synth.log_period_grid(0.1, 20.0, 40), [1.0, 0.5, 1.0 / 3.0, 2.0,
                                               1.0 / 1440.0 * 97]])
    _say("bins", cadence, t.size)
    for P in periods:
        for nbins in (200, 1000, 4096):
            g = bls.bls_debug_phase_bins(plan, t, P, nbins)
            o, *_ = oracle.bins(t, np.ones_like(t), None, P, nbins)
            assert np.array_equal(g, o), (cadence, P, nbins,
                                          int(np.sum(g != o)))


def test_device_api_reports_bad_period(bls):
    import torch
    b = synth.uniform_batch(2, 300, 50, 100, seed=80)
    per = b.periods.copy()
    per[7] = -1.0
    dev = torch.device("cuda:0")
    _say("device bad period")
    m = per.size * 2
    with bls.Plan(max_curves=4, max_points=4096, max_periods=4096) as p:
        args = [torch.tensor(a, device=dev) for a in (b.t, b.x, per)]
        outs = [torch.empty(m, device=dev, dtype=torch.float32),
                torch.empty(m, device=dev, dtype=torch.float32),
                torch.empty(m, device=dev, dtype=torch.int32),
                torch.empty(m, device=dev, dtype=torch.int32),
                torch.empty(2, device=dev, dtype=torch.int64)]
        bls.bls_search_device(p.handle, b.n_off, args[0], args[1], None,
                              args[2], None, 100, 0.01, 0.1, *outs)
        with pytest.raises(bls.BlsError) as ei:
            bls.bls_synchronize(p.handle)
        assert "trial period" in str(ei.value)


def test_detection_statistics(bls):
    """GPU detection on the GPU's periodogram equals the oracle's detection
    on the same SR values (identical inputs: identical peaks); end to end it
    agrees with the oracle's detection on the oracle's own periodogram."""
    import torch
    b = synth.uniform_batch(8, 1500, 4000, 200, seed=81, inj_prob=0.5)
    dev = torch.device("cuda:0")
    _say("detection")
    m = b.periods.size
    t = torch.tensor(b.t, device=dev)
    x = torch.tensor(b.x, device=dev)
    per = torch.tensor(b.periods, device=dev)
    outs = [torch.empty(m * 8, device=dev, dtype=torch.float32),
            torch.empty(m * 8, device=dev, dtype=torch.float32),
            torch.empty(m * 8, device=dev, dtype=torch.int32),
            torch.empty(m * 8, device=dev, dtype=torch.int32),
            torch.empty(8, device=dev, dtype=torch.int64)]
    with bls.Plan(max_curves=8, max_points=1 << 16, max_periods=1 << 16) as p:
        bls.bls_search_device(p.handle, b.n_off, t, x, None, per, None, 200,
                              0.01, 0.1, *outs)
        bls.bls_synchronize(p.handle)
        det = bls.bls_detect_device(p.handle, b.n_off, per, None, 200, 0.01,
                                    0.1, outs[0], max_peaks=6, window=0.01,
                                    sde_threshold=6.0)
    sr = outs[0].cpu().numpy()
    for c in range(8):
        g = det[c]
        src = sr[c * m:(c + 1) * m].astype(np.float64)
        o = oracle.detect(src, b.periods, max_peaks=6, window=0.01,
                          threshold=6.0)
        assert np.array_equal(g["peak_index"], o["peak_index"]), c
        for k in ("mean", "std", "sde"):
            assert abs(g[k if k == "sde" else k + "_sr"] - o[k]) <= \
                1e-12 * max(abs(o[k]), 1e-30), (c, k)
        assert g["candidate"] == o["candidate"]
        lc = b.curve(c)
        oo = _orc(lc)
        oe = oracle.detect(oo.sr, b.periods, max_peaks=6, window=0.01,
                           threshold=6.0)
        assert abs(g["sde"] - oe["sde"]) <= 1e-5 * oe["sde"]
        assert g["peak_index"][0] in np.flatnonzero(
            oo.sr >= (1 - 1e-5) * oo.sr.max())


def test_detection_crafted_periodograms(bls):
    """GPU detection of crafted SR arrays (float32, as the search writes
    them) equals the oracle's detection of the same values: peak indices
    bit-exact, statistics to FP64 rounding.  The cases drive the kernel's
    candidate buckets through rescans, cross-slice suppression, ties and the
    early stop."""
    import torch
    cases = synth.detection_periodograms()
    dev = torch.device("cuda:0")
    nc = len(cases)
    _say("detection crafted", nc)
    srs = [np.asarray(c[0], np.float32) for c in cases]
    p_off = np.concatenate([[0], np.cumsum([s.size for s in srs])])
    per = torch.tensor(np.concatenate([c[1] for c in cases]), device=dev)
    srd = torch.tensor(np.concatenate(srs), device=dev)
    n_off = np.arange(nc + 1, dtype=np.int64) * 4
    with bls.Plan(max_curves=nc, max_points=1 << 12, max_periods=1 << 16) as p:
        for mp, win in sorted({(c[2], c[3]) for c in cases}):
            det = bls.bls_detect_device(p.handle, n_off, per, p_off, 200,
                                        0.01, 0.1, srd, max_peaks=mp,
                                        window=win, sde_threshold=3.0)
            for c, case in enumerate(cases):
                if (case[2], case[3]) != (mp, win):
                    continue
                o = oracle.detect(srs[c].astype(np.float64), case[1],
                                  max_peaks=mp, window=win, threshold=3.0)
                g = det[c]
                assert np.array_equal(g["peak_index"], o["peak_index"]), \
                    (c, g["peak_index"], o["peak_index"])
                assert np.array_equal(g["peak_sr"].astype(np.float64),
                                      o["peak_sr"]), c
                for k in ("mean", "std", "sde"):
                    gv = g[k if k == "sde" else k + "_sr"]
                    assert abs(gv - o[k]) <= 1e-12 * max(abs(o[k]), 1e-30), \
                        (c, k, gv, o[k])
                assert g["candidate"] == o["candidate"], c


def test_detection_beyond_a_million_periods(bls):
    """Detection of periodograms longer than 2^20 periods (the kernel keeps
    no per-period state in LDS, so their length is limited only by the
    batch): two curves of 2^21 + 3 periods, random SR with a few strong
    peaks and their harmonics, 16 peaks; indices bit-exact against the
    oracle."""
    import torch
    rng = np.random.default_rng(85)
    m = (1 << 21) + 3
    per = np.geomspace(0.1, 30.0, m)
    srs = []
    for c in range(2):
        sr = rng.gamma(2.0, 0.5, m).astype(np.float32)
        for P in (0.7 + c, 2.3, 5.1):
            for h in (1.0, 0.5, 2.0, 1.0 / 3.0, 3.0):
                j = int(np.argmin(np.abs(per - h * P)))
                sr[max(j - 50, 0):j + 50] += np.float32(20.0 / h)
        srs.append(sr)
    _say("detection long periodograms", m)
    dev = torch.device("cuda:0")
    per_d = torch.tensor(per, device=dev)
    sr_d = torch.tensor(np.concatenate(srs), device=dev)
    with bls.Plan(max_curves=2, max_points=1 << 12, max_periods=2 * m) as p:
        det = bls.bls_detect_device(p.handle, np.array([0, 4, 8]), per_d, None,
                                    200, 0.01, 0.1, sr_d, max_peaks=16,
                                    window=0.002, sde_threshold=5.0)
    for c in range(2):
        o = oracle.detect(srs[c].astype(np.float64), per, max_peaks=16,
                          window=0.002, threshold=5.0)
        g = det[c]
        assert np.array_equal(g["peak_index"], o["peak_index"]), c
        for k in ("mean", "std", "sde"):
            gv = g[k if k == "sde" else k + "_sr"]
            assert abs(gv - o[k]) <= 1e-12 * max(abs(o[k]), 1e-30), (c, k)
        assert g["candidate"] == o["candidate"]


def test_single_bin_boxes(bls, plan):
    """kmax = 1 (20 bins, q up to 0.05): each period's histogram is its bins
    plus one clamp word, so the LDS tile must hold nbins + 1 words per
    period; every period of a full tile is checked."""
    b = synth.uniform_batch(6, 700, 400, 20, seed=91, inj_prob=0.5)
    _say("single-bin boxes", b.ncurves, b.periods.size)
    assert bls.bls_width_range(20, 0.01, 0.05) == (1, 1)
    res = bls.bls_search_batch(plan, b.n_off, b.t, b.x, None, b.periods,
                               None, 20, 0.01, 0.05)
    m = b.periods.size
    for c in range(b.ncurves):
        lc = b.curve(c)
        lc.qmin, lc.qmax = 0.01, 0.05
        g = {k: (v[c * m:(c + 1) * m] if k != "best_index" else v[c])
             for k, v in res.items()}
        check_curve(lc, g, _orc(lc), label="kmax1-%d" % c)
