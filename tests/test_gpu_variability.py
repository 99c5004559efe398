"""High-variability pre-search on the GPU against the FP64 oracle.

RMS values and bin statistics agree to FP64 rounding (the sums run in a
different order); bins, counts and flags are integers and must be equal,
except where a value sits within rounding of a clipping or flag threshold,
which the checks below detect and report.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
RTOL = 1e-12


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
    p = bls.Plan(max_curves=1 << 17, max_points=1 << 25, max_periods=16)
    yield p.handle
    p.close()


def _run(bls, plan, x, w, n_off, mag, chip_off, nmagbins, **kw):
    import torch
    dev = torch.device("cuda:0")
    nc, nk = len(n_off) - 1, len(chip_off) - 1
    out = dict(rms=torch.empty(nc, device=dev, dtype=torch.float64),
               bin=torch.empty(nc, device=dev, dtype=torch.int32),
               flag=torch.empty(nc, device=dev, dtype=torch.int32),
               bin_mean=torch.empty(nk * nmagbins, device=dev, dtype=torch.float64),
               bin_std=torch.empty(nk * nmagbins, device=dev, dtype=torch.float64),
               bin_count=torch.empty(nk * nmagbins, device=dev, dtype=torch.int32))
    bls.bls_variability_device(
        plan, n_off, torch.tensor(x, device=dev),
        None if w is None else torch.tensor(w, device=dev),
        torch.tensor(mag, device=dev), chip_off, nmagbins, out, **kw)
    return {k: v.cpu().numpy() for k, v in out.items()}


def _compare(g, o, nk, nb, flag_sigma=2.0):
    # RMS to rounding, NaN where the oracle has NaN
    on = np.isnan(o["rms"])
    assert np.array_equal(np.isnan(g["rms"]), on)
    assert np.all(np.abs(g["rms"][~on] - o["rms"][~on])
                  <= RTOL * np.abs(o["rms"][~on]) + 1e-300)
    assert np.array_equal(g["bin"], o["bin"])
    cnt = g["bin_count"].reshape(nk, nb)
    bad_bins = np.argwhere(cnt != o["count"])
    assert bad_bins.size == 0, bad_bins[:5]
    mean = g["bin_mean"].reshape(nk, nb)
    std = g["bin_std"].reshape(nk, nb)
    # The mean and the population deviation of a set move by at most the
    # largest change of a member, so the members' RMS differences bound
    # theirs (a tight bin amplifies relative error by rms / std).
    dr = np.max(np.abs(g["rms"][~on] - o["rms"][~on]), initial=0.0)
    for name, gv, ov in (("mean", mean, o["mean"]), ("std", std, o["std"])):
        nan = np.isnan(ov)
        assert np.array_equal(np.isnan(gv), nan), name
        assert np.all(np.abs(gv[~nan] - ov[~nan])
                      <= RTOL * np.abs(ov[~nan]) + 2 * dr + 1e-300), name
    diff = np.flatnonzero(g["flag"] != o["flag"])
    for s in diff:        # only values within rounding of their threshold
        b = o["bin"][s]
        k = np.searchsorted(_compare.chip_off, s, side="right") - 1
        thr = o["mean"][k, b] + flag_sigma * o["std"][k, b]
        assert abs(o["rms"][s] - thr) <= 1e-12 * thr, (s, o["rms"][s], thr)
    return len(diff)


@pytest.mark.parametrize("nstars,nchips,nmagbins,kw", [
    (300, 1, 60, {}),
    (2000, 3, 60, dict(clip_sigma=2.0, max_iter=10)),
    (5000, 11, 60, dict(max_iter=0)),
    (777, 4, 4096, dict(width=0.001)),
    (3000, 1, 1, dict(width=10.0)),      # one bin, 750 members per wave
    (6000, 1, 1, dict(width=10.0)),      # beyond a wave's LDS list: rescan
    (5000, 2, 2, dict(width=3.0, clip_sigma=2.5, max_iter=20)),
    # (clip 1 would shrink sets to two members that sit exactly one
    # deviation from their mean: a tie that rounding decides)
    (3000, 7, 30, dict(clip_sigma=1.5, max_iter=64, min_stars=10)),
])
def test_small_fields(bls, plan, nstars, nchips, nmagbins, kw):
    b, mag, chip_off, _ = synth.variability_field(nstars, nchips,
                                                  seed=500 + nstars)
    args = dict(origin=14.0)
    args.update(kw)
    _say("variability", nstars, nchips, nmagbins, kw)
    g = _run(bls, plan, b.x, None, b.n_off, mag, chip_off, nmagbins, **args)
    o = oracle.variability(b.x, None, b.n_off, mag, chip_off, nmagbins,
                           **args)
    _compare.chip_off = chip_off
    assert _compare(g, o, nchips, nmagbins, args.get("flag_sigma", 2.0)) == 0


def test_edge_cases(bls, plan):
    """Invalid and empty stars, out-of-range magnitudes, empty chips, zero
    weights, a bin whose clipping empties it, identical values."""
    rng = np.random.default_rng(3)
    b, mag, _, _ = synth.variability_field(400, 1, seed=77)
    x = b.x.copy()
    n_off = b.n_off.copy()
    x[n_off[5] + 2] = np.nan                  # invalid star 5
    mag = mag.copy()
    mag[7] = 99.0                              # out of range
    mag[8] = np.nan
    mag[9] = 13.0                              # below origin
    w = rng.choice([0.0, 1.0, 2.0], x.size)
    w[n_off[:-1]] = 1.0
    w[n_off[11]:n_off[12]] = 0.0               # star 11: no kept value
    chip_off = np.array([0, 0, 150, 150, 400, 400], np.int64)  # empty chips
    _say("variability edge cases")
    g = _run(bls, plan, x, w, n_off, mag, chip_off, 60, origin=14.0)
    o = oracle.variability(x, w, n_off, mag, chip_off, 60, origin=14.0)
    _compare.chip_off = chip_off
    assert _compare(g, o, 5, 60) == 0
    assert g["flag"][5] == -1 and g["flag"][11] == -1
    assert g["bin"][7] == -1 and g["bin"][8] == -1 and g["bin"][9] == -1
    # identical stars; then two values that a tight clip drops entirely
    vals = [0.5] * 6 + [0.0, 2.0]
    xs = np.concatenate([[v, -v] for v in vals])
    no = np.arange(0, 2 * len(vals) + 1, 2, dtype=np.int64)
    m2 = np.array([12.05] * 6 + [12.15] * 2)
    for clip in (0.5, 3.0):
        _say("variability tiny bins", clip)
        g = _run(bls, plan, xs, None, no, m2, [0, 8], 2, origin=12.0,
                 clip_sigma=clip, min_stars=1)
        o = oracle.variability(xs, None, no, m2, [0, 8], 2, origin=12.0,
                               clip_sigma=clip, min_stars=1)
        _compare.chip_off = np.array([0, 8])
        assert _compare(g, o, 1, 2) == 0


def test_errors(bls, plan):
    b, mag, chip_off, _ = synth.variability_field(50, 2, seed=8)
    for kw, st in ((dict(nmagbins=4097), bls.BLS_ERR_CAPACITY),
                   (dict(max_iter=65), bls.BLS_ERR_CAPACITY),
                   (dict(width=0.0), bls.BLS_ERR_INVALID_ARG),
                   (dict(chip_off=np.array([0, 20, 49])), bls.BLS_ERR_INVALID_ARG)):
        a = dict(nmagbins=10, chip_off=chip_off)
        a.update(kw)
        nmb = a.pop("nmagbins")
        co = a.pop("chip_off")
        _say("variability error", kw)
        with pytest.raises(bls.BlsError) as ei:
            _run(bls, plan, b.x, None, b.n_off, mag, co, nmb, origin=14.0, **a)
        assert ei.value.status == st


def test_full_field(bls, plan):
    """One pointing at full size: 100000 stars on 11 chips, 60 bins."""
    b, mag, chip_off, var = synth.variability_field()
    _say("variability full", b.ncurves, b.total_points())
    g = _run(bls, plan, b.x, None, b.n_off, mag, chip_off, 60, origin=14.0)
    o = oracle.variability(b.x, None, b.n_off, mag, chip_off, 60, origin=14.0)
    _compare.chip_off = chip_off
    nd = _compare(g, o, 11, 60)
    _say("variability full: flag differences at thresholds", nd)
    assert (g["flag"][var] == 1).mean() > 0.9
