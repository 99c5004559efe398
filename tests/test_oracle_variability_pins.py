"""Pins of the oracle's high-variability pre-search (CPU only).

A star's stability is the population RMS of its values; the expected
stability per (chip, 0.1-mag bin) is an iterated sigma-clipped mean; stars
above it by more than 2 deviations are flagged (readings V1-V4 in
bls_oracle.c).  Pinned against numpy's RMS, scipy's sigma clipping, and
hand-worked bins.
"""
import numpy as np
import pytest
from scipy import stats

import oracle


def _stars_with_rms(values):
    """One two-point curve per value v: points +v and -v, RMS exactly |v|."""
    x = np.concatenate([[v, -v] for v in values]).astype(np.float64)
    n_off = np.arange(0, 2 * len(values) + 1, 2, dtype=np.int64)
    return x, n_off


def test_rms_is_population_std():
    rng = np.random.default_rng(1)
    n = rng.integers(1, 300, 40)
    n_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    x = rng.normal(1.0, 0.01, n_off[-1]) * rng.uniform(0.5, 2, n_off[-1])
    r = oracle.variability(x, None, n_off, np.full(40, 15.0), [0, 40], 10,
                           origin=14.0)
    for c in range(40):
        seg = x[n_off[c]:n_off[c + 1]]
        assert abs(r["rms"][c] - np.std(seg)) <= 1e-14 * max(np.std(seg), 1e-300)
    # zero weights drop points; other weights do not weigh the RMS
    w = rng.choice([0.0, 1.0, 3.0], n_off[-1])
    for c in range(40):
        w[n_off[c]] = 1.0
    r2 = oracle.variability(x, w, n_off, np.full(40, 15.0), [0, 40], 10,
                            origin=14.0)
    for c in range(40):
        seg = x[n_off[c]:n_off[c + 1]][w[n_off[c]:n_off[c + 1]] > 0]
        assert abs(r2["rms"][c] - np.std(seg)) <= 1e-14 * max(np.std(seg), 1e-300)


@pytest.mark.parametrize("seed,clip", [(0, 3.0), (1, 2.0), (2, 1.5), (3, 2.5)])
def test_clipping_matches_scipy_sigmaclip(seed, clip):
    rng = np.random.default_rng(seed)
    vals = np.abs(np.concatenate([rng.normal(0.01, 0.002, 120),
                                  rng.uniform(0.02, 0.2, 12)]))
    rng.shuffle(vals)
    x, n_off = _stars_with_rms(vals)
    mag = np.full(vals.size, 16.05)
    r = oracle.variability(x, None, n_off, mag, [0, vals.size], 1,
                           origin=16.0, width=0.1, clip_sigma=clip,
                           max_iter=1000, flag_sigma=2.0)
    kept = stats.sigmaclip(vals, clip, clip).clipped
    assert r["count"][0, 0] == kept.size
    assert abs(r["mean"][0, 0] - kept.mean()) <= 1e-15
    assert abs(r["std"][0, 0] - kept.std()) <= 1e-15
    thr = kept.mean() + 2.0 * kept.std()
    assert np.array_equal(r["flag"], (vals > thr).astype(np.int32))


def test_hand_worked_bin():
    # rms values 1,1,1,1,10: mean 2.8, deviation 3.6
    x, n_off = _stars_with_rms([1.0, 1.0, 10.0, 1.0, 1.0])
    mag = np.full(5, 12.1)
    # clip 3: 10 is 2 deviations out, kept; flag above 2.8 + 1.5*3.6 = 8.2
    r = oracle.variability(x, None, n_off, mag, [0, 5], 1, origin=12.0,
                           clip_sigma=3.0, flag_sigma=1.5)
    assert r["count"][0, 0] == 5
    assert abs(r["mean"][0, 0] - 2.8) < 1e-15 and abs(r["std"][0, 0] - 3.6) < 1e-15
    assert r["flag"].tolist() == [0, 0, 1, 0, 0]
    # clip 1.5: 10 is dropped, the rest have deviation 0 and 10 is flagged
    r = oracle.variability(x, None, n_off, mag, [0, 5], 1, origin=12.0,
                           clip_sigma=1.5, flag_sigma=2.0)
    assert r["count"][0, 0] == 4
    assert r["mean"][0, 0] == 1.0 and r["std"][0, 0] == 0.0
    assert r["flag"].tolist() == [0, 0, 1, 0, 0]
    # no clipping rounds: every member counts and 10 < 2.8 + 2.5*3.6 = 11.8
    r = oracle.variability(x, None, n_off, mag, [0, 5], 1, origin=12.0,
                           clip_sigma=1.5, max_iter=0, flag_sigma=2.5)
    assert r["count"][0, 0] == 5 and r["flag"].tolist() == [0, 0, 0, 0, 0]
    # too few stars after clipping: nothing flagged
    r = oracle.variability(x, None, n_off, mag, [0, 5], 1, origin=12.0,
                           clip_sigma=1.5, flag_sigma=2.0, min_stars=5)
    assert r["flag"].tolist() == [0] * 5
    # exactly min_stars members left is enough
    r = oracle.variability(x, None, n_off, mag, [0, 5], 1, origin=12.0,
                           clip_sigma=1.5, flag_sigma=2.0, min_stars=4)
    assert r["flag"].tolist() == [0, 0, 1, 0, 0]


def test_one_clipping_round_at_a_time():
    # 1,1,1,1,1,1,5,50: round 1 drops 50 only (5 is within 1.2 deviations),
    # round 2 drops 5; max_iter=1 stops after the first drop.
    v = [1.0] * 6 + [5.0, 50.0]
    x, n_off = _stars_with_rms(v)
    mag = np.full(8, 12.1)
    r1 = oracle.variability(x, None, n_off, mag, [0, 8], 1, origin=12.0,
                            clip_sigma=1.2, max_iter=1)
    assert r1["count"][0, 0] == 7
    assert abs(r1["mean"][0, 0] - np.mean(v[:7])) < 1e-15
    r2 = oracle.variability(x, None, n_off, mag, [0, 8], 1, origin=12.0,
                            clip_sigma=1.2, max_iter=2)
    assert r2["count"][0, 0] == 6 and r2["std"][0, 0] == 0.0


def test_bins_chips_and_invalid_stars():
    # width 0.25 is exact: mag 12.0 is the first edge of bin 8 from origin 10
    vals = [0.01, 0.01, 0.01, 0.2, 0.01, 0.01, 0.01, 0.2, 0.5, 0.5]
    mag = np.array([12.0, 12.1, 12.2, 12.24, 11.99, 11.9, 11.8, 11.76, 9.99,
                    np.nan])
    x, n_off = _stars_with_rms(vals)
    x[2 * 9] = np.inf                           # star 9 invalid
    r = oracle.variability(x, None, n_off, mag, [0, 10], 12, origin=10.0,
                           width=0.25, clip_sigma=3.0, flag_sigma=1.0)
    assert r["bin"].tolist() == [8, 8, 8, 8, 7, 7, 7, 7, -1, -1]
    assert r["flag"][8] == 0 and r["flag"][9] == -1 and np.isnan(r["rms"][9])
    assert r["count"][0, 8] == 4 and r["count"][0, 7] == 4
    assert r["flag"][[3, 7]].tolist() == [1, 1]
    assert r["count"][0, 0] == 0 and np.isnan(r["mean"][0, 0])
    # the same stars split over two chips are binned separately
    r2 = oracle.variability(x, None, n_off, mag, [0, 4, 10], 12,
                            origin=10.0, width=0.25, clip_sigma=3.0,
                            flag_sigma=1.0)
    assert r2["count"][0, 8] == 4 and r2["count"][1, 8] == 0
    assert r2["count"][1, 7] == 4 and r2["count"][0, 7] == 0
    assert np.array_equal(r2["flag"], r["flag"])


def test_star_order_within_a_chip_only_rounds():
    rng = np.random.default_rng(9)
    vals = np.abs(rng.normal(0.01, 0.003, 500))
    mag = rng.uniform(14, 18, 500)
    x, n_off = _stars_with_rms(vals)
    r = oracle.variability(x, None, n_off, mag, [0, 500], 40, origin=14.0)
    perm = rng.permutation(500)
    xp, n_offp = _stars_with_rms(vals[perm])
    rp = oracle.variability(xp, None, n_offp, mag[perm], [0, 500], 40,
                            origin=14.0)
    assert np.array_equal(rp["flag"], r["flag"][perm])
    assert np.array_equal(rp["count"], r["count"])
    ok = r["count"] > 0
    assert np.allclose(rp["mean"][ok], r["mean"][ok], rtol=1e-13, atol=0)


@pytest.mark.parametrize("kw", [dict(width=0.0), dict(clip_sigma=0.0),
                                dict(max_iter=-1), dict(min_stars=0),
                                dict(chip_off=[0, 3])])
def test_invalid_arguments(kw):
    x, n_off = _stars_with_rms([1.0, 2.0, 3.0, 4.0])
    a = dict(x=x, w=None, n_off=n_off, mag=np.full(4, 12.0),
             chip_off=[0, 4], nmagbins=4)
    a.update(kw)
    with pytest.raises(oracle.OracleError):
        oracle.variability(**a)
