"""Comparison of GPU results with the FP64 oracle (test helper).

Acceptance rule (the search maximises over boxes and over periods, so where
several answers are equally correct only what is unique is compared):

* SR of every period within REL_TOL relative of the oracle (0 where the
  oracle finds no box, and then no box on the GPU either);
* the GPU's box (j, k) equals the oracle's, or the oracle's own statistic
  at the GPU's box is within REL_TOL of the oracle's best (a near-tie);
* the best period index equals the oracle's, or every period whose oracle SR
  lies within REL_TOL of the maximum is acceptable.
"""
from __future__ import annotations

import numpy as np

import oracle

REL_TOL = 1e-5


def oracle_box_sr(lc, period, j, k, nbins):
    """The oracle's FP64 SR of box (j, k) at one period, from its bins."""
    _, hw, hs, hn = oracle.bins(lc.t, lc.x, lc.w, period, nbins)
    idx = [(j + m) % nbins for m in range(k)]
    R = float(np.sum(hw[idx]))
    S = float(np.sum(hs[idx]))
    W = float(np.sum(hw))
    den = R * (W - R)
    return 0.0 if den <= 0 else float(np.sqrt(S * S / den))


def check_curve(lc, gpu, orc, tol=REL_TOL, sr_key="sr", label=""):
    """Assert the acceptance rule for one curve; returns error statistics."""
    sr_g = np.asarray(gpu[sr_key], dtype=np.float64)
    js_g = np.asarray(gpu["jstart"])
    ks_g = np.asarray(gpu["kwidth"])
    sr_o = orc.sr
    none_o = orc.kwidth < 0
    assert np.all(sr_g[none_o] == 0.0), label + ": SR where the oracle has no box"
    assert np.all(ks_g[none_o] < 0), label + ": box where the oracle has none"
    some = ~none_o
    rel = np.abs(sr_g[some] - sr_o[some]) / sr_o[some]
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= tol, "%s: max rel SR error %.3g at period %d" % (
        label, worst, int(np.flatnonzero(some)[np.argmax(rel)]))
    mism = np.flatnonzero(some & ((js_g != orc.jstart) | (ks_g != orc.kwidth)))
    for p in mism:
        alt = oracle_box_sr(lc, lc.periods[p], int(js_g[p]), int(ks_g[p]),
                            lc.nbins)
        assert alt >= (1 - tol) * sr_o[p], (
            "%s: period %d GPU box (%d,%d) SR %.9g vs oracle (%d,%d) %.9g" % (
                label, p, js_g[p], ks_g[p], alt, orc.jstart[p],
                orc.kwidth[p], sr_o[p]))
    match = some & (js_g == orc.jstart) & (ks_g == orc.kwidth)
    if "depth" in gpu:
        dg = np.asarray(gpu["depth"], dtype=np.float64)[match]
        do = orc.depth[match]
        drel = np.abs(dg - do) / np.abs(do)
        assert drel.size == 0 or drel.max() <= 10 * tol, (
            "%s: depth rel err %.3g" % (label, drel.max()))
    bi = int(gpu["best_index"])
    if bi != orc.best_index:
        top = sr_o.max()
        near = np.flatnonzero(sr_o >= (1 - tol) * top)
        assert bi in near, "%s: best index %d not in oracle near-ties %s" % (
            label, bi, near[:10])
    return dict(max_rel=worst,
                p99_rel=float(np.percentile(rel, 99)) if rel.size else 0.0,
                box_mismatch=int(mism.size))
