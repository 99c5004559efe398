"""Pins of the FP64 oracle against things other than itself (CPU only).

The paper (Law et al. 2011, section 2.2.2) prints no formula and no worked
example, so the oracle is pinned by: hand-derived fixtures (tests/golden),
an independent unbinned brute force, closed forms of noiseless boxes, an
independent least-squares library fit, exact rational bin arithmetic, a
bound, invariances, and a prefix-sum reformulation of the box sums.  Each
test says which plausible mistake it would catch.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from tests.bruteforce import unbinned_best

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "box_fixtures.json")


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ---------------------------------------------------------------- fixtures
def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_golden_fixture(case):
    """Hand-derived worked examples (sign, wrap, weights, ties, dropping)."""
    r = oracle.search(case["t"], case["x"], case["w"], [case["period"]],
                      case["nbins"], case["qmin"], case["qmax"],
                      dip_only=case["dip_only"])
    e = case["expected"]
    assert r.jstart[0] == e["jstart"] and r.kwidth[0] == e["kwidth"]
    if e["sr"] == 0.0:
        assert r.sr[0] == 0.0 and math.isnan(r.depth[0])
    else:
        assert _rel(r.sr[0], e["sr"]) < 1e-12
        assert _rel(r.depth[0], e["depth"]) < 1e-10
    assert r.best_index == 0


# ------------------------------------------------------ P1: brute force
def _distinct_bin_curve(rng, n, period, nbins):
    """Reject-sample times until every point has a bin of its own."""
    while True:
        t = np.sort(synth.T_START + rng.uniform(0, 20, n))
        x = 1.0 + 0.01 * rng.standard_normal(n)
        b, _, _, _ = oracle.bins(t, x, None, period, nbins)
        if len(set(b.tolist())) == n:
            return t, x


@pytest.mark.parametrize("seed", range(6))
def test_p1_binned_equals_unbinned_when_bins_are_fine(seed):
    """Every point in its own bin and all widths allowed => the binned search
    sees every cyclic run of points, so its max equals the unbinned max.
    Catches wrong phase order, a broken wrap, a dropped term or a wrong max."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(4, 9))
    nbins = 4096
    periods = rng.uniform(0.3, 3.0, 2)
    weighted = seed % 2 == 1
    for P in periods:
        t, x = _distinct_bin_curve(rng, n, P, nbins)
        w = rng.uniform(0.5, 2.0, n) if weighted else None
        r = oracle.search(t, x, w, [P], nbins, 1e-6, 0.99999)
        assert r.kmin == 1 and r.kmax == nbins - 1
        v, _ = unbinned_best(t, x, w, P)
        assert _rel(r.sr[0] ** 2, v) < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_p1_binned_never_beats_unbinned(seed):
    """Coarse bins: binned boxes are a subset of cyclic runs, so <=."""
    rng = np.random.default_rng(200 + seed)
    n = 9
    t = np.sort(synth.T_START + rng.uniform(0, 10, n))
    x = 1.0 + 0.02 * rng.standard_normal(n)
    periods = rng.uniform(0.2, 2.0, 5)
    r = oracle.search(t, x, None, periods, 8, 0.1, 0.5)
    for p, P in enumerate(periods):
        v, _ = unbinned_best(t, x, None, P)
        assert r.sr[p] ** 2 <= v * (1 + 1e-12)


def test_p1_dip_only_matches_unbinned():
    rng = np.random.default_rng(7)
    n, nbins = 7, 4096
    P = 1.3
    t, x = _distinct_bin_curve(rng, n, P, nbins)
    r = oracle.search(t, x, None, [P], nbins, 1e-6, 0.99999, dip_only=True)
    v, _ = unbinned_best(t, x, None, P, dip_only=True)
    assert _rel(r.sr[0] ** 2, v) < 1e-12


# -------------------------------------------- bins vs exact rationals
def test_bins_match_exact_rational_phase():
    """The bin of each point equals floor(frac(d/P) * nbins) evaluated in exact
    rational arithmetic on the same doubles, except within rounding reach of
    a bin edge.  Catches a wrong t0, f or phase formula."""
    rng = np.random.default_rng(11)
    t = np.sort(synth.T_START + rng.uniform(0, 120, 400))
    x = np.ones_like(t)
    for P in (0.1, 0.37, 1.7, 19.9):
        nbins = 1000
        b, _, _, hn = oracle.bins(t, x, None, P, nbins)
        t0 = Fraction(float(t.min()))
        fP = Fraction(float(P))
        assert hn.sum() == t.size
        for i in range(t.size):
            d = Fraction(float(t[i] - t.min()))      # the one rounded step
            assert abs(float(d - (Fraction(float(t[i])) - t0))) < 1e-9
            ph = (d / fP) % 1
            exact = ph * nbins
            eb = int(math.floor(exact))
            if eb != b[i]:
                edge = min(abs(exact - eb), abs(exact - eb - 1))
                assert float(edge) < 1e-7, (P, i, eb, b[i])


# --------------------------------------------- P2: noiseless closed form
def _inject_on_oracle_bins(rng, t, P, nbins, k0, weighted, delta, wrap):
    b, _, _, hn = oracle.bins(t, np.ones_like(t), None, P, nbins)
    for _ in range(1000):
        j0 = int(nbins - 1 - rng.integers(0, k0 - 1)) if wrap else int(
            rng.integers(1, nbins - k0 - 1))
        ins = [(j0 + m) % nbins for m in range(k0)]
        edges = [ins[0], ins[-1], (j0 - 1) % nbins, (j0 + k0) % nbins]
        if all(hn[e] > 0 for e in edges):
            break
    else:
        pytest.skip("no box with non-empty edges")
    inbox = np.isin(b, ins)
    c = 1.37
    x = np.where(inbox, c - delta, c)
    w = rng.uniform(0.5, 2.0, t.size) if weighted else None
    ww = np.ones_like(t) if w is None else w
    r_frac = math.fsum(ww[inbox]) / math.fsum(ww)
    return x, w, j0, r_frac


@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("wrap", [False, True])
def test_p2_noiseless_box_closed_form(weighted, wrap):
    """x = c - delta on a box of the oracle's own bins at period P*:
    SR = delta sqrt(r(1-r)), box = (j0, k0), step = delta, and no period
    beats P*.  Catches a wrong formula, sign, or window bookkeeping."""
    rng = np.random.default_rng(31 + weighted + 2 * wrap)
    t = synth.nightly_times(rng, 300)
    periods = synth.log_period_grid(0.3, 5.0, 400)
    ps = 137
    nbins, k0, delta = 100, 6, 0.03
    x, w, j0, r = _inject_on_oracle_bins(rng, t, periods[ps], nbins, k0,
                                         weighted, delta, wrap)
    res = oracle.search(t, x, w, periods, nbins, 0.02, 0.15)
    assert res.jstart[ps] == j0 and res.kwidth[ps] == k0
    assert _rel(res.sr[ps], delta * math.sqrt(r * (1 - r))) < 1e-12
    assert _rel(res.depth[ps], delta) < 1e-10
    assert np.all(res.sr <= res.sr[ps] * (1 + 1e-12))


# ------------------------------------------------------ P3: variance bound
def test_p3_variance_bound():
    lc = synth.small_curve(5, 500, nperiods=300, nbins=80)
    r = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                      lc.qmax)
    xbar = math.fsum(lc.x) / lc.n
    var = math.fsum((xi - xbar) ** 2 for xi in lc.x) / lc.n
    assert _rel(r.sumwy2 / r.W, var) < 1e-12
    assert np.all(r.sr ** 2 <= var * (1 + 1e-12))
    assert np.any(r.sr > 0)


# ------------------------------------------------ P4: least-squares library
def _wls_chi2(A, x, w):
    sw = np.sqrt(w)
    coef, *_ = np.linalg.lstsq(A * sw[:, None], x * sw, rcond=None)
    res = x - A @ coef
    return float(np.sum(w * res * res)), coef


@pytest.mark.parametrize("weighted", [False, True])
def test_p4_lstsq_identity_for_returned_box(weighted):
    """W SR^2 equals the chi^2 drop between numpy lstsq fits of [1] and
    [1, box indicator]; the fitted step equals -depth.  Pins the statistic to
    an independent library routine rather than to its own formula."""
    lc = synth.small_curve(9, 300, nperiods=40, nbins=50, weighted=weighted)
    r = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                      lc.qmax)
    w = np.ones(lc.n) if lc.w is None else lc.w
    one = np.ones((lc.n, 1))
    chi0, _ = _wls_chi2(one, lc.x, w)
    for p in range(0, 40, 7):
        b, _, _, _ = oracle.bins(lc.t, lc.x, lc.w, lc.periods[p], lc.nbins)
        j, k = int(r.jstart[p]), int(r.kwidth[p])
        inbox = np.isin(b, [(j + m) % lc.nbins for m in range(k)])
        A = np.column_stack([one[:, 0], inbox.astype(float)])
        chi1, coef = _wls_chi2(A, lc.x, w)
        assert _rel(chi0 - chi1, r.W * r.sr[p] ** 2) < 1e-8
        assert _rel(-coef[1], r.depth[p]) < 1e-8


def test_p4_lstsq_max_over_all_boxes():
    """The best box is the lstsq-best over every (j, k) box (small nbins)."""
    lc = synth.small_curve(13, 120, nperiods=3, nbins=16, qmin=0.07,
                           qmax=0.3)
    r = oracle.search(lc.t, lc.x, None, lc.periods, lc.nbins, lc.qmin,
                      lc.qmax)
    one = np.ones((lc.n, 1))
    w = np.ones(lc.n)
    chi0, _ = _wls_chi2(one, lc.x, w)
    for p in range(3):
        b, _, _, _ = oracle.bins(lc.t, lc.x, None, lc.periods[p], lc.nbins)
        best = 0.0
        for j in range(lc.nbins):
            for k in range(r.kmin, r.kmax + 1):
                inbox = np.isin(b, [(j + m) % lc.nbins for m in range(k)])
                if inbox.sum() == 0 or inbox.sum() == lc.n:
                    continue
                A = np.column_stack([one[:, 0], inbox.astype(float)])
                chi1, _ = _wls_chi2(A, lc.x, w)
                best = max(best, chi0 - chi1)
        assert _rel(best, r.W * r.sr[p] ** 2) < 1e-8


# ----------------------------------------------------- P5-P7 invariances
@pytest.fixture(scope="module")
def noisy():
    lc = synth.small_curve(21, 400, nperiods=120, nbins=60)
    r = oracle.search(lc.t, lc.x, None, lc.periods, lc.nbins, lc.qmin,
                      lc.qmax)
    return lc, r


@pytest.mark.parametrize("C,tol", [(0.5, 1e-10), (-0.5, 1e-10), (1e3, 1e-8)])
def test_p5_offset_invariance(noisy, C, tol):
    """x + C leaves SR, j, k unchanged.  The tolerance grows with C because
    the FP64 mean of values near C carries a rounding error of about
    n eps C / n, which shifts every residual by the same amount."""
    lc, r = noisy
    r2 = oracle.search(lc.t, lc.x + C, None, lc.periods, lc.nbins, lc.qmin,
                       lc.qmax)
    assert np.max(np.abs(r2.sr - r.sr) / r.sr) < tol
    assert np.array_equal(r2.jstart, r.jstart)
    assert np.array_equal(r2.kwidth, r.kwidth)


@pytest.mark.parametrize("a", [3.0, -2.0, 0.5])
def test_p6_flux_scale(noisy, a):
    lc, r = noisy
    r2 = oracle.search(lc.t, a * lc.x, None, lc.periods, lc.nbins, lc.qmin,
                       lc.qmax)
    assert np.max(np.abs(r2.sr - abs(a) * r.sr) / r.sr) < 1e-12
    assert np.max(np.abs(r2.depth - a * r.depth) / np.abs(r.depth)) < 1e-10
    assert np.array_equal(r2.jstart, r.jstart)


def test_p6_weight_scale_and_sign():
    lc = synth.small_curve(22, 300, nperiods=80, nbins=50, weighted=True)
    r = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                      lc.qmax)
    r2 = oracle.search(lc.t, lc.x, 7.3 * lc.w, lc.periods, lc.nbins,
                       lc.qmin, lc.qmax)
    assert np.max(np.abs(r2.sr - r.sr) / r.sr) < 1e-12
    assert np.array_equal(r2.kwidth, r.kwidth)
    r3 = oracle.search(lc.t, -lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                       lc.qmax)
    assert np.max(np.abs(r3.sr - r.sr) / r.sr) < 1e-12
    assert np.max(np.abs(r3.depth + r.depth) / np.abs(r.depth)) < 1e-10


def _all_box_values(hw, hs, hn, kmin, kmax, W, n):
    """(j, k) -> (v, S) over all boxes, by prefix-sum differences."""
    nb = hw.size
    ew = np.concatenate([[0.0], np.cumsum(np.concatenate([hw, hw]))])
    es = np.concatenate([[0.0], np.cumsum(np.concatenate([hs, hs]))])
    en = np.concatenate([[0], np.cumsum(np.concatenate([hn, hn]))])
    out = {}
    for j in range(nb):
        for k in range(kmin, kmax + 1):
            R = ew[j + k] - ew[j]
            S = es[j + k] - es[j]
            nin = en[j + k] - en[j]
            if nin < 1 or nin > n - 1:
                continue
            out[(j, k)] = (S * S / (R * (W - R)), S)
    return out


def test_p6_dip_only_selects_negative_boxes():
    """Dip-only on x equals the best S<0 box; on -x the best S>0 box of x."""
    lc = synth.small_curve(23, 250, nperiods=10, nbins=40)
    for sign in (1.0, -1.0):
        r = oracle.search(lc.t, sign * lc.x, None, lc.periods, lc.nbins,
                          lc.qmin, lc.qmax, dip_only=True)
        for p in range(10):
            _, hw, hs, hn = oracle.bins(lc.t, lc.x, None, lc.periods[p],
                                        lc.nbins)
            vals = _all_box_values(hw, hs, hn, r.kmin, r.kmax, r.W, r.n)
            best = max((v for v, S in vals.values() if sign * S < 0),
                       default=0.0)
            assert _rel(r.sr[p] ** 2, best) < 1e-9
            if r.kwidth[p] > 0:
                assert r.depth[p] > 0


def test_p7_permutation_invariance(noisy):
    lc, r = noisy
    perm = np.random.default_rng(3).permutation(lc.n)
    r2 = oracle.search(lc.t[perm], lc.x[perm], None, lc.periods, lc.nbins,
                       lc.qmin, lc.qmax)
    assert np.max(np.abs(r2.sr - r.sr) / r.sr) < 1e-12
    assert np.array_equal(r2.jstart, r.jstart)
    assert np.array_equal(r2.kwidth, r.kwidth)
    b1, *_ = oracle.bins(lc.t, lc.x, None, lc.periods[5], lc.nbins)
    b2, *_ = oracle.bins(lc.t[perm], lc.x[perm], None, lc.periods[5],
                         lc.nbins)
    assert np.array_equal(b1[perm], b2)


# ------------------------------------------------ P8: internal consistency
@pytest.mark.parametrize("weighted", [False, True])
def test_p8_window_sums_match_prefix_differences(weighted):
    lc = synth.small_curve(41, 500, nperiods=12, nbins=70, weighted=weighted)
    r = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                      lc.qmax)
    for p in range(12):
        _, hw, hs, hn = oracle.bins(lc.t, lc.x, lc.w, lc.periods[p],
                                    lc.nbins)
        vals = _all_box_values(hw, hs, hn, r.kmin, r.kmax, r.W, r.n)
        best = max(v for v, _ in vals.values())
        assert _rel(r.sr[p] ** 2, best) < 1e-10
        v_at = vals[(int(r.jstart[p]), int(r.kwidth[p]))][0]
        assert _rel(v_at, best) < 1e-10


def _tie_curve(used, low):
    nbins = 64
    offs = np.array([0.0] + [(b + 0.5) / nbins for b in used[1:]])
    x = np.where(np.isin(used, low), 0.95, 1.0)
    return synth.T_START + offs, x


def test_p8_empty_bin_ties_go_to_smallest_width_then_start():
    """Equal-valued boxes: the same point set reached through extra empty bins
    goes to the smallest width; two disjoint boxes with bit-identical sums go
    to the smallest start.  64 bins, widths 1..6; low pairs in bins 0-1 and
    40-41, single normal points in bins 10, 20, 30, 55 (no window of 6 bins
    holds two normal points)."""
    nbins = 64
    used = [0, 1, 10, 20, 30, 40, 41, 55]
    t, x = _tie_curve(used, [0, 1, 40, 41])
    b, *_ = oracle.bins(t, x, None, 1.0, nbins)
    assert b.tolist() == used
    r = oracle.search(t, x, None, [1.0], nbins, 0.02, 0.1)
    assert r.kmin == 1 and r.kmax == 6
    # (0,2) ties exactly with (40,2) and with wider boxes such as (63,3),
    # (62,4), (0,3) and (39,3) that add only empty bins
    assert (r.jstart[0], r.kwidth[0]) == (0, 2)
    # one low pair, in bins 40-41: the pair is returned, not a wider box
    used2 = [0, 10, 20, 30, 40, 41, 55]
    t2, x2 = _tie_curve(used2, [40, 41])
    r2 = oracle.search(t2, x2, None, [1.0], nbins, 0.02, 0.1)
    assert (r2.jstart[0], r2.kwidth[0]) == (40, 2)


# ------------------------------------------------------- P9: recovery
def test_p9_recovers_injected_period_config1():
    lc = synth.config1()
    r = oracle.search(lc.t, lc.x, lc.w, lc.periods, lc.nbins, lc.qmin,
                      lc.qmax)
    P = lc.periods[r.best_index]
    ok = [abs(P - a) / a < 0.01 for a in (1.7, 0.85, 3.4)]
    assert any(ok), P


# --------------------------------------------------- invalid input
@pytest.mark.parametrize("bad", [
    dict(nbins=1), dict(qmin=0.0), dict(qmax=1.0), dict(qmin=0.3, qmax=0.2),
    dict(periods=[1.0, -1.0]), dict(periods=[np.nan]), dict(periods=[]),
    dict(min_in_points=0)])
def test_invalid_arguments_rejected(bad):
    lc = synth.small_curve(1, 50, nperiods=4, nbins=20)
    kw = dict(periods=lc.periods, nbins=20, qmin=0.05, qmax=0.2)
    kw.update(bad)
    mip = kw.pop("min_in_points", 1)
    with pytest.raises(oracle.OracleError):
        oracle.search(lc.t, lc.x, None, kw["periods"], kw["nbins"],
                      kw["qmin"], kw["qmax"], min_in_points=mip)


def test_invalid_data_rejected():
    lc = synth.small_curve(1, 50, nperiods=4, nbins=20)
    x = lc.x.copy()
    x[3] = np.nan
    with pytest.raises(oracle.OracleError):
        oracle.search(lc.t, x, None, lc.periods, 20, 0.05, 0.2)
    w = np.ones(lc.n)
    w[2] = -1
    with pytest.raises(oracle.OracleError):
        oracle.search(lc.t, lc.x, w, lc.periods, 20, 0.05, 0.2)
    w = np.zeros(lc.n)
    w[0] = 1
    with pytest.raises(oracle.OracleError):      # one kept point
        oracle.search(lc.t, lc.x, w, lc.periods, 20, 0.05, 0.2)
    # NaN flux on a zero-weight point is dropped, not an error
    w = np.ones(lc.n)
    w[3] = 0.0
    r = oracle.search(lc.t, x, w, lc.periods, 20, 0.05, 0.2)
    assert r.n == lc.n - 1


def test_min_in_points_rule():
    """A lone low point is found with min_in_points=1 and excluded at 2."""
    t = synth.T_START + np.array([0.0, 0.15, 0.25, 0.35, 0.45, 0.55, 0.65,
                                  0.75])
    x = np.array([1.0, 1.0, 1.0, 0.8, 1.0, 1.0, 1.0, 1.0])
    r1 = oracle.search(t, x, None, [1.0], 10, 0.1, 0.4)
    assert (r1.jstart[0], r1.kwidth[0]) == (3, 1)
    r2 = oracle.search(t, x, None, [1.0], 10, 0.1, 0.4, min_in_points=2)
    assert r2.kwidth[0] >= 2
