"""Pins of the oracle's injection-recovery (CPU only).

The oracle injects box eclipses into copies of one cadence by folding each
point at the injected period (readings I1-I3 in bls_oracle.c), searches each
copy and applies the recovery rule I4 to its detection statistics.  These
tests pin the injection without folding, on the time axis, with exact
rational arithmetic; by closed forms of a regular cadence; and the whole
chain by the closed form of a noiseless box aligned to the search's bins,
whose statistic no other period can exceed.

Exactness: times are an HJD-like origin plus multiples of 2^-8 day, periods
powers of two and phases and duty cycles multiples of 2^-6, so every FP64
operation of the fold is exact and its eclipses coincide with time intervals.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle

T_START = 2455000.5


def binary_times(rng, n, span_days):
    k = np.sort(rng.choice(np.arange(int(span_days * 256)), n, replace=False))
    return T_START + k / 256.0


def in_eclipse_time_domain(t, keep, P, phi, q):
    """Eclipse m covers [t0 + (m + phi) P, t0 + (m + phi + q) P) on the time
    axis (t0 = earliest kept time); rational arithmetic, no folding."""
    t0 = min(Fraction(float(x)) for x, k in zip(t, keep) if k)
    P, phi, q = Fraction(P), Fraction(phi), Fraction(q)
    out = np.zeros(len(t), bool)
    for i, x in enumerate(t):
        if not keep[i]:
            continue
        d = Fraction(float(x)) - t0
        m = (d / P - phi).__floor__()
        out[i] = (m + phi) * P <= d < (m + phi + q) * P
    return out


@pytest.mark.parametrize("seed", range(8))
def test_inject_matches_time_domain(seed):
    rng = np.random.default_rng(400 + seed)
    n = int(rng.integers(20, 400))
    t = binary_times(rng, n, 40)
    w = None
    keep = np.ones(n, bool)
    if seed % 2:
        w = rng.uniform(0.5, 2.0, n)
        drop = rng.random(n) < 0.2
        w[drop] = 0.0
        keep = ~drop
    ninj = 5
    P = 2.0 ** rng.integers(-3, 4, ninj)
    phi = rng.integers(0, 64, ninj) / 64.0
    q = rng.integers(1, 32, ninj) / 64.0
    depth = rng.uniform(0.001, 0.05, ninj)
    base = 1.0 + 0.01 * rng.standard_normal((ninj, n))
    x = oracle.inject(t, w, base, P, phi, q, depth)
    for i in range(ninj):
        ecl = in_eclipse_time_domain(t, keep, P[i], phi[i], q[i])
        want = np.where(ecl, base[i] - depth[i], base[i])
        assert np.array_equal(x[i], want), "injection %d" % i


def test_inject_dropped_points_and_zero_depth():
    rng = np.random.default_rng(7)
    t = binary_times(rng, 300, 30)
    base = 1.0 + 0.01 * rng.standard_normal((3, t.size))
    w = np.ones(t.size)
    w[0] = 0.0              # the earliest time is not an observation
    x = oracle.inject(t, w, base, [0.5, 1.0, 2.0], [0.25, 0.5, 0.0],
                      [0.125, 0.25, 0.5], [0.0, 0.02, 0.03])
    assert np.array_equal(x[0], base[0])
    assert x[1, 0] == base[1, 0] and x[2, 0] == base[2, 0]
    # phases start at the earliest kept time, not at t[0]
    keep = w > 0
    ecl = in_eclipse_time_domain(t, keep, 1.0, 0.5, 0.25)
    assert np.array_equal(x[1] != base[1], ecl)


@pytest.mark.parametrize("per_cycle,q", [(64, 0.125), (96, 0.25), (40, 0.5)])
def test_inject_regular_cadence_count(per_cycle, q):
    """A regular cadence of per_cycle points per period over whole cycles:
    exactly q * per_cycle points of every cycle are in eclipse."""
    cycles = 11
    P = 1.0
    s = Fraction(1, per_cycle)
    t = np.array([float(T_START + k * s) for k in range(cycles * per_cycle)])
    assert all(Fraction(float(x)) == T_START + k * s for k, x in enumerate(t))
    base = np.ones((1, t.size))
    x = oracle.inject(t, None, base, P, 0.0, q, 0.01)
    assert int(np.sum(x[0] < 1.0)) == cycles * int(q * per_cycle)
    # shifting the eclipse by a whole number of points keeps the count
    x2 = oracle.inject(t, None, base, P, 3.0 / per_cycle, q, 0.01)
    assert int(np.sum(x2[0] < 1.0)) == int(np.sum(x[0] < 1.0))


def test_recovery_rule():
    thr, tol = 7.0, 0.01
    assert oracle.recovered(1.0, 7.0, 1.0, thr, tol)
    assert not oracle.recovered(1.0, 6.999, 1.0, thr, tol)
    assert oracle.recovered(2.0 * 1.009, 9.0, 2.0, thr, tol)
    assert not oracle.recovered(2.0 * 1.011, 9.0, 2.0, thr, tol)
    assert oracle.recovered(1.0, 9.0, 2.0, thr, tol)        # half
    assert oracle.recovered(4.0, 9.0, 2.0, thr, tol)        # double
    assert not oracle.recovered(6.0, 9.0, 2.0, thr, tol)    # triple
    assert not oracle.recovered(2.0 / 3.0, 9.0, 2.0, thr, tol)
    assert not oracle.recovered(float("nan"), 9.0, 2.0, thr, tol)


@pytest.mark.parametrize("seed", range(3))
def test_recovery_noiseless_aligned_box(seed):
    """Noiseless curve with one box injected at a trial period P* whose phase
    and duty cycle are whole bins of a power-of-two bin count: the eclipse is
    exactly the search's box (j0, k0), so its SR is delta sqrt(r (1 - r)) and
    no period exceeds it (the residual of a two-level fit is not negative);
    the best period is P*, an equal-SR period, or an alias, and the rule
    decides by the threshold alone."""
    rng = np.random.default_rng(500 + seed)
    nb = 64
    t = binary_times(rng, 600, 50)
    grid = np.exp(np.linspace(np.log(0.3), np.log(5.0), 400))
    pstar_i = int(rng.integers(50, 350))
    pstar = grid[pstar_i]
    j0, k0 = int(rng.integers(0, nb)), int(rng.integers(2, 6))
    delta = 0.03
    base = np.ones((1, t.size))
    r = oracle.recovery(t, None, base, pstar, j0 / nb, k0 / nb, delta, grid,
                        nb, 1.0 / nb, 6.0 / nb, sde_threshold=0.0)
    x = r["flux"][0]
    o = r["results"][0]
    inbox = x < 1.0
    rr = inbox.mean()
    assert 0 < inbox.sum() < t.size
    sr_star = delta * np.sqrt(rr * (1 - rr))
    assert o.sr[pstar_i] == pytest.approx(sr_star, rel=1e-12)
    assert o.sr.max() <= sr_star * (1 + 1e-12)
    b = int(r["best_index"][0])
    assert o.sr[b] == pytest.approx(sr_star, rel=1e-12)
    expect = oracle.recovered(grid[b], r["sde"][0], pstar, 0.0, 0.01)
    assert r["recovered"][0] == int(expect)
    if b == pstar_i:
        assert r["recovered"][0] == 1
    never = oracle.recovery(t, None, base, pstar, j0 / nb, k0 / nb, delta,
                            grid, nb, 1.0 / nb, 6.0 / nb,
                            sde_threshold=float("inf"))
    assert never["recovered"][0] == 0
