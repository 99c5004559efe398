"""Pins of the oracle's unbinned box search (CPU only).

The oracle enumerates cyclic runs of phase-sorted points and admits a run
when some box of duty cycle in [qmin, qmax] holds exactly it (readings
U1-U3 in bls_oracle.c).  Pinned by: the independent unbinned brute force
(every run, no duration limit), a direct search over boxes placed at all
critical phases with membership tested point by point, the closed form of
a noiseless box, the binned search (whose boxes are a subset), and
invariances.
"""
import math

import numpy as np
import pytest

import oracle
from tests.bruteforce import unbinned_best


def _phases(t, period):
    t0 = min(t)
    return [((ti - t0) / period) % 1.0 for ti in t]


def box_search(t, x, w, period, qmin, qmax):
    """Best S^2/(R(W-R)) over boxes [a, a+q) of phase, q in [qmin, qmax].

    Membership is tested directly, point by point.  In the (a, q) plane the
    held set is constant on the cells cut out by the lines a = phi_i,
    a + q = phi_j (mod 1), q = qmin and q = qmax; every cell has a vertex,
    and the lines through a vertex leave wedges of at least 45 degrees, so
    probing a small step from every vertex in 24 directions visits every
    cell.
    """
    w = [1.0] * len(t) if w is None else list(w)
    n = len(t)
    ph = _phases(t, period)
    W = math.fsum(w)
    xbar = math.fsum(wi * xi for wi, xi in zip(w, x)) / W
    verts = []
    for q in (qmin, qmax):
        for p in ph:
            verts += [(p, q), (p - q, q)]
    for pi in ph:
        for pj in ph:
            q = (pj - pi) % 1.0
            if qmin <= q <= qmax:
                verts.append((pi, q))
    step = 1e-9
    dirs = [(math.cos(math.radians(7.5 + 15 * k)),
             math.sin(math.radians(7.5 + 15 * k))) for k in range(24)]
    best = 0.0
    best_set = frozenset()
    seen = set()
    for (va, vq) in verts:
        for (da, dq) in dirs:
            a, q = va + step * da, vq + step * dq
            if not qmin <= q <= qmax:
                continue
            idx = frozenset(i for i in range(n) if (ph[i] - a) % 1.0 < q)
            if not idx or len(idx) == n or idx in seen:
                continue
            seen.add(idx)
            R = math.fsum(w[i] for i in idx)
            S = math.fsum(w[i] * (x[i] - xbar) for i in idx)
            v = S * S / (R * (W - R))
            if v > best:
                best, best_set = v, idx
    return best, best_set


def _run_set(t, P, first, last):
    """Points from first to last in (phase, index) order, cyclically."""
    ph = _phases(t, P)
    order = sorted(range(len(t)), key=lambda i: (ph[i], i))
    a, b = order.index(first), order.index(last)
    if b >= a:
        return order[a:b + 1]
    return order[a:] + order[:b + 1]


def _stat(x, idx):
    W = len(x)
    xbar = math.fsum(x) / W
    R = len(idx)
    S = math.fsum(x[i] - xbar for i in idx)
    return S * S / (R * (W - R))


def _curve(seed, n, binary=True):
    rng = np.random.default_rng(seed)
    if binary:   # times on a 2^-10 grid: exact phases at power-of-two periods
        t = np.sort(rng.choice(np.arange(0, 8 * 1024), n, replace=False)) / 1024.0
    else:
        t = np.sort(rng.uniform(0, 8, n))
    x = rng.normal(0, 1, n)
    return t, x


@pytest.mark.parametrize("seed", range(8))
def test_matches_unbinned_brute_force(seed):
    t, x = _curve(seed, 9, binary=False)
    rng = np.random.default_rng(50 + seed)
    w = rng.uniform(0.5, 2.0, t.size) if seed % 2 else None
    P = float(rng.uniform(0.3, 3.0))
    o = oracle.unbinned(t, x, w, [P], 1e-9, 1 - 1e-9)
    bv, bset = unbinned_best(t, x, w, P)
    assert abs(o["sr"][0] ** 2 - bv) <= 1e-12 * bv


@pytest.mark.parametrize("seed,qmin,qmax", [(1, 0.05, 0.2), (2, 0.1, 0.15),
                                            (3, 0.01, 0.5), (4, 0.2, 0.21),
                                            (5, 0.3, 0.6), (6, 0.02, 0.04)])
def test_matches_direct_box_search(seed, qmin, qmax):
    t, x = _curve(seed, 11, binary=False)
    rng = np.random.default_rng(70 + seed)
    for P in rng.uniform(0.2, 4.0, 4):
        o = oracle.unbinned(t, x, None, [P], qmin, qmax)
        bv, bset = box_search(list(t), list(x), None, P, qmin, qmax)
        assert abs(o["sr"][0] ** 2 - bv) <= 1e-12 * max(bv, 1e-300), (P, qmin)
        if bv > 0:
            # the reported run reaches the maximum (a set and its complement
            # tie for unit weights, so the run itself is what is checked)
            run = _run_set(t, P, o["first"][0], o["last"][0])
            assert abs(_stat(x, run) - bv) <= 1e-12 * bv


def test_noiseless_box_closed_form():
    # 400 points uniform in phase at P = 1; x = -delta inside [0.3, 0.38)
    n, delta = 400, 0.125
    t = (np.arange(n) + 0.5) / n + 7.0
    t = np.concatenate([[7.0], t])          # t0 = 7, phase = t - 7
    ph = t - 7.0
    x = np.where((ph >= 0.3) & (ph < 0.38), -delta, 0.0)
    o = oracle.unbinned(t, x, None, [1.0], 0.05, 0.1)
    W = t.size
    R = int(np.sum(x < 0))
    assert abs(o["sr"][0] - delta * math.sqrt(R * (W - R)) / W) < 1e-12
    assert abs(o["depth"][0] - delta) < 1e-12
    inbox = np.flatnonzero(x < 0)
    assert o["first"][0] == inbox[0] and o["last"][0] == inbox[-1]


@pytest.mark.parametrize("seed", range(4))
def test_binned_boxes_never_beat_unbinned(seed):
    rng = np.random.default_rng(90 + seed)
    t = np.sort(rng.uniform(0, 30, 300))
    x = rng.normal(0, 1, 300)
    per = np.exp(rng.uniform(np.log(0.3), np.log(5), 40))
    nb = int(rng.choice([20, 50, 100]))
    b = oracle.search(t, x, None, per, nb, 0.05, 0.2)
    qlo = b.kmin / nb * (1 - 1e-9)
    qhi = b.kmax / nb * (1 + 1e-9)
    u = oracle.unbinned(t, x, None, per, qlo, qhi)
    assert np.all(u["sr"] >= b.sr * (1 - 1e-12))


def test_invariances_and_options():
    t, x = _curve(12, 60, binary=False)
    rng = np.random.default_rng(13)
    w = rng.uniform(0.5, 2, t.size)
    per = np.exp(np.linspace(np.log(0.4), np.log(3), 25))
    base = oracle.unbinned(t, x, w, per, 0.03, 0.2)
    sh = oracle.unbinned(t, x + 123.0, w, per, 0.03, 0.2)
    assert np.allclose(sh["sr"], base["sr"], rtol=1e-9, atol=0)
    sc = oracle.unbinned(t, x, 8.0 * w, per, 0.03, 0.2)
    assert np.allclose(sc["sr"], base["sr"], rtol=1e-12, atol=0)
    perm = rng.permutation(t.size)
    pm = oracle.unbinned(t[perm], x[perm], w[perm], per, 0.03, 0.2)
    assert np.allclose(pm["sr"], base["sr"], rtol=1e-12, atol=0)
    assert np.array_equal(perm[pm["first"]], base["first"])
    neg = oracle.unbinned(t, -x, w, per, 0.03, 0.2)
    assert np.allclose(neg["sr"], base["sr"], rtol=1e-12, atol=0)
    dip = oracle.unbinned(t, x, w, per, 0.03, 0.2, dip_only=True)
    assert np.all(dip["sr"] <= base["sr"] * (1 + 1e-15))
    assert np.all(np.nan_to_num(dip["depth"], nan=1.0) > 0)
    # zero-weight points are dropped; indices still refer to the input
    w0 = w.copy()
    w0[::5] = 0.0
    z = oracle.unbinned(t, x, w0, per, 0.03, 0.2)
    keep = np.flatnonzero(w0 > 0)
    zz = oracle.unbinned(t[keep], x[keep], w[keep], per, 0.03, 0.2)
    assert np.array_equal(z["sr"], zz["sr"])
    assert np.array_equal(z["first"], keep[zz["first"]])
    mp = oracle.unbinned(t, x, w, per, 0.03, 0.2, min_in_points=6)
    assert np.all(mp["sr"] <= base["sr"] * (1 + 1e-15))


def test_ties_and_degenerate_cases():
    # all points at one phase: no box separates them
    t = np.full(10, 3.0)
    o = oracle.unbinned(t, np.arange(10.0), None, [1.0], 0.01, 0.5)
    assert o["sr"][0] == 0 and o["first"][0] == -1 and np.isnan(o["depth"][0])
    # two groups of equal phases: only whole groups can be taken
    t = np.array([0.0, 0.0, 0.0, 0.5, 0.5, 0.5]) + 10.0
    x = np.array([1.0, 1.0, 1.0, -1.0, -1.0, -1.0])
    o = oracle.unbinned(t, x, None, [1.0], 0.01, 0.3)
    assert abs(o["sr"][0] - 1.0) < 1e-15        # S^2/(R(W-R)) = 9/9
    assert o["first"][0] == 0 and o["last"][0] == 2
    with pytest.raises(oracle.OracleError):
        oracle.unbinned(t, x, None, [1.0], 0.0, 0.3)
