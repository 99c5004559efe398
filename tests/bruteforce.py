"""Unbinned brute-force BLS for tiny inputs -- written independently of the oracle.

For one trial period, the points are ordered by phase frac((t - t0)/P) and
every proper cyclic run of consecutive points (1 <= size <= n - 1) is tried as
the in-box set.  Sums use math.fsum (exactly rounded), so this is the
least-squares box statistic S^2 / (R (W - R)) of the box-least-squares method
cited in Law et al. 2011, section 2.2.2, evaluated exhaustively without bins.
A binned search's boxes are a subset of these runs, so its best value can
never exceed this one, and it reaches it when every point has its own bin.
"""
from __future__ import annotations

import math
from typing import Optional, Sequence, Tuple


def unbinned_best(t: Sequence[float], x: Sequence[float],
                  w: Optional[Sequence[float]], period: float,
                  dip_only: bool = False) -> Tuple[float, frozenset]:
    """Largest S^2/(R(W-R)) over cyclic runs in phase order, and its run."""
    if w is None:
        w = [1.0] * len(t)
    pts = [(float(ti), float(xi), float(wi))
           for ti, xi, wi in zip(t, x, w) if wi != 0.0]
    n = len(pts)
    t0 = min(p[0] for p in pts)
    W = math.fsum(p[2] for p in pts)
    xbar = math.fsum(p[2] * p[1] for p in pts) / W
    order = sorted(range(n), key=lambda i: ((pts[i][0] - t0) / period) % 1.0)
    best_v, best_set = 0.0, frozenset()
    for s in range(n):
        for size in range(1, n):
            idx = [order[(s + m) % n] for m in range(size)]
            R = math.fsum(pts[i][2] for i in idx)
            S = math.fsum(pts[i][2] * (pts[i][1] - xbar) for i in idx)
            if dip_only and not S < 0.0:
                continue
            v = S * S / (R * (W - R))
            if v > best_v:
                best_v, best_set = v, frozenset(idx)
    return best_v, best_set
