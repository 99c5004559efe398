"""Pins of the oracle's eclipse detection efficiency (CPU only).

The oracle folds the cadence and counts, per trial eclipse epoch, the distinct
eclipse events that fall on observations (readings W1-W4 in bls_oracle.c).
These tests pin it without folding: in the time domain, by closed forms of the
daytime alias the paper's detection-efficiency figure describes, and by the
one-period limit on seeing two eclipses.

Exactness: times are multiples of 2^-10, periods powers of two and nphase a
power of two, so d f, its fractional part and phase * nphase are all exact
and the binned epochs coincide with time intervals.
"""
import numpy as np
import pytest

import oracle


def events_in_time(t, P, nphase, k, j):
    """Distinct eclipse events at offset j, counted on the time axis.

    Event e covers [t0 + (e + j/nphase) P, t0 + (e + (j + k)/nphase) P); it is
    observed when some time lies inside.  No folding, no bins.
    """
    ts = np.sort(np.asarray(t, np.float64))
    t0 = ts[0]
    e_lo = int(np.floor((ts[0] - t0) / P)) - 2
    e_hi = int(np.ceil((ts[-1] - t0) / P)) + 2
    seen = 0
    for e in range(e_lo, e_hi + 1):
        a = t0 + (e + j / nphase) * P
        b = t0 + (e + (j + k) / nphase) * P
        i = np.searchsorted(ts, a, side="left")
        if i < ts.size and ts[i] < b:
            seen += 1
    return seen


def brute(t, P, nphase, k, m):
    return sum(events_in_time(t, P, nphase, k, j) >= m for j in range(nphase))


def binary_cadence(rng, nights, per_night, span):
    """Nightly blocks of observations at multiples of 2^-10 day."""
    out = []
    for d in range(nights):
        if rng.random() < 0.25:           # weather: lose the night
            continue
        start = rng.integers(0, 1024 - span)
        s = np.sort(rng.choice(np.arange(start, start + span), per_night,
                               replace=False))
        out.append(d + s / 1024.0)
    return np.concatenate(out)


@pytest.mark.parametrize("seed", range(6))
def test_matches_time_domain_count(seed):
    rng = np.random.default_rng(100 + seed)
    t = binary_cadence(rng, nights=int(rng.integers(3, 12)),
                       per_night=int(rng.integers(3, 20)), span=300)
    nphase = int(rng.choice([16, 32, 64]))
    periods = [0.25, 0.5, 1.0, 2.0, 4.0]
    for P in periods:
        k = int(rng.integers(1, nphase // 3))
        D = k * P / nphase                       # exact: k whole bins
        for m in (1, 2, 3):
            got = oracle.eclipse_window(t, None, [P], nphase, D, m)[0]
            assert got == brute(t, P, nphase, k, m), (P, k, m)


@pytest.mark.parametrize("L,k,nights", [(20, 3, 5), (1, 1, 2), (40, 10, 3),
                                        (60, 5, 7)])
def test_integer_day_alias_closed_form(L, k, nights):
    # P = 1 day: every night shows the same L phase bins, so an epoch shows
    # an eclipse on every night or on none; it does iff its k-bin window
    # meets the L observed bins: L + k - 1 of the 64 epochs.
    nphase = 64
    t = np.concatenate([d + np.arange(7, 7 + L) / 64.0 for d in range(nights)])
    for m in range(1, nights + 1):
        got = oracle.eclipse_window(t, None, [1.0], nphase, k / 64.0, m)[0]
        assert got == L + k - 1, m
    assert oracle.eclipse_window(t, None, [1.0], nphase, k / 64.0,
                                 nights + 1)[0] == 0
    # a duration far below one bin still takes one bin: L epochs
    assert oracle.eclipse_window(t, None, [1.0], nphase, 1e-9, 2)[0] == L


def test_one_cycle_of_dense_coverage():
    # Observations fill exactly one cycle [t0, t0 + P).  An unwrapped window
    # sees one event; a window that wraps past the end of the cycle sees the
    # eclipse at the start of the data and the next one, P later: k - 1 of
    # the epochs show two eclipses, all of them show one.
    nphase, P = 64, 2.0
    t = np.arange(0, 2048) / 1024.0
    for k in (1, 2, 5, 17):
        D = k * P / nphase
        assert oracle.eclipse_window(t, None, [P], nphase, D, 2)[0] == k - 1
        assert oracle.eclipse_window(t, None, [P], nphase, D, 1)[0] == nphase
        assert oracle.eclipse_window(t, None, [P], nphase, D, 3)[0] == 0


def test_baseline_shorter_than_a_period_sees_at_most_one():
    # Two events are P apart; points less than P (1 - (k + 1)/nphase) apart
    # can never show both.
    rng = np.random.default_rng(7)
    nphase, P, k = 64, 4.0, 6
    span = P * (1 - (k + 1) / nphase) * 0.999
    t = np.sort(rng.uniform(0, span, 500))
    assert oracle.eclipse_window(t, None, [P], nphase, k * P / nphase, 2)[0] == 0
    assert oracle.eclipse_window(t, None, [P], nphase, k * P / nphase, 1)[0] > 0


def test_dense_coverage_of_three_cycles_sees_every_epoch():
    nphase = 128
    t = np.arange(0, 3 * 1024 + 1) / 1024.0         # [0, 3] dense
    per = np.array([0.5, 0.75, 1.0])
    for m in (1, 2, 3):
        got = oracle.eclipse_window(t, None, per, nphase, 0.01, m)
        assert got.tolist() == [nphase] * 3, m


def test_shift_and_order_invariance_and_zero_weights():
    rng = np.random.default_rng(11)
    t = binary_cadence(rng, nights=9, per_night=15, span=400)
    per = np.exp(np.linspace(np.log(0.3), np.log(3.0), 200))
    base = oracle.eclipse_window(t, None, per, 100, 0.02, 2)
    assert np.array_equal(
        base, oracle.eclipse_window(t + 1024.0, None, per, 100, 0.02, 2))
    perm = rng.permutation(t.size)
    assert np.array_equal(
        base, oracle.eclipse_window(t[perm], None, per, 100, 0.02, 2))
    # extra points of weight 0 are not observations
    junk = rng.uniform(t.min(), t.max(), 50)
    tt = np.concatenate([t, junk])
    w = np.concatenate([np.ones(t.size), np.zeros(50)])
    assert np.array_equal(
        base, oracle.eclipse_window(tt, w, per, 100, 0.02, 2))
    # more required eclipses never observe more epochs
    m1 = oracle.eclipse_window(t, None, per, 100, 0.02, 1)
    m3 = oracle.eclipse_window(t, None, per, 100, 0.02, 3)
    assert np.all(m1 >= base) and np.all(base >= m3)


def test_long_duration_clamps_to_full_cycle():
    t = np.arange(0, 200) / 64.0
    # duration longer than the period: k = nphase, every point is in eclipse
    got = oracle.eclipse_window(t, None, [0.5], 32, 5.0, 2)[0]
    assert got == 32
    # a tiny duration rounds to one bin
    got1 = oracle.eclipse_window(t, None, [1.0], 64, 1e-9, 2)[0]
    assert got1 == oracle.eclipse_window(t, None, [1.0], 64, 1 / 64.0, 2)[0]


@pytest.mark.parametrize("kw", [dict(nphase=0), dict(duration=0.0),
                                dict(duration=float("nan")),
                                dict(min_eclipses=0), dict(periods=[-1.0])])
def test_invalid_inputs(kw):
    args = dict(t=np.arange(10.0), w=None, periods=[1.0], nphase=16,
                duration=0.1, min_eclipses=2)
    args.update(kw)
    with pytest.raises(oracle.OracleError):
        oracle.eclipse_window(**args)
