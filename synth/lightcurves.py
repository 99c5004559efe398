"""Seeded synthetic light curves shaped like the PTF/M-dwarfs survey data.

The survey data (Law et al. 2011, section 2.1 and Table 1: 15-25 min
cadence, about 5 h per night, 1-3 month runs, 140-300 epochs, millimag to
10% precision, HJD times) is not available, so these generators stand in for
it.  Every array is drawn from numpy ``Generator(PCG64)`` streams seeded from
a fixed base seed, one child ``SeedSequence`` per curve, so any curve can be
regenerated alone.

Workload recipes (sizes per the benchmark configurations):

* plain:    1 curve, N = 1000, nightly 8-h windows over 60 nights, sigma 0.01,
            one box P = 1.7 d, depth 0.02, duty cycle 0.03; 5000 log-spaced
            periods 0.2-10 d; 200 bins; q in [0.01, 0.10].
* uniform:  4096 curves x N = 2000, sigma ~ U(0.005, 0.02), 20% with a box
            (depth U(0.005, 0.05), P log-U(0.3, 5), q U(0.01, 0.05)), unit
            weights; 20000 shared log periods 0.2-10 d; 300 bins.
* uneven:   10000 curves, N log-U[200, 10000], U{5000..40000} periods each in
            0.2-10 d, U{200..500} bins, weights 1/sigma_i^2 with
            sigma_i = sigma * U(0.8, 1.2).
* long:     256 curves x N = 50000 on a 1-minute grid over 120 nights,
            sigma 0.003, every curve with a box (q U(0.005, 0.05), depth
            log-U(0.002, 0.02), P log-U(0.1, 20)); 100000 shared periods
            0.1-20 d; 1000 bins; q in [0.005, 0.05].
* cadence:  observing runs of single fields (eclipse detection efficiency):
            U{30..90} nights, each lost to weather with probability 0.3; on a
            clear night a 4.5-h window opening 0.1-0.15 d after the night's
            integer HJD holds exposures every U(15, 25) min; 64 fields share
            100000 log periods 0.1-10 d, 1000 trial epochs, eclipses 0.02 d.
* field:    one pointing's stars for the variability pre-search: 100000
            stars on 11 chips, R magnitudes U(14, 20), U{140..300} epochs,
            noise sqrt(0.003^2 + (0.01 * 10^(0.4 (m - 17)))^2) mag, 3% of
            stars variable (sinusoid, amplitude U(0.02, 0.3) mag, period
            log-U(0.1, 10) d); values are magnitudes.
* serving:  Poisson arrivals; each request N log-U[500, 20000], U{5000..100000}
            periods in 0.2-10 d, U{200..1000} bins, q in [0.01, 0.10], 20%
            with a box.

This module draws inputs only; it holds none of the search's arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Iterator, List, Optional

import numpy as np

T_START = 2455000.5          # HJD-scale epoch, like the survey's times
_BASE_SEED = 17010           # base seed i of configuration i is 17010 + i


@dataclass
class LightCurve:
    t: np.ndarray                    # [n] float64 times (days)
    x: np.ndarray                    # [n] float64 fluxes (normalised to ~1)
    w: Optional[np.ndarray]          # [n] float64 weights, or None (unit)
    periods: np.ndarray              # [m] float64 trial periods (days)
    nbins: int
    qmin: float
    qmax: float
    truth: dict = field(default_factory=dict)   # injected box, if any

    @property
    def n(self) -> int:
        return int(self.t.shape[0])


@dataclass
class Batch:
    """Curves packed end to end (CSR offsets)."""
    t: np.ndarray                    # [sum n] float64
    x: np.ndarray                    # [sum n] float64
    w: Optional[np.ndarray]          # [sum n] float64 or None
    n_off: np.ndarray                # [ncurves + 1] int64
    periods: np.ndarray              # shared grid [m], or packed [sum m]
    p_off: Optional[np.ndarray]      # [ncurves + 1] int64, None = shared grid
    nbins: np.ndarray                # [ncurves] int32
    qmin: np.ndarray                 # [ncurves] float64
    qmax: np.ndarray                 # [ncurves] float64
    truth: List[dict] = field(default_factory=list)

    @property
    def ncurves(self) -> int:
        return int(self.n_off.shape[0] - 1)

    def nperiods(self, c: int) -> int:
        if self.p_off is None:
            return int(self.periods.shape[0])
        return int(self.p_off[c + 1] - self.p_off[c])

    def curve(self, c: int) -> LightCurve:
        a, b = int(self.n_off[c]), int(self.n_off[c + 1])
        if self.p_off is None:
            per = self.periods
        else:
            per = self.periods[int(self.p_off[c]):int(self.p_off[c + 1])]
        return LightCurve(self.t[a:b], self.x[a:b],
                          None if self.w is None else self.w[a:b], per,
                          int(self.nbins[c]), float(self.qmin[c]),
                          float(self.qmax[c]),
                          self.truth[c] if self.truth else {})

    def total_points(self) -> int:
        return int(self.n_off[-1])

    def trial_points(self) -> int:
        """Sum over curves of N_c * nperiods_c."""
        n = np.diff(self.n_off).astype(np.float64)
        if self.p_off is None:
            return int(np.sum(n) * self.periods.shape[0])
        return int(np.sum(n * np.diff(self.p_off)))


def log_period_grid(pmin: float, pmax: float, m: int) -> np.ndarray:
    """m log-spaced periods: P_i = pmin * exp(i ln(pmax/pmin) / (m - 1))."""
    if m == 1:
        return np.array([pmin], np.float64)
    i = np.arange(m, dtype=np.float64)
    return pmin * np.exp(i * (np.log(pmax / pmin) / (m - 1)))


def nightly_times(rng: np.random.Generator, n: int, nights: int = 60,
                  window_h: float = 8.0, t_start: float = T_START) -> np.ndarray:
    """n sorted epochs inside nightly windows: t = t_start + d + 0.1 + U(0, h)."""
    d = rng.integers(0, nights, size=n).astype(np.float64)
    u = rng.uniform(0.0, window_h / 24.0, size=n)
    return np.sort(t_start + d + 0.1 + u)


def minute_grid_times(n: int, nights: int = 120, per_night: int = 417,
                      t_start: float = T_START) -> np.ndarray:
    """Regular 1-minute cadence, per_night samples from 0.1 d each night."""
    d = np.repeat(np.arange(nights, dtype=np.float64), per_night)
    s = np.tile(np.arange(per_night, dtype=np.float64), nights)
    t = t_start + d + 0.1 + s / 1440.0
    if n > t.shape[0]:
        raise ValueError("grid holds only %d epochs" % t.shape[0])
    return t[:n].copy()


def inject_box(t: np.ndarray, period: float, q: float, phi0: float,
               depth: float, t_start: float = T_START) -> np.ndarray:
    """Flux drop of a continuous periodic box (duty cycle q, start phase phi0)."""
    ph = np.mod((t - t_start) / period - phi0, 1.0)
    return np.where(ph < q, -depth, 0.0)


def _curve(rng, n, sigma, times, inj_prob, depth_rng, period_rng, q_rng,
           log_depth=False, weighted=False):
    t = times
    noise_sigma = np.full(n, sigma)
    if weighted:
        noise_sigma = sigma * rng.uniform(0.8, 1.2, size=n)
    x = 1.0 + noise_sigma * rng.standard_normal(n)
    truth = {}
    if rng.uniform() < inj_prob:
        if log_depth:
            depth = float(np.exp(rng.uniform(np.log(depth_rng[0]),
                                             np.log(depth_rng[1]))))
        else:
            depth = float(rng.uniform(*depth_rng))
        per = float(np.exp(rng.uniform(np.log(period_rng[0]),
                                       np.log(period_rng[1]))))
        q = float(rng.uniform(*q_rng))
        phi0 = float(rng.uniform())
        x = x + inject_box(t, per, q, phi0, depth)
        truth = dict(period=per, depth=depth, q=q, phi0=phi0)
    w = 1.0 / noise_sigma ** 2 if weighted else None
    return t, x, w, truth


def config1(seed: int = _BASE_SEED + 1) -> LightCurve:
    """Plain single curve: N = 1000, one box at P = 1.7 d."""
    rng = np.random.default_rng(seed)
    n = 1000
    t = nightly_times(rng, n)
    x = 1.0 + 0.01 * rng.standard_normal(n)
    phi0 = float(rng.uniform())
    x = x + inject_box(t, 1.7, 0.03, phi0, 0.02)
    return LightCurve(t, x, None, log_period_grid(0.2, 10.0, 5000), 200,
                      0.01, 0.10,
                      dict(period=1.7, depth=0.02, q=0.03, phi0=phi0))


def uniform_batch(ncurves: int, n: int, nperiods: int, nbins: int,
                  seed: int, pmin: float = 0.2, pmax: float = 10.0,
                  qmin: float = 0.01, qmax: float = 0.10,
                  inj_prob: float = 0.2) -> Batch:
    """Equal-length curves on nightly windows sharing one period grid."""
    children = np.random.SeedSequence(seed).spawn(ncurves)
    ts, xs, truth = [], [], []
    for c in range(ncurves):
        rng = np.random.default_rng(children[c])
        sigma = float(rng.uniform(0.005, 0.02))
        t = nightly_times(rng, n)
        t, x, _, tr = _curve(rng, n, sigma, t, inj_prob, (0.005, 0.05),
                             (0.3, 5.0), (0.01, 0.05))
        ts.append(t)
        xs.append(x)
        truth.append(tr)
    n_off = np.arange(ncurves + 1, dtype=np.int64) * n
    return Batch(np.concatenate(ts), np.concatenate(xs), None, n_off,
                 log_period_grid(pmin, pmax, nperiods), None,
                 np.full(ncurves, nbins, np.int32),
                 np.full(ncurves, qmin), np.full(ncurves, qmax), truth)


def config2(ncurves: int = 4096) -> Batch:
    """Uniform batch: 4096 x N = 2000, 20000 shared periods, 300 bins."""
    return uniform_batch(ncurves, 2000, 20000, 300, _BASE_SEED + 2)


def uneven_batch(ncurves: int, seed: int, n_range=(200, 10000),
                 np_range=(5000, 40000), nbins_range=(200, 500),
                 weighted: bool = True, pmin: float = 0.2, pmax: float = 10.0,
                 qmin: float = 0.01, qmax: float = 0.10,
                 inj_prob: float = 0.2) -> Batch:
    """Curves of log-uniform length, each with its own period grid and bins."""
    children = np.random.SeedSequence(seed).spawn(ncurves)
    ts, xs, ws, ps, truth = [], [], [], [], []
    ns = np.empty(ncurves, np.int64)
    nps = np.empty(ncurves, np.int64)
    nb = np.empty(ncurves, np.int32)
    for c in range(ncurves):
        rng = np.random.default_rng(children[c])
        n = int(round(np.exp(rng.uniform(np.log(n_range[0]),
                                         np.log(n_range[1])))))
        m = int(rng.integers(np_range[0], np_range[1] + 1))
        nb[c] = int(rng.integers(nbins_range[0], nbins_range[1] + 1))
        sigma = float(rng.uniform(0.005, 0.02))
        t = nightly_times(rng, n)
        t, x, w, tr = _curve(rng, n, sigma, t, inj_prob, (0.005, 0.05),
                             (0.3, 5.0), (0.01, 0.05), weighted=weighted)
        ts.append(t)
        xs.append(x)
        if weighted:
            ws.append(w)
        ps.append(log_period_grid(pmin, pmax, m))
        truth.append(tr)
        ns[c] = n
        nps[c] = m
    n_off = np.concatenate([[0], np.cumsum(ns)]).astype(np.int64)
    p_off = np.concatenate([[0], np.cumsum(nps)]).astype(np.int64)
    return Batch(np.concatenate(ts), np.concatenate(xs),
                 np.concatenate(ws) if weighted else None, n_off,
                 np.concatenate(ps), p_off, nb, np.full(ncurves, qmin),
                 np.full(ncurves, qmax), truth)


def config3(ncurves: int = 10000) -> Batch:
    """Uneven weighted batch: 10000 curves, N log-U[200, 10000]."""
    return uneven_batch(ncurves, _BASE_SEED + 3)


def config4(ncurves: int = 256, n: int = 50000, nperiods: int = 100000,
            nbins: int = 1000) -> Batch:
    """High-cadence long baseline: 1-minute grid over 120 nights."""
    children = np.random.SeedSequence(_BASE_SEED + 4).spawn(ncurves)
    t = minute_grid_times(n)
    ts, xs, truth = [], [], []
    for c in range(ncurves):
        rng = np.random.default_rng(children[c])
        _, x, _, tr = _curve(rng, n, 0.003, t, 1.0, (0.002, 0.02),
                             (0.1, 20.0), (0.005, 0.05), log_depth=True)
        ts.append(t)
        xs.append(x)
        truth.append(tr)
    n_off = np.arange(ncurves + 1, dtype=np.int64) * n
    return Batch(np.concatenate(ts), np.concatenate(xs), None, n_off,
                 log_period_grid(0.1, 20.0, nperiods), None,
                 np.full(ncurves, nbins, np.int32), np.full(ncurves, 0.005),
                 np.full(ncurves, 0.05), truth)


def serving_requests(nreq: int, rate: float, seed: int = _BASE_SEED + 5,
                     n_range=(500, 20000), np_range=(5000, 100000),
                     nbins_range=(200, 1000)) -> Iterator[tuple]:
    """Yield (arrival_time_s, LightCurve) with exponential inter-arrivals."""
    ss = np.random.SeedSequence(seed)
    arr_rng = np.random.default_rng(ss.spawn(1)[0])
    children = ss.spawn(nreq)
    t_arr = 0.0
    for r in range(nreq):
        t_arr += float(arr_rng.exponential(1.0 / rate))
        rng = np.random.default_rng(children[r])
        n = int(round(np.exp(rng.uniform(np.log(n_range[0]),
                                         np.log(n_range[1])))))
        m = int(rng.integers(np_range[0], np_range[1] + 1))
        nb = int(rng.integers(nbins_range[0], nbins_range[1] + 1))
        sigma = float(rng.uniform(0.005, 0.02))
        t = nightly_times(rng, n)
        t, x, _, tr = _curve(rng, n, sigma, t, 0.2, (0.005, 0.05),
                             (0.3, 5.0), (0.01, 0.05))
        yield t_arr, LightCurve(t, x, None, log_period_grid(0.2, 10.0, m),
                                nb, 0.01, 0.10, tr)


def small_curve(seed: int, n: int, nperiods: int = 64, nbins: int = 64,
                qmin: float = 0.02, qmax: float = 0.2, weighted: bool = False,
                pmin: float = 0.3, pmax: float = 5.0, nights: int = 30,
                inject: bool = True) -> LightCurve:
    """A small curve for tests: nightly cadence, optional box and weights."""
    rng = np.random.default_rng(seed)
    t = nightly_times(rng, n, nights=nights)
    t, x, w, tr = _curve(rng, n, 0.01, t, 1.0 if inject else 0.0,
                         (0.01, 0.05), (pmin, pmax), (0.02, 0.08),
                         weighted=weighted)
    return LightCurve(t, x, w, log_period_grid(pmin, pmax, nperiods), nbins,
                      qmin, qmax, tr)


def survey_cadence(rng: np.random.Generator, nights: int = 60,
                   weather: float = 0.3, hours: float = 4.5,
                   cadence_min=(15.0, 25.0),
                   t_start: float = T_START) -> np.ndarray:
    """Exposure times of one field's run (Table 1 cadence, weather losses)."""
    out = []
    for d in range(nights):
        if rng.uniform() < weather:
            continue
        t = t_start + d + 0.1 + rng.uniform(0.0, 0.05)
        end = t + hours / 24.0
        while t < end:
            out.append(t)
            t += rng.uniform(*cadence_min) / 1440.0
    if not out:                      # keep at least one exposure
        out.append(t_start + 0.1)
    return np.asarray(out, np.float64)


def cadence_batch(ncadences: int = 64, nperiods: int = 100000,
                  seed: int = _BASE_SEED + 6, pmin: float = 0.1,
                  pmax: float = 10.0) -> Batch:
    """Many fields' cadences on one shared log period grid (times only)."""
    ss = np.random.SeedSequence(seed)
    ts = []
    for child in ss.spawn(ncadences):
        rng = np.random.default_rng(child)
        ts.append(survey_cadence(rng, nights=int(rng.integers(30, 91))))
    n = np.array([t.shape[0] for t in ts], np.int64)
    n_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    t = np.concatenate(ts)
    return Batch(t, np.zeros_like(t), None, n_off,
                 log_period_grid(pmin, pmax, nperiods), None,
                 np.full(ncadences, 2, np.int32), np.full(ncadences, 0.1),
                 np.full(ncadences, 0.1))


def variability_field(nstars: int = 100000, nchips: int = 11,
                      seed: int = _BASE_SEED + 7, var_frac: float = 0.03):
    """Stars of one pointing (magnitudes over time) for the pre-search.

    Returns (Batch of magnitude light curves, mag [nstars], chip_off
    [nchips + 1], variable [nstars] bool).
    """
    rng = np.random.default_rng(seed)
    mag = rng.uniform(14.0, 20.0, nstars)
    n = rng.integers(140, 301, nstars)
    n_off = np.concatenate([[0], np.cumsum(n)]).astype(np.int64)
    sig = np.sqrt(0.003 ** 2 + (0.01 * 10 ** (0.4 * (mag - 17.0))) ** 2)
    var = rng.uniform(size=nstars) < var_frac
    t = T_START + rng.uniform(0.0, 90.0, n_off[-1])
    star = np.repeat(np.arange(nstars), n)
    x = mag[star] + sig[star] * rng.standard_normal(n_off[-1])
    amp = rng.uniform(0.02, 0.3, nstars) * var
    per = np.exp(rng.uniform(np.log(0.1), np.log(10.0), nstars))
    x = x + amp[star] * np.sin(2 * np.pi * t / per[star])
    chip_off = np.linspace(0, nstars, nchips + 1).round().astype(np.int64)
    b = Batch(t, x, None, n_off, np.array([1.0]), None,
              np.full(nstars, 2, np.int32), np.full(nstars, 0.1),
              np.full(nstars, 0.1))
    return b, mag, chip_off, var


def detection_periodograms(seed: int = _BASE_SEED + 9):
    """Crafted periodograms for the detection step: a list of (SR, periods,
    max_peaks, window).  Strides of 256 match the slices one workgroup's
    threads take, so the cases reach the corners of a parallel peak search:
    the largest values crowded into one slice, suppression across slices,
    ties, an early stop, fewer periods than threads."""
    rng = np.random.default_rng(seed)
    cases = []
    # The 24 largest values all in one 256-stride slice (indices 3 mod 256):
    # more than a thread keeps of its slice at once, so 16 peaks make it
    # look again (its buckets are rescanned).
    m = 256 * 30 + 17
    sr = rng.uniform(0.0, 1.0, m)
    sr[3 + 256 * np.arange(24)] = 2.0 + rng.uniform(0.0, 1.0, 24)
    cases.append((sr, np.geomspace(1.0, 40.0, m), 16, 1e-6))
    # Same slice, but its peaks are wiped out by harmonics of a peak elsewhere:
    # suppression across slices, then rescans.
    per = np.geomspace(0.5, 40.0, m)
    sr = rng.uniform(0.0, 1.0, m)
    top = 5 + 256 * np.arange(20)
    sr[top] = 2.0 + rng.uniform(0.0, 1.0, 20)
    j = int(np.argmin(np.abs(per - 2.0 * per[top[4]])))
    sr[j] = 9.0
    cases.append((sr, per, 16, 0.05))
    # Heavy ties: few distinct values, the smallest index must win each tie.
    m = 256 * 12 + 200
    sr = np.round(rng.uniform(0.0, 1.0, m) * 3.0) / 3.0
    cases.append((sr, np.linspace(1.0, 30.0, m), 16, 0.002))
    # A wide window: every peak suppresses large stretches, every slice
    # empties its list many times.
    sr = rng.gamma(2.0, 1.0, m)
    cases.append((sr, np.linspace(0.3, 30.0, m), 16, 0.3))
    # Few positive values (zeros and negatives otherwise): the search stops
    # early; npeaks < max_peaks.
    sr = np.zeros(m)
    sr[rng.choice(m, 5, replace=False)] = rng.uniform(0.1, 1.0, 5)
    sr[rng.choice(m, 50, replace=False)] = -0.5
    cases.append((sr, np.linspace(1.0, 30.0, m), 16, 0.0))
    # Fewer periods than threads, a single period, a slice of exactly 9.
    for mm in (1, 7, 255, 256 * 9):
        cases.append((rng.uniform(0.0, 1.0, mm), np.linspace(1.0, 9.0, mm),
                      16, 0.01))
    # All SR equal and positive: std 0, sde 0, peaks by index only.
    cases.append((np.full(700, 0.25), np.linspace(1.0, 2.0, 700), 5, 0.0))
    return cases


@dataclass
class InjectionSet:
    """One cadence, its per-injection flux realizations and box eclipses,
    and the trial grid of the search (inputs of the injection-recovery)."""
    t: np.ndarray            # [n] cadence times
    w: Optional[np.ndarray]  # [n] weights or None
    base: np.ndarray         # [ninj, n] fluxes before injection
    period: np.ndarray       # [ninj] injected period (d)
    phase: np.ndarray        # [ninj] start phase in [0, 1)
    q: np.ndarray            # [ninj] duty cycle
    depth: np.ndarray        # [ninj] depth (flux units)
    periods: np.ndarray      # [nperiods] trial grid
    nbins: int
    qmin: float
    qmax: float


def injection_set(ninj: int = 4096, seed: int = _BASE_SEED + 10,
                  nperiods: int = 20000, nbins: int = 300,
                  sigma: float = 0.01, depth_range=(0.003, 0.03),
                  q_range=(0.01, 0.05), period_range=(0.3, 10.0),
                  weighted: bool = False, nights: int = 60) -> InjectionSet:
    """Box eclipses of log-uniform period, random phase, duty cycle and depth
    in copies of one survey cadence, each with its own Gaussian noise."""
    rng = np.random.default_rng(seed)
    t = survey_cadence(rng, nights=nights)
    n = t.shape[0]
    w = None
    if weighted:
        w = 1.0 / (sigma * rng.uniform(0.8, 1.2, n)) ** 2
        w[rng.random(n) < 0.03] = 0.0           # a few rejected exposures
    lo, hi = np.log(period_range[0]), np.log(period_range[1])
    period = np.exp(rng.uniform(lo, hi, ninj))
    phase = rng.uniform(0.0, 1.0, ninj)
    q = rng.uniform(*q_range, ninj)
    depth = rng.uniform(*depth_range, ninj)
    base = 1.0 + sigma * rng.standard_normal((ninj, n))
    return InjectionSet(t, w, base, period, phase, q, depth,
                        log_period_grid(0.2, 10.0, nperiods), nbins, 0.01,
                        0.10)
