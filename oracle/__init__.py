"""FP64 CPU oracle for the binned BLS periodogram -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports it and it
never imports the GPU library; the two share no code.

The arithmetic lives in ``bls_oracle.c`` (plain C, FP64, no fast math), which
states the method (Law et al. 2011, section 2.2.2, and the box-least-squares
statistic it cites) and every reading of it.  This module only builds that
file with gcc and marshals numpy arrays into it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bls_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_bls.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FP contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


class _Prep(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("t0", ctypes.c_double),
                ("W", ctypes.c_double), ("xbar", ctypes.c_double),
                ("sumwy2", ctypes.c_double), ("kmin", ctypes.c_int32),
                ("kmax", ctypes.c_int32)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build(force=True)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.bls_oracle_search.argtypes = [
        P, P, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32,
        ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
        ctypes.c_int32, P, P, P, P, P, P]
    lib.bls_oracle_search.restype = ctypes.c_int
    lib.bls_oracle_bins.argtypes = [
        P, P, P, ctypes.c_int64, ctypes.c_double, ctypes.c_int32, P, P, P, P]
    lib.bls_oracle_bins.restype = ctypes.c_int64
    lib.bls_oracle_detect.argtypes = [
        P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double,
        ctypes.c_double, P, P, P, P, P, P, P, P]
    lib.bls_oracle_detect.restype = ctypes.c_int
    lib.bls_oracle_eclipse_window.argtypes = [
        P, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32,
        ctypes.c_double, ctypes.c_int32, ctypes.c_int32, P]
    lib.bls_oracle_eclipse_window.restype = ctypes.c_int
    lib.bls_oracle_variability.argtypes = [
        P, P, P, ctypes.c_int64, P, P, ctypes.c_int64, ctypes.c_double,
        ctypes.c_double, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
        ctypes.c_double, ctypes.c_int32, P, P, P, P, P, P]
    lib.bls_oracle_variability.restype = ctypes.c_int
    lib.bls_oracle_unbinned.argtypes = [
        P, P, P, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_double,
        ctypes.c_double, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
        P, P, P, P, P]
    lib.bls_oracle_unbinned.restype = ctypes.c_int
    lib.bls_oracle_inject.argtypes = [
        P, P, ctypes.c_int64, P, ctypes.c_int32, P, P, P, P, P]
    lib.bls_oracle_inject.restype = ctypes.c_int
    lib.bls_oracle_recovered.argtypes = [ctypes.c_double] * 5
    lib.bls_oracle_recovered.restype = ctypes.c_int
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(ValueError):
    pass


@dataclass
class OracleResult:
    sr: np.ndarray         # [nperiods] float64
    depth: np.ndarray      # [nperiods] float64 (NaN where no box)
    jstart: np.ndarray     # [nperiods] int32 (-1 where no box)
    kwidth: np.ndarray     # [nperiods] int32 (-1 where no box)
    best_index: int
    n: int
    t0: float
    W: float
    xbar: float
    sumwy2: float
    kmin: int
    kmax: int

    def phase(self, nbins: int) -> np.ndarray:
        out = self.jstart / float(nbins)
        return np.where(self.jstart < 0, np.nan, out)

    def duration(self, periods, nbins: int) -> np.ndarray:
        out = self.kwidth * np.asarray(periods, np.float64) / float(nbins)
        return np.where(self.kwidth < 0, np.nan, out)


def search(t, x, w, periods, nbins, qmin, qmax, *, min_in_points=1,
           dip_only=False, nthreads=0) -> OracleResult:
    """Periodogram of one light curve (see bls_oracle.c for the definition)."""
    lib = _load()
    t = _f64(t)
    x = _f64(x)
    w = None if w is None else _f64(w)
    periods = _f64(periods)
    n = t.shape[0]
    if x.shape[0] != n or (w is not None and w.shape[0] != n):
        raise OracleError("length mismatch")
    m = periods.shape[0]
    sr = np.empty(m, np.float64)
    depth = np.empty(m, np.float64)
    js = np.empty(m, np.int32)
    ks = np.empty(m, np.int32)
    best = ctypes.c_int64(-1)
    prep = _Prep()
    st = lib.bls_oracle_search(
        _ptr(t), _ptr(x), _ptr(w), n, _ptr(periods), m, int(nbins),
        float(qmin), float(qmax), int(min_in_points), int(bool(dip_only)),
        int(nthreads), _ptr(sr), _ptr(depth), _ptr(js), _ptr(ks),
        ctypes.byref(best), ctypes.byref(prep))
    if st != 0:
        raise OracleError("oracle rejected the input (status %d)" % st)
    return OracleResult(sr, depth, js, ks, int(best.value), int(prep.n),
                        prep.t0, prep.W, prep.xbar, prep.sumwy2,
                        int(prep.kmin), int(prep.kmax))


def bins(t, x, w, period, nbins):
    """Bin index of every kept point, and the per-bin sums, at one period.

    Returns (bins[int32, n_kept], hw[nbins], hs[nbins], hn[int64, nbins]).
    """
    lib = _load()
    t = _f64(t)
    x = _f64(x)
    w = None if w is None else _f64(w)
    n = t.shape[0]
    b = np.empty(n, np.int32)
    hw = np.empty(nbins, np.float64)
    hs = np.empty(nbins, np.float64)
    hn = np.empty(nbins, np.int64)
    m = lib.bls_oracle_bins(_ptr(t), _ptr(x), _ptr(w), n, float(period),
                            int(nbins), _ptr(b), _ptr(hw), _ptr(hs), _ptr(hn))
    if m < 0:
        raise OracleError("oracle rejected the input (status %d)" % m)
    return b[:m], hw, hs, hn


def detect(sr, periods, max_peaks=8, window=0.01, threshold=7.0):
    """Detection statistics of one periodogram (see bls_oracle.h)."""
    lib = _load()
    sr = _f64(sr)
    periods = _f64(periods)
    m = sr.shape[0]
    mean, std, sde = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    pi = np.full(max(max_peaks, 1), -1, np.int64)
    ps = np.zeros(max(max_peaks, 1))
    pd = np.zeros(max(max_peaks, 1))
    npk, cand = ctypes.c_int32(), ctypes.c_int32()
    st = lib.bls_oracle_detect(_ptr(sr), _ptr(periods), m, int(max_peaks),
                               float(window), float(threshold),
                               ctypes.byref(mean), ctypes.byref(std),
                               ctypes.byref(sde), _ptr(pi), _ptr(ps),
                               _ptr(pd), ctypes.byref(npk),
                               ctypes.byref(cand))
    if st != 0:
        raise OracleError("oracle rejected the input (status %d)" % st)
    k = npk.value
    return dict(mean=mean.value, std=std.value, sde=sde.value,
                peak_index=pi[:k], peak_sr=ps[:k], peak_sde=pd[:k],
                candidate=bool(cand.value))


def eclipse_window(t, w, periods, nphase, duration, min_eclipses=2,
                   nthreads=0):
    """Observed-epoch counts of the eclipse detection efficiency.

    Returns int32 [nperiods]: for each period, how many of the nphase trial
    eclipse epochs give at least min_eclipses distinct eclipses that fall on
    kept observations (readings W1-W4 in bls_oracle.c); divide by nphase for
    the efficiency.
    """
    lib = _load()
    t = _f64(t)
    w = None if w is None else _f64(w)
    periods = _f64(periods)
    if w is not None and w.shape[0] != t.shape[0]:
        raise OracleError("length mismatch")
    out = np.empty(periods.shape[0], np.int32)
    st = lib.bls_oracle_eclipse_window(
        _ptr(t), _ptr(w), t.shape[0], _ptr(periods), periods.shape[0],
        int(nphase), float(duration), int(min_eclipses), int(nthreads),
        _ptr(out))
    if st != 0:
        raise OracleError("oracle rejected the input (status %d)" % st)
    return out


def variability(x, w, n_off, mag, chip_off, nmagbins, origin=0.0, width=0.1,
                clip_sigma=3.0, max_iter=5, flag_sigma=2.0, min_stars=3):
    """High-variability pre-search (readings V1-V4 in bls_oracle.c).

    Returns a dict: rms, bin, flag per star; mean, std, count per
    (chip, magnitude bin), shaped [nchips, nmagbins].
    """
    lib = _load()
    x = _f64(x)
    w = None if w is None else _f64(w)
    n_off = np.ascontiguousarray(n_off, np.int64)
    chip_off = np.ascontiguousarray(chip_off, np.int64)
    mag = _f64(mag)
    nc = n_off.shape[0] - 1
    nk = chip_off.shape[0] - 1
    if mag.shape[0] != nc or n_off[-1] != x.shape[0]:
        raise OracleError("length mismatch")
    rms = np.empty(nc)
    b = np.empty(nc, np.int32)
    f = np.empty(nc, np.int32)
    bm = np.empty(nk * nmagbins)
    bs = np.empty(nk * nmagbins)
    bc = np.empty(nk * nmagbins, np.int32)
    st = lib.bls_oracle_variability(
        _ptr(x), _ptr(w), _ptr(n_off), nc, _ptr(mag), _ptr(chip_off), nk,
        float(origin), float(width), int(nmagbins), float(clip_sigma),
        int(max_iter), float(flag_sigma), int(min_stars), _ptr(rms), _ptr(b),
        _ptr(f), _ptr(bm), _ptr(bs), _ptr(bc))
    if st != 0:
        raise OracleError("oracle rejected the input (status %d)" % st)
    return dict(rms=rms, bin=b, flag=f, mean=bm.reshape(nk, nmagbins),
                std=bs.reshape(nk, nmagbins), count=bc.reshape(nk, nmagbins))


def unbinned(t, x, w, periods, qmin, qmax, *, min_in_points=1,
             dip_only=False, nthreads=0):
    """Unbinned periodogram of one light curve (readings U1-U3).

    Returns a dict: sr, depth [nperiods] float64; first, last [nperiods]
    int32 input indices of the best box's first and last points in phase
    order (-1 where no box); best_index.
    """
    lib = _load()
    t = _f64(t)
    x = _f64(x)
    w = None if w is None else _f64(w)
    periods = _f64(periods)
    n, m = t.shape[0], periods.shape[0]
    sr = np.empty(m)
    depth = np.empty(m)
    first = np.empty(m, np.int32)
    last = np.empty(m, np.int32)
    best = ctypes.c_int64(-1)
    st = lib.bls_oracle_unbinned(
        _ptr(t), _ptr(x), _ptr(w), n, _ptr(periods), m, float(qmin),
        float(qmax), int(min_in_points), int(bool(dip_only)), int(nthreads),
        _ptr(sr), _ptr(depth), _ptr(first), _ptr(last), ctypes.byref(best))
    if st != 0:
        raise OracleError("oracle rejected the input (status %d)" % st)
    return dict(sr=sr, depth=depth, first=first, last=last,
                best_index=int(best.value))


def inject(t, w, base, period, phase, q, depth) -> np.ndarray:
    """Box eclipses injected into copies of one cadence (readings I1-I3 of
    bls_oracle.c); base: [ninj, n] fluxes before injection.  Returns the
    injected fluxes [ninj, n]."""
    lib = _load()
    t = _f64(t)
    w = None if w is None else _f64(w)
    n = t.shape[0]
    base = _f64(base).reshape(-1, n)
    ninj = base.shape[0]
    prm = [_f64(np.broadcast_to(v, (ninj,))) for v in (period, phase, q, depth)]
    out = np.empty((ninj, n), np.float64)
    st = lib.bls_oracle_inject(_ptr(t), _ptr(w), n, _ptr(base), ninj,
                               *[_ptr(v) for v in prm], _ptr(out))
    if st != 0:
        raise OracleError("oracle rejected the input (status %d)" % st)
    return out


def recovered(best_period, sde, p_inj, sde_threshold, ptol) -> bool:
    """Recovery rule I4 of bls_oracle.c."""
    return bool(_load().bls_oracle_recovered(
        float(best_period), float(sde), float(p_inj), float(sde_threshold),
        float(ptol)))


def recovery(t, w, base, period, phase, q, depth, periods, nbins, qmin, qmax,
             *, window=0.01, sde_threshold=7.0, ptol=0.01, nthreads=0,
             which=None):
    """Injection-recovery of one cadence: inject, search each copy over the
    trial grid, take its detection statistics, apply rule I4.

    which: indices of the injections to run (all by default).  Returns a dict
    of arrays over those injections: recovered (int), best_index, sde, and
    the oracle results (list of OracleResult) and injected fluxes."""
    x = inject(t, w, base, period, phase, q, depth)
    ninj = x.shape[0]
    idx = np.arange(ninj) if which is None else np.asarray(which)
    pr = _f64(np.broadcast_to(period, (ninj,)))
    periods = _f64(periods)
    rec, best, sdes, res = [], [], [], []
    for i in idx:
        o = search(t, x[i], w, periods, nbins, qmin, qmax, nthreads=nthreads)
        d = detect(o.sr, periods, max_peaks=1, window=window,
                   threshold=sde_threshold)
        rec.append(int(recovered(periods[o.best_index], d["sde"], pr[i],
                                 sde_threshold, ptol)))
        best.append(o.best_index)
        sdes.append(d["sde"])
        res.append(o)
    return dict(recovered=np.array(rec, np.int32),
                best_index=np.array(best, np.int64), sde=np.array(sdes),
                results=res, flux=x[idx])
