"""Python face of the C ABI: same names, argument marshalling only."""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import _lib as L


class BlsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (status %d): %s" % (bls_status_string(status),
                                                  status, message))
        self.status = status
        self.message = message


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):          # torch tensor (device memory)
        return C.c_void_p(a.data_ptr())
    return a.ctypes.data_as(C.c_void_p)


def _check(st: int, plan=None):
    if st != L.BLS_OK:
        raise BlsError(st, bls_last_error(plan))


# ------------------------------------------------------------------ basics
def bls_status_string(status: int) -> str:
    return L.load().bls_status_string(int(status)).decode()


def bls_last_error(plan=None) -> str:
    buf = C.create_string_buffer(1024)
    L.load().bls_last_error(plan, buf, 1024)
    return buf.value.decode(errors="replace")


def bls_width_range(nbins: int, qmin: float, qmax: float):
    """(kmin, kmax) of a duty-cycle range, per the library's rule."""
    kmin, kmax = C.c_int32(), C.c_int32()
    _check(L.load().bls_width_range(int(nbins), float(qmin), float(qmax),
                                    C.byref(kmin), C.byref(kmax)))
    return kmin.value, kmax.value


def bls_plan_config_init(**overrides) -> L.BlsPlanConfig:
    cfg = L.BlsPlanConfig()
    L.load().bls_plan_config_init(C.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


def bls_plan_create(cfg: Optional[L.BlsPlanConfig] = None, **overrides):
    if cfg is None:
        cfg = bls_plan_config_init(**overrides)
    plan = C.c_void_p()
    st = L.load().bls_plan_create(C.byref(plan), C.byref(cfg))
    if st != L.BLS_OK:
        raise BlsError(st, bls_last_error(None))
    return plan


def bls_plan_destroy(plan) -> None:
    if plan:
        L.load().bls_plan_destroy(plan)


def bls_synchronize(plan) -> None:
    _check(L.load().bls_synchronize(plan), plan)


def bls_get_stream(plan) -> int:
    s = C.c_void_p()
    _check(L.load().bls_get_stream(plan, C.byref(s)), plan)
    return s.value or 0


def bls_last_stats(plan) -> dict:
    s = L.BlsCallStats()
    _check(L.load().bls_last_stats(plan, C.byref(s)), plan)
    return {f: getattr(s, f) for f, _ in L.BlsCallStats._fields_}


def bls_kernel_times(plan, max_count: int = 64) -> list:
    """Search-kernel durations (ms) of the plan's calls since the last reset,
    oldest first (HIP events around each launch on the plan's stream)."""
    buf = (C.c_float * max(int(max_count), 1))()
    n = C.c_int32(0)
    _check(L.load().bls_kernel_times(plan, buf, int(max_count), C.byref(n)),
           plan)
    return [float(buf[i]) for i in range(n.value)]


def bls_kernel_times_reset(plan) -> None:
    _check(L.load().bls_kernel_times_reset(plan), plan)


def bls_debug_phase_bins(plan, times, period: float, nbins: int):
    """Phase bin the device assigns to each point at one period (diagnostic)."""
    t = _f64(times)
    out = np.empty(t.shape[0], np.int32)
    _check(L.load().bls_debug_phase_bins(plan, _ptr(t), t.shape[0],
                                         float(period), int(nbins),
                                         _ptr(out)), plan)
    return out


# ------------------------------------------------------------------ search
def bls_search(plan, times, flux, weights, periods, nbins, qmin, qmax):
    """One light curve in host memory; returns a dict of numpy arrays."""
    t, x = _f64(times), _f64(flux)
    w = None if weights is None else _f64(weights)
    p = _f64(periods)
    m = p.shape[0]
    out = dict(sr=np.empty(m), phase=np.empty(m), duration=np.empty(m),
               depth=np.empty(m), jstart=np.empty(m, np.int32),
               kwidth=np.empty(m, np.int32))
    best = C.c_int64(-1)
    st = L.load().bls_search(
        plan, _ptr(t), _ptr(x), _ptr(w), t.shape[0], _ptr(p), m, int(nbins),
        float(qmin), float(qmax), _ptr(out["sr"]), _ptr(out["phase"]),
        _ptr(out["duration"]), _ptr(out["depth"]), _ptr(out["jstart"]),
        _ptr(out["kwidth"]), C.byref(best))
    _check(st, plan)
    out["best_index"] = best.value
    return out


@dataclass
class _BatchArgs:
    struct: L.BlsBatch
    keep: list
    nresults: int
    ncurves: int


def _batch(n_off, times, flux, weights, periods, p_off, nbins, qmin, qmax,
           device: bool) -> _BatchArgs:
    keep = []
    b = L.BlsBatch()
    n_off = np.ascontiguousarray(n_off, dtype=np.int64)
    keep.append(n_off)
    nc = n_off.shape[0] - 1
    b.ncurves = nc
    b.n_off = n_off.ctypes.data
    if device:
        arrs = [times, flux, weights, periods]
    else:
        arrs = [_f64(times), _f64(flux),
                None if weights is None else _f64(weights), _f64(periods)]
    keep += arrs
    b.times, b.flux = _ptr(arrs[0]).value, _ptr(arrs[1]).value
    b.weights = None if arrs[2] is None else _ptr(arrs[2]).value
    b.periods = _ptr(arrs[3]).value
    if p_off is None:
        b.p_off = None
        b.nperiods_shared = int(arrs[3].shape[0])
        nres = nc * b.nperiods_shared
    else:
        po = np.ascontiguousarray(p_off, dtype=np.int64)
        keep.append(po)
        b.p_off = po.ctypes.data
        b.nperiods_shared = 0
        nres = int(po[-1])
    if np.ndim(nbins) == 0:
        b.nbins_all, b.nbins = int(nbins), None
    else:
        nb = np.ascontiguousarray(nbins, dtype=np.int32)
        keep.append(nb)
        b.nbins = nb.ctypes.data
    for name in ("qmin", "qmax"):
        v = qmin if name == "qmin" else qmax
        if np.ndim(v) == 0:
            setattr(b, name + "_all", float(v))
            setattr(b, name, None)
        else:
            a = _f64(v)
            keep.append(a)
            setattr(b, name, a.ctypes.data)
    return _BatchArgs(b, keep, nres, nc)


def bls_search_batch(plan, n_off, times, flux, weights, periods, p_off,
                     nbins, qmin, qmax):
    """Many curves in host memory (CSR); returns a dict of numpy arrays."""
    ba = _batch(n_off, times, flux, weights, periods, p_off, nbins, qmin,
                qmax, device=False)
    m = ba.nresults
    out = dict(sr=np.empty(m), phase=np.empty(m), duration=np.empty(m),
               depth=np.empty(m), jstart=np.empty(m, np.int32),
               kwidth=np.empty(m, np.int32),
               best_index=np.empty(ba.ncurves, np.int64))
    r = L.BlsResults(*[out[k].ctypes.data for k in
                       ("sr", "phase", "duration", "depth", "jstart",
                        "kwidth", "best_index")])
    _check(L.load().bls_search_batch(plan, C.byref(ba.struct), C.byref(r)),
           plan)
    return out


def bls_search_device(plan, n_off, times, flux, weights, periods, p_off,
                      nbins, qmin, qmax, sr, depth, jstart, kwidth,
                      best_index):
    """Device tensors in, device tensors out; asynchronous on the plan stream.

    times/flux/weights/periods/sr/depth/jstart/kwidth/best_index are torch
    tensors on the plan's device (float64 inputs; float32 sr/depth, int32
    jstart/kwidth, int64 best_index).  Call bls_synchronize before reading.
    """
    ba = _batch(n_off, times, flux, weights, periods, p_off, nbins, qmin,
                qmax, device=True)
    o = L.BlsDeviceResults(sr.data_ptr(), depth.data_ptr(), jstart.data_ptr(),
                           kwidth.data_ptr(), best_index.data_ptr())
    _check(L.load().bls_search_device(plan, C.byref(ba.struct), C.byref(o)),
           plan)


def bls_search_device_noalloc(n_off, times, flux, weights, periods, p_off,
                              nbins, qmin, qmax, sr, depth, jstart, kwidth,
                              best_index, flags=0, min_in_points=1,
                              stream=None):
    """bls_search_device without a plan: allocates nothing, works in the
    library's fixed per-GPU scratch array; asynchronous on `stream` (a
    torch.cuda.Stream, a raw hipStream_t as int, or None for the default
    stream) of the current device.  Synchronize the stream before reading.
    """
    ba = _batch(n_off, times, flux, weights, periods, p_off, nbins, qmin,
                qmax, device=True)
    o = L.BlsDeviceResults(sr.data_ptr(), depth.data_ptr(), jstart.data_ptr(),
                           kwidth.data_ptr(), best_index.data_ptr())
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    _check(L.load().bls_search_device_noalloc(
        C.byref(ba.struct), C.byref(o), int(flags), int(min_in_points),
        C.c_void_p(stream) if stream else None))


def bls_injection_recovery_device(plan, times, weights, base_flux,
                                  inj_period, inj_phase, inj_q, inj_depth,
                                  periods, nbins, qmin, qmax, window=0.01,
                                  sde_threshold=7.0, ptol=0.01, sr=None,
                                  flux=None):
    """Injection-recovery of one cadence (synchronous).

    times/weights/periods: torch float64 device tensors ([n], [n] or None,
    [nperiods]); base_flux: device float64 [ninj, n] (or flat); inj_*: host
    arrays [ninj].  sr (device float32 [ninj * nperiods]) and flux (device
    float64 [ninj * n]) optionally receive the periodograms and the injected
    fluxes.  Returns a dict of numpy arrays: recovered (1, 0, -1 for invalid
    data), best_index, sde.
    """
    n = int(times.shape[0])
    prm = [_f64(np.broadcast_to(np.asarray(v, np.float64), (len(inj_period),)))
           for v in (inj_period, inj_phase, inj_q, inj_depth)]
    ninj = prm[0].shape[0]
    cfg = L.BlsRecoveryConfig()
    cfg.ninj, cfg.nbins, cfg.n = ninj, int(nbins), n
    cfg.times = times.data_ptr()
    cfg.weights = None if weights is None else weights.data_ptr()
    cfg.base_flux = base_flux.data_ptr()
    cfg.inj_period, cfg.inj_phase, cfg.inj_q, cfg.inj_depth = \
        [v.ctypes.data for v in prm]
    cfg.periods = periods.data_ptr()
    cfg.nperiods = int(periods.shape[0])
    cfg.qmin, cfg.qmax = float(qmin), float(qmax)
    cfg.window, cfg.sde_threshold, cfg.ptol = (float(window),
                                               float(sde_threshold),
                                               float(ptol))
    rec = np.empty(ninj, np.int32)
    best = np.empty(ninj, np.int64)
    sde = np.empty(ninj, np.float64)
    o = L.BlsRecoveryResults(rec.ctypes.data, best.ctypes.data,
                             sde.ctypes.data,
                             None if sr is None else sr.data_ptr(),
                             None if flux is None else flux.data_ptr())
    _check(L.load().bls_injection_recovery_device(plan, C.byref(cfg),
                                                  C.byref(o)), plan)
    return dict(recovered=rec, best_index=best, sde=sde)


def bls_search_unbinned_device(plan, n_off, times, flux, weights, periods,
                               p_off, qmin, qmax, sr, depth, first_point,
                               last_point, best_index):
    """Unbinned search on device tensors; asynchronous on the plan stream.

    As bls_search_device without nbins; first_point/last_point (int32)
    receive the curve-relative input indices of each best box's first and
    last points in phase order.  Call bls_synchronize before reading.
    """
    ba = _batch(n_off, times, flux, weights, periods, p_off, 2, qmin, qmax,
                device=True)
    o = L.BlsUnbinnedResults(sr.data_ptr(), depth.data_ptr(),
                             first_point.data_ptr(), last_point.data_ptr(),
                             best_index.data_ptr())
    _check(L.load().bls_search_unbinned_device(plan, C.byref(ba.struct),
                                               C.byref(o)), plan)


def bls_detect_device(plan, n_off, periods, p_off, nbins, qmin, qmax, sr,
                      max_peaks=8, window=0.01, sde_threshold=7.0):
    """Detection statistics of each curve's periodogram (device SR tensor).

    Returns a list of dicts (mean_sr, std_sr, sde, candidate, peak_index,
    peak_sr, peak_sde), one per curve.
    """
    ba = _batch(n_off, periods, periods, None, periods, p_off, nbins, qmin,
                qmax, device=True)
    out = (L.BlsDetection * ba.ncurves)()
    _check(L.load().bls_detect_device(plan, C.byref(ba.struct),
                                      C.c_void_p(sr.data_ptr()),
                                      int(max_peaks), float(window),
                                      float(sde_threshold), out), plan)
    res = []
    for d in out:
        k = d.npeaks
        res.append(dict(mean_sr=d.mean_sr, std_sr=d.std_sr, sde=d.sde,
                        candidate=bool(d.candidate),
                        peak_index=np.array(d.peak_index[:k], np.int64),
                        peak_sr=np.array(d.peak_sr[:k], np.float32),
                        peak_sde=np.array(d.peak_sde[:k], np.float32)))
    return res


def bls_eclipse_window_device(plan, n_off, times, periods, p_off, nphase,
                              duration, min_eclipses, observed,
                              weights=None):
    """Observed-epoch counts of the eclipse detection efficiency.

    times, periods, weights (or None) and observed (int32) are device
    tensors; observed receives, per cadence and period, how many of the
    nphase trial eclipse epochs show at least min_eclipses eclipses on kept
    observations (divide by nphase for the efficiency).  Synchronous.
    """
    ba = _batch(n_off, times, times, weights, periods, p_off, 2, 0.1, 0.1,
                device=True)
    _check(L.load().bls_eclipse_window_device(
        plan, C.byref(ba.struct), int(nphase), float(duration),
        int(min_eclipses), C.c_void_p(observed.data_ptr())), plan)


def bls_variability_device(plan, n_off, flux, weights, mag, chip_off,
                           nmagbins, out, origin=0.0, width=0.1,
                           clip_sigma=3.0, max_iter=5, flag_sigma=2.0,
                           min_stars=3):
    """High-variability pre-search on device tensors.

    flux, weights (or None) and mag are device tensors (float64); out is a
    dict of device tensors: rms (f64), bin and flag (int32) per curve;
    bin_mean, bin_std (f64) and bin_count (int32) per (chip, bin).  n_off
    and chip_off are host arrays.  Synchronous.
    """
    ba = _batch(n_off, flux, flux, weights, flux, None, 2, 0.1, 0.1,
                device=True)
    co = np.ascontiguousarray(chip_off, dtype=np.int64)
    cfg = L.BlsVariabilityConfig()
    cfg.nchips = co.shape[0] - 1
    cfg.nmagbins = int(nmagbins)
    cfg.chip_off = co.ctypes.data
    cfg.mag = mag.data_ptr()
    cfg.origin, cfg.width = float(origin), float(width)
    cfg.clip_sigma, cfg.flag_sigma = float(clip_sigma), float(flag_sigma)
    cfg.max_iter, cfg.min_stars = int(max_iter), int(min_stars)
    res = L.BlsVariabilityResults()
    for k in ("rms", "bin", "flag", "bin_mean", "bin_std", "bin_count"):
        setattr(res, k, out[k].data_ptr())
    _check(L.load().bls_variability_device(plan, C.byref(ba.struct),
                                           C.byref(cfg), C.byref(res)), plan)


class Plan:
    """Owning wrapper of a bls_plan (closes on exit)."""

    def __init__(self, **cfg):
        self.handle = bls_plan_create(**cfg)

    def close(self):
        if self.handle:
            bls_plan_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving
def bls_server_config_init(**overrides) -> L.BlsServerConfig:
    cfg = L.BlsServerConfig()
    L.load().bls_server_config_init(C.byref(cfg))
    for k, v in overrides.items():
        setattr(cfg, k, v)
    return cfg


def _server_error(srv) -> str:
    buf = C.create_string_buffer(1024)
    L.load().bls_server_last_error(srv, buf, 1024)
    return buf.value.decode(errors="replace")


def bls_server_create(cfg: Optional[L.BlsServerConfig] = None, **overrides):
    if cfg is None:
        cfg = bls_server_config_init(**overrides)
    srv = C.c_void_p()
    st = L.load().bls_server_create(C.byref(srv), C.byref(cfg))
    if st != L.BLS_OK:
        raise BlsError(st, _server_error(None))
    return srv


def bls_server_submit(srv, times, flux, weights, periods, nbins, qmin,
                      qmax) -> int:
    """Queue one request (inputs are copied); returns its ticket."""
    t, x = _f64(times), _f64(flux)
    w = None if weights is None else _f64(weights)
    p = _f64(periods)
    req = L.BlsRequest(t.ctypes.data, x.ctypes.data,
                       None if w is None else w.ctypes.data, t.shape[0],
                       p.ctypes.data, p.shape[0], int(nbins), 0, float(qmin),
                       float(qmax))
    ticket = C.c_uint64()
    st = L.load().bls_server_submit(srv, C.byref(req), C.byref(ticket))
    if st != L.BLS_OK:
        raise BlsError(st, _server_error(srv))
    return ticket.value


def _result_dict(r: L.BlsResult) -> dict:
    m = int(r.nperiods)
    out = dict(status=int(r.status), best_index=int(r.best_index),
               submit_s=r.submit_s, admit_s=r.admit_s, done_s=r.done_s)
    if r.status == L.BLS_OK and m > 0:
        out["sr"] = np.ctypeslib.as_array(
            C.cast(r.sr, C.POINTER(C.c_float)), (m,)).copy()
        out["depth"] = np.ctypeslib.as_array(
            C.cast(r.depth, C.POINTER(C.c_float)), (m,)).copy()
        out["jstart"] = np.ctypeslib.as_array(
            C.cast(r.jstart, C.POINTER(C.c_int32)), (m,)).copy()
        out["kwidth"] = np.ctypeslib.as_array(
            C.cast(r.kwidth, C.POINTER(C.c_int32)), (m,)).copy()
    return out


def bls_server_poll(srv, ticket: int):
    """Result dict, or None while the request is still in flight."""
    r = L.BlsResult()
    st = L.load().bls_server_poll(srv, C.c_uint64(ticket), C.byref(r))
    if st == L.BLS_ERR_BUSY:
        return None
    if st != L.BLS_OK:
        raise BlsError(st, _server_error(srv))
    return _result_dict(r)


def bls_server_wait(srv, ticket: int, timeout_s: float = 60.0) -> dict:
    r = L.BlsResult()
    st = L.load().bls_server_wait(srv, C.c_uint64(ticket), C.byref(r),
                                  float(timeout_s))
    if st != L.BLS_OK:
        raise BlsError(st, _server_error(srv))
    return _result_dict(r)


def bls_server_release(srv, ticket: int) -> None:
    st = L.load().bls_server_release(srv, C.c_uint64(ticket))
    if st != L.BLS_OK:
        raise BlsError(st, _server_error(srv))


def bls_server_get_stats(srv) -> dict:
    s = L.BlsServerStats()
    st = L.load().bls_server_get_stats(srv, C.byref(s))
    if st != L.BLS_OK:
        raise BlsError(st, _server_error(srv))
    return {f: getattr(s, f) for f, _ in L.BlsServerStats._fields_}


def bls_server_reset_stats(srv) -> None:
    L.load().bls_server_reset_stats(srv)


def bls_server_drain(srv, timeout_s: float = 60.0) -> None:
    st = L.load().bls_server_drain(srv, float(timeout_s))
    if st != L.BLS_OK:
        raise BlsError(st, _server_error(srv))


def bls_server_destroy(srv) -> None:
    if srv:
        L.load().bls_server_destroy(srv)
