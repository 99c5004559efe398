"""ctypes binding of libbls_mi355x.so (the C ABI of include/bls.h).

Argument marshalling only: every step of the search runs in the HIP
library.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbls_mi355x.so")

BLS_OK = 0
BLS_ERR_INVALID_ARG = -1
BLS_ERR_NO_MEMORY = -2
BLS_ERR_DEVICE = -3
BLS_ERR_CAPACITY = -4
BLS_ERR_BUSY = -5
BLS_ERR_TIMEOUT = -6

BLS_DIP_ONLY = 1 << 0
BLS_NO_GRAPH = 1 << 1
BLS_NO_AUTOTUNE = 1 << 2
BLS_MAX_NBINS = 4096
BLS_NOALLOC_MAX_CURVES = 64
BLS_NOALLOC_MAX_POINTS = 1 << 20
BLS_NOALLOC_SCRATCH_BYTES = 16 * (1 << 20) + 16384


class BlsPlanConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_curves", C.c_int32),
                ("max_points", C.c_int64), ("max_periods", C.c_int64),
                ("max_nbins", C.c_int32), ("min_in_points", C.c_int32),
                ("flags", C.c_uint32), ("reserved", C.c_int32),
                ("hip_stream", C.c_void_p)]


class BlsBatch(C.Structure):
    _fields_ = [("ncurves", C.c_int32), ("nbins_all", C.c_int32),
                ("n_off", C.c_void_p), ("times", C.c_void_p),
                ("flux", C.c_void_p), ("weights", C.c_void_p),
                ("p_off", C.c_void_p), ("periods", C.c_void_p),
                ("nperiods_shared", C.c_int64), ("nbins", C.c_void_p),
                ("qmin", C.c_void_p), ("qmax", C.c_void_p),
                ("qmin_all", C.c_double), ("qmax_all", C.c_double)]


class BlsResults(C.Structure):
    _fields_ = [("sr", C.c_void_p), ("phase", C.c_void_p),
                ("duration", C.c_void_p), ("depth", C.c_void_p),
                ("jstart", C.c_void_p), ("kwidth", C.c_void_p),
                ("best_index", C.c_void_p)]


class BlsDeviceResults(C.Structure):
    _fields_ = [("sr", C.c_void_p), ("depth", C.c_void_p),
                ("jstart", C.c_void_p), ("kwidth", C.c_void_p),
                ("best_index", C.c_void_p)]


class BlsCallStats(C.Structure):
    _fields_ = [("search_ms", C.c_double), ("total_ms", C.c_double),
                ("trial_points", C.c_double), ("box_evals", C.c_double),
                ("work_items", C.c_int64), ("grid", C.c_int32),
                ("block", C.c_int32), ("lds_bytes", C.c_int32),
                ("graph_replayed", C.c_int32)]


BLS_MAX_PEAKS = 16


class BlsDetection(C.Structure):
    _fields_ = [("mean_sr", C.c_double), ("std_sr", C.c_double),
                ("sde", C.c_double), ("npeaks", C.c_int32),
                ("candidate", C.c_int32),
                ("peak_index", C.c_int64 * BLS_MAX_PEAKS),
                ("peak_sr", C.c_float * BLS_MAX_PEAKS),
                ("peak_sde", C.c_float * BLS_MAX_PEAKS)]


class BlsUnbinnedResults(C.Structure):
    _fields_ = [("sr", C.c_void_p), ("depth", C.c_void_p),
                ("first_point", C.c_void_p), ("last_point", C.c_void_p),
                ("best_index", C.c_void_p)]


class BlsVariabilityConfig(C.Structure):
    _fields_ = [("nchips", C.c_int32), ("nmagbins", C.c_int32),
                ("chip_off", C.c_void_p), ("mag", C.c_void_p),
                ("origin", C.c_double), ("width", C.c_double),
                ("clip_sigma", C.c_double), ("flag_sigma", C.c_double),
                ("max_iter", C.c_int32), ("min_stars", C.c_int32)]


class BlsVariabilityResults(C.Structure):
    _fields_ = [("rms", C.c_void_p), ("bin", C.c_void_p),
                ("flag", C.c_void_p), ("bin_mean", C.c_void_p),
                ("bin_std", C.c_void_p), ("bin_count", C.c_void_p)]


class BlsRecoveryConfig(C.Structure):
    _fields_ = [("ninj", C.c_int32), ("nbins", C.c_int32), ("n", C.c_int64),
                ("times", C.c_void_p), ("weights", C.c_void_p),
                ("base_flux", C.c_void_p), ("inj_period", C.c_void_p),
                ("inj_phase", C.c_void_p), ("inj_q", C.c_void_p),
                ("inj_depth", C.c_void_p), ("periods", C.c_void_p),
                ("nperiods", C.c_int64), ("qmin", C.c_double),
                ("qmax", C.c_double), ("window", C.c_double),
                ("sde_threshold", C.c_double), ("ptol", C.c_double)]


class BlsRecoveryResults(C.Structure):
    _fields_ = [("recovered", C.c_void_p), ("best_index", C.c_void_p),
                ("sde", C.c_void_p), ("sr", C.c_void_p), ("flux", C.c_void_p)]


class BlsRequest(C.Structure):
    _fields_ = [("times", C.c_void_p), ("flux", C.c_void_p),
                ("weights", C.c_void_p), ("n", C.c_int64),
                ("periods", C.c_void_p), ("nperiods", C.c_int64),
                ("nbins", C.c_int32), ("reserved", C.c_int32),
                ("qmin", C.c_double), ("qmax", C.c_double)]


class BlsResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32),
                ("nperiods", C.c_int64), ("sr", C.c_void_p),
                ("depth", C.c_void_p), ("jstart", C.c_void_p),
                ("kwidth", C.c_void_p), ("best_index", C.c_int64),
                ("submit_s", C.c_double), ("admit_s", C.c_double),
                ("done_s", C.c_double)]


class BlsServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("admitted", C.c_int64),
                ("completed", C.c_int64), ("failed", C.c_int64),
                ("queued", C.c_int64), ("active", C.c_int64),
                ("ticks", C.c_int64), ("p50_ms", C.c_double),
                ("p99_ms", C.c_double), ("mean_ms", C.c_double),
                ("max_ms", C.c_double), ("trial_points", C.c_double),
                ("box_evals", C.c_double), ("busy_s", C.c_double),
                ("wall_s", C.c_double), ("device_bytes_in_use", C.c_int64),
                ("device_bytes_peak", C.c_int64)]


class BlsServerConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("max_slots", C.c_int32),
                ("arena_bytes", C.c_int64), ("max_nbins", C.c_int32),
                ("min_in_points", C.c_int32), ("flags", C.c_uint32),
                ("reserved", C.c_int32), ("tick_cost", C.c_double),
                ("max_request_points", C.c_int64),
                ("max_request_periods", C.c_int64)]


_lib = None


def load():
    """Load the HIP library; raises if it is missing (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    # One HIP runtime per process: torch bundles its own libamdhip64.so.7.
    # Loading torch first makes this library bind to that same runtime
    # (same soname) instead of a second copy, which would leave torch
    # without devices.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            "libbls_mi355x.so is not built; run "
            "`python -m paper_1112_1701_amd.build` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "bls_plan_config_init": (None, [P]),
        "bls_plan_create": (C.c_int, [P, P]),
        "bls_plan_destroy": (C.c_int, [P]),
        "bls_search": (C.c_int, [P, P, P, P, I64, P, I64, I32, D, D, P, P, P,
                                 P, P, P, P]),
        "bls_search_batch": (C.c_int, [P, P, P]),
        "bls_search_device": (C.c_int, [P, P, P]),
        "bls_synchronize": (C.c_int, [P]),
        "bls_get_stream": (C.c_int, [P, P]),
        "bls_width_range": (C.c_int, [I32, D, D, P, P]),
        "bls_last_error": (C.c_int, [P, P, C.c_size_t]),
        "bls_status_string": (C.c_char_p, [C.c_int]),
        "bls_last_stats": (C.c_int, [P, P]),
        "bls_kernel_times": (C.c_int, [P, P, I32, P]),
        "bls_kernel_times_reset": (C.c_int, [P]),
        "bls_debug_phase_bins": (C.c_int, [P, P, I64, D, I32, P]),
        "bls_detect_device": (C.c_int, [P, P, P, I32, D, D, P]),
        "bls_eclipse_window_device": (C.c_int, [P, P, I32, D, I32, P]),
        "bls_variability_device": (C.c_int, [P, P, P, P]),
        "bls_search_unbinned_device": (C.c_int, [P, P, P]),
        "bls_search_device_noalloc": (C.c_int, [P, P, C.c_uint32, I32, P]),
        "bls_injection_recovery_device": (C.c_int, [P, P, P]),
    }
    optional = {
        "bls_server_config_init": (None, [P]),
        "bls_server_create": (C.c_int, [P, P]),
        "bls_server_submit": (C.c_int, [P, P, P]),
        "bls_server_poll": (C.c_int, [P, C.c_uint64, P]),
        "bls_server_wait": (C.c_int, [P, C.c_uint64, P, D]),
        "bls_server_release": (C.c_int, [P, C.c_uint64]),
        "bls_server_get_stats": (C.c_int, [P, P]),
        "bls_server_reset_stats": (C.c_int, [P]),
        "bls_server_drain": (C.c_int, [P, D]),
        "bls_server_last_error": (C.c_int, [P, P, C.c_size_t]),
        "bls_server_destroy": (C.c_int, [P]),
    }
    for name, (res, args) in list(sig.items()) + list(optional.items()):
        if name in optional and not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib
