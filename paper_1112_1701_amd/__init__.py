"""MI355X (gfx950) box-least-squares periodogram.

The search (Law et al. 2011, section 2.2.2: phase each light curve at every
trial period and test a range of box durations and phases with the
box-least-squares statistic) runs entirely in the HIP library
``libbls_mi355x.so`` behind the C ABI of ``include/bls.h``.  This package is
the thin Python binding: functions carry the C names and only marshal
numpy arrays, torch device tensors and ctypes structures.  PyTorch is used
for device memory and streams only.
"""
from .api import (  # noqa: F401
    BlsError,
    bls_plan_config_init,
    bls_plan_create,
    bls_plan_destroy,
    bls_search,
    bls_search_batch,
    bls_search_device,
    bls_search_device_noalloc,
    bls_synchronize,
    bls_get_stream,
    bls_width_range,
    bls_last_error,
    bls_status_string,
    bls_last_stats,
    bls_kernel_times,
    bls_kernel_times_reset,
    bls_debug_phase_bins,
    bls_detect_device,
    bls_eclipse_window_device,
    bls_variability_device,
    bls_search_unbinned_device,
    bls_injection_recovery_device,
    bls_server_config_init,
    bls_server_create,
    bls_server_submit,
    bls_server_poll,
    bls_server_wait,
    bls_server_release,
    bls_server_get_stats,
    bls_server_reset_stats,
    bls_server_drain,
    bls_server_destroy,
    Plan,
)
from ._lib import (  # noqa: F401
    BLS_OK, BLS_ERR_INVALID_ARG, BLS_ERR_NO_MEMORY, BLS_ERR_DEVICE,
    BLS_ERR_CAPACITY, BLS_ERR_BUSY, BLS_ERR_TIMEOUT, BLS_DIP_ONLY,
    BLS_NO_GRAPH, BLS_NO_AUTOTUNE, BLS_MAX_NBINS, LIB_PATH,
    BLS_NOALLOC_MAX_CURVES, BLS_NOALLOC_MAX_POINTS, BLS_NOALLOC_SCRATCH_BYTES,
)
