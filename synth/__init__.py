"""Seeded synthetic light curves and trial-period grids.

Shared by the tests, the benchmark and the smoke check.  It only draws
inputs: times on a survey-like cadence, Gaussian noise and injected box
dips.  It contains none of the search's arithmetic.
"""
from .lightcurves import (  # noqa: F401
    LightCurve,
    Batch,
    T_START,
    log_period_grid,
    nightly_times,
    minute_grid_times,
    inject_box,
    config1,
    config2,
    config3,
    config4,
    serving_requests,
    uniform_batch,
    uneven_batch,
    small_curve,
    survey_cadence,
    cadence_batch,
    variability_field,
    detection_periodograms,
    InjectionSet,
    injection_set,
)
