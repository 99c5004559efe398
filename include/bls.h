/*
 * bls.h -- C ABI of the MI355X (gfx950) box-least-squares periodogram.
 *
 * The operation (Law et al. 2011, section 2.2.2, "A Parallel Eclipse Search
 * Using Graphics Processing Units"): each light curve is phased at every
 * trial period and a range of box durations and phases is tested with the
 * box-least-squares statistic the section cites (Kovacs et al. 2002).  For
 * one curve with times t_i, fluxes x_i and weights w_i (points with w_i = 0
 * are dropped first):
 *
 *   t0 = min t_i,  d_i = t_i - t0,  W = sum w_i,  xbar = sum w_i x_i / W;
 *   per trial period P: f = 1/P, phase_i = frac(d_i f),
 *   bin_i = min(trunc(phase_i * nbins), nbins - 1);
 *   a box is bins j, j+1, ..., j+k-1 (mod nbins) with
 *   kmin = max(1, lround(qmin nbins)) <= k <= kmax = min(nbins-1, lround(qmax nbins));
 *   R = sum_{box} w_i,  S = sum_{box} w_i (x_i - xbar),
 *   v = S^2 / (R (W - R)), valid iff min_in_points <= points in box <= n - 1
 *   (and S < 0 with BLS_DIP_ONLY);
 *   SR = sqrt(max v) over valid boxes with v > 0 (0 if none), exact ties to
 *   the smallest k, then the smallest j;
 *   depth = -S W / (R (W - R)) of that box (> 0 for a dip),
 *   phase = j / nbins (box start, relative to t0),
 *   duration = k P / nbins,
 *   best_index = first period with the largest SR.
 *
 * A period with no valid box reports SR = 0, jstart = kwidth = -1 and NaN
 * phase, duration and depth.
 *
 * Precision: the phase is computed in FP64 with the operation order above,
 * so bins are those of an FP64 evaluation; per-bin sums are exact
 * fixed-point integers; box sums and the statistic are FP32.  SR agrees with
 * an FP64 evaluation to about 1e-6 relative.  Values and weights are encoded
 * relative to the curve's largest |w y| and largest w (30 bits), so the error
 * grows with the ratio of the largest value to the noise: within 1e-5 for a
 * 1e4-sigma outlier, reaching 1e-5 near 1e5 sigma.
 *
 * Conventions: every function returns a bls_status.  No function throws.
 * Caller-owned host arrays are never retained after a synchronous call
 * returns.  A plan is not thread-safe; distinct plans are independent.
 */
#ifndef BLS_MI355X_H
#define BLS_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BLS_API_VERSION 1
#define BLS_MAX_NBINS 4096          /* largest nbins a plan accepts */

typedef enum {
    BLS_OK = 0,
    BLS_ERR_INVALID_ARG = -1,   /* bad shape, parameter or data            */
    BLS_ERR_NO_MEMORY = -2,     /* host or device allocation failed        */
    BLS_ERR_DEVICE = -3,        /* a HIP call failed; see bls_last_error    */
    BLS_ERR_CAPACITY = -4,      /* shape exceeds the plan's capacities      */
    BLS_ERR_BUSY = -5,          /* result not ready yet (serving)           */
    BLS_ERR_TIMEOUT = -6        /* wait timed out (serving)                 */
} bls_status;

/* Plan flags. */
enum {
    BLS_DIP_ONLY = 1u << 0,     /* only boxes below the mean (S < 0) count  */
    BLS_NO_GRAPH = 1u << 1,     /* never capture/replay HIP graphs          */
    BLS_NO_AUTOTUNE = 1u << 2   /* use the built-in tile table              */
};

typedef struct bls_plan bls_plan;

/* Plan configuration.  Initialise with bls_plan_config_init. */
typedef struct {
    int32_t device;         /* HIP device ordinal                              */
    int32_t max_curves;     /* curves per call                                 */
    int64_t max_points;     /* total points per call (all curves)              */
    int64_t max_periods;    /* total per-period results per call               */
    int32_t max_nbins;      /* <= BLS_MAX_NBINS                                */
    int32_t min_in_points;  /* minimum points inside a valid box (>= 1)        */
    uint32_t flags;         /* BLS_DIP_ONLY | BLS_NO_GRAPH | BLS_NO_AUTOTUNE   */
    int32_t reserved;
    void *hip_stream;       /* hipStream_t to run on; NULL = plan-owned stream */
} bls_plan_config;

/* Defaults: device 0, 1 curve, 2^20 points, 2^20 periods, max_nbins 4096,
 * min_in_points 1, no flags, plan-owned stream. */
void bls_plan_config_init(bls_plan_config *cfg);

/* Create a plan: allocates device buffers sized by cfg on cfg->device.
 * *out receives the plan (NULL on error).  Errors: INVALID_ARG (bad cfg),
 * NO_MEMORY, DEVICE. */
int bls_plan_create(bls_plan **out, const bls_plan_config *cfg);

/* Release a plan and its device memory.  NULL is accepted. */
int bls_plan_destroy(bls_plan *plan);

/*
 * One light curve, host arrays (the signature of the method's statement).
 *   times, flux: [n]; weights: [n] or NULL for unit weights.
 *   periods: [nperiods] trial periods, finite and > 0.
 *   nbins: phase bins (2..max_nbins); qmin, qmax: box duty-cycle range,
 *   0 < qmin <= qmax < 1.
 * Outputs, [nperiods] each, caller-owned, any may be NULL: sr, phase,
 * duration, depth (doubles), jstart, kwidth (box start bin and width);
 * best_index: first period index with the largest SR (may be NULL).
 * Synchronous.  On any error the outputs are untouched.  The first host-array
 * call on a plan pins a host staging buffer sized for the plan's limits
 * (24 B per point plus 8 B per result, or 16 B per result, the larger),
 * kept until bls_plan_destroy; without pinned memory the copies run from
 * the caller's pageable arrays.
 * Errors: INVALID_ARG (non-finite time or flux of a kept point, negative or
 * non-finite weight, fewer than 2 kept points, bad period, nbins or q range,
 * kmin > kmax), CAPACITY (n, nperiods or nbins above the plan's limits),
 * DEVICE, NO_MEMORY.
 */
int bls_search(bls_plan *plan, const double *times, const double *flux,
               const double *weights, int64_t n, const double *periods,
               int64_t nperiods, int32_t nbins, double qmin, double qmax,
               double *sr, double *phase, double *duration, double *depth,
               int32_t *jstart, int32_t *kwidth, int64_t *best_index);

/*
 * Many light curves packed end to end (CSR).  Curve c owns points
 * [n_off[c], n_off[c+1]) of times/flux/weights and periods
 * [p_off[c], p_off[c+1]) of periods; with p_off == NULL every curve uses
 * periods[0 .. nperiods_shared).  nbins/qmin/qmax are per-curve arrays, or
 * NULL to use nbins_all/qmin_all/qmax_all.  Curve c's per-period results
 * are stored from r_off(c) = p_off ? p_off[c] : c * nperiods_shared.
 * n_off, p_off, nbins, qmin and qmax are always host arrays; whether times,
 * flux, weights and periods are host or device pointers depends on the call.
 */
typedef struct {
    int32_t ncurves;
    int32_t nbins_all;
    const int64_t *n_off;       /* [ncurves + 1], n_off[0] == 0, non-decreasing */
    const double *times;
    const double *flux;
    const double *weights;      /* NULL = unit weights                       */
    const int64_t *p_off;       /* [ncurves + 1] or NULL (shared grid)       */
    const double *periods;
    int64_t nperiods_shared;
    const int32_t *nbins;       /* [ncurves] or NULL                         */
    const double *qmin;         /* [ncurves] or NULL                         */
    const double *qmax;         /* [ncurves] or NULL                         */
    double qmin_all;
    double qmax_all;
} bls_batch;

/* Host result arrays for bls_search_batch, indexed as described above;
 * any may be NULL.  best_index has one entry per curve. */
typedef struct {
    double *sr;
    double *phase;
    double *duration;
    double *depth;
    int32_t *jstart;
    int32_t *kwidth;
    int64_t *best_index;
} bls_results;

/* Batch of curves in host memory: one persistent launch for the whole
 * batch.  Synchronous; outputs untouched on error.  Errors as bls_search. */
int bls_search_batch(bls_plan *plan, const bls_batch *batch,
                     const bls_results *out);

/* Device result arrays for bls_search_device (device pointers, all
 * required): FP32 SR and depth, box start and width, and per-curve best
 * period index. */
typedef struct {
    float *sr;
    float *depth;
    int32_t *jstart;
    int32_t *kwidth;
    int64_t *best_index;
} bls_device_results;

/*
 * Batch whose times, flux, weights and periods are DEVICE pointers on the
 * plan's device; results go to device arrays.  Shapes and parameters are
 * checked on the host before anything is queued; the data itself is checked
 * on the device.  Asynchronous on the plan's stream: the device arrays are
 * borrowed until bls_synchronize returns.  Curves whose data is invalid get
 * SR = NaN and are reported by bls_synchronize.  Repeated calls with the
 * same batch description replay captured HIP graphs.  Several calls may be
 * queued on one plan without synchronizing in between, with the same or
 * different batches: a call that must rewrite the plan's staged batch
 * description first waits (on the host) until the copies of the queued
 * calls have read it.  They share the plan's prepared-point scratch, so
 * they run one after the other in stream order.
 */
int bls_search_device(bls_plan *plan, const bls_batch *batch,
                      const bls_device_results *out);

/*
 * bls_search_device for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  No plan: the call allocates nothing (no hipMalloc or hipFree,
 * no pinned or heap host memory) and works in a fixed scratch array that
 * the library holds in each GPU's memory until the process ends
 * (BLS_NOALLOC_SCRATCH_BYTES per GPU: prepared points, curve descriptors,
 * work segments and counters).
 *   batch: as for bls_search_device (times, flux, weights, periods on the
 *   current HIP device; n_off, p_off, nbins, qmin, qmax host arrays), at most
 *   BLS_NOALLOC_MAX_CURVES curves and BLS_NOALLOC_MAX_POINTS points in all,
 *   nbins <= BLS_MAX_NBINS.
 *   out: as for bls_search_device.
 *   flags: BLS_DIP_ONLY or 0; min_in_points >= 1 (as a plan's).
 *   hip_stream: the hipStream_t to queue on (NULL: the default stream).
 * Runs on the calling thread's current HIP device, asynchronously on
 * hip_stream, with the built-in tile table (no tuning); results equal
 * bls_search_device's.  A curve whose data is invalid gets SR = NaN and
 * jstart = kwidth = -1 (nothing is read back to report it).
 * Every call on one GPU shares that GPU's scratch, which keeps the last
 * call's contents: calls queued on one stream run one after the other,
 * calls on different streams (or threads) that overlap on one GPU race.
 * Errors, checked on the host before anything is queued (message via
 * bls_last_error(NULL, ...)): INVALID_ARG (as bls_search_device, or flags),
 * CAPACITY (more curves or points than the limits above, a histogram that
 * does not fit a workgroup's LDS), DEVICE.
 */
#define BLS_NOALLOC_MAX_CURVES 64
#define BLS_NOALLOC_MAX_POINTS (1 << 20)
#define BLS_NOALLOC_SCRATCH_BYTES (16u * (1u << 20) + 16384u)
int bls_search_device_noalloc(const bls_batch *batch,
                              const bls_device_results *out, uint32_t flags,
                              int32_t min_in_points, void *hip_stream);

/* Wait for the plan's queued work.  Returns INVALID_ARG if a curve of the
 * last bls_search_device call had invalid data (message names the first
 * such curve), DEVICE on a HIP error. */
int bls_synchronize(bls_plan *plan);

/* The hipStream_t the plan runs on. */
int bls_get_stream(const bls_plan *plan, void **stream);

/* Widths a (nbins, qmin, qmax) triple selects, per the rule above. */
int bls_width_range(int32_t nbins, double qmin, double qmax, int32_t *kmin,
                    int32_t *kmax);

/* Message of the plan's most recent error (empty if none); NUL-terminated,
 * truncated to len.  plan may be NULL for errors of bls_plan_create. */
int bls_last_error(const bls_plan *plan, char *buf, size_t len);

/* Static description of a status code. */
const char *bls_status_string(int status);

/*
 * Unbinned search: box edges fall between data points instead of on a
 * phase-bin grid (the range of durations and phases of section 2.2.2 taken
 * to the limit of the data).  Per curve and trial period, the kept points
 * are ordered by phase (t0 = min kept time, phase = frac((t - t0) / P) in
 * FP64, ties by input order); a box is a cyclic run of m consecutive points
 * of that order, 1 <= m <= n - 1, that some box of duty cycle q in
 * [qmin, qmax] of the period holds exactly: the run does not split equal
 * phases, its phase span (first to last point) is below qmax and the phase
 * distance between its two outside neighbours exceeds qmin (1 when they are
 * the same point).  Validity, statistic and tie rules are those of the
 * binned search, ties going to the smaller m, then to the earlier start in
 * phase order.
 * batch: as for bls_search_device (device times, flux, weights, periods);
 * nbins is ignored and qmin/qmax are phase fractions; at most 2^20 points
 * per curve (curves above 4096 points keep their per-point arrays in a
 * plan-owned device workspace instead of LDS, about 36 bytes per point per
 * resident workgroup, at most about 1 GiB, and run slower).  out: device arrays [results]: FP32 SR and depth, and the
 * input indices (within the curve) of the best box's first and last points
 * in phase order (-1 where no box); best_index per curve.  Asynchronous on
 * the plan's stream: bls_synchronize reports invalid data.  Errors:
 * INVALID_ARG, CAPACITY (a curve above 2^20 points, plan limits), DEVICE,
 * NO_MEMORY (the workspace of long curves).
 */
typedef struct {
    float *sr;
    float *depth;
    int32_t *first_point;
    int32_t *last_point;
    int64_t *best_index;
} bls_unbinned_results;

int bls_search_unbinned_device(bls_plan *plan, const bls_batch *batch,
                               const bls_unbinned_results *out);

/*
 * Detection statistics of each curve's periodogram (the step after the
 * search: the signal detection efficiency of the cited BLS statistic and
 * the strongest peaks).  Per curve, over its m trial periods:
 *   mean_sr, std_sr: mean and population standard deviation of SR;
 *   sde = (max SR - mean_sr) / std_sr (0 if std_sr is 0);
 *   peaks: up to max_peaks (<= BLS_MAX_PEAKS), each the largest SR among
 *   periods not yet suppressed (ties: smallest index); a peak at P suppresses
 *   every period P' with |P' - h P| <= window * h P, h in {1, 1/2, 2, 1/3, 3};
 *   the search stops when no unsuppressed period has SR > 0;
 *   peak_sde = (peak SR - mean_sr) / std_sr; candidate = sde >= sde_threshold.
 * batch: as for bls_search_device (periods are device pointers); sr: device
 * [results] as written by bls_search_device for that batch.  out: host
 * [ncurves].  Synchronous on the plan's stream.  Errors: INVALID_ARG,
 * CAPACITY, DEVICE.
 */
#define BLS_MAX_PEAKS 16
typedef struct {
    double mean_sr;
    double std_sr;
    double sde;
    int32_t npeaks;
    int32_t candidate;
    int64_t peak_index[BLS_MAX_PEAKS];
    float peak_sr[BLS_MAX_PEAKS];
    float peak_sde[BLS_MAX_PEAKS];
} bls_detection;

int bls_detect_device(bls_plan *plan, const bls_batch *batch, const float *sr,
                      int32_t max_peaks, double window, double sde_threshold,
                      bls_detection *out);

/*
 * Eclipse detection efficiency of observing cadences: the chance that at
 * least min_eclipses eclipses of a binary with a given period fall on
 * observations, given the real cadence with its daytime and weather gaps
 * (the simulation behind the paper's detection-efficiency figure, section
 * 5, Discussion and conclusions).  Per cadence and trial period P (f = 1/P):
 *   the kept times (weight > 0; all if weights is NULL) are folded into
 *   nphase phase bins as in the search (t0 = min kept time, bin =
 *   min(trunc(frac((t - t0) f) nphase), nphase - 1), FP64);
 *   the eclipse of trial epoch j (0 <= j < nphase) covers bins j .. j+k-1
 *   modulo nphase, k = lround(duration f nphase) clamped to [1, nphase];
 *   a point of cycle floor((t - t0) f) in bin b lies in that cycle's eclipse
 *   when b >= j and in the previous cycle's when the window wrapped (b < j);
 *   observed[r] = number of epochs j with at least min_eclipses distinct
 *   eclipses holding a kept point; the efficiency is observed[r] / nphase.
 * cadences: a bls_batch whose times, weights and periods are DEVICE pointers
 * (flux, nbins, qmin, qmax are ignored); each cadence needs >= 1 point.
 * observed: DEVICE int32 [results], indexed as bls_search_device's results.
 * nphase <= BLS_MAX_NBINS; duration > 0 in the units of the times;
 * min_eclipses 1 or 2.  Synchronous on the plan's stream.  Errors:
 * INVALID_ARG (bad arguments; a cadence with a non-finite kept time, a bad
 * weight, no kept point or a bad period: its results are -1), CAPACITY
 * (plan limits, or more than 2^29 cycles in one cadence), DEVICE.
 */
int bls_eclipse_window_device(bls_plan *plan, const bls_batch *cadences,
                              int32_t nphase, double duration,
                              int32_t min_eclipses, int32_t *observed);

/*
 * Injection-recovery: the detection efficiency of a cadence through the
 * search itself (the paper's detection-efficiency simulations on real
 * cadences, section 5, Discussion and conclusions, with each simulated
 * eclipse found by the box search and its detection statistic instead of
 * only counted on the cadence).  Every injection is a copy of one cadence
 * with its own flux realization and one box eclipse:
 *   t0 = min kept time (weight > 0; all points if weights is NULL), d = t - t0;
 *   injection i (period P_i > 0, start phase phi_i in [0, 1), duty cycle q_i
 *   in (0, 1), finite depth delta_i), in FP64 with this operation order:
 *   f = 1/P_i, c = d f, u = c - phi_i, v = u - floor(u); a kept point with
 *   v < q_i gets flux base_i - delta_i, every other point base_i.
 * Each copy is searched over the shared trial grid (nbins, qmin, qmax) as by
 * bls_search_device, and its periodogram's detection statistics are taken
 * as by bls_detect_device (window); the injection is recovered when SDE >=
 * sde_threshold and the best period P_b (first period of the largest SR)
 * satisfies |P_b - h P_i| <= ptol h P_i for some h in {1, 1/2, 2}.
 * The batch is ninj copies of n points: ninj <= max_curves, ninj * n <=
 * max_points and ninj * nperiods <= max_periods of the plan.
 */
typedef struct {
    int32_t ninj;               /* injections                                */
    int32_t nbins;              /* phase bins of the search                  */
    int64_t n;                  /* points of the cadence (>= 2)              */
    const double *times;        /* DEVICE [n]                                */
    const double *weights;      /* DEVICE [n] or NULL (unit weights)         */
    const double *base_flux;    /* DEVICE [ninj * n], injection-major        */
    const double *inj_period;   /* host [ninj]                               */
    const double *inj_phase;    /* host [ninj]                               */
    const double *inj_q;        /* host [ninj]                               */
    const double *inj_depth;    /* host [ninj]                               */
    const double *periods;      /* DEVICE [nperiods] trial grid              */
    int64_t nperiods;
    double qmin, qmax;          /* box duty-cycle range of the search        */
    double window;              /* detection: relative suppression window    */
    double sde_threshold;
    double ptol;                /* relative period tolerance (>= 0)          */
} bls_recovery_config;

typedef struct {
    int32_t *recovered;         /* host [ninj]: 1, 0, or -1 for a copy with
                                   invalid data or trial periods (required)  */
    int64_t *best_index;        /* host [ninj] or NULL                       */
    double *sde;                /* host [ninj] or NULL                       */
    float *sr;                  /* DEVICE [ninj * nperiods] or NULL: the
                                   periodograms, injection-major             */
    double *flux;               /* DEVICE [ninj * n] or NULL: the injected
                                   fluxes                                    */
} bls_recovery_results;

/* Synchronous on the plan's stream.  Errors: INVALID_ARG (arguments, an
 * injection parameter, nbins or q range), CAPACITY (plan limits), DEVICE,
 * NO_MEMORY.  Copies with invalid data are reported in recovered (-1), not
 * as an error. */
int bls_injection_recovery_device(bls_plan *plan,
                                  const bls_recovery_config *cfg,
                                  const bls_recovery_results *out);

/*
 * High-variability pre-search (the step before the box search, section
 * 2.2.1): stars much more variable than others of similar magnitude on the
 * same chip are flagged.  Per star c (a curve of the batch):
 *   rms[c] = population RMS about the mean of its kept values (weight > 0,
 *   all if weights is NULL), unweighted; a star with no kept value, a
 *   non-finite kept value or a bad weight is invalid (rms NaN, bin -1,
 *   flag -1);
 *   bin[c] = floor((mag[c] - origin) / width) when in [0, nmagbins), else
 *   -1 (also for a non-finite magnitude).
 * Per (chip k, bin b), over the valid stars of chip k in bin b (chip k holds
 * stars chip_off[k] .. chip_off[k+1]-1): the clipped set starts as all of
 * them; a round takes its mean and population deviation and drops members
 * outside [mean - clip_sigma dev, mean + clip_sigma dev]; rounds repeat until
 * one drops nothing or max_iter rounds have dropped members; bin_mean,
 * bin_std and bin_count describe the final set (NaN, NaN, 0 if the bin has
 * no star).  When bin_count >= min_stars every star of the bin with
 * rms > bin_mean + flag_sigma bin_std gets flag 1; other valid stars 0.
 * The paper's choices: width 0.1 mag, flag_sigma 2.
 */
typedef struct {
    int32_t nchips;
    int32_t nmagbins;           /* 1 .. 4096 bins per chip                  */
    const int64_t *chip_off;    /* host [nchips + 1]; chip_off[nchips] ==
                                   ncurves, non-decreasing                  */
    const double *mag;          /* DEVICE [ncurves] reference magnitudes    */
    double origin;              /* lower edge of bin 0                      */
    double width;               /* bin width (> 0)                          */
    double clip_sigma;          /* > 0                                      */
    double flag_sigma;          /* >= 0                                     */
    int32_t max_iter;           /* 0 .. 64 clipping rounds                  */
    int32_t min_stars;          /* >= 1                                     */
} bls_variability_config;

/* Device result arrays (all required). */
typedef struct {
    double *rms;                /* [ncurves]                                */
    int32_t *bin;               /* [ncurves]                                */
    int32_t *flag;              /* [ncurves]                                */
    double *bin_mean;           /* [nchips * nmagbins], chip-major          */
    double *bin_std;            /* [nchips * nmagbins]                      */
    int32_t *bin_count;         /* [nchips * nmagbins]                      */
} bls_variability_results;

/* curves: a bls_batch whose flux and weights are DEVICE pointers (times,
 * periods, nbins, qmin, qmax are ignored; curves may be empty).
 * Synchronous on the plan's stream.  Errors: INVALID_ARG, CAPACITY (more
 * curves than max_curves, nmagbins or max_iter above their limits), DEVICE,
 * NO_MEMORY. */
int bls_variability_device(bls_plan *plan, const bls_batch *curves,
                           const bls_variability_config *cfg,
                           const bls_variability_results *out);

/*
 * Diagnostic: the phase bin the search kernel assigns to each point of one
 * curve (unit weights) at one trial period, computed by the same device
 * code (t0 = min time, d = t - t0, f = 1/P, bin = min(trunc(frac(d f)
 * nbins), nbins - 1), all FP64).  times: host [n], finite; bins: host [n]
 * output.  Synchronous.  For checking bin-exact agreement with an FP64
 * reference.  Errors: INVALID_ARG, CAPACITY (n above max_points), DEVICE.
 */
int bls_debug_phase_bins(bls_plan *plan, const double *times, int64_t n,
                         double period, int32_t nbins, int32_t *bins);

/* Timing and shape of the plan's last search, unbinned-search,
 * eclipse-window, variability or detection call.  search_ms covers the
 * call's kernels.  For the eclipse window trial_points is points x periods
 * and box_evals periods x nphase epoch decisions; for the variability
 * pre-search, points and stars; for detection, the periods scanned; for the
 * unbinned search box_evals estimates the run steps as the sum of
 * n * qmax * n * nperiods. */
typedef struct {
    double search_ms;       /* main kernel(s), device time (HIP events)     */
    double total_ms;        /* whole call as queued on the stream           */
    double trial_points;    /* sum over curves of N_c * nperiods_c          */
    double box_evals;       /* sum over curves of nbins * nwidths * nperiods */
    int64_t work_items;     /* (curve, period tile) items                   */
    int32_t grid;           /* workgroups of the persistent launch          */
    int32_t block;          /* threads per workgroup                        */
    int32_t lds_bytes;      /* dynamic LDS per workgroup                    */
    int32_t graph_replayed; /* 1 if the call replayed a captured graph      */
} bls_call_stats;

int bls_last_stats(const bls_plan *plan, bls_call_stats *out);

/* Device durations of the search kernel (or unbinned kernel) launches of
 * the plan's search calls since the last bls_kernel_times_reset, measured by
 * HIP events recorded on the plan's stream right before and after each
 * launch (graph replays included: the kernel is its own graph).  Waits for
 * the plan's stream, then writes the most recent min(max, available)
 * durations in ms, oldest first, to ms[] and their number to *count; the
 * plan keeps the last 64.  Errors: INVALID_ARG, DEVICE. */
int bls_kernel_times(bls_plan *plan, float *ms, int32_t max, int32_t *count);
int bls_kernel_times_reset(bls_plan *plan);

/* ------------------------------------------------------------------ serving
 * A request loop with continuous batching.  Requests (one light curve with
 * its own trial-period grid, bins and duty-cycle range) are queued by
 * bls_server_submit, which copies the inputs and returns at once.  A
 * scheduler thread admits queued requests while device memory (points and
 * periods of the request arena) and slots are free, keeps every admitted
 * curve resident on the device, and issues persistent launches ("ticks")
 * that hold period tiles of all admitted requests at once: the oldest
 * requests get most of each tick, and every admitted request gets at least
 * one tile, so newly admitted work overlaps with work already running.  A
 * request's results are identical to those of bls_search on the same input.
 */
typedef struct bls_server bls_server;

typedef struct {
    int32_t device;
    int32_t max_slots;            /* requests resident on the device at once  */
    int64_t arena_bytes;          /* device bytes of resident requests at once
                                     (40 per point, 24 per trial period, any
                                     mix; twice this much is reserved)        */
    int32_t max_nbins;            /* <= BLS_MAX_NBINS                          */
    int32_t min_in_points;        /* as for a plan                             */
    uint32_t flags;               /* BLS_DIP_ONLY                              */
    int32_t reserved;
    double tick_cost;             /* work per launch, in point-period units
                                     (N*periods + 1.6*box evaluations); 0 = auto */
    int64_t max_request_points;   /* largest N accepted (<= 2^24)              */
    int64_t max_request_periods;  /* largest period grid accepted              */
} bls_server_config;

/* One request: host arrays, copied by bls_server_submit. */
typedef struct {
    const double *times;
    const double *flux;
    const double *weights;        /* NULL = unit weights */
    int64_t n;
    const double *periods;
    int64_t nperiods;
    int32_t nbins;
    int32_t reserved;
    double qmin;
    double qmax;
} bls_request;

/* A finished request.  The arrays belong to the server and stay valid
 * until bls_server_release(ticket).  They sit in the server's pinned result
 * pool when it had room for them (pageable memory otherwise, which costs
 * the scheduler a wait per request): releasing finished requests promptly
 * keeps later ones in the pool. */
typedef struct {
    int32_t status;               /* BLS_OK or the request's error             */
    int32_t reserved;
    int64_t nperiods;
    const float *sr;              /* [nperiods] SR                             */
    const float *depth;           /* [nperiods] depth (NaN: no box)            */
    const int32_t *jstart;        /* [nperiods] box start bin (-1: no box)     */
    const int32_t *kwidth;        /* [nperiods] box width in bins (-1: none)   */
    int64_t best_index;           /* first period with the largest SR          */
    double submit_s;              /* server clock (s since creation)           */
    double admit_s;
    double done_s;
} bls_result;

typedef struct {
    int64_t submitted, admitted, completed, failed, queued, active, ticks;
    double p50_ms, p99_ms, mean_ms, max_ms;  /* submit -> done, completed requests */
    double trial_points;          /* sum N*nperiods of completed requests      */
    double box_evals;             /* box evaluations of completed requests     */
    double busy_s;                /* device time of the launches               */
    double wall_s;                /* wall time since creation or reset         */
    int64_t device_bytes_in_use;
    int64_t device_bytes_peak;
} bls_server_stats;

/* Defaults: device 0, 256 slots, 4 GiB arena, max_nbins 4096, min_in_points
 * 1, no flags, automatic tick size, N <= 2^20, nperiods <= 2^20. */
void bls_server_config_init(bls_server_config *cfg);

/* Allocate the arena and start the scheduler thread.  Besides the device
 * arena the server pins host memory: a quarter of arena_bytes (at most 1 GiB)
 * to stage request inputs and half (at most 2 GiB) for finished requests'
 * results; where pinning fails it works from pageable memory.  Errors:
 * INVALID_ARG, NO_MEMORY, DEVICE (message via bls_server_last_error(NULL,
 * ...)). */
int bls_server_create(bls_server **out, const bls_server_config *cfg);

/* Queue a request; non-blocking; inputs are copied.  *ticket identifies it.
 * Errors (no ticket issued): INVALID_ARG (same checks as bls_search),
 * CAPACITY (larger than the limits or than the whole arena). */
int bls_server_submit(bls_server *srv, const bls_request *req, uint64_t *ticket);

/* BUSY while the request is queued or running; BLS_OK with *out filled when
 * done (out->status holds the request's own status); INVALID_ARG for an
 * unknown or released ticket. */
int bls_server_poll(bls_server *srv, uint64_t ticket, bls_result *out);

/* As poll, but waits up to timeout_s seconds (TIMEOUT if still running). */
int bls_server_wait(bls_server *srv, uint64_t ticket, bls_result *out,
                    double timeout_s);

/* Free a finished request's results; INVALID_ARG if unknown or not done. */
int bls_server_release(bls_server *srv, uint64_t ticket);

/* Counters and latency percentiles since creation or the last reset. */
int bls_server_get_stats(bls_server *srv, bls_server_stats *out);
int bls_server_reset_stats(bls_server *srv);

/* Wait until no request is queued or running (TIMEOUT after timeout_s). */
int bls_server_drain(bls_server *srv, double timeout_s);

/* Message of the server's last error (srv NULL: of bls_server_create). */
int bls_server_last_error(const bls_server *srv, char *buf, size_t len);

/* Stop the scheduler (waiting for running launches) and free everything.
 * NULL is accepted. */
int bls_server_destroy(bls_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* BLS_MI355X_H */
