/*
 * FP64 CPU oracle for the binned box-least-squares (BLS) periodogram.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may build, load
 * or call it; the GPU library never includes, links or calls anything here,
 * and nothing here includes or calls the GPU library.
 *
 * What is computed (Law et al. 2011, section 2.2.2 "A Parallel Eclipse Search
 * Using Graphics Processing Units": every trial period is tried, the light
 * curve is phased at it, and a range of box durations and phases is tested;
 * the BLS statistic itself is the one of Kovacs et al. 2002 that the section
 * cites): for every trial period the weighted least-squares fit of a
 * two-level step function ("box") over phase bins, reported as the signal
 * residue SR = sqrt(S^2 / (R (W - R))) of the best box.
 *
 * Conventions that the paper leaves open are fixed in bls_oracle.c next to
 * the code that implements them.
 */
#ifndef BLS_ORACLE_H
#define BLS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    BLS_ORACLE_OK = 0,
    BLS_ORACLE_INVALID = -1,
    BLS_ORACLE_NOMEM = -2
};

/* Per-curve quantities of the preparation step (oracle step 1-4). */
typedef struct {
    int64_t n;      /* points kept (weight > 0)                      */
    double  t0;     /* reference epoch = min time over kept points    */
    double  W;      /* sum of weights                                 */
    double  xbar;   /* weighted mean flux                             */
    double  sumwy2; /* sum w (x - xbar)^2                             */
    int32_t kmin;   /* narrowest box, in bins                         */
    int32_t kmax;   /* widest box, in bins                            */
} bls_oracle_prep;

/*
 * Full periodogram of one light curve.
 *   t, x: [n] times and fluxes; w: [n] weights or NULL (unit weights).
 *   periods: [nperiods] trial periods (> 0).
 *   min_in_points: minimum kept points inside a valid box (>= 1).
 *   dip_only: non-zero => only boxes whose mean is below the rest count.
 *   nthreads: OpenMP threads over periods (<= 0: OpenMP default).
 * Outputs (any may be NULL), [nperiods] each: sr, depth, jstart, kwidth;
 * best_index: first period with the largest SR; prep: per-curve numbers.
 * Returns BLS_ORACLE_OK or BLS_ORACLE_INVALID (outputs untouched).
 */
int bls_oracle_search(const double *t, const double *x, const double *w,
                      int64_t n, const double *periods, int64_t nperiods,
                      int32_t nbins, double qmin, double qmax,
                      int32_t min_in_points, int32_t dip_only, int32_t nthreads,
                      double *sr, double *depth, int32_t *jstart,
                      int32_t *kwidth, int64_t *best_index,
                      bls_oracle_prep *prep);

/*
 * The phase bins and per-bin sums of one period (oracle step 5), over the
 * kept points in their input order.  bins: [n_kept]; hw, hs: [nbins] double;
 * hn: [nbins] int64.  Any output may be NULL.  Returns the number of kept
 * points, or BLS_ORACLE_INVALID.
 */
int64_t bls_oracle_bins(const double *t, const double *x, const double *w,
                        int64_t n, double period, int32_t nbins,
                        int32_t *bins, double *hw, double *hs, int64_t *hn);

/*
 * Detection statistics of one periodogram (the step after the search).
 *   sr, periods: [m]; the statistic is the signal detection efficiency of the
 *   BLS method the paper cites: SDE = (SR_max - mean SR) / std SR, with the
 *   mean and the population standard deviation over the m periods (SDE = 0
 *   when the deviation is 0).
 *   Peaks: up to max_peaks, each the largest SR among periods not yet
 *   suppressed (ties: smallest index); a peak at P* suppresses every period P
 *   with |P - h P*| <= window * h P* for h in {1, 1/2, 2, 1/3, 3}; the search
 *   stops early when no unsuppressed period has SR > 0.
 * Outputs: mean, std, sde; peak_index/peak_sr/peak_sde [max_peaks]; npeaks;
 * candidate = (sde >= threshold).
 */
int bls_oracle_detect(const double *sr, const double *periods, int64_t m,
                      int32_t max_peaks, double window, double threshold,
                      double *mean, double *std, double *sde,
                      int64_t *peak_index, double *peak_sr, double *peak_sde,
                      int32_t *npeaks, int32_t *candidate);

/*
 * Eclipse detection efficiency of an observing cadence (readings W1-W4 in
 * bls_oracle.c).  t: [n] times; w: [n] weights or NULL (weight 0 = not an
 * observation); periods: [nperiods]; nphase: trial eclipse epochs per period;
 * duration: eclipse length in the units of t; min_eclipses >= 1.
 * observed: [nperiods] output, the number of the nphase epochs for which at
 * least min_eclipses distinct eclipses fall on kept observations.
 */
int bls_oracle_eclipse_window(const double *t, const double *w, int64_t n,
                              const double *periods, int64_t nperiods,
                              int32_t nphase, double duration,
                              int32_t min_eclipses, int32_t nthreads,
                              int32_t *observed);

/*
 * High-variability pre-search (readings V1-V4 in bls_oracle.c).
 *   x, w: packed values and weights (w NULL = unit), n_off [ncurves + 1];
 *   mag: [ncurves] reference magnitudes; chip_off [nchips + 1]: the stars of
 *   chip k are [chip_off[k], chip_off[k+1]); magnitude bins of the given
 *   width from origin, nmagbins per chip.
 * Outputs: rms, bin, flag [ncurves]; bin_mean, bin_std, bin_count
 * [nchips * nmagbins] (mean and deviation NaN for an empty bin).
 */
int bls_oracle_variability(const double *x, const double *w,
                           const int64_t *n_off, int64_t ncurves,
                           const double *mag, const int64_t *chip_off,
                           int64_t nchips, double origin, double width,
                           int32_t nmagbins, double clip_sigma,
                           int32_t max_iter, double flag_sigma,
                           int32_t min_stars, double *rms, int32_t *bin,
                           int32_t *flag, double *bin_mean, double *bin_std,
                           int32_t *bin_count);

/*
 * Unbinned variant (readings U1-U3 in bls_oracle.c): boxes are the cyclic
 * runs of phase-sorted kept points that some box of duty cycle in
 * [qmin, qmax] holds exactly.  Inputs as bls_oracle_search without nbins.
 * Outputs [nperiods] (any may be NULL): sr, depth, first_point and
 * last_point (input indices of the best box's first and last points in
 * phase order, -1 if none); best_index as reading R8.
 */
int bls_oracle_unbinned(const double *t, const double *x, const double *w,
                        int64_t n, const double *periods, int64_t nperiods,
                        double qmin, double qmax, int32_t min_in_points,
                        int32_t dip_only, int32_t nthreads, double *sr,
                        double *depth, int32_t *first_point,
                        int32_t *last_point, int64_t *best_index);

/*
 * Box eclipses injected into copies of one cadence (readings I1-I3 in
 * bls_oracle.c).  t, w: [n] (w may be NULL); base: [ninj * n] fluxes before
 * injection, injection-major; period, phase, q, depth: [ninj].  x: [ninj * n]
 * output.  Returns BLS_ORACLE_OK, or BLS_ORACLE_INVALID (no kept point).
 */
int bls_oracle_inject(const double *t, const double *w, int64_t n,
                      const double *base, int32_t ninj, const double *period,
                      const double *phase, const double *q,
                      const double *depth, double *x);

/* Recovery rule I4: 1 when sde >= sde_threshold and best_period is within
 * ptol h p_inj of h p_inj for some h in {1, 1/2, 2}, else 0. */
int bls_oracle_recovered(double best_period, double sde, double p_inj,
                         double sde_threshold, double ptol);

#ifdef __cplusplus
}
#endif

#endif /* BLS_ORACLE_H */
