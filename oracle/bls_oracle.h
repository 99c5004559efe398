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

#ifdef __cplusplus
}
#endif

#endif /* BLS_ORACLE_H */
