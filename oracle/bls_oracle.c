/*
 * FP64 CPU oracle for the binned BLS periodogram -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * build, load or call this file.  It shares no code, header, table or helper
 * with the GPU library.  Build: gcc -O2 -ffp-contract=off -fopenmp (no fast
 * math), so every multiply and add below is one correctly rounded IEEE
 * double operation in the order written.
 *
 * Source of the method: Law et al. 2011, section 2.2.2 ("A Parallel Eclipse
 * Search Using Graphics Processing Units").  The section applies a standard
 * box-least-squares search (it cites Kovacs, Zucker & Mazeh 2002 and Tingley
 * 2003 for the statistic) that phases each light curve at every trial period
 * and then tries a range of transit durations and phases.  The section gives
 * no formulas, so the statistic is restated here from its least-squares
 * meaning:
 *
 *   A box B is a set of phase bins.  Fitting x = H outside B and x = L inside
 *   B by weighted least squares gives L and H as the weighted means inside
 *   and outside.  With R = sum_{i in B} w_i, S = sum_{i in B} w_i (x_i - xbar)
 *   and W = sum_i w_i, the drop in chi^2 against a constant is
 *   W * S^2 / (R (W - R)); the signal residue is SR = sqrt(S^2/(R (W - R))).
 *   The fitted step is H - L = -S W / (R (W - R)) (positive for a dip).
 *
 * Readings where the paper is silent (each is also listed in the design
 * notes of the repository):
 *   R1  boxes are whole phase bins; nbins bins of equal width in phase;
 *   R2  reference epoch t0 = min time over kept points; d = t - t0;
 *   R3  phase = frac(d * f) with f = 1/P computed once per period; the bin
 *       is trunc(phase * nbins), clamped to nbins - 1;
 *   R4  widths kmin = max(1, lround(qmin nbins)) .. kmax = min(nbins - 1,
 *       lround(qmax nbins)); boxes may wrap from the last bin to the first;
 *   R5  points with weight 0 are dropped before anything else; a NULL weight
 *       array means unit weights; negative or non-finite weights, and
 *       non-finite times or fluxes of kept points, are invalid input;
 *   R6  a box is valid iff min_in_points <= (kept points inside) <= n - 1,
 *       R (W - R) > 0 and, in dip-only mode, S < 0;
 *   R7  only valid boxes with S^2/(R(W-R)) > 0 are candidates; the best is
 *       the largest value, exact ties going to the smaller width k, then the
 *       smaller start bin j; a period with no candidate has SR = 0,
 *       j = k = -1 and depth NaN;
 *   R8  best_index is the first period with the largest SR.
 */
#include "bls_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Kept points after step 1: their own arrays, in input order. */
typedef struct {
    int64_t n;
    double *d;  /* t - t0           */
    double *w;  /* weight           */
    double *y;  /* x - xbar         */
} kept_curve;

static void free_kept(kept_curve *kc)
{
    free(kc->d);
    free(kc->w);
    free(kc->y);
    kc->d = kc->w = kc->y = NULL;
}

/* Widths from the duty-cycle range (reading R4). */
static void width_range(int32_t nbins, double qmin, double qmax,
                        int32_t *kmin, int32_t *kmax)
{
    long lo = lround(qmin * (double)nbins);
    long hi = lround(qmax * (double)nbins);
    if (lo < 1) lo = 1;
    if (hi > nbins - 1) hi = nbins - 1;
    *kmin = (int32_t)lo;
    *kmax = (int32_t)hi;
}

/*
 * Steps 1-3: drop zero-weight points, check the rest, take the weighted
 * mean, centre the fluxes and measure times from the earliest kept point
 * (readings R2 and R5).  Plain sequential double sums.
 */
static int prepare(const double *t, const double *x, const double *w,
                   int64_t n, kept_curve *kc, bls_oracle_prep *prep)
{
    memset(kc, 0, sizeof(*kc));
    if (n < 0 || t == NULL || x == NULL)
        return BLS_ORACLE_INVALID;

    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        double wi = w ? w[i] : 1.0;
        if (!isfinite(wi) || wi < 0.0)
            return BLS_ORACLE_INVALID;
        if (wi == 0.0)
            continue;
        if (!isfinite(t[i]) || !isfinite(x[i]))
            return BLS_ORACLE_INVALID;
        ++m;
    }
    if (m < 2)
        return BLS_ORACLE_INVALID;

    kc->n = m;
    kc->d = (double *)malloc((size_t)m * sizeof(double));
    kc->w = (double *)malloc((size_t)m * sizeof(double));
    kc->y = (double *)malloc((size_t)m * sizeof(double));
    if (!kc->d || !kc->w || !kc->y) {
        free_kept(kc);
        return BLS_ORACLE_NOMEM;
    }

    double W = 0.0, wx = 0.0, t0 = INFINITY;
    int64_t k = 0;
    for (int64_t i = 0; i < n; ++i) {
        double wi = w ? w[i] : 1.0;
        if (wi == 0.0)
            continue;
        kc->w[k] = wi;
        kc->d[k] = t[i];     /* times for now; made relative below */
        kc->y[k] = x[i];     /* fluxes for now; centred below      */
        W = W + wi;
        wx = wx + wi * x[i];
        if (t[i] < t0)
            t0 = t[i];
        ++k;
    }
    if (!(W > 0.0) || !isfinite(W)) {
        free_kept(kc);
        return BLS_ORACLE_INVALID;
    }
    double xbar = wx / W;
    double sumwy2 = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        kc->d[i] = kc->d[i] - t0;
        kc->y[i] = kc->y[i] - xbar;
        sumwy2 = sumwy2 + kc->w[i] * kc->y[i] * kc->y[i];
    }
    if (prep) {
        prep->n = m;
        prep->t0 = t0;
        prep->W = W;
        prep->xbar = xbar;
        prep->sumwy2 = sumwy2;
    }
    return BLS_ORACLE_OK;
}

/* Reading R3: the phase bin of time offset d at frequency f = 1/P. */
static int32_t phase_bin(double d, double f, int32_t nbins)
{
    double c = d * f;
    double phase = c - floor(c);
    int32_t b = (int32_t)(phase * (double)nbins);
    if (b >= nbins)
        b = nbins - 1;
    return b;
}

/* Step 5: fold the kept points at one period and sum them per bin. */
static void fold_and_bin(const kept_curve *kc, double period, int32_t nbins,
                         double *hw, double *hs, int64_t *hn, int32_t *bins)
{
    double f = 1.0 / period;
    for (int32_t b = 0; b < nbins; ++b) {
        hw[b] = 0.0;
        hs[b] = 0.0;
        hn[b] = 0;
    }
    for (int64_t i = 0; i < kc->n; ++i) {
        int32_t b = phase_bin(kc->d[i], f, nbins);
        if (bins)
            bins[i] = b;
        hw[b] = hw[b] + kc->w[i];
        hs[b] = hs[b] + kc->w[i] * kc->y[i];
        hn[b] = hn[b] + 1;
    }
}

typedef struct {
    double v;       /* S^2 / (R (W - R)) of the best box, 0 if none */
    double S, R;
    int32_t j, k;   /* -1, -1 if none */
} box_best;

/*
 * Step 6: every start bin j and width k in [kmin, kmax], bins taken modulo
 * nbins (readings R4, R6, R7).  The window sums for one start are running
 * sums over its bins, never differences of prefix sums.
 */
static box_best scan_boxes(const double *hw, const double *hs,
                           const int64_t *hn, int32_t nbins, int32_t kmin,
                           int32_t kmax, int64_t n, double W,
                           int32_t min_in_points, int32_t dip_only)
{
    box_best best;
    best.v = 0.0;
    best.S = best.R = 0.0;
    best.j = best.k = -1;

    for (int32_t j = 0; j < nbins; ++j) {
        double R = 0.0, S = 0.0;
        int64_t nin = 0;
        for (int32_t m = 0; m < kmax; ++m) {
            int32_t b = (j + m) % nbins;
            R = R + hw[b];
            S = S + hs[b];
            nin = nin + hn[b];
            int32_t k = m + 1;
            if (k < kmin)
                continue;
            if (nin < min_in_points || nin > n - 1)
                continue;
            if (dip_only && !(S < 0.0))
                continue;
            double den = R * (W - R);
            if (!(den > 0.0))
                continue;
            double v = (S * S) / den;
            if (!(v > 0.0))
                continue;
            int better = 0;
            if (v > best.v)
                better = 1;
            else if (v == best.v) {
                if (k < best.k)
                    better = 1;
                else if (k == best.k && j < best.j)
                    better = 1;
            }
            if (better) {
                best.v = v;
                best.S = S;
                best.R = R;
                best.j = j;
                best.k = k;
            }
        }
    }
    return best;
}

int bls_oracle_search(const double *t, const double *x, const double *w,
                      int64_t n, const double *periods, int64_t nperiods,
                      int32_t nbins, double qmin, double qmax,
                      int32_t min_in_points, int32_t dip_only, int32_t nthreads,
                      double *sr, double *depth, int32_t *jstart,
                      int32_t *kwidth, int64_t *best_index,
                      bls_oracle_prep *prep)
{
    if (nperiods < 1 || periods == NULL || nbins < 2 || min_in_points < 1)
        return BLS_ORACLE_INVALID;
    if (!(qmin > 0.0) || !(qmax < 1.0) || !(qmin <= qmax))
        return BLS_ORACLE_INVALID;
    for (int64_t p = 0; p < nperiods; ++p)
        if (!isfinite(periods[p]) || !(periods[p] > 0.0))
            return BLS_ORACLE_INVALID;
    int32_t kmin, kmax;
    width_range(nbins, qmin, qmax, &kmin, &kmax);
    if (kmin > kmax)
        return BLS_ORACLE_INVALID;

    kept_curve kc;
    bls_oracle_prep pr;
    int st = prepare(t, x, w, n, &kc, &pr);
    if (st != BLS_ORACLE_OK)
        return st;
    pr.kmin = kmin;
    pr.kmax = kmax;

    double *p_sr = (double *)malloc((size_t)nperiods * sizeof(double));
    if (!p_sr) {
        free_kept(&kc);
        return BLS_ORACLE_NOMEM;
    }
    int failed = 0;

#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        double *hw = (double *)malloc((size_t)nbins * sizeof(double));
        double *hs = (double *)malloc((size_t)nbins * sizeof(double));
        int64_t *hn = (int64_t *)malloc((size_t)nbins * sizeof(int64_t));
        if (!hw || !hs || !hn) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        }
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 16)
#endif
        for (int64_t p = 0; p < nperiods; ++p) {
            if (!hw || !hs || !hn)
                continue;
            fold_and_bin(&kc, periods[p], nbins, hw, hs, hn, NULL);
            box_best b = scan_boxes(hw, hs, hn, nbins, kmin, kmax, kc.n,
                                    pr.W, min_in_points, dip_only);
            p_sr[p] = sqrt(b.v);
            if (sr)
                sr[p] = p_sr[p];
            if (jstart)
                jstart[p] = b.j;
            if (kwidth)
                kwidth[p] = b.k;
            if (depth)
                depth[p] = (b.k < 0) ? NAN
                                     : -b.S * pr.W / (b.R * (pr.W - b.R));
        }
        free(hw);
        free(hs);
        free(hn);
    }

    if (!failed) {
        /* Reading R8: first period with the largest SR. */
        int64_t bi = 0;
        for (int64_t p = 1; p < nperiods; ++p)
            if (p_sr[p] > p_sr[bi])
                bi = p;
        if (best_index)
            *best_index = bi;
        if (prep)
            *prep = pr;
    }
    free(p_sr);
    free_kept(&kc);
    return failed ? BLS_ORACLE_NOMEM : BLS_ORACLE_OK;
}

int64_t bls_oracle_bins(const double *t, const double *x, const double *w,
                        int64_t n, double period, int32_t nbins,
                        int32_t *bins, double *hw, double *hs, int64_t *hn)
{
    if (nbins < 2 || !isfinite(period) || !(period > 0.0))
        return BLS_ORACLE_INVALID;
    kept_curve kc;
    int st = prepare(t, x, w, n, &kc, NULL);
    if (st != BLS_ORACLE_OK)
        return st;
    double *lw = (double *)malloc((size_t)nbins * sizeof(double));
    double *ls = (double *)malloc((size_t)nbins * sizeof(double));
    int64_t *ln = (int64_t *)malloc((size_t)nbins * sizeof(int64_t));
    if (!lw || !ls || !ln) {
        free(lw);
        free(ls);
        free(ln);
        free_kept(&kc);
        return BLS_ORACLE_NOMEM;
    }
    fold_and_bin(&kc, period, nbins, lw, ls, ln, bins);
    if (hw)
        memcpy(hw, lw, (size_t)nbins * sizeof(double));
    if (hs)
        memcpy(hs, ls, (size_t)nbins * sizeof(double));
    if (hn)
        memcpy(hn, ln, (size_t)nbins * sizeof(int64_t));
    int64_t m = kc.n;
    free(lw);
    free(ls);
    free(ln);
    free_kept(&kc);
    return m;
}
