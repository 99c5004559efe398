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

/*
 * Detection statistics (signal detection efficiency of the cited BLS
 * statistic, plus alias-suppressed peaks); see bls_oracle.h for the rules.
 * Reading: the window is relative to the peak period, and the harmonic set
 * is fixed at 1/3, 1/2, 1, 2, 3.
 */
int bls_oracle_detect(const double *sr, const double *periods, int64_t m,
                      int32_t max_peaks, double window, double threshold,
                      double *mean, double *std, double *sde,
                      int64_t *peak_index, double *peak_sr, double *peak_sde,
                      int32_t *npeaks, int32_t *candidate)
{
    static const double harmonics[5] = {1.0, 0.5, 2.0, 1.0 / 3.0, 3.0};
    if (m < 1 || !sr || !periods || max_peaks < 0 || !(window >= 0.0))
        return BLS_ORACLE_INVALID;

    double sum = 0.0;
    for (int64_t p = 0; p < m; ++p)
        sum = sum + sr[p];
    double mu = sum / (double)m;
    double ss = 0.0;
    for (int64_t p = 0; p < m; ++p)
        ss = ss + (sr[p] - mu) * (sr[p] - mu);
    double sd = sqrt(ss / (double)m);
    double best = sr[0];
    for (int64_t p = 1; p < m; ++p)
        if (sr[p] > best)
            best = sr[p];
    double s = sd > 0.0 ? (best - mu) / sd : 0.0;

    unsigned char *off = (unsigned char *)calloc((size_t)m, 1);
    if (!off)
        return BLS_ORACLE_NOMEM;
    int32_t k = 0;
    while (k < max_peaks) {
        int64_t pk = -1;
        for (int64_t p = 0; p < m; ++p)
            if (!off[p] && sr[p] > 0.0 && (pk < 0 || sr[p] > sr[pk]))
                pk = p;
        if (pk < 0)
            break;
        peak_index[k] = pk;
        peak_sr[k] = sr[pk];
        peak_sde[k] = sd > 0.0 ? (sr[pk] - mu) / sd : 0.0;
        ++k;
        for (int64_t p = 0; p < m; ++p) {
            for (int h = 0; h < 5; ++h) {
                double c = harmonics[h] * periods[pk];
                if (fabs(periods[p] - c) <= window * c) {
                    off[p] = 1;
                    break;
                }
            }
        }
    }
    free(off);
    *mean = mu;
    *std = sd;
    *sde = s;
    *npeaks = k;
    *candidate = s >= threshold ? 1 : 0;
    return BLS_ORACLE_OK;
}

/*
 * Eclipse detection efficiency of an observing cadence (the simulation
 * behind the paper's detection-efficiency figure, section 5, Discussion and
 * conclusions: the chance that at least two eclipses of a binary of given
 * period fall on observations, given the real cadence with its daytime and
 * weather gaps).  Readings:
 *   W1  only the times matter; points with weight 0 are not observations
 *       (a NULL weight array keeps every point); t0 = min kept time;
 *   W2  eclipse epochs are a grid of nphase phase offsets j / nphase; the
 *       eclipse starting at offset j covers the k phase bins j .. j+k-1
 *       (modulo nphase) of the fold of reading R3 with nphase bins, where
 *       k = lround(duration * f * nphase) clamped to [1, nphase], f = 1/P;
 *   W3  a point of cycle E = floor(d f) in bin b lies in eclipse event E when
 *       b >= j and in event E - 1 when the window wrapped past the end of the
 *       cycle (b < j); an event is observed when at least one point lies in
 *       it;
 *   W4  observed[p] = number of offsets j with at least min_eclipses
 *       distinct observed events; the efficiency is observed[p] / nphase.
 * Events are counted here by sorting the event numbers of the in-eclipse
 * points of each offset; nothing is shared across offsets.
 */
static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int bls_oracle_eclipse_window(const double *t, const double *w, int64_t n,
                              const double *periods, int64_t nperiods,
                              int32_t nphase, double duration,
                              int32_t min_eclipses, int32_t nthreads,
                              int32_t *observed)
{
    if (!t || !periods || !observed || n < 1 || nperiods < 1 || nphase < 1 ||
        !(duration > 0.0) || !isfinite(duration) || min_eclipses < 1)
        return BLS_ORACLE_INVALID;
    for (int64_t p = 0; p < nperiods; ++p)
        if (!isfinite(periods[p]) || !(periods[p] > 0.0))
            return BLS_ORACLE_INVALID;
    int64_t m = 0;
    double t0 = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double wi = w ? w[i] : 1.0;
        if (!isfinite(wi) || wi < 0.0)
            return BLS_ORACLE_INVALID;
        if (wi == 0.0)
            continue;
        if (!isfinite(t[i]))
            return BLS_ORACLE_INVALID;
        if (t[i] < t0)
            t0 = t[i];
        ++m;
    }
    if (m < 1)
        return BLS_ORACLE_INVALID;
    double *d = (double *)malloc((size_t)m * sizeof(double));
    if (!d)
        return BLS_ORACLE_NOMEM;
    for (int64_t i = 0, k = 0; i < n; ++i)
        if (!w || w[i] != 0.0)
            d[k++] = t[i] - t0;

    int fail = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel reduction(| : fail)
#endif
    {
        int32_t *bin = (int32_t *)malloc((size_t)m * sizeof(int32_t));
        int64_t *cyc = (int64_t *)malloc((size_t)m * sizeof(int64_t));
        int64_t *ev = (int64_t *)malloc((size_t)m * sizeof(int64_t));
        if (!bin || !cyc || !ev)
            fail = 1;
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
        for (int64_t p = 0; p < nperiods; ++p) {
            if (fail)
                continue;
            double f = 1.0 / periods[p];
            long kw = lround(duration * f * (double)nphase);
            if (kw < 1)
                kw = 1;
            if (kw > nphase)
                kw = nphase;
            for (int64_t i = 0; i < m; ++i) {
                double c = d[i] * f;
                double e = floor(c);
                cyc[i] = (int64_t)e;
                bin[i] = phase_bin(d[i], f, nphase);
            }
            int32_t count = 0;
            for (int32_t j = 0; j < nphase; ++j) {
                int64_t ne = 0;
                for (int64_t i = 0; i < m; ++i) {
                    int32_t off = bin[i] - j;
                    if (off < 0)
                        off += nphase;
                    if (off < kw)
                        ev[ne++] = bin[i] >= j ? cyc[i] : cyc[i] - 1;
                }
                qsort(ev, (size_t)ne, sizeof(int64_t), cmp_i64);
                int64_t distinct = 0;
                for (int64_t q = 0; q < ne; ++q)
                    if (q == 0 || ev[q] != ev[q - 1])
                        ++distinct;
                if (distinct >= min_eclipses)
                    ++count;
            }
            observed[p] = count;
        }
        free(bin);
        free(cyc);
        free(ev);
    }
    free(d);
    return fail ? BLS_ORACLE_NOMEM : BLS_ORACLE_OK;
}

/*
 * High-variability pre-search (section 2.2.1, "High-variability source
 * searches"): the photometric stability expected at a star's magnitude is
 * a sigma-clipped average over the stars of the same chip in 0.1-mag bins;
 * stars more variable than that by more than 2 sigma are flagged.
 * Readings:
 *   V1  a star's stability is the population RMS about the mean of its kept
 *       values (weight > 0, NULL weights keep all), unweighted, in the
 *       values' own units; a star with no kept value, or a non-finite kept
 *       value or bad weight, is invalid (flag -1, in no bin);
 *   V2  its magnitude bin is floor((mag - origin) / width); stars whose bin
 *       falls outside [0, nmagbins), or whose magnitude is not finite, are in
 *       no bin (flag 0);
 *   V3  per (chip, bin) the clipped set starts as all member stars, in star
 *       order; a round takes the mean and population deviation of the set
 *       and drops every member farther than clip_sigma deviations from the
 *       mean (inclusive bounds keep a member exactly at the limit); rounds
 *       repeat until one drops nothing or max_iter rounds have dropped
 *       something; the bin's mean and deviation are those of the final set;
 *   V4  a member star is flagged when its stability exceeds the bin mean by
 *       more than flag_sigma deviations and the final set holds at least
 *       min_stars stars.
 */
static void mean_std(const double *v, int64_t n, double *mu, double *sd)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s = s + v[i];
    double m = s / (double)n;
    double ss = 0.0;
    for (int64_t i = 0; i < n; ++i)
        ss = ss + (v[i] - m) * (v[i] - m);
    *mu = m;
    *sd = sqrt(ss / (double)n);
}

int bls_oracle_variability(const double *x, const double *w,
                           const int64_t *n_off, int64_t ncurves,
                           const double *mag, const int64_t *chip_off,
                           int64_t nchips, double origin, double width,
                           int32_t nmagbins, double clip_sigma,
                           int32_t max_iter, double flag_sigma,
                           int32_t min_stars, double *rms, int32_t *bin,
                           int32_t *flag, double *bin_mean, double *bin_std,
                           int32_t *bin_count)
{
    if (!x || !n_off || !mag || !chip_off || ncurves < 1 || nchips < 1 ||
        nmagbins < 1 || !(width > 0.0) || !isfinite(origin) ||
        !isfinite(width) || !(clip_sigma > 0.0) || max_iter < 0 ||
        !(flag_sigma >= 0.0) || min_stars < 1 || n_off[0] != 0 ||
        chip_off[0] != 0 || chip_off[nchips] != ncurves)
        return BLS_ORACLE_INVALID;

    /* V1, V2: per star */
    for (int64_t c = 0; c < ncurves; ++c) {
        int64_t a = n_off[c], b = n_off[c + 1];
        int64_t m = 0;
        int bad = 0;
        double s = 0.0;
        for (int64_t i = a; i < b; ++i) {
            double wi = w ? w[i] : 1.0;
            if (!isfinite(wi) || wi < 0.0) {
                bad = 1;
                continue;
            }
            if (wi == 0.0)
                continue;
            if (!isfinite(x[i]))
                bad = 1;
            s = s + x[i];
            ++m;
        }
        flag[c] = 0;
        bin[c] = -1;
        if (bad || m == 0) {
            rms[c] = NAN;
            flag[c] = -1;
            continue;
        }
        double mu = s / (double)m;
        double ss = 0.0;
        for (int64_t i = a; i < b; ++i) {
            double wi = w ? w[i] : 1.0;
            if (wi == 0.0)
                continue;
            ss = ss + (x[i] - mu) * (x[i] - mu);
        }
        rms[c] = sqrt(ss / (double)m);
        if (isfinite(mag[c])) {
            double q = floor((mag[c] - origin) / width);
            if (q >= 0.0 && q < (double)nmagbins)
                bin[c] = (int32_t)q;
        }
    }

    /* V3, V4: per chip and bin */
    double *vals = (double *)malloc((size_t)ncurves * sizeof(double));
    double *next = (double *)malloc((size_t)ncurves * sizeof(double));
    if (!vals || !next) {
        free(vals);
        free(next);
        return BLS_ORACLE_NOMEM;
    }
    for (int64_t k = 0; k < nchips; ++k) {
        for (int32_t b = 0; b < nmagbins; ++b) {
            int64_t cnt = 0;
            for (int64_t c = chip_off[k]; c < chip_off[k + 1]; ++c)
                if (bin[c] == b && flag[c] >= 0)
                    vals[cnt++] = rms[c];
            int64_t slot = k * nmagbins + b;
            if (cnt == 0) {
                bin_mean[slot] = NAN;
                bin_std[slot] = NAN;
                bin_count[slot] = 0;
                continue;
            }
            double mu, sd;
            mean_std(vals, cnt, &mu, &sd);
            for (int32_t it = 0; it < max_iter; ++it) {
                int64_t kept = 0;
                for (int64_t i = 0; i < cnt; ++i)
                    if (vals[i] >= mu - clip_sigma * sd &&
                        vals[i] <= mu + clip_sigma * sd)
                        next[kept++] = vals[i];
                if (kept == cnt)
                    break;
                memcpy(vals, next, (size_t)kept * sizeof(double));
                cnt = kept;
                mean_std(vals, cnt, &mu, &sd);
            }
            bin_mean[slot] = mu;
            bin_std[slot] = sd;
            bin_count[slot] = (int32_t)cnt;
            if (cnt < min_stars)
                continue;
            for (int64_t c = chip_off[k]; c < chip_off[k + 1]; ++c)
                if (bin[c] == b && flag[c] >= 0 &&
                    rms[c] > mu + flag_sigma * sd)
                    flag[c] = 1;
        }
    }
    free(vals);
    free(next);
    return BLS_ORACLE_OK;
}

/*
 * Unbinned variant: box edges fall between data points instead of on a
 * phase-bin grid, so every subset of points that some box of duty cycle in
 * [qmin, qmax] can hold is tried (the range of durations and phases of
 * section 2.2.2 taken to the limit of the data, as in the unbinned form of
 * the cited statistic).  Readings, beyond R2, R3 (phase only, no bin), R5,
 * R6 and the statistic:
 *   U1  kept points are ordered by phase, ties by input order;
 *   U2  a box [a, a + q) of phase (cyclic) holds a cyclic run of m
 *       consecutive points of that order, 1 <= m <= n - 1, starting at
 *       sorted position r; with prev, first, last, next the positions
 *       r - 1, r, r + m - 1, r + m (mod n) and forward phase distances
 *       (one added when the step passes the end of the order), some box
 *       with q in [qmin, qmax] holds exactly that run iff
 *         dist(prev, first) > 0, dist(last, next) > 0,
 *         span = dist(first, last) < qmax and gap = dist(prev, next) > qmin
 *       (gap = 1 when prev and next are the same point);
 *   U3  the best box has the largest S^2/(R (W - R)); ties go to the
 *       smaller m, then the smaller r; first_point and last_point are the
 *       input indices of its first and last points (-1 if none).
 */
typedef struct {
    double ph;
    int64_t k;      /* index among kept points */
} ph_key;

static int cmp_ph(const void *a, const void *b)
{
    const ph_key *x = (const ph_key *)a, *y = (const ph_key *)b;
    if (x->ph < y->ph)
        return -1;
    if (x->ph > y->ph)
        return 1;
    return (x->k > y->k) - (x->k < y->k);
}

/* Forward phase distance from sorted position i to j (U2). */
static double fwd(const ph_key *o, int64_t i, int64_t j)
{
    if (j > i)
        return o[j].ph - o[i].ph;
    return (o[j].ph + 1.0) - o[i].ph;
}

int bls_oracle_unbinned(const double *t, const double *x, const double *w,
                        int64_t n, const double *periods, int64_t nperiods,
                        double qmin, double qmax, int32_t min_in_points,
                        int32_t dip_only, int32_t nthreads, double *sr,
                        double *depth, int32_t *first_point,
                        int32_t *last_point, int64_t *best_index)
{
    if (nperiods < 1 || periods == NULL || min_in_points < 1 ||
        !(qmin > 0.0) || !(qmax < 1.0) || !(qmin <= qmax))
        return BLS_ORACLE_INVALID;
    for (int64_t p = 0; p < nperiods; ++p)
        if (!isfinite(periods[p]) || !(periods[p] > 0.0))
            return BLS_ORACLE_INVALID;
    kept_curve kc;
    bls_oracle_prep pr;
    int st = prepare(t, x, w, n, &kc, &pr);
    if (st != BLS_ORACLE_OK)
        return st;
    const int64_t m = kc.n;
    int64_t *orig = (int64_t *)malloc((size_t)m * sizeof(int64_t));
    double *p_sr = (double *)malloc((size_t)nperiods * sizeof(double));
    if (!orig || !p_sr) {
        free(orig);
        free(p_sr);
        free_kept(&kc);
        return BLS_ORACLE_NOMEM;
    }
    for (int64_t i = 0, k = 0; i < n; ++i)
        if (!w || w[i] != 0.0)
            orig[k++] = i;
    int failed = 0;

#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        ph_key *o = (ph_key *)malloc((size_t)m * sizeof(ph_key));
        if (!o) {
#ifdef _OPENMP
#pragma omp atomic write
#endif
            failed = 1;
        }
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
        for (int64_t p = 0; p < nperiods; ++p) {
            if (!o)
                continue;
            double f = 1.0 / periods[p];
            for (int64_t i = 0; i < m; ++i) {
                double c = kc.d[i] * f;
                o[i].ph = c - floor(c);
                o[i].k = i;
            }
            qsort(o, (size_t)m, sizeof(ph_key), cmp_ph);
            double bv = 0.0, bS = 0.0, bR = 0.0;
            int64_t bm = -1, br = -1;
            for (int64_t r = 0; r < m; ++r) {
                int64_t prev = (r + m - 1) % m;
                if (!(fwd(o, prev, r) > 0.0))
                    continue;
                double R = 0.0, S = 0.0;
                for (int64_t len = 1; len <= m - 1; ++len) {
                    int64_t last = (r + len - 1) % m;
                    int64_t next = (r + len) % m;
                    int64_t q = o[last].k;
                    R = R + kc.w[q];
                    S = S + kc.w[q] * kc.y[q];
                    double span = len == 1 ? 0.0 : fwd(o, r, last);
                    if (!(span < qmax))
                        break;
                    if (!(fwd(o, last, next) > 0.0))
                        continue;
                    double gap = prev == next ? 1.0 : fwd(o, prev, next);
                    if (!(gap > qmin))
                        continue;
                    if (len < min_in_points)
                        continue;
                    if (dip_only && !(S < 0.0))
                        continue;
                    double den = R * (pr.W - R);
                    if (!(den > 0.0))
                        continue;
                    double v = (S * S) / den;
                    if (!(v > 0.0))
                        continue;
                    if (v > bv || (v == bv && (len < bm ||
                                               (len == bm && r < br)))) {
                        bv = v;
                        bS = S;
                        bR = R;
                        bm = len;
                        br = r;
                    }
                }
            }
            p_sr[p] = sqrt(bv);
            if (sr)
                sr[p] = p_sr[p];
            if (depth)
                depth[p] = bm < 0 ? NAN : -bS * pr.W / (bR * (pr.W - bR));
            if (first_point)
                first_point[p] = bm < 0 ? -1 : (int32_t)orig[o[br].k];
            if (last_point)
                last_point[p] =
                    bm < 0 ? -1 : (int32_t)orig[o[(br + bm - 1) % m].k];
        }
        free(o);
    }
    if (!failed && best_index) {
        int64_t bi = 0;
        for (int64_t p = 1; p < nperiods; ++p)
            if (p_sr[p] > p_sr[bi])
                bi = p;
        *best_index = bi;
    }
    free(orig);
    free(p_sr);
    free_kept(&kc);
    return failed ? BLS_ORACLE_NOMEM : BLS_ORACLE_OK;
}

/*
 * Injection of box eclipses into copies of one cadence, and the recovery
 * rule: the paper's detection-efficiency simulations (section 5, Discussion
 * and conclusions: eclipses of a binary of given period on the real
 * cadences) taken through the search itself.  Readings:
 *   I1  the phase origin is t0 = min kept time (weight > 0; all points with
 *       a NULL weight array), as for the search; d = t - t0;
 *   I2  injection i (period P, start phase phi in [0, 1), duty cycle q,
 *       depth delta) covers the points with frac(d / P - phi) < q, in the
 *       FP64 order f = 1/P, c = d f, u = c - phi, v = u - floor(u);
 *   I3  an injected point's flux is base - delta, every other point keeps
 *       base (dropped points too: the search ignores them);
 *   I4  an injection is recovered when its periodogram's detection
 *       statistic SDE is at least the threshold and its best period P_b
 *       (first period of largest SR) lies within ptol h P of h P for h in
 *       {1, 1/2, 2} (the injected period or its first aliases).
 */
int bls_oracle_inject(const double *t, const double *w, int64_t n,
                      const double *base, int32_t ninj, const double *period,
                      const double *phase, const double *q,
                      const double *depth, double *x)
{
    if (n < 1 || ninj < 1 || !t || !base || !period || !phase || !q ||
        !depth || !x)
        return BLS_ORACLE_INVALID;
    double t0 = INFINITY;
    int64_t kept = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (w && !(w[i] > 0.0))
            continue;
        if (t[i] < t0)
            t0 = t[i];
        ++kept;
    }
    if (kept == 0)
        return BLS_ORACLE_INVALID;
    for (int32_t k = 0; k < ninj; ++k) {
        const double f = 1.0 / period[k];
        const double *b = base + (int64_t)k * n;
        double *o = x + (int64_t)k * n;
        for (int64_t i = 0; i < n; ++i) {
            const int keep = !w || w[i] > 0.0;
            const double d = t[i] - t0;
            const double c = d * f;
            const double u = c - phase[k];
            const double v = u - floor(u);
            o[i] = (keep && v < q[k]) ? b[i] - depth[k] : b[i];
        }
    }
    return BLS_ORACLE_OK;
}

int bls_oracle_recovered(double best_period, double sde, double p_inj,
                         double sde_threshold, double ptol)
{
    if (!(sde >= sde_threshold))
        return 0;
    static const double h[3] = {1.0, 0.5, 2.0};
    for (int i = 0; i < 3; ++i) {
        const double target = h[i] * p_inj;
        if (fabs(best_period - target) <= ptol * target)
            return 1;
    }
    return 0;
}
