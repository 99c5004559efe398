// gfx950 kernels of the BLS periodogram (Law et al. 2011, section 2.2.2:
// phase each light curve at every trial period, then test a range of box
// durations and phases with the box-least-squares statistic it cites).
//
//   prep_kernel     one workgroup per curve: drop zero-weight points, t0,
//                   weighted mean, centring, fixed-point encoding (FP64)
//   search_kernel   persistent: each workgroup pulls (curve, period tile)
//                   items from a global counter; per item it folds the
//                   curve at T periods into exact LDS histograms (one 64-bit
//                   LDS atomic per point and period), turns them into FP32
//                   bins, scans every start bin x width with running window
//                   sums, and keeps the best box per period with a 64-bit
//                   LDS atomic max on (value, -index)
//   fill_kernel / best_index_kernel  counter and per-curve key set-up and
//                   read-out (plain kernels so that the sequence can be
//                   captured in a HIP graph)
//   unbinned_kernel box edges between points: per (curve, period) item the
//                   phases ordered in LDS and every run of consecutive points
//                   scored with exact sums
//   detect_kernel   one workgroup per periodogram: SR statistics in one pass
//                   and the strongest peaks with harmonic suppression, taken
//                   from per-thread candidate lists
//   window_prep_kernel / window_kernel  eclipse detection efficiency of a
//                   cadence: per (cadence, period tile) the smallest and
//                   largest cycle in each phase bin, then one decision per
//                   trial eclipse epoch
//   var_rms_kernel / var_clip_kernel  high-variability pre-search: per-star
//                   RMS, then per (chip, magnitude bin) clipped statistics
//                   and the flagged stars
//
// No FP contraction anywhere (-ffp-contract=off): the phase is computed with
// exactly the FP64 operation sequence of its definition so that every point
// falls into the same bin as in an FP64 evaluation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "bls_device.h"
#include "../../include/bls.h"

namespace bls {
namespace {

// ------------------------------------------------------------------ prep
__device__ inline void block_sum2(double &a, double &b, double *sa, double *sb) {
  const int tid = threadIdx.x;
  sa[tid] = a;
  sb[tid] = b;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      sa[tid] = sa[tid] + sa[tid + s];
      sb[tid] = sb[tid] + sb[tid + s];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
  __syncthreads();
}

// Count, mean and sum of squared deviations of the workgroup's values from
// each thread's own (n, mean, m2), merged pairwise in a fixed tree (the
// update of Chan, Golub and LeVeque); threads without values hold n = 0.
__device__ inline void block_chan(double &n, double &mean, double &m2, double *sa, double *sb,
                                  double *sc) {
  const int tid = threadIdx.x;
  sa[tid] = n;
  sb[tid] = mean;
  sc[tid] = m2;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const double na = sa[tid], nb = sa[tid + s];
      if (nb > 0.0) {
        if (na > 0.0) {
          const double nn = na + nb;
          const double delta = sb[tid + s] - sb[tid];
          const double fb = nb / nn;
          sb[tid] = sb[tid] + delta * fb;
          sc[tid] = sc[tid] + sc[tid + s] + delta * delta * na * fb;
          sa[tid] = nn;
        } else {
          sa[tid] = nb;
          sb[tid] = sb[tid + s];
          sc[tid] = sc[tid + s];
        }
      }
    }
    __syncthreads();
  }
  n = sa[0];
  mean = sb[0];
  m2 = sc[0];
  __syncthreads();
}

__device__ inline void block_minmax(double &mn, double &mx, double *sa, double *sb) {
  const int tid = threadIdx.x;
  sa[tid] = mn;
  sb[tid] = mx;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      sa[tid] = fmin(sa[tid], sa[tid + s]);
      sb[tid] = fmax(sb[tid], sb[tid + s]);
    }
    __syncthreads();
  }
  mn = sa[0];
  mx = sb[0];
  __syncthreads();
}

__device__ inline void block_isum2(long long &a, long long &b, long long *sa, long long *sb) {
  const int tid = threadIdx.x;
  sa[tid] = a;
  sb[tid] = b;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      sa[tid] += sa[tid + s];
      sb[tid] += sb[tid + s];
    }
    __syncthreads();
  }
  a = sa[0];
  b = sb[0];
  __syncthreads();
}

// Exponent e with |v| 2^e < 2^bits for every |v| <= m (0 if m == 0).
__device__ inline int scale_exponent(double m, int bits) {
  if (!(m > 0.0)) return 0;
  int ex;
  frexp(m, &ex);  // m = f 2^ex, f in [0.5, 1)
  return bits - ex;
}

__global__ __launch_bounds__(kBlock) void prep_kernel(PrepArgs a) {
  __shared__ double sa[kBlock];
  __shared__ double sb[kBlock];
  __shared__ long long ia[kBlock];
  __shared__ long long ib[kBlock];

  const int c = blockIdx.x;
  if (c >= a.ncurves) return;
  CurveDesc *cd = a.curves + c;
  const int64_t off = cd->n_off;
  const int64_t n = cd->n;
  const int qbits = cd->qbits;
  const bool weighted = a.w != nullptr;
  const int tid = threadIdx.x;

  // Pass 1: validity, kept count, t0, sum w, sum w x.
  long long cnt = 0, bad = 0;
  double tmin = INFINITY, sw = 0.0, swx = 0.0;
  for (int64_t i = tid; i < n; i += kBlock) {
    const double wi = weighted ? a.w[off + i] : 1.0;
    if (!(wi >= 0.0) || isinf(wi)) {
      bad = 1;
      continue;
    }
    if (wi == 0.0) continue;
    const double ti = a.t[off + i];
    const double xi = a.x[off + i];
    if (!isfinite(ti) || !isfinite(xi)) {
      bad = 1;
      continue;
    }
    ++cnt;
    tmin = fmin(tmin, ti);
    sw = sw + wi;
    swx = swx + wi * xi;
  }
  // Trial periods of this curve (device-side inputs are checked here).
  long long badp = 0, unused0 = 0;
  if (cd->check_periods) {
    for (int64_t i = tid; i < cd->nperiods; i += kBlock) {
      const double P = a.periods[cd->p_off + i];
      if (!isfinite(P) || !(P > 0.0)) badp = 1;
    }
  }
  block_isum2(badp, unused0, ia, ib);
  block_isum2(cnt, bad, ia, ib);
  block_sum2(sw, swx, sa, sb);
  double tmax_unused = -INFINITY;
  block_minmax(tmin, tmax_unused, sa, sb);

  if (badp != 0 || bad != 0 || cnt < 2 || !(sw > 0.0) || !isfinite(sw)) {
    if (tid == 0) {
      cd->status = badp ? kCurveBadPeriod : bad ? kCurveBadData : kCurveTooFew;
      cd->n_eff = (int32_t)cnt;
    }
    // zero the encoded points so that no kernel reads garbage
    for (int64_t i = tid; i < n; i += kBlock) {
      a.dt[off + i] = 0.0;
      a.q[off + i] = 0;
      if (weighted) a.qw[off + i] = -1;
    }
    return;
  }
  const double W = weighted ? sw : (double)cnt;
  const double xbar = swx / sw;

  // Cadence: the lower median of 64 gaps between consecutive input times,
  // sampled evenly along the curve (the fold spaces its lanes by it; any
  // value is correct, a good one only makes the fold faster).
  if (tid < 64) {
    const int64_t i = (int64_t)tid * (n - 1) / 64;
    float g = fabsf((float)(a.t[off + i + 1] - a.t[off + i]));
    if (!isfinite(g)) g = INFINITY;
    int rank = 0;
    for (int k = 0; k < 64; ++k) {
      const float o = __shfl(g, k, 64);
      rank += (o < g) || (o == g && k < tid);
    }
    if (rank == 31) cd->cadence = g;
  }

  // Pass 2: largest |w (x - xbar)| and largest w, for the fixed-point scales.
  double my = 0.0, mw = 0.0;
  for (int64_t i = tid; i < n; i += kBlock) {
    const double wi = weighted ? a.w[off + i] : 1.0;
    if (wi == 0.0) continue;
    const double yi = a.x[off + i] - xbar;
    const double v = weighted ? wi * yi : yi;
    my = fmax(my, fabs(v));
    mw = fmax(mw, wi);
  }
  double dummy = 0.0;
  block_minmax(dummy, my, sa, sb);
  dummy = 0.0;
  block_minmax(dummy, mw, sa, sb);
  const int es = scale_exponent(my, qbits);
  const int ew = weighted ? scale_exponent(mw, qbits) : qbits;

  // Pass 3: encode; exact totals of the encoded weights and values.
  long long sqw = 0, sq = 0;
  for (int64_t i = tid; i < n; i += kBlock) {
    const double wi = weighted ? a.w[off + i] : 1.0;
    if (wi == 0.0) {
      a.dt[off + i] = 0.0;
      a.q[off + i] = 0;
      if (weighted) a.qw[off + i] = -1;
      continue;
    }
    const double yi = a.x[off + i] - xbar;
    const double v = weighted ? wi * yi : yi;
    a.dt[off + i] = a.t[off + i] - tmin;
    const int qi = __double2int_rn(ldexp(v, es));
    a.q[off + i] = qi;
    sq += qi;
    if (weighted) {
      const int qwi = __double2int_rn(ldexp(wi, ew));
      a.qw[off + i] = qwi;
      sqw += qwi;
    }
  }
  block_isum2(sqw, sq, ia, ib);

  if (tid == 0) {
    cd->t0 = tmin;
    cd->W = W;
    cd->xbar = xbar;
    cd->es = es;
    cd->ew = ew;
    cd->out_scale = ldexp(1.0, ew - es);
    cd->Wf = weighted ? (float)ldexp((double)sqw, -qbits) : (float)cnt;
    // |sums| < 2^53, so both totals are exact in FP64
    cd->Wtot = weighted ? ldexp((double)sqw, -qbits) : (double)cnt;
    cd->Stot = ldexp((double)sq, -qbits);
    cd->n_eff = (int32_t)cnt;
    cd->status = kCurveOk;
  }
}

// ---------------------------------------------------------------- search
// One bin word holds (count << shift) + sum of signed fixed-point values.
// |sum| < 2^46 < 2^(shift - 1), so the sum is the sign-extended low field
// and the count is what remains above it.
struct BinWord {
  long long sum;
  unsigned count;
};

__device__ inline BinWord decode_word(unsigned long long u, int shift) {
  BinWord w;
  const int hi = 64 - shift;
  w.sum = ((long long)(u << hi)) >> hi;
  // a negative sum borrowed one from the count field
  w.count = (unsigned)(u >> shift) - (unsigned)(w.sum >> 63);
  return w;
}

// Correctly rounded float of an integer with |v| < 2^47: both halves convert
// exactly and the fused multiply-add rounds once.
__device__ inline float int47_to_float(long long v) {
  const int hi = (int)(v >> 24);
  const unsigned lo = (unsigned)v & 0xFFFFFFu;
  return fmaf((float)hi, 16777216.0f, (float)lo);
}

// trunc(frac(d f) nbins) with the FP64 operation order of the definition.
// For finite c >= 0, c - floor(c) is exact and below 1, so v_fract_f64
// returns exactly that value.  The result lies in [0, nbins]; nbins itself
// (phase so close to 1 that the product rounds up) is the clamp case of the
// definition.
__device__ inline int raw_bin(double d, double f, double nbd) {
  const double c = d * f;
  const double ph = __builtin_amdgcn_fract(c);
  return (int)(ph * nbd);
}

__device__ inline int phase_bin(double d, double f, double nbd, unsigned nbm1) {
  return (int)min((unsigned)raw_bin(d, f, nbd), nbm1);
}

// A 64-bit value every lane holds alike, moved to scalar registers.
__device__ inline int64_t uniform_i64(int64_t v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((uint64_t)v & 0xFFFFFFFFu));
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Lane spacing of the fold for one work item, in units of kPPT points:
// 1, 2 or 4 (a chunk is kBlock / 64 = 4 waves of 64 lanes).  On a dense
// cadence, points close in time fall into one bin at long periods, and
// lanes of one LDS atomic on the same word are serialised.  The gap is
// the smallest that puts adjacent lanes half a bin apart in phase at the
// tile's longest period (fmin = its smallest frequency); cadence is the
// curve's median time step.  Where lanes are that far apart already, the
// contiguous layout (gap 1) is the faster one.
static_assert(kBlock == 256 && kPPT == 4, "the fold's lane layout assumes 4 waves of 4 points");

__device__ inline int fold_lane_gap(double fmin, int nbins, float cadence) {
  // x = (lane step in time) / (bin width in time at the longest period)
  const double x = fmin * (double)nbins * (double)kPPT * (double)cadence;
  return !(x < 0.5) || !(x > 0.0) ? 1 : x >= 0.25 ? 2 : 4;
}

// Whether a tile's fold merges a thread's consecutive same-bin points: when
// one cadence step advances the phase by less than a bin at the tile's
// longest period (frequency fmin), unless the launch fixes the choice
// (policy 1: always, 2: never).  Any answer is correct; this one only picks
// the faster fold.
__device__ inline bool fold_merges(double fmin, int nbins, float cadence, int policy) {
  if (policy != 0) return policy == 1;
  const double x = fmin * (double)nbins * (double)cadence;
  return !(x >= 1.0);
}

// Fold and bin one chunk of kBlock * kPPT points into the tile's histograms.
// Each thread takes kPPT consecutive points, so the 64 lanes of one atomic
// instruction hold points kPPT apart in time: their phases (hence bins and
// LDS banks) are far less correlated than those of 64 consecutive points of
// a sorted light curve, which cuts same-bin and same-bank collisions.
// Each period's histogram plane starts HS words after the previous one: nb
// bins, the word after them (it catches the clamp case and is added to bin
// nb - 1 when the histogram is decoded, later the start of the wrap-around
// copy), and padding that keeps the scan's reads free of bank conflicts.
// Weighted curves use two such planes per period, A (count, weight) then B
// (weighted signal), each contiguous so that the lanes of one atomic spread
// over all LDS banks.
// MERGE: consecutive points of a thread that share a bin are summed first;
// without it every point is one atomic (tiles whose periods are short
// against the cadence, where neighbours almost never share a bin).
template <bool WEIGHTED, bool FULL, bool MERGE>
__device__ inline void fold_chunk(const SearchArgs &a, const CurveDesc &cd, int64_t base,
                                  int np, const double *s_f, unsigned long long *s_hist,
                                  int HS, int gap) {
  const int tid = threadIdx.x;
  // The chunk's first point and the points left from there, kept in scalar
  // registers.
  const int64_t off = uniform_i64(cd.n_off + base);
  const int64_t left = uniform_i64(cd.n - base);
  // Each thread takes kPPT consecutive points; the lanes of a wave are
  // kPPT gap points apart and the waves interleave (gap 1, 2 or 4).  The
  // gap passes through an opaque copy so that the compiler recomputes this
  // per chunk instead of holding it in VGPRs through the item.
  asm volatile("" : "+s"(gap));
  const int w = tid >> 6, l = tid & 63;
  const int k0 = kPPT * (l * gap + (w & (gap - 1))) + 64 * kPPT * gap * (w >> (gap >> 1));
  const double *dt = a.dt + off;
  const int32_t *q = a.q + off;
  const int32_t *qw = WEIGHTED ? a.qw + off : nullptr;
  const double nbd = (double)cd.nbins;
  const unsigned long long one = 1ull << cd.shift;
  double d[kPPT];
  unsigned long long va[kPPT];
  unsigned long long vb[kPPT];
  bool ok[kPPT];
#pragma unroll
  for (int r = 0; r < kPPT; ++r) {
    const int k = k0 + r;
    ok[r] = FULL || (int64_t)k < left;
    d[r] = 0.0;
    va[r] = 0;
    vb[r] = 0;
    if (ok[r]) {
      d[r] = dt[k];
      const long long qi = q[k];
      if (WEIGHTED) {
        const int qwi = qw[k];
        va[r] = qwi >= 0 ? one + (unsigned long long)(long long)qwi : 0ull;
        vb[r] = (unsigned long long)qi;
      } else {
        va[r] = one + (unsigned long long)qi;
      }
    }
  }
  constexpr int wpb = WEIGHTED ? 2 : 1;
  for (int t = 0; t < np; ++t) {
    const double f = s_f[t];
    unsigned long long *h = s_hist + (size_t)t * HS * wpb;
    // A thread's consecutive points that share a bin (common at long
    // periods) are summed in registers and sent as one atomic.
    int bin[kPPT];
#pragma unroll
    for (int r = 0; r < kPPT; ++r) bin[r] = raw_bin(d[r], f, nbd);
    if (!MERGE) {
#pragma unroll
      for (int r = 0; r < kPPT; ++r) {
        if (FULL || ok[r]) {
          __hip_atomic_fetch_add(h + bin[r], va[r], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
          if (WEIGHTED)
            __hip_atomic_fetch_add(h + HS + bin[r], vb[r], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        }
      }
      continue;
    }
    unsigned long long accA = 0, accB = 0;
#pragma unroll
    for (int r = 0; r < kPPT; ++r) {
      if (FULL || ok[r]) {
        accA += va[r];
        if (WEIGHTED) accB += vb[r];
        const int rn = r + 1 < kPPT ? r + 1 : r;
        const bool run_ends = r == kPPT - 1 || !(FULL || ok[rn]) || bin[rn] != bin[r];
        if (run_ends) {
          __hip_atomic_fetch_add(h + bin[r], accA, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          if (WEIGHTED)
            __hip_atomic_fetch_add(h + HS + bin[r], accB, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
          accA = 0;
          accB = 0;
        }
      }
    }
  }
}

// Exact test of one box against a lane's best (bn, bd): divide-free
// comparison v > v_best, validity on exact counts, dip-only sign.
template <bool WEIGHTED, bool DIP, bool MIP1>
__device__ __forceinline__ void consider(float R, float S, float C, float d, int m, float nmax1,
                                         float mipf, float &bn, float &bd, int &bm) {
  const float num = S * S;
  const float den = R * d;
  bool ok = num * bd > bn * den;
  if (WEIGHTED) {
    ok = ok & (C <= nmax1) & (C >= mipf) & (den > 0.0f);
  } else {
    ok = ok & (d >= 1.0f);  // at least one point outside the box
    if (!MIP1) ok = ok & (R >= mipf);
  }
  if (DIP) ok = ok & (S < 0.0f);
  if (ok) {
    bn = num;
    bd = den;
    bm = m;
  }
}

// One lane task, unit weights: every width kmin..kmax from start bin j (h
// points at bin j of the period's histogram; the wrap-around copy follows
// the last bin).  Counts are exact integers in FP32, so d = W - R is kept by
// subtraction.  Widths are screened four at a time against theta: a box
// beats theta only if S^2 >= theta R d, and over four consecutive widths
// R d = R (W - R) is concave in the growing R, so its least value is at the
// first or the last of the four, while S^2 is at most the largest of the
// four |S|^2.  A group passing that bound is taken again box by box, each
// box screened alone and, if it passes, given the exact test.
template <bool DIP, bool MIP1>
__device__ __forceinline__ void scan_task_unit(const float2 *h, int kmin, int kmax, float Wf,
                                               float thr, float mipf, float &bn, float &bd,
                                               int &bm) {
  float d = Wf, S = 0.0f;
  int m = 0;
  for (; m < kmin - 1; ++m) {
    const float2 e = h[m];
    d -= e.x;
    S += e.y;
  }
  bn = 0.0f;
  bd = 1.0f;
  bm = -1;
  for (; m + 4 <= kmax; m += 4) {
    const float2 e0 = h[m], e1 = h[m + 1], e2 = h[m + 2], e3 = h[m + 3];
    const float d0 = d - e0.x, S0 = S + e0.y;
    const float d1 = d0 - e1.x, S1 = S0 + e1.y;
    const float d2 = d1 - e2.x, S2 = S1 + e2.y;
    const float d3 = d2 - e3.x, S3 = S2 + e3.y;
    const float sm = fmaxf(fmaxf(fabsf(S0), fabsf(S1)), fmaxf(fabsf(S2), fabsf(S3)));
    const float g = fminf((Wf - d0) * d0, (Wf - d3) * d3);
    if (sm * sm >= thr * g) {
      // Rare: the four boxes again from the group's start, in the same
      // operations (so the same values).
      float dd = d, SS = S;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float2 e = h[m + i];
        dd -= e.x;
        SS += e.y;
        const float R = Wf - dd;
        if (SS * SS >= thr * (R * dd))
          consider<false, DIP, MIP1>(R, SS, 0.f, dd, m + i, 0.f, mipf, bn, bd, bm);
      }
    }
    d = d3;
    S = S3;
  }
  for (; m < kmax; ++m) {
    const float2 e = h[m];
    d -= e.x;
    S += e.y;
    const float R = Wf - d;
    if (S * S >= thr * (R * d)) consider<false, DIP, MIP1>(R, S, 0.f, d, m, 0.f, mipf, bn, bd, bm);
  }
}

// Exact test of one weighted box that passed the screen.  Its point count,
// needed only for the validity test, is summed here from the count bins
// (hc) rather than carried through the scan; without need_counts (no box
// can hold every point and one point makes a box valid) R (W - R) > 0
// alone decides validity.
template <bool DIP>
__device__ __forceinline__ void consider_w(float R, float S, float d, int m, const float2 *hc,
                                           bool need_counts, float nmax1, float mipf, float &bn,
                                           float &bd, int &bm) {
  const float num = S * S;
  const float den = R * d;
  bool ok = (num * bd > bn * den) & (den > 0.0f);
  if (DIP) ok = ok & (S < 0.0f);
  if (ok && need_counts) {
    float C = 0.0f;
    for (int i = 0; i <= m; ++i) C += hc[i].x;
    ok = (C <= nmax1) & (C >= mipf);
  }
  if (ok) {
    bn = num;
    bd = den;
    bm = m;
  }
}

// One lane task, weighted curves.  R is a running sum of the box's weight
// (positive terms, so its relative error stays within k roundings) and
// d = W - R is formed per box.  The screen is that of unit weights: R (W - R)
// is concave in the growing R, so four consecutive widths are bounded by
// the larger |S| of the four and the smaller R (W - R) of the first and the
// last (ha: the period's (R, S) bins from start j; hc: their counts in .x,
// read only for boxes that pass).
template <bool DIP>
__device__ __forceinline__ void scan_task_weighted(const float2 *ha, const float2 *hc, int kmin,
                                                   int kmax, float Wf, float thr, float nmax1,
                                                   float mipf, bool need_counts, float &bn,
                                                   float &bd, int &bm) {
  float R = 0.0f, S = 0.0f;
  int m = 0;
  for (; m < kmin - 1; ++m) {
    const float2 e = ha[m];
    R += e.x;
    S += e.y;
  }
  bn = 0.0f;
  bd = 1.0f;
  bm = -1;
  for (; m + 4 <= kmax; m += 4) {
    const float2 e0 = ha[m], e1 = ha[m + 1], e2 = ha[m + 2], e3 = ha[m + 3];
    const float R0 = R + e0.x, S0 = S + e0.y;
    const float R1 = R0 + e1.x, S1 = S0 + e1.y;
    const float R2 = R1 + e2.x, S2 = S1 + e2.y;
    const float R3 = R2 + e3.x, S3 = S2 + e3.y;
    const float sm = fmaxf(fmaxf(fabsf(S0), fabsf(S1)), fmaxf(fabsf(S2), fabsf(S3)));
    const float g = fminf(R0 * (Wf - R0), R3 * (Wf - R3));
    if (sm * sm >= thr * g) {
      float RR = R, SS = S;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float2 e = ha[m + i];
        RR += e.x;
        SS += e.y;
        const float dd = Wf - RR;
        if (SS * SS >= thr * (RR * dd))
          consider_w<DIP>(RR, SS, dd, m + i, hc, need_counts, nmax1, mipf, bn, bd, bm);
      }
    }
    R = R3;
    S = S3;
  }
  for (; m < kmax; ++m) {
    const float2 e = ha[m];
    R += e.x;
    S += e.y;
    const float d = Wf - R;
    if (S * S >= thr * (R * d)) consider_w<DIP>(R, S, d, m, hc, need_counts, nmax1, mipf, bn, bd, bm);
  }
}

// Boxes wider than half the bins, evaluated through their complement: the
// k' = nb - k bins that follow the box.  A wide box's own sums cancel (the
// values are centred), so its signal is taken as Stot - S' from the exact
// total and the complement's short running sum, its weight as W - R', and
// the weight outside it is R'.  One lane task is complement start j1 with
// widths k' = k1lo .. k1hi, i.e. boxes (j1 + k' mod nb, nb - k').  Exact
// ties go to the smaller k, i.e. the larger k', hence >= along the task.
// Returns the task's best key (0 if none).  h: (R, S) bins from j1; hc:
// their counts in .x (weighted curves; unit weights count in .x of h).
template <bool WEIGHTED, bool DIP>
__device__ inline unsigned long long scan_task_complement(const float2 *h, const float2 *hc,
                                                          int j1, int k1lo, int k1hi, int nb,
                                                          float Wf, float Stot, float neff,
                                                          float mipf) {
  float R1 = 0.0f, S1 = 0.0f, C1 = 0.0f;
  float bn = 0.0f, bd = 1.0f;
  int bk = -1;
  for (int m = 0; m < k1hi; ++m) {
    const float2 e = h[m];
    R1 += e.x;
    S1 += e.y;
    if (WEIGHTED) C1 += hc[m].x;
    if (m + 1 < k1lo) continue;
    const float Sin = Stot - S1;
    const float num = Sin * Sin;
    const float den = (Wf - R1) * R1;
    // points in the box: neff - (points outside), at least mip, at most neff - 1
    const float cout = WEIGHTED ? C1 : R1;
    bool ok = (num > 0.0f) & (den > 0.0f) & (num * bd >= bn * den) & (cout >= 1.0f) &
              (neff - cout >= mipf);
    if (DIP) ok = ok & (Sin < 0.0f);
    if (ok) {
      bn = num;
      bd = den;
      bk = m + 1;
    }
  }
  if (bk < 0) return 0ull;
  const int k = nb - bk;
  const int j = j1 + bk >= nb ? j1 + bk - nb : j1 + bk;
  const float v = bn * __builtin_amdgcn_rcpf(bd);
  const unsigned idx = __umul24((unsigned)k, (unsigned)nb) + (unsigned)j;
  return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(0xFFFFFFFFu - idx);
}

// Key of a lane's best box: its value (any consistent rounding; exact ties
// compare equal), then the smaller width and start.
__device__ __forceinline__ unsigned long long box_key(float bn, float bd, int bm, int j, int nb) {
  const float v = bn * __builtin_amdgcn_rcpf(bd);
  const unsigned idx = __umul24((unsigned)(bm + 1), (unsigned)nb) + (unsigned)j;
  return ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(0xFFFFFFFFu - idx);
}

// Seed of a weighted curve's per-period best before the scan: kSeeds boxes
// of width kmin with start bins spread over the period (a box may run into
// the wrap-around copy), each evaluated as a lane task evaluates it: the same
// sums in the same order, the same validity test and the same key.  Without
// it the first round of lane tasks screens against zero and sends every box
// to the exact test, whose count sums make that costly for weighted curves.
// Seed keys are keys of valid boxes, so the period's largest key stands.
constexpr int kSeeds = 32;

template <bool DIP>
__device__ inline void seed_best_weighted(const unsigned long long *s_hist,
                                          unsigned long long *s_best, const int *s_nonempty,
                                          int np, int nb, int HS, int kmin, int kmax, float Wf,
                                          float nmax1, float mipf, bool mip1) {
  for (int q = threadIdx.x; q < np * kSeeds; q += kBlock) {
    const int t = q / kSeeds;
    const int j = (int)(__umul24((unsigned)(q % kSeeds), (unsigned)nb) / kSeeds);
    const float2 *h =
        reinterpret_cast<const float2 *>(s_hist) + __umul24((unsigned)t, (unsigned)(2 * HS)) + j;
    float R = 0.0f, S = 0.0f;
    for (int i = 0; i < kmin; ++i) {
      const float2 e = h[i];
      R += e.x;
      S += e.y;
    }
    float bn = 0.0f, bd = 1.0f;
    int bm = -1;
    const bool need_counts = !(mip1 && s_nonempty[t] > kmax);
    consider_w<DIP>(R, S, Wf - R, kmin - 1, h + HS, need_counts, nmax1, mipf, bn, bd, bm);
    if (bm >= 0)
      __hip_atomic_fetch_max(&s_best[t], box_key(bn, bd, bm, j, nb), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// The same seed for unit weights: kSeeds boxes of width kmin, each summed
// and tested exactly as a lane task sums and tests it (d by subtraction
// from W, S by addition, in bin order).
template <bool DIP, bool MIP1>
__device__ inline void seed_best_unit(const unsigned long long *s_hist,
                                      unsigned long long *s_best, int np, int nb, int HS,
                                      int kmin, float Wf, float mipf) {
  for (int q = threadIdx.x; q < np * kSeeds; q += kBlock) {
    const int t = q / kSeeds;
    const int j = (int)(__umul24((unsigned)(q % kSeeds), (unsigned)nb) / kSeeds);
    const float2 *h =
        reinterpret_cast<const float2 *>(s_hist) + __umul24((unsigned)t, (unsigned)HS) + j;
    float d = Wf, S = 0.0f;
    for (int i = 0; i < kmin; ++i) {
      const float2 e = h[i];
      d -= e.x;
      S += e.y;
    }
    float bn = 0.0f, bd = 1.0f;
    int bm = -1;
    consider<false, DIP, MIP1>(Wf - d, S, 0.f, d, kmin - 1, 0.f, mipf, bn, bd, bm);
    if (bm >= 0)
      __hip_atomic_fetch_max(&s_best[t], box_key(bn, bd, bm, j, nb), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Next work item of a persistent workgroup (thread 0 only): items of its
// own partition first, then of the others in turn; -1 once all are taken.
// done_mask remembers the partitions found empty.
__device__ inline long long next_item(const SearchArgs &a, unsigned &done_mask) {
  const int np = a.nparts;
  const int home = (int)(blockIdx.x % (unsigned)np);
  for (int k = 0; k < np; ++k) {
    const int x = home + k < np ? home + k : home + k - np;
    if (done_mask & (1u << x)) continue;
    const unsigned long long it =
        __hip_atomic_fetch_add(a.counter + x, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long item = a.part_begin[x] + (long long)it;
    if (item < a.part_begin[x + 1]) return item;
    done_mask |= 1u << x;
  }
  return -1;
}

// A claimed work item and its place: curve and tile (period, for the
// unbinned search) within the curve.
struct ItemRef {
  long long item;
  int curve;
  int tile;
};

// The segment of the last claimed item, kept in thread 0's registers:
// items of a partition are claimed in increasing order, so the next one
// usually falls in the same segment and needs no memory access to place.
struct SegCache {
  long long lo, hi;  // items [lo, hi) of the segment
  int curve, tile0;
};

// Claim the next item and place it (thread 0 only).
__device__ inline ItemRef claim_item(const SearchArgs &a, unsigned &done_mask, SegCache &sc) {
  ItemRef r;
  r.item = next_item(a, done_mask);
  r.curve = 0;
  r.tile = 0;
  if (r.item < 0) return r;
  if (!(r.item >= sc.lo && r.item < sc.hi)) {
    int lo = 0, hi = a.nseg - 1;  // last s with seg_start[s] <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.seg_start[mid] <= r.item)
        lo = mid;
      else
        hi = mid - 1;
    }
    sc.lo = a.seg_start[lo];
    sc.hi = a.seg_start[lo + 1];
    sc.curve = a.seg_curve[lo];
    sc.tile0 = a.seg_tile0[lo];
  }
  r.curve = sc.curve;
  r.tile = sc.tile0 + (int)(r.item - sc.lo);
  return r;
}

// Unit-weight kernels are held to 64 VGPRs (8 waves per SIMD): with tiles of
// up to 7 periods, 8 workgroups then fit a CU's LDS and registers alike, at
// the price of a few spills in the item set-up.  Where the tile's LDS allows
// no more than 6 workgroups per CU anyway, the WIDE copy (80 VGPRs, no
// spills) runs instead; weighted kernels always have 80.
template <bool WEIGHTED, bool DIP, bool WIDE>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((WEIGHTED || WIDE) ? 6 : 8)))
void search_kernel(SearchArgs a) {
  extern __shared__ __align__(16) unsigned long long s_hist[];
  __shared__ double s_f[kTileMax];
  __shared__ unsigned long long s_best[kTileMax];
  __shared__ int s_nonempty[kTileMax];
  // results of the item's periods, written out together at its end
  __shared__ float s_rsr[kGroupMax];
  __shared__ float s_rdp[kGroupMax];
  __shared__ int s_rjk[kGroupMax];      // j & 0xFFFF | k << 16
  __shared__ unsigned long long s_gkey;  // the item's largest (SR, ~period)
  __shared__ long long s_item;
  __shared__ int s_curve;
  __shared__ int s_p0, s_gp0, s_gp1, s_t, s_edge;

  const int tid = threadIdx.x;
  constexpr int wpb = WEIGHTED ? 2 : 1;
  // A work item is a group of consecutive periods of one curve, searched one
  // tile of periods per pass of this loop; the tile's results are staged in
  // LDS and the group's are written out together after its last tile.
  // Thread 0 claims the next group one step ahead, while the workgroup
  // works, so the claim's atomic and lookups are off the path.  The group
  // being searched (its item, curve, periods [gp0, gp1), tile t and the
  // current tile's start p0) lives in LDS, written and read by thread 0, so
  // the tile body keeps the register footprint of one tile.
  unsigned done_mask = 0u;
  SegCache sc = {0, 0, 0, 0};
  ItemRef nx = {-1, 0, 0};
  if (tid == 0) {
    nx = claim_item(a, done_mask, sc);
    s_p0 = 0;
    s_t = 0;
    s_gp1 = 0;
  }

  for (;;) {
    if (tid == 0) {
      int p0 = s_p0 + s_t;
      int edge = 0;
      if (p0 >= s_gp1) {  // next group (groups are never empty)
        edge = 1;         // first tile of the group
        s_item = nx.item;
        s_curve = nx.curve;
        if (nx.item >= 0) {
          const CurveDesc *d = a.curves + nx.curve;
          const int G = d->group > 0 ? d->group : d->tile;
          const int gp0 = max(0, nx.tile * G - d->galign);
          s_t = d->tile;
          s_gp0 = gp0;
          s_gp1 = min(d->nperiods, (nx.tile + 1) * G - d->galign);
          p0 = gp0;
        }
      }
      if (p0 + s_t >= s_gp1) edge |= 2;  // last tile of the group
      s_p0 = p0;
      s_edge = edge;
    }
    __syncthreads();
    if (s_item < 0) break;
    // Item values are uniform: keep them (and the curve record) scalar.
    const int c = __builtin_amdgcn_readfirstlane(s_curve);
    const int p0 = __builtin_amdgcn_readfirstlane(s_p0);
    const int edge = __builtin_amdgcn_readfirstlane(s_edge);
    __syncthreads();  // everyone has read the item before thread 0 takes the next
    if (tid == 0 && (edge & 1)) nx = claim_item(a, done_mask, sc);

    const CurveDesc cd = a.curves[c];
    const int np = min(cd.tile, __builtin_amdgcn_readfirstlane(s_gp1) - p0);
    // Every item reaches the one barrier at the end of the loop body (no
    // `continue`: a second way into the loop header that skips thread 0's
    // fetch lets the compiler keep the other lanes circling the header
    // barrier without it).
    if (np <= 0) {
    } else if (cd.status != kCurveOk) {
      for (int t = tid; t < np; t += kBlock) {
        const int64_t r = cd.r_off + p0 + t;
        a.sr[r] = NAN;
        a.depth[r] = NAN;
        a.jstart[r] = -1;
        a.kwidth[r] = -1;
      }
    } else {
    if (tid == 0 && (edge & 1)) s_gkey = 0ull;
    const int nb = cd.nbins;
    const int kmin = cd.kmin;
    const int kmax = cd.kmax;
    // Widths up to half the bins are scanned directly, wider ones through
    // their complement; neither reads more than kscan - 1 bins past the end.
    const int kscan = min(kmax, nb >> 1);
    const int HB = nb + max(kscan - 1, 1);  // bins, then clamp word / wrap copy
    const int HS = max(cd.hstride, HB);     // words between periods' planes

    // Clear the tile's histograms; frequencies f = 1/P (IEEE division).
    for (int i = tid; i < np * HS * wpb; i += kBlock) s_hist[i] = 0ull;
    if (tid < np) {
      s_f[tid] = 1.0 / a.periods[cd.p_off + p0 + tid];
      s_best[tid] = 0ull;
      s_nonempty[tid] = 0;
    }
    __syncthreads();
    // the tile's longest period, taken from its ends (period grids are
    // ordered in practice; another choice only changes the speed)
    const double ftile = fmin(s_f[0], s_f[np - 1]);
    const int lanes_gap =
        __builtin_amdgcn_readfirstlane(fold_lane_gap(ftile, cd.nbins, cd.cadence));
    // Merging a thread's same-bin points pays only where one cadence step
    // moves the phase by less than a bin at the tile's longest period.
    const bool merge = fold_merges(ftile, cd.nbins, cd.cadence, a.fold_policy);

    // Fold and bin: points in registers, reused for every period of the tile.
    for (int64_t base = 0; base < cd.n; base += (int64_t)kBlock * kPPT) {
      if (base + (int64_t)kBlock * kPPT <= cd.n) {
        if (merge)
          fold_chunk<WEIGHTED, true, true>(a, cd, base, np, s_f, s_hist, HS, lanes_gap);
        else
          fold_chunk<WEIGHTED, true, false>(a, cd, base, np, s_f, s_hist, HS, lanes_gap);
      } else {
        fold_chunk<WEIGHTED, false, true>(a, cd, base, np, s_f, s_hist, HS, 1);
      }
    }
    __syncthreads();

    // Exact integer bins -> FP32 in place (the clamp word joins bin nb - 1).
    {
      const float qscale = ldexpf(1.0f, -cd.qbits);
      int t = tid / nb, b = tid - (tid / nb) * nb;
      const int dt = kBlock / nb, db = kBlock - (kBlock / nb) * nb;
      for (; t < np;) {
        unsigned long long *w = s_hist + (size_t)t * HS * wpb + b;
        unsigned long long w0 = w[0];
        unsigned long long w1 = WEIGHTED ? w[HS] : 0ull;
        if (b == nb - 1) {
          w0 += w[1];
          if (WEIGHTED) w1 += w[HS + 1];
        }
        const BinWord bw = decode_word(w0, cd.shift);
        if (WEIGHTED) {
          // A slot <- (R, S) of the bin, B slot <- (count, 0)
          *reinterpret_cast<float2 *>(w) =
              make_float2(int47_to_float(bw.sum) * qscale, int47_to_float((long long)w1) * qscale);
          *reinterpret_cast<float2 *>(w + HS) = make_float2((float)bw.count, 0.0f);
          if (bw.count != 0u)
            __hip_atomic_fetch_add(&s_nonempty[t], 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
          float2 *o = reinterpret_cast<float2 *>(w);
          *o = make_float2((float)bw.count, int47_to_float(bw.sum) * qscale);
        }
        t += dt;
        b += db;
        if (b >= nb) {
          b -= nb;
          ++t;
        }
      }
    }
    __syncthreads();
    // Wrap-around: bins 0 .. kscan-2 repeated after bin nb-1.
    if (kscan > 1) {
      const int ext = kscan - 1;
      for (int i = tid; i < np * ext; i += kBlock) {
        const int t = i / ext;
        const int e = i - t * ext;
        unsigned long long *src = s_hist + (size_t)t * HS * wpb + e;
        src[nb] = src[0];
        if (WEIGHTED) src[HS + nb] = src[HS];
      }
    }
    __syncthreads();
    if (WEIGHTED && kmin <= kscan) {
      seed_best_weighted<DIP>(s_hist, s_best, s_nonempty, np, nb, HS, kmin, kmax, cd.Wf,
                              (float)(cd.n_eff - 1), (float)a.min_in_points,
                              a.min_in_points <= 1);
      __syncthreads();
    } else if (!WEIGHTED && kmin <= kscan && a.seed_unit) {
      if (a.min_in_points <= 1)
        seed_best_unit<DIP, true>(s_hist, s_best, np, nb, HS, kmin, cd.Wf, 0.f);
      else
        seed_best_unit<DIP, false>(s_hist, s_best, np, nb, HS, kmin, cd.Wf,
                                   (float)a.min_in_points);
      __syncthreads();
    }

    // Box scan.  Lane task = (start bin j, period t), start-bin major, so that
    // the per-period best found by earlier tasks (s_best) is already a good
    // lower bound theta when later tasks run.  Boxes are screened against a
    // slightly relaxed theta; only those that pass get the exact comparison,
    // validity test and index bookkeeping.  The largest box always passes,
    // so the result is that of the full comparison.
    //
    // The relaxation covers the rounding of the screen's products (a few
    // units of 2^-24), the departure of the rounded R (W - R) from a concave
    // function of R, and for weighted curves the rounding of the running
    // weight R itself (k terms); at least 2^-14.
    if (kmin <= kscan) {
      const float Wf = cd.Wf;
      const float nmax1 = (float)(cd.n_eff - 1);
      const float mipf = (float)a.min_in_points;
      const bool mip1 = a.min_in_points <= 1;
      const float margin =
          fmaxf(0x1p-14f, (float)((WEIGHTED ? 2 : 1) * kscan + 16) * 0x1p-24f);
      int j = tid / np, t = tid - (tid / np) * np;
      const int dj = kBlock / np, dtt = kBlock - (kBlock / np) * np;
      for (; j < nb;) {
        const float theta = __uint_as_float((unsigned)(s_best[t] >> 32));
        const float thr = theta * (1.0f - margin);
        float bn, bd;
        int bm;
        if (WEIGHTED) {
          const float2 *ha = reinterpret_cast<const float2 *>(s_hist) +
                             __umul24((unsigned)t, (unsigned)(2 * HS)) + j;
          const bool need_counts = !(mip1 && s_nonempty[t] > kmax);
          scan_task_weighted<DIP>(ha, ha + HS, kmin, kscan, Wf, thr, nmax1, mipf, need_counts, bn,
                                  bd, bm);
        } else {
          const float2 *h =
              reinterpret_cast<const float2 *>(s_hist) + __umul24((unsigned)t, (unsigned)HS) + j;
          if (mip1)
            scan_task_unit<DIP, true>(h, kmin, kscan, Wf, thr, mipf, bn, bd, bm);
          else
            scan_task_unit<DIP, false>(h, kmin, kscan, Wf, thr, mipf, bn, bd, bm);
        }
        if (bm >= 0)
          __hip_atomic_fetch_max(&s_best[t], box_key(bn, bd, bm, j, nb), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        t += dtt;
        j += dj;
        if (t >= np) {
          t -= np;
          ++j;
        }
      }
    }
    // Widths above half the bins (only when kmax allows them): through the
    // complement, without a screen.
    if (kmax > kscan) {
      const int k1lo = nb - kmax;
      const int k1hi = nb - max(kmin, kscan + 1);
      const float Stot = (float)cd.Stot;
      const float neff = (float)cd.n_eff;
      const float mipf = (float)a.min_in_points;
      for (int q = tid; q < np * nb; q += kBlock) {
        const int j1 = q / np, t = q - (q / np) * np;
        const float2 *h = reinterpret_cast<const float2 *>(s_hist) +
                          __umul24((unsigned)t, (unsigned)(WEIGHTED ? 2 * HS : HS)) + j1;
        const unsigned long long key = scan_task_complement<WEIGHTED, DIP>(
            h, h + HS, j1, k1lo, k1hi, nb, cd.Wf, Stot, neff, mipf);
        if (key != 0ull)
          __hip_atomic_fetch_max(&s_best[t], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    __syncthreads();

    // Per period: the winning box's sums again in FP64 from the bins, the
    // statistic and depth from them.  A box wider than half the bins is
    // summed through its complement, with the exact totals.
    if (tid < np) {
      const int t = tid;
      const int p = p0 + t;
      const int g = p - s_gp0;  // staging slot
      const unsigned long long key = s_best[t];
      float srf = 0.0f;
      if (key == 0ull) {
        s_rsr[g] = 0.0f;
        s_rdp[g] = NAN;
        s_rjk[g] = -1;
      } else {
        const unsigned idx = 0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull);
        const int k = (int)(idx / (unsigned)nb);
        const int j = (int)(idx - (unsigned)k * (unsigned)nb);
        const float2 *plane =
            reinterpret_cast<const float2 *>(s_hist + (size_t)t * HS * (WEIGHTED ? 2 : 1));
        const bool wide = 2 * k > nb;
        const int s0 = wide ? (j + k >= nb ? j + k - nb : j + k) : j;
        const int len = wide ? nb - k : k;
        double Rs = 0.0, Ss = 0.0;
        for (int m = 0; m < len; ++m) {
          const float2 e = plane[s0 + m];
          Rs += (double)e.x;
          Ss += (double)e.y;
        }
        const double W = cd.Wtot;
        const double R = wide ? W - Rs : Rs;        // weight in the box
        const double D = wide ? Rs : W - Rs;        // weight outside it
        const double S = wide ? cd.Stot - Ss : Ss;  // signal in the box
        const double den = R * D;
        const double sr = sqrt(S * S / den) * cd.out_scale;
        const double depth = -S * W / den * cd.out_scale;
        srf = (float)sr;
        s_rsr[g] = srf;
        s_rdp[g] = (float)depth;
        s_rjk[g] = (j & 0xFFFF) | (k << 16);
      }
      __hip_atomic_fetch_max(&s_gkey,
                             ((unsigned long long)__float_as_uint(srf) << 32) |
                                 (unsigned long long)(0xFFFFFFFFu - (unsigned)p),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    // After the group's last tile: its results, consecutive periods of the
    // curve, written out together (whole result lines where groups are
    // line-aligned), and one global update of the curve's best key.
    if (edge & 2) {
      __syncthreads();
      const int gp0 = s_gp0;
      const int ng = s_gp1 - gp0;
      for (int t = tid; t < ng; t += kBlock) {
        const int64_t r = cd.r_off + gp0 + t;
        const int jk = s_rjk[t];
        a.sr[r] = s_rsr[t];
        a.depth[r] = s_rdp[t];
        a.jstart[r] = (int)(short)(jk & 0xFFFF);
        a.kwidth[r] = jk >> 16;
      }
      if (tid == 0)
        __hip_atomic_fetch_max(a.best_key + c, s_gkey, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    }  // valid item
    __syncthreads();
  }
}

__global__ void bins_kernel(const double *dt, int64_t n, const double *period, int32_t nbins,
                            int32_t *bins) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double f = 1.0 / period[0];
    bins[i] = phase_bin(dt[i], f, (double)nbins, (unsigned)(nbins - 1));
  }
}

// ------------------------------------------------------------- detection
// One workgroup per curve: mean and population deviation of SR (FP64), then
// peaks largest first, a peak at P suppressing every P' within
// window * hP of hP for h in {1, 1/2, 2, 1/3, 3}.
//
// Peaks without a pass per peak: while the deviation pass reads SR, every
// thread keeps the kDetList largest keys of its slice of periods (p = tid +
// kBlock j, positive SR only) with their periods.  A key is (SR bits, ~p),
// unique, and orders periods as the peaks are chosen (larger SR, then the
// smaller index).  For each peak a thread offers its largest entry not yet
// suppressed, the workgroup takes the largest offer, and every thread tests
// its remaining entries against the new peak.  A thread whose entries are all
// used up while its slice holds more positive values scans its slice again
// against every peak so far and refills its list.
// List length: each entry costs four VGPRs and insertion work in the
// deviation pass; too short a list runs out near strong peaks and their
// harmonics, and a refill re-reads the slice.  On 20000-period periodograms
// of 2000-point curves, 12 is fastest for 8 peaks (8: refills set the
// kernel's tail; 16: the pass loses occupancy).
constexpr int kDetList = 12;
constexpr int kDetBatch = 8;   // loads in flight per pass
constexpr int kDetRefill = 4;  // loads in flight per refill (registers)

__global__ __launch_bounds__(kBlock) void detect_kernel(DetectArgs a) {
  __shared__ double sa[kBlock];
  __shared__ double sb[kBlock];
  __shared__ double sc[kBlock];
  __shared__ unsigned long long s_key[kBlock / 64];  // one offer per wave
  __shared__ double s_peak[BLS_MAX_PEAKS];
  const int c = blockIdx.x;
  if (c >= a.ncurves) return;
  const DetectDesc dd = a.desc[c];
  const int64_t m = dd.nperiods;
  const float *sr = a.sr + dd.r_off;
  const double *per = a.periods + dd.p_off;
  bls_detection *out = reinterpret_cast<bls_detection *>(a.out) + c;
  const int tid = threadIdx.x;

  // One pass over SR.  A thread reads its slice kDetBatch values at a time
  // (whole batches, then the tail) and keeps: the running count, mean and sum
  // of squared deviations of its values, each batch merged in by the pairwise
  // update of Chan, Golub and LeVeque (one value at a time in the tail); its
  // largest value; and its list (descending keys).  The workgroup merges the
  // threads' statistics the same way, in a fixed tree.
  unsigned long long top[kDetList];
#pragma unroll
  for (int i = 0; i < kDetList; ++i) top[i] = 0ull;
  int npos = 0;  // positive SR values in this thread's slice
  double cn = 0.0, cmean = 0.0, cm2 = 0.0, mx = -INFINITY;
  auto take = [&](float v, int64_t p) {
    mx = fmax(mx, (double)v);
    if (v > 0.0f) {
      ++npos;
      unsigned long long key = ((unsigned long long)__float_as_uint(v) << 32) |
                               (unsigned long long)(0xFFFFFFFFu - (unsigned)p);
      if (key > top[kDetList - 1]) {
#pragma unroll
        for (int i = 0; i < kDetList; ++i) {
          if (key > top[i]) {
            const unsigned long long o = top[i];
            top[i] = key;
            key = o;
          }
        }
      }
    }
  };
  const int64_t full = m - (int64_t)(kDetBatch - 1) * kBlock;  // p0 < full: whole batch
  int64_t p0 = tid;
  for (; p0 < full; p0 += kDetBatch * kBlock) {
    float v[kDetBatch];
#pragma unroll
    for (int u = 0; u < kDetBatch; ++u) v[u] = sr[p0 + (int64_t)u * kBlock];
    double bs = 0.0;
#pragma unroll
    for (int u = 0; u < kDetBatch; ++u) bs = bs + (double)v[u];
    const double bmean = bs * (1.0 / kDetBatch);  // exact: a power of two
    double bm2 = 0.0;
#pragma unroll
    for (int u = 0; u < kDetBatch; ++u) {
      const double dv = (double)v[u] - bmean;
      bm2 = bm2 + dv * dv;
    }
    const double nn = cn + (double)kDetBatch;
    const double delta = bmean - cmean;
    const double fb = (double)kDetBatch / nn;
    cmean = cmean + delta * fb;
    cm2 = cm2 + bm2 + delta * delta * cn * fb;
    cn = nn;
#pragma unroll
    for (int u = 0; u < kDetBatch; ++u) take(v[u], p0 + (int64_t)u * kBlock);
  }
  for (int64_t p = p0; p < m; p += kBlock) {
    const float v = sr[p];
    cn = cn + 1.0;
    const double delta = (double)v - cmean;
    cmean = cmean + delta / cn;
    cm2 = cm2 + delta * ((double)v - cmean);
    take(v, p);
  }
  block_chan(cn, cmean, cm2, sa, sb, sc);
  double mn = INFINITY;
  block_minmax(mn, mx, sa, sb);
  const double mean = cmean;
  const double sd = sqrt(cm2 / (double)m);
  const double sde = sd > 0.0 ? (mx - mean) / sd : 0.0;

  auto key_index = [](unsigned long long key) -> int64_t {
    return (int64_t)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
  };
  double tper[kDetList];
  unsigned dead = 0u;  // bit i: entry i empty, taken or suppressed
#pragma unroll
  for (int i = 0; i < kDetList; ++i) {
    tper[i] = top[i] ? per[key_index(top[i])] : 0.0;
    if (!top[i]) dead |= 1u << i;
  }
  bool more = npos > kDetList;  // the slice holds values the list dropped
  const double harm[5] = {1.0, 0.5, 2.0, 1.0 / 3.0, 3.0};
  auto suppressed = [&](double Pp, double P) {
    bool off = false;
    for (int h = 0; h < 5; ++h) {
      const double cp = harm[h] * P;
      if (fabs(Pp - cp) <= a.window * cp) off = true;
    }
    return off;
  };

  int k = 0;
  for (; k < a.max_peaks; ++k) {
    if (dead == (1u << kDetList) - 1u && more) {
      // Refill the list with the slice's largest entries free of every peak
      // so far.  Only a value that would enter the list is tested; one that
      // would not, or one pushed out, leaves `more` set (a later refill
      // tests it then).
#pragma unroll
      for (int i = 0; i < kDetList; ++i) top[i] = 0ull;
      more = false;
      auto retake = [&](float v, double Pp, int64_t p) {
        if (!(v > 0.0f)) return;
        unsigned long long key = ((unsigned long long)__float_as_uint(v) << 32) |
                                 (unsigned long long)(0xFFFFFFFFu - (unsigned)p);
        if (key < top[kDetList - 1]) {
          more = true;
          return;
        }
        bool off = false;
        for (int j = 0; j < k; ++j) off = off || suppressed(Pp, s_peak[j]);
        if (off) return;
        if (top[kDetList - 1]) more = true;  // the last entry drops out
#pragma unroll
        for (int i = 0; i < kDetList; ++i) {
          if (key > top[i]) {
            const unsigned long long o = top[i];
            top[i] = key;
            key = o;
          }
        }
      };
      // Loads in batches, as in the passes above: a refill is a chain of
      // dependent loads otherwise.
      const int64_t rfull = m - (int64_t)(kDetRefill - 1) * kBlock;
      int64_t q0 = tid;
      for (; q0 < rfull; q0 += kDetRefill * kBlock) {
        float v[kDetRefill];
        double pp[kDetRefill];
#pragma unroll
        for (int u = 0; u < kDetRefill; ++u) {
          v[u] = sr[q0 + (int64_t)u * kBlock];
          pp[u] = per[q0 + (int64_t)u * kBlock];
        }
#pragma unroll
        for (int u = 0; u < kDetRefill; ++u) retake(v[u], pp[u], q0 + (int64_t)u * kBlock);
      }
      for (int64_t q = q0; q < m; q += kBlock) retake(sr[q], per[q], q);
      dead = 0u;
#pragma unroll
      for (int i = 0; i < kDetList; ++i) {
        tper[i] = top[i] ? per[key_index(top[i])] : 0.0;
        if (!top[i]) dead |= 1u << i;
      }
    }
    unsigned long long offer = 0ull;
    int mine = -1;
#pragma unroll
    for (int i = kDetList - 1; i >= 0; --i)
      if (!((dead >> i) & 1u)) {
        offer = top[i];
        mine = i;
      }
    // Largest offer: across the wave by shuffles, across the waves in LDS.
    // (Every read of s_key for the previous peak happened before the barrier
    // that published that peak's period.)
    unsigned long long wbest = offer;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long x = __shfl_xor(wbest, o);
      wbest = x > wbest ? x : wbest;
    }
    if ((tid & 63) == 0) s_key[tid >> 6] = wbest;
    __syncthreads();
    unsigned long long key = s_key[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w) key = s_key[w] > key ? s_key[w] : key;
    if (key == 0ull) break;
    if (offer == key) {  // the owner: its entry's period for everyone
#pragma unroll
      for (int i = 0; i < kDetList; ++i)
        if (i == mine) s_peak[k] = tper[i];
    }
    __syncthreads();
    const double P = s_peak[k];
    const int64_t pk = key_index(key);
    const float vk = __uint_as_float((unsigned)(key >> 32));
    if (tid == 0) {
      out->peak_index[k] = pk;
      out->peak_sr[k] = vk;
      out->peak_sde[k] = sd > 0.0 ? (float)(((double)vk - mean) / sd) : 0.0f;
    }
    // The suppression test of every entry, harmonic by harmonic (the same
    // products as the refill's test, so the two agree bit for bit).
#pragma unroll
    for (int h = 0; h < 5; ++h) {
      const double cp = harm[h] * P;
      const double wc = a.window * cp;
#pragma unroll
      for (int i = 0; i < kDetList; ++i)
        if (fabs(tper[i] - cp) <= wc) dead |= 1u << i;
    }
  }
  if (tid == 0) {
    out->mean_sr = mean;
    out->std_sr = sd;
    out->sde = sde;
    out->npeaks = k;
    out->candidate = sde >= a.threshold ? 1 : 0;
    for (int i = k; i < BLS_MAX_PEAKS; ++i) {
      out->peak_index[i] = -1;
      out->peak_sr[i] = 0.0f;
      out->peak_sde[i] = 0.0f;
    }
  }
}

// ------------------------------------------------------- eclipse window
// Detection efficiency of a cadence.  Per trial period the kept times are
// folded with the phase bins of the search (nphase bins); every bin keeps the
// smallest and largest cycle number floor(d f) of the points in it.  The
// eclipse starting at offset j covers bins j .. j+k-1 of one cycle, the
// bins past the end of the cycle belonging to the eclipse one cycle earlier,
// so over its window the eclipse numbers seen are cycle (bins >= j) and
// cycle - 1 (wrapped bins); two distinct eclipses are observed exactly when
// the largest such number exceeds the smallest, one when any bin is filled.

__global__ __launch_bounds__(kBlock) void window_prep_kernel(WindowArgs a) {
  __shared__ double sa[kBlock];
  __shared__ double sb[kBlock];
  const int c = blockIdx.x;
  if (c >= a.ncurves) return;
  WindowDesc *wd = a.desc + c;
  const int64_t off = wd->n_off, n = wd->n;
  const int tid = threadIdx.x;
  double tmin = INFINITY, tmax = -INFINITY, bad = 0.0, kept = 0.0;
  for (int64_t i = tid; i < n; i += kBlock) {
    const double wi = a.w ? a.w[off + i] : 1.0;
    if (!(wi >= 0.0) || isinf(wi)) {
      bad = 1.0;
      continue;
    }
    if (wi == 0.0) continue;
    const double ti = a.t[off + i];
    if (!isfinite(ti)) {
      bad = 1.0;
      continue;
    }
    kept = kept + 1.0;
    tmin = fmin(tmin, ti);
    tmax = fmax(tmax, ti);
  }
  double badp = 0.0;
  if (wd->check_periods) {
    for (int64_t i = tid; i < wd->nperiods; i += kBlock) {
      const double P = a.periods[wd->p_off + i];
      if (!isfinite(P) || !(P > 0.0)) badp = 1.0;
    }
  }
  block_sum2(bad, kept, sa, sb);
  double mx = badp;
  block_minmax(tmin, mx, sa, sb);
  double lo = INFINITY;
  block_minmax(lo, tmax, sa, sb);
  if (tid == 0) {
    wd->t0 = tmin;
    wd->dmax = tmax - tmin;
    wd->status = bad > 0.0 ? kCurveBadData
                 : kept < 1.0 ? kCurveTooFew
                 : mx > 0.0 ? kCurveBadPeriod
                            : kCurveOk;
  }
}

constexpr int kCycleEmptyLo = 0x3fffffff;   // min of an empty bin
constexpr int kCycleEmptyHi = -0x3fffffff;  // max of an empty bin

// Integer wave sum through DPP moves (registers only): lanes exchange within
// quads, half rows and rows, then rows are combined by row_bcast; lane 63
// holds the total, which every lane receives.  Lanes a DPP step does not
// write keep 0, so they add nothing.
template <int CTRL, int ROWS>
__device__ inline int dpp_i32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);
}

__device__ inline int wave_isum(int v) {
  v += dpp_i32<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v += dpp_i32<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v += dpp_i32<0x141, 0xf>(v);  // row_half_mirror
  v += dpp_i32<0x140, 0xf>(v);  // row_mirror
  v += dpp_i32<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_i32<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return __builtin_amdgcn_readlane(v, 63);
}

// The decision of every window of one period in one pass over its entries.
// Entries are the nphase bins followed by the first k-1 bins again, one
// cycle earlier (entry nb + b is bin b with its cycle numbers minus one), so
// the window at offset j is the k entries j .. j+k-1 of E[0, L), L = nb+k-1.
// A window holds two distinct eclipse numbers exactly when D(j) <= j+k-1,
// where D(j) is the first entry at which its entries from j on hold two:
//   NF(i)  first filled entry >= i;
//   B(p)   filled p that is mixed (min < max), or whose previous filled
//          entry is mixed or has another cycle number;
//   NB(i)  first p >= i with B(p);
//   G(f)   f if f is mixed, else NB(f+1) (the filled entries between are
//          single-valued with f's number, and NB(f+1) is the first that is
//          not);
//   D(j) = G(NF(j)).
// With one eclipse required every filled entry counts as mixed, and D(j) =
// NF(j).  D(j) >= j, and no window reaches past L-1, so entries from L on
// (read from any bin) decide nothing.
//
// One wave takes the period: lane l owns the s consecutive entries
// [l s, l s + s), s odd so that the lanes' strided reads spread over the
// LDS banks.  The lane walks its entries downwards keeping the next filled
// entry p: at a filled entry q, B(p) follows from p and q alone (q is p's
// previous filled entry), so NB(q+1) is p when B(p), else NB(p+1), and G(q)
// follows.  Above the lane's last filled entry NB is NB past the lane,
// carried as kWinOut until a wave scan supplies it.  Three wave scans join
// the lanes: the last filled entry of the lanes before (for the B of the
// lane's first filled entry), NB past the lane (a suffix minimum of the
// lanes' first B), and the G of the first filled entry after the lane (for
// the windows after its last filled entry).
constexpr int kWinInf = 0x3fffffff;   // no such entry
constexpr int kWinOut = 0x3ffffffe;   // NB past the lane, not yet known
// A filled entry's key: its cycle number when single-valued, kWinMix + its
// position when mixed, so that B(p) (seen from p's previous filled entry q)
// is key(p) != key(q).  Cycle numbers are at most kMaxCycle < kWinMix.
constexpr int kWinMix = 0x40000000;
constexpr int kWinNone = -0x7fffffff;  // no filled entry

template <int GAP>
__device__ __forceinline__ int window_period(const int2 *row, int nb, int k) {
  const int lane = threadIdx.x & 63;
  const int L = nb + k - 1;
  const int s = ((L + 63) >> 6) | 1;
  const int base = lane * s;
  // Lane nb / s holds entry nb at offset nb % s: above that offset the
  // lanes from it on hold wrapped entries, below it those after it.  Within
  // each part a lane's entries are all wrapped or none are, so cycle numbers
  // are compared as stored and the next filled entry's number is moved into
  // the unwrapped frame where the lane crosses.
  const int sl = nb / s, mc = nb - sl * s;
  const int wa = lane >= sl ? 1 : 0, wb = lane > sl ? 1 : 0;
  // the next filled entry (none yet: a key no entry has makes the first
  // one found take NB(q+1) = p_pos = kWinOut)
  int p_pos = kWinOut, p_key = kWinNone, p_nb = kWinOut;
  int g = kWinInf;      // G of the next filled entry = D of the entries so far
  int last = -1;        // the lane's last filled entry
  int olo = kWinInf;    // lowest entry whose D is NB past the lane
  int cnt = 0;
  auto step = [&](int m, const int2 *r, int kk) {
    const int x = base + m;
    const int2 v = r[x];
    const bool fl = v.x <= v.y;
    const bool mx = GAP ? v.x < v.y : fl;
    const int key = mx ? x + kWinMix : v.x;
    const int nq = key != p_key ? p_pos : p_nb;
    const int gq = mx ? x : nq;
    p_pos = fl ? x : p_pos;
    p_key = fl ? key : p_key;
    p_nb = fl ? nq : p_nb;
    g = fl ? gq : g;
    last = max(last, fl ? x : -1);
    olo = g == kWinOut ? x : olo;
    cnt += g < x + kk ? 1 : 0;
  };
  // wrapped entries x read bin x - nb; entries from L on decide nothing:
  // a lane holding only such entries reads the first s bins, the lane
  // holding entry L reads up to s - 2 entries past the period's wrapped
  // copy (into the next period or the workspace's padding).  Only unwrapped
  // entries start windows.
  const bool idle = base >= L;
  const int2 *ra = row - (idle ? base : wa * nb), *rb = row - (idle ? base : wb * nb);
  const int ka = wa ? 0 : k, kb = wb ? 0 : k;
  for (int m = s - 1; m >= mc; --m) step(m, ra, ka);
  if (p_key < kWinMix) p_key -= wa - wb;
  for (int m = mc - 1; m >= 0; --m) step(m, rb, kb);
  if (p_key < kWinMix) p_key -= wb;
  // the lane's first filled entry is p (G(p) = g), its last one `last`
  const bool any = last >= 0;
  int l_key = kWinNone;
  if (any) {
    // (an entry from L on, read from any bin, decides nothing)
    const int wrap = last >= nb ? 1 : 0;
    const int2 v = row[min(last - wrap * nb, nb - 1)];
    l_key = (GAP ? v.x < v.y : true) ? last + kWinMix : v.x - wrap;
  }
  // the key of the last filled entry of the lanes before
  int xs = l_key;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(xs, d, 64);
    if (lane >= d && xs == kWinNone) xs = y;
  }
  int carry = __shfl_up(xs, 1, 64);
  if (lane == 0) carry = kWinNone;
  const bool bf = any && (carry != kWinNone ? carry != p_key : p_key >= kWinMix);
  // the lane's first B: its first filled entry, or NB past it
  int nbx = bf ? p_pos : (any && p_nb != kWinOut ? p_nb : kWinInf);
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_down(nbx, d, 64);
    if (lane + d < 64) nbx = min(nbx, y);
  }
  int nb_out = __shfl_down(nbx, 1, 64);
  if (lane == 63) nb_out = kWinInf;
  // entries olo .. last have D = NB past the lane
  if (any && olo <= last && nb_out < kWinInf)
    cnt += max(0, min(last + 1, nb) - max(olo, nb_out - k + 1));
  // the entries after the last filled one have D = G of the next filled
  // entry of the lanes after
  int gx = any ? (g == kWinOut ? nb_out : g) : -1;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_down(gx, d, 64);
    if (lane + d < 64 && gx < 0) gx = y;
  }
  int gc = __shfl_down(gx, 1, 64);
  if (lane == 63) gc = -1;
  if (gc >= 0 && gc < kWinInf)
    cnt += max(0, min(base + s, nb) - max(max(last + 1, base), gc - k + 1));
  return wave_isum(cnt);
}

template <int GAP>
__global__ __launch_bounds__(kBlock) void window_kernel(WindowArgs a) {
  extern __shared__ int2 s_mm[];            // [tile][nphase] (min, max cycle), padding
  __shared__ double s_f[kTileMax];
  __shared__ int s_k[kTileMax];
  static_assert(sizeof(s_f) + sizeof(s_k) == kWindowStaticLds, "window kernel static LDS");
  const int tid = threadIdx.x;
  const int nb = a.nphase;
  const double nbd = (double)nb;
  const unsigned nbm1 = (unsigned)(nb - 1);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

  // A workgroup's items increase, so its cadence only moves forward: keep
  // the current one and the first item of the next.
  int cur = 0;
  int64_t next0 = a.ncurves > 1 ? a.desc[1].item0 : a.nitems;
  WindowDesc wd = a.desc[0];
  // The cadence's times (d = t - t0, kept points only) stay in registers
  // across the workgroup's items of that cadence when it has at most
  // kBlock * kWinRegs points; longer cadences are read again per item.
  constexpr int kWinRegs = 8;
  double dreg[kWinRegs];
  bool kreg[kWinRegs];
  int cached = -1;
  for (int64_t item = blockIdx.x; item < a.nitems; item += gridDim.x) {
    if (item >= next0) {
      while (cur + 1 < a.ncurves && a.desc[cur + 1].item0 <= item) ++cur;
      wd = a.desc[cur];
      next0 = cur + 1 < a.ncurves ? a.desc[cur + 1].item0 : a.nitems;
    }
    const int p0 = (int)(item - wd.item0) * a.tile;
    const int np = min(a.tile, wd.nperiods - p0);
    int32_t *out = a.observed + wd.r_off + p0;
    // One barrier sequence for every item: invalid cadences fall through to
    // the barrier at the end of the loop body rather than `continue`.
    if (wd.status != kCurveOk) {
      if (tid < np) out[tid] = -1;
    } else {
    if (tid < np) {
      const double f = 1.0 / a.periods[wd.p_off + p0 + tid];
      const double kr = __builtin_round(a.duration * f * nbd);
      s_f[tid] = f;
      s_k[tid] = kr < 1.0 ? 1 : kr > nbd ? nb : (int)kr;
      if (wd.dmax * f >= (double)kMaxCycle) atomicOr(a.overflow, 1u);
    }
    for (int i = tid; i < np * nb; i += kBlock) s_mm[i] = make_int2(kCycleEmptyLo, kCycleEmptyHi);
    __syncthreads();

    // Fold: cycle numbers per bin (clamped at kMaxCycle, which the item's
    // set-up has flagged: the largest d f of the cadence is its last kept
    // time's).
    auto fold_point = [&](double d, double f, int2 *row) {
      const double cyc = d * f;
      const double e = floor(cyc);
      const int b = (int)min((unsigned)(int)(__builtin_amdgcn_fract(cyc) * nbd), nbm1);
      const int ei = (int)fmin(e, (double)kMaxCycle);
      int *w2 = reinterpret_cast<int *>(row + b);
      atomicMin(w2, ei);
      atomicMax(w2 + 1, ei);
    };
    if (wd.n <= (int64_t)kBlock * kWinRegs) {
      if (cached != cur) {
#pragma unroll
        for (int r = 0; r < kWinRegs; ++r) {
          const int64_t i = tid + (int64_t)kBlock * r;
          const bool in = i < wd.n;
          const double wi = in ? (a.w ? a.w[wd.n_off + i] : 1.0) : 0.0;
          kreg[r] = in && wi != 0.0;
          dreg[r] = kreg[r] ? a.t[wd.n_off + i] - wd.t0 : 0.0;
        }
        cached = cur;
      }
      for (int t = 0; t < np; ++t) {
        const double f = s_f[t];
#pragma unroll
        for (int r = 0; r < kWinRegs; ++r)
          if (kreg[r]) fold_point(dreg[r], f, s_mm + t * nb);
      }
    } else {
      for (int t = 0; t < np; ++t) {
        const double f = s_f[t];
        for (int64_t i = tid; i < wd.n; i += kBlock) {
          const double wi = a.w ? a.w[wd.n_off + i] : 1.0;
          if (wi == 0.0) continue;
          fold_point(a.t[wd.n_off + i] - wd.t0, f, s_mm + t * nb);
        }
      }
    }
    __syncthreads();

    // Windows: one wave per period.
    for (int t = wave; t < np; t += kBlock / 64) {
      const int k = __builtin_amdgcn_readfirstlane(s_k[t]);
      const int c = window_period<GAP>(s_mm + t * nb, nb, k);
      if ((tid & 63) == 0) out[t] = c;
    }
    }  // valid cadence
    __syncthreads();
  }
}

// ------------------------------------------------- variability pre-search
// Stability of every star (population RMS of its kept values) and its
// magnitude bin, then per (chip, bin) an iterated sigma-clipped mean and
// deviation and the stars above it by flag_sigma deviations.  All sums run
// in FP64 in a fixed lane order combined by a fixed butterfly, so results do
// not depend on scheduling.

// Wave sums in a fixed order, through DPP moves (registers only, no LDS
// round trip per step): lanes exchange within quads, then half rows and rows
// of 16 (every lane then holds its row's sum), then row 0 is added into row
// 1 and row 2 into row 3 (row_bcast:15), then rows 0-1 into rows 2-3
// (row_bcast:31); lane 63 holds the total, which is read out to every lane.
// Lanes a DPP step does not write keep 0, so they add nothing.

template <int CTRL, int ROWS>
__device__ inline double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i32<CTRL, ROWS>((int)(unsigned)(b & 0xffffffffll));
  const int hi = dpp_i32<CTRL, ROWS>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ inline double wave_sum(double v) {
  v = v + dpp_f64<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = v + dpp_f64<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
  v = v + dpp_f64<0x141, 0xf>(v);  // row_half_mirror
  v = v + dpp_f64<0x140, 0xf>(v);  // row_mirror
  v = v + dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = v + dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}


// Sums over each half of a wave (lanes 0-31 and 32-63) in a fixed order:
// the steps of wave_sum up to row_bcast:15, which leave the halves' totals
// in lanes 31 and 63; every lane receives its own half's total.
__device__ inline double half_sum(double v) {
  v = v + dpp_f64<0xb1, 0xf>(v);
  v = v + dpp_f64<0x4e, 0xf>(v);
  v = v + dpp_f64<0x141, 0xf>(v);
  v = v + dpp_f64<0x140, 0xf>(v);
  v = v + dpp_f64<0x142, 0xa>(v);
  const long long b = __double_as_longlong(v);
  const int lo0 = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), 31);
  const int hi0 = __builtin_amdgcn_readlane((int)(b >> 32), 31);
  const int lo1 = __builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffll), 63);
  const int hi1 = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  const bool upper = (threadIdx.x & 32) != 0;
  const int lo = upper ? lo1 : lo0, hi = upper ? hi1 : hi0;
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

__device__ inline int half_isum(int v) {
  v += dpp_i32<0xb1, 0xf>(v);
  v += dpp_i32<0x4e, 0xf>(v);
  v += dpp_i32<0x141, 0xf>(v);
  v += dpp_i32<0x140, 0xf>(v);
  v += dpp_i32<0x142, 0xa>(v);
  const int t0 = __builtin_amdgcn_readlane(v, 31), t1 = __builtin_amdgcn_readlane(v, 63);
  return (threadIdx.x & 32) ? t1 : t0;
}

// Half a wave per star (two stars per wave, so half as many waves wait on
// memory): the mean, then the mean squared deviation (two passes, as the
// definition reads).  A star of up to 320 values is loaded once into
// registers (10 per lane, all loads in flight together) and both passes run
// there; longer stars take the second pass from memory again.  Every lane
// stays active through the sums: a half past the last star works on an
// empty one and writes nothing.
constexpr int kVarLanes = 32;
constexpr int kVarRegs = 10;

__global__ __launch_bounds__(kBlock) void var_rms_kernel(VarArgs a) {
  const int lane = threadIdx.x & (kVarLanes - 1);
  const int c = blockIdx.x * (kBlock / kVarLanes) + (threadIdx.x / kVarLanes);
  const bool live = c < a.ncurves;
  // The star's offsets and magnitude are loaded together up front (one
  // round trip before the values, none after them).
  const int64_t off = live ? a.n_off[c] : 0;
  const int64_t n = live ? a.n_off[c + 1] - off : 0;
  const double mag = live ? a.mag[c] : 0.0;
  const double *x = a.x + off;
  const double *w = a.w ? a.w + off : nullptr;
  int cnt = 0, bad = 0;
  double s = 0.0;
  double xv[kVarRegs];
  bool kv[kVarRegs];
#pragma unroll
  for (int u = 0; u < kVarRegs; ++u) {   // lanes past the end keep nothing
    xv[u] = 0.0;
    kv[u] = false;
  }
  for (int64_t i0 = lane; i0 < n; i0 += kVarLanes * kVarRegs) {
#pragma unroll
    for (int u = 0; u < kVarRegs; ++u) {
      const int64_t i = i0 + kVarLanes * u;
      xv[u] = i < n ? x[i] : 0.0;
      const double wi = i < n ? (w ? w[i] : 1.0) : 0.0;
      if (!(wi >= 0.0) || isinf(wi)) bad = 1;
      kv[u] = wi > 0.0 && !isinf(wi);
    }
#pragma unroll
    for (int u = 0; u < kVarRegs; ++u) {
      if (!kv[u]) continue;
      if (!isfinite(xv[u])) bad = 1;
      s = s + xv[u];
      ++cnt;
    }
  }
  s = half_sum(s);
  cnt = half_isum(cnt);
  bad = half_isum(bad);
  const double mu = s / (double)cnt;
  double ss = 0.0;
  if (!bad && cnt > 0) {
    if (n <= kVarLanes * kVarRegs) {
#pragma unroll
      for (int u = 0; u < kVarRegs; ++u) {
        if (!kv[u]) continue;
        const double dv = xv[u] - mu;
        ss = ss + dv * dv;
      }
    } else {
      for (int64_t i = lane; i < n; i += kVarLanes) {
        const double wi = w ? w[i] : 1.0;
        if (wi == 0.0) continue;
        const double dv = x[i] - mu;
        ss = ss + dv * dv;
      }
    }
  }
  ss = half_sum(ss);
  if (lane != 0 || !live) return;
  if (bad || cnt == 0) {
    a.rms[c] = __longlong_as_double(0x7ff8000000000000ll);
    a.bin[c] = -1;
    a.flag[c] = -1;
    return;
  }
  a.rms[c] = sqrt(ss / (double)cnt);
  a.flag[c] = 0;
  int b = -1;
  if (isfinite(mag)) {
    const double q = floor((mag - a.origin) / a.width);
    if (q >= 0.0 && q < (double)a.nmagbins) b = (int)q;
  }
  a.bin[c] = b;
}

constexpr int kVarRegionCap = 1024;  // members one wave keeps in LDS

// Sum over the workgroup in a fixed order: wave butterflies, then the four
// wave totals in wave order; every thread receives the same value.
__device__ inline double block_sum_fixed(double v, double *s_red) {
  v = wave_sum(v);
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) s_red[wv] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kBlock / 64; ++w) t = t + s_red[w];
  __syncthreads();
  return t;
}

// One workgroup per (chip, bin).  Each wave scans a quarter of the chip's
// stars and keeps its members in its own LDS region, so the regions in wave
// order list the members in star order; a wave with more members than its
// region holds sends the whole task to rescanning the chip instead.
__global__ __launch_bounds__(kBlock) void var_clip_kernel(VarArgs a) {
  __shared__ int s_list[kBlock / 64][kVarRegionCap];
  __shared__ double s_val[kBlock / 64][kVarRegionCap];     // members' RMS
  __shared__ unsigned char s_alive[kBlock / 64][kVarRegionCap];
  __shared__ int s_wcnt[kBlock / 64];
  __shared__ double s_red[kBlock / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int64_t task = blockIdx.x;
  if (task >= (int64_t)a.nchips * a.nmagbins) return;
  const int k = (int)(task / a.nmagbins);
  const int b = (int)(task - (int64_t)k * a.nmagbins);
  const int c0 = (int)a.chip_off[k], c1 = (int)a.chip_off[k + 1];
  const int quarter = (c1 - c0 + 3) / 4;
  const int w0 = min(c1, c0 + wv * quarter), w1 = min(c1, w0 + quarter);

  // Members of this wave's quarter, in star order, all alive; eight chunks
  // of bin numbers are loaded together per round.
  int cnt_w = 0;
  const unsigned long long below = (1ull << lane) - 1ull;
  for (int base = w0; base < w1; base += 64 * 8) {
    int bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int st = base + 64 * u + lane;
      bv[u] = st < w1 ? a.bin[st] : -1;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int st = base + 64 * u + lane;
      const bool mem = bv[u] == b;
      const unsigned long long mask = __ballot(mem);
      if (mem) {
        const int pos = cnt_w + __popcll(mask & below);
        if (pos < kVarRegionCap) s_list[wv][pos] = st;
        a.alive[st] = 1;
      }
      cnt_w += __popcll(mask);
    }
  }
  if (lane == 0) s_wcnt[wv] = cnt_w;
  __syncthreads();
  int cnt0 = 0;
  bool fits = true;
  for (int w = 0; w < kBlock / 64; ++w) {
    cnt0 += s_wcnt[w];
    fits = fits && s_wcnt[w] <= kVarRegionCap;
  }
  const double qnan = __longlong_as_double(0x7ff8000000000000ll);
  if (cnt0 == 0) {
    if (tid == 0) {
      a.bin_mean[task] = qnan;
      a.bin_std[task] = qnan;
      a.bin_count[task] = 0;
    }
    return;  // uniform: every thread saw cnt0 == 0
  }
  // Visit the members in star order: the regions in wave order (value and
  // alive flag in LDS, gathered once), or a rescan of the chip when a region
  // overflowed.  f(value, alive flag, star).
  if (fits) {
    for (int w = 0; w < kBlock / 64; ++w)
      for (int i = tid; i < s_wcnt[w]; i += kBlock) {
        s_val[w][i] = a.rms[s_list[w][i]];
        s_alive[w][i] = 1;
      }
    __syncthreads();
  }
  auto for_members = [&](auto f) {
    if (fits) {
      for (int w = 0; w < kBlock / 64; ++w)
        for (int i = tid; i < s_wcnt[w]; i += kBlock)
          f(s_val[w][i], s_alive[w][i], s_list[w][i]);
    } else {
      for (int st = c0 + tid; st < c1; st += kBlock)
        if (a.bin[st] == b) f(a.rms[st], a.alive[st], st);
    }
  };
  int cnt = cnt0;
  double mu = 0.0, sd = 0.0;
  for (int it = 0;; ++it) {
    double sum = 0.0;
    for_members([&](double v, unsigned char &alive, int) {
      if (alive) sum = sum + v;
    });
    mu = block_sum_fixed(sum, s_red) / (double)cnt;
    double ss = 0.0;
    for_members([&](double v, unsigned char &alive, int) {
      if (alive) {
        const double dv = v - mu;
        ss = ss + dv * dv;
      }
    });
    sd = sqrt(block_sum_fixed(ss, s_red) / (double)cnt);
    if (it >= a.max_iter) break;
    const double lo = mu - a.clip_sigma * sd, hi = mu + a.clip_sigma * sd;
    double drop = 0.0;
    for_members([&](double v, unsigned char &alive, int) {
      if (alive && !(v >= lo && v <= hi)) {
        alive = 0;
        drop = drop + 1.0;
      }
    });
    const int dropped = (int)block_sum_fixed(drop, s_red);
    if (dropped == 0) break;
    cnt -= dropped;
  }
  if (tid == 0) {
    a.bin_mean[task] = mu;
    a.bin_std[task] = sd;
    a.bin_count[task] = cnt;
  }
  if (cnt < a.min_stars) return;
  const double thr = mu + a.flag_sigma * sd;
  for_members([&](double v, unsigned char &, int st) {
    if (v > thr) a.flag[st] = 1;
  });
}

// ------------------------------------------------------ unbinned search
// Box edges between data points: per period the kept points are put in
// phase order (ties by index) and every cyclic run that some box with duty
// cycle in [qlo, qhi] holds exactly is scored.  The order is found without a
// comparison sort: a counting sort on a fine phase grid (about one point per
// cell) groups the points, and each point's rank is its cell's start plus
// the number of cell mates that precede it.  Sums over a run are exact:
// FP64 sums of the integer fixed-point values of the prep pass, below 2^53.

__host__ __device__ inline int pow2_at_least(int n) {
  int m = 1;
  while (m < n) m <<= 1;
  return m;
}

// Forward phase distance from sorted position i (phase pi) to j (phase pj),
// one cycle added when the step passes the end of the order.
__device__ inline double fwd_phase(double pi, double pj, int i, int j) {
  return j > i ? pj - pi : (pj + 1.0) - pi;
}

// GLOB: the per-point arrays live in the workgroup's slice of a device
// workspace instead of LDS (curves longer than LDS holds); the steps are the
// same, only slower.
template <bool WEIGHTED, bool DIP, bool GLOB>
__global__ __launch_bounds__(kBlock) void unbinned_kernel(SearchArgs a) {
  extern __shared__ __align__(16) unsigned char s_lds[];
  __shared__ long long s_item;
  __shared__ int s_curve;
  __shared__ int s_per;
  __shared__ unsigned long long s_vbits;
  __shared__ unsigned long long s_theta;
  __shared__ unsigned int s_tie;
  __shared__ long long s_bestS, s_bestR;
  __shared__ long long s_wsum[kBlock / 64];
  __shared__ int s_part[kBlock];

  const int tid = threadIdx.x;
  const int N = a.ucap;
  const int Mc = pow2_at_least(N);
  unsigned char *s_raw = GLOB ? a.uws + (int64_t)blockIdx.x * a.uws_stride : s_lds;
  double *ph_u = reinterpret_cast<double *>(s_raw);
  double *sph = ph_u + N;
  int *sq = reinterpret_cast<int *>(sph + N);
  int *sidx = sq + N;
  int *grp = sidx + N;
  int *cnt = grp + N;
  int *sw = cnt + Mc + 1;   // weighted only

  unsigned done_mask = 0u;
  SegCache sc = {0, 0, 0, 0};
  ItemRef nx = {-1, 0, 0};
  if (tid == 0) nx = claim_item(a, done_mask, sc);  // one item ahead
  for (;;) {
    if (tid == 0) {
      s_item = nx.item;
      s_curve = nx.curve;
      s_per = nx.tile;
    }
    __syncthreads();
    if (s_item < 0) break;
    const int c = __builtin_amdgcn_readfirstlane(s_curve);
    const int p = __builtin_amdgcn_readfirstlane(s_per);
    __syncthreads();
    if (tid == 0) nx = claim_item(a, done_mask, sc);

    const CurveDesc cd = a.curves[c];
    const int64_t r_out = cd.r_off + p;
    // Every item, valid or not, reaches the one barrier at the end of the
    // loop body: a `continue` here would give the loop header a second way
    // in that skips thread 0's fetch, and the compiler may then keep the
    // other lanes circling the header barrier without thread 0.
    if (cd.status != kCurveOk) {
      if (tid == 0) {
        a.sr[r_out] = NAN;
        a.depth[r_out] = NAN;
        a.jstart[r_out] = -1;
        a.kwidth[r_out] = -1;
      }
    } else {
    const int n = (int)cd.n;
    const int M = pow2_at_least(n);
    const double Md = (double)M;
    const double f = 1.0 / a.periods[cd.p_off + p];
    const double *dt = a.dt + cd.n_off;
    const int32_t *q = a.q + cd.n_off;
    const int32_t *qw = WEIGHTED ? a.qw + cd.n_off : nullptr;

    // Phases and fine-grid cells; dropped points go to the extra cell M.
    for (int i = tid; i <= M; i += kBlock) cnt[i] = 0;
    if (tid == 0) {
      s_vbits = 0ull;
      s_theta = 0ull;
      s_tie = 0xFFFFFFFFu;
    }
    __syncthreads();
    long long wsum = 0;
    for (int i = tid; i < n; i += kBlock) {
      const bool kept = WEIGHTED ? qw[i] >= 0 : true;
      const double ph = __builtin_amdgcn_fract(dt[i] * f);
      ph_u[i] = kept ? ph : 2.0;
      const int cell = kept ? (int)min((unsigned)(int)(ph * Md), (unsigned)(M - 1)) : M;
      atomicAdd(&cnt[cell], 1);
      if (WEIGHTED && kept) wsum += qw[i];
    }
    __syncthreads();
    // Exclusive scan of the M + 1 cell counts (runs per thread, then a
    // sequential pass over the 256 run totals).
    {
      const int per = (M + 1 + kBlock - 1) / kBlock;
      const int b0 = min(M + 1, tid * per), b1 = min(M + 1, b0 + per);
      int run = 0;
      for (int b = b0; b < b1; ++b) run += cnt[b];
      s_part[tid] = run;
      __syncthreads();
      if (tid == 0) {
        int acc = 0;
        for (int i = 0; i < kBlock; ++i) {
          const int v = s_part[i];
          s_part[i] = acc;
          acc += v;
        }
      }
      __syncthreads();
      int acc = s_part[tid];
      for (int b = b0; b < b1; ++b) {
        const int v = cnt[b];
        cnt[b] = acc;
        acc += v;
      }
    }
    __syncthreads();
    // Scatter into cells (any order inside a cell); cnt becomes cell ends.
    for (int i = tid; i < n; i += kBlock) {
      const double ph = ph_u[i];
      const int cell = ph < 1.5 ? (int)min((unsigned)(int)(ph * Md), (unsigned)(M - 1)) : M;
      grp[atomicAdd(&cnt[cell], 1)] = i;
    }
    __syncthreads();
    // Rank = cell start + cell mates before this point in (phase, index).
    for (int i = tid; i < n; i += kBlock) {
      const double ph = ph_u[i];
      const int cell = ph < 1.5 ? (int)min((unsigned)(int)(ph * Md), (unsigned)(M - 1)) : M;
      const int b = cell == 0 ? 0 : cnt[cell - 1];
      const int e = cnt[cell];
      int rank = b;
      for (int k = b; k < e; ++k) {
        const int j = grp[k];
        const double pj = ph_u[j];
        rank += (pj < ph || (pj == ph && j < i)) ? 1 : 0;
      }
      sph[rank] = ph;
      sq[rank] = q[i];
      sidx[rank] = i;
      if (WEIGHTED) sw[rank] = qw[i];
    }
    long long W = 0;
    if (WEIGHTED) {
      for (int o = 32; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o, 64);
      if ((tid & 63) == 0) s_wsum[tid >> 6] = wsum;
    }
    __syncthreads();
    const int nk = M == 0 ? 0 : cnt[M - 1];  // kept points come first
    if (WEIGHTED) {
      for (int k = 0; k < kBlock / 64; ++k) W += s_wsum[k];
    } else {
      W = nk;
    }
    const double Wd = (double)W;
    const double qlo = cd.qlo, qhi = cd.qhi;

    // Runs from every start position, four run steps per iteration with
    // their values loaded together, up to the longest run a box shorter than
    // qhi in phase can hold.  S and R are summed in FP64, which is
    // exact here (|q|, w < 2^qbits with qbits <= 63 - 2 bitlen(n) keep
    // every partial sum below 2^53 at any curve length).  Each step is screened against theta,
    // the best value any lane of the workgroup has found so far in this
    // period (s_theta, raised as lanes improve; the lanes' final bests go to
    // s_vbits as before): a run with
    // S^2 < theta (1 - 2^-20) R (W - R) can be neither the best nor a tie
    // of it, so it skips the admissibility tests and the exact comparison.
    // Candidates are compared without a division (S^2 / den against the
    // lane's best as cross products).
    double bnum = 0.0, bden = 1.0;
    unsigned int btie = 0xFFFFFFFFu;
    double bS = 0.0, bR = 0.0;
    for (int r = tid; r < nk; r += kBlock) {
      const int prev = r == 0 ? nk - 1 : r - 1;
      const double ph_r = sph[r], ph_prev = sph[prev];
      if (!(fwd_phase(ph_prev, ph_r, prev, r) > 0.0)) continue;
      const unsigned long long tb =
          __hip_atomic_load(&s_theta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      double thr = __longlong_as_double((long long)tb) * (1.0 - 0x1p-20);
      // Longest run from r that a box with duty cycle below qhi can hold:
      // the span from r grows along the phase order, so it is found by
      // bisection (a run of one point spans nothing).
      int lmax = 1;
      {
        int hi = nk - 1;
        while (lmax < hi) {
          const int mid = (lmax + hi + 1) >> 1;
          int e = r + mid - 1;
          if (e >= nk) e -= nk;
          if (fwd_phase(ph_r, sph[e], r, e) < qhi)
            lmax = mid;
          else
            hi = mid - 1;
        }
      }
      double S = 0.0, R = 0.0;
      int e0 = r;  // first position of the next group of four
      for (int len = 1; len <= lmax; len += 4) {
        int idx[4];
        idx[0] = e0;
#pragma unroll
        for (int u = 1; u < 4; ++u) idx[u] = idx[u - 1] + 1 == nk ? 0 : idx[u - 1] + 1;
        int qv[4], wv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          qv[u] = sq[idx[u]];
          wv[u] = WEIGHTED ? sw[idx[u]] : 1;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int L = len + u;
          if (L > lmax) break;
          S += (double)qv[u];
          R += WEIGHTED ? (double)wv[u] : 1.0;
          if (DIP && !(S < 0.0)) continue;
          const double den = R * (Wd - R);
          const double num = S * S;
          if (num < thr * den) continue;
          // Rare: the run passed the screen; its edges must be admissible.
          const int e = idx[u];
          const int next = e + 1 == nk ? 0 : e + 1;
          const double pe = sph[e], pn = sph[next];
          if (!(fwd_phase(pe, pn, e, next) > 0.0)) continue;
          const double gap = prev == next ? 1.0 : fwd_phase(ph_prev, pn, prev, next);
          if (!(gap > qlo)) continue;
          if (L < a.min_in_points) continue;
          if (!(den > 0.0) || S == 0.0) continue;
          const double lhs = num * bden, rhs = bnum * den;
          const unsigned int tie = (unsigned)L * (unsigned)nk + (unsigned)r;
          if (lhs > rhs || (lhs == rhs && tie < btie)) {
            bnum = num;
            bden = den;
            btie = tie;
            bS = S;
            bR = R;
            const double v = num / den;
            thr = fmax(thr, v * (1.0 - 0x1p-20));
            __hip_atomic_fetch_max(&s_theta, (unsigned long long)__double_as_longlong(v),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          }
        }
        e0 = idx[3] + 1 == nk ? 0 : idx[3] + 1;
      }
    }
    const double bv = bnum > 0.0 ? bnum / bden : 0.0;
    const unsigned long long vb = (unsigned long long)__double_as_longlong(bv);
    if (bv > 0.0) atomicMax(&s_vbits, vb);
    __syncthreads();
    if (bv > 0.0 && vb == s_vbits) atomicMin(&s_tie, btie);
    __syncthreads();
    if (bv > 0.0 && vb == s_vbits && btie == s_tie) {
      s_bestS = (long long)bS;  // exact integers
      s_bestR = (long long)bR;
    }
    __syncthreads();
    if (tid == 0) {
      float srf = 0.0f;
      if (s_vbits == 0ull) {
        a.sr[r_out] = 0.0f;
        a.depth[r_out] = NAN;
        a.jstart[r_out] = -1;
        a.kwidth[r_out] = -1;
      } else {
        const int len = (int)(s_tie / (unsigned)nk);
        const int r = (int)(s_tie - (unsigned)len * (unsigned)nk);
        const double scale = WEIGHTED ? ldexp(1.0, cd.ew - cd.es) : ldexp(1.0, -cd.es);
        const double v = __longlong_as_double((long long)s_vbits);
        const double Rd = (double)s_bestR;
        const double den = Rd * (Wd - Rd);
        srf = (float)(sqrt(v) * scale);
        a.sr[r_out] = srf;
        a.depth[r_out] = (float)(-(double)s_bestS * Wd / den * scale);
        a.jstart[r_out] = sidx[r];
        a.kwidth[r_out] = sidx[(r + len - 1) % nk];
      }
      const unsigned long long ckey = ((unsigned long long)__float_as_uint(srf) << 32) |
                                      (unsigned long long)(0xFFFFFFFFu - (unsigned)p);
      __hip_atomic_fetch_max(a.best_key + c, ckey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    }  // valid curve
    __syncthreads();
  }
}

template <bool W, bool D, bool G>
const void *unbinned_fn() {
  return reinterpret_cast<const void *>(&unbinned_kernel<W, D, G>);
}

const void *pick_unbinned(bool weighted, bool dip, bool glob) {
  if (glob) {
    if (weighted) return dip ? unbinned_fn<true, true, true>() : unbinned_fn<true, false, true>();
    return dip ? unbinned_fn<false, true, true>() : unbinned_fn<false, false, true>();
  }
  if (weighted) return dip ? unbinned_fn<true, true, false>() : unbinned_fn<true, false, false>();
  return dip ? unbinned_fn<false, true, false>() : unbinned_fn<false, false, false>();
}

__global__ void fill_kernel(unsigned long long *counter, unsigned long long *keys, int32_t nkeys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kMaxParts && counter) counter[i] = 0ull;
  if (i < nkeys) keys[i] = 0ull;
}

__global__ void best_index_kernel(unsigned long long *keys, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const unsigned long long k = keys[i];
    keys[i] = (unsigned long long)(0xFFFFFFFFu - (unsigned)(k & 0xFFFFFFFFull));
  }
}

template <bool W, bool D, bool WIDE = false>
const void *search_fn() {
  return reinterpret_cast<const void *>(&search_kernel<W, D, WIDE>);
}

const void *pick_narrow(bool weighted, bool dip) {
  if (weighted) return dip ? search_fn<true, true>() : search_fn<true, false>();
  return dip ? search_fn<false, true>() : search_fn<false, false>();
}

// The unit-weight kernel copy for a tile of hist_bytes of LDS: the 64-VGPR
// copy where its LDS lets more than 6 workgroups share a CU, the 80-VGPR one
// otherwise (BLS_WIDE_REGS=0/1 forces the choice).
const void *pick(bool weighted, bool dip, int hist_bytes) {
  if (weighted) return pick_narrow(true, dip);
  int wide = -1;
  if (const char *e = getenv("BLS_WIDE_REGS")) wide = atoi(e) != 0 ? 1 : 0;
  if (wide < 0) {
    const void *fn = pick_narrow(false, dip);
    int blocks = 0;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, hist_bytes) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, kBlock, (size_t)hist_bytes) !=
            hipSuccess)
      return fn;
    wide = blocks <= 6 ? 1 : 0;
  }
  if (!wide) return pick_narrow(false, dip);
  return dip ? search_fn<false, true, true>() : search_fn<false, false, true>();
}

}  // namespace

int launch_fill(unsigned long long *counter, unsigned long long *keys, int32_t nkeys,
                void *stream) {
  const int n = nkeys > 1 ? nkeys : 1;
  hipLaunchKernelGGL(fill_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     counter, keys, nkeys);
  return (int)hipGetLastError();
}

int launch_prep(const PrepArgs &a, void *stream) {
  if (a.ncurves <= 0) return 0;
  hipLaunchKernelGGL(prep_kernel, dim3(a.ncurves), dim3(kBlock), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_search(const SearchArgs &a, bool weighted, bool dip_only, int grid, void *stream) {
  if (a.nitems <= 0) return 0;
  const void *fn = pick(weighted, dip_only, a.hist_bytes);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, a.hist_bytes);
  if (e != hipSuccess) return (int)e;
  void *args[] = {const_cast<SearchArgs *>(&a)};
  e = hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, (size_t)a.hist_bytes,
                      (hipStream_t)stream);
  if (e != hipSuccess) return (int)e;
  return (int)hipGetLastError();
}

int launch_bins(const double *dt, int64_t n, const double *period, int32_t nbins, int32_t *bins,
                void *stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(bins_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     (hipStream_t)stream, dt, n, period, nbins, bins);
  return (int)hipGetLastError();
}

int launch_detect(const DetectArgs &a, void *stream) {
  if (a.ncurves <= 0) return 0;
  hipLaunchKernelGGL(detect_kernel, dim3(a.ncurves), dim3(kBlock), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

int launch_best_index(unsigned long long *keys, int32_t n, void *stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(best_index_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     keys, n);
  return (int)hipGetLastError();
}

int launch_window(const WindowArgs &a, int grid, void *stream) {
  if (a.ncurves <= 0) return 0;
  hipLaunchKernelGGL(window_prep_kernel, dim3(a.ncurves), dim3(kBlock), 0, (hipStream_t)stream,
                     a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.nitems <= 0) return (int)e;
  const int lds = window_lds_bytes(a.tile, a.nphase);
  const void *fn = a.min_eclipses >= 2 ? reinterpret_cast<const void *>(&window_kernel<1>)
                                       : reinterpret_cast<const void *>(&window_kernel<0>);
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  if (e != hipSuccess) return (int)e;
  void *args[] = {const_cast<WindowArgs *>(&a)};
  e = hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, (size_t)lds, (hipStream_t)stream);
  if (e != hipSuccess) return (int)e;
  return (int)hipGetLastError();
}

int launch_variability(const VarArgs &a, void *stream) {
  if (a.ncurves <= 0 || a.nchips <= 0) return 0;
  hipStream_t s = (hipStream_t)stream;
  const int per = kBlock / kVarLanes;
  hipLaunchKernelGGL(var_rms_kernel, dim3((a.ncurves + per - 1) / per), dim3(kBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return (int)e;
  const int64_t tasks = (int64_t)a.nchips * a.nmagbins;
  hipLaunchKernelGGL(var_clip_kernel, dim3((unsigned)tasks), dim3(kBlock), 0, s, a);
  return (int)hipGetLastError();
}

int window_blocks_per_cu(int lds_bytes, int *blocks) {
  const void *fn = reinterpret_cast<const void *>(&window_kernel<1>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return (int)e;
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, (size_t)lds_bytes);
}

int64_t unbinned_lds_bytes(int n, bool weighted) {
  const int64_t N = n < 1 ? 1 : n;
  const int64_t M = pow2_at_least((int)N);
  return 8 * N + 8 * N + 4 * N + 4 * N + 4 * N + 4 * (M + 1) + (weighted ? 4 * N : 0);
}

int launch_unbinned(const SearchArgs &a, bool weighted, bool dip_only, int grid, void *stream) {
  if (a.nitems <= 0) return 0;
  const void *fn = pick_unbinned(weighted, dip_only, a.uws != nullptr);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, a.hist_bytes);
  if (e != hipSuccess) return (int)e;
  void *args[] = {const_cast<SearchArgs *>(&a)};
  e = hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, (size_t)a.hist_bytes,
                      (hipStream_t)stream);
  if (e != hipSuccess) return (int)e;
  return (int)hipGetLastError();
}

int unbinned_blocks_per_cu(bool weighted, bool dip_only, bool glob, int lds_bytes,
                           int *blocks) {
  const void *fn = pick_unbinned(weighted, dip_only, glob);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return (int)e;
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, (size_t)lds_bytes);
}

int search_blocks_per_cu(bool weighted, bool dip_only, int hist_bytes, int *blocks) {
  const void *fn = pick(weighted, dip_only, hist_bytes);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, hist_bytes);
  if (e != hipSuccess) return (int)e;
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, (size_t)hist_bytes);
}

}  // namespace bls
