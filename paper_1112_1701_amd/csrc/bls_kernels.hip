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
//
// The unbinned search (bls_unbinned.hip), the detection statistics
// (bls_detect.hip), the eclipse detection efficiency (bls_window.hip) and
// the high-variability pre-search (bls_variability.hip) have sources of
// their own; the work-item claim is shared through bls_items.h.
//
// No FP contraction anywhere (-ffp-contract=off): the phase is computed with
// exactly the FP64 operation sequence of its definition so that every point
// falls into the same bin as in an FP64 evaluation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include "bls_block.h"
#include "bls_device.h"
#include "bls_items.h"
#include "../../include/bls.h"

namespace bls {
namespace {

// ------------------------------------------------------------------ prep
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
// one cadence step advances the phase by less than 0.3 bins at the tile's
// longest period (frequency fmin), so that runs of about three points or
// more share a bin, unless the launch fixes the choice (policy 1: always,
// 2: never).  The merge costs VALU operations on every point and saves one
// LDS atomic per point it joins; shorter runs do not repay it.  A weighted
// point saves two atomics, and there the merge pays from one bin per step.
// Any answer is correct; this one only picks the faster fold.
__device__ inline bool fold_merges(double fmin, int nbins, float cadence, int policy,
                                   bool weighted) {
  if (policy != 0) return policy == 1;
  const double x = fmin * (double)nbins * (double)cadence;
  return !(x >= (weighted ? 1.0 : 0.3));
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
    const bool merge = fold_merges(ftile, cd.nbins, cd.cadence, a.fold_policy, WEIGHTED);

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

int launch_best_index(unsigned long long *keys, int32_t n, void *stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(best_index_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     keys, n);
  return (int)hipGetLastError();
}

int search_blocks_per_cu(bool weighted, bool dip_only, int hist_bytes, int *blocks) {
  const void *fn = pick(weighted, dip_only, hist_bytes);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, hist_bytes);
  if (e != hipSuccess) return (int)e;
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, (size_t)hist_bytes);
}

}  // namespace bls
