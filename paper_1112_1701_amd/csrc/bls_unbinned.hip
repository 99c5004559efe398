// gfx950 kernel of the unbinned box search (box edges between data points,
// a range of durations and phases taken to the data, section 2.2.2).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "bls_device.h"
#include "bls_items.h"
#include "../../include/bls.h"

namespace bls {
namespace {

// ------------------------------------------------------ unbinned search
// Box edges between data points: per period the kept points are put in
// phase order (ties by index) and every cyclic run that some box with duty
// cycle in [qlo, qhi] holds exactly is scored.  The order is found without a
// comparison sort: a counting sort on a fine phase grid (about one point per
// cell) groups the points, and each point's rank is its cell's start plus
// the number of cell mates that precede it.  Sums over a run are exact:
// differences of FP64 prefix sums of the integer fixed-point values of the
// prep pass, all below 2^53.  Runs are screened eight ends at a time by a
// bound from the prefix sums' extremes over those ends; only windows that
// can hold the best run are scored run by run.

__host__ __device__ inline int pow2_at_least(int n) {
  int m = 1;
  while (m < n) m <<= 1;
  return m;
}

// Array stride of the per-point arrays for curves of up to n points: even,
// so that every 8-byte array of the layout stays 8-byte aligned.
__host__ __device__ inline int unbinned_stride(int n) { return n < 1 ? 2 : (n + 1) & ~1; }

// Run ends screened together by one bound (the window of the walk).
constexpr int kUnbRun = 8;

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
  __shared__ double s_wtot[2 * (kBlock / 64)];
  __shared__ int s_part[kBlock / 64];

  const int tid = threadIdx.x;
  const int N = unbinned_stride(a.ucap);
  unsigned char *s_raw = GLOB ? a.uws + (int64_t)blockIdx.x * a.uws_stride : s_lds;
  double *ph_u = reinterpret_cast<double *>(s_raw);
  double *sph = ph_u + N;
  int *sidx = reinterpret_cast<int *>(sph + N);
  int *sq = sidx + N;
  int *sw = sq + N;  // weighted only
  int *grp = sw + (WEIGHTED ? N : 0);
  int *cnt = grp + N;
  // After the ranking: the prefix sums of the values over the unsorted
  // phases, those of the weights over grp and the cell counts (weighted;
  // unit weights keep the cell counts, which place the longest runs), and
  // the window bounds over the values and the next array (the weights or
  // grp), 8 bytes per point.
  double *Pq = ph_u;
  double *Pw = reinterpret_cast<double *>(grp);
  float2 *Mb = reinterpret_cast<float2 *>(sq);

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
    // Exclusive scan of the M + 1 cell counts: a run of cells per thread,
    // a scan of the run totals across each wave, then across the waves.
    {
      const int per = (M + 1 + kBlock - 1) / kBlock;
      const int b0 = min(M + 1, tid * per), b1 = min(M + 1, b0 + per);
      int run = 0;
      for (int b = b0; b < b1; ++b) run += cnt[b];
      int x = run;
      const int lane = tid & 63;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
      }
      if (lane == 63) s_part[tid >> 6] = x;
      __syncthreads();
      int acc = x - run;
      for (int w = 0; w < (tid >> 6); ++w) acc += s_part[w];
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

    // Prefix sums in phase order, Pq[i] = q summed over ranks 0..i (and Pw
    // for the weights), in FP64: every partial sum is an integer below 2^53
    // (|q|, w < 2^31 and at most 2^20 points), so each is exact and a run's
    // sum is a difference of two of them, exact as well.  A thread takes a
    // contiguous chunk: its total, a scan of the totals across the
    // workgroup, then the chunk's running sums.
    {
      const int per = (nk + kBlock - 1) / kBlock;
      const int cb = min(nk, tid * per), ce = min(nk, cb + per);
      double tq = 0.0, tw = 0.0;
      for (int i = cb; i < ce; ++i) {
        tq += (double)sq[i];
        if (WEIGHTED) tw += (double)sw[i];
      }
      double xq = tq, xw = tw;  // inclusive scan across the wave
      const int lane = tid & 63;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const double yq = __shfl_up(xq, o, 64);
        const double yw = WEIGHTED ? __shfl_up(xw, o, 64) : 0.0;
        if (lane >= o) {
          xq += yq;
          if (WEIGHTED) xw += yw;
        }
      }
      if (lane == 63) {
        s_wtot[tid >> 6] = xq;
        if (WEIGHTED) s_wtot[kBlock / 64 + (tid >> 6)] = xw;
      }
      __syncthreads();  // every thread has read nk and the weight total
      double rq = xq - tq, rw = xw - tw;
      for (int w = 0; w < (tid >> 6); ++w) {
        rq += s_wtot[w];
        if (WEIGHTED) rw += s_wtot[kBlock / 64 + w];
      }
      for (int i = cb; i < ce; ++i) {
        rq += (double)sq[i];
        Pq[i] = rq;
        if (WEIGHTED) {
          rw += (double)sw[i];
          Pw[i] = rw;
        }
      }
    }
    __syncthreads();
    const double Tq = nk > 0 ? Pq[nk - 1] : 0.0;
    const double Tw = WEIGHTED ? (nk > 0 ? Pw[nk - 1] : 0.0) : Wd;
    // Prefix sum at an unwrapped rank x < 2 nk (one cycle's total added past
    // the end of the order).
    auto pq_at = [&](int x) { return x >= nk ? Pq[x - nk] + Tq : Pq[x]; };
    auto pw_at = [&](int x) { return x >= nk ? Pw[x - nk] + Tw : Pw[x]; };

    // Window bounds: for every rank i the largest and smallest prefix sum
    // over the kUnbRun unwrapped ranks i .. i + kUnbRun - 1, as floats
    // rounded outwards (a bound needs no more).
    for (int i = tid; i < nk; i += kBlock) {
      double hi = -INFINITY, lo = INFINITY;
      if (i + kUnbRun <= nk) {  // no wrap: the loads go out together
        double v[kUnbRun];
#pragma unroll
        for (int b = 0; b < kUnbRun; ++b) v[b] = Pq[i + b];
#pragma unroll
        for (int b = 0; b < kUnbRun; ++b) {
          hi = fmax(hi, v[b]);
          lo = fmin(lo, v[b]);
        }
      } else {
        for (int b = 0; b < kUnbRun; ++b) {
          int x = i + b, wraps = 0;
          while (x >= nk) {
            x -= nk;
            ++wraps;
          }
          const double v = Pq[x] + (double)wraps * Tq;
          hi = fmax(hi, v);
          lo = fmin(lo, v);
        }
      }
      float fh = (float)hi, fl = (float)lo;
      if ((double)fh < hi) fh = nextafterf(fh, INFINITY);
      if ((double)fl > lo) fl = nextafterf(fl, -INFINITY);
      Mb[i] = make_float2(fh, fl);
    }
    __syncthreads();

    // The longest run from start r that a box with duty cycle below qhi can
    // hold: runs end at r + L - 1, and the span from r grows along the
    // phase order, so the first end u past r whose span reaches qhi gives
    // L = u - r (at most nk - 1; a run of one point spans nothing).  With
    // unit weights the fine grid of the sort places phase(r) + qhi near that
    // end: the first rank of its cell is the guess, and exact span tests
    // move it to the boundary (about one point per cell).  Weighted curves
    // have no room left for the cell counts and bisect.
    auto spans_less = [&](int r, double ph_r, int u) {  // end u unwrapped
      const int e = u >= nk ? u - nk : u;
      return fwd_phase(ph_r, sph[e], r, e) < qhi;
    };
    auto longest_run = [&](int r) {
      const double ph_r = sph[r];
      if (WEIGHTED) {
        int lmax = 1, hi = nk - 1;
        while (lmax < hi) {
          const int mid = (lmax + hi + 1) >> 1;
          if (spans_less(r, ph_r, r + mid - 1))
            lmax = mid;
          else
            hi = mid - 1;
        }
        return lmax;
      }
      if (nk <= 2) return 1;
      const double t = ph_r + qhi;
      const bool wr = t >= 1.0;
      const int cell = (int)min((unsigned)(int)((wr ? t - 1.0 : t) * Md), (unsigned)(M - 1));
      int u = (cell == 0 ? 0 : cnt[cell - 1]) + (wr ? nk : 0);
      const int lo = r + 1, hi = r + nk - 1;
      u = min(max(u, lo), hi);
      while (u < hi && spans_less(r, ph_r, u)) ++u;
      while (u > lo && !spans_less(r, ph_r, u - 1)) --u;
      return u - r;
    };

    // Runs from every start position.  A run of L points from start r has
    // S = P(r + L - 1) - P(r - 1) and R = L (or the same difference of the
    // weight sums), exact, as above.  Runs are screened against theta, the
    // best value any lane of the workgroup has found so far in this period
    // (s_theta holds it relaxed, theta (1 - 2^-20), raised as lanes improve;
    // the lanes' final bests go to s_vbits): a run with
    // S^2 < theta (1 - 2^-20) R (W - R) can be neither
    // the best nor a tie of it.  The ends are taken kUnbRun at a time, and a
    // window of ends is screened as a whole first: S^2 is at most the
    // largest |S| over the window (from the window's prefix-sum bounds;
    // only negative S for dips), and R (W - R) is concave in the growing R,
    // so its least value over the window is at the first or the last end.
    // Only a window that passes has its ends scored one by one: the
    // admissibility tests of the edges and the exact comparison, without a
    // division (S^2 / den against the lane's best as cross products).
    double bnum = 0.0, bden = 1.0;
    unsigned int btie = 0xFFFFFFFFu;
    double bS = 0.0, bR = 0.0;
    for (int r = tid; r < nk; r += kBlock) {
      const int prev = r == 0 ? nk - 1 : r - 1;
      const double ph_r = sph[r], ph_prev = sph[prev];
      if (!(fwd_phase(ph_prev, ph_r, prev, r) > 0.0)) continue;
      double thr = 0.0;
      const int lmax = longest_run(r);
      const int eEnd = r + lmax - 1;  // last end, unwrapped
      const double base = r == 0 ? 0.0 : Pq[r - 1];
      const double wbase = WEIGHTED ? (r == 0 ? 0.0 : Pw[r - 1]) : 0.0;
      // Window bounds against base, and base less one cycle's total past
      // the end of the order: every quantity but the float bound is an
      // integer below 2^53, so up and dn, rounded, still bound S.
      const double base_w = base - Tq;
      double Ru = 1.0;  // R of the window's first end (unit weights)
      const double Rend = (double)lmax;
      for (int e = r; e <= eEnd; e += kUnbRun, Ru += (double)kUnbRun) {
        // theta (already relaxed) as the other lanes have raised it so far
        // (a relaxed read: any value it returns is one some run reached)
        const unsigned long long tb =
            __hip_atomic_load(&s_theta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        thr = fmax(thr, __longlong_as_double((long long)tb));
        const bool wr = e >= nk;
        const float2 mb = Mb[wr ? e - nk : e];
        const double bb = wr ? base_w : base;
        const double up = (double)mb.x - bb;  // >= every S of the window
        const double dn = bb - (double)mb.y;  // >= every -S
        const double sm = DIP ? fmax(dn, 0.0) : fmax(fmax(up, dn), 0.0);
        double R1, R2;
        if (WEIGHTED) {
          R1 = pw_at(e) - wbase;
          R2 = pw_at(min(e + kUnbRun - 1, eEnd)) - wbase;
        } else {
          R1 = Ru;
          R2 = fmin(Ru + (double)(kUnbRun - 1), Rend);
        }
        const double g = fmin(R1 * (Wd - R1), R2 * (Wd - R2));
        if (!(sm * sm >= thr * g)) continue;
        const int eL = min(e + kUnbRun - 1, eEnd);
        // The window's ends in two halves, each half's loads together.
        constexpr int kHalf = kUnbRun / 2;
#pragma unroll
        for (int h = 0; h < kUnbRun; h += kHalf) {
          if (e + h > eL) break;
          double Pv[kHalf], Wv[kHalf];
#pragma unroll
          for (int u = 0; u < kHalf; ++u) {
            const int x = min(e + h + u, eEnd);
            Pv[u] = pq_at(x);
            if (WEIGHTED) Wv[u] = pw_at(x);
          }
#pragma unroll
          for (int u = 0; u < kHalf; ++u) {
            if (e + h + u > eL) break;
            const int L = e + h + u - r + 1;
            const double S = Pv[u] - base, R = WEIGHTED ? Wv[u] - wbase : (double)L;
            if (DIP && !(S < 0.0)) continue;
            const double den = R * (Wd - R);
            const double num = S * S;
            if (num < thr * den) continue;
            // Rare: the run passed the screen; its edges must be admissible.
            const int x = e + h + u >= nk ? e + h + u - nk : e + h + u;
            const int next = x + 1 == nk ? 0 : x + 1;
            const double pe = sph[x], pn = sph[next];
            if (!(fwd_phase(pe, pn, x, next) > 0.0)) continue;
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
              const double vr = num / den * (1.0 - 0x1p-20);  // relaxed
              thr = fmax(thr, vr);
              __hip_atomic_fetch_max(&s_theta, (unsigned long long)__double_as_longlong(vr),
                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
          }
        }
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

}  // namespace

int64_t unbinned_lds_bytes(int n, bool weighted) {
  const int64_t N = unbinned_stride(n);
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

}  // namespace bls
