// gfx950 kernels of the eclipse detection efficiency of a cadence (the
// chance that at least two eclipses of a target at a given period fall on
// observations, section 5).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "bls_block.h"
#include "bls_device.h"
#include "../../include/bls.h"

namespace bls {
namespace {

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
    // (eight loads in flight per thread: a shared grid is checked by one
    // workgroup)
#pragma unroll 8
    for (int64_t i = tid; i < wd->nperiods; i += kBlock) {
      const double P = a.periods[wd->p_off + i];
      if (!isfinite(P) || !(P > 0.0)) badp = 1.0;
    }
  }
  const int anybadp = __syncthreads_or(badp > 0.0 ? 1 : 0);
  block_sum2(bad, kept, sa, sb);
  block_minmax(tmin, tmax, sa, sb);
  if (tid == 0) {
    wd->t0 = tmin;
    wd->dmax = tmax - tmin;
    wd->status = bad > 0.0 ? kCurveBadData
                 : kept < 1.0 ? kCurveTooFew
                 : anybadp ? kCurveBadPeriod
                           : kCurveOk;
  }
}

constexpr int kCycleEmptyLo = 0x3fffffff;   // min of an empty bin
constexpr int kCycleEmptyHi = -0x3fffffff;  // max of an empty bin

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

}  // namespace

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


int window_blocks_per_cu(int lds_bytes, int *blocks) {
  const void *fn = reinterpret_cast<const void *>(&window_kernel<1>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
  if (e != hipSuccess) return (int)e;
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, (size_t)lds_bytes);
}

}  // namespace bls
