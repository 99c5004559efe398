// gfx950 kernels of the high-variability pre-search of a field (per-star
// RMS, then sigma-clipped statistics per chip and magnitude bin).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "bls_block.h"
#include "bls_device.h"
#include "../../include/bls.h"

namespace bls {
namespace {

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

}  // namespace

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

}  // namespace bls
