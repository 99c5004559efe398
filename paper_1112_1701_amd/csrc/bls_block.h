// Workgroup and wave reductions shared by the kernels.  Every reduction
// runs in a fixed order (a fixed tree over threads, fixed DPP steps over
// lanes), so results do not depend on scheduling.
#pragma once
#include <hip/hip_runtime.h>

#include <math.h>

#include "bls_device.h"

namespace bls {
namespace {

// Sums of two values over the workgroup.
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

// Minimum and maximum over the workgroup.
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

}  // namespace
}  // namespace bls
