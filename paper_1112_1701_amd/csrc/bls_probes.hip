// Micro-benchmarks of the gfx950 rates the search kernel's design rests on
// (libbls_probes.so, include/bls_probes.h): LDS atomic throughput by width
// and type at random addresses, LDS 64-bit read throughput by lane pattern,
// and VALU issue rates of independent FP32 / FP64 / integer chains.  Each
// probe is one timed launch of a kernel whose every access stays inside its
// own LDS array and whose results are written out, so nothing is optimised
// away.  Measurement tooling: the search never calls it.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "../../include/bls_probes.h"

namespace {

constexpr int kBlock = 256;
constexpr int kWords = 4096;  // LDS words (8 B) of the atomic and read probes

// xorshift32 per lane: addresses spread over the histogram.
__device__ inline unsigned next_rand(unsigned &s) {
  s ^= s << 13;
  s ^= s >> 17;
  s ^= s << 5;
  return s;
}

template <int KIND>
__global__ __launch_bounds__(kBlock) void lds_atomic_kernel(int iters, int span,
                                                            unsigned long long *out) {
  __shared__ unsigned long long h[kWords];
  for (int i = threadIdx.x; i < kWords; i += kBlock) h[i] = 0ull;
  __syncthreads();
  unsigned s = 2654435761u * (blockIdx.x * kBlock + threadIdx.x + 1);
  const unsigned mask = (unsigned)(span - 1);  // span: a power of two <= kWords
  for (int it = 0; it < iters; ++it) {
    const unsigned a = next_rand(s) & mask;
    if (KIND == BLS_PROBE_ADD_U64) {
      __hip_atomic_fetch_add(&h[a], 1ull + a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else if (KIND == BLS_PROBE_ADD_U32) {
      __hip_atomic_fetch_add(reinterpret_cast<unsigned *>(h) + a, 1u + a, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
      __hip_atomic_fetch_add(reinterpret_cast<float *>(h) + a, 1.0f, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_WORKGROUP);
    }
  }
  __syncthreads();
  unsigned long long acc = 0ull;
  for (int i = threadIdx.x; i < kWords; i += kBlock) acc += h[i];
  out[blockIdx.x * kBlock + threadIdx.x] = acc;
}

// 64-bit reads: lane l of each 16-lane group reads word base + l * lane_stride
// (+ a per-iteration offset), i.e. the bank pattern of one clock of the scan.
__global__ __launch_bounds__(kBlock) void lds_read_kernel(int iters, int lane_stride,
                                                          unsigned long long *out) {
  __shared__ unsigned long long h[kWords];
  for (int i = threadIdx.x; i < kWords; i += kBlock) h[i] = (unsigned long long)i * 3u;
  __syncthreads();
  const int l = threadIdx.x & 15;
  const int base = (threadIdx.x >> 4) & 7;
  unsigned long long acc = 0ull;
  for (int it = 0; it < iters; ++it) {
    const int a = (base + l * lane_stride + (it & 63)) & (kWords - 1);
    acc += h[a];
  }
  out[blockIdx.x * kBlock + threadIdx.x] = acc;
}

// VALU issue: kChains independent dependency chains per lane.
constexpr int kChains = 8;

template <int KIND>
__global__ __launch_bounds__(kBlock) void valu_kernel(int iters, double *out) {
  const int tid = blockIdx.x * kBlock + threadIdx.x;
  if (KIND == BLS_PROBE_FMA_F32 || KIND == BLS_PROBE_ADD_F32V) {
    float v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = 1.0f + 1e-7f * (float)(tid + c);
    // a per-lane addend in a register: no literal operand in the loop
    const float k = 1e-8f * (float)(threadIdx.x & 7);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < kChains; ++c)
        v[c] = KIND == BLS_PROBE_FMA_F32 ? fmaf(v[c], 0.5f, k) : v[c] + k;
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[tid] = s;
  } else if (KIND == BLS_PROBE_MUL_F64) {
    double v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = 1.0 + 1e-12 * (double)(tid + c);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) v[c] = v[c] * 0.9999999999;
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[tid] = s;
  } else {
    unsigned v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = (unsigned)(tid * 7 + c);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) v[c] = (v[c] << 3) + 0x9E3779B9u;
    }
    unsigned s = 0u;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out[tid] = (double)s;
  }
}

int timed(hipEvent_t a, hipEvent_t b, double *ms) {
  hipError_t e = hipEventSynchronize(b);
  float f = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
  *ms = f;
  return (int)e;
}

template <class Launch>
int run(int grid, size_t out_bytes, Launch launch, double *ms) {
  void *out = nullptr;
  hipError_t e = hipMalloc(&out, out_bytes);
  if (e != hipSuccess) return (int)e;
  hipEvent_t a = nullptr, b = nullptr;
  if ((e = hipEventCreate(&a)) == hipSuccess && (e = hipEventCreate(&b)) == hipSuccess) {
    launch(out);  // warm-up
    (void)hipEventRecord(a, nullptr);
    launch(out);
    (void)hipEventRecord(b, nullptr);
    e = (hipError_t)timed(a, b, ms);
    if (e == hipSuccess) e = hipGetLastError();
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(out);
  (void)grid;
  return (int)e;
}

}  // namespace

extern "C" int bls_probe_lds_atomic(int kind, int span, int iters, int grid, double *ms) {
  if (!ms || iters < 1 || grid < 1 || span < 1 || span > kWords || (span & (span - 1)) ||
      (kind != BLS_PROBE_ADD_U64 && kind != BLS_PROBE_ADD_U32 && kind != BLS_PROBE_ADD_F32))
    return -1;
  const size_t bytes = (size_t)grid * kBlock * sizeof(unsigned long long);
  return run(grid, bytes, [&](void *o) {
    auto *out = static_cast<unsigned long long *>(o);
    if (kind == BLS_PROBE_ADD_U64)
      hipLaunchKernelGGL(lds_atomic_kernel<BLS_PROBE_ADD_U64>, dim3(grid), dim3(kBlock), 0, 0,
                         iters, span, out);
    else if (kind == BLS_PROBE_ADD_U32)
      hipLaunchKernelGGL(lds_atomic_kernel<BLS_PROBE_ADD_U32>, dim3(grid), dim3(kBlock), 0, 0,
                         iters, span, out);
    else
      hipLaunchKernelGGL(lds_atomic_kernel<BLS_PROBE_ADD_F32>, dim3(grid), dim3(kBlock), 0, 0,
                         iters, span, out);
  }, ms);
}

extern "C" int bls_probe_lds_read(int lane_stride, int iters, int grid, double *ms) {
  if (!ms || iters < 1 || grid < 1 || lane_stride < 0 || lane_stride > 256) return -1;
  const size_t bytes = (size_t)grid * kBlock * sizeof(unsigned long long);
  return run(grid, bytes, [&](void *o) {
    hipLaunchKernelGGL(lds_read_kernel, dim3(grid), dim3(kBlock), 0, 0, iters, lane_stride,
                       static_cast<unsigned long long *>(o));
  }, ms);
}

extern "C" int bls_probe_valu(int kind, int iters, int grid, double *ms) {
  if (!ms || iters < 1 || grid < 1 ||
      (kind != BLS_PROBE_FMA_F32 && kind != BLS_PROBE_MUL_F64 && kind != BLS_PROBE_MAD_U32 &&
       kind != BLS_PROBE_ADD_F32V))
    return -1;
  const size_t bytes = (size_t)grid * kBlock * sizeof(double);
  return run(grid, bytes, [&](void *o) {
    auto *out = static_cast<double *>(o);
    if (kind == BLS_PROBE_FMA_F32)
      hipLaunchKernelGGL(valu_kernel<BLS_PROBE_FMA_F32>, dim3(grid), dim3(kBlock), 0, 0, iters,
                         out);
    else if (kind == BLS_PROBE_MUL_F64)
      hipLaunchKernelGGL(valu_kernel<BLS_PROBE_MUL_F64>, dim3(grid), dim3(kBlock), 0, 0, iters,
                         out);
    else if (kind == BLS_PROBE_ADD_F32V)
      hipLaunchKernelGGL(valu_kernel<BLS_PROBE_ADD_F32V>, dim3(grid), dim3(kBlock), 0, 0, iters,
                         out);
    else
      hipLaunchKernelGGL(valu_kernel<BLS_PROBE_MAD_U32>, dim3(grid), dim3(kBlock), 0, 0, iters,
                         out);
  }, ms);
}
