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
// No FP contraction anywhere (-ffp-contract=off): the phase is computed with
// exactly the FP64 operation sequence of its definition so that every point
// falls into the same bin as in an FP64 evaluation.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "bls_device.h"

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
  block_isum2(cnt, bad, ia, ib);
  block_sum2(sw, swx, sa, sb);
  double tmax_unused = -INFINITY;
  block_minmax(tmin, tmax_unused, sa, sb);

  if (bad != 0 || cnt < 2 || !(sw > 0.0) || !isfinite(sw)) {
    if (tid == 0) {
      cd->status = bad ? kCurveBadData : kCurveTooFew;
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

  // Pass 3: encode.
  long long sqw = 0, unused = 0;
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
    a.q[off + i] = __double2int_rn(ldexp(v, es));
    if (weighted) {
      const int qwi = __double2int_rn(ldexp(wi, ew));
      a.qw[off + i] = qwi;
      sqw += qwi;
    }
  }
  block_isum2(sqw, unused, ia, ib);

  if (tid == 0) {
    cd->t0 = tmin;
    cd->W = W;
    cd->xbar = xbar;
    cd->es = es;
    cd->ew = ew;
    cd->out_scale = ldexp(1.0, ew - es);
    cd->Wf = weighted ? (float)ldexp((double)sqw, -qbits) : (float)cnt;
    cd->n_eff = (int32_t)cnt;
    cd->status = kCurveOk;
  }
}

// ---------------------------------------------------------------- search
// One bin word holds (count << shift) + sum of signed fixed-point values;
// the sum needs fewer than shift - 1 bits, so it is the sign-extended low
// field and the count is what remains above it.
__device__ inline void decode_word(unsigned long long u, int shift, long long &sum,
                                   unsigned long long &count) {
  const int hi = 64 - shift;
  sum = ((long long)(u << hi)) >> hi;
  count = (u - (unsigned long long)sum) >> shift;
}

// Phase bin with the FP64 operation order of the definition.
__device__ inline int phase_bin(double d, double f, double nbd, int nbm1) {
  const double c = d * f;
  const double ph = c - floor(c);
  const int b = (int)(ph * nbd);
  return min(max(b, 0), nbm1);
}

template <bool WEIGHTED, bool FULL>
__device__ inline void fold_chunk(const SearchArgs &a, const CurveDesc &cd, int64_t base,
                                  int np, const double *s_f, unsigned long long *s_hist,
                                  int HB) {
  const int tid = threadIdx.x;
  const int64_t off = cd.n_off;
  const int64_t n = cd.n;
  const int nb = cd.nbins;
  const double nbd = (double)nb;
  const unsigned long long one = 1ull << cd.shift;
  double d[kPPT];
  unsigned long long va[kPPT];
  unsigned long long vb[kPPT];
  bool ok[kPPT];
#pragma unroll
  for (int r = 0; r < kPPT; ++r) {
    const int64_t i = base + (int64_t)r * kBlock + tid;
    ok[r] = FULL || i < n;
    d[r] = 0.0;
    va[r] = 0;
    vb[r] = 0;
    if (ok[r]) {
      d[r] = a.dt[off + i];
      const long long qi = a.q[off + i];
      if (WEIGHTED) {
        const int qwi = a.qw[off + i];
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
    unsigned long long *h = s_hist + (size_t)t * HB * wpb;
#pragma unroll
    for (int r = 0; r < kPPT; ++r) {
      if (FULL || ok[r]) {
        const int b = phase_bin(d[r], f, nbd, nb - 1);
        __hip_atomic_fetch_add(h + b * wpb, va[r], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
        if (WEIGHTED)
          __hip_atomic_fetch_add(h + b * wpb + 1, vb[r], __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
  }
}

// (t, j) of a flattened index over np rows of nb entries.
__device__ inline void split_index(int idx, int nb, float inv_nb, int &t, int &j) {
  t = (int)((float)idx * inv_nb);
  j = idx - t * nb;
  if (j < 0) {
    --t;
    j += nb;
  } else if (j >= nb) {
    ++t;
    j -= nb;
  }
}

template <bool WEIGHTED, bool DIP>
__global__ __launch_bounds__(kBlock) void search_kernel(SearchArgs a) {
  extern __shared__ __align__(16) unsigned long long s_hist[];
  __shared__ double s_f[kTileMax];
  __shared__ unsigned long long s_best[kTileMax];
  __shared__ long long s_item;
  __shared__ int s_curve;
  __shared__ int s_tile;

  const int tid = threadIdx.x;
  constexpr int wpb = WEIGHTED ? 2 : 1;

  for (;;) {
    if (tid == 0) {
      const unsigned long long it =
          __hip_atomic_fetch_add(a.counter, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_item = (long long)it;
      if ((long long)it < a.nitems) {
        int lo = 0, hi = a.nseg - 1;  // last s with seg_start[s] <= it
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (a.seg_start[mid] <= (long long)it)
            lo = mid;
          else
            hi = mid - 1;
        }
        s_curve = a.seg_curve[lo];
        s_tile = a.seg_tile0[lo] + (int)((long long)it - a.seg_start[lo]);
      }
    }
    __syncthreads();
    if (s_item >= a.nitems) break;
    // Item values are uniform: keep them (and the curve record) scalar.
    const int c = __builtin_amdgcn_readfirstlane(s_curve);
    const int tile = __builtin_amdgcn_readfirstlane(s_tile);
    __syncthreads();  // everyone has read the item before thread 0 takes the next

    const CurveDesc cd = a.curves[c];
    const int p0 = tile * cd.tile;
    const int np = min(cd.tile, cd.nperiods - p0);
    if (np <= 0) continue;

    if (cd.status != kCurveOk) {
      for (int t = tid; t < np; t += kBlock) {
        const int64_t r = cd.r_off + p0 + t;
        a.sr[r] = NAN;
        a.depth[r] = NAN;
        a.jstart[r] = -1;
        a.kwidth[r] = -1;
      }
      continue;
    }

    const int nb = cd.nbins;
    const int kmin = cd.kmin;
    const int kmax = cd.kmax;
    const int HB = nb + kmax - 1;  // bins plus the wrap-around copy

    // Clear the tile's histograms; frequencies f = 1/P (IEEE division).
    for (int i = tid; i < np * nb * wpb; i += kBlock) {
      int t, b;
      split_index(i / wpb, nb, 1.0f / (float)nb, t, b);
      s_hist[((size_t)t * HB + b) * wpb + (i % wpb)] = 0ull;
    }
    if (tid < np) {
      s_f[tid] = 1.0 / a.periods[cd.p_off + p0 + tid];
      s_best[tid] = 0ull;
    }
    __syncthreads();

    // Fold and bin: points in registers, reused for every period of the tile.
    for (int64_t base = 0; base < cd.n; base += (int64_t)kBlock * kPPT) {
      if (base + (int64_t)kBlock * kPPT <= cd.n)
        fold_chunk<WEIGHTED, true>(a, cd, base, np, s_f, s_hist, HB);
      else
        fold_chunk<WEIGHTED, false>(a, cd, base, np, s_f, s_hist, HB);
    }
    __syncthreads();

    // Exact integer bins -> FP32 (count, sum) in place.
    const float inv_nb = 1.0f / (float)nb;
    const float qscale = ldexpf(1.0f, -cd.qbits);
    for (int i = tid; i < np * nb; i += kBlock) {
      int t, b;
      split_index(i, nb, inv_nb, t, b);
      unsigned long long *w = s_hist + ((size_t)t * HB + b) * wpb;
      long long sa;
      unsigned long long ca;
      decode_word(w[0], cd.shift, sa, ca);
      if (WEIGHTED) {
        const long long sb = (long long)w[1];
        float4 *o = reinterpret_cast<float4 *>(w);
        *o = make_float4((float)sa * qscale, (float)sb * qscale, (float)ca, 0.0f);
      } else {
        float2 *o = reinterpret_cast<float2 *>(w);
        *o = make_float2((float)ca, (float)sa * qscale);
      }
    }
    __syncthreads();
    // Wrap-around: bins 0 .. kmax-2 repeated after bin nb-1.
    if (kmax > 1) {
      const int ext = kmax - 1;
      const float inv_ext = 1.0f / (float)ext;
      for (int i = tid; i < np * ext; i += kBlock) {
        int t, e;
        split_index(i, ext, inv_ext, t, e);
        unsigned long long *src = s_hist + ((size_t)t * HB + e) * wpb;
        unsigned long long *dst = s_hist + ((size_t)t * HB + nb + e) * wpb;
        dst[0] = src[0];
        if (WEIGHTED) dst[1] = src[1];
      }
    }
    __syncthreads();

    // Box scan: lane task = (period t, start bin j); running sums over widths.
    const float Wf = cd.Wf;
    const float nmax1 = (float)(cd.n_eff - 1);
    const float mipf = (float)a.min_in_points;
    const bool mip1 = a.min_in_points <= 1;
    for (int task = tid; task < np * nb; task += kBlock) {
      int t, j;
      split_index(task, nb, inv_nb, t, j);
      float R = 0.0f, S = 0.0f, C = 0.0f;
      float bn = 0.0f, bd = 1.0f;
      int bm = -1;
      if (WEIGHTED) {
        const float4 *h = reinterpret_cast<const float4 *>(s_hist) + (size_t)t * HB + j;
        int m = 0;
        for (; m < kmin - 1; ++m) {
          const float4 e = h[m];
          R += e.x;
          S += e.y;
          C += e.z;
        }
        for (; m < kmax; ++m) {
          const float4 e = h[m];
          R += e.x;
          S += e.y;
          C += e.z;
          const float den = R * (Wf - R);
          const float num = S * S;
          bool better = (num * bd > bn * den) & (C <= nmax1) & (C >= mipf) & (den > 0.0f);
          if (DIP) better &= (S < 0.0f);
          bn = better ? num : bn;
          bd = better ? den : bd;
          bm = better ? m : bm;
        }
      } else {
        const float2 *h = reinterpret_cast<const float2 *>(s_hist) + (size_t)t * HB + j;
        int m = 0;
        for (; m < kmin - 1; ++m) {
          const float2 e = h[m];
          R += e.x;
          S += e.y;
        }
        if (mip1) {
          for (; m < kmax; ++m) {
            const float2 e = h[m];
            R += e.x;
            S += e.y;
            const float dd = Wf - R;
            const float den = R * dd;
            const float num = S * S;
            bool better = (num * bd > bn * den) & (dd >= 1.0f);
            if (DIP) better &= (S < 0.0f);
            bn = better ? num : bn;
            bd = better ? den : bd;
            bm = better ? m : bm;
          }
        } else {
          for (; m < kmax; ++m) {
            const float2 e = h[m];
            R += e.x;
            S += e.y;
            const float dd = Wf - R;
            const float den = R * dd;
            const float num = S * S;
            bool better = (num * bd > bn * den) & (dd >= 1.0f) & (R >= mipf);
            if (DIP) better &= (S < 0.0f);
            bn = better ? num : bn;
            bd = better ? den : bd;
            bm = better ? m : bm;
          }
        }
      }
      (void)C;
      if (bm >= 0) {
        const float v = bn / bd;
        const unsigned idx = (unsigned)((bm + 1) * nb + j);
        const unsigned long long key =
            ((unsigned long long)__float_as_uint(v) << 32) | (unsigned long long)(0xFFFFFFFFu - idx);
        __hip_atomic_fetch_max(&s_best[t], key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
    }
    __syncthreads();

    // Per period: re-sum the winning box in scan order, write the result.
    if (tid < np) {
      const int t = tid;
      const int p = p0 + t;
      const int64_t r = cd.r_off + p;
      const unsigned long long key = s_best[t];
      float srf = 0.0f;
      if (key == 0ull) {
        a.sr[r] = 0.0f;
        a.depth[r] = NAN;
        a.jstart[r] = -1;
        a.kwidth[r] = -1;
      } else {
        const unsigned idx = 0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull);
        const int k = (int)(idx / (unsigned)nb);
        const int j = (int)(idx - (unsigned)k * (unsigned)nb);
        float R = 0.0f, S = 0.0f;
        if (WEIGHTED) {
          const float4 *h = reinterpret_cast<const float4 *>(s_hist) + (size_t)t * HB + j;
          for (int m = 0; m < k; ++m) {
            R += h[m].x;
            S += h[m].y;
          }
        } else {
          const float2 *h = reinterpret_cast<const float2 *>(s_hist) + (size_t)t * HB + j;
          for (int m = 0; m < k; ++m) {
            R += h[m].x;
            S += h[m].y;
          }
        }
        const double Rd = (double)R;
        const double den = Rd * ((double)Wf - Rd);
        const double Sd = (double)S;
        const double sr = sqrt(Sd * Sd / den) * cd.out_scale;
        const double depth = -Sd * (double)Wf / den * cd.out_scale;
        srf = (float)sr;
        a.sr[r] = srf;
        a.depth[r] = (float)depth;
        a.jstart[r] = j;
        a.kwidth[r] = k;
      }
      const unsigned long long ckey = ((unsigned long long)__float_as_uint(srf) << 32) |
                                      (unsigned long long)(0xFFFFFFFFu - (unsigned)p);
      __hip_atomic_fetch_max(a.best_key + c, ckey, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
  }
}

__global__ void fill_kernel(unsigned long long *counter, unsigned long long *keys, int32_t nkeys) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && counter) *counter = 0ull;
  if (i < nkeys) keys[i] = 0ull;
}

__global__ void best_index_kernel(unsigned long long *keys, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const unsigned long long k = keys[i];
    keys[i] = (unsigned long long)(0xFFFFFFFFu - (unsigned)(k & 0xFFFFFFFFull));
  }
}

template <bool W, bool D>
const void *search_fn() {
  return reinterpret_cast<const void *>(&search_kernel<W, D>);
}

const void *pick(bool weighted, bool dip) {
  if (weighted) return dip ? search_fn<true, true>() : search_fn<true, false>();
  return dip ? search_fn<false, true>() : search_fn<false, false>();
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
  const void *fn = pick(weighted, dip_only);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, a.hist_bytes);
  if (e != hipSuccess) return (int)e;
  void *args[] = {const_cast<SearchArgs *>(&a)};
  e = hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, (size_t)a.hist_bytes,
                      (hipStream_t)stream);
  if (e != hipSuccess) return (int)e;
  return (int)hipGetLastError();
}

int launch_best_index(unsigned long long *keys, int32_t n, void *stream) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(best_index_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                     keys, n);
  return (int)hipGetLastError();
}

int search_blocks_per_cu(bool weighted, bool dip_only, int hist_bytes, int *blocks) {
  const void *fn = pick(weighted, dip_only);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, hist_bytes);
  if (e != hipSuccess) return (int)e;
  return (int)hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kBlock, (size_t)hist_bytes);
}

}  // namespace bls
