// gfx950 kernel of the detection statistics of a periodogram (the SDE of
// the BLS peak and the strongest peaks with their harmonics suppressed).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "bls_block.h"
#include "bls_device.h"
#include "../../include/bls.h"

namespace bls {
namespace {

// ------------------------------------------------------------- detection
// One workgroup per curve: mean and population deviation of SR (FP64), then
// peaks largest first, a peak at P suppressing every P' within
// window * hP of hP for h in {1, 1/2, 2, 1/3, 3}.
//
// Peaks without a pass per peak.  The deviation pass reads a thread's slice
// of periods (p = tid + kBlock j) kDetBatch values at a time, and batch lane
// u keeps a bucket: the two largest keys among the slice's values with
// j = u (mod kDetBatch), positive SR only.  A key is (SR bits, ~p): unique,
// and ordered as the peaks are chosen (larger SR, then the smaller index).
// A thread's current entry is its largest bucket key; before it is offered
// it is tested against the peaks it has not met (its period is read then).
// The workgroup takes the largest offer.  An entry that is taken or
// suppressed leaves its bucket, whose next key is its second, or, once that
// is used up, the largest one below it, found (with the one after) by
// rescanning the bucket's values (every kDetBatch-th of the slice).  A
// thread so always offers the largest free key of its slice, and the peaks
// are exactly those of a peak-by-peak search.  In the pass a bucket costs a
// compare or two per value; the sorted list of 12 keys this replaces cost a
// 12-step chain per inserted value, about 34 of a 78-value slice, which was
// most of the kernel's time.  (Buckets of one key rescan twice as often;
// three or four keys, or 16 or 32 buckets, cost more in registers than they
// save.)
constexpr int kDetBatch = 8;   // loads in flight per pass; buckets per thread
constexpr int kDetRescan = 4;  // loads in flight per bucket rescan

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
  // largest value; and its buckets.  The workgroup merges the threads'
  // statistics the same way, in a fixed tree.
  auto keyof = [](float v, int64_t p) {
    return ((unsigned long long)__float_as_uint(v) << 32) |
           (unsigned long long)(0xFFFFFFFFu - (unsigned)p);
  };
  // bkey[u]: the bucket's largest key; bkey2[u]: the next one below it (0:
  // none known, found by a rescan when needed)
  unsigned long long bkey[kDetBatch], bkey2[kDetBatch];
#pragma unroll
  for (int u = 0; u < kDetBatch; ++u) {
    bkey[u] = 0ull;
    bkey2[u] = 0ull;
  }
  double cn = 0.0, cmean = 0.0, cm2 = 0.0, mx = -INFINITY;
  auto take = [&](int u, float v, int64_t p) {
    mx = fmax(mx, (double)v);
    if (v > 0.0f) {
      const unsigned long long key = keyof(v, p);
      if (key > bkey2[u]) {
        const bool top = key > bkey[u];
        bkey2[u] = top ? bkey[u] : key;
        bkey[u] = top ? key : bkey[u];
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
    for (int u = 0; u < kDetBatch; ++u) take(u, v[u], p0 + (int64_t)u * kBlock);
  }
  // the tail: fewer than kDetBatch values, lane u's in bucket u
#pragma unroll
  for (int u = 0; u < kDetBatch - 1; ++u) {
    const int64_t p = p0 + (int64_t)u * kBlock;
    if (p < m) {
      const float v = sr[p];
      cn = cn + 1.0;
      const double delta = (double)v - cmean;
      cmean = cmean + delta / cn;
      cm2 = cm2 + delta * ((double)v - cmean);
      take(u, v, p);
    }
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
  const double harm[5] = {1.0, 0.5, 2.0, 1.0 / 3.0, 3.0};
  auto suppressed = [&](double Pp, double P) {
    bool off = false;
    for (int h = 0; h < 5; ++h) {
      const double cp = harm[h] * P;
      if (fabs(Pp - cp) <= a.window * cp) off = true;
    }
    return off;
  };
  // The two largest keys below `bound` among bucket u's values (0: none).
  auto rescan = [&](int u, unsigned long long bound, unsigned long long &best,
                    unsigned long long &second) {
    const int64_t step = (int64_t)kDetBatch * kBlock;
    best = 0ull;
    second = 0ull;
    auto see = [&](float v, int64_t p) {
      if (v > 0.0f) {
        const unsigned long long key = keyof(v, p);
        if (key < bound && key > second) {
          const bool top = key > best;
          second = top ? best : key;
          best = top ? key : best;
        }
      }
    };
    int64_t q = tid + (int64_t)u * kBlock;
    for (; q + (kDetRescan - 1) * step < m; q += kDetRescan * step) {
      float v[kDetRescan];
#pragma unroll
      for (int r = 0; r < kDetRescan; ++r) v[r] = sr[q + r * step];
#pragma unroll
      for (int r = 0; r < kDetRescan; ++r) see(v[r], q + r * step);
    }
    for (; q < m; q += step) see(sr[q], q);
  };
  // The current entry: the largest bucket key, its bucket and period, and
  // how many peaks it has been tested against.
  unsigned long long ckey = 0ull;
  int cu = 0, tested = 0;
  double curP = 0.0;
  auto pick = [&]() {
    ckey = 0ull;
    cu = 0;
#pragma unroll
    for (int u = 0; u < kDetBatch; ++u)
      if (bkey[u] > ckey) {
        ckey = bkey[u];
        cu = u;
      }
    curP = ckey ? per[key_index(ckey)] : 0.0;
    tested = 0;
  };
  auto pop = [&]() {  // the current entry leaves its bucket
    unsigned long long b1 = 0ull, b2 = 0ull;
#pragma unroll
    for (int u = 0; u < kDetBatch; ++u)
      if (u == cu) b1 = bkey2[u];
    if (b1 == 0ull) rescan(cu, ckey, b1, b2);  // the next key is not known
#pragma unroll
    for (int u = 0; u < kDetBatch; ++u)
      if (u == cu) {
        bkey[u] = b1;
        bkey2[u] = b2;
      }
    pick();
  };
  pick();

  int k = 0;
  for (; k < a.max_peaks; ++k) {
    // The current entry against the peaks it has not met; a suppressed one
    // gives way to the next.
    while (ckey != 0ull && tested < k) {
      bool off = false;
      for (int j = tested; j < k; ++j) off = off || suppressed(curP, s_peak[j]);
      if (!off) {
        tested = k;
        break;
      }
      pop();
    }
    const unsigned long long offer = ckey;
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
    const bool mine = offer == key;  // keys are unique: one owner
    if (mine) s_peak[k] = curP;
    __syncthreads();
    const int64_t pk = key_index(key);
    const float vk = __uint_as_float((unsigned)(key >> 32));
    if (tid == 0) {
      out->peak_index[k] = pk;
      out->peak_sr[k] = vk;
      out->peak_sde[k] = sd > 0.0 ? (float)(((double)vk - mean) / sd) : 0.0f;
    }
    if (mine) pop();  // the owner's entry is taken
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

}  // namespace

int launch_detect(const DetectArgs &a, void *stream) {
  if (a.ncurves <= 0) return 0;
  hipLaunchKernelGGL(detect_kernel, dim3(a.ncurves), dim3(kBlock), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace bls
