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
  const double harm[5] = {1.0, 0.5, 2.0, 1.0 / 3.0, 3.0};
  auto suppressed = [&](double Pp, double P) {
    bool off = false;
    for (int h = 0; h < 5; ++h) {
      const double cp = harm[h] * P;
      if (fabs(Pp - cp) <= a.window * cp) off = true;
    }
    return off;
  };
  // A thread offers its largest entry that is neither taken nor suppressed
  // by a peak so far.  The entries' periods are read lazily: only the
  // current entry's (top[0]), tested against the peaks it has not met yet
  // when it is about to be offered.  Read for all entries at once, the
  // periods cost more than twice the pass (random reads that together touch
  // nearly every line of the period grid in every workgroup); most entries
  // are never offered.  An entry that is taken or suppressed is popped and
  // the next one becomes current; the next entry's period is read one pop
  // ahead, so that a pop does not wait on memory.
  double curP = top[0] ? per[key_index(top[0])] : 0.0;
  double nextP = top[1] ? per[key_index(top[1])] : 0.0;
  auto pop = [&]() {
#pragma unroll
    for (int i = 0; i + 1 < kDetList; ++i) top[i] = top[i + 1];
    top[kDetList - 1] = 0ull;
    curP = nextP;
    nextP = top[1] ? per[key_index(top[1])] : 0.0;
  };
  int tested = 0;               // peaks the current entry has been tested against
  bool more = npos > kDetList;  // the slice holds values the list dropped

  int k = 0;
  for (; k < a.max_peaks; ++k) {
    // The current entry against the peaks it has not met; suppressed ones
    // give way to the next.
    while (top[0] != 0ull && tested < k) {
      bool off = false;
      for (int j = tested; j < k; ++j) off = off || suppressed(curP, s_peak[j]);
      if (!off) {
        tested = k;
        break;
      }
      pop();
      tested = 0;
    }
    if (top[0] == 0ull && more) {
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
      curP = top[0] ? per[key_index(top[0])] : 0.0;
      nextP = top[1] ? per[key_index(top[1])] : 0.0;
      tested = k;  // the refill tested its entries against every peak so far
    }
    const unsigned long long offer = top[0];
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
    if (mine) {  // the owner's entry is taken
      pop();
      tested = 0;
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

}  // namespace

int launch_detect(const DetectArgs &a, void *stream) {
  if (a.ncurves <= 0) return 0;
  hipLaunchKernelGGL(detect_kernel, dim3(a.ncurves), dim3(kBlock), 0, (hipStream_t)stream, a);
  return (int)hipGetLastError();
}

}  // namespace bls
