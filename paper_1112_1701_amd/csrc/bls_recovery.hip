// Injection-recovery of one cadence (bls_injection_recovery_device): box
// eclipses injected into copies of the cadence on the device, every copy
// searched by the batched search and its periodogram's detection statistics
// taken, then the recovery rule applied.  This is the paper's detection-
// efficiency simulation on real cadences (section 5, Discussion and
// conclusions) taken through the search itself.
//
//   cadence_t0_kernel  one workgroup: t0 = min kept time of the cadence
//   inject_kernel      per (injection, point): the batch's times, weights
//                      and injected fluxes, injection-major
//
// The injected fluxes follow the FP64 operation order of the definition in
// include/bls.h, so the device and an FP64 evaluation put exactly the same
// points in eclipse.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "bls_plan.h"

namespace bls {
namespace {

struct InjParam {
  double f;       // 1 / P (IEEE division on the host)
  double phase;   // start phase in [0, 1)
  double q;       // duty cycle
  double depth;
};

__global__ __launch_bounds__(kBlock) void cadence_t0_kernel(const double *t, const double *w,
                                                            int64_t n, double *t0) {
  __shared__ double s[kBlock];
  double m = INFINITY;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) {
    const bool keep = w == nullptr || w[i] > 0.0;
    if (keep) m = fmin(m, t[i]);
  }
  s[threadIdx.x] = m;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) s[threadIdx.x] = fmin(s[threadIdx.x], s[threadIdx.x + k]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *t0 = s[0];
}

struct InjectArgs {
  const double *t;
  const double *w;
  const double *base;
  const InjParam *prm;
  const double *t0;
  int64_t n;
  int64_t total;      // ninj * n
  double *t_out;
  double *w_out;      // nullptr without weights
  double *x_out;
};

__global__ __launch_bounds__(kBlock) void inject_kernel(InjectArgs a) {
  const double t0 = *a.t0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x; g < a.total; g += stride) {
    const int64_t k = g / a.n;
    const int64_t i = g - k * a.n;
    const double ti = a.t[i];
    const double wi = a.w ? a.w[i] : 1.0;
    const bool keep = a.w == nullptr || wi > 0.0;
    const InjParam p = a.prm[k];
    const double d = ti - t0;
    const double c = d * p.f;
    const double u = c - p.phase;
    const double v = u - floor(u);
    const double b = a.base[g];
    a.t_out[g] = ti;
    if (a.w_out) a.w_out[g] = wi;
    a.x_out[g] = (keep && v < p.q) ? b - p.depth : b;
  }
}

int fail(bls_plan *p, int st, const char *msg) { return set_error(p, st, std::string(msg)); }

}  // namespace
}  // namespace bls

using namespace bls;

extern "C" int bls_injection_recovery_device(bls_plan *p, const bls_recovery_config *cf,
                                             const bls_recovery_results *out) {
  if (!p) return BLS_ERR_INVALID_ARG;
  p->last_error.clear();
  if (!cf || !out || !out->recovered)
    return fail(p, BLS_ERR_INVALID_ARG, "config and out->recovered are required");
  const int32_t ninj = cf->ninj;
  const int64_t n = cf->n;
  if (ninj < 1 || n < 2 || !cf->times || !cf->base_flux || !cf->inj_period ||
      !cf->inj_phase || !cf->inj_q || !cf->inj_depth || !cf->periods || cf->nperiods < 1)
    return fail(p, BLS_ERR_INVALID_ARG,
                "need ninj >= 1, n >= 2, nperiods >= 1 and every input array");
  if (!(cf->window >= 0.0) || !isfinite(cf->window) || isnan(cf->sde_threshold) ||
      !(cf->ptol >= 0.0) || !isfinite(cf->ptol))
    return fail(p, BLS_ERR_INVALID_ARG, "need a finite window >= 0, a threshold, ptol >= 0");
  std::vector<InjParam> prm(ninj);
  for (int32_t k = 0; k < ninj; ++k) {
    const double P = cf->inj_period[k], ph = cf->inj_phase[k], q = cf->inj_q[k],
                 dep = cf->inj_depth[k];
    if (!isfinite(P) || !(P > 0.0) || !(ph >= 0.0) || !(ph < 1.0) || !(q > 0.0) ||
        !(q < 1.0) || !isfinite(dep)) {
      char m[160];
      snprintf(m, sizeof m,
               "injection %d: period %g, phase %g, q %g, depth %g (need P > 0, 0 <= phase < 1,"
               " 0 < q < 1, finite depth)",
               k, P, ph, q, dep);
      return fail(p, BLS_ERR_INVALID_ARG, m);
    }
    prm[k].f = 1.0 / P;
    prm[k].phase = ph;
    prm[k].q = q;
    prm[k].depth = dep;
  }
  // The batch: ninj copies of the cadence sharing the trial grid.
  if ((int64_t)ninj * n > p->cfg.max_points || ninj > p->cfg.max_curves ||
      (int64_t)ninj * cf->nperiods > p->cfg.max_periods)
    return fail(p, BLS_ERR_CAPACITY,
                "injections x points, injections or injections x periods exceed the plan");
  std::vector<int64_t> n_off(ninj + 1);
  for (int32_t k = 0; k <= ninj; ++k) n_off[k] = (int64_t)k * n;
  int st = ensure_staging(p);
  if (st != BLS_OK) return st;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  bls_batch b;
  memset(&b, 0, sizeof b);
  b.ncurves = ninj;
  b.nbins_all = cf->nbins;
  b.n_off = n_off.data();
  b.times = p->d_t;
  b.flux = p->d_x;
  b.weights = cf->weights ? p->d_w : nullptr;
  b.p_off = nullptr;
  b.periods = cf->periods;
  b.nperiods_shared = cf->nperiods;
  b.qmin_all = cf->qmin;
  b.qmax_all = cf->qmax;
  std::string err;
  st = validate_batch(p->cfg, b, false, p->shapes, err);
  if (st != BLS_OK) return set_error(p, st, err);
  const bool weighted = cf->weights != nullptr;
  TileChoice tc = choose_tiles(p, p->shapes, weighted);
  PlannedBatch pb;
  st = plan_batch(p, p->shapes, weighted, tc, pb);
  if (st != BLS_OK) return st;
  p->graph_valid = false;  // descriptors were rewritten
  st = ensure_recovery_buffers(p);
  if (st != BLS_OK) return st;

  hipStream_t s = p->stream;
  if ((e = hipEventRecord(p->ev_begin, s)) != hipSuccess) return hip_error(p, e, "event");
  // a synchronous upload: prm lives on this function's stack
  if ((e = hipMemcpyAsync(p->d_inj, prm.data(), sizeof(InjParam) * ninj, hipMemcpyHostToDevice,
                          s)) != hipSuccess ||
      (e = hipStreamSynchronize(s)) != hipSuccess)
    return hip_error(p, e, "upload injections");
  hipLaunchKernelGGL(cadence_t0_kernel, dim3(1), dim3(kBlock), 0, s, cf->times, cf->weights, n,
                     p->d_inj_t0);
  if ((e = hipGetLastError()) != hipSuccess) return hip_error(p, e, "launch t0");
  InjectArgs ia;
  ia.t = cf->times;
  ia.w = cf->weights;
  ia.base = cf->base_flux;
  ia.prm = reinterpret_cast<const InjParam *>(p->d_inj);
  ia.t0 = p->d_inj_t0;
  ia.n = n;
  ia.total = (int64_t)ninj * n;
  ia.t_out = p->d_t;
  ia.w_out = weighted ? p->d_w : nullptr;
  ia.x_out = p->d_x;
  const int64_t blocks = std::min<int64_t>((ia.total + kBlock - 1) / kBlock, 8 * 1024);
  hipLaunchKernelGGL(inject_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, ia);
  if ((e = hipGetLastError()) != hipSuccess) return hip_error(p, e, "launch injection");
  if (out->flux &&
      (e = hipMemcpyAsync(out->flux, p->d_x, sizeof(double) * ia.total, hipMemcpyDeviceToDevice,
                          s)) != hipSuccess)
    return hip_error(p, e, "copy injected fluxes");

  st = enqueue_search(p, pb, p->d_t, p->d_x, weighted ? p->d_w : nullptr, cf->periods, p->d_sr,
                      p->d_depth, p->d_j, p->d_k, p->d_best);
  if (st != BLS_OK) return st;
  st = enqueue_detect_shared(p, ninj, cf->periods, cf->nperiods, p->d_sr, 1, cf->window,
                             cf->sde_threshold);
  if (st != BLS_OK) return st;
  if ((e = hipEventRecord(p->ev_end, s)) != hipSuccess) return hip_error(p, e, "event");
  const int64_t nres = (int64_t)ninj * cf->nperiods;
  if (out->sr &&
      (e = hipMemcpyAsync(out->sr, p->d_sr, sizeof(float) * nres, hipMemcpyDeviceToDevice, s)) !=
          hipSuccess)
    return hip_error(p, e, "copy periodograms");
  std::vector<bls_detection> det(ninj);
  std::vector<double> grid(cf->nperiods);
  if ((e = hipMemcpyAsync(det.data(), p->d_detect_out, sizeof(bls_detection) * ninj,
                          hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(grid.data(), cf->periods, sizeof(double) * cf->nperiods,
                          hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_error(p, e, "download detections");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_error(p, e, "injection recovery");
  std::vector<int32_t> bad(ninj, 0);
  st = device_status_flags(p, ninj, bad.data());
  if (st != BLS_OK) return st;

  // Rule: SDE >= threshold and the best period within ptol h P of h P,
  // h in {1, 1/2, 2}; invalid copies (bad data or trial periods) get -1.
  static const double kAlias[3] = {1.0, 0.5, 2.0};
  for (int32_t k = 0; k < ninj; ++k) {
    const bls_detection &d = det[k];
    const int64_t bi = d.npeaks > 0 ? d.peak_index[0] : -1;
    int32_t rec = 0;
    if (bad[k]) {
      rec = -1;
    } else if (bi >= 0 && d.sde >= cf->sde_threshold) {
      const double pb = grid[bi];
      for (double h : kAlias) {
        const double target = h * cf->inj_period[k];
        if (fabs(pb - target) <= cf->ptol * target) rec = 1;
      }
    }
    out->recovered[k] = rec;
    if (out->best_index) out->best_index[k] = bad[k] ? -1 : bi;
    if (out->sde) out->sde[k] = bad[k] ? NAN : d.sde;
  }
  float ms = 0.f;
  p->stats.search_ms = last_kernel_ms(p);
  (void)hipEventElapsedTime(&ms, p->ev_begin, p->ev_end);
  p->stats.total_ms = ms;
  fill_stats(p, pb, false);
  p->last = pb;
  return BLS_OK;
}
