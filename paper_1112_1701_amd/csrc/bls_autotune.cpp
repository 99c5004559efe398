// Autotuner for the search launch: picks the period tile T (periods per work
// item) for a batch's dominant shape.  T sets the histogram LDS footprint,
// hence how many workgroups a CU holds, and how often a curve's points are
// re-read per period.  Candidates are timed on synthetic prepared data of
// the same shape (written straight into the plan's scratch arrays, which
// the real prep overwrites afterwards); the winner is cached per shape
// bucket in memory and, when BLS_AUTOTUNE_CACHE names a file, on disk.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "bls_plan.h"

namespace bls {
namespace {

std::mutex g_cache_mu;
std::map<uint64_t, TileChoice> g_cache;

struct Bucket {
  int n_log2, nbins_b, kmax_b, weighted, dip;
  uint64_t key() const {
    return ((uint64_t)n_log2 << 40) | ((uint64_t)nbins_b << 24) | ((uint64_t)kmax_b << 8) |
           ((uint64_t)weighted << 1) | (uint64_t)dip;
  }
};

template <class T>
T median_of(std::vector<T> v) {
  std::nth_element(v.begin(), v.begin() + v.size() / 2, v.end());
  return v[v.size() / 2];
}

bool load_disk(uint64_t key, TileChoice &tc) {
  const char *path = getenv("BLS_AUTOTUNE_CACHE");
  if (!path || !*path) return false;
  FILE *f = fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    unsigned long long k;
    int budget, cap, occ;
    if (sscanf(line, "bls-tile-v2 %llx %d %d %d", &k, &budget, &cap, &occ) == 4 && k == key) {
      tc.lds_budget = budget;
      tc.tile_cap = cap;
      tc.occupancy = occ;
      found = true;  // the last entry wins
    }
  }
  fclose(f);
  return found;
}

void save_disk(uint64_t key, const TileChoice &tc, double ms) {
  const char *path = getenv("BLS_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  FILE *f = fopen(path, "a");
  if (!f) return;
  fprintf(f, "bls-tile-v2 %llx %d %d %d %.4f\n", (unsigned long long)key, tc.lds_budget,
          tc.tile_cap, tc.occupancy, ms);
  fclose(f);
}

__global__ void synth_prepped(double *dt, int32_t *q, int32_t *qw, int64_t n, int qmax_abs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // integer hash of the index: spread times over 60 days, small signed values
  unsigned h = (unsigned)i * 2654435761u;
  h ^= h >> 15;
  h *= 2246822519u;
  h ^= h >> 13;
  dt[i] = 60.0 * (double)(h >> 8) * (1.0 / 16777216.0);
  q[i] = (int32_t)(h % (2u * (unsigned)qmax_abs + 1u)) - qmax_abs;
  if (qw) qw[i] = 1 << 20;
}

__global__ void synth_periods(double *per, int m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) per[i] = 0.2 * exp((double)i * log(50.0) / (double)(m > 1 ? m - 1 : 1));
}

// Time one search launch of the sample batch with tile T.
double time_candidate(bls_plan *p, std::vector<CurveShape> &shapes, bool weighted, int T,
                      double *per, float *sr, float *depth, int32_t *js, int32_t *ks,
                      unsigned long long *keys, int nreps) {
  TileChoice tc;
  const int wpb = weighted ? 2 : 1;
  tc.lds_budget = T * hist_stride(shapes[0].nbins, shapes[0].kmax, T, weighted) * 8 * wpb;
  tc.tile_cap = T;
  PlannedBatch pb;
  if (plan_batch(p, shapes, weighted, tc, pb) != BLS_OK) return -1.0;
  // prep fields of the synthetic curves: every point kept, unit scale
  for (int c = 0; c < pb.ncurves; ++c) {
    CurveDesc &d = p->h_curves[c];
    d.status = kCurveOk;
    d.n_eff = (int32_t)d.n;
    d.Wf = weighted ? (float)ldexp((double)d.n * (double)(1 << 20), -d.qbits) : (float)d.n;
    d.out_scale = 1.0;
  }
  hipStream_t st = p->stream;
  if (hipMemcpyAsync(p->d_curves, p->h_curves, sizeof(CurveDesc) * pb.ncurves,
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(p->d_seg_start, p->h_seg_start, sizeof(int64_t) * (pb.nseg + 1),
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(p->d_seg_curve, p->h_seg_curve, sizeof(int32_t) * pb.nseg,
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(p->d_seg_tile0, p->h_seg_tile0, sizeof(int32_t) * pb.nseg,
                     hipMemcpyHostToDevice, st) != hipSuccess ||
      desc_mark(p) != BLS_OK)
    return -1.0;
  SearchArgs a;
  a.curves = p->d_curves;
  a.periods = per;
  a.dt = p->d_dt;
  a.q = p->d_q;
  a.qw = weighted ? p->d_qw : nullptr;
  a.seg_start = p->d_seg_start;
  a.seg_curve = p->d_seg_curve;
  a.seg_tile0 = p->d_seg_tile0;
  a.nseg = pb.nseg;
  a.min_in_points = p->cfg.min_in_points;
  a.nitems = pb.nitems;
  a.counter = p->d_counter;
  a.sr = sr;
  a.depth = depth;
  a.jstart = js;
  a.kwidth = ks;
  a.best_key = keys;
  a.hist_bytes = pb.hist_bytes;
  a.ucap = 0;
  a.uws = nullptr;
  a.uws_stride = 0;
  a.fold_policy = 0;
  a.seed_unit = 1;
  single_partition(a);
  const bool dip = (p->cfg.flags & BLS_DIP_ONLY) != 0;
  double best = 1e30;
  for (int r = 0; r < nreps; ++r) {
    if (launch_fill(p->d_counter, keys, pb.ncurves, st) != 0) return -1.0;
    if (hipEventRecord(p->ev_search0, st) != hipSuccess) return -1.0;
    if (launch_search(a, weighted, dip, pb.grid, st) != 0) return -1.0;
    if (hipEventRecord(p->ev_search1, st) != hipSuccess) return -1.0;
    if (hipEventSynchronize(p->ev_search1) != hipSuccess) return -1.0;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p->ev_search0, p->ev_search1) != hipSuccess) return -1.0;
    best = std::min(best, (double)ms);
  }
  return best;
}

TileChoice tune(bls_plan *p, const Bucket &bk, const CurveShape &rep, bool weighted) {
  TileChoice def = default_tiles(weighted);
  // Sample: enough items for a few dozen per workgroup at the mid-size
  // tiles, so a candidate is timed in the steady state of the persistent
  // grid rather than its ramp-up and tail (at 1024 periods per curve the
  // 8- and 12-period tiles differed by less than the run-to-run noise).
  const int64_t n = std::max<int64_t>(2, std::min<int64_t>(rep.n, p->cfg.max_points / 4));
  int ncurves = (int)std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(
      64, p->cfg.max_curves), p->cfg.max_points / n));
  const int m = 8192;
  if ((int64_t)ncurves * m > p->cfg.max_periods) ncurves = (int)std::max<int64_t>(1, p->cfg.max_periods / m);
  if (ncurves < 1 || (int64_t)ncurves * m > p->cfg.max_periods) return def;

  double *per = nullptr;
  float *sr = nullptr, *depth = nullptr;
  int32_t *js = nullptr, *ks = nullptr;
  unsigned long long *keys = nullptr;
  const size_t nres = (size_t)ncurves * m;
  bool ok = device_alloc((void **)&per, 8 * m) == hipSuccess &&
            device_alloc((void **)&sr, 4 * nres) == hipSuccess &&
            device_alloc((void **)&depth, 4 * nres) == hipSuccess &&
            device_alloc((void **)&js, 4 * nres) == hipSuccess &&
            device_alloc((void **)&ks, 4 * nres) == hipSuccess &&
            device_alloc((void **)&keys, 8 * ncurves) == hipSuccess;
  TileChoice best_tc = def;
  if (ok) {
    const int64_t total = n * ncurves;
    const int qmax_abs = 1 << 12;
    hipLaunchKernelGGL(synth_prepped, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       p->stream, p->d_dt, p->d_q, weighted ? p->d_qw : nullptr, total,
                       qmax_abs);
    hipLaunchKernelGGL(synth_periods, dim3((m + 255) / 256), dim3(256), 0, p->stream, per, m);
    std::vector<CurveShape> shapes(ncurves);
    for (int c = 0; c < ncurves; ++c) {
      shapes[c] = rep;
      shapes[c].n_off = (int64_t)c * n;
      shapes[c].n = n;
      shapes[c].p_off = 0;
      shapes[c].r_off = (int64_t)c * m;
      shapes[c].nperiods = m;
    }
    const int wpb = weighted ? 2 : 1;
    double best_rate = 0.0;
    // Tiles of 4, 5, 7, 8, 9 and 16 periods can read bins free of LDS bank
    // conflicts, 6, 10 and 12 cannot; 7 is the largest that lets eight
    // unit-weight workgroups share a CU at 300 bins.
    const int cands[] = {1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 16, 24, 32};
    for (int T : cands) {
      if (T > kTileMax) break;
      const int per_period = hist_stride(rep.nbins, rep.kmax, T, weighted) * 8 * wpb;
      if (T * per_period > p->max_lds - 1024) break;
      const double ms = time_candidate(p, shapes, weighted, T, per, sr, depth, js, ks, keys, 3);
      if (ms <= 0.0) continue;
      const double rate = 1.0 / ms;  // same work for every candidate
      if (rate > best_rate * 1.02) {  // prefer the smaller tile on near-ties
        best_rate = rate;
        best_tc.lds_budget = T * per_period;
        best_tc.tile_cap = T;
        best_tc.occupancy = 0;
      }
    }
    if (best_rate > 0.0) save_disk(bk.key(), best_tc, 1.0 / best_rate);
  }
  for (void *d : {(void *)per, (void *)sr, (void *)depth, (void *)js, (void *)ks, (void *)keys})
    if (d) (void)hipFree(d);
  (void)hipGetLastError();
  return best_tc;
}

}  // namespace

// Box evaluations of a call below which it is not worth tuning for
// (about 20 ms of search at the measured 3e12 evaluations per second).
constexpr double kTuneMinEvals = 6e10;

TileChoice choose_tiles(bls_plan *p, const std::vector<CurveShape> &shapes, bool weighted) {
  TileChoice tc = default_tiles(weighted);
  bool env = false;
  if (const char *s = getenv("BLS_LDS_BUDGET")) tc.lds_budget = atoi(s), env = true;
  if (const char *s = getenv("BLS_TILE_CAP")) tc.tile_cap = atoi(s), env = true;
  if (const char *s = getenv("BLS_OCCUPANCY")) tc.occupancy = atoi(s), env = true;
  if (env || (p->cfg.flags & BLS_NO_AUTOTUNE) || shapes.empty()) return tc;
  // Tuning a new shape costs about 0.1 s of device time; a call with less
  // work than that many box evaluations keeps the built-in table.
  double evals = 0.0;
  for (const CurveShape &s : shapes)
    evals += (double)s.nbins * (double)(s.kmax - s.kmin + 1) * (double)s.nperiods;
  if (evals < kTuneMinEvals) {
    // The built-in table, with the tile cut so that the call has work items
    // for two workgroups per CU.  Tiles any smaller only add per-item work:
    // one 1000-point curve x 5000 periods (200 bins) took 69 / 50 / 62 /
    // 93 us with tiles of 18 / 8 / 4 / 2 periods.
    int64_t periods = 0;
    for (const CurveShape &s : shapes) periods += s.nperiods;
    const int64_t cap = std::max<int64_t>(1, periods / (2 * (int64_t)std::max(p->num_cus, 1)));
    tc.tile_cap = (int)std::min<int64_t>(tc.tile_cap, cap);
    return tc;
  }

  // Dominant shape: median points, bins and widths over the batch.
  std::vector<int64_t> ns;
  std::vector<int> nbs, kms;
  for (const CurveShape &s : shapes) {
    ns.push_back(s.n);
    nbs.push_back(s.nbins);
    kms.push_back(s.kmax);
  }
  CurveShape rep = shapes[0];
  rep.n = median_of(ns);
  rep.nbins = median_of(nbs);
  rep.kmax = median_of(kms);
  rep.kmin = std::min(rep.kmin, rep.kmax);
  Bucket bk;
  bk.n_log2 = (int)ceil(log2((double)rep.n));
  bk.nbins_b = (rep.nbins + 31) / 32;
  bk.kmax_b = (rep.kmax + 7) / 8;
  bk.weighted = weighted ? 1 : 0;
  bk.dip = (p->cfg.flags & BLS_DIP_ONLY) ? 1 : 0;
  const uint64_t key = bk.key();
  if (p->tuned_valid && p->tuned_key == key) return p->tuned;
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      p->tuned = it->second;
      p->tuned_key = key;
      p->tuned_valid = true;
      return it->second;
    }
  }
  TileChoice got;
  if (!load_disk(key, got)) got = tune(p, bk, rep, weighted);
  {
    std::lock_guard<std::mutex> g(g_cache_mu);
    g_cache[key] = got;
  }
  p->tuned = got;
  p->tuned_key = key;
  p->tuned_valid = true;
  return got;
}

}  // namespace bls
