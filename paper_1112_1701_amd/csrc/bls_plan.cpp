// Host runtime of the BLS library: plan creation, validation, planning of
// (curve, period tile) work items, launch sequencing, HIP graph replay and
// the C ABI of include/bls.h.
//
// The operation and its conventions are those stated in include/bls.h (Law
// et al. 2011, section 2.2.2, and the box-least-squares statistic it cites).
#include "bls_plan.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>
#include <unordered_map>

namespace bls {
namespace {

// Message of the calling thread's last error without a plan (plan creation,
// the plan-free search); a fixed buffer, so that recording it allocates
// nothing.
thread_local char g_create_error[256];
std::atomic<long long> g_alloc_count{0};

uint64_t fnv1a(uint64_t h, const void *data, size_t bytes) {
  const unsigned char *p = static_cast<const unsigned char *>(data);
  for (size_t i = 0; i < bytes; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

template <class T>
uint64_t mix(uint64_t h, const T &v) {
  return fnv1a(h, &v, sizeof(T));
}

int cbits_of(int64_t n) {
  int b = 0;
  while (b < 63 && (int64_t(1) << b) <= n) ++b;
  return b;  // bit length of n
}

void free_dev(void *p) {
  if (p) (void)hipFree(p);
}

}  // namespace

hipError_t device_alloc(void **ptr, size_t bytes) {
  *ptr = nullptr;
  const long long k = ++g_alloc_count;
  const char *hook = getenv("BLS_DEBUG_FAIL_ALLOC");
  if (hook && *hook) {
    // "N": the N-th device allocation of the process fails; "all": every one
    // ("pinned" leaves device allocations alone and refuses the host-array
    // path's pinned staging instead).
    if (strcmp(hook, "all") == 0 || atoll(hook) == k) return hipErrorOutOfMemory;
  }
  return hipMalloc(ptr, bytes > 0 ? bytes : 1);
}

int set_error(bls_plan *p, int status, const std::string &msg) {
  if (p)
    p->last_error = msg;
  else
    snprintf(g_create_error, sizeof g_create_error, "%s", msg.c_str());
  return status;
}

int set_error_noplan(int status, const char *msg) {
  snprintf(g_create_error, sizeof g_create_error, "%s", msg);
  return status;
}

int hip_error(bls_plan *p, hipError_t e, const char *what) {
  std::string m = std::string(what) + ": " + hipGetErrorString(e);
  return set_error(p, e == hipErrorOutOfMemory ? BLS_ERR_NO_MEMORY : BLS_ERR_DEVICE, m);
}

int width_range(int32_t nbins, double qmin, double qmax, int32_t *kmin, int32_t *kmax) {
  if (nbins < 2 || !(qmin > 0.0) || !(qmax < 1.0) || !(qmin <= qmax)) return BLS_ERR_INVALID_ARG;
  long lo = lround(qmin * (double)nbins);
  long hi = lround(qmax * (double)nbins);
  if (lo < 1) lo = 1;
  if (hi > nbins - 1) hi = nbins - 1;
  if (kmin) *kmin = (int32_t)lo;
  if (kmax) *kmax = (int32_t)hi;
  return lo <= hi ? BLS_OK : BLS_ERR_INVALID_ARG;
}

namespace {

// Cycles the scan's 64-bit LDS reads take for the first rounds of lane tasks
// of one workgroup when consecutive periods' planes are S float2 apart.  The
// LDS serves such reads 16 lanes at a time from 32 banks of 4 bytes: a group
// of 16 lanes takes as many cycles as the busiest bank has accesses.  Lane
// task q is (start bin, period) = divmod(q, tile); every lane reads at the
// same offset m past its own start, which moves all banks alike, so m = 0.
int scan_read_cycles(int S, int tile, int nbins) {
  int cycles = 0;
  for (int round = 0; round < 4; ++round) {
    for (int g = 0; g < kBlock / 16; ++g) {
      int bank[32] = {0};
      int worst = 0;
      for (int l = 0; l < 16; ++l) {
        const int q = round * kBlock + g * 16 + l;
        const int j = q / tile, t = q - (q / tile) * tile;
        if (j >= nbins) continue;
        const int b0 = (int)((2 * ((int64_t)t * S + j)) & 31);
        worst = std::max(worst, ++bank[b0]);
        worst = std::max(worst, ++bank[(b0 + 1) & 31]);
      }
      cycles += worst;
    }
  }
  return cycles;
}

// Banks depend on S mod 16 only; the cost of each residue is kept.
int cached_read_cycles(int S, int tile, int nbins) {
  static std::mutex mu;
  static std::unordered_map<uint64_t, int> memo;
  const int nb = std::min(nbins, 4 * kBlock);  // lanes reach no further start bin
  const uint64_t key = ((uint64_t)nb << 16) | ((uint64_t)tile << 4) | (uint64_t)(S & 15);
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
  }
  const int c = scan_read_cycles(S & 15, tile, nb);
  std::lock_guard<std::mutex> g(mu);
  memo.emplace(key, c);
  return c;
}

}  // namespace

int hist_words(int nbins, int kmax) {
  // widths above nbins / 2 are scanned through their complement, so no
  // read reaches more than min(kmax, nbins / 2) - 1 bins past the end
  return nbins + std::max(std::min(kmax, nbins / 2) - 1, 1);
}

int hist_stride(int nbins, int kmax, int tile, bool weighted, bool memo) {
  const int hb = hist_words(nbins, kmax);
  const int wpb = weighted ? 2 : 1;  // the scan reads the first plane of wpb
  int best = hb, best_cost = 0;
  for (int hs = hb; hs < hb + 16; ++hs) {
    const int c = memo ? cached_read_cycles(hs * wpb, tile, nbins)
                       : scan_read_cycles((hs * wpb) & 15, tile, std::min(nbins, 4 * kBlock));
    if (hs == hb || c < best_cost) {
      best = hs;
      best_cost = c;
    }
  }
  return best;
}

void fit_tile(int nbins, int kmax, int64_t nperiods, int lds_budget, int tile_cap,
              bool weighted, int *tile, int *stride, bool memo) {
  const int wpb = weighted ? 2 : 1;
  int T = std::max(1, lds_budget / (hist_words(nbins, kmax) * 8 * wpb));
  T = std::min(T, std::min(tile_cap, kTileMax));
  T = (int)std::min<int64_t>(T, std::max<int64_t>(nperiods, 1));
  T = std::max(T, 1);
  int hs = hist_stride(nbins, kmax, T, weighted, memo);
  while (T > 1 && T * hs * 8 * wpb > lds_budget) {
    --T;
    hs = hist_stride(nbins, kmax, T, weighted, memo);
  }
  *tile = T;
  *stride = hs;
}

namespace {
// Message sink of validate_batch_into: a caller-owned character buffer.
struct ErrBuf {
  char *buf;
  size_t len;
  ErrBuf &operator=(const char *m) {
    if (buf && len) snprintf(buf, len, "%s", m);
    return *this;
  }
};
}  // namespace

void fill_curve_desc(const CurveShape &s, bool weighted, const TileChoice &tc,
                     bool check_periods, bool memo, CurveDesc &d) {
  memset(&d, 0, sizeof d);
  d.n_off = s.n_off;
  d.n = s.n;
  d.p_off = s.p_off;
  d.r_off = s.r_off;
  d.nperiods = s.nperiods;
  d.nbins = s.nbins;
  d.kmin = s.kmin;
  d.kmax = s.kmax;
  const int cb = cbits_of(s.n);
  d.shift = 64 - cb;
  d.qbits = std::min(kQBitsMax, 63 - 2 * cb);
  d.weighted = weighted ? 1 : 0;
  d.check_periods = check_periods ? 1 : 0;
  // bins, then the clamp word / wrap-around copy, per period and plane,
  // padded against LDS bank conflicts, as the kernel lays them out
  int T = 1, hs = 0;
  fit_tile(s.nbins, s.kmax, s.nperiods, tc.lds_budget, tc.tile_cap, weighted, &T, &hs, memo);
  d.tile = T;
  d.hstride = hs;
}

int validate_batch_into(const bls_plan_config &cfg, const bls_batch &b, bool check_data,
                        CurveShape *shapes, int shapes_cap, char *err_buf, size_t err_len,
                        bool binned) {
  ErrBuf err{err_buf, err_len};
  char msg[256];
  if (b.ncurves < 1 || b.n_off == nullptr || b.times == nullptr || b.flux == nullptr ||
      b.periods == nullptr) {
    err = "batch needs ncurves >= 1 and non-NULL n_off, times, flux, periods";
    return BLS_ERR_INVALID_ARG;
  }
  if (b.ncurves > cfg.max_curves) {
    snprintf(msg, sizeof msg, "%d curves exceed the plan's max_curves %d", b.ncurves,
             cfg.max_curves);
    err = msg;
    return BLS_ERR_CAPACITY;
  }
  if (b.n_off[0] != 0) {
    err = "n_off[0] must be 0";
    return BLS_ERR_INVALID_ARG;
  }
  if (b.p_off == nullptr && b.nperiods_shared < 1) {
    err = "shared period grid needs nperiods_shared >= 1";
    return BLS_ERR_INVALID_ARG;
  }
  if (b.p_off != nullptr && b.p_off[0] != 0) {
    err = "p_off[0] must be 0";
    return BLS_ERR_INVALID_ARG;
  }
  if (shapes_cap < b.ncurves) {
    err = "shape buffer smaller than the batch";
    return BLS_ERR_CAPACITY;
  }
  int64_t total_results = 0;
  for (int c = 0; c < b.ncurves; ++c) {
    CurveShape &s = shapes[c];
    s.n_off = b.n_off[c];
    s.n = b.n_off[c + 1] - b.n_off[c];
    if (s.n < 2) {
      snprintf(msg, sizeof msg, "curve %d has %lld points (need >= 2)", c, (long long)s.n);
      err = msg;
      return BLS_ERR_INVALID_ARG;
    }
    if (s.n > (int64_t(1) << 24)) {
      snprintf(msg, sizeof msg, "curve %d has %lld points (at most 2^24)", c, (long long)s.n);
      err = msg;
      return BLS_ERR_CAPACITY;
    }
    int64_t np;
    if (b.p_off) {
      s.p_off = b.p_off[c];
      np = b.p_off[c + 1] - b.p_off[c];
      s.r_off = s.p_off;
    } else {
      s.p_off = 0;
      np = b.nperiods_shared;
      s.r_off = (int64_t)c * b.nperiods_shared;
    }
    if (np < 1 || np > INT32_MAX) {
      snprintf(msg, sizeof msg, "curve %d has %lld trial periods", c, (long long)np);
      err = msg;
      return BLS_ERR_INVALID_ARG;
    }
    s.nperiods = (int32_t)np;
    total_results += np;
    const double qmin = b.qmin ? b.qmin[c] : b.qmin_all;
    const double qmax = b.qmax ? b.qmax[c] : b.qmax_all;
    if (!binned) {
      s.nbins = 0;
      s.kmin = s.kmax = 0;
      if (!(qmin > 0.0) || !(qmax < 1.0) || !(qmin <= qmax)) {
        snprintf(msg, sizeof msg, "curve %d: bad duty-cycle range [%g, %g]", c, qmin, qmax);
        err = msg;
        return BLS_ERR_INVALID_ARG;
      }
      if (s.n > kUnbinnedMaxPointsGlobal) {
        snprintf(msg, sizeof msg, "curve %d has %lld points (the unbinned search takes at most %d)",
                 c, (long long)s.n, kUnbinnedMaxPointsGlobal);
        err = msg;
        return BLS_ERR_CAPACITY;
      }
      continue;
    }
    s.nbins = b.nbins ? b.nbins[c] : b.nbins_all;
    if (s.nbins < 2) {
      snprintf(msg, sizeof msg, "curve %d: nbins %d < 2", c, s.nbins);
      err = msg;
      return BLS_ERR_INVALID_ARG;
    }
    if (s.nbins > cfg.max_nbins) {
      snprintf(msg, sizeof msg, "curve %d: nbins %d exceeds max_nbins %d", c, s.nbins,
               cfg.max_nbins);
      err = msg;
      return BLS_ERR_CAPACITY;
    }
    if (width_range(s.nbins, qmin, qmax, &s.kmin, &s.kmax) != BLS_OK) {
      snprintf(msg, sizeof msg, "curve %d: bad duty-cycle range [%g, %g] for %d bins", c, qmin,
               qmax, s.nbins);
      err = msg;
      return BLS_ERR_INVALID_ARG;
    }
  }
  const int64_t total_points = b.n_off[b.ncurves];
  if (total_points > cfg.max_points) {
    snprintf(msg, sizeof msg, "%lld points exceed the plan's max_points %lld",
             (long long)total_points, (long long)cfg.max_points);
    err = msg;
    return BLS_ERR_CAPACITY;
  }
  if (total_results > cfg.max_periods) {
    snprintf(msg, sizeof msg, "%lld results exceed the plan's max_periods %lld",
             (long long)total_results, (long long)cfg.max_periods);
    err = msg;
    return BLS_ERR_CAPACITY;
  }
  if (!check_data) return BLS_OK;

  // Host data: periods, then points (zero-weight points are dropped first).
  const int64_t nper_total = b.p_off ? b.p_off[b.ncurves] : b.nperiods_shared;
  for (int64_t i = 0; i < nper_total; ++i) {
    const double P = b.periods[i];
    if (!isfinite(P) || !(P > 0.0)) {
      snprintf(msg, sizeof msg, "trial period %lld is %g (must be finite and > 0)",
               (long long)i, P);
      err = msg;
      return BLS_ERR_INVALID_ARG;
    }
  }
  for (int c = 0; c < b.ncurves; ++c) {
    const CurveShape &s = shapes[c];
    int64_t kept = 0;
    double W = 0.0;
    for (int64_t i = s.n_off; i < s.n_off + s.n; ++i) {
      const double w = b.weights ? b.weights[i] : 1.0;
      if (!(w >= 0.0) || isinf(w)) {
        snprintf(msg, sizeof msg, "curve %d point %lld: weight %g (must be finite, >= 0)", c,
                 (long long)(i - s.n_off), w);
        err = msg;
        return BLS_ERR_INVALID_ARG;
      }
      if (w == 0.0) continue;
      if (!isfinite(b.times[i]) || !isfinite(b.flux[i])) {
        snprintf(msg, sizeof msg, "curve %d point %lld: non-finite time or flux", c,
                 (long long)(i - s.n_off));
        err = msg;
        return BLS_ERR_INVALID_ARG;
      }
      ++kept;
      W += w;
    }
    if (kept < 2 || !(W > 0.0) || !isfinite(W)) {
      snprintf(msg, sizeof msg, "curve %d: %lld points with positive weight (need >= 2)", c,
               (long long)kept);
      err = msg;
      return BLS_ERR_INVALID_ARG;
    }
  }
  return BLS_OK;
}

int validate_batch(const bls_plan_config &cfg, const bls_batch &b, bool check_data,
                   std::vector<CurveShape> &shapes, std::string &err, bool binned) {
  if (b.ncurves >= 1 && b.ncurves <= cfg.max_curves) shapes.resize(b.ncurves);
  char buf[256] = "";
  const int st = validate_batch_into(cfg, b, check_data, shapes.data(), (int)shapes.size(), buf,
                                     sizeof buf, binned);
  if (st != BLS_OK) err = buf;
  return st;
}

// Segments of the batch, grouped by work partition.  Curves go to the
// partitions round-robin in descending cost, so each partition (one per XCD:
// the device dispatches workgroups to its XCDs round-robin) gets a similar
// share, largest first, and every curve's period tiles stay in one XCD's L2:
// the curve is fetched by one L2 and adjacent tiles' partial result lines
// merge there before write-back.
void layout_partitions(bls_plan *p, const std::vector<double> &cost,
                       const std::vector<int64_t> &items_of, PlannedBatch &out) {
  const int nc = (int)cost.size();
  p->order.resize(nc);
  std::iota(p->order.begin(), p->order.end(), 0);
  std::stable_sort(p->order.begin(), p->order.end(),
                   [&](int a, int b) { return cost[a] > cost[b]; });
  // Few curves (fewer than two per XCD) share one partition: splitting them
  // would only make most workgroups probe empty partitions first.
  const int np =
      (p->num_cus > 0 && p->num_cus % kMaxParts == 0 && nc >= 2 * kMaxParts) ? kMaxParts : 1;
  int64_t items = 0;
  int s = 0;
  for (int x = 0; x < np; ++x) {
    out.part_begin[x] = items;
    for (int k = x; k < nc; k += np) {
      const int c = p->order[k];
      p->h_seg_start[s] = items;
      p->h_seg_curve[s] = c;
      p->h_seg_tile0[s] = 0;
      items += items_of[c];
      ++s;
    }
  }
  for (int x = np; x <= kMaxParts; ++x) out.part_begin[x] = items;
  p->h_seg_start[nc] = items;
  out.nparts = np;
  out.nseg = nc;
  out.nitems = items;
}

int item_group(const bls_plan *p, const std::vector<CurveShape> &shapes) {
  if (const char *e = getenv("BLS_ITEM_GROUP")) {
    const int g = atoi(e);  // 0: one tile per item; kGroupMax: groups
    return g == kGroupMax ? kGroupMax : 0;
  }
  int64_t periods = 0;
  for (const CurveShape &s : shapes) periods += s.nperiods;
  // at least four groups per workgroup of a full grid (eight per CU)
  const int64_t want = (int64_t)kGroupMax * 4 * 8 * std::max(p->num_cus, 1);
  return periods >= want ? kGroupMax : 0;
}

int plan_batch(bls_plan *p, const std::vector<CurveShape> &shapes, bool weighted,
               const TileChoice &tc, PlannedBatch &out) {
  const int nc = (int)shapes.size();
  // queued copies (or graph replays) may still read the pinned descriptors
  const int ws = desc_wait(p);
  if (ws != BLS_OK) return ws;
  const int wpb = weighted ? 2 : 1;
  out = PlannedBatch{};
  out.ncurves = nc;
  out.weighted = weighted;

  // Work items: groups of kGroupMax consecutive periods, aligned to whole
  // result lines and written out together, when the batch has enough of
  // them for several items per resident workgroup; one tile each otherwise.
  const int G = item_group(p, shapes);
  // Per-curve tile: as many periods as fit the LDS budget, at least one.
  int hist_bytes = 0;
  std::vector<double> item_cost(nc);
  for (int c = 0; c < nc; ++c) {
    const CurveShape &s = shapes[c];
    CurveDesc &d = p->h_curves[c];
    // each distinct period range is checked once (a shared grid by curve 0)
    fill_curve_desc(s, weighted, tc, c == 0 || s.p_off != shapes[0].p_off, true, d);
    const int T = d.tile;
    if (G > 0) {
      d.group = G;
      d.galign = (int32_t)(s.r_off % G);
    }
    hist_bytes = std::max(hist_bytes, T * d.hstride * 8 * wpb);
    const double nw = (double)(s.kmax - s.kmin + 1);
    item_cost[c] = (double)(G > 0 ? G : T) * ((double)s.n + 1.6 * (double)s.nbins * nw);
    out.total_points += s.n;
    out.total_results += s.nperiods;
    out.trial_points += (double)s.n * (double)s.nperiods;
    out.box_evals += (double)s.nbins * nw * (double)s.nperiods;
  }
  if (hist_bytes > p->max_lds - 1024) {
    return set_error(p, BLS_ERR_CAPACITY,
                     "one period's histogram needs " + std::to_string(hist_bytes) +
                         " bytes of LDS, more than a workgroup has");
  }

  // Largest items first within each XCD partition, so the persistent grid
  // drains evenly.
  std::vector<int64_t> items_of(nc);
  for (int c = 0; c < nc; ++c) {
    const CurveDesc &d = p->h_curves[c];
    items_of[c] = d.group > 0 ? ((int64_t)d.nperiods + d.galign + d.group - 1) / d.group
                              : (d.nperiods + d.tile - 1) / d.tile;
  }
  layout_partitions(p, item_cost, items_of, out);
  const int64_t items = out.nitems;
  out.hist_bytes = hist_bytes;

  int per_cu = 0;
  hipError_t e = (hipError_t)search_blocks_per_cu(weighted, (p->cfg.flags & BLS_DIP_ONLY) != 0,
                                                  hist_bytes, &per_cu);
  if (e != hipSuccess) return hip_error(p, e, "occupancy query");
  if (per_cu < 1) return set_error(p, BLS_ERR_CAPACITY, "search kernel does not fit a CU");
  if (tc.occupancy > 0) per_cu = std::min(per_cu, tc.occupancy);
  const int64_t grid = std::min<int64_t>(items, (int64_t)p->num_cus * per_cu);
  out.grid = (int32_t)std::max<int64_t>(grid, 1);
  return BLS_OK;
}

int desc_wait(bls_plan *p) {
  if (!p->desc_pending) return BLS_OK;
  hipError_t e = hipEventSynchronize(p->ev_desc);
  if (e != hipSuccess) return hip_error(p, e, "wait for descriptor uploads");
  p->desc_pending = false;
  return BLS_OK;
}

int desc_mark(bls_plan *p) {
  hipError_t e = hipEventRecord(p->ev_desc, p->stream);
  if (e != hipSuccess) return hip_error(p, e, "event record");
  p->desc_pending = true;
  return BLS_OK;
}

int ring_begin(bls_plan *p) {
  const int slot = (int)(p->k_recorded % bls_plan::kTimeRing);
  hipError_t e = hipEventRecord(p->ev_k0[slot], p->stream);
  return e == hipSuccess ? BLS_OK : hip_error(p, e, "event record");
}

int ring_end(bls_plan *p) {
  const int slot = (int)(p->k_recorded % bls_plan::kTimeRing);
  hipError_t e = hipEventRecord(p->ev_k1[slot], p->stream);
  if (e != hipSuccess) return hip_error(p, e, "event record");
  ++p->k_recorded;
  return BLS_OK;
}

int enqueue_pre(bls_plan *p, const PlannedBatch &pb, const double *t, const double *x,
                const double *w, const double *periods, int64_t *best) {
  hipStream_t st = p->stream;
  hipError_t e;
  const int nc = pb.ncurves;
  e = hipMemcpyAsync(p->d_curves, p->h_curves, sizeof(CurveDesc) * nc, hipMemcpyHostToDevice,
                     st);
  if (e != hipSuccess) return hip_error(p, e, "upload curve descriptors");
  e = hipMemcpyAsync(p->d_seg_start, p->h_seg_start, sizeof(int64_t) * (pb.nseg + 1),
                     hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_error(p, e, "upload segments");
  e = hipMemcpyAsync(p->d_seg_curve, p->h_seg_curve, sizeof(int32_t) * pb.nseg,
                     hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_error(p, e, "upload segments");
  e = hipMemcpyAsync(p->d_seg_tile0, p->h_seg_tile0, sizeof(int32_t) * pb.nseg,
                     hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_error(p, e, "upload segments");

  unsigned long long *keys = reinterpret_cast<unsigned long long *>(best);
  e = (hipError_t)launch_fill(p->d_counter, keys, nc, st);
  if (e != hipSuccess) return hip_error(p, e, "launch fill");

  PrepArgs pa;
  pa.curves = p->d_curves;
  pa.periods = periods;
  pa.ncurves = nc;
  pa.t = t;
  pa.x = x;
  pa.w = w;
  pa.dt = p->d_dt;
  pa.q = p->d_q;
  pa.qw = p->d_qw;
  e = (hipError_t)launch_prep(pa, st);
  if (e != hipSuccess) return hip_error(p, e, "launch prep");
  return BLS_OK;
}

int enqueue_kernel(bls_plan *p, const PlannedBatch &pb, const double *periods, float *sr,
                   float *depth, int32_t *js, int32_t *ks, int64_t *best, bool unbinned) {
  SearchArgs sa;
  sa.curves = p->d_curves;
  sa.periods = periods;
  sa.dt = p->d_dt;
  sa.q = p->d_q;
  sa.qw = pb.weighted ? p->d_qw : nullptr;
  sa.seg_start = p->d_seg_start;
  sa.seg_curve = p->d_seg_curve;
  sa.seg_tile0 = p->d_seg_tile0;
  sa.nseg = pb.nseg;
  sa.min_in_points = p->cfg.min_in_points;
  sa.nitems = pb.nitems;
  sa.counter = p->d_counter;
  sa.sr = sr;
  sa.depth = depth;
  sa.jstart = js;
  sa.kwidth = ks;
  sa.best_key = reinterpret_cast<unsigned long long *>(best);
  sa.hist_bytes = pb.hist_bytes;
  sa.ucap = pb.ucap;
  sa.uws = pb.uws;
  sa.uws_stride = pb.uws_stride;
  sa.fold_policy = 0;
  sa.seed_unit = 1;
  if (const char *fm = getenv("BLS_FOLD_MERGE")) sa.fold_policy = atoi(fm) == 1 ? 1 : 2;
  if (const char *su = getenv("BLS_SEED_UNIT")) sa.seed_unit = atoi(su) != 0 ? 1 : 0;
  sa.nparts = pb.nparts;
  sa.pad_parts = 0;
  for (int x = 0; x <= kMaxParts; ++x) sa.part_begin[x] = pb.part_begin[x];
  const bool dip = (p->cfg.flags & BLS_DIP_ONLY) != 0;
  hipError_t e = unbinned ? (hipError_t)launch_unbinned(sa, pb.weighted, dip, pb.grid, p->stream)
                          : (hipError_t)launch_search(sa, pb.weighted, dip, pb.grid, p->stream);
  if (e != hipSuccess) return hip_error(p, e, "launch search");
  return BLS_OK;
}

int enqueue_post(bls_plan *p, const PlannedBatch &pb, int64_t *best) {
  hipError_t e = (hipError_t)launch_best_index(reinterpret_cast<unsigned long long *>(best),
                                               pb.ncurves, p->stream);
  if (e != hipSuccess) return hip_error(p, e, "launch best index");
  return BLS_OK;
}

int enqueue_search(bls_plan *p, const PlannedBatch &pb, const double *t, const double *x,
                   const double *w, const double *periods, float *sr, float *depth, int32_t *js,
                   int32_t *ks, int64_t *best, bool unbinned) {
  int st = enqueue_pre(p, pb, t, x, w, periods, best);
  if (st == BLS_OK) st = desc_mark(p);
  if (st == BLS_OK) st = ring_begin(p);
  if (st == BLS_OK) st = enqueue_kernel(p, pb, periods, sr, depth, js, ks, best, unbinned);
  if (st == BLS_OK) st = ring_end(p);
  if (st == BLS_OK) st = enqueue_post(p, pb, best);
  return st;
}

TileChoice default_tiles(bool weighted) {
  TileChoice tc;
  // The same 32 KB for both paths: one-curve calls on uneven weighted curves
  // ran at 1.97e11 trial-period points/s with it, against 1.92e11 with 40 KB
  // and 1.94e11 with 24 KB.
  (void)weighted;
  tc.lds_budget = 32768;
  tc.tile_cap = kTileMax;
  tc.occupancy = 0;
  return tc;
}

double last_kernel_ms(bls_plan *p) {
  if (p->k_recorded == 0) return 0.0;
  const int slot = (int)((p->k_recorded - 1) % bls_plan::kTimeRing);
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, p->ev_k0[slot], p->ev_k1[slot]) != hipSuccess) return 0.0;
  return ms;
}

void fill_stats(bls_plan *p, const PlannedBatch &pb, bool replayed) {
  p->stats.trial_points = pb.trial_points;
  p->stats.box_evals = pb.box_evals;
  p->stats.work_items = pb.nitems;
  p->stats.grid = pb.grid;
  p->stats.block = kBlock;
  p->stats.lds_bytes = pb.hist_bytes;
  p->stats.graph_replayed = replayed ? 1 : 0;
}

int ensure_staging(bls_plan *p) {
  if (p->staging) return BLS_OK;
  const size_t np = (size_t)p->cfg.max_points, nr = (size_t)p->cfg.max_periods,
               nc = (size_t)p->cfg.max_curves;
  struct {
    void **ptr;
    size_t bytes;
  } req[] = {{(void **)&p->d_t, np * 8},      {(void **)&p->d_x, np * 8},
             {(void **)&p->d_w, np * 8},      {(void **)&p->d_periods, nr * 8},
             {(void **)&p->d_sr, nr * 4},     {(void **)&p->d_depth, nr * 4},
             {(void **)&p->d_j, nr * 4},      {(void **)&p->d_k, nr * 4},
             {(void **)&p->d_best, nc * 8}};
  for (auto &r : req) {
    hipError_t e = device_alloc(r.ptr, r.bytes);
    if (e != hipSuccess) {
      for (auto &q : req) {
        free_dev(*q.ptr);
        *q.ptr = nullptr;
      }
      return hip_error(p, e, "allocate host-path staging");
    }
  }
  p->staging = true;
  return BLS_OK;
}

int check_device_status(bls_plan *p, int ncurves) {
  std::vector<CurveDesc> cds(ncurves);
  hipError_t e = hipMemcpy(cds.data(), p->d_curves, sizeof(CurveDesc) * ncurves,
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(p, e, "read curve status");
  for (int c = 0; c < ncurves; ++c) {
    if (cds[c].status != kCurveOk) {
      char msg[160];
      snprintf(msg, sizeof msg, "curve %d: %s", c,
               cds[c].status == kCurveBadData
                   ? "non-finite time/flux of a kept point, or a negative/non-finite weight"
               : cds[c].status == kCurveBadPeriod
                   ? "a trial period is not finite and > 0"
                   : "fewer than two points with positive weight");
      return set_error(p, BLS_ERR_INVALID_ARG, msg);
    }
  }
  return BLS_OK;
}


// Per-curve validity flags of the last prep (1 where the curve's data or
// trial periods were invalid), read back from the device descriptors.
int device_status_flags(bls_plan *p, int ncurves, int32_t *bad) {
  std::vector<CurveDesc> cds(ncurves);
  hipError_t e = hipMemcpy(cds.data(), p->d_curves, sizeof(CurveDesc) * ncurves,
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_error(p, e, "read curve status");
  for (int c = 0; c < ncurves; ++c) bad[c] = cds[c].status != kCurveOk ? 1 : 0;
  return BLS_OK;
}

int ensure_detect_buffers(bls_plan *p) {
  if (p->d_detect_desc) return BLS_OK;
  hipError_t e;
  if ((e = device_alloc((void **)&p->d_detect_desc, sizeof(DetectDesc) * p->cfg.max_curves)) ||
      (e = device_alloc((void **)&p->d_detect_out, sizeof(bls_detection) * p->cfg.max_curves))) {
    if (p->d_detect_desc) (void)hipFree(p->d_detect_desc);
    p->d_detect_desc = nullptr;
    p->d_detect_out = nullptr;
    return hip_error(p, e, "allocate detection buffers");
  }
  return BLS_OK;
}

int enqueue_detect_shared(bls_plan *p, int ncurves, const double *periods, int64_t nperiods,
                          const float *sr, int max_peaks, double window, double threshold) {
  int st = ensure_detect_buffers(p);
  if (st != BLS_OK) return st;
  std::vector<DetectDesc> dd(ncurves);
  for (int c = 0; c < ncurves; ++c) {
    dd[c].p_off = 0;
    dd[c].r_off = (int64_t)c * nperiods;
    dd[c].nperiods = nperiods;
  }
  hipStream_t s = p->stream;
  // a synchronous upload: dd lives on this function's stack
  hipError_t e = hipMemcpyAsync(p->d_detect_desc, dd.data(), sizeof(DetectDesc) * ncurves,
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_error(p, e, "upload detection descriptors");
  DetectArgs a;
  a.desc = p->d_detect_desc;
  a.periods = periods;
  a.sr = sr;
  a.out = p->d_detect_out;
  a.ncurves = ncurves;
  a.max_peaks = max_peaks;
  a.window = window;
  a.threshold = threshold;
  if ((e = (hipError_t)launch_detect(a, s)) != hipSuccess) return hip_error(p, e, "launch detection");
  return BLS_OK;
}

int ensure_recovery_buffers(bls_plan *p) {
  if (p->d_inj) return BLS_OK;
  hipError_t e;
  if ((e = device_alloc((void **)&p->d_inj, 32 * (size_t)p->cfg.max_curves)) ||
      (e = device_alloc((void **)&p->d_inj_t0, sizeof(double)))) {
    if (p->d_inj) (void)hipFree(p->d_inj);
    p->d_inj = nullptr;
    p->d_inj_t0 = nullptr;
    return hip_error(p, e, "allocate injection buffers");
  }
  return BLS_OK;
}

}  // namespace bls

using namespace bls;

namespace {

// Duration of the most recent bracketed kernel launch (the stream must have
// reached its end event); 0 if there is none.
// Host-array search of a validated batch (shared by bls_search and
// bls_search_batch).
// f(i0, i1) over [0, n) in contiguous pieces on up to 16 host threads, one
// piece per `grain` items at least (the calling thread takes the last).
template <class F>
void par_ranges(int64_t n, int64_t grain, F f) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int64_t nt = std::max<int64_t>(
      1, std::min<int64_t>((int64_t)std::min(hw, 16u), n / std::max<int64_t>(grain, 1)));
  std::vector<std::thread> th;
  int64_t i0 = 0;
  for (int64_t t = 0; t + 1 < nt; ++t) {
    const int64_t i1 = n * (t + 1) / nt;
    try {
      th.emplace_back(f, i0, i1);
    } catch (...) {
      f(i0, i1);  // no thread: this one does the piece
    }
    i0 = i1;
  }
  f(i0, n);
  for (auto &x : th) x.join();
}

// Copy of `bytes` between host buffers on several threads (a single thread
// copies at a fraction of the memory bandwidth).
void par_copy(void *dst, const void *src, size_t bytes) {
  par_ranges((int64_t)bytes, int64_t(8) << 20, [&](int64_t i0, int64_t i1) {
    memcpy((char *)dst + i0, (const char *)src + i0, (size_t)(i1 - i0));
  });
}

// Pinned staging for the host API, sized once for the plan's limits: the
// inputs (times, flux, weights, periods) or the results (SR, depth, first
// and last bin, best index), whichever is larger.  False if pinned memory
// is not available (the host API then copies from pageable memory).
bool ensure_host_stage(bls_plan *p) {
  if (p->h_stage) return true;
  // BLS_DEBUG_FAIL_ALLOC=pinned: behave as if pinned memory were refused
  const char *hook = getenv("BLS_DEBUG_FAIL_ALLOC");
  if (hook && strcmp(hook, "pinned") == 0) return false;
  const size_t np = (size_t)p->cfg.max_points, nr = (size_t)p->cfg.max_periods,
               nc = (size_t)p->cfg.max_curves;
  const size_t in = 3 * np * 8 + nr * 8 + 256, res = 4 * nr * 4 + nc * 8 + 256;
  const size_t bytes = std::max(in, res);
  if (hipHostMalloc((void **)&p->h_stage, bytes, 0) != hipSuccess) {
    p->h_stage = nullptr;
    return false;
  }
  p->h_stage_bytes = bytes;
  return true;
}

int host_search(bls_plan *p, const bls_batch &b, const std::vector<CurveShape> &shapes,
                const bls_results &out) {
  int st = ensure_staging(p);
  if (st != BLS_OK) return st;
  const bool weighted = b.weights != nullptr;
  TileChoice tc = choose_tiles(p, shapes, weighted);
  PlannedBatch pb;
  st = plan_batch(p, shapes, weighted, tc, pb);
  if (st != BLS_OK) return st;
  p->graph_valid = false;  // descriptors were rewritten

  const int64_t npts = b.n_off[b.ncurves];
  const int64_t nper = b.p_off ? b.p_off[b.ncurves] : b.nperiods_shared;
  hipStream_t s = p->stream;
  hipError_t e;
  // Inputs through the pinned staging when there is one: a threaded copy
  // into it, then DMA (pageable copies run at a fraction of that rate).  The
  // previous call's copies from or into it ended with that call.
  const bool pinned = ensure_host_stage(p);
  const double *src_t = b.times, *src_x = b.flux, *src_w = b.weights, *src_p = b.periods;
  if (pinned) {
    double *st = reinterpret_cast<double *>(p->h_stage);
    double *sx = st + npts, *sw = sx + npts, *sp = sw + (weighted ? npts : 0);
    par_copy(st, b.times, (size_t)npts * 8);
    par_copy(sx, b.flux, (size_t)npts * 8);
    if (weighted) par_copy(sw, b.weights, (size_t)npts * 8);
    par_copy(sp, b.periods, (size_t)nper * 8);
    src_t = st;
    src_x = sx;
    src_w = weighted ? sw : nullptr;
    src_p = sp;
  }
  if ((e = hipEventRecord(p->ev_begin, s)) != hipSuccess) return hip_error(p, e, "event");
  if ((e = hipMemcpyAsync(p->d_t, src_t, npts * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_error(p, e, "upload times");
  if ((e = hipMemcpyAsync(p->d_x, src_x, npts * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_error(p, e, "upload flux");
  if (weighted &&
      (e = hipMemcpyAsync(p->d_w, src_w, npts * 8, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_error(p, e, "upload weights");
  if ((e = hipMemcpyAsync(p->d_periods, src_p, nper * 8, hipMemcpyHostToDevice, s)) !=
      hipSuccess)
    return hip_error(p, e, "upload periods");
  st = enqueue_search(p, pb, p->d_t, p->d_x, weighted ? p->d_w : nullptr, p->d_periods, p->d_sr,
                      p->d_depth, p->d_j, p->d_k, p->d_best);
  if (st != BLS_OK) return st;
  if ((e = hipEventRecord(p->ev_end, s)) != hipSuccess) return hip_error(p, e, "event");

  // Results into the pinned staging (the uploads from it have run by then:
  // same stream), else into pageable vectors.
  const int64_t nres = pb.total_results;
  std::vector<float> v_sr, v_depth;
  std::vector<int32_t> v_js, v_ks;
  std::vector<int64_t> v_best;
  float *sr, *depth;
  int32_t *js, *ks;
  int64_t *best;
  if (pinned) {
    best = reinterpret_cast<int64_t *>(p->h_stage);
    sr = reinterpret_cast<float *>(best + b.ncurves);
    depth = sr + nres;
    js = reinterpret_cast<int32_t *>(depth + nres);
    ks = js + nres;
  } else {
    v_sr.resize(nres);
    v_depth.resize(nres);
    v_js.resize(nres);
    v_ks.resize(nres);
    v_best.resize(b.ncurves);
    sr = v_sr.data();
    depth = v_depth.data();
    js = v_js.data();
    ks = v_ks.data();
    best = v_best.data();
  }
  if ((e = hipMemcpyAsync(sr, p->d_sr, nres * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(depth, p->d_depth, nres * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(js, p->d_j, nres * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(ks, p->d_k, nres * 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
      (e = hipMemcpyAsync(best, p->d_best, b.ncurves * 8, hipMemcpyDeviceToHost, s)) !=
          hipSuccess)
    return hip_error(p, e, "download results");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_error(p, e, "search");
  st = check_device_status(p, b.ncurves);
  if (st != BLS_OK) return st;

  float ms = 0.f;
  p->stats.search_ms = last_kernel_ms(p);
  (void)hipEventElapsedTime(&ms, p->ev_begin, p->ev_end);
  p->stats.total_ms = ms;
  fill_stats(p, pb, false);

  // Results: (value, box) per period at r_off; phase and duration from j, k.
  // Up to 40 B are written per result: host threads take contiguous curve
  // ranges.
  par_ranges(b.ncurves, std::max<int64_t>(1, (int64_t)b.ncurves * (int64_t(1) << 20) /
                                                 std::max<int64_t>(nres, 1)),
             [&](int64_t c0, int64_t c1) {
    for (int64_t c = c0; c < c1; ++c) {
      const CurveShape &cs = shapes[c];
      const double *per = b.periods + cs.p_off;
      for (int32_t i = 0; i < cs.nperiods; ++i) {
        const int64_t r = cs.r_off + i;
        const bool none = ks[r] < 0;
        if (out.sr) out.sr[r] = (double)sr[r];
        if (out.depth) out.depth[r] = none ? NAN : (double)depth[r];
        if (out.jstart) out.jstart[r] = js[r];
        if (out.kwidth) out.kwidth[r] = ks[r];
        if (out.phase) out.phase[r] = none ? NAN : (double)js[r] / (double)cs.nbins;
        if (out.duration) out.duration[r] = none ? NAN : (double)ks[r] * per[i] / (double)cs.nbins;
      }
      if (out.best_index) out.best_index[c] = best[c];
    }
  });
  p->last = pb;
  return BLS_OK;
}

uint64_t batch_signature(const bls_plan *p, const bls_batch &b, const bls_device_results &o) {
  uint64_t h = 1469598103934665603ull;
  h = mix(h, b.ncurves);
  h = mix(h, b.times);
  h = mix(h, b.flux);
  h = mix(h, b.weights);
  h = mix(h, b.periods);
  h = mix(h, b.nperiods_shared);
  h = mix(h, b.nbins_all);
  h = mix(h, b.qmin_all);
  h = mix(h, b.qmax_all);
  h = fnv1a(h, b.n_off, sizeof(int64_t) * (b.ncurves + 1));
  if (b.p_off) h = fnv1a(h, b.p_off, sizeof(int64_t) * (b.ncurves + 1));
  if (b.nbins) h = fnv1a(h, b.nbins, sizeof(int32_t) * b.ncurves);
  if (b.qmin) h = fnv1a(h, b.qmin, sizeof(double) * b.ncurves);
  if (b.qmax) h = fnv1a(h, b.qmax, sizeof(double) * b.ncurves);
  h = mix(h, o.sr);
  h = mix(h, o.depth);
  h = mix(h, o.jstart);
  h = mix(h, o.kwidth);
  h = mix(h, o.best_index);
  h = mix(h, p->cfg.flags);
  h = mix(h, p->cfg.min_in_points);
  return h;
}

void drop_graph(bls_plan *p) {
  for (int g = 0; g < 3; ++g) {
    if (p->gexec[g]) (void)hipGraphExecDestroy(p->gexec[g]);
    if (p->graph[g]) (void)hipGraphDestroy(p->graph[g]);
    p->gexec[g] = nullptr;
    p->graph[g] = nullptr;
  }
  p->graph_valid = false;
}

// Capture one part of the launch sequence into graph g and instantiate it.
template <class F>
int capture_part(bls_plan *p, int g, F &&enqueue) {
  hipError_t e = hipStreamBeginCapture(p->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_error(p, e, "begin capture");
  const int st = enqueue();
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(p->stream, &graph);
  if (st != BLS_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_error(p, e, "end capture");
  p->graph[g] = graph;
  e = hipGraphInstantiate(&p->gexec[g], graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_error(p, e, "instantiate graph");
  return BLS_OK;
}

// Replay the three captured parts, the search kernel between the timing
// ring's events and the descriptor mark after the uploads.
int launch_graphs(bls_plan *p) {
  hipError_t e = hipGraphLaunch(p->gexec[0], p->stream);
  if (e != hipSuccess) return hip_error(p, e, "graph launch");
  int st = desc_mark(p);
  if (st == BLS_OK) st = ring_begin(p);
  if (st != BLS_OK) return st;
  if ((e = hipGraphLaunch(p->gexec[1], p->stream)) != hipSuccess)
    return hip_error(p, e, "graph launch");
  st = ring_end(p);
  if (st != BLS_OK) return st;
  if ((e = hipGraphLaunch(p->gexec[2], p->stream)) != hipSuccess)
    return hip_error(p, e, "graph launch");
  return BLS_OK;
}

}  // namespace

extern "C" {

void bls_plan_config_init(bls_plan_config *cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof *cfg);
  cfg->device = 0;
  cfg->max_curves = 1;
  cfg->max_points = int64_t(1) << 20;
  cfg->max_periods = int64_t(1) << 20;
  cfg->max_nbins = BLS_MAX_NBINS;
  cfg->min_in_points = 1;
  cfg->flags = 0;
  cfg->hip_stream = nullptr;
}

int bls_plan_create(bls_plan **out, const bls_plan_config *cfg_in) {
  if (!out) return set_error(nullptr, BLS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  bls_plan_config cfg;
  if (cfg_in)
    cfg = *cfg_in;
  else
    bls_plan_config_init(&cfg);
  if (cfg.min_in_points <= 0) cfg.min_in_points = 1;
  if (cfg.max_curves < 1 || cfg.max_points < 2 || cfg.max_periods < 1 || cfg.max_nbins < 2 ||
      cfg.max_nbins > BLS_MAX_NBINS || cfg.max_curves > (1 << 30))
    return set_error(nullptr, BLS_ERR_INVALID_ARG, "bad plan capacities");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0)
    return set_error(nullptr, BLS_ERR_DEVICE, "no HIP device available");
  if (cfg.device < 0 || cfg.device >= ndev)
    return set_error(nullptr, BLS_ERR_INVALID_ARG, "device ordinal out of range");

  bls_plan *p = new (std::nothrow) bls_plan();
  if (!p) return set_error(nullptr, BLS_ERR_NO_MEMORY, "host allocation");
  p->cfg = cfg;
  p->device = cfg.device;
  auto fail = [&](int st) {
    snprintf(g_create_error, sizeof g_create_error, "%s", p->last_error.c_str());
    bls_plan_destroy(p);
    return st;
  };
  if ((e = hipSetDevice(p->device)) != hipSuccess) return fail(hip_error(p, e, "set device"));
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, p->device)) != hipSuccess)
    return fail(hip_error(p, e, "device properties"));
  p->num_cus = prop.multiProcessorCount;
  p->max_lds = (int)prop.sharedMemPerBlock;
  if (cfg.hip_stream) {
    p->stream = (hipStream_t)cfg.hip_stream;
  } else {
    if ((e = hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking)) != hipSuccess)
      return fail(hip_error(p, e, "create stream"));
    p->own_stream = true;
  }
  for (hipEvent_t *ev : {&p->ev_begin, &p->ev_search0, &p->ev_search1, &p->ev_end, &p->ev_desc})
    if ((e = hipEventCreate(ev)) != hipSuccess) return fail(hip_error(p, e, "create event"));
  for (int i = 0; i < bls_plan::kTimeRing; ++i)
    if ((e = hipEventCreate(&p->ev_k0[i])) != hipSuccess ||
        (e = hipEventCreate(&p->ev_k1[i])) != hipSuccess)
      return fail(hip_error(p, e, "create event"));

  const size_t nc = (size_t)cfg.max_curves, npt = (size_t)cfg.max_points;
  struct {
    void **ptr;
    size_t bytes;
  } req[] = {{(void **)&p->d_curves, sizeof(CurveDesc) * nc},
             {(void **)&p->d_seg_start, sizeof(int64_t) * (nc + 1)},
             {(void **)&p->d_seg_curve, sizeof(int32_t) * nc},
             {(void **)&p->d_seg_tile0, sizeof(int32_t) * nc},
             {(void **)&p->d_dt, 8 * npt},
             {(void **)&p->d_q, 4 * npt},
             {(void **)&p->d_qw, 4 * npt},
             {(void **)&p->d_counter, 64}};
  for (auto &r : req)
    if ((e = device_alloc(r.ptr, r.bytes)) != hipSuccess)
      return fail(hip_error(p, e, "allocate plan buffers"));
  if ((e = hipHostMalloc((void **)&p->h_curves, sizeof(CurveDesc) * nc, 0)) != hipSuccess ||
      (e = hipHostMalloc((void **)&p->h_seg_start, sizeof(int64_t) * (nc + 1), 0)) !=
          hipSuccess ||
      (e = hipHostMalloc((void **)&p->h_seg_curve, sizeof(int32_t) * nc, 0)) != hipSuccess ||
      (e = hipHostMalloc((void **)&p->h_seg_tile0, sizeof(int32_t) * nc, 0)) != hipSuccess)
    return fail(hip_error(p, e, "allocate pinned descriptors"));
  *out = p;
  return BLS_OK;
}

int bls_plan_destroy(bls_plan *p) {
  if (!p) return BLS_OK;
  if (p->stream) (void)hipStreamSynchronize(p->stream);
  drop_graph(p);
  for (void *d : {(void *)p->d_detect_desc, (void *)p->d_detect_out,
                  (void *)p->d_window_desc, (void *)p->d_window_flag,
                  (void *)p->d_var_noff, (void *)p->d_var_alive, (void *)p->d_var_chip,
                  (void *)p->d_uws})
    free_dev(d);
  for (void *d : {(void *)p->d_curves, (void *)p->d_seg_start, (void *)p->d_seg_curve,
                  (void *)p->d_seg_tile0, (void *)p->d_dt, (void *)p->d_q, (void *)p->d_qw,
                  (void *)p->d_counter, (void *)p->d_t, (void *)p->d_x, (void *)p->d_w,
                  (void *)p->d_periods, (void *)p->d_sr, (void *)p->d_depth, (void *)p->d_j,
                  (void *)p->d_k, (void *)p->d_best})
    free_dev(d);
  for (void *h : {(void *)p->h_curves, (void *)p->h_seg_start, (void *)p->h_seg_curve,
                  (void *)p->h_seg_tile0, (void *)p->h_stage})
    if (h) (void)hipHostFree(h);
  for (hipEvent_t ev : {p->ev_begin, p->ev_search0, p->ev_search1, p->ev_end, p->ev_desc})
    if (ev) (void)hipEventDestroy(ev);
  for (int i = 0; i < bls_plan::kTimeRing; ++i) {
    if (p->ev_k0[i]) (void)hipEventDestroy(p->ev_k0[i]);
    if (p->ev_k1[i]) (void)hipEventDestroy(p->ev_k1[i]);
  }
  if (p->own_stream && p->stream) (void)hipStreamDestroy(p->stream);
  delete p;
  return BLS_OK;
}

int bls_search(bls_plan *p, const double *times, const double *flux, const double *weights,
               int64_t n, const double *periods, int64_t nperiods, int32_t nbins, double qmin,
               double qmax, double *sr, double *phase, double *duration, double *depth,
               int32_t *jstart, int32_t *kwidth, int64_t *best_index) {
  if (!p) return BLS_ERR_INVALID_ARG;
  if (n < 0 || nperiods < 1)
    return set_error(p, BLS_ERR_INVALID_ARG, "need n >= 2 and nperiods >= 1");
  int64_t n_off[2] = {0, n};
  bls_batch b;
  memset(&b, 0, sizeof b);
  b.ncurves = 1;
  b.n_off = n_off;
  b.times = times;
  b.flux = flux;
  b.weights = weights;
  b.p_off = nullptr;
  b.periods = periods;
  b.nperiods_shared = nperiods;
  b.nbins_all = nbins;
  b.qmin_all = qmin;
  b.qmax_all = qmax;
  bls_results o{sr, phase, duration, depth, jstart, kwidth, best_index};
  return bls_search_batch(p, &b, &o);
}

int bls_search_batch(bls_plan *p, const bls_batch *b, const bls_results *out) {
  if (!p) return BLS_ERR_INVALID_ARG;
  if (!b || !out) return set_error(p, BLS_ERR_INVALID_ARG, "batch and out must be non-NULL");
  p->last_error.clear();
  std::string err;
  int st = validate_batch(p->cfg, *b, true, p->shapes, err);
  if (st != BLS_OK) return set_error(p, st, err);
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  return host_search(p, *b, p->shapes, *out);
}

int bls_search_device(bls_plan *p, const bls_batch *b, const bls_device_results *o) {
  if (!p) return BLS_ERR_INVALID_ARG;
  if (!b || !o || !o->sr || !o->depth || !o->jstart || !o->kwidth || !o->best_index)
    return set_error(p, BLS_ERR_INVALID_ARG, "batch and every device result array are required");
  p->last_error.clear();
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  const bool use_graph = (p->cfg.flags & BLS_NO_GRAPH) == 0;
  const uint64_t sig = batch_signature(p, *b, *o);
  if (use_graph && p->graph_valid && sig == p->graph_sig) {
    if ((e = hipEventRecord(p->ev_begin, p->stream)) != hipSuccess) return hip_error(p, e, "event");
    int st = launch_graphs(p);
    if (st != BLS_OK) return st;
    if ((e = hipEventRecord(p->ev_end, p->stream)) != hipSuccess) return hip_error(p, e, "event");
    fill_stats(p, p->last, true);
    return BLS_OK;
  }
  std::string err;
  int st = validate_batch(p->cfg, *b, false, p->shapes, err);
  if (st != BLS_OK) return set_error(p, st, err);
  if (p->gexec[0]) {
    // replays of the old graphs may still be queued: let them finish before
    // their executables go
    if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_error(p, e, "synchronize");
    drop_graph(p);
  }
  const bool weighted = b->weights != nullptr;
  TileChoice tc = choose_tiles(p, p->shapes, weighted);
  PlannedBatch pb;
  st = plan_batch(p, p->shapes, weighted, tc, pb);
  if (st != BLS_OK) return st;
  p->last = pb;
  if ((e = hipEventRecord(p->ev_begin, p->stream)) != hipSuccess) return hip_error(p, e, "event");
  if (use_graph) {
    st = capture_part(p, 0, [&] {
      return enqueue_pre(p, pb, b->times, b->flux, b->weights, b->periods, o->best_index);
    });
    if (st == BLS_OK)
      st = capture_part(p, 1, [&] {
        return enqueue_kernel(p, pb, b->periods, o->sr, o->depth, o->jstart, o->kwidth,
                              o->best_index, false);
      });
    if (st == BLS_OK) st = capture_part(p, 2, [&] { return enqueue_post(p, pb, o->best_index); });
    if (st == BLS_OK) st = launch_graphs(p);
    if (st != BLS_OK) {
      drop_graph(p);
      return st;
    }
    p->graph_sig = sig;
    p->graph_valid = true;
  } else {
    st = enqueue_search(p, pb, b->times, b->flux, b->weights, b->periods, o->sr, o->depth,
                        o->jstart, o->kwidth, o->best_index);
    if (st != BLS_OK) return st;
  }
  if ((e = hipEventRecord(p->ev_end, p->stream)) != hipSuccess) return hip_error(p, e, "event");
  fill_stats(p, pb, false);
  return BLS_OK;
}

int bls_search_unbinned_device(bls_plan *p, const bls_batch *b, const bls_unbinned_results *o) {
  if (!p) return BLS_ERR_INVALID_ARG;
  if (!b || !o || !o->sr || !o->depth || !o->first_point || !o->last_point || !o->best_index)
    return set_error(p, BLS_ERR_INVALID_ARG, "batch and every device result array are required");
  p->last_error.clear();
  std::string err;
  int st = validate_batch(p->cfg, *b, false, p->shapes, err, false);
  if (st != BLS_OK) return set_error(p, st, err);
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  const bool weighted = b->weights != nullptr;
  const int nc = b->ncurves;
  PlannedBatch pb;
  pb.ncurves = nc;
  pb.weighted = weighted;
  std::vector<double> cost(nc);
  int ucap = 1;
  // the pinned descriptors are rewritten: a captured search graph goes
  // stale, and queued copies may still read them
  p->graph_valid = false;
  st = desc_wait(p);
  if (st != BLS_OK) return st;
  for (int c = 0; c < nc; ++c) {
    const CurveShape &s = p->shapes[c];
    CurveDesc &d = p->h_curves[c];
    memset(&d, 0, sizeof d);
    d.n_off = s.n_off;
    d.n = s.n;
    d.p_off = s.p_off;
    d.r_off = s.r_off;
    d.nperiods = s.nperiods;
    d.nbins = 0;
    const int cb = cbits_of(s.n);
    d.shift = 64 - cb;
    d.qbits = std::min(kQBitsMax, 63 - 2 * cb);
    d.weighted = weighted ? 1 : 0;
    d.check_periods = (c == 0 || s.p_off != p->shapes[0].p_off) ? 1 : 0;
    d.tile = 1;
    d.qlo = b->qmin ? b->qmin[c] : b->qmin_all;
    d.qhi = b->qmax ? b->qmax[c] : b->qmax_all;
    ucap = std::max<int>(ucap, (int)s.n);
    // a start's run covers about qhi * n points
    cost[c] = (double)s.n * (1.0 + d.qhi * (double)s.n);
    pb.total_points += s.n;
    pb.total_results += s.nperiods;
    pb.trial_points += (double)s.n * (double)s.nperiods;
    pb.box_evals += (double)s.n * d.qhi * (double)s.n * (double)s.nperiods;
  }
  std::vector<int64_t> items_of(nc);
  for (int c = 0; c < nc; ++c) items_of[c] = p->h_curves[c].nperiods;
  layout_partitions(p, cost, items_of, pb);
  const int64_t items = pb.nitems;
  pb.ucap = ucap;
  // Curves up to kUnbinnedMaxPoints keep their per-point arrays in LDS;
  // longer ones in a device workspace slice per workgroup.
  const bool glob = ucap > kUnbinnedMaxPoints;
  const int64_t arrays = unbinned_lds_bytes(ucap, weighted);
  pb.hist_bytes = glob ? 0 : (int32_t)arrays;
  if (pb.hist_bytes > p->max_lds - 2048)
    return set_error(p, BLS_ERR_CAPACITY, "curve too long for the unbinned search's LDS");
  int per_cu = 0;
  if ((e = (hipError_t)unbinned_blocks_per_cu(weighted, (p->cfg.flags & BLS_DIP_ONLY) != 0, glob,
                                              pb.hist_bytes, &per_cu)) != hipSuccess)
    return hip_error(p, e, "occupancy query");
  if (per_cu < 1) return set_error(p, BLS_ERR_CAPACITY, "unbinned kernel does not fit a CU");
  int64_t grid = std::min<int64_t>(items, (int64_t)p->num_cus * per_cu);
  if (glob) {
    // at most about 1 GiB of workspace (at least 32 workgroups)
    const int64_t stride = (arrays + 255) & ~(int64_t)255;
    grid = std::min<int64_t>(grid, std::max<int64_t>(32, ((int64_t)1 << 30) / stride));
    const int64_t need = grid * stride;
    if (need > p->uws_bytes) {
      // queued unbinned searches may still use the old workspace
      if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_error(p, e, "synchronize");
      free_dev(p->d_uws);
      p->d_uws = nullptr;
      p->uws_bytes = 0;
      if ((e = device_alloc((void **)&p->d_uws, (size_t)need)) != hipSuccess)
        return hip_error(p, e, "allocate unbinned workspace");
      p->uws_bytes = need;
    }
    pb.uws = p->d_uws;
    pb.uws_stride = stride;
  }
  pb.grid = (int32_t)std::max<int64_t>(1, grid);
  p->last = pb;
  if ((e = hipEventRecord(p->ev_begin, p->stream)) != hipSuccess) return hip_error(p, e, "event");
  st = enqueue_search(p, pb, b->times, b->flux, b->weights, b->periods, o->sr, o->depth,
                      o->first_point, o->last_point, o->best_index, true);
  if (st != BLS_OK) return st;
  if ((e = hipEventRecord(p->ev_end, p->stream)) != hipSuccess) return hip_error(p, e, "event");
  fill_stats(p, pb, false);
  return BLS_OK;
}

int bls_detect_device(bls_plan *p, const bls_batch *b, const float *sr, int32_t max_peaks,
                      double window, double sde_threshold, bls_detection *out) {
  if (!p) return BLS_ERR_INVALID_ARG;
  if (!b || !sr || !out || max_peaks < 0 || max_peaks > BLS_MAX_PEAKS || !(window >= 0.0) ||
      !isfinite(window) || isnan(sde_threshold))
    return set_error(p, BLS_ERR_INVALID_ARG,
                     "need batch, sr, out, 0 <= max_peaks <= 16, finite window >= 0");
  std::string err;
  std::vector<CurveShape> shapes;
  int st = validate_batch(p->cfg, *b, false, shapes, err);
  if (st != BLS_OK) return set_error(p, st, err);
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  const int nc = b->ncurves;
  std::vector<DetectDesc> dd(nc);
  for (int c = 0; c < nc; ++c) {
    dd[c].p_off = shapes[c].p_off;
    dd[c].r_off = shapes[c].r_off;
    dd[c].nperiods = shapes[c].nperiods;
  }
  st = ensure_detect_buffers(p);
  if (st != BLS_OK) return st;
  hipStream_t s = p->stream;
  if ((e = hipMemcpyAsync(p->d_detect_desc, dd.data(), sizeof(DetectDesc) * nc,
                          hipMemcpyHostToDevice, s)))
    return hip_error(p, e, "upload detection descriptors");
  DetectArgs a;
  a.desc = p->d_detect_desc;
  a.periods = b->periods;
  a.sr = sr;
  a.out = p->d_detect_out;
  a.ncurves = nc;
  a.max_peaks = max_peaks;
  a.window = window;
  a.threshold = sde_threshold;
  if ((e = hipEventRecord(p->ev_search0, s)) != hipSuccess) return hip_error(p, e, "event");
  if ((e = (hipError_t)launch_detect(a, s))) return hip_error(p, e, "launch detection");
  if ((e = hipEventRecord(p->ev_search1, s)) != hipSuccess) return hip_error(p, e, "event");
  if ((e = hipMemcpyAsync(out, p->d_detect_out, sizeof(bls_detection) * nc,
                          hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s)))
    return hip_error(p, e, "detection");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, p->ev_search0, p->ev_search1);
  p->stats = bls_call_stats{};
  p->stats.search_ms = p->stats.total_ms = ms;
  double m_total = 0.0;
  for (int c = 0; c < nc; ++c) m_total += (double)dd[c].nperiods;
  p->stats.trial_points = m_total;
  p->stats.block = kBlock;
  p->stats.grid = nc;
  return BLS_OK;
}

int bls_eclipse_window_device(bls_plan *p, const bls_batch *b, int32_t nphase, double duration,
                              int32_t min_eclipses, int32_t *observed) {
  if (!p) return BLS_ERR_INVALID_ARG;
  char msg[200];
  if (!b || !observed || b->ncurves < 1 || !b->n_off || !b->times || !b->periods)
    return set_error(p, BLS_ERR_INVALID_ARG,
                     "need a batch with ncurves >= 1, n_off, times, periods, and observed");
  if (nphase < 1 || nphase > BLS_MAX_NBINS || !(duration > 0.0) || !isfinite(duration) ||
      (min_eclipses != 1 && min_eclipses != 2))
    return set_error(p, BLS_ERR_INVALID_ARG,
                     "need 1 <= nphase <= 4096, finite duration > 0, min_eclipses 1 or 2");
  if (b->ncurves > p->cfg.max_curves) return set_error(p, BLS_ERR_CAPACITY, "too many cadences");
  if (b->n_off[0] != 0 || (b->p_off && b->p_off[0] != 0) ||
      (!b->p_off && b->nperiods_shared < 1))
    return set_error(p, BLS_ERR_INVALID_ARG, "n_off[0] and p_off[0] must be 0, grid non-empty");
  const int nc = b->ncurves;
  // up to 32 KB of LDS per workgroup (four periods at 1000 phase bins, one
  // per wave in the window pass): five workgroups per CU
  const int tile = std::max(
      1, std::min(kTileMax, ((32 << 10) - kWindowStaticLds - 8 * window_pad(nphase)) /
                                (8 * nphase)));
  std::vector<WindowDesc> wd(nc);
  int64_t items = 0, results = 0;
  for (int c = 0; c < nc; ++c) {
    WindowDesc &d = wd[c];
    memset(&d, 0, sizeof d);
    d.n_off = b->n_off[c];
    d.n = b->n_off[c + 1] - b->n_off[c];
    const int64_t np = b->p_off ? b->p_off[c + 1] - b->p_off[c] : b->nperiods_shared;
    if (d.n < 1 || np < 1 || np > INT32_MAX) {
      snprintf(msg, sizeof msg, "cadence %d has %lld points and %lld periods (need >= 1 each)", c,
               (long long)d.n, (long long)np);
      return set_error(p, BLS_ERR_INVALID_ARG, msg);
    }
    d.p_off = b->p_off ? b->p_off[c] : 0;
    d.r_off = b->p_off ? b->p_off[c] : (int64_t)c * b->nperiods_shared;
    d.nperiods = (int32_t)np;
    d.check_periods = (b->p_off || c == 0) ? 1 : 0;
    d.item0 = items;
    items += (np + tile - 1) / tile;
    results += np;
  }
  if (b->n_off[nc] > p->cfg.max_points || results > p->cfg.max_periods)
    return set_error(p, BLS_ERR_CAPACITY, "points or periods exceed the plan's limits");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  if (!p->d_window_desc) {
    if ((e = device_alloc((void **)&p->d_window_desc, sizeof(WindowDesc) * p->cfg.max_curves)) ||
        (e = device_alloc((void **)&p->d_window_flag, sizeof(unsigned int)))) {
      if (p->d_window_desc) (void)hipFree(p->d_window_desc);
      p->d_window_desc = nullptr;
      p->d_window_flag = nullptr;
      return hip_error(p, e, "allocate eclipse-window buffers");
    }
  }
  const int lds = window_lds_bytes(tile, nphase);
  int per_cu = 0;
  if ((e = (hipError_t)window_blocks_per_cu(lds, &per_cu)) != hipSuccess)
    return hip_error(p, e, "window occupancy");
  const int64_t grid = std::min<int64_t>(items, (int64_t)std::max(per_cu, 1) * p->num_cus * 4);
  hipStream_t s = p->stream;
  const unsigned int zero = 0;
  if ((e = hipMemcpyAsync(p->d_window_desc, wd.data(), sizeof(WindowDesc) * nc,
                          hipMemcpyHostToDevice, s)) ||
      (e = hipMemcpyAsync(p->d_window_flag, &zero, sizeof zero, hipMemcpyHostToDevice, s)))
    return hip_error(p, e, "upload window descriptors");
  WindowArgs a;
  a.desc = p->d_window_desc;
  a.ncurves = nc;
  a.tile = tile;
  a.nitems = items;
  a.t = b->times;
  a.w = b->weights;
  a.periods = b->periods;
  a.observed = observed;
  a.nphase = nphase;
  a.min_eclipses = min_eclipses;
  a.duration = duration;
  a.overflow = p->d_window_flag;
  if ((e = hipEventRecord(p->ev_search0, s)) != hipSuccess) return hip_error(p, e, "event");
  if ((e = (hipError_t)launch_window(a, (int)grid, s))) return hip_error(p, e, "launch window");
  if ((e = hipEventRecord(p->ev_search1, s)) != hipSuccess) return hip_error(p, e, "event");
  unsigned int flag = 0;
  if ((e = hipMemcpyAsync(wd.data(), p->d_window_desc, sizeof(WindowDesc) * nc,
                          hipMemcpyDeviceToHost, s)) ||
      (e = hipMemcpyAsync(&flag, p->d_window_flag, sizeof flag, hipMemcpyDeviceToHost, s)) ||
      (e = hipStreamSynchronize(s)))
    return hip_error(p, e, "eclipse window");
  {
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, p->ev_search0, p->ev_search1);
    p->stats = bls_call_stats{};
    p->stats.search_ms = p->stats.total_ms = ms;
    double pp = 0.0, dec = 0.0;
    for (int c = 0; c < nc; ++c) {
      pp += (double)wd[c].n * (double)wd[c].nperiods;
      dec += (double)wd[c].nperiods * (double)nphase;
    }
    p->stats.trial_points = pp;
    p->stats.box_evals = dec;
    p->stats.work_items = items;
    p->stats.grid = (int32_t)grid;
    p->stats.block = kBlock;
    p->stats.lds_bytes = lds;
  }
  for (int c = 0; c < nc; ++c) {
    if (wd[c].status != kCurveOk) {
      snprintf(msg, sizeof msg, "cadence %d: %s", c,
               wd[c].status == kCurveBadData     ? "non-finite kept time or a bad weight"
               : wd[c].status == kCurveBadPeriod ? "a trial period is not finite and > 0"
                                                 : "no point with positive weight");
      return set_error(p, BLS_ERR_INVALID_ARG, msg);
    }
  }
  if (flag)
    return set_error(p, BLS_ERR_CAPACITY, "a cadence spans more than 2^29 cycles of a period");
  return BLS_OK;
}

int bls_variability_device(bls_plan *p, const bls_batch *b, const bls_variability_config *cfg,
                           const bls_variability_results *o) {
  if (!p) return BLS_ERR_INVALID_ARG;
  if (!b || !cfg || !o || !b->n_off || !b->flux || !cfg->chip_off || !cfg->mag || !o->rms ||
      !o->bin || !o->flag || !o->bin_mean || !o->bin_std || !o->bin_count)
    return set_error(p, BLS_ERR_INVALID_ARG,
                     "need batch (n_off, flux), config (chip_off, mag) and every result array");
  const int nc = b->ncurves, nk = cfg->nchips;
  if (nc < 1 || nk < 1 || cfg->nmagbins < 1 || !(cfg->width > 0.0) || !isfinite(cfg->width) ||
      !isfinite(cfg->origin) || !(cfg->clip_sigma > 0.0) || !(cfg->flag_sigma >= 0.0) ||
      cfg->max_iter < 0 || cfg->min_stars < 1)
    return set_error(p, BLS_ERR_INVALID_ARG,
                     "need ncurves, nchips, nmagbins >= 1, finite origin, width > 0, "
                     "clip_sigma > 0, flag_sigma >= 0, max_iter >= 0, min_stars >= 1");
  if (nc > p->cfg.max_curves || cfg->nmagbins > kVarMaxBins || cfg->max_iter > kVarMaxIter)
    return set_error(p, BLS_ERR_CAPACITY,
                     "more curves than max_curves, nmagbins > 4096 or max_iter > 64");
  if (b->n_off[0] != 0 || cfg->chip_off[0] != 0 || cfg->chip_off[nk] != nc)
    return set_error(p, BLS_ERR_INVALID_ARG, "n_off[0], chip_off[0] must be 0; "
                                             "chip_off[nchips] must equal ncurves");
  for (int c = 0; c < nc; ++c)
    if (b->n_off[c + 1] < b->n_off[c])
      return set_error(p, BLS_ERR_INVALID_ARG, "n_off must be non-decreasing");
  for (int k = 0; k < nk; ++k)
    if (cfg->chip_off[k + 1] < cfg->chip_off[k])
      return set_error(p, BLS_ERR_INVALID_ARG, "chip_off must be non-decreasing");
  if (b->n_off[nc] > p->cfg.max_points)
    return set_error(p, BLS_ERR_CAPACITY, "points exceed the plan's max_points");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  if (!p->d_var_noff) {
    const size_t mc = (size_t)p->cfg.max_curves;
    if ((e = device_alloc((void **)&p->d_var_noff, 8 * (mc + 1))) ||
        (e = device_alloc((void **)&p->d_var_alive, mc))) {
      free_dev(p->d_var_noff);
      free_dev(p->d_var_alive);
      p->d_var_noff = nullptr;
      p->d_var_alive = nullptr;
      return hip_error(p, e, "allocate variability scratch");
    }
  }
  if (nk > p->var_chip_cap) {
    free_dev(p->d_var_chip);
    p->d_var_chip = nullptr;
    p->var_chip_cap = 0;
    if ((e = device_alloc((void **)&p->d_var_chip, 8 * ((size_t)nk + 1))))
      return hip_error(p, e, "allocate chip offsets");
    p->var_chip_cap = nk;
  }
  hipStream_t s = p->stream;
  if ((e = hipMemcpyAsync(p->d_var_noff, b->n_off, 8 * ((size_t)nc + 1), hipMemcpyHostToDevice,
                          s)) ||
      (e = hipMemcpyAsync(p->d_var_chip, cfg->chip_off, 8 * ((size_t)nk + 1),
                          hipMemcpyHostToDevice, s)))
    return hip_error(p, e, "upload offsets");
  VarArgs a;
  memset(&a, 0, sizeof a);
  a.ncurves = nc;
  a.nchips = nk;
  a.nmagbins = cfg->nmagbins;
  a.max_iter = cfg->max_iter;
  a.min_stars = cfg->min_stars;
  a.n_off = p->d_var_noff;
  a.chip_off = p->d_var_chip;
  a.x = b->flux;
  a.w = b->weights;
  a.mag = cfg->mag;
  a.origin = cfg->origin;
  a.width = cfg->width;
  a.clip_sigma = cfg->clip_sigma;
  a.flag_sigma = cfg->flag_sigma;
  a.rms = o->rms;
  a.bin = o->bin;
  a.flag = o->flag;
  a.bin_mean = o->bin_mean;
  a.bin_std = o->bin_std;
  a.bin_count = o->bin_count;
  a.alive = p->d_var_alive;
  if ((e = hipEventRecord(p->ev_search0, s)) != hipSuccess) return hip_error(p, e, "event");
  if ((e = (hipError_t)launch_variability(a, s))) return hip_error(p, e, "launch variability");
  if ((e = hipEventRecord(p->ev_search1, s)) != hipSuccess) return hip_error(p, e, "event");
  if ((e = hipStreamSynchronize(s))) return hip_error(p, e, "variability");
  float ms = 0.f;
  (void)hipEventElapsedTime(&ms, p->ev_search0, p->ev_search1);
  p->stats = bls_call_stats{};
  p->stats.search_ms = p->stats.total_ms = ms;
  p->stats.trial_points = (double)b->n_off[nc];
  p->stats.box_evals = (double)nc;
  p->stats.block = kBlock;
  return BLS_OK;
}

int bls_debug_phase_bins(bls_plan *p, const double *times, int64_t n, double period,
                         int32_t nbins, int32_t *bins) {
  if (!p) return BLS_ERR_INVALID_ARG;
  if (!times || !bins || n < 2 || !isfinite(period) || !(period > 0.0) || nbins < 2)
    return set_error(p, BLS_ERR_INVALID_ARG, "need times, bins, n >= 2, period > 0, nbins >= 2");
  if (n > p->cfg.max_points || n > (int64_t(1) << 24))
    return set_error(p, BLS_ERR_CAPACITY, "n exceeds the plan's max_points");
  for (int64_t i = 0; i < n; ++i)
    if (!isfinite(times[i])) return set_error(p, BLS_ERR_INVALID_ARG, "non-finite time");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  int st = ensure_staging(p);
  if (st != BLS_OK) return st;
  p->graph_valid = false;
  st = desc_wait(p);
  if (st != BLS_OK) return st;
  CurveDesc &d = p->h_curves[0];
  memset(&d, 0, sizeof d);
  d.n = n;
  d.nperiods = 1;
  d.nbins = nbins;
  const int cb = cbits_of(n);
  d.shift = 64 - cb;
  d.qbits = std::min(kQBitsMax, 63 - 2 * cb);
  hipStream_t s = p->stream;
  if ((e = hipMemcpyAsync(p->d_curves, p->h_curves, sizeof(CurveDesc), hipMemcpyHostToDevice,
                          s)) != hipSuccess ||
      (e = hipMemcpyAsync(p->d_t, times, n * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(p->d_periods, &period, 8, hipMemcpyHostToDevice, s)) != hipSuccess)
    return hip_error(p, e, "upload");
  if ((st = desc_mark(p)) != BLS_OK) return st;
  PrepArgs pa;
  pa.curves = p->d_curves;
  pa.periods = p->d_periods;
  pa.ncurves = 1;
  pa.t = p->d_t;
  pa.x = p->d_t;  // any finite flux: only the time offsets are used
  pa.w = nullptr;
  pa.dt = p->d_dt;
  pa.q = p->d_q;
  pa.qw = p->d_qw;
  if ((e = (hipError_t)launch_prep(pa, s)) != hipSuccess) return hip_error(p, e, "launch prep");
  if ((e = (hipError_t)launch_bins(p->d_dt, n, p->d_periods, nbins, p->d_j, s)) != hipSuccess)
    return hip_error(p, e, "launch bins");
  if ((e = hipMemcpyAsync(bins, p->d_j, n * 4, hipMemcpyDeviceToHost, s)) != hipSuccess)
    return hip_error(p, e, "download bins");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_error(p, e, "synchronize");
  return BLS_OK;
}

int bls_synchronize(bls_plan *p) {
  if (!p) return BLS_ERR_INVALID_ARG;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_error(p, e, "synchronize");
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, p->ev_begin, p->ev_end) == hipSuccess) p->stats.total_ms = ms;
  p->desc_pending = false;
  p->stats.search_ms = last_kernel_ms(p);
  if (p->last.ncurves > 0) return check_device_status(p, p->last.ncurves);
  return BLS_OK;
}

int bls_get_stream(const bls_plan *p, void **stream) {
  if (!p || !stream) return BLS_ERR_INVALID_ARG;
  *stream = (void *)p->stream;
  return BLS_OK;
}

int bls_width_range(int32_t nbins, double qmin, double qmax, int32_t *kmin, int32_t *kmax) {
  return width_range(nbins, qmin, qmax, kmin, kmax);
}

int bls_last_error(const bls_plan *p, char *buf, size_t len) {
  if (!buf || len == 0) return BLS_ERR_INVALID_ARG;
  const char *m = p ? p->last_error.c_str() : g_create_error;
  const size_t n = std::min(len - 1, strlen(m));
  memcpy(buf, m, n);
  buf[n] = '\0';
  return BLS_OK;
}

const char *bls_status_string(int status) {
  switch (status) {
    case BLS_OK: return "ok";
    case BLS_ERR_INVALID_ARG: return "invalid argument";
    case BLS_ERR_NO_MEMORY: return "out of memory";
    case BLS_ERR_DEVICE: return "device (HIP) error";
    case BLS_ERR_CAPACITY: return "exceeds plan capacity";
    case BLS_ERR_BUSY: return "not ready";
    case BLS_ERR_TIMEOUT: return "timed out";
    default: return "unknown status";
  }
}

int bls_last_stats(const bls_plan *p, bls_call_stats *out) {
  if (!p || !out) return BLS_ERR_INVALID_ARG;
  *out = p->stats;
  return BLS_OK;
}

int bls_kernel_times(bls_plan *p, float *ms, int32_t max, int32_t *count) {
  if (!p || !count || max < 0 || (max > 0 && !ms)) return BLS_ERR_INVALID_ARG;
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_error(p, e, "set device");
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_error(p, e, "synchronize");
  const int64_t avail = std::min<int64_t>(p->k_recorded - p->k_base, bls_plan::kTimeRing);
  const int64_t n = std::min<int64_t>(avail, max);
  // the most recent n launches, oldest first
  for (int64_t i = 0; i < n; ++i) {
    const int64_t k = p->k_recorded - n + i;
    const int slot = (int)(k % bls_plan::kTimeRing);
    float v = 0.f;
    if ((e = hipEventElapsedTime(&v, p->ev_k0[slot], p->ev_k1[slot])) != hipSuccess)
      return hip_error(p, e, "event timing");
    ms[i] = v;
  }
  *count = (int32_t)n;
  return BLS_OK;
}

int bls_kernel_times_reset(bls_plan *p) {
  if (!p) return BLS_ERR_INVALID_ARG;
  p->k_base = p->k_recorded;
  return BLS_OK;
}

}  // extern "C"
