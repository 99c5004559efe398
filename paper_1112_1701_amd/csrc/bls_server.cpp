// Serving loop of the BLS library: requests are admitted by device memory,
// stay resident on the device, and are searched by persistent launches
// ("ticks") that mix period tiles of every admitted request (continuous
// batching).  The arithmetic is the search kernel's, so a request's results
// equal those of bls_search on the same input.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "bls_plan.h"
#include "bls_sched.h"

namespace bls {
namespace {

constexpr int kTickBuffers = 2;          // launches in flight
constexpr int64_t kBytesPerPoint = 40;   // t, x, w, dt (8 B), q, qw (4 B)
constexpr int64_t kBytesPerPeriod = 24;  // periods (8 B), sr, depth, jstart, kwidth (4 B)
constexpr size_t kArenaAlign = 64;       // elements

thread_local std::string g_server_create_error;

struct Req {
  uint64_t ticket = 0;
  // inputs: in the pinned pool when it had room (async copies), else here
  std::vector<double> t, x, w, per;
  size_t pin_off = Arena::kFail;
  const double *pt = nullptr, *px = nullptr, *pw = nullptr, *pper = nullptr;
  bool weighted = false;
  int32_t nbins = 0, kmin = 0, kmax = 0;
  int64_t n = 0, np = 0;
  double submit_s = 0, admit_s = 0, done_s = 0;
  int status = BLS_ERR_BUSY;
  bool finished = false;
  // results: in the pinned result pool when it had room (copied without a
  // wait), else in these vectors; o_* point at whichever holds them
  size_t res_off = Arena::kFail;
  std::vector<float> sr, depth;
  std::vector<int32_t> js, ks;
  const float *o_sr = nullptr, *o_depth = nullptr;
  const int32_t *o_js = nullptr, *o_ks = nullptr;
  int64_t best = -1;
  int slot = -1;
  size_t pt_off = 0, pr_off = 0;
  int32_t tile = 1, hstride = 0, ntiles = 0, issued = 0, done_tiles = 0;
  double item_cost = 0;
  uint64_t order = 0;
  double pp = 0, evals = 0;
};

// One tick: period tiles of every kind of admitted request, unit-weight
// segments first (nu of them), then weighted ones; each kind is its own
// persistent launch of the tick, back to back on the server's stream.
struct Tick {
  int buf = 0;
  int nu = 0;
  std::vector<TickSegment> segs;
};

// Result copies of the requests a tick finished, queued on the copy stream;
// ev completes when they have landed in the pinned result pool.
struct Collect {
  hipEvent_t ev = nullptr;
  std::vector<Req *> reqs;
};

// Bytes of a request's block in the pinned result pool: SR, depth, first and
// last bin (4 B per period each, in that order), the best key (8 B) and the
// curve status (4 B, padded).
size_t result_bytes(int64_t np) { return 16 * (size_t)np + 16; }

// Device bytes a request holds while resident (arena elements, aligned).
int64_t request_bytes(int64_t n, int64_t np) {
  const int64_t a = (int64_t)kArenaAlign;
  return ((n + a - 1) / a * a) * kBytesPerPoint + ((np + a - 1) / a * a) * kBytesPerPeriod;
}

int cbits_of(int64_t n) {
  int b = 0;
  while (b < 63 && (int64_t(1) << b) <= n) ++b;
  return b;
}

}  // namespace
}  // namespace bls

using namespace bls;

struct bls_server {
  bls_server_config cfg{};
  int device = 0;
  int num_cus = 0;
  int max_lds = 0;
  // stream: the ticks; up_stream: admitted requests' uploads and prep, which
  // the next tick waits for (ev_up); copy_stream: result copies
  hipStream_t stream = nullptr, copy_stream = nullptr, up_stream = nullptr;
  hipEvent_t ev_up = nullptr;
  bool up_pending = false;

  int64_t cap_pts = 0, cap_per = 0;
  int64_t arena_budget = 0;   // bytes of resident requests allowed at once
  int64_t bytes_peak = 0;     // largest bytes held at once (both regions)
  double *d_t = nullptr, *d_x = nullptr, *d_w = nullptr, *d_dt = nullptr, *d_per = nullptr;
  void *d_txw = nullptr;  // d_t, d_x, d_w: one block, cap_pts apart
  int32_t *d_q = nullptr, *d_qw = nullptr, *d_js = nullptr, *d_ks = nullptr;
  float *d_sr = nullptr, *d_depth = nullptr;
  void *d_res = nullptr;  // d_sr, d_depth, d_js, d_ks: one block, cap_per apart
  CurveDesc *d_curves = nullptr, *h_curves = nullptr;
  unsigned long long *d_keys = nullptr;
  // a tick's segment arrays (starts, curves, first tiles), packed for its
  // segment count into one block per buffer and sent in one copy
  char *d_seg[kTickBuffers] = {}, *h_seg[kTickBuffers] = {};
  int64_t *d_seg_start[kTickBuffers] = {};
  int32_t *d_seg_curve[kTickBuffers] = {}, *d_seg_tile0[kTickBuffers] = {};
  unsigned long long *d_counter[kTickBuffers] = {};
  hipEvent_t ev_s[kTickBuffers] = {}, ev_e[kTickBuffers] = {};
  bool buf_busy[kTickBuffers] = {};

  Arena pts_arena, per_arena;
  char *h_pool = nullptr;   // pinned staging for request inputs
  Arena pool_arena;
  char *h_res = nullptr;    // pinned result pool (blocks of result_bytes)
  Arena res_arena;
  std::deque<Collect> collecting;
  std::vector<hipEvent_t> ev_free;
  std::vector<Req *> slots;
  std::deque<Req *> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Req>> reqs;
  std::deque<Tick> inflight;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::thread thr;
  bool stop = false;
  uint64_t next_ticket = 1, next_order = 1;

  int64_t submitted = 0, admitted = 0, completed = 0, failed = 0, ticks = 0;
  double pp_done = 0, evals_done = 0, busy_s = 0;
  std::chrono::steady_clock::time_point t0, t_reset;
  LatencyLog lat;
  std::string last_error;
  int lds_budget = 32768;
  double tick_cost = 0;
  int device_error = 0;
};

namespace {

double now_s(const bls_server *s) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t0).count();
}

int srv_error(bls_server *s, int st, const std::string &msg) {
  if (s)
    s->last_error = msg;
  else
    g_server_create_error = msg;
  return st;
}

int srv_hip(bls_server *s, hipError_t e, const char *what) {
  return srv_error(s, e == hipErrorOutOfMemory ? BLS_ERR_NO_MEMORY : BLS_ERR_DEVICE,
                   std::string(what) + ": " + hipGetErrorString(e));
}

// Fail every unfinished request (device error in the scheduler).
void fail_all(bls_server *s, int st) {
  for (auto &kv : s->reqs) {
    Req *r = kv.second.get();
    if (!r->finished) {
      r->finished = true;
      r->status = st;
      r->done_s = now_s(s);
      s->failed++;
    }
  }
  s->pending.clear();
  for (auto &sl : s->slots) sl = nullptr;
  s->cv_done.notify_all();
}

// Device work for a newly admitted request: inputs, descriptor, prep, key,
// on the upload stream (they overlap the ticks in flight).
hipError_t start_request(bls_server *s, Req *r) {
  CurveDesc &d = s->h_curves[r->slot];
  memset(&d, 0, sizeof d);
  d.n_off = (int64_t)r->pt_off;
  d.n = r->n;
  d.p_off = (int64_t)r->pr_off;
  d.r_off = (int64_t)r->pr_off;
  d.nperiods = (int32_t)r->np;
  d.nbins = r->nbins;
  d.kmin = r->kmin;
  d.kmax = r->kmax;
  d.tile = r->tile;
  d.hstride = r->hstride;
  const int cb = cbits_of(r->n);
  d.shift = 64 - cb;
  d.qbits = std::min(kQBitsMax, 63 - 2 * cb);
  d.weighted = r->weighted ? 1 : 0;
  d.check_periods = 0;  // checked on the host at submit
  hipStream_t st = s->up_stream;
  hipError_t e;
  const size_t n = (size_t)r->n, np = (size_t)r->np;
  if (r->pin_off != Arena::kFail) {
    // staged rows at equal pitch in the pinned pool: one pitched copy
    const size_t step = (size_t)(r->px - r->pt) * 8;
    if ((e = hipMemcpy2DAsync(s->d_t + r->pt_off, (size_t)s->cap_pts * 8, r->pt, step, n * 8,
                              r->weighted ? 3 : 2, hipMemcpyHostToDevice, st)))
      return e;
  } else if ((e = hipMemcpyAsync(s->d_t + r->pt_off, r->pt, n * 8, hipMemcpyHostToDevice, st)) ||
             (e = hipMemcpyAsync(s->d_x + r->pt_off, r->px, n * 8, hipMemcpyHostToDevice, st)) ||
             (r->weighted && (e = hipMemcpyAsync(s->d_w + r->pt_off, r->pw, n * 8,
                                                 hipMemcpyHostToDevice, st)))) {
    return e;
  }
  if ((e = hipMemcpyAsync(s->d_per + r->pr_off, r->pper, np * 8, hipMemcpyHostToDevice,
                          st)) ||
      (e = hipMemcpyAsync(s->d_curves + r->slot, &d, sizeof d, hipMemcpyHostToDevice, st)))
    return e;
  if ((e = (hipError_t)launch_fill(nullptr, s->d_keys + r->slot, 1, st))) return e;
  PrepArgs pa;
  pa.curves = s->d_curves + r->slot;
  pa.periods = s->d_per;
  pa.ncurves = 1;
  pa.t = s->d_t;
  pa.x = s->d_x;
  pa.w = r->weighted ? s->d_w : nullptr;
  pa.dt = s->d_dt;
  pa.q = s->d_q;
  pa.qw = s->d_qw;
  return (hipError_t)launch_prep(pa, st);
}

// One persistent launch over segments [s0, s0 + n) of the tick's arrays;
// seg_start holds n + 1 entries from sbase.
hipError_t launch_kind(bls_server *s, int b, bool weighted, int s0, int sbase, int n,
                       int64_t items, int hist_bytes, unsigned long long *counter) {
  if (n == 0 || items == 0) return hipSuccess;
  SearchArgs a;
  memset(&a, 0, sizeof a);
  a.curves = s->d_curves;
  a.periods = s->d_per;
  a.dt = s->d_dt;
  a.q = s->d_q;
  a.qw = weighted ? s->d_qw : nullptr;
  a.seg_start = s->d_seg_start[b] + sbase;
  a.seg_curve = s->d_seg_curve[b] + s0;
  a.seg_tile0 = s->d_seg_tile0[b] + s0;
  a.nseg = n;
  a.min_in_points = s->cfg.min_in_points;
  a.nitems = items;
  a.counter = counter;
  a.sr = s->d_sr;
  a.depth = s->d_depth;
  a.jstart = s->d_js;
  a.kwidth = s->d_ks;
  a.best_key = s->d_keys;
  a.hist_bytes = hist_bytes;
  single_partition(a);
  const bool dip = (s->cfg.flags & BLS_DIP_ONLY) != 0;
  int per_cu = 1;
  hipError_t e = (hipError_t)search_blocks_per_cu(weighted, dip, hist_bytes, &per_cu);
  if (e != hipSuccess) return e;
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)s->num_cus *
                                                                          std::max(per_cu, 1)));
  return (hipError_t)launch_search(a, weighted, dip, (int)grid, s->stream);
}

hipError_t launch_tick(bls_server *s, Tick &tk) {
  const int b = tk.buf;
  const int nseg = (int)tk.segs.size();
  const int nu = tk.nu, nw = nseg - nu;
  // seg_start: the unit-weight launch's nu + 1 entries, then the weighted
  // launch's nw + 1; seg_curve and seg_tile0: nu, then nw entries.  Packed
  // in that order: 8 (nseg + 2) + 4 nseg + 4 nseg bytes.
  const size_t o_curve = 8 * (size_t)(nseg + 2), o_tile0 = o_curve + 4 * (size_t)nseg;
  int64_t *h_start = reinterpret_cast<int64_t *>(s->h_seg[b]);
  int32_t *h_curve = reinterpret_cast<int32_t *>(s->h_seg[b] + o_curve);
  int32_t *h_tile0 = reinterpret_cast<int32_t *>(s->h_seg[b] + o_tile0);
  s->d_seg_start[b] = reinterpret_cast<int64_t *>(s->d_seg[b]);
  s->d_seg_curve[b] = reinterpret_cast<int32_t *>(s->d_seg[b] + o_curve);
  s->d_seg_tile0[b] = reinterpret_cast<int32_t *>(s->d_seg[b] + o_tile0);
  int64_t items[2] = {0, 0};
  int hist[2] = {0, 0};
  for (int i = 0; i < nseg; ++i) {
    const TickSegment &g = tk.segs[i];
    const int kind = i < nu ? 0 : 1;
    h_start[i + kind] = items[kind];
    h_curve[i] = g.slot;
    h_tile0[i] = g.tile0;
    items[kind] += g.ntiles;
    const Req *r = s->slots[g.slot];
    hist[kind] = std::max(hist[kind], r->tile * r->hstride * 8 * (kind ? 2 : 1));
  }
  h_start[nu] = items[0];
  h_start[nseg + 1] = items[1];
  hipStream_t st = s->stream;
  hipError_t e;
  if ((e = hipMemcpyAsync(s->d_seg[b], s->h_seg[b], o_tile0 + 4 * (size_t)nseg,
                          hipMemcpyHostToDevice, st)))
    return e;
  // eight counters: the unit-weight launch takes the first, the weighted the fifth
  if ((e = (hipError_t)launch_fill(s->d_counter[b], nullptr, 0, st))) return e;
  if ((e = hipEventRecord(s->ev_s[b], st))) return e;
  if ((e = launch_kind(s, b, false, 0, 0, nu, items[0], hist[0], s->d_counter[b]))) return e;
  if ((e = launch_kind(s, b, true, nu, nu + 1, nw, items[1], hist[1], s->d_counter[b] + 4)))
    return e;
  return hipEventRecord(s->ev_e[b], st);
}

// Results of a finished request (the tick that completed its last tile has
// finished, so nothing on the device still writes them).  With a block in
// the pinned result pool the copies are queued on the copy stream and the
// request completes once they have landed (*queued); without one they are
// copied into host vectors at once.
hipError_t collect_request(bls_server *s, Req *r, bool *queued) {
  const size_t np = (size_t)r->np;
  hipStream_t cs = s->copy_stream;
  hipError_t e;
  *queued = false;
  if (r->res_off != Arena::kFail) {
    char *b = s->h_res + r->res_off;
    // the four result arrays are rows of one pitched block on the device
    if ((e = hipMemcpy2DAsync(b, np * 4, s->d_sr + r->pr_off, (size_t)s->cap_per * 4, np * 4, 4,
                              hipMemcpyDeviceToHost, cs)) ||
        (e = hipMemcpyAsync(b + 16 * np, s->d_keys + r->slot, 8, hipMemcpyDeviceToHost, cs)) ||
        (e = hipMemcpyAsync(b + 16 * np + 8, &s->d_curves[r->slot].status, 4,
                            hipMemcpyDeviceToHost, cs)))
      return e;
    *queued = true;
    return hipSuccess;
  }
  r->sr.resize(np);
  r->depth.resize(np);
  r->js.resize(np);
  r->ks.resize(np);
  unsigned long long key = 0;
  int32_t status = 0;
  if ((e = hipMemcpyAsync(r->sr.data(), s->d_sr + r->pr_off, np * 4, hipMemcpyDeviceToHost, cs)) ||
      (e = hipMemcpyAsync(r->depth.data(), s->d_depth + r->pr_off, np * 4, hipMemcpyDeviceToHost,
                          cs)) ||
      (e = hipMemcpyAsync(r->js.data(), s->d_js + r->pr_off, np * 4, hipMemcpyDeviceToHost, cs)) ||
      (e = hipMemcpyAsync(r->ks.data(), s->d_ks + r->pr_off, np * 4, hipMemcpyDeviceToHost, cs)) ||
      (e = hipMemcpyAsync(&key, s->d_keys + r->slot, 8, hipMemcpyDeviceToHost, cs)) ||
      (e = hipMemcpyAsync(&status, &s->d_curves[r->slot].status, 4, hipMemcpyDeviceToHost, cs)) ||
      (e = hipStreamSynchronize(cs)))
    return e;
  r->o_sr = r->sr.data();
  r->o_depth = r->depth.data();
  r->o_js = r->js.data();
  r->o_ks = r->ks.data();
  r->best = (int64_t)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
  r->status = status == kCurveOk ? BLS_OK : BLS_ERR_INVALID_ARG;
  return hipSuccess;
}

// Key, status and result pointers of a request whose queued copies landed.
void read_pinned_results(bls_server *s, Req *r) {
  const size_t np = (size_t)r->np;
  const char *b = s->h_res + r->res_off;
  unsigned long long key = 0;
  int32_t status = 0;
  memcpy(&key, b + 16 * np, 8);
  memcpy(&status, b + 16 * np + 8, 4);
  r->o_sr = reinterpret_cast<const float *>(b);
  r->o_depth = r->o_sr + np;
  r->o_js = reinterpret_cast<const int32_t *>(r->o_depth + np);
  r->o_ks = r->o_js + np;
  r->best = (int64_t)(0xFFFFFFFFu - (unsigned)(key & 0xFFFFFFFFull));
  r->status = status == kCurveOk ? BLS_OK : BLS_ERR_INVALID_ARG;
}

// A request whose results are on the host: its device room and slot go back
// (the lock is held).
void complete_request(bls_server *s, Req *r) {
  r->done_s = now_s(s);
  r->finished = true;
  s->slots[r->slot] = nullptr;
  s->pts_arena.release(r->pt_off);
  if (r->pin_off != Arena::kFail) {
    s->pool_arena.release(r->pin_off);  // its copies finished long ago
    r->pin_off = Arena::kFail;
  }
  s->per_arena.release(r->pr_off);
  if (r->status == BLS_OK) {
    s->completed++;
    s->pp_done += r->pp;
    s->evals_done += r->evals;
    s->lat.add((r->done_s - r->submit_s) * 1e3);
  } else {
    s->failed++;
  }
}

void scheduler(bls_server *s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  int next_buf = 0;
  while (!s->stop) {
    bool progressed = false;

    // 1. Completed ticks: count tiles, finish requests, free their memory.
    while (!s->inflight.empty()) {
      Tick &tk = s->inflight.front();
      hipError_t q = hipEventQuery(s->ev_e[tk.buf]);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) {
        s->device_error = BLS_ERR_DEVICE;
        srv_hip(s, q, "search launch");
        fail_all(s, BLS_ERR_DEVICE);
        s->inflight.clear();
        break;
      }
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, s->ev_s[tk.buf], s->ev_e[tk.buf]) == hipSuccess)
        s->busy_s += ms * 1e-3;
      std::vector<Req *> done;
      for (const TickSegment &g : tk.segs) {
        Req *r = s->slots[g.slot];
        if (!r) continue;
        r->done_tiles += g.ntiles;
        if (r->done_tiles == r->ntiles) done.push_back(r);
      }
      s->buf_busy[tk.buf] = false;
      s->inflight.pop_front();
      if (!done.empty()) {
        Collect col;
        std::vector<Req *> now;  // copied at once (no room in the result pool)
        lk.unlock();
        hipError_t e = hipSuccess;
        for (Req *r : done) {
          bool queued = false;
          if (e == hipSuccess) e = collect_request(s, r, &queued);
          (queued ? col.reqs : now).push_back(r);
        }
        if (e == hipSuccess && !col.reqs.empty()) {
          if (!s->ev_free.empty()) {
            col.ev = s->ev_free.back();
            s->ev_free.pop_back();
          } else {
            e = hipEventCreateWithFlags(&col.ev, hipEventDisableTiming);
          }
          if (e == hipSuccess) e = hipEventRecord(col.ev, s->copy_stream);
        }
        lk.lock();
        if (e != hipSuccess) {
          if (col.ev) s->ev_free.push_back(col.ev);
          s->device_error = BLS_ERR_DEVICE;
          srv_hip(s, e, "collect results");
          fail_all(s, BLS_ERR_DEVICE);
          break;
        }
        for (Req *r : now) complete_request(s, r);
        if (!now.empty()) s->cv_done.notify_all();
        if (!col.reqs.empty()) s->collecting.push_back(std::move(col));
      }
      progressed = true;
    }
    if (s->device_error) break;

    // 1b. Result copies that have landed: their requests are done.
    while (!s->collecting.empty()) {
      Collect &col = s->collecting.front();
      hipError_t q = hipEventQuery(col.ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) {
        s->device_error = BLS_ERR_DEVICE;
        srv_hip(s, q, "result copies");
        fail_all(s, BLS_ERR_DEVICE);
        break;
      }
      for (Req *r : col.reqs) {
        read_pinned_results(s, r);
        complete_request(s, r);
      }
      s->ev_free.push_back(col.ev);
      s->collecting.pop_front();
      s->cv_done.notify_all();
      progressed = true;
    }
    if (s->device_error) break;

    // 2. Admission, oldest first, while a slot and arena room are free.
    std::vector<Req *> admitted;
    while (!s->pending.empty()) {
      Req *r = s->pending.front();
      int slot = -1;
      for (int i = 0; i < (int)s->slots.size(); ++i)
        if (!s->slots[i]) {
          slot = i;
          break;
        }
      if (slot < 0) break;
      const int64_t held = (int64_t)(s->pts_arena.in_use() * kBytesPerPoint +
                                     s->per_arena.in_use() * kBytesPerPeriod);
      if (held + request_bytes(r->n, r->np) > s->arena_budget) break;
      const size_t po = s->pts_arena.alloc((size_t)r->n);
      if (po == Arena::kFail) break;
      const size_t pr = s->per_arena.alloc((size_t)r->np);
      if (pr == Arena::kFail) {
        s->pts_arena.release(po);
        break;
      }
      s->bytes_peak = std::max(s->bytes_peak,
                               (int64_t)(s->pts_arena.in_use() * kBytesPerPoint +
                                         s->per_arena.in_use() * kBytesPerPeriod));
      r->slot = slot;
      r->pt_off = po;
      r->pr_off = pr;
      r->admit_s = now_s(s);
      r->order = s->next_order++;
      s->slots[slot] = r;
      s->pending.pop_front();
      s->admitted++;
      admitted.push_back(r);
    }

    // 3. Next launch if a buffer is free and tiles remain.
    bool have_tick = false;
    Tick tk;
    if (!s->buf_busy[next_buf]) {
      std::vector<SlotWork> work;
      for (int i = 0; i < (int)s->slots.size(); ++i) {
        Req *r = s->slots[i];
        if (r && r->issued < r->ntiles)
          work.push_back({i, r->order, r->ntiles, r->issued, r->item_cost});
      }
      if (!work.empty()) {
        tk.buf = next_buf;
        tk.segs = build_tick(work, s->tick_cost, 1);
        // unit-weight segments first: each kind is one launch of the tick
        std::stable_partition(tk.segs.begin(), tk.segs.end(), [&](const TickSegment &g) {
          return !s->slots[g.slot]->weighted;
        });
        tk.nu = 0;
        for (const TickSegment &g : tk.segs) tk.nu += s->slots[g.slot]->weighted ? 0 : 1;
        for (const SlotWork &wk : work) s->slots[wk.slot]->issued = wk.next_tile;
        have_tick = !tk.segs.empty();
      }
    }

    // Device work outside the lock (requests and slots stay put: only this
    // thread frees them).
    if (!admitted.empty() || have_tick) {
      lk.unlock();
      hipError_t e = hipSuccess;
      for (Req *r : admitted)
        if (e == hipSuccess) e = start_request(s, r);
      if (e == hipSuccess && !admitted.empty()) {
        e = hipEventRecord(s->ev_up, s->up_stream);
        s->up_pending = true;
      }
      // a tick holds tiles of every admitted request: it starts after their
      // uploads and prep
      if (e == hipSuccess && have_tick && s->up_pending) {
        e = hipStreamWaitEvent(s->stream, s->ev_up, 0);
        s->up_pending = false;
      }
      if (e == hipSuccess && have_tick) e = launch_tick(s, tk);
      lk.lock();
      if (e != hipSuccess) {
        s->device_error = BLS_ERR_DEVICE;
        srv_hip(s, e, "enqueue");
        fail_all(s, BLS_ERR_DEVICE);
        break;
      }
      if (have_tick) {
        s->buf_busy[tk.buf] = true;
        s->inflight.push_back(std::move(tk));
        s->ticks++;
        next_buf = (next_buf + 1) % kTickBuffers;
      }
      progressed = true;
    }

    if (!progressed) {
      if (s->inflight.empty() && s->collecting.empty())
        s->cv_work.wait_for(lk, std::chrono::milliseconds(50));
      else
        s->cv_work.wait_for(lk, std::chrono::microseconds(50));
    }
  }
  lk.unlock();
  (void)hipStreamSynchronize(s->stream);
}

}  // namespace

extern "C" {

void bls_server_config_init(bls_server_config *cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof *cfg);
  cfg->device = 0;
  cfg->max_slots = 256;
  cfg->arena_bytes = int64_t(4) << 30;
  cfg->max_nbins = BLS_MAX_NBINS;
  cfg->min_in_points = 1;
  cfg->flags = 0;
  cfg->tick_cost = 0.0;
  cfg->max_request_points = int64_t(1) << 20;
  cfg->max_request_periods = int64_t(1) << 20;
}

int bls_server_destroy(bls_server *s);

int bls_server_create(bls_server **out, const bls_server_config *cfg_in) {
  if (!out) return srv_error(nullptr, BLS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  bls_server_config cfg;
  if (cfg_in)
    cfg = *cfg_in;
  else
    bls_server_config_init(&cfg);
  if (cfg.min_in_points <= 0) cfg.min_in_points = 1;
  if (cfg.max_slots < 1 || cfg.max_slots > 65536 || cfg.arena_bytes < (1 << 20) ||
      cfg.max_nbins < 2 || cfg.max_nbins > BLS_MAX_NBINS || cfg.max_request_points < 2 ||
      cfg.max_request_points > (int64_t(1) << 24) || cfg.max_request_periods < 1 ||
      cfg.max_request_periods > INT32_MAX || cfg.tick_cost < 0.0)
    return srv_error(nullptr, BLS_ERR_INVALID_ARG, "bad server configuration");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0)
    return srv_error(nullptr, BLS_ERR_DEVICE, "no HIP device available");
  if (cfg.device < 0 || cfg.device >= ndev)
    return srv_error(nullptr, BLS_ERR_INVALID_ARG, "device ordinal out of range");

  bls_server *s = new (std::nothrow) bls_server();
  if (!s) return srv_error(nullptr, BLS_ERR_NO_MEMORY, "host allocation");
  s->cfg = cfg;
  s->device = cfg.device;
  s->t0 = s->t_reset = std::chrono::steady_clock::now();
  auto fail = [&](int st) {
    g_server_create_error = s->last_error;
    bls_server_destroy(s);
    return st;
  };
  if ((e = hipSetDevice(s->device))) return fail(srv_hip(s, e, "set device"));
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, s->device))) return fail(srv_hip(s, e, "properties"));
  s->num_cus = prop.multiProcessorCount;
  s->max_lds = (int)prop.sharedMemPerBlock;
  if ((e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking)) ||
      (e = hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking)) ||
      (e = hipStreamCreateWithFlags(&s->up_stream, hipStreamNonBlocking)) ||
      (e = hipEventCreateWithFlags(&s->ev_up, hipEventDisableTiming)))
    return fail(srv_hip(s, e, "create streams"));

  // Arena: point arrays and period arrays in two address ranges, each able
  // to take the whole byte budget, so that any mix of request shapes fits;
  // admission counts the bytes both ranges hold against the budget (the
  // reservation is twice arena_bytes).
  s->arena_budget = cfg.arena_bytes;
  s->cap_pts = cfg.arena_bytes / kBytesPerPoint;
  s->cap_per = cfg.arena_bytes / kBytesPerPeriod;
  const size_t P = (size_t)s->cap_pts, Q = (size_t)s->cap_per, M = (size_t)cfg.max_slots;
  struct {
    void **ptr;
    size_t bytes;
  } req[] = {{(void **)&s->d_txw, 24 * P},     {(void **)&s->d_dt, 8 * P},
             {(void **)&s->d_q, 4 * P},        {(void **)&s->d_qw, 4 * P},
             {(void **)&s->d_per, 8 * Q},      {(void **)&s->d_res, 16 * Q},
             {(void **)&s->d_curves, sizeof(CurveDesc) * M},
             {(void **)&s->d_keys, 8 * M}};
  for (auto &r : req)
    if ((e = device_alloc(r.ptr, r.bytes))) return fail(srv_hip(s, e, "allocate arena"));
  // times, values and weights as rows of one block, and the result arrays
  // as rows of another, so that one pitched copy moves a request's rows
  s->d_t = static_cast<double *>(s->d_txw);
  s->d_x = s->d_t + P;
  s->d_w = s->d_x + P;
  s->d_sr = static_cast<float *>(s->d_res);
  s->d_depth = s->d_sr + Q;
  s->d_js = reinterpret_cast<int32_t *>(s->d_depth + Q);
  s->d_ks = s->d_js + Q;
  for (int b = 0; b < kTickBuffers; ++b) {
    if ((e = device_alloc((void **)&s->d_seg[b], 16 * (M + 1))) ||
        (e = device_alloc((void **)&s->d_counter[b], 64)))
      return fail(srv_hip(s, e, "allocate tick buffers"));
    if ((e = hipHostMalloc((void **)&s->h_seg[b], 16 * (M + 1), 0)))
      return fail(srv_hip(s, e, "allocate pinned tick buffers"));
    if ((e = hipEventCreate(&s->ev_s[b])) || (e = hipEventCreate(&s->ev_e[b])))
      return fail(srv_hip(s, e, "create events"));
  }
  if ((e = hipHostMalloc((void **)&s->h_curves, sizeof(CurveDesc) * M, 0)))
    return fail(srv_hip(s, e, "allocate pinned descriptors"));
  s->pts_arena.reset(P, kArenaAlign);
  s->per_arena.reset(Q, kArenaAlign);
  s->slots.assign(M, nullptr);
  {
    // pinned staging: a quarter of the device arena, at most 1 GiB; requests
    // that do not fit are staged in pageable memory instead
    const size_t pool = (size_t)std::min<int64_t>(cfg.arena_bytes / 4, int64_t(1) << 30);
    if (hipHostMalloc((void **)&s->h_pool, pool, 0) == hipSuccess)
      s->pool_arena.reset(pool, 256);
    else
      s->h_pool = nullptr;
    // pinned results: half the device arena, at most 2 GiB (a finished
    // request holds its block until it is released); results that do not fit
    // are copied into pageable memory with a wait instead
    const size_t rpool = (size_t)std::min<int64_t>(cfg.arena_bytes / 2, int64_t(2) << 30);
    if (hipHostMalloc((void **)&s->h_res, rpool, 0) == hipSuccess)
      s->res_arena.reset(rpool, 256);
    else
      s->h_res = nullptr;
  }
  // 20 KB of LDS per request tile leaves room for 8 workgroups per CU.  On
  // the serving sweep it beat the batch path's 32 KB (p99 at 1000 requests/s
  // 8.5-9.1 ms against 10.4-10.7, saturation about 4% higher) and 16 KB;
  // one-curve batch calls, by contrast, are faster with 32 KB tiles.
  s->lds_budget = 20480;
  // about 40 launches' worth of work per second at full rate keeps launch
  // overhead negligible while new requests wait at most a few milliseconds
  s->tick_cost = cfg.tick_cost > 0.0 ? cfg.tick_cost : 4.0e9;
  s->thr = std::thread(scheduler, s);
  *out = s;
  return BLS_OK;
}

int bls_server_submit(bls_server *s, const bls_request *q, uint64_t *ticket) {
  if (!s) return BLS_ERR_INVALID_ARG;
  if (!q || !ticket) return srv_error(s, BLS_ERR_INVALID_ARG, "request and ticket are required");
  if (q->n > s->cfg.max_request_points || q->nperiods > s->cfg.max_request_periods) {
    std::lock_guard<std::mutex> g(s->mu);
    return srv_error(s, BLS_ERR_CAPACITY, "request exceeds max_request_points/periods");
  }
  if (q->nbins > s->cfg.max_nbins) {
    std::lock_guard<std::mutex> g(s->mu);
    return srv_error(s, BLS_ERR_CAPACITY, "nbins exceeds max_nbins");
  }
  // Same checks as the single-curve search, on the host.
  int64_t n_off[2] = {0, q->n};
  bls_batch b;
  memset(&b, 0, sizeof b);
  b.ncurves = 1;
  b.n_off = n_off;
  b.times = q->times;
  b.flux = q->flux;
  b.weights = q->weights;
  b.periods = q->periods;
  b.nperiods_shared = q->nperiods;
  b.nbins_all = q->nbins;
  b.qmin_all = q->qmin;
  b.qmax_all = q->qmax;
  bls_plan_config pc;
  bls_plan_config_init(&pc);
  pc.max_points = q->n > 2 ? q->n : 2;
  pc.max_periods = q->nperiods > 1 ? q->nperiods : 1;
  pc.max_nbins = s->cfg.max_nbins;
  std::vector<CurveShape> shapes;
  std::string err;
  int st = q->n < 2 ? BLS_ERR_INVALID_ARG : validate_batch(pc, b, true, shapes, err);
  if (st != BLS_OK) {
    std::lock_guard<std::mutex> g(s->mu);
    return srv_error(s, st, q->n < 2 ? "need n >= 2" : err);
  }
  const CurveShape &cs = shapes[0];
  auto r = std::make_unique<Req>();
  r->n = q->n;
  r->np = q->nperiods;
  r->nbins = cs.nbins;
  r->kmin = cs.kmin;
  r->kmax = cs.kmax;
  r->weighted = q->weights != nullptr;
  {
    const size_t n8 = (size_t)q->n * 8, p8 = (size_t)q->nperiods * 8;
    const size_t need = 3 * ((n8 + 255) & ~size_t(255)) + p8;
    size_t off = Arena::kFail;
    if (s->h_pool || s->h_res) {
      std::lock_guard<std::mutex> g(s->mu);
      if (s->h_pool) off = s->pool_arena.alloc(need);
      if (s->h_res) r->res_off = s->res_arena.alloc(result_bytes(q->nperiods));
    }
    if (off != Arena::kFail) {
      char *base = s->h_pool + off;
      const size_t step = (n8 + 255) & ~size_t(255);
      double *dt_ = (double *)base, *dx = (double *)(base + step),
             *dw = (double *)(base + 2 * step), *dp = (double *)(base + 3 * step);
      memcpy(dt_, q->times, n8);
      memcpy(dx, q->flux, n8);
      if (r->weighted) memcpy(dw, q->weights, n8);
      memcpy(dp, q->periods, p8);
      r->pin_off = off;
      r->pt = dt_;
      r->px = dx;
      r->pw = r->weighted ? dw : nullptr;
      r->pper = dp;
    } else {
      r->t.assign(q->times, q->times + q->n);
      r->x.assign(q->flux, q->flux + q->n);
      if (r->weighted) r->w.assign(q->weights, q->weights + q->n);
      r->per.assign(q->periods, q->periods + q->nperiods);
      r->pt = r->t.data();
      r->px = r->x.data();
      r->pw = r->weighted ? r->w.data() : nullptr;
      r->pper = r->per.data();
    }
  }
  const int wpb = r->weighted ? 2 : 1;
  int T = 1, hs = 0;
  fit_tile(r->nbins, r->kmax, r->np, s->lds_budget, kTileMax, r->weighted, &T, &hs);
  const int per_period = hs * 8 * wpb;
  r->tile = T;
  r->hstride = hs;
  r->ntiles = (int32_t)((r->np + T - 1) / T);
  const double nw = (double)(r->kmax - r->kmin + 1);
  r->item_cost = (double)T * ((double)r->n + 1.6 * (double)r->nbins * nw);
  r->pp = (double)r->n * (double)r->np;
  r->evals = (double)r->nbins * nw * (double)r->np;

  std::lock_guard<std::mutex> g(s->mu);
  int reject = BLS_OK;
  if (s->device_error)
    reject = srv_error(s, BLS_ERR_DEVICE, "server stopped after a device error");
  else if (request_bytes(r->n, r->np) > s->arena_budget || !s->pts_arena.fits_ever((size_t)r->n) ||
           !s->per_arena.fits_ever((size_t)r->np) || per_period > s->max_lds - 1024)
    reject = srv_error(s, BLS_ERR_CAPACITY, "request larger than the server's device arena");
  if (reject != BLS_OK) {
    if (r->pin_off != Arena::kFail) s->pool_arena.release(r->pin_off);
    if (r->res_off != Arena::kFail) s->res_arena.release(r->res_off);
    return reject;
  }
  r->ticket = s->next_ticket++;
  r->submit_s = now_s(s);
  *ticket = r->ticket;
  s->pending.push_back(r.get());
  s->reqs[r->ticket] = std::move(r);
  s->submitted++;
  s->cv_work.notify_one();
  return BLS_OK;
}

static void fill_result(const Req *r, bls_result *out) {
  memset(out, 0, sizeof *out);
  out->status = r->status;
  out->nperiods = r->status == BLS_OK ? r->np : 0;
  out->sr = r->o_sr;
  out->depth = r->o_depth;
  out->jstart = r->o_js;
  out->kwidth = r->o_ks;
  out->best_index = r->best;
  out->submit_s = r->submit_s;
  out->admit_s = r->admit_s;
  out->done_s = r->done_s;
}

int bls_server_poll(bls_server *s, uint64_t ticket, bls_result *out) {
  if (!s || !out) return BLS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return srv_error(s, BLS_ERR_INVALID_ARG, "unknown ticket");
  if (!it->second->finished) return BLS_ERR_BUSY;
  fill_result(it->second.get(), out);
  return BLS_OK;
}

int bls_server_wait(bls_server *s, uint64_t ticket, bls_result *out, double timeout_s) {
  if (!s || !out) return BLS_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return srv_error(s, BLS_ERR_INVALID_ARG, "unknown ticket");
  Req *r = it->second.get();
  const auto deadline =
      std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(0.0, timeout_s));
  while (!r->finished) {
    if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !r->finished)
      return BLS_ERR_TIMEOUT;
  }
  fill_result(r, out);
  return BLS_OK;
}

int bls_server_release(bls_server *s, uint64_t ticket) {
  if (!s) return BLS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end() || !it->second->finished)
    return srv_error(s, BLS_ERR_INVALID_ARG, "unknown or unfinished ticket");
  if (it->second->res_off != Arena::kFail) s->res_arena.release(it->second->res_off);
  s->reqs.erase(it);
  return BLS_OK;
}

int bls_server_get_stats(bls_server *s, bls_server_stats *out) {
  if (!s || !out) return BLS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->admitted = s->admitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->queued = (int64_t)s->pending.size();
  int64_t active = 0;
  for (Req *r : s->slots) active += r != nullptr;
  out->active = active;
  out->ticks = s->ticks;
  out->p50_ms = s->lat.percentile(50.0);
  out->p99_ms = s->lat.percentile(99.0);
  out->mean_ms = s->lat.mean();
  out->max_ms = s->lat.max();
  out->trial_points = s->pp_done;
  out->box_evals = s->evals_done;
  out->busy_s = s->busy_s;
  out->wall_s =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - s->t_reset).count();
  out->device_bytes_in_use =
      (int64_t)(s->pts_arena.in_use() * kBytesPerPoint + s->per_arena.in_use() * kBytesPerPeriod);
  out->device_bytes_peak = s->bytes_peak;
  return BLS_OK;
}

int bls_server_reset_stats(bls_server *s) {
  if (!s) return BLS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> g(s->mu);
  s->submitted = s->admitted = s->completed = s->failed = s->ticks = 0;
  s->pp_done = s->evals_done = s->busy_s = 0.0;
  s->lat.clear();
  s->t_reset = std::chrono::steady_clock::now();
  return BLS_OK;
}

int bls_server_drain(bls_server *s, double timeout_s) {
  if (!s) return BLS_ERR_INVALID_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  const auto deadline =
      std::chrono::steady_clock::now() + std::chrono::duration<double>(std::max(0.0, timeout_s));
  auto idle = [&] {
    if (!s->pending.empty()) return false;
    for (Req *r : s->slots)
      if (r) return false;
    return true;
  };
  while (!idle()) {
    if (s->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !idle())
      return BLS_ERR_TIMEOUT;
  }
  return s->device_error ? BLS_ERR_DEVICE : BLS_OK;
}

int bls_server_last_error(const bls_server *s, char *buf, size_t len) {
  if (!buf || len == 0) return BLS_ERR_INVALID_ARG;
  const std::string &m = s ? s->last_error : g_server_create_error;
  const size_t n = std::min(len - 1, m.size());
  memcpy(buf, m.data(), n);
  buf[n] = '\0';
  return BLS_OK;
}

int bls_server_destroy(bls_server *s) {
  if (!s) return BLS_OK;
  if (s->thr.joinable()) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->thr.join();
  }
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
  if (s->up_stream) (void)hipStreamSynchronize(s->up_stream);
  for (void *d : {s->d_txw, (void *)s->d_dt,
                  (void *)s->d_q, (void *)s->d_qw, (void *)s->d_per, s->d_res,
                  (void *)s->d_curves, (void *)s->d_keys})
    if (d) (void)hipFree(d);
  for (const Collect &c : s->collecting)
    if (c.ev) (void)hipEventDestroy(c.ev);
  for (hipEvent_t ev : s->ev_free) (void)hipEventDestroy(ev);
  for (int b = 0; b < kTickBuffers; ++b) {
    for (void *d : {(void *)s->d_seg[b], (void *)s->d_counter[b]})
      if (d) (void)hipFree(d);
    if (s->h_seg[b]) (void)hipHostFree(s->h_seg[b]);
    if (s->ev_s[b]) (void)hipEventDestroy(s->ev_s[b]);
    if (s->ev_e[b]) (void)hipEventDestroy(s->ev_e[b]);
  }
  if (s->h_curves) (void)hipHostFree(s->h_curves);
  if (s->h_pool) (void)hipHostFree(s->h_pool);
  if (s->h_res) (void)hipHostFree(s->h_res);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  if (s->up_stream) (void)hipStreamDestroy(s->up_stream);
  if (s->ev_up) (void)hipEventDestroy(s->ev_up);
  delete s;
  return BLS_OK;
}

}  // extern "C"
