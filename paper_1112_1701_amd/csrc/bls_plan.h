// Plan object and host-side planning shared by the C ABI, the autotuner and
// the serving scheduler.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/bls.h"
#include "bls_device.h"

namespace bls {

// Launch shape chosen per batch (by the tuner or the built-in table).
struct TileChoice {
  int lds_budget = 32768;   // dynamic LDS bytes per workgroup to aim for
  int tile_cap = kTileMax;  // upper bound on periods per work item
  int occupancy = 0;        // workgroups per CU to launch (0 = max resident)
};

// A fully planned call: descriptors in pinned host memory, ready to upload.
struct PlannedBatch {
  int32_t ncurves = 0;
  bool weighted = false;
  int64_t total_points = 0;
  int64_t total_results = 0;
  int64_t nitems = 0;
  int32_t nseg = 0;
  int32_t hist_bytes = 0;
  int32_t grid = 0;
  double trial_points = 0.0;
  double box_evals = 0.0;
  int32_t ucap = 0;         // unbinned search: largest curve (points)
  unsigned char *uws = nullptr;  // unbinned search: workspace of long curves
  int64_t uws_stride = 0;        // its bytes per workgroup
  int32_t nparts = 1;       // work partitions (XCDs)
  int64_t part_begin[bls::kMaxParts + 1] = {};
};

// Per-curve shape after validation (host only).
struct CurveShape {
  int64_t n_off, n, p_off, r_off;
  int32_t nperiods, nbins, kmin, kmax;
};

}  // namespace bls

struct bls_plan {
  bls_plan_config cfg{};
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int num_cus = 0;
  int max_lds = 0;

  // device working set
  bls::CurveDesc *d_curves = nullptr;
  int64_t *d_seg_start = nullptr;
  int32_t *d_seg_curve = nullptr;
  int32_t *d_seg_tile0 = nullptr;
  double *d_dt = nullptr;
  int32_t *d_q = nullptr;
  int32_t *d_qw = nullptr;
  unsigned long long *d_counter = nullptr;

  // host-API staging (allocated on first use)
  bool staging = false;
  double *d_t = nullptr, *d_x = nullptr, *d_w = nullptr, *d_periods = nullptr;
  float *d_sr = nullptr, *d_depth = nullptr;
  int32_t *d_j = nullptr, *d_k = nullptr;
  int64_t *d_best = nullptr;
  // pinned host staging of the host API (allocated on first use): a call's
  // inputs on the way in, its results on the way out
  char *h_stage = nullptr;
  size_t h_stage_bytes = 0;

  // detection buffers (allocated on first use)
  bls::DetectDesc *d_detect_desc = nullptr;
  void *d_detect_out = nullptr;

  // injection-recovery buffers (allocated on first use): per-injection
  // parameters [max_curves] and the cadence's t0
  void *d_inj = nullptr;
  double *d_inj_t0 = nullptr;

  // unbinned search of long curves: per-workgroup workspace (grown as needed)
  unsigned char *d_uws = nullptr;
  int64_t uws_bytes = 0;

  // eclipse-window buffers (allocated on first use)
  bls::WindowDesc *d_window_desc = nullptr;
  unsigned int *d_window_flag = nullptr;

  // variability pre-search scratch (allocated on first use, grown as needed)
  int64_t *d_var_noff = nullptr;      // [max_curves + 1]
  uint8_t *d_var_alive = nullptr;     // [max_curves]
  int64_t *d_var_chip = nullptr;      // [var_chip_cap + 1]
  int64_t var_chip_cap = 0;

  // pinned host descriptors
  bls::CurveDesc *h_curves = nullptr;
  int64_t *h_seg_start = nullptr;
  int32_t *h_seg_curve = nullptr;
  int32_t *h_seg_tile0 = nullptr;

  // graph cache for bls_search_device: the launch sequence is captured as
  // three graphs (uploads, fill and prep; the search kernel; the best-index
  // read-out) so that the search kernel's own duration can be bracketed by
  // events on every replay
  hipGraph_t graph[3] = {nullptr, nullptr, nullptr};
  hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
  uint64_t graph_sig = 0;
  bool graph_valid = false;

  hipEvent_t ev_begin = nullptr, ev_search0 = nullptr, ev_search1 = nullptr,
             ev_end = nullptr;

  // The pinned descriptors above are read by queued copies (or graph
  // replays) until ev_desc, recorded after them, completes; a call that
  // rewrites them first waits for it.
  hipEvent_t ev_desc = nullptr;
  bool desc_pending = false;

  // Search-kernel durations of the last kTimeRing calls: events recorded
  // just before and after each search (or unbinned) kernel launch.
  static constexpr int kTimeRing = 64;
  hipEvent_t ev_k0[kTimeRing] = {};
  hipEvent_t ev_k1[kTimeRing] = {};
  int64_t k_recorded = 0;   // kernel launches bracketed so far
  int64_t k_base = 0;       // value of k_recorded at the last reset

  bls::PlannedBatch last;
  bls_call_stats stats{};
  std::string last_error;
  std::vector<bls::CurveShape> shapes;   // scratch for planning
  std::vector<int> order;                // scratch for planning
  bool tuned_valid = false;
  uint64_t tuned_key = 0;
  bls::TileChoice tuned;
};

namespace bls {

// Validation of a batch description and its parameters (host only; no
// device access).  With check_data, also the host data arrays.  Without
// binned, nbins is ignored and each curve's duty-cycle range is checked as
// phase limits (0 < qmin <= qmax < 1) with at most kUnbinnedMaxPoints points.
int validate_batch(const bls_plan_config &cfg, const bls_batch &b, bool check_data,
                   std::vector<CurveShape> &shapes, std::string &err, bool binned = true);
// The same into caller-owned storage (no heap use): shapes has room for
// shapes_cap curves; a failure's message goes to err (NUL-terminated).
int validate_batch_into(const bls_plan_config &cfg, const bls_batch &b, bool check_data,
                        CurveShape *shapes, int shapes_cap, char *err, size_t err_len,
                        bool binned = true);
// Host fields of one curve's descriptor (prep fields zero): fixed-point
// layout, and the period tile and plane stride that fit tc's LDS budget.
// memo: keep the bank-conflict costs of plane strides in the process-wide
// cache (false: compute them afresh, with no heap use).
void fill_curve_desc(const CurveShape &s, bool weighted, const TileChoice &tc,
                     bool check_periods, bool memo, CurveDesc &d);

// Segments grouped into work partitions (one per XCD), curves assigned
// round-robin in descending cost; items_of[c] = work items of curve c.
void layout_partitions(bls_plan *p, const std::vector<double> &cost,
                       const std::vector<int64_t> &items_of, PlannedBatch &out);

// Periods per work item of a batch: kGroupMax when the batch has at least
// four such groups per workgroup of a full grid (the kernel then writes each
// item's results as whole lines), else 0 (one period tile per item).  The
// environment variable BLS_ITEM_GROUP (0 or kGroupMax) overrides the choice.
int item_group(const bls_plan *p, const std::vector<CurveShape> &shapes);

// Fill the pinned descriptors for a validated batch and size the launch.
int plan_batch(bls_plan *p, const std::vector<CurveShape> &shapes, bool weighted,
               const TileChoice &tc, PlannedBatch &out);

// The launch sequence of a search, in three parts: (1) upload descriptors,
// clear counters and keys, prep; (2) the search kernel (with unbinned, the
// unbinned kernel: js and ks then receive the first and last point of each
// best box); (3) per-curve best index.  Nothing here records events, so each
// part can be captured into a graph.
int enqueue_pre(bls_plan *p, const PlannedBatch &pb, const double *t, const double *x,
                const double *w, const double *periods, int64_t *best);
int enqueue_kernel(bls_plan *p, const PlannedBatch &pb, const double *periods, float *sr,
                   float *depth, int32_t *js, int32_t *ks, int64_t *best, bool unbinned);
int enqueue_post(bls_plan *p, const PlannedBatch &pb, int64_t *best);
// All three, with ev_desc after the uploads and the kernel bracketed by the
// timing ring's events (streams that are not capturing).
int enqueue_search(bls_plan *p, const PlannedBatch &pb, const double *t, const double *x,
                   const double *w, const double *periods, float *sr, float *depth,
                   int32_t *js, int32_t *ks, int64_t *best, bool unbinned = false);
// Wait until no queued copy or graph still reads the pinned descriptors.
int desc_wait(bls_plan *p);
// Mark the pinned descriptors as read by work queued so far on the stream.
int desc_mark(bls_plan *p);
// Events of the timing ring around the next kernel launch.
int ring_begin(bls_plan *p);
int ring_end(bls_plan *p);

int set_error(bls_plan *p, int status, const std::string &msg);
// The calling thread's error without a plan (what bls_last_error(NULL)
// returns), recorded without heap use.
int set_error_noplan(int status, const char *msg);
int hip_error(bls_plan *p, hipError_t e, const char *what);
int width_range(int32_t nbins, double qmin, double qmax, int32_t *kmin, int32_t *kmax);

// Search-kernel duration of the last bracketed launch (ms; 0 if none).
double last_kernel_ms(bls_plan *p);
// Call statistics of a planned batch.
void fill_stats(bls_plan *p, const PlannedBatch &pb, bool replayed);
// Device buffers of the host-array calls (max_points, max_periods,
// max_curves sized), allocated on first use.
int ensure_staging(bls_plan *p);
// INVALID_ARG naming the first curve whose prep found invalid data.
int check_device_status(bls_plan *p, int ncurves);
// Per-curve flags (1: invalid data or trial periods) of the last prep.
int device_status_flags(bls_plan *p, int ncurves, int32_t *bad);
// Detection buffers (max_curves descriptors and results), on first use.
int ensure_detect_buffers(bls_plan *p);
// Queue the detection kernel over ncurves periodograms of one shared grid,
// curve c's SR at sr[c * nperiods]; results in p->d_detect_out.
int enqueue_detect_shared(bls_plan *p, int ncurves, const double *periods, int64_t nperiods,
                          const float *sr, int max_peaks, double window, double threshold);
// Injection-recovery buffers, on first use.
int ensure_recovery_buffers(bls_plan *p);

// Device allocation with the optional failure-injection hook.
hipError_t device_alloc(void **ptr, size_t bytes);

// LDS words (64-bit) one period's histogram plane needs: the bins, then the
// clamp word / wrap-around copy of the first min(kmax, nbins / 2) - 1 bins.
int hist_words(int nbins, int kmax);
// Words between consecutive periods' planes for a tile of `tile` periods:
// at least hist_words, padded so that the scan's 64-bit reads, served 16
// lanes at a time across 32 four-byte banks, meet as few bank conflicts as
// the layout allows (lane task (start bin, period) = divmod(lane, tile)).
int hist_stride(int nbins, int kmax, int tile, bool weighted, bool memo = true);
// Periods per work item that fit an LDS budget (at least one, at most
// tile_cap and nperiods) and the padded stride that goes with it.
void fit_tile(int nbins, int kmax, int64_t nperiods, int lds_budget, int tile_cap,
              bool weighted, int *tile, int *stride, bool memo = true);

// Tile choice for a batch: autotuned (cached) unless disabled.
TileChoice choose_tiles(bls_plan *p, const std::vector<CurveShape> &shapes, bool weighted);
// The built-in table the tuner starts from.
TileChoice default_tiles(bool weighted);

}  // namespace bls
