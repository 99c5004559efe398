// Internal layout shared by the host runtime and the gfx950 kernels.
//
// Data layout in HBM (one call, all curves packed end to end):
//   prep_dt[i]  f64  t_i - t0 of point i (0 for dropped points)
//   prep_q[i]   i32  round(y_i 2^es) (unit weights) or round(w_i y_i 2^es)
//   prep_qw[i]  i32  round(w_i 2^ew), -1 for a dropped (zero-weight) point
//                    (weighted curves only)
//   curves[c]   CurveDesc, host fields first, prep fields written on device
//   seg_*       work segments: items [seg_start[s], seg_start[s+1]) are the
//               period tiles seg_tile0[s] + ... of curve seg_curve[s]
#pragma once
#include <stdint.h>

namespace bls {

constexpr int kBlock = 256;        // threads per workgroup
constexpr int kTileMax = 32;       // largest period tile
constexpr int kGroupMax = 32;      // largest group of periods per work item
constexpr int kPPT = 4;            // points held in registers per thread
constexpr int kQBitsMax = 30;      // fixed-point magnitude bits per point
constexpr int kMaxParts = 8;       // work partitions (one per XCD)

enum CurveStatus : int32_t {
  kCurveOk = 0,
  kCurveBadData = 1,    // non-finite kept time/flux, bad weight
  kCurveTooFew = 2,     // fewer than two kept points or zero total weight
  kCurveBadPeriod = 3,  // a trial period that is not finite and > 0
};

struct CurveDesc {
  // ---- written by the host planner
  int64_t n_off;        // first point in the packed arrays
  int64_t n;            // input points (including zero-weight ones)
  int64_t p_off;        // first trial period
  int64_t r_off;        // first result slot
  int32_t nperiods;
  int32_t nbins;
  int32_t kmin;
  int32_t kmax;
  int32_t tile;         // periods per work item
  int32_t shift;        // count field starts at this bit of a bin word
  int32_t qbits;        // magnitude bits of a point's fixed-point value
  int32_t weighted;     // 1 if a weight array is present
  int32_t check_periods;  // 1: prep checks this curve's trial periods
  int32_t hstride;      // LDS words between periods' histogram planes (>= bins + wrap)
  // ---- written by the prep kernel
  double t0;            // min time over kept points
  double W;             // sum of weights (FP64)
  double xbar;          // weighted mean flux (FP64)
  double out_scale;     // SR and depth of scan units -> flux units
  float Wf;             // total weight in scan units
  int32_t n_eff;        // kept points
  int32_t status;       // CurveStatus
  int32_t es;           // exponent of the S fixed-point scale
  int32_t ew;           // exponent of the weight fixed-point scale
  float cadence;        // median gap between consecutive input times (sampled)
  // ---- unbinned search only (host)
  double qlo;           // duty-cycle limits of a box, in phase
  double qhi;
  // ---- written by the prep kernel: exact totals in scan units (sums of the
  // fixed-point values times 2^-qbits), for boxes evaluated through their
  // complement and for the reported statistic
  double Wtot;          // total weight (the kept count for unit weights)
  double Stot;          // total signal (about 0: the values are centred)
  // ---- written by the host planner: work items are groups of `group`
  // consecutive periods (0: one tile), searched `tile` at a time; the first
  // group of the curve is `galign` periods short, so that later groups start
  // where the result index is a multiple of `group`
  int32_t group;
  int32_t galign;
};

struct PrepArgs {
  CurveDesc *curves;
  const double *periods;
  int32_t ncurves;
  const double *t;
  const double *x;
  const double *w;      // nullptr: unit weights
  double *dt;
  int32_t *q;
  int32_t *qw;
};

struct SearchArgs {
  const CurveDesc *curves;
  const double *periods;
  const double *dt;
  const int32_t *q;
  const int32_t *qw;
  const int64_t *seg_start;   // [nseg + 1]
  const int32_t *seg_curve;   // [nseg]
  const int32_t *seg_tile0;   // [nseg]
  int32_t nseg;
  int32_t min_in_points;
  int64_t nitems;
  unsigned long long *counter;  // kMaxParts work counters, zeroed before the launch
  float *sr;
  float *depth;
  int32_t *jstart;
  int32_t *kwidth;
  unsigned long long *best_key;  // per curve, zeroed before the launch
  int32_t hist_bytes;         // dynamic LDS for histograms
  int32_t ucap;               // unbinned search: largest curve (points)
  // unbinned search of curves above kUnbinnedMaxPoints: a device workspace
  // of uws_stride bytes per workgroup holds the per-point arrays (nullptr:
  // they are in LDS)
  unsigned char *uws;
  int64_t uws_stride;
  // fold of the binned search: 0 merges a thread's same-bin points where the
  // cadence makes that likely, 1 always, 2 never (equal results)
  int32_t fold_policy;
  // unit weights: seed each period's best with a few boxes before the scan
  // (1) or start the scan from zero (0); equal results
  int32_t seed_unit;
  // Work partitions: items [part_begin[x], part_begin[x+1]) belong to
  // partition x, which workgroups with blockIdx.x % nparts == x drain first
  // (workgroups are dispatched to the XCDs round-robin, so a partition's
  // curves stay in one XCD's L2); counter[x] counts its items taken.
  int32_t nparts;
  int32_t pad_parts;
  int64_t part_begin[kMaxParts + 1];
};

// One partition over all items (callers without an XCD split).
inline void single_partition(SearchArgs &a) {
  a.nparts = 1;
  a.pad_parts = 0;
  for (int x = 0; x <= kMaxParts; ++x) a.part_begin[x] = x == 0 ? 0 : a.nitems;
}

// Unbinned search: bytes of per-point arrays for curves of up to n points
// (LDS, or a workspace slice per workgroup above kUnbinnedMaxPoints).
int64_t unbinned_lds_bytes(int n, bool weighted);
int launch_unbinned(const SearchArgs &a, bool weighted, bool dip_only, int grid, void *stream);
int unbinned_blocks_per_cu(bool weighted, bool dip_only, bool glob, int lds_bytes, int *blocks);
constexpr int kUnbinnedMaxPoints = 4096;         // per-point arrays in LDS
constexpr int kUnbinnedMaxPointsGlobal = 1 << 20;  // in a device workspace

struct DetectDesc {
  int64_t p_off;     // first trial period of the curve
  int64_t r_off;     // first result of the curve
  int64_t nperiods;
};

struct DetectArgs {
  const DetectDesc *desc;
  const double *periods;
  const float *sr;
  void *out;          // bls_detection [ncurves]
  int32_t ncurves;
  int32_t max_peaks;
  double window;
  double threshold;
};

// Eclipse detection efficiency of an observing cadence (window function).
struct WindowDesc {
  int64_t n_off;        // first point of the cadence
  int64_t n;            // its points (including zero-weight ones)
  int64_t p_off;        // first trial period
  int64_t r_off;        // first result slot
  int64_t item0;        // first work item (period tile) of this cadence
  int32_t nperiods;
  int32_t check_periods;  // 1: the prep pass checks this cadence's periods
  double t0;            // min kept time (written on the device)
  double dmax;          // max kept time - t0 (written on the device)
  int32_t status;       // CurveStatus (written on the device)
  int32_t pad;
};

struct WindowArgs {
  WindowDesc *desc;
  int32_t ncurves;
  int32_t tile;         // periods per work item
  int64_t nitems;
  const double *t;
  const double *w;      // nullptr: every point is an observation
  const double *periods;
  int32_t *observed;
  int32_t nphase;
  int32_t min_eclipses; // 1 or 2
  double duration;
  unsigned int *overflow;  // set when a cycle number exceeds kMaxCycle
};
constexpr int kMaxCycle = 1 << 29;

// Eclipse-window workspace: per period the nphase bins, (min, max) cycle
// numbers as two int32, then padding: the window pass reads up to s - 2
// entries past a period's wrapped copy without using them, s the entries
// per lane (at most the value below, for windows of nphase bins).
constexpr int window_pad(int nphase) { return ((2 * nphase - 1 + 63) >> 6) | 1; }
constexpr int window_lds_bytes(int tile, int nphase) {
  return (tile * nphase + window_pad(nphase)) * 8;
}
// Static LDS of the window kernel (period frequencies and window lengths).
constexpr int kWindowStaticLds = kTileMax * (8 + 4);

int launch_window(const WindowArgs &a, int grid, void *stream);

// High-variability pre-search.
constexpr int kVarMaxBins = 4096;   // magnitude bins per chip
constexpr int kVarMaxIter = 64;     // clipping rounds

struct VarArgs {
  int32_t ncurves;
  int32_t nchips;
  int32_t nmagbins;
  int32_t max_iter;
  int32_t min_stars;
  int32_t pad;
  const int64_t *n_off;     // device [ncurves + 1]
  const int64_t *chip_off;  // device [nchips + 1]
  const double *x;
  const double *w;          // nullptr: unit weights
  const double *mag;
  double origin;
  double width;
  double clip_sigma;
  double flag_sigma;
  double *rms;              // [ncurves]
  int32_t *bin;             // [ncurves]
  int32_t *flag;            // [ncurves]
  double *bin_mean;         // [nchips * nmagbins]
  double *bin_std;
  int32_t *bin_count;
  uint8_t *alive;           // [ncurves] scratch: in the clipped set
};

int launch_variability(const VarArgs &a, void *stream);
int window_blocks_per_cu(int lds_bytes, int *blocks);

// Launch wrappers (bls_kernels.hip).  All return hipError_t as int.
int launch_detect(const DetectArgs &a, void *stream);
int launch_fill(unsigned long long *counter, unsigned long long *keys,
                int32_t nkeys,
                void *stream);
int launch_prep(const PrepArgs &a, void *stream);
int launch_search(const SearchArgs &a, bool weighted, bool dip_only, int grid,
                  void *stream);
int launch_best_index(unsigned long long *keys, int32_t n, void *stream);
// Phase bin of every prepared point at one period (diagnostic).
int launch_bins(const double *dt, int64_t n, const double *period, int32_t nbins, int32_t *bins,
                void *stream);
// Workgroups of the search kernel one CU holds at this LDS size.
int search_blocks_per_cu(bool weighted, bool dip_only, int hist_bytes,
                         int *blocks);

}  // namespace bls
