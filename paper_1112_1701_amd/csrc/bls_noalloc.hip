// Plan-free search (bls_search_device_noalloc): the launch sequence of
// bls_search_device -- descriptors, fill, prep, search, best index -- with
// its working set in a fixed device array instead of plan allocations, for
// callers that cannot allocate (code under HIP graph capture, serving
// loops, harnesses that forbid hipMalloc).
//
// The array, `scratch`, lives in every GPU's memory from the library's load
// until the process ends.  Host code never passes its name to a kernel or a
// copy (on the host that name is only a stand-in, not a device address): on
// a call's first use of a device, with that device current,
// hipGetSymbolAddress gives the device's own address of the array, which is
// kept per device and used from then on.  The curve descriptors, which
// bls_search_device uploads from pinned host memory, are written here by a
// small kernel from its by-value arguments, so the call needs no host
// staging either and every step is a kernel launch.
#include <hip/hip_runtime.h>

#include <stdio.h>
#include <string.h>

#include <mutex>

#include "bls_plan.h"

namespace bls {
namespace {

constexpr int kNaCurves = BLS_NOALLOC_MAX_CURVES;
constexpr int64_t kNaPoints = BLS_NOALLOC_MAX_POINTS;

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Layout of the scratch array: prepared points (t - t0 as f64, fixed-point
// signal and weight as i32), then curve descriptors, work segments and the
// partition counters.
constexpr size_t kOffDt = 0;
constexpr size_t kOffQ = align256(kOffDt + sizeof(double) * kNaPoints);
constexpr size_t kOffQw = align256(kOffQ + sizeof(int32_t) * kNaPoints);
constexpr size_t kOffCurves = align256(kOffQw + sizeof(int32_t) * kNaPoints);
constexpr size_t kOffSegStart = align256(kOffCurves + sizeof(CurveDesc) * kNaCurves);
constexpr size_t kOffSegCurve = align256(kOffSegStart + sizeof(int64_t) * (kNaCurves + 1));
constexpr size_t kOffSegTile0 = align256(kOffSegCurve + sizeof(int32_t) * kNaCurves);
constexpr size_t kOffCounter = align256(kOffSegTile0 + sizeof(int32_t) * kNaCurves);
constexpr size_t kScratchBytes = align256(kOffCounter + sizeof(unsigned long long) * kMaxParts);
static_assert(kScratchBytes <= BLS_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds its stated size");

static __device__ __align__(256) unsigned char scratch[BLS_NOALLOC_SCRATCH_BYTES];

// Per device: the address of its copy of the array and what the launch
// sizing needs, taken once with the device current.
constexpr int kMaxDevices = 64;
struct DeviceState {
  bool ready = false;
  unsigned char *ptr = nullptr;
  int num_cus = 0;
  int max_lds = 0;
};
DeviceState g_dev[kMaxDevices];
std::mutex g_dev_mu;

int device_state(int dev, DeviceState &out) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_error_noplan(BLS_ERR_DEVICE, "device ordinal beyond the supported range");
  std::lock_guard<std::mutex> g(g_dev_mu);
  DeviceState &s = g_dev[dev];
  if (!s.ready) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return set_error_noplan(BLS_ERR_DEVICE, "hipGetSymbolAddress of the scratch array failed");
    int cus = 0, lds = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess)
      return set_error_noplan(BLS_ERR_DEVICE, "device attribute query failed");
    s.ptr = static_cast<unsigned char *>(p);
    s.num_cus = cus;
    s.max_lds = lds;
    s.ready = true;
  }
  out = s;
  return BLS_OK;
}

// Curve descriptors and segments of up to kDescPerLaunch curves, passed by
// value; one thread per curve writes them into the scratch array.
constexpr int kDescPerLaunch = 16;
struct DescArgs {
  CurveDesc desc[kDescPerLaunch];
  int64_t seg_start[kDescPerLaunch];
  int32_t seg_curve[kDescPerLaunch];
  int32_t first;        // segment (and descriptor slot) of entry 0
  int32_t count;
  int32_t last;         // 1: also write seg_start[nseg] = nitems
  int32_t nseg;
  int64_t nitems;
  CurveDesc *curves;
  int64_t *seg_start_out;
  int32_t *seg_curve_out;
  int32_t *seg_tile0_out;
};
static_assert(sizeof(DescArgs) <= 4000, "descriptor arguments exceed the kernel argument space");

__global__ void desc_kernel(DescArgs a) {
  const int i = threadIdx.x;
  if (i < a.count) {
    const int s = a.first + i;
    const int c = a.seg_curve[i];
    a.curves[c] = a.desc[i];
    a.seg_start_out[s] = a.seg_start[i];
    a.seg_curve_out[s] = c;
    a.seg_tile0_out[s] = 0;
  }
  if (i == 0 && a.last) a.seg_start_out[a.nseg] = a.nitems;
}

}  // namespace
}  // namespace bls

using namespace bls;

extern "C" int bls_search_device_noalloc(const bls_batch *b, const bls_device_results *o,
                                         uint32_t flags, int32_t min_in_points,
                                         void *hip_stream) {
  if (!b || !o || !o->sr || !o->depth || !o->jstart || !o->kwidth || !o->best_index)
    return set_error_noplan(BLS_ERR_INVALID_ARG,
                            "batch and every device result array are required");
  if ((flags & ~(uint32_t)BLS_DIP_ONLY) != 0)
    return set_error_noplan(BLS_ERR_INVALID_ARG, "flags other than BLS_DIP_ONLY");
  if (min_in_points < 1) return set_error_noplan(BLS_ERR_INVALID_ARG, "min_in_points < 1");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess)
    return set_error_noplan(BLS_ERR_DEVICE, "no current HIP device");
  DeviceState ds;
  int st = device_state(dev, ds);
  if (st != BLS_OK) return st;

  // Shapes and parameters, against the scratch array's limits.
  bls_plan_config cfg;
  bls_plan_config_init(&cfg);
  cfg.device = dev;
  cfg.max_curves = kNaCurves;
  cfg.max_points = kNaPoints;
  cfg.max_periods = INT64_MAX;
  cfg.max_nbins = BLS_MAX_NBINS;
  cfg.min_in_points = min_in_points;
  cfg.flags = flags;
  CurveShape shapes[kNaCurves];
  char err[256] = "";
  st = validate_batch_into(cfg, *b, false, shapes, kNaCurves, err, sizeof err);
  if (st != BLS_OK) return set_error_noplan(st, err);
  const int nc = b->ncurves;
  const bool weighted = b->weights != nullptr;
  const int wpb = weighted ? 2 : 1;

  // Built-in tile table; tiles cut so that the call has work items for two
  // workgroups per CU (as for untuned small plan calls).
  TileChoice tc = default_tiles(weighted);
  int64_t periods = 0;
  for (int c = 0; c < nc; ++c) periods += shapes[c].nperiods;
  const int64_t cap = periods / (2 * (int64_t)(ds.num_cus > 0 ? ds.num_cus : 1));
  tc.tile_cap = (int)(cap < 1 ? 1 : cap < tc.tile_cap ? cap : tc.tile_cap);

  CurveDesc desc[kNaCurves];
  double cost[kNaCurves];
  int64_t items_of[kNaCurves];
  int hist_bytes = 0;
  for (int c = 0; c < nc; ++c) {
    const CurveShape &s = shapes[c];
    fill_curve_desc(s, weighted, tc, c == 0 || s.p_off != shapes[0].p_off, false, desc[c]);
    const int T = desc[c].tile;
    const int hb = T * desc[c].hstride * 8 * wpb;
    if (hb > hist_bytes) hist_bytes = hb;
    const double nw = (double)(s.kmax - s.kmin + 1);
    cost[c] = (double)T * ((double)s.n + 1.6 * (double)s.nbins * nw);
    items_of[c] = (s.nperiods + T - 1) / T;
  }
  if (hist_bytes > ds.max_lds - 1024)
    return set_error_noplan(BLS_ERR_CAPACITY,
                            "one period's histogram needs more LDS than a workgroup has");

  // One partition; segments in descending item cost (insertion sort).
  int order[kNaCurves];
  for (int c = 0; c < nc; ++c) {
    int k = c;
    while (k > 0 && cost[order[k - 1]] < cost[c]) {
      order[k] = order[k - 1];
      --k;
    }
    order[k] = c;
  }
  int64_t seg_start[kNaCurves];
  int64_t nitems = 0;
  for (int s = 0; s < nc; ++s) {
    seg_start[s] = nitems;
    nitems += items_of[order[s]];
  }

  int per_cu = 0;
  hipError_t e = (hipError_t)search_blocks_per_cu(weighted, (flags & BLS_DIP_ONLY) != 0,
                                                  hist_bytes, &per_cu);
  if (e != hipSuccess) return set_error_noplan(BLS_ERR_DEVICE, "occupancy query failed");
  if (per_cu < 1) return set_error_noplan(BLS_ERR_CAPACITY, "search kernel does not fit a CU");
  int64_t grid = (int64_t)ds.num_cus * per_cu;
  if (nitems < grid) grid = nitems;
  if (grid < 1) grid = 1;

  // Addresses inside this device's copy of the array.
  unsigned char *base = ds.ptr;
  double *d_dt = reinterpret_cast<double *>(base + kOffDt);
  int32_t *d_q = reinterpret_cast<int32_t *>(base + kOffQ);
  int32_t *d_qw = reinterpret_cast<int32_t *>(base + kOffQw);
  CurveDesc *d_curves = reinterpret_cast<CurveDesc *>(base + kOffCurves);
  int64_t *d_seg_start = reinterpret_cast<int64_t *>(base + kOffSegStart);
  int32_t *d_seg_curve = reinterpret_cast<int32_t *>(base + kOffSegCurve);
  int32_t *d_seg_tile0 = reinterpret_cast<int32_t *>(base + kOffSegTile0);
  unsigned long long *d_counter = reinterpret_cast<unsigned long long *>(base + kOffCounter);
  hipStream_t stream = (hipStream_t)hip_stream;

  // Descriptors and segments, kDescPerLaunch curves per launch.
  for (int s0 = 0; s0 < nc; s0 += kDescPerLaunch) {
    DescArgs da;
    memset(&da, 0, sizeof da);
    da.first = s0;
    da.count = nc - s0 < kDescPerLaunch ? nc - s0 : kDescPerLaunch;
    da.last = s0 + da.count == nc ? 1 : 0;
    da.nseg = nc;
    da.nitems = nitems;
    da.curves = d_curves;
    da.seg_start_out = d_seg_start;
    da.seg_curve_out = d_seg_curve;
    da.seg_tile0_out = d_seg_tile0;
    for (int i = 0; i < da.count; ++i) {
      const int c = order[s0 + i];
      da.desc[i] = desc[c];
      da.seg_start[i] = seg_start[s0 + i];
      da.seg_curve[i] = c;
    }
    hipLaunchKernelGGL(desc_kernel, dim3(1), dim3(64), 0, stream, da);
    if ((e = hipGetLastError()) != hipSuccess)
      return set_error_noplan(BLS_ERR_DEVICE, "launch of the descriptor kernel failed");
  }
  unsigned long long *keys = reinterpret_cast<unsigned long long *>(o->best_index);
  if ((e = (hipError_t)launch_fill(d_counter, keys, nc, stream)) != hipSuccess)
    return set_error_noplan(BLS_ERR_DEVICE, "launch of the fill kernel failed");

  PrepArgs pa;
  pa.curves = d_curves;
  pa.periods = b->periods;
  pa.ncurves = nc;
  pa.t = b->times;
  pa.x = b->flux;
  pa.w = b->weights;
  pa.dt = d_dt;
  pa.q = d_q;
  pa.qw = d_qw;
  if ((e = (hipError_t)launch_prep(pa, stream)) != hipSuccess)
    return set_error_noplan(BLS_ERR_DEVICE, "launch of the prep kernel failed");

  SearchArgs sa;
  memset(&sa, 0, sizeof sa);
  sa.curves = d_curves;
  sa.periods = b->periods;
  sa.dt = d_dt;
  sa.q = d_q;
  sa.qw = weighted ? d_qw : nullptr;
  sa.seg_start = d_seg_start;
  sa.seg_curve = d_seg_curve;
  sa.seg_tile0 = d_seg_tile0;
  sa.nseg = nc;
  sa.min_in_points = min_in_points;
  sa.nitems = nitems;
  sa.counter = d_counter;
  sa.sr = o->sr;
  sa.depth = o->depth;
  sa.jstart = o->jstart;
  sa.kwidth = o->kwidth;
  sa.best_key = keys;
  sa.hist_bytes = hist_bytes;
  sa.ucap = 0;
  single_partition(sa);
  if ((e = (hipError_t)launch_search(sa, weighted, (flags & BLS_DIP_ONLY) != 0, (int)grid,
                                     stream)) != hipSuccess)
    return set_error_noplan(BLS_ERR_DEVICE, "launch of the search kernel failed");
  if ((e = (hipError_t)launch_best_index(keys, nc, stream)) != hipSuccess)
    return set_error_noplan(BLS_ERR_DEVICE, "launch of the best-index kernel failed");
  return BLS_OK;
}
