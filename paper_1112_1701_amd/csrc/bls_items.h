// Work items of the persistent kernels: claiming the next item from the
// XCD-partitioned counters and placing it in its segment (curve, tile).
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "bls_device.h"

namespace bls {
namespace {

// Next work item of a persistent workgroup (thread 0 only): items of its
// own partition first, then of the others in turn; -1 once all are taken.
// done_mask remembers the partitions found empty.
__device__ inline long long next_item(const SearchArgs &a, unsigned &done_mask) {
  const int np = a.nparts;
  const int home = (int)(blockIdx.x % (unsigned)np);
  for (int k = 0; k < np; ++k) {
    const int x = home + k < np ? home + k : home + k - np;
    if (done_mask & (1u << x)) continue;
    const unsigned long long it =
        __hip_atomic_fetch_add(a.counter + x, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const long long item = a.part_begin[x] + (long long)it;
    if (item < a.part_begin[x + 1]) return item;
    done_mask |= 1u << x;
  }
  return -1;
}

// A claimed work item and its place: curve and tile (period, for the
// unbinned search) within the curve.
struct ItemRef {
  long long item;
  int curve;
  int tile;
};

// The segment of the last claimed item, kept in thread 0's registers:
// items of a partition are claimed in increasing order, so the next one
// usually falls in the same segment and needs no memory access to place.
struct SegCache {
  long long lo, hi;  // items [lo, hi) of the segment
  int curve, tile0;
};

// Claim the next item and place it (thread 0 only).
__device__ inline ItemRef claim_item(const SearchArgs &a, unsigned &done_mask, SegCache &sc) {
  ItemRef r;
  r.item = next_item(a, done_mask);
  r.curve = 0;
  r.tile = 0;
  if (r.item < 0) return r;
  if (!(r.item >= sc.lo && r.item < sc.hi)) {
    int lo = 0, hi = a.nseg - 1;  // last s with seg_start[s] <= item
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.seg_start[mid] <= r.item)
        lo = mid;
      else
        hi = mid - 1;
    }
    sc.lo = a.seg_start[lo];
    sc.hi = a.seg_start[lo + 1];
    sc.curve = a.seg_curve[lo];
    sc.tile0 = a.seg_tile0[lo];
  }
  r.curve = sc.curve;
  r.tile = sc.tile0 + (int)(r.item - sc.lo);
  return r;
}

}  // namespace
}  // namespace bls
