// Host-side scheduling pieces of the serving loop, free of any HIP call so
// that they can be compiled and tested on a machine without a GPU:
//   Arena        first-fit allocator over one device allocation (offsets)
//   TickBuilder  continuous batching: which (request, period tiles) go into
//                the next persistent launch
//   LatencyLog   latency percentiles
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <algorithm>
#include <map>
#include <vector>

namespace bls {

// First-fit allocator over [0, capacity) with coalescing of free neighbours.
// Offsets are aligned to `align` bytes (a power of two).
class Arena {
 public:
  explicit Arena(size_t capacity = 0, size_t align = 256) { reset(capacity, align); }

  void reset(size_t capacity, size_t align) {
    align_ = align;
    capacity_ = capacity & ~(align - 1);
    free_.clear();
    used_.clear();
    in_use_ = 0;
    if (capacity_ > 0) free_[0] = capacity_;
  }

  static constexpr size_t kFail = ~size_t(0);

  // Offset of a block of at least `bytes`, or kFail.
  size_t alloc(size_t bytes) {
    const size_t need = round_up(bytes == 0 ? 1 : bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= need) {
        const size_t off = it->first;
        const size_t rest = it->second - need;
        free_.erase(it);
        if (rest > 0) free_[off + need] = rest;
        used_[off] = need;
        in_use_ += need;
        peak_ = std::max(peak_, in_use_);
        return off;
      }
    }
    return kFail;
  }

  // Return a block; false if `off` is not an allocated block.
  bool release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return false;
    size_t start = off, len = u->second;
    used_.erase(u);
    in_use_ -= len;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    return true;
  }

  bool fits_ever(size_t bytes) const { return round_up(bytes == 0 ? 1 : bytes) <= capacity_; }
  size_t capacity() const { return capacity_; }
  size_t in_use() const { return in_use_; }
  size_t peak() const { return peak_; }
  size_t largest_free() const {
    size_t m = 0;
    for (auto &f : free_) m = std::max(m, f.second);
    return m;
  }
  size_t free_blocks() const { return free_.size(); }
  size_t round_up(size_t b) const { return (b + align_ - 1) & ~(align_ - 1); }

 private:
  size_t align_ = 256, capacity_ = 0, in_use_ = 0, peak_ = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  std::map<size_t, size_t> used_;  // offset -> length
};

// Work remaining on one admitted request.
struct SlotWork {
  int slot;            // index of the request's slot
  uint64_t order;      // admission order (smaller = older)
  int32_t ntiles;      // period tiles of the request
  int32_t next_tile;   // first tile not yet issued
  double item_cost;    // relative cost of one tile
};

struct TickSegment {
  int slot;
  int32_t tile0;
  int32_t ntiles;
};

// Continuous batching: fill one launch with up to `budget` cost units of
// tiles, oldest requests first, but give every active request at least
// `min_tiles` tiles so that newly admitted requests start at once and
// overlap on the device with the ones already running.
inline std::vector<TickSegment> build_tick(std::vector<SlotWork> &work, double budget,
                                           int32_t min_tiles) {
  std::vector<TickSegment> out;
  std::vector<SlotWork *> act;
  for (auto &w : work)
    if (w.next_tile < w.ntiles) act.push_back(&w);
  std::sort(act.begin(), act.end(),
            [](const SlotWork *a, const SlotWork *b) { return a->order < b->order; });
  // first pass: a minimum share for every active request
  double spent = 0.0;
  for (SlotWork *w : act) {
    const int32_t take = std::min(min_tiles, w->ntiles - w->next_tile);
    if (take <= 0) continue;
    out.push_back({w->slot, w->next_tile, take});
    w->next_tile += take;
    spent += take * w->item_cost;
  }
  // second pass: the rest of the budget, oldest first
  for (SlotWork *w : act) {
    if (spent >= budget) break;
    const int32_t left = w->ntiles - w->next_tile;
    if (left <= 0) continue;
    int32_t take = left;
    if (w->item_cost > 0.0) {
      const double can = (budget - spent) / w->item_cost;
      if (can < (double)take) take = std::max<int32_t>(1, (int32_t)can);
    }
    // merge with this slot's first-pass segment when contiguous
    bool merged = false;
    for (auto &s : out)
      if (s.slot == w->slot && s.tile0 + s.ntiles == w->next_tile) {
        s.ntiles += take;
        merged = true;
        break;
      }
    if (!merged) out.push_back({w->slot, w->next_tile, take});
    w->next_tile += take;
    spent += take * w->item_cost;
  }
  return out;
}

// Latency samples (milliseconds) and their percentiles.
class LatencyLog {
 public:
  void add(double ms) { v_.push_back(ms); }
  void clear() { v_.clear(); }
  size_t size() const { return v_.size(); }
  // Nearest-rank percentile (q in [0, 100]); 0 if empty.
  double percentile(double q) const {
    if (v_.empty()) return 0.0;
    std::vector<double> s(v_);
    std::sort(s.begin(), s.end());
    size_t rank = (size_t)((q / 100.0) * (double)s.size() + 0.999999999);
    if (rank < 1) rank = 1;
    if (rank > s.size()) rank = s.size();
    return s[rank - 1];
  }
  double mean() const {
    if (v_.empty()) return 0.0;
    double t = 0;
    for (double x : v_) t += x;
    return t / (double)v_.size();
  }
  double max() const {
    double m = 0;
    for (double x : v_) m = std::max(m, x);
    return m;
  }

 private:
  std::vector<double> v_;
};

}  // namespace bls
