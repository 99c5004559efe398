"""Host-side scheduling pieces of the serving loop (no GPU): the arena
allocator, the continuous-batching tick builder and latency percentiles,
compiled with g++ from the library's own header and checked against simple
models."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1112_1701_amd", "csrc")

DRIVER = r'''
#include "bls_sched.h"
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>
using namespace bls;
#define CHECK(c) do { if (!(c)) { printf("FAIL line %d: %s\n", __LINE__, #c); return 1; } } while (0)
int main() {
  // Arena: random alloc/free against an interval model.
  {
    Arena a(1 << 20, 256);
    std::mt19937 rng(7);
    std::map<size_t, size_t> live;  // off -> rounded len
    for (int it = 0; it < 20000; ++it) {
      if (live.empty() || rng() % 3) {
        size_t b = 1 + rng() % 20000;
        size_t off = a.alloc(b);
        if (off == Arena::kFail) { CHECK(a.largest_free() < a.round_up(b)); continue; }
        CHECK(off % 256 == 0);
        CHECK(off + a.round_up(b) <= a.capacity());
        for (auto &kv : live) CHECK(off + a.round_up(b) <= kv.first || kv.first + kv.second <= off);
        live[off] = a.round_up(b);
      } else {
        auto it2 = live.begin();
        std::advance(it2, rng() % live.size());
        CHECK(a.release(it2->first));
        live.erase(it2);
      }
      size_t used = 0; for (auto &kv : live) used += kv.second;
      CHECK(used == a.in_use());
    }
    for (auto &kv : live) CHECK(a.release(kv.first));
    CHECK(a.in_use() == 0 && a.free_blocks() == 1 && a.largest_free() == a.capacity());
    CHECK(!a.release(12345));
    CHECK(!a.fits_ever((1 << 20) + 1));
  }
  // Tick builder: budget, order, minimum share, no tile issued twice.
  {
    std::vector<SlotWork> w = {{0, 5, 10, 0, 1.0}, {1, 2, 4, 0, 2.0}, {2, 9, 3, 0, 1.0}};
    auto t1 = build_tick(w, 6.0, 1);
    // every active request gets a tile; oldest (order 2 = slot 1) first
    CHECK(t1.size() >= 3);
    CHECK(t1[0].slot == 1);
    double cost = 0; std::map<int,int> got;
    for (auto &s : t1) { cost += s.ntiles * (s.slot == 1 ? 2.0 : 1.0); got[s.slot] += s.ntiles; }
    CHECK(got[0] >= 1 && got[1] >= 1 && got[2] >= 1);
    CHECK(cost <= 6.0 + 2.0);
    // drain: repeated ticks issue each tile exactly once and in order
    std::vector<std::vector<int>> seen(3);
    for (auto &s : t1) for (int k = 0; k < s.ntiles; ++k) seen[s.slot].push_back(s.tile0 + k);
    for (int rep = 0; rep < 100; ++rep) {
      auto t = build_tick(w, 3.0, 1);
      if (t.empty()) break;
      for (auto &s : t) for (int k = 0; k < s.ntiles; ++k) seen[s.slot].push_back(s.tile0 + k);
    }
    int nt[3] = {10, 4, 3};
    for (int i = 0; i < 3; ++i) {
      CHECK((int)seen[i].size() == nt[i]);
      for (int k = 0; k < nt[i]; ++k) CHECK(seen[i][k] == k);
    }
    CHECK(build_tick(w, 10.0, 1).empty());
  }
  // Latency percentiles (nearest rank).
  {
    LatencyLog l;
    CHECK(l.percentile(50) == 0.0);
    for (int i = 1; i <= 100; ++i) l.add(i);
    CHECK(l.percentile(50) == 50.0 && l.percentile(99) == 99.0 && l.percentile(100) == 100.0);
    CHECK(l.max() == 100.0 && l.mean() == 50.5);
  }
  printf("OK\n");
  return 0;
}
'''


def test_sched_pieces_compile_and_pass():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        exe = os.path.join(d, "t")
        open(src, "w").write(DRIVER)
        subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall",
                               "-fsanitize=address,undefined", "-I" + CSRC,
                               src, "-o", exe])
        out = subprocess.run([exe], capture_output=True, text=True)
        assert out.returncode == 0 and out.stdout.strip() == "OK", out.stdout
