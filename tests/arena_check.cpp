// Randomised check of mgr::ArenaFit (the service's workspace allocator)
// against a brute-force granule map: every allocation is the lowest free run
// that fits, live ranges never overlap and stay inside the arena, and after
// everything is released the arena is one free range again.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "mgr_arena.hpp"

int main(int argc, char **argv) {
  const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
  std::mt19937_64 rng(seed);
  const size_t G = mgr::ArenaFit::kGranule;
  for (int round = 0; round < 200; ++round) {
    const size_t ngran = 1 + rng() % 400;
    mgr::ArenaFit a(ngran * G + rng() % G);  // a size that is not a whole number of granules
    if (a.size() != ngran * G) return std::printf("size %zu\n", a.size()), 1;
    std::vector<char> used(ngran, 0);
    struct Live { size_t off, bytes; };
    std::vector<Live> live;
    for (int op = 0; op < 500; ++op) {
      if (!live.empty() && rng() % 3 == 0) {
        const size_t i = rng() % live.size();
        a.release(live[i].off, live[i].bytes);
        const size_t g0 = live[i].off / G, ng = mgr::ArenaFit::round_up(live[i].bytes) / G;
        for (size_t g = g0; g < g0 + ng; ++g) used[g] = 0;
        live.erase(live.begin() + (long)i);
        continue;
      }
      const size_t bytes = rng() % 4 == 0 ? 0 : 1 + rng() % (ngran * G / 4 + 1);
      const size_t ng = mgr::ArenaFit::round_up(bytes) / G;
      // brute force: lowest run of ng free granules
      long want = -1;
      for (size_t g = 0; ng > 0 && g + ng <= ngran; ++g) {
        size_t k = 0;
        while (k < ng && !used[g + k]) ++k;
        if (k == ng) { want = (long)g; break; }
      }
      size_t off = 12345;
      const bool ok = a.alloc(bytes, off);
      if (ng == 0) {
        if (!ok || off != 0) return std::printf("zero-byte alloc\n"), 1;
        continue;
      }
      if (ok != (want >= 0)) return std::printf("round %d op %d: alloc %d, brute force %ld\n", round, op, ok, want), 1;
      if (!ok) continue;
      if (off != (size_t)want * G) return std::printf("round %d op %d: off %zu want %zu\n", round, op, off, (size_t)want * G), 1;
      for (size_t g = want; g < (size_t)want + ng; ++g) {
        if (used[g]) return std::printf("overlap\n"), 1;
        used[g] = 1;
      }
      live.push_back({off, bytes});
    }
    // free ranges are exactly the unused granule runs, coalesced
    size_t g = 0;
    auto it = a.free_ranges().begin();
    while (g < ngran) {
      if (used[g]) { ++g; continue; }
      size_t e = g;
      while (e < ngran && !used[e]) ++e;
      if (it == a.free_ranges().end() || it->first != g * G || it->second != (e - g) * G)
        return std::printf("round %d: free map differs at granule %zu\n", round, g), 1;
      ++it;
      g = e;
    }
    if (it != a.free_ranges().end()) return std::printf("extra free range\n"), 1;
    for (auto &l : live) a.release(l.off, l.bytes);
    if (a.free_ranges().size() != 1 || a.free_ranges().begin()->second != a.size())
      return std::printf("round %d: not coalesced after release\n", round), 1;
  }
  std::printf("ok\n");
  return 0;
}
