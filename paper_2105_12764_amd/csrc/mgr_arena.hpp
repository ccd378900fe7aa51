// mgr_arena.hpp -- first-fit allocation of byte ranges inside one arena, in
// 256-byte granules, with free ranges coalesced on release.  Host-side
// bookkeeping only (the service hands the ranges out as request workspaces);
// not thread-safe: the caller serialises access.
#pragma once

#include <cstddef>
#include <iterator>
#include <map>

namespace mgr {

class ArenaFit {
 public:
  explicit ArenaFit(size_t bytes = 0) { reset(bytes); }

  void reset(size_t bytes) {
    free_.clear();
    size_ = bytes / kGranule * kGranule;
    if (size_) free_[0] = size_;
  }

  static size_t round_up(size_t bytes) { return (bytes + kGranule - 1) / kGranule * kGranule; }
  size_t size() const { return size_; }

  // Lowest free offset that holds `bytes` (rounded up); false if none does.
  // A zero-byte request succeeds at offset 0 and takes nothing.
  bool alloc(size_t bytes, size_t &off) {
    bytes = round_up(bytes);
    if (bytes == 0) {
      off = 0;
      return true;
    }
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      off = it->first;
      const size_t rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      return true;
    }
    return false;
  }

  // Return a range from alloc(bytes) (same `bytes`), merging it with free
  // neighbours.
  void release(size_t off, size_t bytes) {
    bytes = round_up(bytes);
    if (bytes == 0) return;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }

  // Free ranges, offset -> bytes (for checks).
  const std::map<size_t, size_t> &free_ranges() const { return free_; }

  static constexpr size_t kGranule = 256;

 private:
  size_t size_ = 0;
  std::map<size_t, size_t> free_;
};

}  // namespace mgr
