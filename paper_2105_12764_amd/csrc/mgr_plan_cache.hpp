// mgr_plan_cache.hpp -- the plan cache's bookkeeping, free of any GPU call so
// that it can be checked on the host (tests/plan_cache_check.cpp).
//
// Lifetime rule.  A plan owns device tables whose addresses are baked into
// the kernel arguments of every launch that uses it.  Three kinds of owner
// hold a plan through a shared_ptr:
//   * the cache (least recently used entries are dropped beyond a bound);
//   * a call in progress (a batch holds the plans of all its fields until it
//     has enqueued them);
//   * a captured HIP graph: the call that records launches into a graph
//     hands one reference to a graph user object, whose release callback
//     runs when the graph and every executable made from it are destroyed.
// The tables are freed when the last owner lets go.  A user-object callback
// may not call the GPU runtime, and freeing tables does (hipFree), so the
// callback only moves its reference into a pending list (`Deferred`); an
// ordinary library call, outside any capture, drops the pending references
// later.
#pragma once

#include <cstddef>
#include <list>
#include <memory>
#include <mutex>
#include <utility>
#include <vector>

namespace mgr {

// Least-recently-used map from K to shared_ptr<V>, at most `cap` entries.
// Not thread-safe by itself: the caller holds its own lock.  Entries it
// drops are handed back to the caller, who releases them after unlocking
// (the last release of a plan frees device memory).
template <typename K, typename V>
class LruCache {
 public:
  explicit LruCache(size_t cap) : cap_(cap < 1 ? 1 : cap) {}

  // The entry for k, moved to the front; nullptr if absent.
  std::shared_ptr<V> find(const K &k) {
    for (auto it = items_.begin(); it != items_.end(); ++it)
      if (it->first == k) {
        items_.splice(items_.begin(), items_, it);
        return items_.front().second;
      }
    return nullptr;
  }

  // Inserts (or replaces) k at the front; entries beyond the capacity are
  // appended to `dropped`.
  void insert(const K &k, std::shared_ptr<V> v, std::vector<std::shared_ptr<V>> &dropped) {
    for (auto it = items_.begin(); it != items_.end(); ++it)
      if (it->first == k) {
        dropped.push_back(std::move(it->second));
        items_.erase(it);
        break;
      }
    items_.emplace_front(k, std::move(v));
    while (items_.size() > cap_) {
      dropped.push_back(std::move(items_.back().second));
      items_.pop_back();
    }
  }

  void clear(std::vector<std::shared_ptr<V>> &dropped) {
    for (auto &e : items_) dropped.push_back(std::move(e.second));
    items_.clear();
  }

  size_t size() const { return items_.size(); }
  size_t capacity() const { return cap_; }

 private:
  size_t cap_;
  std::list<std::pair<K, std::shared_ptr<V>>> items_;
};

// References released by callbacks that must not destroy what they hold.
template <typename V>
class Deferred {
 public:
  // A heap holder of one reference, to be passed to a release callback as
  // its user pointer.
  static std::shared_ptr<V> *hold(std::shared_ptr<V> v) { return new std::shared_ptr<V>(std::move(v)); }

  // The callback's body: takes over the holder's reference without
  // releasing it (the object is not destroyed here) and frees the holder.
  void release(std::shared_ptr<V> *h) {
    std::lock_guard<std::mutex> lk(mu_);
    pending_.push_back(std::move(*h));
    delete h;
  }

  // Drops the pending references (from an ordinary call, never from a
  // callback); returns how many there were.
  size_t drain() {
    std::vector<std::shared_ptr<V>> v;
    {
      std::lock_guard<std::mutex> lk(mu_);
      v.swap(pending_);
    }
    return v.size();  // v's references are released here, after the lock
  }

  size_t pending() {
    std::lock_guard<std::mutex> lk(mu_);
    return pending_.size();
  }

 private:
  std::mutex mu_;
  std::vector<std::shared_ptr<V>> pending_;
};

}  // namespace mgr
