// Host check of the plan cache's bookkeeping (csrc/mgr_plan_cache.hpp):
//  1. LruCache against a plain list model on random insert/find sequences:
//     same order, same entries dropped, never more than the capacity;
//  2. lifetimes: an object is destroyed exactly when its last owner -- the
//     cache, a call in progress, or a graph's holder -- lets go; a holder's
//     release callback (Deferred::release) never destroys anything, and the
//     object is destroyed by Deferred::drain only if no other owner is left.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <random>
#include <set>
#include <vector>

#include "mgr_plan_cache.hpp"

namespace {

std::set<int> g_alive;  // ids of objects not yet destroyed

struct Obj {
  int id;
  explicit Obj(int i) : id(i) { g_alive.insert(i); }
  ~Obj() { g_alive.erase(id); }
};

int fail(const char *what, int a = 0, int b = 0) {
  std::printf("FAIL %s %d %d\n", what, a, b);
  return 1;
}

int check_lru(unsigned seed) {
  std::mt19937 rng(seed);
  for (int round = 0; round < 200; ++round) {
    const size_t cap = 1 + rng() % 8;
    mgr::LruCache<int, Obj> c(cap);
    std::vector<int> model;  // keys, most recent first
    int next_id = 0;
    std::vector<std::shared_ptr<Obj>> dropped;
    for (int op = 0; op < 300; ++op) {
      const int key = (int)(rng() % 12);
      if (rng() % 2) {
        auto v = c.find(key);
        auto it = std::find(model.begin(), model.end(), key);
        if ((v != nullptr) != (it != model.end())) return fail("find presence", key);
        if (it != model.end()) {
          model.erase(it);
          model.insert(model.begin(), key);
        }
      } else {
        dropped.clear();
        c.insert(key, std::make_shared<Obj>(1000000 * round + next_id++), dropped);
        std::vector<int> want_drop;
        auto it = std::find(model.begin(), model.end(), key);
        if (it != model.end()) {
          want_drop.push_back(key);
          model.erase(it);
        }
        model.insert(model.begin(), key);
        while (model.size() > cap) {
          want_drop.push_back(model.back());
          model.pop_back();
        }
        if (dropped.size() != want_drop.size()) return fail("dropped count", (int)dropped.size(), (int)want_drop.size());
      }
      if (c.size() != model.size() || c.size() > cap) return fail("size", (int)c.size(), (int)model.size());
    }
    // every entry the model keeps is still cached
    for (int k : model)
      if (!c.find(k)) return fail("final presence", k);
    dropped.clear();
    c.clear(dropped);
    if (c.size() != 0 || dropped.size() != model.size()) return fail("clear");
  }
  return 0;
}

int check_lifetimes(unsigned seed) {
  std::mt19937 rng(seed);
  for (int round = 0; round < 300; ++round) {
    g_alive.clear();
    const size_t cap = 1 + rng() % 4;
    mgr::LruCache<int, Obj> cache(cap);
    mgr::Deferred<Obj> deferred;
    std::vector<std::shared_ptr<Obj>> calls;     // references of calls in progress
    std::vector<std::shared_ptr<Obj> *> graphs;  // holders given to graphs
    std::vector<std::shared_ptr<Obj>> dropped;
    int next_id = 0;
    for (int op = 0; op < 200; ++op) {
      const int what = (int)(rng() % 6);
      if (what == 0) {  // a call builds a plan and caches it
        auto p = std::make_shared<Obj>(next_id++);
        dropped.clear();
        cache.insert((int)(rng() % 6), p, dropped);
        calls.push_back(p);
        dropped.clear();  // the dropped entries are released outside the lock
      } else if (what == 1 && !calls.empty()) {  // a call under capture retains its plan in the graph
        graphs.push_back(mgr::Deferred<Obj>::hold(calls.back()));
      } else if (what == 2 && !calls.empty()) {  // a call returns
        calls.pop_back();
      } else if (what == 3 && !graphs.empty()) {  // a graph is destroyed: the callback runs
        const size_t i = rng() % graphs.size();
        const int id = (*graphs[i])->id;
        const size_t before = g_alive.size();
        deferred.release(graphs[i]);
        graphs.erase(graphs.begin() + (long)i);
        if (g_alive.size() != before || !g_alive.count(id)) return fail("callback destroyed an object", id);
      } else if (what == 4) {  // an ordinary call drains the pending references
        deferred.drain();
      } else if (what == 5 && rng() % 8 == 0) {
        dropped.clear();
        cache.clear(dropped);
        dropped.clear();
      }
      // every live object has an owner, and every owned object is alive
      std::set<int> owned;
      for (auto &p : calls) owned.insert(p->id);
      for (auto *h : graphs) owned.insert((*h)->id);
      for (int k = 0; k < 6; ++k)  // (find reorders the cache, which does not matter here)
        if (auto v = cache.find(k)) owned.insert(v->id);
      const size_t pend = deferred.pending();
      if (pend == 0 && owned != g_alive) return fail("ownership", (int)owned.size(), (int)g_alive.size());
      if (pend > 0)
        for (int id : owned)
          if (!g_alive.count(id)) return fail("owned object destroyed", id);
    }
    calls.clear();
    for (auto *h : graphs) deferred.release(h);
    graphs.clear();
    dropped.clear();
    cache.clear(dropped);
    dropped.clear();
    deferred.drain();
    if (!g_alive.empty()) return fail("leak", (int)g_alive.size());
  }
  return 0;
}

}  // namespace

int main(int argc, char **argv) {
  const unsigned seed = argc > 1 ? (unsigned)std::atoi(argv[1]) : 1u;
  if (check_lru(seed)) return 1;
  if (check_lifetimes(seed)) return 1;
  std::printf("ok\n");
  return 0;
}
