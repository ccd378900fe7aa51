// mgr_timing.cpp -- per-kernel HIP-event timing behind mgr_timing_* (mgr.h).
#include "mgr_timing.hpp"

#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mgr.h"

namespace mgr {

namespace {

struct Pending {
  int kernel;
  hipEvent_t start, stop;
  double bytes;
};

struct Totals {
  std::string name;
  long long launches = 0;
  double ms = 0.0;
  double bytes = 0.0;
};

std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<hipEvent_t> g_free;
std::vector<Pending> g_pending;
std::vector<Totals> g_totals;
std::map<std::string, int> g_index;

hipEvent_t take_event() {
  if (!g_free.empty()) {
    hipEvent_t e = g_free.back();
    g_free.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Waits for every pending record and folds it into the totals.
void drain_locked() {
  for (const Pending &p : g_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
      Totals &t = g_totals[p.kernel];
      t.launches += 1;
      t.ms += ms;
      t.bytes += p.bytes;
    }
    g_free.push_back(p.start);
    g_free.push_back(p.stop);
  }
  g_pending.clear();
}

thread_local int g_quiet = 0;  // TimingOff guards active on this thread

}  // namespace

TimingOff::TimingOff() { ++g_quiet; }
TimingOff::~TimingOff() { --g_quiet; }

bool timing_enabled() { return g_quiet == 0 && g_on.load(std::memory_order_relaxed); }

TimedLaunch::TimedLaunch(hipStream_t s, const std::string &name, double alg_bytes) : stream_(s) {
  if (!timing_enabled()) return;
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_index.find(name);
  int k;
  if (it == g_index.end()) {
    k = (int)g_totals.size();
    g_index[name] = k;
    g_totals.push_back(Totals{name});
  } else {
    k = it->second;
  }
  hipEvent_t a = take_event(), b = take_event();
  if (!a || !b) return;
  if (hipEventRecord(a, s) != hipSuccess) return;
  g_pending.push_back(Pending{k, a, b, alg_bytes});
  slot_ = (int)g_pending.size() - 1;
}

TimedLaunch::~TimedLaunch() {
  if (slot_ < 0) return;
  std::lock_guard<std::mutex> lk(g_mu);
  if (slot_ < (int)g_pending.size()) (void)hipEventRecord(g_pending[slot_].stop, stream_);
}

}  // namespace mgr

extern "C" {

mgr_status mgr_timing_enable(int on) {
  mgr::g_on.store(on != 0);
  return MGR_OK;
}

void mgr_timing_reset(void) {
  std::lock_guard<std::mutex> lk(mgr::g_mu);
  mgr::drain_locked();
  mgr::g_totals.clear();
  mgr::g_index.clear();
}

int mgr_timing_count(void) {
  std::lock_guard<std::mutex> lk(mgr::g_mu);
  mgr::drain_locked();
  return (int)mgr::g_totals.size();
}

mgr_status mgr_timing_get(int index, const char **name, int64_t *launches, double *total_ms,
                          double *alg_bytes) {
  std::lock_guard<std::mutex> lk(mgr::g_mu);
  mgr::drain_locked();
  if (index < 0 || index >= (int)mgr::g_totals.size()) return MGR_ERR_INVALID_ARG;
  const mgr::Totals &t = mgr::g_totals[index];
  if (name) *name = t.name.c_str();
  if (launches) *launches = t.launches;
  if (total_ms) *total_ms = t.ms;
  if (alg_bytes) *alg_bytes = t.bytes;
  return MGR_OK;
}

}  // extern "C"
