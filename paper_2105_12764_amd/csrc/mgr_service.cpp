// mgr_service.cpp -- a refactoring service: a stream of decompose /
// recompose requests admitted by HBM footprint and run on a few streams.
//
// Requests are admitted first-in first-out while the in-flight footprint --
// every admitted request's input, output and workspace bytes -- stays
// within the service's budget.  Workspace comes from one arena allocated at
// creation (first fit, coalescing on release), so no request allocates
// device memory.  A request's plan (the library's tables for its shape,
// coordinates and level count) is built or found by the submitting thread
// before the service lock is taken, so a new shape's table upload does not
// hold up the other requests.  An admitted request is enqueued on the internal stream
// with the fewest requests running, followed by an event; one waiter thread
// per stream retires its requests in order, releases their budget and
// workspace, and admits what waits.  Times are host steady-clock
// milliseconds: submit, start (enqueued) and done (the waiter saw the event).
// A request's coordinates are freed once it is enqueued; its record (about
// a hundred bytes: status and times) stays until the service is destroyed.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/mgr.h"
#include "mgr_api_internal.hpp"
#include "mgr_arena.hpp"

namespace {

thread_local std::string g_service_error;

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  bool recompose = false;
  int ndim = 0;
  int64_t shape[4] = {0, 0, 0, 0};
  std::vector<std::vector<double>> coords;  // host copies (empty: uniform)
  mgr_dtype dtype = MGR_FLOAT64;
  int nlevels = 0;
  const void *in = nullptr;
  void *out = nullptr;
  size_t ws_bytes = 0, footprint = 0, ws_off = 0;
  int stream = -1;
  hipEvent_t ev = nullptr;
  double t_submit = 0, t_start = 0, t_done = 0;
  bool done = false;
  mgr_status status = MGR_OK;
};

}  // namespace

struct mgr_service {
  int device = 0;
  size_t budget = 0, in_flight = 0;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  mgr::ArenaFit fit;  // workspace ranges of the arena
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request *> pending;
  std::vector<std::deque<Request *>> running;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> waiters;
  std::vector<std::unique_ptr<Request>> all;  // index = ticket - 1
  bool stop = false;

  // Enqueue waiting requests in order while budget and workspace allow
  // (caller holds mu).
  void admit() {
    while (!pending.empty()) {
      Request *r = pending.front();
      if (in_flight + r->footprint > budget) return;
      size_t off = 0;
      if (!fit.alloc(r->ws_bytes, off)) return;
      pending.pop_front();
      r->ws_off = off;
      in_flight += r->footprint;
      size_t best = 0;
      for (size_t k = 1; k < running.size(); ++k)
        if (running[k].size() < running[best].size()) best = k;
      r->stream = (int)best;
      std::vector<const double *> cp(r->ndim, nullptr);
      for (int k = 0; k < r->ndim && !r->coords.empty(); ++k) cp[k] = r->coords[k].data();
      const double *const *carg = r->coords.empty() ? nullptr : cp.data();
      void *ws = r->ws_bytes ? (void *)(arena + off) : nullptr;
      r->t_start = now_ms();
      const mgr_status s =
          r->recompose ? mgr_recompose(r->ndim, r->shape, carg, r->dtype, r->nlevels, r->in, r->out, ws,
                                       r->ws_bytes, streams[best])
                       : mgr_decompose(r->ndim, r->shape, carg, r->dtype, r->nlevels, r->in, r->out, ws,
                                       r->ws_bytes, streams[best]);
      r->status = s;
      // the library keeps its own tables: the request needs its coordinates no more
      std::vector<std::vector<double>>().swap(r->coords);
      if (s == MGR_OK && hipEventRecord(r->ev, streams[best]) != hipSuccess) {
        (void)hipGetLastError();
        r->status = MGR_ERR_DEVICE;
      }
      running[best].push_back(r);  // the waiter retires it (also on failure)
    }
  }

  void waiter(size_t k) {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv.wait(lk, [&] { return stop || !running[k].empty(); });
      if (running[k].empty()) return;  // stop requested and nothing left
      Request *r = running[k].front();
      lk.unlock();
      if (r->status == MGR_OK && hipEventSynchronize(r->ev) != hipSuccess) {
        (void)hipGetLastError();
        r->status = MGR_ERR_DEVICE;
      }
      const double t = now_ms();
      lk.lock();
      running[k].pop_front();
      r->t_done = t;
      r->done = true;
      in_flight -= r->footprint;
      fit.release(r->ws_off, r->ws_bytes);
      (void)hipEventDestroy(r->ev);
      r->ev = nullptr;
      admit();
      cv.notify_all();
    }
  }
};

namespace {

mgr_status sfail(mgr_status s, const std::string &m) {
  g_service_error = m;
  return s;
}

}  // namespace

extern "C" {

mgr_status mgr_service_create(size_t budget_bytes, int nstreams, mgr_service **svc) {
  if (!svc) return sfail(MGR_ERR_INVALID_ARG, "svc is NULL");
  *svc = nullptr;
  if (budget_bytes < 4096) return sfail(MGR_ERR_INVALID_ARG, "budget too small");
  if (nstreams < 1 || nstreams > 16) return sfail(MGR_ERR_INVALID_ARG, "nstreams must be in 1..16");
  try {
    auto s = std::make_unique<mgr_service>();
    if (hipGetDevice(&s->device) != hipSuccess) {
      (void)hipGetLastError();
      return sfail(MGR_ERR_DEVICE, "hipGetDevice failed");
    }
    s->budget = budget_bytes;
    // Workspace against footprint (mgr_workspace_size): three FP64 grids of
    // the level-1 shape and one of the level-2 shape (4-D: three FP64 coarse
    // grids and nt FP64 coarse space slices), each rounded up to 256 bytes.
    // A dimension of m >= 3 nodes keeps m/2 + 1 <= 3m/4 of them (m = 4 is
    // the worst) and a dimension of 2 keeps both, so the level-1 grid holds
    // at most 3/4 of the N nodes and the level-2 grid at most 1/2 (4-D: the
    // coarse grids at most 3/4, the slices at most N).  The workspace is then
    // at most 22N bytes (4-D: 26N) plus 1 KiB of rounding, against a
    // footprint of 2Ns bytes (s >= 4) plus the workspace: below 0.77 of the
    // footprint plus 1 KiB.  An arena of 4/5 of the budget plus 1 MiB
    // therefore holds any request whose footprint is within the budget; an
    // in-flight set whose workspaces do not fit together waits for a release
    // (with nothing in flight the arena is empty, so the head request always
    // fits eventually).
    s->arena_bytes = std::min(budget_bytes, budget_bytes / 5 * 4 + ((size_t)1 << 20));
    s->arena_bytes = mgr::ArenaFit::round_up(s->arena_bytes);
    if (hipMalloc((void **)&s->arena, s->arena_bytes) != hipSuccess) {
      (void)hipGetLastError();
      return sfail(MGR_ERR_OUT_OF_MEMORY, "workspace arena allocation failed");
    }
    s->fit.reset(s->arena_bytes);
    s->running.resize(nstreams);
    s->streams.assign(nstreams, nullptr);
    for (int k = 0; k < nstreams; ++k)
      if (hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        for (int q = 0; q < k; ++q) (void)hipStreamDestroy(s->streams[q]);
        (void)hipFree(s->arena);
        return sfail(MGR_ERR_DEVICE, "stream creation failed");
      }
    mgr_service *raw = s.get();
    for (int k = 0; k < nstreams; ++k) raw->waiters.emplace_back([raw, k] { raw->waiter((size_t)k); });
    *svc = s.release();
    return MGR_OK;
  } catch (...) {
    return sfail(MGR_ERR_OUT_OF_MEMORY, "service creation failed");
  }
}

mgr_status mgr_service_submit(mgr_service *svc, int recompose, int ndim, const int64_t *shape,
                              const double *const *coords, mgr_dtype dtype, int nlevels, const void *in,
                              void *out, uint64_t *ticket) {
  if (!svc || !ticket) return sfail(MGR_ERR_INVALID_ARG, "svc and ticket must be non-NULL");
  if (ndim < 1 || ndim > 4 || !shape) return sfail(MGR_ERR_INVALID_ARG, "ndim must be 1..4 with a shape");
  size_t ws = 0;
  mgr_status s = mgr_workspace_size(ndim, shape, dtype, nlevels, &ws);
  if (s != MGR_OK) return sfail(s, mgr_last_error());
  if (!in || !out) return sfail(MGR_ERR_INVALID_ARG, "in and out must be non-NULL device pointers");
  // build (or find) the request's plan here, outside the service lock; a
  // request whose arguments the library rejects fails when it is enqueued
  // and reports its status through mgr_service_result
  {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != svc->device) (void)hipSetDevice(svc->device);
    (void)mgr::prepare_plan(ndim, shape, coords, nlevels);
    if (cur >= 0 && cur != svc->device) (void)hipSetDevice(cur);
    (void)hipGetLastError();
  }
  try {
    auto r = std::make_unique<Request>();
    r->recompose = recompose != 0;
    r->ndim = ndim;
    size_t n = 1;
    for (int k = 0; k < ndim; ++k) {
      r->shape[k] = shape[k];
      n *= (size_t)shape[k];
    }
    if (coords) {
      r->coords.resize(ndim);
      for (int k = 0; k < ndim; ++k) {
        if (coords[k]) r->coords[k].assign(coords[k], coords[k] + shape[k]);
        else {
          r->coords[k].resize(shape[k]);
          for (int64_t i = 0; i < shape[k]; ++i) r->coords[k][i] = (double)i;
        }
      }
    }
    r->dtype = dtype;
    r->nlevels = nlevels;
    r->in = in;
    r->out = out;
    r->ws_bytes = ws;
    r->footprint = 2 * n * (dtype == MGR_FLOAT64 ? 8 : 4) + ws;
    if (r->footprint > svc->budget) return sfail(MGR_ERR_UNSUPPORTED, "request larger than the service budget");
    if (mgr::ArenaFit::round_up(ws) > svc->arena_bytes)
      return sfail(MGR_ERR_UNSUPPORTED, "request workspace larger than the service arena");
    if (hipEventCreateWithFlags(&r->ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return sfail(MGR_ERR_DEVICE, "hipEventCreate failed");
    }
    std::lock_guard<std::mutex> lk(svc->mu);
    r->ticket = svc->all.size() + 1;
    r->t_submit = now_ms();
    *ticket = r->ticket;
    svc->pending.push_back(r.get());
    svc->all.push_back(std::move(r));
    svc->admit();
    svc->cv.notify_all();
    return MGR_OK;
  } catch (...) {
    return sfail(MGR_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

mgr_status mgr_service_wait_all(mgr_service *svc) {
  if (!svc) return sfail(MGR_ERR_INVALID_ARG, "svc is NULL");
  std::unique_lock<std::mutex> lk(svc->mu);
  svc->cv.wait(lk, [&] {
    if (!svc->pending.empty()) return false;
    for (auto &q : svc->running)
      if (!q.empty()) return false;
    return true;
  });
  return MGR_OK;
}

mgr_status mgr_service_result(mgr_service *svc, uint64_t ticket, int *done, mgr_status *status,
                              double *queue_ms, double *latency_ms) {
  if (!svc) return sfail(MGR_ERR_INVALID_ARG, "svc is NULL");
  std::lock_guard<std::mutex> lk(svc->mu);
  if (ticket == 0 || ticket > svc->all.size()) return sfail(MGR_ERR_INVALID_ARG, "unknown ticket");
  const Request &r = *svc->all[ticket - 1];
  if (done) *done = r.done ? 1 : 0;
  if (status) *status = r.status;
  if (queue_ms) *queue_ms = r.t_start > 0 ? r.t_start - r.t_submit : -1.0;
  if (latency_ms) *latency_ms = r.done ? r.t_done - r.t_submit : -1.0;
  return MGR_OK;
}

mgr_status mgr_service_destroy(mgr_service *svc) {
  if (!svc) return MGR_OK;
  mgr_service_wait_all(svc);
  {
    std::lock_guard<std::mutex> lk(svc->mu);
    svc->stop = true;
  }
  svc->cv.notify_all();
  for (auto &t : svc->waiters) t.join();
  {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != svc->device) (void)hipSetDevice(svc->device);
    // the recomposition helper streams the library registered for these streams
    mgr::forget_helpers(svc->streams.data(), (int)svc->streams.size());
    if (cur >= 0 && cur != svc->device) (void)hipSetDevice(cur);
  }
  for (auto &s : svc->streams) (void)hipStreamDestroy(s);
  (void)hipFree(svc->arena);
  delete svc;
  return MGR_OK;
}

const char *mgr_service_last_error(void) { return g_service_error.c_str(); }

}  // extern "C"
