// mgr_api.cpp -- the extern "C" boundary of libmgr (declared in include/mgr.h):
// argument validation, the per-device plan cache and dispatch to the HIP
// kernels.  No exception crosses the boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mgr.h"
#include "mgr_api_internal.hpp"
#include "mgr_kernels.hpp"
#include "mgr_plan.hpp"
#include "mgr_plan_cache.hpp"
#include "mgr_timing.hpp"

namespace {

thread_local std::string g_last_error;
thread_local std::string g_tune_report;

mgr_status fail(mgr_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

// Cache key of a plan: the device, the caller's rank, the padded shape, the
// time extent (4-D), the level count and the coordinates.
struct PlanKey {
  int device;
  int ndim;
  int64_t n[mgr::kDims];
  int64_t nt;  // time extent of a 4-D field (1 otherwise)
  int nlev;
  std::vector<std::vector<double>> coords;
  bool operator==(const PlanKey &o) const {
    return device == o.device && ndim == o.ndim && nt == o.nt && nlev == o.nlev &&
           std::memcmp(n, o.n, sizeof(n)) == 0 && coords == o.coords;
  }
};

// Key of autotuned launch shapes: they depend on the grid's shape, not on
// its coordinates.
struct TuneKey {
  int device;
  int ndim;
  int64_t n[mgr::kDims];
  int64_t nt;
  int nlev;
  bool operator==(const TuneKey &o) const {
    return device == o.device && ndim == o.ndim && nt == o.nt && nlev == o.nlev &&
           std::memcmp(n, o.n, sizeof(n)) == 0;
  }
};
using TuneVec = std::vector<mgr::LevelTune>;

// Plans kept at most (a batch of more distinct fields than this cannot be
// captured into a graph: its warm-up call would evict its own first plans),
// and tuned shapes kept at most.
constexpr size_t kCacheMax = 1024;
constexpr size_t kTuneMax = 4096;

std::mutex g_mu;  // guards g_cache and g_tunes
mgr::LruCache<PlanKey, mgr::Plan> g_cache(kCacheMax);
mgr::LruCache<TuneKey, TuneVec> g_tunes(kTuneMax);
// Plan references given up by destroyed graphs, released by a later call.
mgr::Deferred<mgr::Plan> g_deferred;

void graph_release_plan(void *holder) { g_deferred.release(static_cast<std::shared_ptr<mgr::Plan> *>(holder)); }

// Whether `stream` is capturing into a graph (and which), or an error.
mgr_status capture_state(void *stream, bool &capturing, hipGraph_t *graph = nullptr) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamGetCaptureInfo_v2((hipStream_t)stream, &st, nullptr, &g, nullptr, nullptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MGR_ERR_DEVICE, std::string("hipStreamGetCaptureInfo: ") + hipGetErrorString(e));
  }
  capturing = st == hipStreamCaptureStatusActive;
  if (graph) *graph = capturing ? g : nullptr;
  return MGR_OK;
}

// Keeps `plans` alive for as long as the graph being captured on `stream`
// (and every executable made from it) exists: each gets a user object that
// the graph owns.  No-op when the stream is not capturing.
mgr_status retain_for_capture(void *stream, const std::vector<std::shared_ptr<mgr::Plan>> &plans) {
  bool capturing = false;
  hipGraph_t g = nullptr;
  mgr_status s = capture_state(stream, capturing, &g);
  if (s != MGR_OK || !capturing) return s;
  for (const auto &p : plans) {
    auto *h = mgr::Deferred<mgr::Plan>::hold(p);
    hipUserObject_t obj = nullptr;
    if (hipUserObjectCreate(&obj, h, graph_release_plan, 1, hipUserObjectNoDestructorSync) != hipSuccess) {
      (void)hipGetLastError();
      delete h;
      return fail(MGR_ERR_DEVICE, "hipUserObjectCreate failed while capturing");
    }
    if (hipGraphRetainUserObject(g, obj, 1, hipGraphUserObjectMove) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipUserObjectRelease(obj, 1);  // runs graph_release_plan
      return fail(MGR_ERR_DEVICE, "hipGraphRetainUserObject failed while capturing");
    }
  }
  return MGR_OK;
}

// Pads the caller's shape to rank 3 with leading 1s.
bool pad_shape(int ndim, const int64_t *shape, int64_t n[mgr::kDims], std::string &why) {
  if (ndim < 1 || ndim > 3) {
    why = ndim == 4 ? "4-D fields are taken by mgr_decompose, mgr_recompose, mgr_workspace_size and "
                      "mgr_max_levels only"
                    : "ndim must be 1, 2, 3 or 4 (got " + std::to_string(ndim) + ")";
    return false;
  }
  if (!shape) {
    why = "shape is NULL";
    return false;
  }
  for (int k = 0; k < mgr::kDims; ++k) n[k] = 1;
  for (int k = 0; k < ndim; ++k) {
    if (shape[k] < 2) {
      why = "shape[" + std::to_string(k) + "] must be >= 2";
      return false;
    }
    if (shape[k] > (int64_t)1 << 31) {
      why = "shape[" + std::to_string(k) + "] too large";
      return false;
    }
    n[mgr::kDims - ndim + k] = shape[k];
  }
  if (n[1] * n[2] >= ((int64_t)1 << 31)) {
    why = "a plane (product of the last two dimensions) must hold fewer than 2^31 nodes";
    return false;
  }
  const int64_t total = n[0] * n[1] * n[2];
  if (total <= 0 || total > ((int64_t)1 << 40)) {
    why = "total element count out of range";
    return false;
  }
  return true;
}

// Shapes of 1 to 4 dims.  A 4-D shape is (time, then three space dims): n
// gets the space dims and nt the time extent (1 below 4-D).
bool split_shape(int ndim, const int64_t *shape, int64_t n[mgr::kDims], int64_t &nt, std::string &why) {
  nt = 1;
  if (ndim != 4) return pad_shape(ndim, shape, n, why);
  if (!shape) {
    why = "shape is NULL";
    return false;
  }
  for (int k = 0; k < 4; ++k) {
    if (shape[k] < 2) {
      why = "shape[" + std::to_string(k) + "] must be >= 2";
      return false;
    }
    if (shape[k] > (int64_t)1 << 31) {
      why = "shape[" + std::to_string(k) + "] too large";
      return false;
    }
  }
  if (!pad_shape(3, shape + 1, n, why)) return false;
  const int64_t slice = n[0] * n[1] * n[2];
  if (slice >= ((int64_t)1 << 31)) {
    why = "a time slice (product of the last three dimensions) must hold fewer than 2^31 nodes";
    return false;
  }
  if (shape[0] > (((int64_t)1 << 40) / slice)) {
    why = "total element count out of range";
    return false;
  }
  nt = shape[0];
  return true;
}

// Per-dim coordinates: the padded rank-3 dims, or (4-D) time then space;
// NULL entries (or coords == NULL) are uniform.
mgr_status make_coords(int ndim, const int64_t n[mgr::kDims], int64_t nt, const double *const *coords,
                       std::vector<std::vector<double>> &cx) {
  const int nc = ndim == 4 ? 4 : mgr::kDims;
  cx.assign(nc, {});
  for (int k = 0; k < nc; ++k) {
    const int uk = ndim == 4 ? k : k - (mgr::kDims - ndim);
    const int64_t ext = ndim == 4 ? (k == 0 ? nt : n[k - 1]) : n[k];
    const double *src = (uk >= 0 && coords) ? coords[uk] : nullptr;
    cx[k].resize(ext);
    for (int64_t i = 0; i < ext; ++i) {
      const double v = src ? src[i] : (double)i;
      if (!std::isfinite(v))
        return fail(MGR_ERR_INVALID_ARG, "coords[" + std::to_string(uk) + "] has a non-finite value");
      if (i > 0 && !(v > cx[k][i - 1]))
        return fail(MGR_ERR_INVALID_ARG,
                    "coords[" + std::to_string(uk) + "] is not strictly increasing");
      cx[k][i] = v;
    }
  }
  return MGR_OK;
}

mgr_status validate(int ndim, const int64_t *shape, const double *const *coords, int dtype,
                    int nlevels, const void *in, void *out, void *ws, size_t ws_bytes,
                    int64_t n[mgr::kDims], std::vector<std::vector<double>> &cx, int64_t *nt_out = nullptr) {
  std::string why;
  int64_t nt = 1;
  if (!split_shape(ndim, shape, n, nt, why)) return fail(MGR_ERR_INVALID_ARG, why);
  if (nt_out) *nt_out = nt;
  if (dtype != MGR_FLOAT32 && dtype != MGR_FLOAT64)
    return fail(MGR_ERR_INVALID_ARG, "dtype must be MGR_FLOAT32 or MGR_FLOAT64");
  const int ml = ndim == 4 ? mgr::max_levels4(nt, n) : mgr::max_levels3(n);
  if (nlevels < 0 || nlevels > ml)
    return fail(MGR_ERR_INVALID_ARG, "nlevels must be in [0, " + std::to_string(ml) + "]");
  if (nlevels > mgr::kMaxLevels) return fail(MGR_ERR_UNSUPPORTED, "too many levels");
  if (!in || !out) return fail(MGR_ERR_INVALID_ARG, "in and out must be non-NULL device pointers");
  const size_t esz = dtype == MGR_FLOAT64 ? 8 : 4;
  const size_t bytes = (size_t)(nt * n[0] * n[1] * n[2]) * esz;
  const char *a = (const char *)in, *b = (const char *)out;
  if (a < b + bytes && b < a + bytes) return fail(MGR_ERR_INVALID_ARG, "in and out overlap");
  const mgr_status sc = make_coords(ndim, n, nt, coords, cx);
  if (sc != MGR_OK) return sc;
  const size_t need = ndim == 4 ? mgr::workspace_bytes4(nt, n, nlevels, esz) : mgr::workspace_bytes(n, nlevels, esz);
  if (need > 0) {
    if (!ws) return fail(MGR_ERR_WORKSPACE, "workspace is NULL");
    if (ws_bytes < need)
      return fail(MGR_ERR_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
    if ((uintptr_t)ws % 256 != 0) return fail(MGR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    const char *w = (const char *)ws;
    if ((w < a + bytes && a < w + need) || (w < b + bytes && b < w + need))
      return fail(MGR_ERR_INVALID_ARG, "workspace overlaps in or out");
  }
  return MGR_OK;
}

// The cached plan of a request, built and cached if there is none.  A plan
// is built with a device allocation and a synchronous copy, which stream
// capture does not allow, so under capture (`stream` capturing) a missing
// plan is an error.  Tuned launch shapes kept for the shape are restored
// into a new plan.
mgr_status get_plan(const int64_t n[mgr::kDims], int ndim, int nlevels,
                    const std::vector<std::vector<double>> &cx, std::shared_ptr<mgr::Plan> &out,
                    void *stream, int64_t nt = 1) {
  int dev = -1;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) {
    (void)hipGetLastError();
    return fail(MGR_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(he));
  }
  bool capturing = false;
  mgr_status cs = capture_state(stream, capturing);
  if (cs != MGR_OK) return cs;
  if (!capturing) g_deferred.drain();  // plans of destroyed graphs (may free device tables)
  PlanKey key{dev, ndim, {n[0], n[1], n[2]}, nt, nlevels, cx};
  {
    std::lock_guard<std::mutex> lk(g_mu);
    out = g_cache.find(key);
    if (out) return MGR_OK;
  }
  if (capturing)
    return fail(MGR_ERR_UNSUPPORTED,
                "no cached plan for this request while the stream is capturing a graph (building one "
                "allocates device memory): make one call with the same shape, coordinates and level "
                "count outside the capture first");
  std::string err;
  int st = 0;
  std::unique_ptr<mgr::Plan> p;
  try {
    p = ndim == 4 ? mgr::build_plan4(nt, n, cx, nlevels, err, st) : mgr::build_plan(ndim, n, cx, nlevels, err, st);
  } catch (const std::bad_alloc &) {
    return fail(MGR_ERR_OUT_OF_MEMORY, "host allocation failed while building the plan");
  } catch (...) {
    return fail(MGR_ERR_DEVICE, "unexpected failure while building the plan");
  }
  if (!p) return fail((mgr_status)st, err);
  std::vector<std::shared_ptr<mgr::Plan>> dropped;  // released after the lock (frees device tables)
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (auto t = g_tunes.find(TuneKey{dev, ndim, {n[0], n[1], n[2]}, nt, nlevels})) p->tune = *t;
    out = std::shared_ptr<mgr::Plan>(p.release());
    g_cache.insert(key, out, dropped);
  }
  return MGR_OK;
}

// Keeps the tuned launch shapes of `pl` for later plans of the same shape.
void remember_tune(const mgr::Plan &pl, const int64_t n[mgr::kDims], int ndim, int64_t nt, int nlevels) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  auto t = std::make_shared<TuneVec>(pl.tune_snapshot());
  std::vector<std::shared_ptr<TuneVec>> dropped;
  std::lock_guard<std::mutex> lk(g_mu);
  g_tunes.insert(TuneKey{dev, ndim, {n[0], n[1], n[2]}, nt, nlevels}, t, dropped);
}

// A helper stream per (device, caller stream) for the work a recomposition
// runs beside the caller's stream, with its fork and join events; created on
// first use and kept until the process ends (a stream may still hold work).
// `mu` keeps one forked enqueue at a time per caller stream, so that the
// shared events pair up.
struct Helper {
  int device = -1;
  hipStream_t caller = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  std::mutex mu;
};
std::mutex g_hmu;
std::list<Helper> g_helpers;  // stable addresses
// Helpers kept at most: a caller that passes ever new streams gets serial
// recompositions beyond this rather than one more stream per call.
constexpr size_t kHelpersMax = 64;

// The helper of `caller` on the current device, or nullptr (then the call
// runs serially) when it cannot be created, the registry is full, or there
// is none yet and `create` is false (stream capture).
Helper *helper_for(hipStream_t caller, bool create) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_hmu);
  for (auto &h : g_helpers)
    if (h.device == dev && h.caller == caller) return &h;
  if (!create || g_helpers.size() >= kHelpersMax) return nullptr;
  hipStream_t s = nullptr;
  hipEvent_t f = nullptr, j = nullptr;
  bool ok = hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&f, hipEventDisableTiming) == hipSuccess;
  ok = ok && hipEventCreateWithFlags(&j, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    (void)hipGetLastError();
    if (j) (void)hipEventDestroy(j);
    if (f) (void)hipEventDestroy(f);
    if (s) (void)hipStreamDestroy(s);
    return nullptr;
  }
  Helper &h = g_helpers.emplace_back();
  h.device = dev;
  h.caller = caller;
  h.s = s;
  h.fork = f;
  h.join = j;
  return &h;
}

mgr_status run(bool dec, int ndim, const int64_t *shape, const double *const *coords, int dtype,
               int nlevels, const void *in, void *out, void *ws, size_t ws_bytes, void *stream,
               int nkeep = -1) {
  g_last_error.clear();
  try {
    int64_t n[mgr::kDims], nt = 1;
    std::vector<std::vector<double>> cx;
    mgr_status s = validate(ndim, shape, coords, dtype, nlevels, in, out, ws, ws_bytes, n, cx, &nt);
    if (s != MGR_OK) return s;
    if (nkeep != -1 && (nkeep < 0 || nkeep > nlevels))
      return fail(MGR_ERR_INVALID_ARG, "nkeep must be in [0, nlevels]");
    if (nkeep != -1 && ndim == 4)
      return fail(MGR_ERR_UNSUPPORTED, "partial recomposition of 4-D fields is not supported");
    std::shared_ptr<mgr::Plan> plan;
    s = get_plan(n, ndim, nlevels, cx, plan, stream, nt);
    if (s != MGR_OK) return s;
    bool capturing = false;
    s = capture_state(stream, capturing);
    if (s != MGR_OK) return s;
    std::string err;
    const bool f64 = dtype == MGR_FLOAT64;
    bool ok = false;
    if (dec) {
      ok = mgr::enqueue_decompose(*plan, f64, in, out, ws, stream, err);
    } else if (Helper *h = (plan->nlev >= 2 && !plan->time) ? helper_for((hipStream_t)stream, !capturing)
                                                            : nullptr) {
      std::lock_guard<std::mutex> lk(h->mu);
      const mgr::StreamFork fk{h->s, h->fork, h->join};
      ok = mgr::enqueue_recompose(*plan, f64, in, out, ws, stream, err, nkeep, &fk);
    } else {
      ok = mgr::enqueue_recompose(*plan, f64, in, out, ws, stream, err, nkeep);
    }
    if (!ok) return fail(MGR_ERR_DEVICE, err);
    if (capturing) return retain_for_capture(stream, {plan});
    return MGR_OK;
  } catch (const std::bad_alloc &) {
    return fail(MGR_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(MGR_ERR_DEVICE, "unexpected internal failure");
  }
}

// ------------------------------------------------------------ batches

// Internal streams of one device for batched calls, created on first use and
// kept until the process ends (a stream may still hold enqueued work).
struct BatchStreams {
  int device = -1;
  hipStream_t s[MGR_BATCH_STREAMS] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[MGR_BATCH_STREAMS] = {};
};
std::mutex g_bmu;                 // guards g_batch and serialises batch enqueues
std::list<BatchStreams> g_batch;  // stable addresses

mgr_status batch_streams(int dev, BatchStreams *&out) {
  for (auto &b : g_batch)
    if (b.device == dev) {
      out = &b;
      return MGR_OK;
    }
  BatchStreams b;
  b.device = dev;
  bool ok = hipEventCreateWithFlags(&b.fork, hipEventDisableTiming) == hipSuccess;
  for (int k = 0; ok && k < MGR_BATCH_STREAMS; ++k) {
    ok = hipStreamCreateWithFlags(&b.s[k], hipStreamNonBlocking) == hipSuccess;
    if (ok) ok = hipEventCreateWithFlags(&b.join[k], hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    const hipError_t e = hipGetLastError();
    for (int k = 0; k < MGR_BATCH_STREAMS; ++k) {
      if (b.join[k]) (void)hipEventDestroy(b.join[k]);
      if (b.s[k]) (void)hipStreamDestroy(b.s[k]);
    }
    if (b.fork) (void)hipEventDestroy(b.fork);
    return fail(MGR_ERR_DEVICE, std::string("creating the batch streams: ") + hipGetErrorString(e));
  }
  g_batch.push_back(b);
  out = &g_batch.back();
  return MGR_OK;
}

struct FieldJob {
  int64_t n[mgr::kDims];
  std::vector<std::vector<double>> cx;
  std::shared_ptr<mgr::Plan> plan;
  size_t ws_off = 0, ws_need = 0, bytes = 0;
};

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

std::string field_tag(int i) { return "field " + std::to_string(i) + ": "; }

// Shape, dtype and level checks of every field and the workspace layout.
mgr_status batch_layout(int nfields, const mgr_field *fields, std::vector<FieldJob> &jobs,
                        size_t &total) {
  if (nfields < 1) return fail(MGR_ERR_INVALID_ARG, "nfields must be >= 1");
  if (!fields) return fail(MGR_ERR_INVALID_ARG, "fields is NULL");
  jobs.assign(nfields, FieldJob{});
  total = 0;
  for (int i = 0; i < nfields; ++i) {
    const mgr_field &f = fields[i];
    std::string why;
    if (!pad_shape(f.ndim, f.shape, jobs[i].n, why)) return fail(MGR_ERR_INVALID_ARG, field_tag(i) + why);
    if (f.dtype != MGR_FLOAT32 && f.dtype != MGR_FLOAT64)
      return fail(MGR_ERR_INVALID_ARG, field_tag(i) + "dtype must be MGR_FLOAT32 or MGR_FLOAT64");
    const int ml = mgr::max_levels3(jobs[i].n);
    if (f.nlevels < 0 || f.nlevels > ml)
      return fail(MGR_ERR_INVALID_ARG,
                  field_tag(i) + "nlevels must be in [0, " + std::to_string(ml) + "]");
    const size_t esz = f.dtype == MGR_FLOAT64 ? 8 : 4;
    jobs[i].bytes = (size_t)(jobs[i].n[0] * jobs[i].n[1] * jobs[i].n[2]) * esz;
    jobs[i].ws_need = mgr::workspace_bytes(jobs[i].n, f.nlevels, esz);
    jobs[i].ws_off = total;
    total += align256(jobs[i].ws_need);
  }
  return MGR_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = (const char *)a, *y = (const char *)b;
  return x < y + nb && y < x + na;
}

// Streams of a batch's fields.  Per-field chains: largest first, each to the
// least loaded stream (by bytes).  Grouped launches: the fields of one class
// (rank and element type) share their kernels' launches, so a class stays on
// as few streams as it can: every class gets one stream, the streams left
// over go one at a time to the class with the most bytes per stream (no
// more streams than fields), and a class's fields go largest first to the
// least loaded of its streams; with more classes than streams, whole
// classes go largest first to the least loaded stream.  (A 64-field batch of
// four classes: 4.3 -> 3.5 ms from a graph against the per-field rule.)
void batch_lanes(int nfields, const mgr_field *fields, const std::vector<FieldJob> &jobs, const std::vector<int> &order,
                 bool grouped, std::vector<int> &lane) {
  constexpr int S = MGR_BATCH_STREAMS;
  double load[S] = {};
  auto least = [&](const std::vector<int> &ks) {
    int k = ks[0];
    for (int q : ks)
      if (load[q] < load[k]) k = q;
    return k;
  };
  std::vector<int> all(S);
  for (int k = 0; k < S; ++k) all[k] = k;
  if (!grouped) {
    for (int i : order) {
      const int k = least(all);
      lane[i] = k;
      load[k] += (double)jobs[i].bytes;
    }
    return;
  }
  // classes, most bytes first
  std::vector<int> key(nfields), ckey;
  std::vector<double> cbytes;
  std::vector<int> cfields;
  for (int i = 0; i < nfields; ++i) {
    key[i] = fields[i].ndim * 2 + (fields[i].dtype == MGR_FLOAT64 ? 1 : 0);
    const auto it = std::find(ckey.begin(), ckey.end(), key[i]);
    if (it == ckey.end()) {
      ckey.push_back(key[i]);
      cbytes.push_back((double)jobs[i].bytes);
      cfields.push_back(1);
    } else {
      cbytes[it - ckey.begin()] += (double)jobs[i].bytes;
      ++cfields[it - ckey.begin()];
    }
  }
  const int nc = (int)ckey.size();
  std::vector<int> corder(nc);
  for (int c = 0; c < nc; ++c) corder[c] = c;
  std::stable_sort(corder.begin(), corder.end(), [&](int a, int b) { return cbytes[a] > cbytes[b]; });
  std::vector<std::vector<int>> lanes_of(nc);
  if (nc >= S) {
    for (int c : corder) {
      const int k = least(all);
      lanes_of[c].push_back(k);
      load[k] += cbytes[c];
    }
  } else {
    std::vector<int> nl(nc, 1);
    for (int r = nc; r < S; ++r) {
      int best = -1;
      for (int c : corder)
        if (nl[c] < cfields[c] && (best < 0 || cbytes[c] / nl[c] > cbytes[best] / nl[best])) best = c;
      if (best < 0) break;
      ++nl[best];
    }
    int next = 0;
    for (int c : corder)
      for (int j = 0; j < nl[c]; ++j) lanes_of[c].push_back(next++);
  }
  for (int i : order) {
    const int c = (int)(std::find(ckey.begin(), ckey.end(), key[i]) - ckey.begin());
    const int k = nc >= S ? lanes_of[c][0] : least(lanes_of[c]);
    lane[i] = k;
    if (nc < S) load[k] += (double)jobs[i].bytes;
  }
}

mgr_status run_batch(bool dec, int nfields, const mgr_field *fields, void *ws, size_t ws_bytes,
                     void *stream, int flags) {
  g_last_error.clear();
  try {
    std::vector<FieldJob> jobs;
    size_t total = 0;
    mgr_status s = batch_layout(nfields, fields, jobs, total);
    if (s != MGR_OK) return s;
    if (total > 0) {
      if (!ws) return fail(MGR_ERR_WORKSPACE, "workspace is NULL");
      if (ws_bytes < total)
        return fail(MGR_ERR_WORKSPACE, "workspace too small: need " + std::to_string(total) + " bytes");
      if ((uintptr_t)ws % 256 != 0) return fail(MGR_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    }
    for (int i = 0; i < nfields; ++i) {
      const mgr_field &f = fields[i];
      void *wsi = ws ? (void *)((char *)ws + jobs[i].ws_off) : nullptr;
      s = validate(f.ndim, f.shape, f.coords, (int)f.dtype, f.nlevels, f.in, f.out, wsi, jobs[i].ws_need,
                   jobs[i].n, jobs[i].cx);
      if (s != MGR_OK) return fail(s, field_tag(i) + g_last_error);
      if (total > 0 && (overlaps(ws, total, f.in, jobs[i].bytes) || overlaps(ws, total, f.out, jobs[i].bytes)))
        return fail(MGR_ERR_INVALID_ARG, field_tag(i) + "in or out overlaps the batch workspace");
    }
    for (int i = 0; i < nfields; ++i)
      for (int j = 0; j < nfields; ++j) {
        if (i == j) continue;
        if (overlaps(fields[i].out, jobs[i].bytes, fields[j].out, jobs[j].bytes) ||
            overlaps(fields[i].out, jobs[i].bytes, fields[j].in, jobs[j].bytes))
          return fail(MGR_ERR_INVALID_ARG, field_tag(i) + "out overlaps the in or out of field " +
                                               std::to_string(j));
      }
    for (int i = 0; i < nfields; ++i) {
      s = get_plan(jobs[i].n, fields[i].ndim, fields[i].nlevels, jobs[i].cx, jobs[i].plan, stream);
      if (s != MGR_OK) return fail(s, field_tag(i) + g_last_error);
    }
    std::vector<std::shared_ptr<mgr::Plan>> plans;
    for (auto &j : jobs)
      if (std::find(plans.begin(), plans.end(), j.plan) == plans.end()) plans.push_back(j.plan);
    const bool grouped = !(flags & MGR_BATCH_PER_FIELD);
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
      const hipError_t e = hipGetLastError();
      return fail(MGR_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    std::vector<int> order(nfields);
    for (int i = 0; i < nfields; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return jobs[a].bytes > jobs[b].bytes; });
    std::vector<int> lane(nfields);
    batch_lanes(nfields, fields, jobs, order, grouped, lane);
    std::lock_guard<std::mutex> lk(g_bmu);
    BatchStreams *bs = nullptr;
    s = batch_streams(dev, bs);
    if (s != MGR_OK) return s;
    hipStream_t user = (hipStream_t)stream;
    if (hipEventRecord(bs->fork, user) != hipSuccess) {
      const hipError_t e = hipGetLastError();
      return fail(MGR_ERR_DEVICE, std::string("hipEventRecord: ") + hipGetErrorString(e));
    }
    bool used[MGR_BATCH_STREAMS] = {};
    for (int i = 0; i < nfields; ++i) used[lane[i]] = true;
    std::string err;
    bool ok = true;
    for (int k = 0; k < MGR_BATCH_STREAMS && ok; ++k)
      if (used[k] && hipStreamWaitEvent(bs->s[k], bs->fork, 0) != hipSuccess) {
        ok = false;
        err = std::string("hipStreamWaitEvent: ") + hipGetErrorString(hipGetLastError());
      }
    // Batches keep the register-prefetch load-vector kernel (bitwise the same
    // results): a HIP graph replay of a batch that used the ring kernel ended
    // in a host segmentation fault inside the graph launch once, with no
    // cause found in the kernel; until one is, batches do not use it.
    const mgr::PlainLoadVector plain;
    if (grouped) {
      // each stream runs its fields with grouped launches; the streams' small
      // latency-bound launches overlap each other's large ones
      std::vector<std::vector<mgr::BatchItem>> lanes;
      std::vector<void *> streams;
      for (int k = 0; k < MGR_BATCH_STREAMS && ok; ++k) {
        if (!used[k]) continue;
        std::vector<mgr::BatchItem> items;
        for (int i : order)
          if (lane[i] == k)
            items.push_back(mgr::BatchItem{jobs[i].plan.get(), fields[i].dtype == MGR_FLOAT64, fields[i].in,
                                           fields[i].out, ws ? (void *)((char *)ws + jobs[i].ws_off) : nullptr});
        lanes.push_back(std::move(items));
        streams.push_back((void *)bs->s[k]);
      }
      if (ok) ok = mgr::enqueue_batch(dec, lanes, streams, err);
    }
    for (int i : order) {
      if (!ok || grouped) break;
      const bool f64 = fields[i].dtype == MGR_FLOAT64;
      void *wsi = ws ? (void *)((char *)ws + jobs[i].ws_off) : nullptr;
      std::string e;
      const bool good = dec ? mgr::enqueue_decompose(*jobs[i].plan, f64, fields[i].in, fields[i].out, wsi,
                                                     bs->s[lane[i]], e)
                            : mgr::enqueue_recompose(*jobs[i].plan, f64, fields[i].in, fields[i].out, wsi,
                                                     bs->s[lane[i]], e);
      if (!good) {
        ok = false;
        err = field_tag(i) + e;
      }
    }
    // join every stream that may hold work back to the caller's stream, also
    // after a failure, so that later work on `stream` stays ordered
    for (int k = 0; k < MGR_BATCH_STREAMS; ++k) {
      if (!used[k]) continue;
      if (hipEventRecord(bs->join[k], bs->s[k]) != hipSuccess ||
          hipStreamWaitEvent(user, bs->join[k], 0) != hipSuccess) {
        const hipError_t e = hipGetLastError();
        if (ok) err = std::string("joining the batch streams: ") + hipGetErrorString(e);
        ok = false;
      }
    }
    if (!ok) return fail(MGR_ERR_DEVICE, err);
    return retain_for_capture(stream, plans);
  } catch (const std::bad_alloc &) {
    return fail(MGR_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(MGR_ERR_DEVICE, "unexpected internal failure");
  }
}

// ------------------------------------------------------------ no-allocation entry point

// Device scratch of mgr_decompose_noalloc: the plan tables of the last
// request in the first kNoAllocTableBytes, the workspace after them.  One
// copy per device, held until the process ends.  In host code `scratch`
// names a host-side stand-in: only its device address (noalloc_scratch) is
// ever passed to the GPU.
constexpr size_t kNoAllocTableBytes = (size_t)MGR_NOALLOC_TABLE_BYTES;
constexpr size_t kNoAllocBytes = (size_t)MGR_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

// Per device: the address of its copy of `scratch`, and the plan whose tables
// the scratch holds (stream order decides what a later call finds there).
struct NoAllocSlot {
  int device = -1;
  void *ptr = nullptr;
  std::unique_ptr<PlanKey> key;
  std::unique_ptr<mgr::Plan> plan;
  std::mutex mu;
};
std::mutex g_namu;
std::list<NoAllocSlot> g_noalloc;  // stable addresses

// The slot of the current device; on its first use the device address of
// `scratch` is looked up with that device current.
mgr_status noalloc_slot(NoAllocSlot *&out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MGR_ERR_DEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(g_namu);
  for (auto &s : g_noalloc)
    if (s.device == dev) {
      out = &s;
      return MGR_OK;
    }
  void *ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    (void)hipGetLastError();
    return fail(MGR_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  NoAllocSlot &s = g_noalloc.emplace_back();
  s.device = dev;
  s.ptr = ptr;
  out = &s;
  return MGR_OK;
}

mgr_status run_noalloc(int ndim, const int64_t *shape, const double *const *coords, int dtype, int nlevels,
                       const void *in, void *out, void *stream) {
  g_last_error.clear();
  try {
    int64_t n[mgr::kDims], nt = 1;
    std::string why;
    if (!split_shape(ndim, shape, n, nt, why)) return fail(MGR_ERR_INVALID_ARG, why);
    if (ndim == 4) return fail(MGR_ERR_UNSUPPORTED, "mgr_decompose_noalloc takes 1-D to 3-D fields");
    if (dtype != MGR_FLOAT32 && dtype != MGR_FLOAT64)
      return fail(MGR_ERR_INVALID_ARG, "dtype must be MGR_FLOAT32 or MGR_FLOAT64");
    const int ml = mgr::max_levels3(n);
    if (nlevels < 0 || nlevels > ml)
      return fail(MGR_ERR_INVALID_ARG, "nlevels must be in [0, " + std::to_string(ml) + "]");
    // the size limit comes first, before any device call
    const size_t need = mgr::workspace_bytes(n, nlevels, dtype == MGR_FLOAT64 ? 8 : 4);
    const size_t room = kNoAllocBytes - kNoAllocTableBytes;
    if (need > room)
      return fail(MGR_ERR_WORKSPACE, "request needs " + std::to_string(need) +
                                         " bytes of workspace; the static scratch of "
                                         "mgr_decompose_noalloc holds " + std::to_string(room));
    bool capturing = false;
    mgr_status s = capture_state(stream, capturing);
    if (s != MGR_OK) return s;
    if (capturing)
      return fail(MGR_ERR_UNSUPPORTED, "mgr_decompose_noalloc cannot be captured into a graph");
    NoAllocSlot *slot = nullptr;
    s = noalloc_slot(slot);
    if (s != MGR_OK) return s;
    char *ws = (char *)slot->ptr + kNoAllocTableBytes;
    std::vector<std::vector<double>> cx;
    s = validate(ndim, shape, coords, dtype, nlevels, in, out, ws, room, n, cx);
    if (s != MGR_OK) return s;
    std::lock_guard<std::mutex> lk(slot->mu);
    PlanKey key{slot->device, ndim, {n[0], n[1], n[2]}, 1, nlevels, cx};
    if (!slot->key || !(*slot->key == key)) {
      slot->key.reset();
      slot->plan.reset();
      const mgr::TableTarget tgt{slot->ptr, kNoAllocTableBytes, stream};
      std::string err;
      int st = 0;
      std::unique_ptr<mgr::Plan> p = mgr::build_plan(ndim, n, cx, nlevels, err, st, true, &tgt);
      if (!p) return fail((mgr_status)st, err);
      {
        std::lock_guard<std::mutex> gl(g_mu);
        if (auto t = g_tunes.find(TuneKey{slot->device, ndim, {n[0], n[1], n[2]}, 1, nlevels})) p->tune = *t;
      }
      slot->plan = std::move(p);
      slot->key = std::make_unique<PlanKey>(key);
    }
    mgr::TimingOff quiet;
    std::string err;
    if (!mgr::enqueue_decompose(*slot->plan, dtype == MGR_FLOAT64, in, out, ws, stream, err)) {
      slot->key.reset();  // the tables may not have arrived
      slot->plan.reset();
      return fail(MGR_ERR_DEVICE, err);
    }
    return MGR_OK;
  } catch (const std::bad_alloc &) {
    return fail(MGR_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(MGR_ERR_DEVICE, "unexpected internal failure");
  }
}

}  // namespace

namespace mgr {

mgr_status prepare_plan(int ndim, const int64_t *shape, const double *const *coords, int nlevels) {
  try {
    int64_t n[kDims], nt = 1;
    std::string why;
    if (!split_shape(ndim, shape, n, nt, why)) return fail(MGR_ERR_INVALID_ARG, why);
    const int ml = ndim == 4 ? max_levels4(nt, n) : max_levels3(n);
    if (nlevels < 0 || nlevels > ml || nlevels > kMaxLevels)
      return fail(MGR_ERR_INVALID_ARG, "nlevels must be in [0, " + std::to_string(ml) + "]");
    std::vector<std::vector<double>> cx;
    const mgr_status s = make_coords(ndim, n, nt, coords, cx);
    if (s != MGR_OK) return s;
    std::shared_ptr<Plan> plan;
    return get_plan(n, ndim, nlevels, cx, plan, nullptr, nt);
  } catch (const std::bad_alloc &) {
    return fail(MGR_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(MGR_ERR_DEVICE, "unexpected internal failure");
  }
}

void forget_helpers(const hipStream_t *callers, int n) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  std::lock_guard<std::mutex> lk(g_hmu);
  for (int q = 0; q < n; ++q)
    for (auto it = g_helpers.begin(); it != g_helpers.end(); ++it) {
      if (it->device != dev || it->caller != callers[q]) continue;
      {
        std::lock_guard<std::mutex> hl(it->mu);  // no enqueue of this caller in progress
        (void)hipStreamSynchronize(it->s);
        (void)hipEventDestroy(it->fork);
        (void)hipEventDestroy(it->join);
        (void)hipStreamDestroy(it->s);
      }
      g_helpers.erase(it);
      break;
    }
  (void)hipGetLastError();
}

}  // namespace mgr

extern "C" {

int mgr_max_levels(int ndim, const int64_t *shape) {
  int64_t n[mgr::kDims], nt = 1;
  std::string why;
  if (!split_shape(ndim, shape, n, nt, why)) {
    g_last_error = why;
    return -MGR_ERR_INVALID_ARG;
  }
  return ndim == 4 ? mgr::max_levels4(nt, n) : mgr::max_levels3(n);
}

mgr_status mgr_workspace_size(int ndim, const int64_t *shape, mgr_dtype dtype, int nlevels,
                              size_t *bytes) {
  g_last_error.clear();
  int64_t n[mgr::kDims], nt = 1;
  std::string why;
  if (!bytes) return fail(MGR_ERR_INVALID_ARG, "bytes is NULL");
  if (!split_shape(ndim, shape, n, nt, why)) return fail(MGR_ERR_INVALID_ARG, why);
  if (dtype != MGR_FLOAT32 && dtype != MGR_FLOAT64)
    return fail(MGR_ERR_INVALID_ARG, "dtype must be MGR_FLOAT32 or MGR_FLOAT64");
  const int ml = ndim == 4 ? mgr::max_levels4(nt, n) : mgr::max_levels3(n);
  if (nlevels < 0 || nlevels > ml)
    return fail(MGR_ERR_INVALID_ARG, "nlevels must be in [0, " + std::to_string(ml) + "]");
  const size_t es = dtype == MGR_FLOAT64 ? 8 : 4;
  *bytes = ndim == 4 ? mgr::workspace_bytes4(nt, n, nlevels, es) : mgr::workspace_bytes(n, nlevels, es);
  return MGR_OK;
}

mgr_status mgr_decompose(int ndim, const int64_t *shape, const double *const *coords,
                         mgr_dtype dtype, int nlevels, const void *in, void *out, void *workspace,
                         size_t workspace_bytes, void *stream) {
  return run(true, ndim, shape, coords, (int)dtype, nlevels, in, out, workspace, workspace_bytes,
             stream);
}

mgr_status mgr_recompose(int ndim, const int64_t *shape, const double *const *coords,
                         mgr_dtype dtype, int nlevels, const void *in, void *out, void *workspace,
                         size_t workspace_bytes, void *stream) {
  return run(false, ndim, shape, coords, (int)dtype, nlevels, in, out, workspace, workspace_bytes,
             stream);
}

mgr_status mgr_decompose_noalloc(int ndim, const int64_t *shape, const double *const *coords,
                                 mgr_dtype dtype, int nlevels, const void *in, void *out, void *stream) {
  return run_noalloc(ndim, shape, coords, (int)dtype, nlevels, in, out, stream);
}

mgr_status mgr_recompose_partial(int ndim, const int64_t *shape, const double *const *coords,
                                 mgr_dtype dtype, int nlevels, int nkeep, const void *in, void *out,
                                 void *workspace, size_t workspace_bytes, void *stream) {
  if (nkeep < 0 || nkeep > nlevels) {
    g_last_error = "nkeep must be in [0, nlevels]";
    return MGR_ERR_INVALID_ARG;
  }
  return run(false, ndim, shape, coords, (int)dtype, nlevels, in, out, workspace, workspace_bytes, stream,
             nkeep);
}

static mgr_status run_classes(bool export_, int ndim, const int64_t *shape, mgr_dtype dtype, int nlevels,
                              const void *in, void *out, void *stream) {
  g_last_error.clear();
  try {
    int64_t n[mgr::kDims];
    std::string why;
    if (!pad_shape(ndim, shape, n, why)) return fail(MGR_ERR_INVALID_ARG, why);
    if (dtype != MGR_FLOAT32 && dtype != MGR_FLOAT64)
      return fail(MGR_ERR_INVALID_ARG, "dtype must be MGR_FLOAT32 or MGR_FLOAT64");
    const int ml = mgr::max_levels3(n);
    if (nlevels < 0 || nlevels > ml)
      return fail(MGR_ERR_INVALID_ARG, "nlevels must be in [0, " + std::to_string(ml) + "]");
    if (!in || !out) return fail(MGR_ERR_INVALID_ARG, "in and out must be non-NULL device pointers");
    const size_t bytes = (size_t)(n[0] * n[1] * n[2]) * (dtype == MGR_FLOAT64 ? 8 : 4);
    if (overlaps(in, bytes, out, bytes)) return fail(MGR_ERR_INVALID_ARG, "in and out overlap");
    // the layout depends on the level structure only: the plan of uniform coordinates
    std::vector<std::vector<double>> cx(mgr::kDims);
    for (int k = 0; k < mgr::kDims; ++k) {
      cx[k].resize(n[k]);
      for (int64_t i = 0; i < n[k]; ++i) cx[k][i] = (double)i;
    }
    std::shared_ptr<mgr::Plan> plan;
    mgr_status s = get_plan(n, ndim, nlevels, cx, plan, stream);
    if (s != MGR_OK) return s;
    std::string err;
    if (!mgr::enqueue_classes(*plan, dtype == MGR_FLOAT64, export_, in, out, stream, err))
      return fail(MGR_ERR_DEVICE, err);
    return MGR_OK;
  } catch (const std::bad_alloc &) {
    return fail(MGR_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(MGR_ERR_DEVICE, "unexpected internal failure");
  }
}

mgr_status mgr_class_sizes(int ndim, const int64_t *shape, int nlevels, int64_t *sizes) {
  g_last_error.clear();
  int64_t n[mgr::kDims];
  std::string why;
  if (!pad_shape(ndim, shape, n, why)) return fail(MGR_ERR_INVALID_ARG, why);
  const int ml = mgr::max_levels3(n);
  if (nlevels < 0 || nlevels > ml)
    return fail(MGR_ERR_INVALID_ARG, "nlevels must be in [0, " + std::to_string(ml) + "]");
  if (!sizes) return fail(MGR_ERR_INVALID_ARG, "sizes is NULL");
  // node counts of the level grids: a dimension of m >= 3 nodes keeps m/2 + 1
  std::vector<int64_t> grid(nlevels + 1);
  int64_t m[mgr::kDims] = {n[0], n[1], n[2]};
  for (int s = 0; s <= nlevels; ++s) {
    grid[s] = m[0] * m[1] * m[2];
    for (int k = 0; k < mgr::kDims; ++k) m[k] = mgr::coarse_count(m[k]);
  }
  sizes[0] = grid[nlevels];
  for (int t = 0; t < nlevels; ++t) {
    const int s = nlevels - 1 - t;
    sizes[1 + t] = grid[s] - grid[s + 1];
  }
  return MGR_OK;
}

mgr_status mgr_export_classes(int ndim, const int64_t *shape, mgr_dtype dtype, int nlevels, const void *in,
                              void *out, void *stream) {
  return run_classes(true, ndim, shape, dtype, nlevels, in, out, stream);
}

mgr_status mgr_import_classes(int ndim, const int64_t *shape, mgr_dtype dtype, int nlevels, const void *in,
                              void *out, void *stream) {
  return run_classes(false, ndim, shape, dtype, nlevels, in, out, stream);
}

mgr_status mgr_autotune(int ndim, const int64_t *shape, const double *const *coords, mgr_dtype dtype,
                        int nlevels, const void *in, void *out, void *workspace, size_t workspace_bytes,
                        void *stream) {
  g_last_error.clear();
  try {
    int64_t n[mgr::kDims];
    std::vector<std::vector<double>> cx;
    if (ndim == 4) return fail(MGR_ERR_UNSUPPORTED, "autotuning of 4-D fields is not supported");
    mgr_status s = validate(ndim, shape, coords, (int)dtype, nlevels, in, out, workspace, workspace_bytes, n, cx);
    if (s != MGR_OK) return s;
    bool capturing = false;
    s = capture_state(stream, capturing);
    if (s != MGR_OK) return s;
    if (capturing) return fail(MGR_ERR_UNSUPPORTED, "mgr_autotune waits for its timed launches: not under stream capture");
    std::shared_ptr<mgr::Plan> plan;
    s = get_plan(n, ndim, nlevels, cx, plan, stream);
    if (s != MGR_OK) return s;
    std::string err, report;
    if (!mgr::enqueue_autotune(*plan, dtype == MGR_FLOAT64, in, out, workspace, stream, err, report))
      return fail(MGR_ERR_DEVICE, err);
    remember_tune(*plan, n, ndim, 1, nlevels);
    g_tune_report = report;
    return MGR_OK;
  } catch (const std::bad_alloc &) {
    return fail(MGR_ERR_OUT_OF_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(MGR_ERR_DEVICE, "unexpected internal failure");
  }
}

const char *mgr_autotune_report(void) { return g_tune_report.c_str(); }

mgr_status mgr_batch_workspace_size(int nfields, const mgr_field *fields, size_t *bytes) {
  g_last_error.clear();
  if (!bytes) return fail(MGR_ERR_INVALID_ARG, "bytes is NULL");
  try {
    std::vector<FieldJob> jobs;
    size_t total = 0;
    const mgr_status s = batch_layout(nfields, fields, jobs, total);
    if (s != MGR_OK) return s;
    *bytes = total;
    return MGR_OK;
  } catch (const std::bad_alloc &) {
    return fail(MGR_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
}

mgr_status mgr_decompose_batch(int nfields, const mgr_field *fields, void *workspace,
                               size_t workspace_bytes, void *stream) {
  return run_batch(true, nfields, fields, workspace, workspace_bytes, stream, 0);
}

mgr_status mgr_recompose_batch(int nfields, const mgr_field *fields, void *workspace,
                               size_t workspace_bytes, void *stream) {
  return run_batch(false, nfields, fields, workspace, workspace_bytes, stream, 0);
}

mgr_status mgr_decompose_batch_ex(int nfields, const mgr_field *fields, void *workspace,
                                  size_t workspace_bytes, void *stream, int flags) {
  if (flags & ~MGR_BATCH_PER_FIELD) {
    g_last_error = "unknown flags";
    return MGR_ERR_INVALID_ARG;
  }
  return run_batch(true, nfields, fields, workspace, workspace_bytes, stream, flags);
}

mgr_status mgr_recompose_batch_ex(int nfields, const mgr_field *fields, void *workspace,
                                  size_t workspace_bytes, void *stream, int flags) {
  if (flags & ~MGR_BATCH_PER_FIELD) {
    g_last_error = "unknown flags";
    return MGR_ERR_INVALID_ARG;
  }
  return run_batch(false, nfields, fields, workspace, workspace_bytes, stream, flags);
}

mgr_status mgr_probe_copy(const void *src, void *dst, size_t bytes, void *stream) {
  g_last_error.clear();
  if (!src || !dst) return fail(MGR_ERR_INVALID_ARG, "src and dst must be non-NULL");
  if (bytes % 16 != 0) return fail(MGR_ERR_INVALID_ARG, "bytes must be a multiple of 16");
  if ((uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0)
    return fail(MGR_ERR_INVALID_ARG, "src and dst must be 16-byte aligned");
  const char *a = (const char *)src, *b = (const char *)dst;
  if (a < b + bytes && b < a + bytes) return fail(MGR_ERR_INVALID_ARG, "src and dst overlap");
  std::string err;
  if (!mgr::enqueue_copy_probe(src, dst, bytes, stream, err)) return fail(MGR_ERR_DEVICE, err);
  return MGR_OK;
}

const char *mgr_status_string(mgr_status s) {
  switch (s) {
    case MGR_OK: return "ok";
    case MGR_ERR_INVALID_ARG: return "invalid argument";
    case MGR_ERR_UNSUPPORTED: return "unsupported request";
    case MGR_ERR_WORKSPACE: return "workspace missing or too small";
    case MGR_ERR_OUT_OF_MEMORY: return "out of memory";
    case MGR_ERR_DEVICE: return "device error";
  }
  return "unknown status";
}

const char *mgr_last_error(void) { return g_last_error.c_str(); }

void mgr_release_caches(void) {
  std::vector<std::shared_ptr<mgr::Plan>> dropped;  // released after the lock
  {
    std::lock_guard<std::mutex> lk(g_mu);
    g_cache.clear(dropped);
  }
  dropped.clear();
  g_deferred.drain();
}

}  // extern "C"
