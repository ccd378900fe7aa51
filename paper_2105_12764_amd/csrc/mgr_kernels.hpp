// mgr_kernels.hpp -- enqueue entry points of the HIP kernels (host side).
#pragma once

#include <string>
#include <vector>

#include "mgr_plan.hpp"

namespace mgr {

// Enqueue one full decomposition / recomposition of `pl` on `stream`.
// Arguments are assumed validated.  Returns false with `err` set when a
// launch fails.
bool enqueue_decompose(const Plan &pl, bool f64, const void *in, void *out, void *ws, void *stream,
                       std::string &err);
bool enqueue_copy_probe(const void *src, void *dst, size_t bytes, void *stream, std::string &err);
// A helper stream and two events for work that a call may run beside its
// own stream (forked after everything already on the stream, joined back
// before the work that needs it).
struct StreamFork {
  void *helper;  // hipStream_t
  void *fork;    // hipEvent_t
  void *join;    // hipEvent_t
};

// nkeep: coefficient classes used, coarsest first (< 0: all).  With `fk`, the
// finest level's load vector and all but its last solve run on the helper
// stream while the coarser levels recompose (same arithmetic, same results).
bool enqueue_recompose(const Plan &pl, bool f64, const void *in, void *out, void *ws, void *stream,
                       std::string &err, int nkeep = -1, const StreamFork *fk = nullptr);

// While one lives on a thread, launches from that thread use the
// register-prefetch load-vector kernel on every level (the batched entry
// points take it; results are bitwise those of the ring kernel).
class PlainLoadVector {
 public:
  PlainLoadVector();
  ~PlainLoadVector();
  PlainLoadVector(const PlainLoadVector &) = delete;
  PlainLoadVector &operator=(const PlainLoadVector &) = delete;
};

// One field of a batch: its plan, type and device buffers (workspace of the
// single-field size).
struct BatchItem {
  const Plan *pl;
  bool f64;
  const void *in;
  void *out;
  void *ws;
};

// Decompose (recompose) every field of a batch with grouped launches, lane
// k's fields on streams[k]: the fields' launch chains are recorded, and for
// each step of the level loop (aligned by level index, finest = 0) the
// launches of one kernel across a lane's fields go out as one grid over their
// blocks, in order on the lane's stream; the lanes' launches are issued
// interleaved.  Same kernels and arithmetic as the single-field calls
// (bitwise the same results).  Fields must have 1 to 3 dims.
bool enqueue_batch(bool dec, const std::vector<std::vector<BatchItem>> &lanes, const std::vector<void *> &streams,
                   std::string &err);

// Reorder a nodal representation into class-contiguous order (export) or
// back (import); src and dst hold prod(shape) elements each.
bool enqueue_classes(const Plan &pl, bool f64, bool export_, const void *src, void *dst, void *stream,
                     std::string &err);

// Tune the plan's launch shapes on `stream` (synchronous: waits for the
// timed launches) and store them in the plan.  Reads `in`; overwrites `out`
// and `ws`.  `report` gets one line per decision.
bool enqueue_autotune(Plan &pl, bool f64, const void *in, void *out, void *ws, void *stream, std::string &err,
                      std::string &report);

}  // namespace mgr
