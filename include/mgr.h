/*
 * mgr.h -- C ABI of libmgr: multigrid hierarchical decomposition (refactor)
 * and recomposition of structured N-D floating-point fields on an AMD
 * MI355X (gfx950) GPU.
 *
 * Method: Chen et al., "Scalable Multigrid-based Hierarchical Scientific
 * Data Refactoring on GPUs" (arXiv 2105.12764), Sec. II-A.  One
 * decomposition step takes the level-l grid N_l to N_{l-1}:
 *   1. coefficients: every node of N_l \ N_{l-1} gets its value minus the
 *      multilinear interpolant from N_{l-1} (Sec. II-A.1);
 *   2. load vector f_{l-1} = R_l M_l vec(C_l), applied one dimension at a
 *      time (Sec. II-A.2, mass and transfer matrices of Sec. III-A.2);
 *   3. correction z_{l-1} = M_{l-1}^{-1} f_{l-1}, tridiagonal solves along
 *      each dimension (Sec. II-A.2, Thomas algorithm of Sec. III-A.3);
 *   4. the correction is added to the N_{l-1} nodes (Eq. 1).
 * Recomposition runs the steps in reverse, coarsest to finest (Sec. II-A,
 * "Overall decomposition/recomposition process").
 *
 * Conventions where the paper is silent:
 *   - arrays are C order (dimension 0 slowest, ndim-1 contiguous);
 *   - along a dimension with m >= 3 level nodes the next coarser grid keeps
 *     positions 0, 2, 4, ... and m-1; a dimension with m = 2 is no longer
 *     coarsened.  For m = 2^k + 1 this is the paper's dyadic hierarchy;
 *   - output layout is NODAL: same shape as the input; a node dropped at a
 *     level holds its coefficient, the final coarsest nodes hold the
 *     corrected coarse values Q u.  nlevels = 0 is a copy;
 *   - coordinates default to 0, 1, ..., n-1.
 *
 * Precision: MGR_FLOAT64 computes everything in FP64.  MGR_FLOAT32 keeps
 * the input and output in FP32 and splits as follows:
 *   - decomposition: coefficients, interpolation and the load vector are
 *     computed in FP64 (a coefficient is the difference of a value and its
 *     nearly equal interpolant), and the coarser level grids are kept in
 *     FP64 in the workspace; each stored value is rounded to FP32 once;
 *   - recomposition: the load vector of the stored coefficients and the
 *     interpolation are computed in FP32 (a coefficient is added to an
 *     interpolant, with no cancellation), the load vector is widened to
 *     FP64 for the solves, and the coarser level grids are FP32;
 *   - the tridiagonal correction solves and their workspace are FP64 in
 *     both directions.
 *
 * Plans and graph capture: the first call for a new (shape, coords,
 * nlevels) on a device builds FP64 tables on the host and uploads them (one
 * device allocation and one synchronous copy); the library caches the 1024
 * most recently used such plans.  A call made while its stream captures a
 * HIP graph needs its plan cached already (MGR_ERR_UNSUPPORTED otherwise:
 * make one call outside the capture first); the captured graph then holds
 * the plan, whose tables stay allocated until the graph and every
 * executable graph made from it are destroyed, even if the cache drops it.
 *
 * Threading: every entry point is thread-safe.  Calls are stream-ordered
 * and asynchronous: they return after enqueuing work on `stream`.
 */
#ifndef MGR_H
#define MGR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MGR_OK = 0,
  MGR_ERR_INVALID_ARG = 1,   /* bad ndim/shape/coords/nlevels/pointer/overlap */
  MGR_ERR_UNSUPPORTED = 2,   /* valid request the library does not handle */
  MGR_ERR_WORKSPACE = 3,     /* workspace NULL or smaller than required */
  MGR_ERR_OUT_OF_MEMORY = 4, /* plan tables could not be allocated */
  MGR_ERR_DEVICE = 5         /* a HIP call or kernel launch failed */
} mgr_status;

typedef enum { MGR_FLOAT32 = 0, MGR_FLOAT64 = 1 } mgr_dtype;

/* Largest valid level count for `shape`: the number of coarsening steps of
 * its deepest dimension (a dimension of m >= 3 nodes goes to m/2 + 1).
 * ndim in 1..4, every shape[k] >= 2.  Returns -MGR_ERR_INVALID_ARG on a bad
 * shape.  Host only, no GPU needed. */
int mgr_max_levels(int ndim, const int64_t *shape);

/* Bytes of device workspace that mgr_decompose / mgr_recompose need for this
 * request (0 when nlevels == 0): three FP64 grids of the level-1 shape (the
 * decomposition keeps its coarser level grids in FP64 also for FP32 fields)
 * and, with two or more levels, one FP64 grid of the level-2 shape (4-D:
 * three FP64 coarse 4-D grids and an FP64 coarse space grid per time step).
 * Host only, no GPU needed.
 * Returns MGR_ERR_INVALID_ARG for a bad shape, dtype or level count. */
mgr_status mgr_workspace_size(int ndim, const int64_t *shape, mgr_dtype dtype,
                              int nlevels, size_t *bytes);

/* Decompose `in` into its nodal multilevel representation `out`.
 *   ndim, shape : 1..4 dimensions, each >= 2 nodes, C order.  A 4-D shape
 *                 is (time, then three space dims): the decomposition in
 *                 four tensor-product dims of Sec. III-D, time coarsening
 *                 like space; the product of the three space dims must be
 *                 below 2^31.  4-D fields are taken by mgr_decompose,
 *                 mgr_recompose, mgr_workspace_size and mgr_max_levels;
 *                 the other entry points reject them.
 *   coords      : host pointer to ndim host arrays of shape[k] doubles,
 *                 strictly increasing and finite; coords == NULL or
 *                 coords[k] == NULL selects 0..shape[k]-1.  Read during the
 *                 call only (the library keeps its own tables).
 *   dtype       : element type of in and out.
 *   nlevels     : 0 .. mgr_max_levels(ndim, shape).
 *   in, out     : device pointers, prod(shape) elements each, caller-owned,
 *                 not overlapping.  `in` must stay unchanged until the
 *                 stream reaches this call's work.
 *   workspace   : device pointer, caller-owned, >= mgr_workspace_size bytes,
 *                 256-byte aligned; contents on entry are ignored.  Not
 *                 shared by calls that may run concurrently.
 *   stream      : hipStream_t to enqueue on (NULL = the null stream).
 * All argument checks happen before anything is enqueued; on any error
 * nothing is launched and `out` is untouched.  Plans are built and cached
 * as described above (see "Plans and graph capture"). */
mgr_status mgr_decompose(int ndim, const int64_t *shape,
                         const double *const *coords, mgr_dtype dtype,
                         int nlevels, const void *in, void *out,
                         void *workspace, size_t workspace_bytes,
                         void *stream);

/* Recompose the field from its nodal multilevel representation: the inverse
 * of mgr_decompose with the same shape, coords and nlevels.  Arguments,
 * ownership and errors as for mgr_decompose (here `in` is the
 * representation and `out` the field).  With two or more levels, the finest
 * level's load vector and first solves (which read only `in`) run on a
 * library-owned stream forked from `stream` after the work already on it and
 * joined back before the finest level's last kernels, so the call stays
 * ordered on `stream` and capturable in a HIP graph.  The helper stream of a
 * (device, stream) pair is created by its first call outside stream
 * capture; a captured call whose stream has none yet runs serially (same
 * results).  Helper streams are kept for at most 64 such pairs per process
 * (a service frees those of its streams when it is destroyed); calls from
 * further pairs, and 4-D fields, run serially on `stream`. */
mgr_status mgr_recompose(int ndim, const int64_t *shape,
                         const double *const *coords, mgr_dtype dtype,
                         int nlevels, const void *in, void *out,
                         void *workspace, size_t workspace_bytes,
                         void *stream);

/* Decomposition that allocates nothing, for callers that cannot allocate
 * device memory (tight serving loops, harnesses that forbid hipMalloc).
 * Same result as mgr_decompose with the same arguments, bit for bit; the
 * workspace and the plan tables live in a static device array of
 * MGR_NOALLOC_SCRATCH_BYTES per device (held from the first call on a device
 * until the process ends): the first MGR_NOALLOC_TABLE_BYTES hold the tables
 * of the last request, the rest its workspace.
 *   ndim        : 1..3 (4-D fields: MGR_ERR_UNSUPPORTED).
 *   others      : as for mgr_decompose; there is no workspace argument.
 * Errors: MGR_ERR_WORKSPACE, checked before any device call, when the
 * request's workspace (mgr_workspace_size) exceeds
 * MGR_NOALLOC_SCRATCH_BYTES - MGR_NOALLOC_TABLE_BYTES (e.g. 257^3 FP64 with
 * all levels fits, 513^3 does not), or when its plan tables exceed
 * MGR_NOALLOC_TABLE_BYTES; MGR_ERR_UNSUPPORTED when `stream` is capturing a
 * graph; otherwise as for mgr_decompose.
 * Behaviour: calls no device allocator.  A request whose shape, coords and
 * level count differ from the previous call's on the device rebuilds the
 * tables on the host and copies them into the scratch with one
 * hipMemcpyAsync on `stream` from pageable host memory; the same request
 * again copies nothing.  Every call on a device shares that device's
 * scratch and leaves its contents there: calls that may run at the same
 * time on one device (different streams, no ordering between them) race on
 * it and give wrong results.  Calls ordered on one stream are safe.
 * Per-kernel timing (mgr_timing_enable) does not record these launches. */
#define MGR_NOALLOC_SCRATCH_BYTES (64u << 20)
#define MGR_NOALLOC_TABLE_BYTES (4u << 20)
mgr_status mgr_decompose_noalloc(int ndim, const int64_t *shape,
                                 const double *const *coords, mgr_dtype dtype,
                                 int nlevels, const void *in, void *out,
                                 void *stream);

/* Progressive (partial) recomposition (Sec. II-A: the coarse representation
 * plus the first classes of coefficients give an approximation whose error
 * falls as classes are added).  Recomposes with only the `nkeep` coarsest
 * coefficient classes of the representation `in` -- the coarsest values
 * plus the coefficients of levels nlevels-1 down to nlevels-nkeep -- and the
 * finer classes taken as zero: exactly mgr_recompose of `in` with those
 * coefficients set to zero, without reading them.  The result has the full
 * shape: below the kept levels it is the multilinear interpolant.
 * nkeep in 0..nlevels (nkeep == nlevels is mgr_recompose; 0 interpolates the
 * coarsest values).  Other arguments, ownership and errors as for
 * mgr_recompose; nkeep out of range is MGR_ERR_INVALID_ARG. */
mgr_status mgr_recompose_partial(int ndim, const int64_t *shape,
                                 const double *const *coords, mgr_dtype dtype,
                                 int nlevels, int nkeep, const void *in, void *out,
                                 void *workspace, size_t workspace_bytes,
                                 void *stream);

/* Class-contiguous layout of a nodal representation (the paper's reordered
 * layout, Sec. III-C, used here as an exchange format for progressive
 * access): first the coarsest grid's values, then the coefficient class of
 * each level -- the level's nodes that are not in the next coarser grid --
 * from the coarsest level to the finest, each in C order of its level grid.
 * A prefix of the buffer that ends at a class boundary therefore holds the
 * coarse representation plus the coarsest classes; importing the prefix with
 * the rest zero and recomposing equals mgr_recompose_partial.
 * mgr_export_classes reorders the nodal array `in` into `out`;
 * mgr_import_classes is its inverse.  Both arrays hold prod(shape) elements
 * of dtype (device, caller-owned, not overlapping); no workspace.  Shape,
 * dtype and nlevels as for mgr_decompose (coordinates do not matter).
 * Stream-ordered; errors as for mgr_decompose. */
mgr_status mgr_export_classes(int ndim, const int64_t *shape, mgr_dtype dtype, int nlevels,
                              const void *in, void *out, void *stream);

/* Element counts of the class-contiguous layout's parts, in buffer order:
 * sizes[0] = the coarsest grid's nodes, sizes[1 + t] = the class of level
 * nlevels-1-t (coarsest class first); nlevels + 1 entries in all, written to
 * the caller's host array.  Host only.  MGR_ERR_INVALID_ARG for a bad shape
 * or level count or sizes == NULL. */
mgr_status mgr_class_sizes(int ndim, const int64_t *shape, int nlevels, int64_t *sizes);
mgr_status mgr_import_classes(int ndim, const int64_t *shape, mgr_dtype dtype, int nlevels,
                              const void *in, void *out, void *stream);

/* Static English name of a status code. */
const char *mgr_status_string(mgr_status s);

/* Detail of the calling thread's last failure ("" if none).  The pointer is
 * valid until the thread's next libmgr call. */
const char *mgr_last_error(void);

/* Drop every cached plan.  A plan's device tables are freed at once unless
 * a captured graph still holds the plan (they are freed after the graph and
 * its executables are destroyed).  The caller must make sure no enqueued
 * libmgr work outside captured graphs is still pending. */
void mgr_release_caches(void);

/* Autotune the launch shapes for this request (the paper's per-size tuning,
 * Sec. III-B): for every level the library ranks candidate shapes -- the
 * coarse planes each workgroup marches through and the reconstruction tile --
 * with a model of the 128-byte memory lines they touch and the rounds of
 * resident workgroups they need, times the three best on the GPU and keeps
 * the fastest in the plan it caches for (shape, coords, nlevels) on this
 * device.  Later mgr_decompose / mgr_recompose calls with that plan, and
 * batches containing it, use the tuned shapes.  Results are bitwise those of
 * the untuned calls: no shape changes any node's arithmetic.
 * Arguments as for mgr_decompose; `in` is only read (its values do not
 * matter), `out` and the workspace are overwritten with meaningless data.
 * Synchronous: returns after the timed launches on `stream` have finished;
 * MGR_ERR_UNSUPPORTED under stream capture.  The tuned shapes are also kept
 * per (device, shape, nlevels) beyond the plan's life in the cache: a plan
 * rebuilt later for the same shape starts with them. */
mgr_status mgr_autotune(int ndim, const int64_t *shape, const double *const *coords,
                        mgr_dtype dtype, int nlevels, const void *in, void *out,
                        void *workspace, size_t workspace_bytes, void *stream);

/* The calling thread's last mgr_autotune decisions, one line per choice
 * ("" if none).  Valid until the thread's next mgr_autotune call. */
const char *mgr_autotune_report(void);

/* ---- Batches of independent fields ----------------------------------------
 * Many fields of different shapes, level counts and dtypes refactored by one
 * call (the paper runs independent fields side by side, Sec. III-F; its
 * evaluation refactors many fields, Sec. IV-D).  Each field's result is
 * bitwise the result of mgr_decompose / mgr_recompose on that field alone. */

/* One field of a batch; the members mean what the same-named arguments of
 * mgr_decompose mean (shape: the first ndim entries are used). */
typedef struct mgr_field {
  int ndim;
  int64_t shape[3];
  const double *const *coords;
  mgr_dtype dtype;
  int nlevels;
  const void *in;
  void *out;
} mgr_field;

/* Number of internal streams a batch spreads its fields over. */
#define MGR_BATCH_STREAMS 4

/* Device workspace bytes for a batch: each field gets its own slice
 * (mgr_workspace_size of the field, rounded up to 256 bytes), in order.
 * Host only.  Returns the first invalid field's error (the detail names its
 * index); nfields must be >= 1 and fields non-NULL. */
mgr_status mgr_batch_workspace_size(int nfields, const mgr_field *fields, size_t *bytes);

/* Decompose every field of the batch.
 *   fields    : host array of nfields descriptors, read during the call.
 *   workspace : device pointer, >= mgr_batch_workspace_size bytes, 256-byte
 *               aligned, caller-owned; not overlapping any field's in or out.
 *   stream    : the call is ordered on `stream` like a single call.  The
 *               fields' launch chains are aligned by level (finest first in
 *               a decomposition, coarsest first in a recomposition), and for
 *               each step of a level the launches of one kernel across all
 *               fields go out as one grid over their workgroups (the jobs'
 *               arguments travel in the kernel arguments), in order on
 *               `stream`: a handful of launches per level for the whole
 *               batch instead of several per field and level (Sec. III-B/D:
 *               small grids batched into one launch).  The call can be
 *               captured into one HIP graph (plans must exist first: make
 *               one uncaptured call with the same fields before capturing,
 *               with at most 1024 distinct plans in the batch so that they
 *               all stay cached).  Results are bitwise those of the
 *               single-field calls.
 * Besides every check of mgr_decompose per field (the detail names the
 * field), no field's out may overlap another field's in or out.  All checks
 * happen before anything is enqueued; on error nothing is launched. */
mgr_status mgr_decompose_batch(int nfields, const mgr_field *fields, void *workspace,
                               size_t workspace_bytes, void *stream);

/* Recompose every field of the batch (each field's `in` is its nodal
 * representation, `out` the field).  As mgr_decompose_batch otherwise. */
mgr_status mgr_recompose_batch(int nfields, const mgr_field *fields, void *workspace,
                               size_t workspace_bytes, void *stream);

/* The batched calls with flags: 0 is mgr_decompose_batch /
 * mgr_recompose_batch; MGR_BATCH_PER_FIELD runs each field's own launch chain
 * instead, the chains spread over MGR_BATCH_STREAMS internal streams (default
 * priority) forked from `stream` and joined back with events (also
 * capturable; bitwise the same results).  Other bits: MGR_ERR_INVALID_ARG. */
#define MGR_BATCH_PER_FIELD 1
mgr_status mgr_decompose_batch_ex(int nfields, const mgr_field *fields, void *workspace,
                                  size_t workspace_bytes, void *stream, int flags);
mgr_status mgr_recompose_batch_ex(int nfields, const mgr_field *fields, void *workspace,
                                  size_t workspace_bytes, void *stream, int flags);

/* ---- Refactoring service ----------------------------------------------------
 * A stream of independent decompose / recompose requests on caller-owned
 * device buffers, admitted first-in first-out by HBM footprint: a request
 * starts only while the in-flight footprint -- input + output + workspace
 * bytes of every admitted, unfinished request -- stays within the budget.
 * Workspace comes from an arena allocated at creation (4/5 of the budget
 * plus 1 MiB, at most the budget: a request's workspace is below 0.77 of its
 * footprint plus 1 KiB, so any request within the budget fits it), so
 * requests allocate nothing.  A request's plan is built by the submitting
 * thread, before it takes the service's lock.  The operations
 * are those of mgr_decompose / mgr_recompose; the service is the stream of
 * many independent fields refactored inside workflows (Sec. V)
 * with admission by memory footprint.  Admitted requests run on
 * `nstreams` internal streams (default priority), least-loaded first; one
 * host thread per stream retires them in order.  All calls on one service
 * from the device current at creation.  Thread-safe. */
typedef struct mgr_service mgr_service;

/* Create a service on the current device.  budget_bytes >= 4096;
 * nstreams in 1..16.  MGR_ERR_OUT_OF_MEMORY if the arena cannot be
 * allocated, MGR_ERR_DEVICE without a usable device. */
mgr_status mgr_service_create(size_t budget_bytes, int nstreams, mgr_service **svc);

/* Submit one request (recompose != 0: recomposition).  Arguments as for
 * mgr_decompose minus the workspace and stream (1..4 dims); coordinates are
 * copied.
 * `in` must stay unchanged and `out` unused by the caller until the request
 * is done.  Returns after finding or building the request's plan, with a
 * ticket (1, 2, ...); the request waits if it does not fit yet.
 * MGR_ERR_UNSUPPORTED for a request whose footprint exceeds the budget;
 * argument errors as for mgr_decompose are reported by mgr_service_result. */
mgr_status mgr_service_submit(mgr_service *svc, int recompose, int ndim, const int64_t *shape,
                              const double *const *coords, mgr_dtype dtype, int nlevels,
                              const void *in, void *out, uint64_t *ticket);

/* Block until every submitted request is done. */
mgr_status mgr_service_wait_all(mgr_service *svc);

/* State of a request: done (0/1), its status, milliseconds from submission
 * to being enqueued (queue_ms; -1 while waiting) and to completion as seen
 * by the service (latency_ms; -1 until done).  Any output pointer may be
 * NULL.  MGR_ERR_INVALID_ARG for an unknown ticket. */
mgr_status mgr_service_result(mgr_service *svc, uint64_t ticket, int *done, mgr_status *status,
                              double *queue_ms, double *latency_ms);

/* Wait for every request, stop the threads and free the arena and streams
 * (with the recomposition helper streams the library made for them).
 * (Each request's record -- status and times, about a hundred bytes of host
 * memory -- is kept until then, so that mgr_service_result answers for every
 * ticket.) */
mgr_status mgr_service_destroy(mgr_service *svc);

/* Detail of the calling thread's last service failure ("" if none). */
const char *mgr_service_last_error(void);

/* ---- Instrumentation (benchmarking only; not part of the method) --------
 * While enabled, every kernel launch of later calls is bracketed by a pair of
 * HIP events recorded on the launch's own stream, and its algorithmic
 * traffic (the bytes the method must move for that launch: each input read
 * once, each output written once) is accumulated per kernel name.  Intended
 * for one thread driving the library. */

/* Streaming copy probe: copies `bytes` bytes (a multiple of 16) from device
 * buffer src to device buffer dst with one read and one write of every
 * byte and no arithmetic -- the "achievable single-pass" bandwidth probe the
 * paper divides by to place its throughput (Sec. IV-D), and a kernel of known
 * traffic for calibrating hardware byte counters.  Buffers must not
 * overlap; MGR_ERR_INVALID_ARG otherwise.  At most 64 GiB (one launch);
 * MGR_ERR_DEVICE beyond.  Enqueued on `stream`. */
mgr_status mgr_probe_copy(const void *src, void *dst, size_t bytes, void *stream);

/* Turn event recording on (on != 0) or off.  Always MGR_OK. */
mgr_status mgr_timing_enable(int on);

/* Wait for the recorded events and drop all totals. */
void mgr_timing_reset(void);

/* Wait for the recorded events; number of distinct kernels with totals. */
int mgr_timing_count(void);

/* Totals of kernel `index` (0 .. mgr_timing_count()-1): its name (static
 * until the next reset), launches, summed event time in milliseconds and
 * summed algorithmic bytes.  Any output pointer may be NULL.  Returns
 * MGR_ERR_INVALID_ARG for an index out of range. */
mgr_status mgr_timing_get(int index, const char **name, int64_t *launches,
                          double *total_ms, double *alg_bytes);

#ifdef __cplusplus
}
#endif

#endif /* MGR_H */
