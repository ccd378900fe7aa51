// mgr_plan.hpp -- host-side plan of one refactoring request: the level
// hierarchy and the FP64 tables every kernel reads (interpolation weights,
// load-vector taps, tridiagonal solve factors, nodal offsets).
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace mgr {

constexpr int kDims = 3;        // internal rank: leading dims of size 1 pad 1-D/2-D
constexpr int kTaps = 5;        // load-vector row: fine positions 2J-2 .. 2J+2
constexpr int kMaxBlocks = 16;  // partitions per line in the register solvers
constexpr int kLongBlocks = 128; // partitions of 64 per line in the long-line solver (its LDS: 64 KB)
constexpr int kMaxLevels = 62;

// Device pointers of the tables of one dimension at one level.
struct DimTabs {
  const int64_t *nodal = nullptr;  // [m] offset of level position i in the finest array
  const double *r = nullptr;       // [m] weight of the right coarse neighbour (fine i)
  const double *W = nullptr;       // [c*5] taps of row J of P^T M (fine 2J-2..2J+2)
  // coarse mass-matrix solve, over coarse positions [c]
  const double *sub = nullptr;     // a_i  (coupling to i-1)
  const double *sup = nullptr;     // e_i  (coupling to i+1)
  // Partition tables, [P*S] (padded past c).  Separator and padding slots
  // hold w = 0, supi = 0, invb = 1, Ls = Rs = 0, so a branch-free interior
  // solve over all S slots of a partition leaves them unchanged.
  const double *w = nullptr;       // block-local elimination factor
  const double *invb = nullptr;    // 1 / block-local pivot
  const double *supi = nullptr;    // e_i inside a block (0 at its last interior position)
  const double *Ls = nullptr;      // response of a block to its left separator
  const double *Rs = nullptr;      // response of a block to its right separator
  const double *sepa = nullptr;    // [P-1] a_s at the separators
  const double *sepe = nullptr;    // [P-1] e_s at the separators
  const double *wr = nullptr;      // [P-1] separator-system elimination factor
  const double *invbr = nullptr;   // [P-1] 1 / separator-system pivot
  const double *gam = nullptr;     // [P-1] separator-system upper coupling
  const double *tw = nullptr;      // [c] whole-line Thomas elimination factor
  const double *tinvb = nullptr;   // [c] whole-line Thomas 1 / pivot
  int S = 0;                       // partition length (0: sequential fallback)
  int P = 1;                       // partitions per line
};

struct Level {
  int64_t m[kDims];   // level-grid extent
  int64_t c[kDims];   // next-coarser extent (== m when not coarsened)
  bool co[kDims];     // coarsened at this step
  DimTabs d[kDims];
};

// Levels small enough to run entirely in one workgroup's LDS (k_tail_dec,
// k_tail_rec): at most kTailNodes nodes and kTailMaxExtent per dimension (the
// tail solves each line with one thread), with all their tables in at most
// kTailDoubles FP64 words and kTailOffsets nodal offsets.
constexpr int kTailNodes = 17 * 17 * 17;
constexpr int kTailMaxExtent = 65;
constexpr int kTailMaxLevels = 16;
constexpr int kTailDoubles = 3072;
constexpr int kTailOffsets = 1024;

// Descriptor of one tail level: extents and the word offsets of its tables
// in the packed tail tables (nodal: into the offset table; the rest: into the
// FP64 table).  Tables of a dimension that is not coarsened are absent except
// nodal and r (all zero).
struct TailLevel {
  int m[kDims], c[kDims], co[kDims];
  int nodal[kDims], r[kDims], W[kDims], sup[kDims], tw[kDims], tinvb[kDims];
};

// Launch shapes of one level chosen by the autotuner; 0 keeps the built-in
// rule.  None of them changes any node's arithmetic.
struct LevelTune {
  int lv_ti[2] = {0, 0};  // load-vector coarse planes per workgroup: decompose, recompose
  int rc_tj = 0, rc_tk = 0, rc_ti = 0;  // reconstruct tile (coarse rows, columns) and planes
};

struct Plan {
  int ndim = 0;                 // caller's rank
  int64_t n[kDims];             // finest shape, padded to rank 3
  int nlev = 0;
  std::vector<Level> lev;       // nlev + 1 entries; lev[nlev] has only nodal tables
  int device = -1;
  void *dev_tables = nullptr;   // one device allocation holding every table (owned)
  size_t table_bytes = 0;
  // A plan built into caller-provided device memory (see TableTarget) owns no
  // device allocation; it keeps the host image its tables were copied from.
  std::vector<char> host_image;
  int64_t max_coarse = 0;       // elements of the largest coarse grid (level 1)
  int tail_start = 0;           // first level run by the single-workgroup tail kernels
  const TailLevel *dev_tail = nullptr;  // [nlev - tail_start + 1], inside dev_tables
  const int64_t *dev_tail_off = nullptr;  // packed nodal offsets of the tail levels
  const double *dev_tail_dbl = nullptr;   // packed FP64 tables of the tail levels
  int tail_noff = 0, tail_ndbl = 0;
  // autotuned launch shapes per level (empty: none); written by the
  // autotuner, read as one snapshot per call
  mutable std::mutex tune_mu;
  std::vector<LevelTune> tune;
  std::vector<LevelTune> tune_snapshot() const {
    std::lock_guard<std::mutex> lk(tune_mu);
    return tune;
  }
  // Four-dimensional fields (Sec. III-D: time as one more tensor-product
  // dimension).  Dim 0 of the caller's shape is taken as time: this plan then
  // covers the three remaining dims (one time slice; no tail levels) and
  // `time` covers dim 0 as a (1, 1, nt) plan.  tpos[s][t] is the finest time
  // index of time position t of the level-s grid.
  std::unique_ptr<Plan> time;
  int64_t nt = 1;
  std::vector<std::vector<int64_t>> tpos;
  ~Plan();
};

// Coarse extent of a level grid with m nodes along a dimension.
inline int64_t coarse_count(int64_t m) { return m < 3 ? m : m / 2 + 1; }

int max_levels3(const int64_t n[kDims]);
// Levels of a 4-D grid (nt time positions, space extents n).
int max_levels4(int64_t nt, const int64_t n[kDims]);

// Device memory the caller provides for a plan's tables: `bytes` at `base`,
// filled by one asynchronous host-to-device copy on `stream`.
struct TableTarget {
  void *base;
  size_t bytes;
  void *stream;  // hipStream_t
};

// Builds tables on the host and uploads them to the current device: into one
// new device allocation (synchronous copy), or, with `target`, into the
// caller's memory (no allocation; status 3 if the tables do not fit).
// Returns nullptr and sets `err` on failure.  `allow_tail` false keeps every
// level on the general kernels.
std::unique_ptr<Plan> build_plan(int ndim, const int64_t n[kDims],
                                 const std::vector<std::vector<double>> &coords,
                                 int nlev, std::string &err, int &status, bool allow_tail = true,
                                 const TableTarget *target = nullptr);
// A 4-D plan: coords holds the time coordinates, then the three space dims'.
std::unique_ptr<Plan> build_plan4(int64_t nt, const int64_t n[kDims],
                                  const std::vector<std::vector<double>> &coords, int nlev,
                                  std::string &err, int &status);

// Three FP64 grids of level 1's size (two level grids, the load vector) and
// (nlev >= 2) one FP64 grid of level 2's size; the same for FP32 fields.
size_t workspace_bytes(const int64_t n[kDims], int nlev, size_t elem_size);
// 4-D: two FP64 coarse level grids, the FP64 load/correction grid and the FP64
// per-slice load vectors (nt slices of the coarse space grid).
size_t workspace_bytes4(int64_t nt, const int64_t n[kDims], int nlev, size_t elem_size);

}  // namespace mgr
