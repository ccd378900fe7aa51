// mgr_plan.hpp -- host-side plan of one refactoring request: the level
// hierarchy and the FP64 tables every kernel reads (interpolation weights,
// load-vector taps, tridiagonal solve factors, nodal offsets).
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

namespace mgr {

constexpr int kDims = 3;        // internal rank: leading dims of size 1 pad 1-D/2-D
constexpr int kTaps = 5;        // load-vector row: fine positions 2J-2 .. 2J+2
constexpr int kMaxBlocks = 16;  // partitions per line in the register solvers
constexpr int kMaxLevels = 62;

// Device pointers of the tables of one dimension at one level.
struct DimTabs {
  const int64_t *nodal = nullptr;  // [m] offset of level position i in the finest array
  const double *r = nullptr;       // [m] weight of the right coarse neighbour (fine i)
  const double *W = nullptr;       // [c*5] taps of row J of P^T M (fine 2J-2..2J+2)
  // coarse mass-matrix solve, over coarse positions [c]
  const double *sub = nullptr;     // a_i  (coupling to i-1)
  const double *sup = nullptr;     // e_i  (coupling to i+1)
  const double *w = nullptr;       // block-local elimination factor
  const double *invb = nullptr;    // 1 / block-local pivot
  const double *Ls = nullptr;      // response of a block to its left separator
  const double *Rs = nullptr;      // response of a block to its right separator
  const double *wr = nullptr;      // [P-1] separator-system elimination factor
  const double *invbr = nullptr;   // [P-1] 1 / separator-system pivot
  const double *gam = nullptr;     // [P-1] separator-system upper coupling
  int S = 0;                       // partition length (0: sequential fallback)
  int P = 1;                       // partitions per line
};

struct Level {
  int64_t m[kDims];   // level-grid extent
  int64_t c[kDims];   // next-coarser extent (== m when not coarsened)
  bool co[kDims];     // coarsened at this step
  DimTabs d[kDims];
};

struct Plan {
  int ndim = 0;                 // caller's rank
  int64_t n[kDims];             // finest shape, padded to rank 3
  int nlev = 0;
  std::vector<Level> lev;       // nlev + 1 entries; lev[nlev] has only nodal tables
  int device = -1;
  void *dev_tables = nullptr;   // one device allocation holding every table
  size_t table_bytes = 0;
  int64_t max_coarse = 0;       // elements of the largest coarse grid (level 1)
  ~Plan();
};

// Coarse extent of a level grid with m nodes along a dimension.
inline int64_t coarse_count(int64_t m) { return m < 3 ? m : m / 2 + 1; }

int max_levels3(const int64_t n[kDims]);

// Builds tables on the host and uploads them to the current device.
// Returns nullptr and sets `err` on failure.
std::unique_ptr<Plan> build_plan(int ndim, const int64_t n[kDims],
                                 const std::vector<std::vector<double>> &coords,
                                 int nlev, std::string &err, int &status);

size_t workspace_bytes(const int64_t n[kDims], int nlev, size_t elem_size);

}  // namespace mgr
