// mgr_kernels.hip -- CDNA4 (gfx950) kernels of the multigrid refactoring
// hot path and the host code that enqueues one decomposition or
// recomposition (arXiv 2105.12764, Sec. II-A; kernel roles of Sec. III-A).
//
// One step l -> l-1 of the decomposition is three launches:
//   k_loadvec   reads the level grid once.  Per plane along dimension 0 it
//               stages a (rows x columns) tile with a two-node halo in LDS,
//               forms the coefficients (value minus the multilinear
//               interpolant, Sec. II-A.1), writes them to their nodal
//               positions, keeps the coarse values compactly (the paper's
//               reordered layout, Sec. III-C) and applies the load-vector
//               operator P^T M along dimensions 2 and 1 in LDS.  Along
//               dimension 0 it keeps a five-plane ring and emits each coarse
//               plane of f = R M C as soon as its taps are complete.  This
//               fuses the paper's coefficient and mass-transfer kernels
//               (GPK, LPK) into one pass over the data.
//   k_solve_*   the correction solves M_{l-1} z = f along each coarsened
//               dimension (Sec. II-A.2; IPK role).  Each line is held in
//               registers, cut into partitions solved independently plus a
//               small separator system (exact, see mgr_plan.cpp), so every
//               solve reads and writes the coarse grid once.  Strided
//               dimensions put 64 adjacent lines on the 64 lanes of a wave
//               (coalesced); the contiguous dimension stages rows through LDS.
//               The last solve of a step applies the correction in its store
//               (coarse <- coarse + z), so no separate pass adds it.
// Recomposition runs the same load-vector and solve kernels on the stored
// coefficients, subtracts z, and k_reconstruct adds the interpolant back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "mgr_kernels.hpp"
#include "mgr_plan.hpp"
#include "mgr_timing.hpp"

namespace mgr {

namespace {

// ------------------------------------------------------------ addressing

// Offset of level node (i, j, k) in an array: per-dimension offset tables
// (nodal positions in the finest array) or plain strides (compact grids).
struct Map3 {
  const int64_t *t0, *t1, *t2;
  int64_t s0, s1;
};

__host__ Map3 compact_map(int64_t m1, int64_t m2) { return Map3{nullptr, nullptr, nullptr, m1 * m2, m2}; }
__host__ Map3 nodal_map(const Level &L) { return Map3{L.d[0].nodal, L.d[1].nodal, L.d[2].nodal, 0, 0}; }

__device__ __forceinline__ int64_t moff(const Map3 &m, int64_t i, int64_t j, int64_t k) {
  return m.t0 ? (m.t0[i] + m.t1[j] + m.t2[k]) : (i * m.s0 + j * m.s1 + k);
}

// Linear interpolation between a (left) and b (right) with the weight r of
// the right node, in the paper's FMA form (Sec. III-E, Table III).
__device__ __forceinline__ double lerp(double a, double b, double r) { return fma(r, b, fma(-r, a, a)); }
__device__ __forceinline__ float lerp(float a, float b, float r) { return fmaf(r, b, fmaf(-r, a, a)); }

// Arithmetic type of the recomposition's stencils: the field's own type (a
// recomposition adds a coefficient to an interpolant, with no cancellation).
// The decomposition always computes in FP64 (see k_loadvec), the correction
// solves too, and the load vector handed to them is FP64.
template <typename T>
using Acc = T;

template <bool CO>
__device__ __forceinline__ bool coarse_pos(int64_t g, int64_t m) {
  return !CO || (g % 2 == 0) || (g == m - 1);
}
template <bool CO>
__device__ __forceinline__ int64_t coarse_idx(int64_t g, int64_t m, int64_t c) {
  return !CO ? g : (g == m - 1 ? c - 1 : g / 2);
}

// ------------------------------------------------------- load-vector kernel

// Coarse rows (dim 1) per tile (each measured at 513^3).  FP32 fields: 8;
// their kernels wait on latency more than on bandwidth and gain more from a
// third resident workgroup per CU (256 threads each) than a taller tile
// saves in halo rows.  FP64 fields: 24 for the finest level's decomposition
// (768 threads, three waves per SIMD at its register count, fewer halo rows),
// 16 for the finest level's recomposition and the nodal levels'
// decomposition (the taller tile is slower there), 8 for the nodal levels'
// recomposition, whose kernels run beside the finest level's on the helper
// stream: twice the workgroups, each half the size, find free slots sooner
// (FP64 recomposition 1.298 -> 1.281 ms; 8 rows slowed the other two).
template <typename T, bool DEC, bool NODAL>
constexpr int kTJ = sizeof(T) == 4 ? 8 : (DEC ? (NODAL ? 16 : 24) : (NODAL ? 8 : 16));
constexpr int TK = 32;  // coarse columns (dim 2) per tile
template <typename T, bool DEC, bool NODAL>
constexpr int kNTHR = kTJ<T, DEC, NODAL> * TK;
// kTJ for a choice made at run time
template <typename T>
int tile_rows(bool dec, bool nodal) {
  return dec ? (nodal ? kTJ<T, true, true> : kTJ<T, true, false>)
             : (nodal ? kTJ<T, false, true> : kTJ<T, false, false>);
}
#define LV_WAVES (DEC ? (sizeof(TS) == 4 ? 4 : 1) : 5)
#define LV_MAXP 128

template <typename T, typename TS = T>
struct LoadArgs {
  const TS *src;  // level grid: field values (decompose) or stored coefficients (recompose)
  Map3 smap;
  T *out;         // decompose: coefficient destination (nodal positions)
  Map3 omap;
  double *F;      // load vector, compact next-level grid (FP64)
  int64_t m0, m1, m2, c0, c1, c2;
  const double *r0, *r1, *r2;
  const double *W0, *W1, *W2;
  int64_t TI;     // coarse planes per workgroup along dim 0
  int gx, gy, gz; // tile grid (dims 2, 1, 0)
  // Time slices of a 4-D level (k_tfine covers the rest of their nodes):
  // decompose with out == nullptr forms the load vector only; recompose with
  // keep_coarse stages the nodes coarse in space too, for a slice all of
  // whose nodes hold coefficients.
  int keep_coarse;
};

// Tile id of this workgroup.  Hardware hands consecutive workgroup ids to
// the 8 XCDs in turn; this mapping gives each XCD one contiguous run of
// tiles so that neighbouring tiles, which share halo rows, share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
  const int q = nb / 8, r = nb % 8;
  const int xcd = bid % 8, local = bid / 8;
  return (xcd < r ? xcd * (q + 1) : r * (q + 1) + (xcd - r) * q) + local;
}

// ------------------------------------------------------------ grouped launches

// Up to N independent jobs of one kernel in a single launch (the batched
// entry points): the jobs' argument structs travel in the kernel arguments,
// and job i takes blocks [start[i], start[i+1]) of the grid.
constexpr int kGroupArgBytes = 3584;  // budget for the jobs' arguments (kernel arguments stay below 4 KB)
template <typename J>
struct Group {
  static constexpr int N = (kGroupArgBytes - 8) / (int)(sizeof(J) + 4) > 0 ? (kGroupArgBytes - 8) / (int)(sizeof(J) + 4) : 1;
  J job[N];
  int start[N + 1];
  int njobs;
};

// Job and block of this workgroup within a group: blocks are numbered so that
// each XCD walks a contiguous run (xcd_tile), then located by the prefix sums.
template <typename J>
__device__ __forceinline__ void group_locate(const Group<J> &g, int &j, int &b) {
  const int t = xcd_tile(blockIdx.x, g.start[g.njobs]);
  j = 0;
  while (j + 1 < g.njobs && g.start[j + 1] <= t) ++j;
  b = t - g.start[j];
}

// One workgroup owns a (TJ x TK) tile of the coarse grid in dims (1, 2) and
// a chunk of TI coarse planes along dim 0.  It walks the fine planes in
// steps of two -- fine plane a = 2I+1 and coarse plane b = 2I+2 -- with the
// next step's values prefetched into registers while the current step
// computes.  Per step, from the staged values U of both planes:
//   * P^T M along dims 2 and 1 (LDS), then along dim 0 from a five-plane
//     register window: f = (P^T M)^{(x)3} U.  By the Galerkin identity
//     P^T M_l P = M_{l-1}, solving M_{l-1} z' = f gives z' = U_c + z, the
//     corrected coarse values, so the load vector is formed from the values
//     and the coefficient computation stays off its critical path;
//   * (decompose) the coefficients U - Pi U_c of both planes, written to
//     their nodal positions: Pi of plane b is its bilinear interpolant
//     (dims 1, 2) from up to four staged neighbours, Pi of plane a the dim-0
//     lerp of the interpolants of the coarse planes on either side.
// Recomposition stages the stored coefficients (zero at the coarse nodes)
// and forms f = (P^T M)^{(x)3} C the same way.
template <typename T, typename TS, bool DEC, bool NODAL, bool CO0, bool CO1, bool CO2>
__device__ __forceinline__ void loadvec_body(const LoadArgs<T, TS> &a, const int tile) {
  // a decomposition forms its coefficients as differences of nearly equal
  // values, so it computes in FP64 whatever the storage type
  using A = std::conditional_t<DEC, double, Acc<T>>;
  // staged planes hold the loaded values, exact in the source type
  using P = TS;
  constexpr int TJ = kTJ<T, DEC, NODAL>, NTHR = kNTHR<T, DEC, NODAL>;
  constexpr int SJ = CO1 ? 2 : 1, HJ = CO1 ? 2 : 0;
  constexpr int SK = CO2 ? 2 : 1, HK = CO2 ? 2 : 0;
  constexpr int NJ = SJ * (TJ - 1) + 1 + 2 * HJ;
  constexpr int NK = SK * (TK - 1) + 1 + 2 * HK;
  constexpr int NE = NJ * NK;
  constexpr int EPT = (NE + NTHR - 1) / NTHR;  // tile elements per thread
  static_assert(EPT <= 8, "the per-thread flags hold 4 bits for each of at most 8 tile elements");
  constexpr int NG = NJ * TK;                  // dim-2 reduced rows of one plane
  __shared__ P sA[NE];      // plane b (coarse along dim 0)
  __shared__ P sB[NE];      // plane a (fine along dim 0)
  __shared__ A sG[2 * NG];  // dim-2 reduced rows of b, then of a
  __shared__ A sR1[DEC ? NJ : 1], sR2[DEC ? NK : 1];  // interpolation weights of rows / columns
  // Tables read inside the plane loop are staged in LDS (or loaded one step
  // ahead with the prefetch): a vector-memory read of a table there would
  // make the compiler wait for the in-flight prefetch loads.
  __shared__ int64_t sPO[NODAL ? LV_MAXP : 1];  // nodal plane offsets of the window
  __shared__ A sStep[2][6];                // per-step dim-0 taps and weight

  const int tid = threadIdx.x;
  const int tx = tile % a.gx, ty = (tile / a.gx) % a.gy, tz = tile / (a.gx * a.gy);
  const int64_t J0 = (int64_t)ty * TJ, K0 = (int64_t)tx * TK;
  const int64_t I0 = (int64_t)tz * a.TI;
  const int64_t I1 = min(I0 + a.TI, a.c0);
  const int64_t fj0 = SJ * J0 - HJ, fk0 = SK * K0 - HK;
  const bool lastJ = J0 + TJ >= a.c1, lastK = K0 + TK >= a.c2, lastI = I1 >= a.c0;
  const int64_t ojb = SJ * J0, oje = lastJ ? a.m1 : SJ * (J0 + TJ);
  const int64_t okb = SK * K0, oke = lastK ? a.m2 : SK * (K0 + TK);
  const int64_t oib = (CO0 ? 2 : 1) * I0;
  const int64_t oie = (DEC && a.out == nullptr) ? oib : (lastI ? a.m0 : (CO0 ? 2 : 1) * I1);

  // per-element constants of this thread's tile elements (same for every plane)
  enum : unsigned { F_IN = 1, F_OWN = 2, F_C1 = 4, F_C2 = 8 };
  unsigned flags = 0;                    // 4 bits per element
  int colS[EPT], colO[NODAL ? EPT : 1];  // in-plane offsets (planes hold < 2^31 nodes)
  colO[0] = 0;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NTHR;
    const int j = e / NK, k = e % NK;
    const int64_t gj = fj0 + j, gk = fk0 + k;
    unsigned f = 0;
    colS[i] = 0;
    if (NODAL) colO[NODAL ? i : 0] = 0;
    if (e < NE && gj >= 0 && gj < a.m1 && gk >= 0 && gk < a.m2) {
      f |= F_IN;
      if (gj >= ojb && gj < oje && gk >= okb && gk < oke) f |= F_OWN;
      if (coarse_pos<CO1>(gj, a.m1)) f |= F_C1;
      if (coarse_pos<CO2>(gk, a.m2)) f |= F_C2;
      colS[i] = (int)(a.smap.t1 ? a.smap.t1[gj] + a.smap.t2[gk] : gj * a.smap.s1 + gk);
      if (DEC && NODAL) colO[NODAL ? i : 0] = (int)(a.omap.t1[gj] + a.omap.t2[gk]);
    }
    flags |= f << (4 * i);
  }
  auto flag_of = [&](int i) -> unsigned { return (flags >> (4 * i)) & 15u; };

  // the (J, K) load-vector entry this thread reduces and emits
  const int hJ = tid / TK, hK = tid % TK;
  const int64_t gJ = J0 + hJ, gK = K0 + hK;
  const bool hOK = gJ < a.c1 && gK < a.c2;
  if (DEC) {
    for (int j = tid; j < NJ; j += NTHR) {
      const int64_t gj = fj0 + j;
      sR1[j] = (CO1 && gj >= 0 && gj < a.m1 && !coarse_pos<CO1>(gj, a.m1)) ? a.r1[gj] : A(0);
    }
    for (int k = tid; k < NK; k += NTHR) {
      const int64_t gk = fk0 + k;
      sR2[k] = (CO2 && gk >= 0 && gk < a.m2 && !coarse_pos<CO2>(gk, a.m2)) ? a.r2[gk] : A(0);
    }
  }

  // plane window [pw0, pw0 + LV_MAXP) of this workgroup (host keeps 2 TI + 3 <= LV_MAXP)
  const int64_t pw0 = CO0 ? max<int64_t>(0, 2 * I0 - 2) : I0;
  if (NODAL) {
    const int64_t *t0 = DEC ? a.omap.t0 : a.smap.t0;
    for (int q = tid; q < LV_MAXP; q += NTHR) sPO[q] = (pw0 + q < a.m0) ? t0[pw0 + q] : 0;
  }
  // plane offsets: the field-side array of a coarser level goes through the nodal tables
  auto src_plane = [&](int64_t p) -> int64_t { return (!DEC && NODAL) ? sPO[p - pw0] : p * a.smap.s0; };
  auto out_plane = [&](int64_t p) -> int64_t { return (DEC && NODAL) ? sPO[p - pw0] : p * a.omap.s0; };

  // loads of one plane into registers.  Branch-free, so that all of them
  // are in flight together: elements outside the grid read the plane's first
  // node (colS = 0) and are masked when staged.
  auto fetch = [&](P (&v)[EPT], int64_t p) {
    const TS *base = a.src + src_plane(p);
#pragma unroll
    for (int i = 0; i < EPT; ++i) v[i] = base[colS[i]];
  };
  // stage a plane into LDS: zero outside the grid and, for recomposition of a
  // plane coarse along dim 0, at the stored coarse values (not coefficients)
  auto stage = [&](P *s, const P (&v)[EPT], bool zero_coarse) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int e = tid + i * NTHR;
      const unsigned f = flag_of(i);
      const bool keep = (f & F_IN) && !(zero_coarse && (f & F_C1) && (f & F_C2));
      if (e < NE) s[e] = keep ? v[i] : P(0);
    }
  };

  // bilinear interpolant (dims 1, 2) at tile element e of the staged plane s,
  // branch-free: along a dimension where the node is coarse both neighbours
  // are the node itself and the weight is 0 (the weight tables hold 0 there)
  auto interp2 = [&](const P *s, int e, unsigned f) -> A {
    if (!(f & F_IN)) return A(0);
    const int dk = (f & F_C2) ? 0 : 1, dj = (f & F_C1) ? 0 : NK;
    const A rk = sR2[e % NK], rj = sR1[e / NK];
    return lerp(lerp((A)s[e - dj - dk], (A)s[e - dj + dk], rk), lerp((A)s[e + dj - dk], (A)s[e + dj + dk], rk),
                rj);
  };

  // P^T M along dim 2 of the staged plane s into sG + off, stored column-major
  // ([K][j]).  Thread t always takes column K = t / RG and rows j = t % RG,
  // t % RG + RG, ...: no divisions, its five taps stay in registers, and
  // consecutive lanes walk rows (odd pitch NK: no LDS bank conflicts).
  constexpr int RG = NTHR / TK;               // row groups per column
  constexpr int RPT = (NJ + RG - 1) / RG;     // rows per thread
  const int rK = tid / RG, rj0 = tid % RG;
  const bool rOK = K0 + rK < a.c2;
  // taps of this thread's dim-2 column and dim-1 row: via LDS into registers
  __shared__ A sW[(TJ + TK) * 5];
  for (int e = tid; e < TK * 5; e += NTHR)
    sW[TJ * 5 + e] = (CO2 && K0 + e / 5 < a.c2) ? a.W2[K0 * 5 + e] : A(0);
  for (int e = tid; e < TJ * 5; e += NTHR)
    sW[e] = (CO1 && J0 + e / 5 < a.c1) ? a.W1[J0 * 5 + e] : A(0);
  __syncthreads();
  // Taps of this thread's dim-2 column and dim-1 row: kept in registers, or
  // -- for the FP32 decomposition, which moves half the bytes of FP64 per
  // step with the same FP64 arithmetic and is latency- rather than
  // memory-bound -- read from LDS where used, which brings it under 128 VGPRs
  // and two resident workgroups per CU (measured faster there, slower for the
  // FP64 and recomposition kernels).
  constexpr bool kTapsInLds = DEC && sizeof(T) == 4;
  A w1r[kTapsInLds ? 1 : 5], w2r[kTapsInLds ? 1 : 5];
  if constexpr (!kTapsInLds) {
#pragma unroll
    for (int o = 0; o < 5; ++o) {
      w2r[o] = sW[TJ * 5 + rK * 5 + o];
      w1r[o] = sW[hJ * 5 + o];
    }
  }
  auto w2 = [&](int o) -> A {
    if constexpr (kTapsInLds) return sW[TJ * 5 + rK * 5 + o];
    else return w2r[o];
  };
  auto w1 = [&](int o) -> A {
    if constexpr (kTapsInLds) return sW[hJ * 5 + o];
    else return w1r[o];
  };
  auto reduce2 = [&](const P *s, int off) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int j = rj0 + q * RG;
      if (j < NJ) {
        A g = A(0);
        if (rOK) {
          if (CO2) {
            const P *row = s + j * NK + 2 * rK;
#pragma unroll
            for (int o = 0; o < 5; ++o) g = fma(w2(o), (A)row[o], g);
          } else {
            g = (A)s[j * NK + rK];
          }
        }
        sG[off + rK * NJ + j] = g;
      }
    }
  };
  // P^T M along dim 1 of the reduced rows at sG + off, for this thread's (J, K)
  auto reduce1 = [&](int off) -> A {
    A h = A(0);
    if (hOK) {
      const A *col = sG + off + hK * NJ;
      if (CO1) {
#pragma unroll
        for (int o = 0; o < 5; ++o) h = fma(w1(o), col[2 * hJ + o], h);
      } else {
        h = col[hJ];
      }
    }
    return h;
  };

  A piPrev[EPT], piNext[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) piPrev[i] = piNext[i] = A(0);
  A h0 = A(0), h1 = A(0), h2 = A(0), h3 = A(0), h4 = A(0);

  // step schedule: with dim 0 coarsened, step I covers fine planes
  // (2I+1, 2I+2) for I in [I0-2, I1-1] and emits F[I] for I >= I0; without,
  // step I is plane I and emits F[I].
  const int64_t sbeg = CO0 ? I0 - 2 : I0, send = I1;  // [sbeg, send)
  auto planes = [&](int64_t I, int64_t &pa, int64_t &pb) {
    if (!CO0) { pa = -1; pb = I; return; }
    pa = 2 * I + 1;
    pb = 2 * I + 2;
    if (!(pa >= 0 && pa < a.m0) || I < I0 - 1) pa = -1;
    if (!(pb >= 0 && pb < a.m0)) pb = -1;
    if (pa >= 0 && pb < 0) { pb = pa; pa = -1; }  // last plane of an even extent is coarse
  };

  // dim-0 taps of step I (threads 0-4) and the dim-0 weight of its fine plane
  // (thread 5), loaded with the step's plane data and staged with it
  // The load is unconditional (every thread reads some valid double) and
  // nothing uses kv before it is staged, so the compiler keeps it in flight
  // with the plane loads; entries are only read where they are meaningful.
  double kv = 0.0;
  auto fetch_consts = [&](int64_t I, int64_t pa) {
    const double *kp = a.r1 ? a.r1 : a.r2;  // any valid table when dim 0 is not coarsened
    if (CO0) {
      const int64_t Ic = min(max(I, (int64_t)0), a.c0 - 1);
      kp = tid < 5 ? a.W0 + Ic * 5 + tid : ((DEC && pa >= 0) ? a.r0 + pa : a.W0);
    }
    kv = *kp;
  };
  P va[EPT], vb[EPT];
  {
    int64_t pa, pb;
    planes(sbeg, pa, pb);
    if (pb >= 0) fetch(vb, pb);
    if (pa >= 0) fetch(va, pa);
    fetch_consts(sbeg, pa);
  }
  for (int64_t I = sbeg; I < send; ++I) {
    int64_t pa, pb;
    planes(I, pa, pb);
    const bool b_in_a_slot = CO0 && pb >= 0 && pb == 2 * I + 1;  // coarse plane in the fine slot
    if (pb >= 0) stage(sA, vb, !DEC && !a.keep_coarse);
    if (pa >= 0) stage(sB, va, false);
    A *kst = sStep[I & 1];
    if (tid < 6) kst[tid] = kv;
    // prefetch the next step while this one computes
    if (I + 1 < send) {
      int64_t qa, qb;
      planes(I + 1, qa, qb);
      if (qb >= 0) fetch(vb, qb);
      if (qa >= 0) fetch(va, qa);
      fetch_consts(I + 1, qa);
    }
    __syncthreads();
    if (pb >= 0) reduce2(sA, 0);
    if (pa >= 0) reduce2(sB, NG);
    if (DEC && pb >= 0) {
      const bool own_p = pb >= oib && pb < oie;
      const int64_t oo = out_plane(pb);
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NTHR;
        const unsigned f = e < NE ? flag_of(i) : 0u;
        piNext[i] = interp2(sA, e, f);
        // Nodes coarse along dims 1 and 2 of a coarse plane belong to the next
        // level, which writes them later.  On the finest level they are
        // written here too (their coefficient is exactly 0): that keeps every
        // written row whole, so no cache line of the output is stored in part.
        if (own_p && (f & F_OWN) && (!NODAL || !((f & F_C1) && (f & F_C2))))
          a.out[oo + (NODAL ? colO[NODAL ? i : 0] : colS[i])] = (T)((A)sA[e] - piNext[i]);
      }
    }
    if (DEC && pa >= 0) {
      const bool own_p = pa >= oib && pa < oie;
      const int64_t oo = out_plane(pa);
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NTHR;
        if (e < NE && own_p && (flag_of(i) & F_OWN))
          a.out[oo + (NODAL ? colO[NODAL ? i : 0] : colS[i])] =
              (T)((A)sB[e] - lerp(piPrev[i], piNext[i], kst[5]));
      }
    }
    __syncthreads();
    const A hb = pb >= 0 ? reduce1(0) : A(0);
    const A ha = pa >= 0 ? reduce1(NG) : A(0);
    if (CO0) {
      h0 = h2;
      h1 = h3;
      h2 = h4;
      h3 = b_in_a_slot ? hb : ha;
      h4 = b_in_a_slot ? A(0) : hb;
      if (I >= I0 && hOK) {
        A f = kst[0] * h0;
        f = fma(kst[1], h1, f);
        f = fma(kst[2], h2, f);
        f = fma(kst[3], h3, f);
        f = fma(kst[4], h4, f);
        a.F[(I * a.c1 + gJ) * a.c2 + gK] = f;
      }
    } else if (hOK) {
      a.F[(I * a.c1 + gJ) * a.c2 + gK] = hb;
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) piPrev[i] = piNext[i];
  }
}

template <typename T, typename TS, bool DEC, bool NODAL, bool CO0, bool CO1, bool CO2>
__global__ void __launch_bounds__((kNTHR<T, DEC, NODAL>), LV_WAVES) k_loadvec(LoadArgs<T, TS> a) {
  loadvec_body<T, TS, DEC, NODAL, CO0, CO1, CO2>(a, xcd_tile(blockIdx.x, a.gx * a.gy * a.gz));
}
template <typename T, typename TS, bool DEC, bool NODAL, bool CO0, bool CO1, bool CO2>
__global__ void __launch_bounds__((kNTHR<T, DEC, NODAL>), LV_WAVES) k_loadvec_group(Group<LoadArgs<T, TS>> g) {
  int j, b;
  group_locate(g, j, b);
  loadvec_body<T, TS, DEC, NODAL, CO0, CO1, CO2>(g.job[j], b);
}

// ------------------------------------------- finest-level load vector, LDS ring

// Zeros read by the global-to-LDS loads of tile elements outside the grid (and,
// in a recomposition, of the stored coarse values, which count as zero).
__device__ __align__(16) double g_zero_words[2];

// LDS-only workgroup barrier: waits for this wave's LDS operations, not for
// its vector-memory loads, so global-to-LDS loads of later stages stay in
// flight across it (__syncthreads would wait for them).  The asm is also a
// compiler barrier for memory accesses.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Waits until at most N vector-memory operations of this wave are
// outstanding (lgkm and exp counters left free).
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt holds 6 bits");
  __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

typedef __attribute__((address_space(3))) void *lds_ptr;

// One 4-byte global-to-LDS load per lane: lane i's word at `src` goes to LDS
// byte address lds + 4 i (`lds` wave-uniform).  Written as asm so that the
// compiler does not see the LDS write: it would otherwise wait for every
// such load in flight before reading any staged plane whose independence it
// cannot prove.  The kernel's own vmcnt waits and LDS barriers order the
// loads with the reads.  One wait state between writing M0 and the load.
// M0 is a reserved register: the compiler warns that it may not honour the
// clobber, so this is safe only while compiled code keeps nothing of its own
// in M0 in the kernels that use it (in the ring kernels every instruction
// naming M0 is this block's write; a CPU test checks the assembly).
__device__ __forceinline__ void lds_dma_dword(const void *src, unsigned lds) {
  asm volatile("s_mov_b32 m0, %0\n\ts_nop 0\n\tglobal_load_lds_dword %1, off" : : "s"(lds), "v"(src) : "memory", "m0");
}

// Finest-level decomposition step (coefficients and load vector), the
// computation of k_loadvec on a level grid stored compactly in C order, with
// the plane pairs staged differently: every
// element of a staged plane comes straight from memory into LDS through
// 4-byte global-to-LDS loads, and NST stages of plane pairs rotate, so the
// loads of the next NST-1 steps are in flight while a step computes (the
// register prefetch of k_loadvec keeps one).  An element outside the grid is
// loaded from g_zero_words.
// Each wave issues the same number of loads for every step (steps past the
// chunk load zeros), so the wait for a stage is a fixed count.  One
// workgroup per compute unit (147 KB of LDS at TJ = 16).
//
// Tiles: TJ x TK coarse rows x columns, except that the last tile along dim
// 1 (dim 2) takes one more coarse row (column) when a single one would be
// left over, as for every 2^k + 1 extent; its staged halo already holds the
// fine nodes that row needs, and threads 0.. compute its load-vector
// entries as extra items beside their own.
template <int TJ>
constexpr int kRingThr = TJ * TK;
template <typename TS, int TJ>
struct RingGeom {
  static constexpr int NTHR = TJ * TK;
  static constexpr int NJ = 2 * TJ + 3, NK = 2 * TK + 3;  // staged rows / columns (two-node halo)
  static constexpr int NE = NJ * NK;
  static constexpr int DW = (int)(sizeof(TS) / 4);         // 4-byte words per element
  static constexpr int NSLOT = (DW * NE + NTHR - 1) / NTHR;  // loads per thread per plane
  static constexpr int PLANE_WORDS = NSLOT * NTHR;          // padded stage plane
  static constexpr int EPT = (NE + NTHR - 1) / NTHR;        // coefficient elements per thread
  static constexpr int NG = NJ * (TK + 1);                  // dim-2 reduced rows of one plane
};
constexpr int RING_MAXTI = 130;  // coarse planes per workgroup at most (step table in LDS)

template <typename T, typename TS, bool CO0, bool CO1, bool CO2, int TJ, int NST>
__global__ void __launch_bounds__(kRingThr<TJ>, 1) k_loadvec_ring(LoadArgs<T, TS> a) {
  using A = double;  // a decomposition computes in FP64 (see k_loadvec)
  using P = TS;
  using G = RingGeom<TS, TJ>;
  constexpr int NTHR = G::NTHR, NJ = G::NJ, NK = G::NK, NE = G::NE, NSLOT = G::NSLOT;
  constexpr int EPT = G::EPT, NG = G::NG, PW = G::PLANE_WORDS;
  static_assert(CO0 && CO1 && CO2, "the ring kernel serves levels coarsened along every dim");
  static_assert(NST == 3, "the step loop is unrolled for three stages");
  static_assert(EPT <= 8, "the per-thread flags hold 4 bits for each of at most 8 tile elements");
  // stages: plane b (coarse along dim 0) and plane a (fine along dim 0) of a step
  __shared__ __align__(16) unsigned sA0[PW], sB0[PW], sA1[PW], sB1[PW], sA2[PW], sB2[PW];
  __shared__ A sG[2 * NG];  // dim-2 reduced rows of b, then of a ([K][j], K <= TK)
  __shared__ A sR1[NJ], sR2[NK];
  __shared__ A sW[(TJ + 1 + TK + 1) * 5];
  __shared__ A sK[CO0 ? (RING_MAXTI + 2) * 6 : 1];  // per-step dim-0 taps and fine-plane weight

  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int tile = xcd_tile(blockIdx.x, a.gx * a.gy * a.gz);
  const int tx = tile % a.gx, ty = (tile / a.gx) % a.gy, tz = tile / (a.gx * a.gy);
  const int64_t J0 = (int64_t)ty * TJ, K0 = (int64_t)tx * TK;
  const int64_t I0 = (int64_t)tz * a.TI;
  const int64_t I1 = min(I0 + a.TI, a.c0);
  const int64_t fj0 = 2 * J0 - 2, fk0 = 2 * K0 - 2;
  const bool lastJ = ty == a.gy - 1, lastK = tx == a.gx - 1, lastI = I1 >= a.c0;
  // coarse rows / columns of this tile (TJ or TK, one more for an absorbed last one)
  const int nJ = (int)min<int64_t>(a.c1 - J0, lastJ ? TJ + 1 : TJ);
  const int nK = (int)min<int64_t>(a.c2 - K0, lastK ? TK + 1 : TK);
  const int64_t ojb = 2 * J0, oje = lastJ ? a.m1 : 2 * (J0 + TJ);
  const int64_t okb = 2 * K0, oke = lastK ? a.m2 : 2 * (K0 + TK);
  const int64_t oib = (CO0 ? 2 : 1) * I0;
  const int64_t oie = lastI ? a.m0 : (CO0 ? 2 : 1) * I1;

  // word offsets of this thread's load slots in a plane (-1: load zero)
  int off[NSLOT];
#pragma unroll
  for (int u = 0; u < NSLOT; ++u) {
    const int w = u * NTHR + tid, e = w / G::DW, h = w % G::DW;
    const int j = e / NK, k = e % NK;
    const int64_t gj = fj0 + j, gk = fk0 + k;
    off[u] = (e < NE && gj >= 0 && gj < a.m1 && gk >= 0 && gk < a.m2) ? (int)(gj * a.smap.s1 + gk) * G::DW + h
                                                                       : -1;
  }
  // per-element constants of this thread's coefficient elements
  enum : unsigned { F_IN = 1, F_OWN = 2, F_C1 = 4, F_C2 = 8 };
  unsigned flags = 0;
  int colS[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = tid + i * NTHR;
    const int j = e / NK, k = e % NK;
    const int64_t gj = fj0 + j, gk = fk0 + k;
    unsigned f = 0;
    colS[i] = 0;
    if (e < NE && gj >= 0 && gj < a.m1 && gk >= 0 && gk < a.m2) {
      f |= F_IN;
      if (gj >= ojb && gj < oje && gk >= okb && gk < oke) f |= F_OWN;
      if (coarse_pos<true>(gj, a.m1)) f |= F_C1;
      if (coarse_pos<true>(gk, a.m2)) f |= F_C2;
      colS[i] = (int)(gj * a.smap.s1 + gk);
    }
    flags |= f << (4 * i);
  }
  auto flag_of = [&](int i) -> unsigned { return (flags >> (4 * i)) & 15u; };

  for (int j = tid; j < NJ; j += NTHR) {
    const int64_t gj = fj0 + j;
    sR1[j] = (gj >= 0 && gj < a.m1 && !coarse_pos<true>(gj, a.m1)) ? a.r1[gj] : A(0);
  }
  for (int k = tid; k < NK; k += NTHR) {
    const int64_t gk = fk0 + k;
    sR2[k] = (gk >= 0 && gk < a.m2 && !coarse_pos<true>(gk, a.m2)) ? a.r2[gk] : A(0);
  }
  // taps: rows 0..TJ (row TJ only if absorbed), then columns 0..TK
  for (int e = tid; e < (TJ + 1) * 5; e += NTHR) sW[e] = (e / 5 < nJ) ? a.W1[J0 * 5 + e] : A(0);
  for (int e = tid; e < (TK + 1) * 5; e += NTHR) sW[(TJ + 1) * 5 + e] = (e / 5 < nK) ? a.W2[K0 * 5 + e] : A(0);

  // step schedule (as k_loadvec): with dim 0 coarsened, step I covers fine
  // planes (2I+1, 2I+2) for I in [I0-2, I1-1] and emits F[I] for I >= I0
  const int64_t sbeg = CO0 ? I0 - 2 : I0, send = I1;
  auto planes = [&](int64_t I, int64_t &pa, int64_t &pb) {
    if (I >= send) { pa = pb = -1; return; }
    if (!CO0) { pa = -1; pb = I; return; }
    pa = 2 * I + 1;
    pb = 2 * I + 2;
    if (!(pa >= 0 && pa < a.m0) || I < I0 - 1) pa = -1;
    if (!(pb >= 0 && pb < a.m0)) pb = -1;
    if (pa >= 0 && pb < 0) { pb = pa; pa = -1; }  // last plane of an even extent is coarse
  };
  if (CO0) {
    for (int q = tid; q < (int)(send - sbeg) * 6; q += NTHR) {
      const int64_t I = sbeg + q / 6;
      const int o = q % 6;
      A v = A(0);
      if (o < 5) {
        v = a.W0[min(max(I, (int64_t)0), a.c0 - 1) * 5 + o];
      } else {
        int64_t pa, pb;
        planes(I, pa, pb);
        if (pa >= 0) v = a.r0[pa];
      }
      sK[q] = v;
    }
  }
  __syncthreads();

  // this thread's taps of its dim-2 column and dim-1 row
  constexpr int RG = NTHR / TK, RPT = (NJ + RG - 1) / RG;
  const int rK = tid / RG, rj0 = tid % RG;
  const int hJ = tid / TK, hK = tid % TK;
  A w1r[5], w2r[5];
#pragma unroll
  for (int o = 0; o < 5; ++o) {
    w2r[o] = sW[(TJ + 1) * 5 + rK * 5 + o];
    w1r[o] = sW[hJ * 5 + o];
  }
  // extra items of an absorbed row / column: item x < nx is the load-vector
  // entry (xj, xk) in tile coordinates, taken by thread x
  const bool xcol = nK > TK, xrow = nJ > TJ;
  const int ncol = xcol ? nJ : 0;           // column TK, rows 0 .. nJ-1
  const int nx = ncol + (xrow ? min(nK, TK) : 0);  // then row TJ, columns 0 .. TK-1
  const bool hasx = tid < nx;
  const int xj = tid < ncol ? tid : TJ, xk = tid < ncol ? TK : tid - ncol;
  A xw1[5];
#pragma unroll
  for (int o = 0; o < 5; ++o) xw1[o] = hasx ? sW[xj * 5 + o] : A(0);

  const bool hOK = hJ < nJ && hK < nK;
  auto reduce2 = [&](const P *sp, int off) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int j = rj0 + q * RG;
      if (j < NJ) {
        A g = A(0);
        if (rK < nK) {
          const P *row = sp + j * NK + 2 * rK;
#pragma unroll
          for (int o = 0; o < 5; ++o) g = fma(w2r[o], (A)row[o], g);
        }
        sG[off + rK * NJ + j] = g;
      }
    }
    if (xcol && tid < NJ) {  // column TK: fine columns 2TK .. 2TK+2 of the tile
      const P *row = sp + tid * NK + 2 * TK;
      A g = A(0);
#pragma unroll
      for (int o = 0; o < 3; ++o) g = fma(sW[(TJ + 1) * 5 + TK * 5 + o], (A)row[o], g);
      sG[off + TK * NJ + tid] = g;
    }
  };
  // P^T M along dim 1 of the reduced rows at sG + off for entry (j, k) with taps w
  auto reduce1 = [&](int off, int j, int k, const A (&w)[5]) -> A {
    const A *col = sG + off + k * NJ + 2 * j;
    if (j == TJ) {  // absorbed row: fine rows 2TJ .. 2TJ+2
      A h = A(0);
#pragma unroll
      for (int o = 0; o < 3; ++o) h = fma(w[o], col[o], h);
      return h;
    }
    A h = A(0);
#pragma unroll
    for (int o = 0; o < 5; ++o) h = fma(w[o], col[o], h);
    return h;
  };

  // bilinear interpolant (dims 1, 2) of tile element e of the staged plane
  auto interp2 = [&](const P *sp, int e, unsigned f) -> A {
    if (!(f & F_IN)) return A(0);
    const int dk = (f & F_C2) ? 0 : 1, dj = (f & F_C1) ? 0 : NK;
    const A rk = sR2[e % NK], rj = sR1[e / NK];
    return lerp(lerp((A)sp[e - dj - dk], (A)sp[e - dj + dk], rk), lerp((A)sp[e + dj - dk], (A)sp[e + dj + dk], rk),
                rj);
  };

  // global-to-LDS loads of step J's planes into stage (dA, dB); every wave
  // issues 2 NSLOT loads whatever J is
  const char *zero = (const char *)g_zero_words;
  auto issue = [&](unsigned *dA, unsigned *dB, int64_t J) {
    int64_t pa, pb;
    planes(J, pa, pb);
    const char *bb = pb >= 0 ? (const char *)(a.src + pb * a.smap.s0) : zero;
    const char *ba = pa >= 0 ? (const char *)(a.src + pa * a.smap.s0) : zero;
    const unsigned la = (unsigned)(uintptr_t)(lds_ptr)dA, lb = (unsigned)(uintptr_t)(lds_ptr)dB;
#pragma unroll
    for (int u = 0; u < NSLOT; ++u) {
      const char *src = (pb >= 0 && off[u] >= 0) ? bb + (int64_t)off[u] * 4 : zero;
      lds_dma_dword(src, __builtin_amdgcn_readfirstlane(la + 4u * (u * NTHR + wave * 64)));
    }
#pragma unroll
    for (int u = 0; u < NSLOT; ++u) {
      const char *src = (pa >= 0 && off[u] >= 0) ? ba + (int64_t)off[u] * 4 : zero;
      lds_dma_dword(src, __builtin_amdgcn_readfirstlane(lb + 4u * (u * NTHR + wave * 64)));
    }
  };

  A piPrev[EPT], piNext[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) piPrev[i] = piNext[i] = A(0);
  A h0 = A(0), h1 = A(0), h2 = A(0), h3 = A(0), h4 = A(0);
  A x0 = A(0), x1 = A(0), x2 = A(0), x3 = A(0), x4 = A(0);  // window of the extra item

  // one step: issue step I + NST - 1 into the stage step I - 1 used, wait for
  // step I's stage, compute
  auto step = [&](int64_t I, const unsigned *cA, const unsigned *cB, unsigned *rA, unsigned *rB) {
    issue(rA, rB, I + NST - 1);
    wait_vm<2 * NSLOT * (NST - 1)>();
    lds_barrier();
    const P *pA = (const P *)cA, *pB = (const P *)cB;
    int64_t pa, pb;
    planes(I, pa, pb);
    const bool b_in_a_slot = CO0 && pb >= 0 && pb == 2 * I + 1;
    const A *kst = sK + (CO0 ? (I - sbeg) * 6 : 0);
    if (pb >= 0) reduce2(pA, 0);
    if (pa >= 0) reduce2(pB, NG);
    if (pb >= 0) {
      const bool own_p = pb >= oib && pb < oie;
      T *oo = a.out + pb * a.omap.s0;
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NTHR;
        const unsigned f = e < NE ? flag_of(i) : 0u;
        piNext[i] = interp2(pA, e, f);
        // the finest level also writes its coarse nodes (coefficient exactly
        // 0, overwritten by the next level) so that every written row is whole
        if (own_p && (f & F_OWN)) oo[colS[i]] = (T)((A)pA[e] - piNext[i]);
      }
    }
    if (pa >= 0) {
      const bool own_p = pa >= oib && pa < oie;
      T *oo = a.out + pa * a.omap.s0;
      const A r0 = kst[5];
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = tid + i * NTHR;
        if (e < NE && own_p && (flag_of(i) & F_OWN)) oo[colS[i]] = (T)((A)pB[e] - lerp(piPrev[i], piNext[i], r0));
      }
    }
    lds_barrier();
    const A hb = (pb >= 0 && hOK) ? reduce1(0, hJ, hK, w1r) : A(0);
    const A ha = (pa >= 0 && hOK) ? reduce1(NG, hJ, hK, w1r) : A(0);
    const A xb = (pb >= 0 && hasx) ? reduce1(0, xj, xk, xw1) : A(0);
    const A xa = (pa >= 0 && hasx) ? reduce1(NG, xj, xk, xw1) : A(0);
    if (CO0) {
      h0 = h2; h1 = h3; h2 = h4;
      h3 = b_in_a_slot ? hb : ha;
      h4 = b_in_a_slot ? A(0) : hb;
      x0 = x2; x1 = x3; x2 = x4;
      x3 = b_in_a_slot ? xb : xa;
      x4 = b_in_a_slot ? A(0) : xb;
      if (I >= I0) {
        if (hOK) {
          A f = kst[0] * h0;
          f = fma(kst[1], h1, f);
          f = fma(kst[2], h2, f);
          f = fma(kst[3], h3, f);
          f = fma(kst[4], h4, f);
          a.F[(I * a.c1 + J0 + hJ) * a.c2 + K0 + hK] = f;
        }
        if (hasx) {
          A f = kst[0] * x0;
          f = fma(kst[1], x1, f);
          f = fma(kst[2], x2, f);
          f = fma(kst[3], x3, f);
          f = fma(kst[4], x4, f);
          a.F[(I * a.c1 + J0 + xj) * a.c2 + K0 + xk] = f;
        }
      }
    } else {
      if (hOK) a.F[(I * a.c1 + J0 + hJ) * a.c2 + K0 + hK] = hb;
      if (hasx) a.F[(I * a.c1 + J0 + xj) * a.c2 + K0 + xk] = xb;
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) piPrev[i] = piNext[i];
  };

  issue(sA0, sB0, sbeg);
  issue(sA1, sB1, sbeg + 1);
  int64_t I = sbeg;
  for (; I + 2 < send; I += 3) {
    step(I, sA0, sB0, sA2, sB2);
    step(I + 1, sA1, sB1, sA0, sB0);
    step(I + 2, sA2, sB2, sA1, sB1);
  }
  if (I < send) step(I, sA0, sB0, sA2, sB2);
  if (I + 1 < send) step(I + 1, sA1, sB1, sA0, sB0);
  wait_vm<0>();  // no load may still write this workgroup's LDS when it ends
}

// ------------------------------------------------------------ correction solves

struct SolveDev {
  const double *sup, *w, *invb, *supi, *Ls, *Rs, *sepa, *sepe, *wr, *invbr, *gam;
};
SolveDev solve_dev(const DimTabs &d) {
  return SolveDev{d.sup, d.w, d.invb, d.supi, d.Ls, d.Rs, d.sepa, d.sepe, d.wr, d.invbr, d.gam};
}

// What the last solve of a step does with its solution z when it stores it:
// keep it in F (FP64), store it as the next level's values (decompose: the
// load vector was formed from the values, so z is the corrected coarse grid)
// compactly or at its nodal positions, or subtract it from the stored coarse
// values (recompose).
enum EpiMode { EPI_Z = 0, EPI_STORE_COMPACT = 1, EPI_STORE_NODAL = 2, EPI_SUB_COMPACT = 3 };

template <typename T>
struct Epi {
  int mode;
  T *dst;        // compact next-level grid (STORE_COMPACT / SUB_COMPACT) or output array (STORE_NODAL)
  Map3 nmap;     // STORE_NODAL: nodal map of the coarse grid
};

template <typename T>
__device__ __forceinline__ void epi_store(const Epi<T> &e, double *F, int64_t idx, int64_t i,
                                          int64_t j, int64_t k, double z) {
  switch (e.mode) {
    case EPI_Z: F[idx] = z; break;
    case EPI_STORE_COMPACT: e.dst[idx] = (T)z; break;
    case EPI_STORE_NODAL: e.dst[moff(e.nmap, i, j, k)] = (T)z; break;
    default: e.dst[idx] = (T)((double)e.dst[idx] - z); break;
  }
}

// Interior solve of one partition held in x[0..S): forward elimination and
// back substitution with the block factors of positions f .. f+S-1.  The
// tables are padded so that the separator slot and the slots past the end
// of the line pass through unchanged: the loop is straight-line code whose
// table reads do not depend on the data, so they can all be in flight
// before the dependent chain needs them.
template <int S>
__device__ __forceinline__ void partition_solve(double (&x)[S], const SolveDev &tb, int64_t f) {
#pragma unroll
  for (int q = 1; q < S; ++q) x[q] = fma(-tb.w[f + q], x[q - 1], x[q]);
  x[S - 1] *= tb.invb[f + S - 1];
#pragma unroll
  for (int q = S - 2; q >= 0; --q) x[q] = fma(-tb.supi[f + q], x[q + 1], x[q]) * tb.invb[f + q];
}

// Separator fix-up of a partition: x -= t_left Ls + t_right Rs (zero at the
// separator and padding slots), then the separator slot takes its value.
template <int S>
__device__ __forceinline__ void partition_fixup(double (&x)[S], const SolveDev &tb, int64_t f, double tl,
                                                double tr, bool has_sep) {
#pragma unroll
  for (int q = 0; q < S; ++q) x[q] = fma(-tl, tb.Ls[f + q], fma(-tr, tb.Rs[f + q], x[q]));
  if (has_sep) x[S - 1] = tr;
}

template <int S>
__device__ __forceinline__ double pick(const double (&x)[S], int q) {
  double v = 0.0;
#pragma unroll
  for (int i = 0; i < S; ++i)
    if (i == q) v = x[i];
  return v;
}

// Separator system of one line: rhs_p = Fs_p - a_s yL_p - e_s yF_{p+1};
// Thomas with the precomputed factors.  Arrays are strided by `ld`.
__device__ __forceinline__ void separator_solve(const SolveDev &tb, int S, int P, const double *yF,
                                                const double *yL, const double *Fs, double *t,
                                                int ld) {
  double g = 0.0;
  for (int sp = 0; sp < P - 1; ++sp) {
    double rhs = Fs[sp * ld] - tb.sepa[sp] * yL[sp * ld] - tb.sepe[sp] * yF[(sp + 1) * ld];
    g = fma(-tb.wr[sp], g, rhs);
    t[sp * ld] = g;
  }
  double nxt = 0.0;
  for (int sp = P - 2; sp >= 0; --sp) {
    nxt = fma(-tb.gam[sp], nxt, t[sp * ld]) * tb.invbr[sp];
    t[sp * ld] = nxt;
  }
}

// Copies a line's solve tables into LDS -- w, invb, supi, Ls, Rs [cp = P*S]
// each, then sepa, sepe, wr, invbr, gam [P] -- with eight loads in flight
// per thread, and returns LDS-backed accessors.  Used by the row solver, whose lanes work on
// different partitions: it is persistent, so a workgroup stages the tables
// once and then walks many blocks of rows, and table reads inside the
// sequential solve chain cost an LDS access instead of a round trip to
// memory.  (In the strided solver a wave shares one partition, and its
// table reads are scalar-cache loads.)
__device__ __forceinline__ SolveDev stage_tables(double *tab, const SolveDev &tg, int cp, int P, int t,
                                                 int nt) {
  const double *src[5] = {tg.w, tg.invb, tg.supi, tg.Ls, tg.Rs};
  const int n = 5 * cp;
  for (int e = t; e < n; e += 8 * nt) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = min(e + u * nt, n - 1);
      v[u] = src[q / cp][q % cp];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (e + u * nt < n) tab[e + u * nt] = v[u];
  }
  for (int q = t; q < P - 1; q += nt) {
    tab[n + q] = tg.sepa[q];
    tab[n + P + q] = tg.sepe[q];
    tab[n + 2 * P + q] = tg.wr[q];
    tab[n + 3 * P + q] = tg.invbr[q];
    tab[n + 4 * P + q] = tg.gam[q];
  }
  return SolveDev{nullptr, tab, tab + cp, tab + 2 * cp, tab + 3 * cp, tab + 4 * cp,
                  tab + n, tab + n + P, tab + n + 2 * P, tab + n + 3 * P, tab + n + 4 * P};
}
__host__ __device__ constexpr int tables_size(int cp, int P) { return 5 * cp + 5 * P; }

// Lines along dim 0 or 1: lane = position along the contiguous dim 2,
// wave = partition.  Element q of partition p of line (outer, k) sits at
// F[outer * so + k + (p*S + q) * sp].
template <typename T>
struct StridedArgs {
  double *F;
  int64_t c, nk, sp, so, c1, c2;
  int P, axis;
  SolveDev tb;
  Epi<T> ep;
};

// Blocks of 64 lines in (outer, k-block) order; `blk` is numbered so that
// consecutive ones run on one XCD: neighbouring k-blocks share the cache
// lines at their ends.
template <typename T, int S>
__device__ __forceinline__ void strided_body(const StridedArgs<T> &A, const int blk) {
  double *F = A.F;
  const int64_t c = A.c, nk = A.nk, sp_ = A.sp, so = A.so;
  const int P = A.P, axis = A.axis;
  const SolveDev &tb = A.tb;
  const Epi<T> &ep = A.ep;
  extern __shared__ double xs[];
  const int lane = threadIdx.x & 63;
  const int p = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (p >= P) {  // a grouped launch sized for a job with more partitions: only meet the barriers
    if (P > 1) {
      __syncthreads();
      __syncthreads();
    }
    return;
  }
  const int nkb = (int)((nk + 63) / 64);
  const int64_t k = (int64_t)(blk % nkb) * 64 + lane;
  const int64_t outer = blk / nkb;
  const bool active = k < nk;
  const int64_t base = outer * so + k;
  const int64_t f = (int64_t)p * S;
  const int nload = p < P - 1 ? S : (int)(c - f);
  const int nint = p < P - 1 ? S - 1 : nload;

  double x[S];
#pragma unroll
  for (int q = 0; q < S; ++q) x[q] = (active && q < nload) ? F[base + (f + q) * sp_] : 0.0;
  partition_solve<S>(x, tb, f);

  double *yF = xs, *yL = xs + P * 64, *Fs = xs + 2 * P * 64, *tt = xs + 3 * P * 64;
  if (P > 1) {
    yF[p * 64 + lane] = x[0];
    yL[p * 64 + lane] = pick<S>(x, nint - 1);
    Fs[p * 64 + lane] = x[S - 1];
    __syncthreads();
    if (p == 0) separator_solve(tb, S, P, yF + lane, yL + lane, Fs + lane, tt + lane, 64);
    __syncthreads();
    const double tl = p > 0 ? tt[(p - 1) * 64 + lane] : 0.0;
    const double tr = p < P - 1 ? tt[p * 64 + lane] : 0.0;
    partition_fixup<S>(x, tb, f, tl, tr, p < P - 1);
  }
  if (!active) return;
  if (ep.mode == EPI_SUB_COMPACT) {
    // read the stored values eight at a time: one memory round trip per
    // eight elements, not one per element
#pragma unroll
    for (int q0 = 0; q0 < S; q0 += 8) {
      T d[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) d[u] = ep.dst[base + (f + min(q0 + u, nload - 1)) * sp_];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q0 + u < nload) ep.dst[base + (f + q0 + u) * sp_] = (T)((double)d[u] - x[q0 + u]);
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < S; ++q) {
    if (q < nload) {
      const int64_t pos = f + q;
      const int64_t idx = base + pos * sp_;
      const int64_t i = axis == 0 ? pos : outer;
      const int64_t j = axis == 0 ? outer : pos;
      epi_store(ep, F, idx, i, j, k, x[q]);
    }
  }
}

// (five waves per SIMD keep two 9-wave workgroups resident per CU at S = 32)
template <typename T, int S>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5))) k_solve_strided(StridedArgs<T> a) {
  strided_body<T, S>(a, xcd_tile(blockIdx.x, gridDim.x));
}
template <typename T, int S>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(5))) k_solve_strided_group(
    Group<StridedArgs<T>> g) {
  int j, b;
  group_locate(g, j, b);
  strided_body<T, S>(g.job[j], b);
}

// Threads of a row-solver workgroup at most: its LDS budget keeps blocks small
// anyway, and the cap leaves each thread room for a whole partition in
// registers.
constexpr int ROWS_THR = 256;

// Lines along the contiguous dim 2: a workgroup stages R consecutive rows in
// LDS (a straight coalesced copy: consecutive rows are contiguous), thread
// (r, p) solves partition p of row r in registers.  Persistent over blocks
// of R rows.
template <typename T>
struct RowsArgs {
  double *F;
  int64_t nrows, c1;
  int c, P, R;
  SolveDev tg;
  Epi<T> ep;
};

// Blocks first, first + stride, ... of R rows.
template <typename T, int S>
__device__ __forceinline__ void rows_body(const RowsArgs<T> &A, const int64_t first, const int64_t stride) {
  double *F = A.F;
  const int64_t nrows = A.nrows, c1 = A.c1;
  const int c = A.c, P = A.P, R = A.R;
  const SolveDev &tg = A.tg;
  const Epi<T> &ep = A.ep;
  extern __shared__ double sm[];
  const int t = threadIdx.x, nt = blockDim.x;
  const SolveDev tb = stage_tables(sm, tg, P * S, P, t, nt);
  double *tile = sm + tables_size(P * S, P);  // [R][c]
  double *ex = tile + (size_t)R * c;       // separator exchange [4][P][R]
  double *yF = ex, *yL = ex + P * R, *Fs = ex + 2 * P * R, *tt = ex + 3 * P * R;
  // threads past R x P (a grouped launch sized for a larger job) stage and
  // store with the others but solve nothing
  const bool solver = t < R * P;
  const int r = t % R, p = solver ? t / R : 0;
  const int64_t f = (int64_t)p * S;
  const int nload = p < P - 1 ? S : (int)(c - f);
  const int nint = p < P - 1 ? S - 1 : nload;
  const int64_t nblocks = (nrows + R - 1) / R;
  for (int64_t blk = first; blk < nblocks; blk += stride) {
    const int64_t row0 = blk * R;
    const int nr = (int)min<int64_t>(R, nrows - row0);
    const int64_t gbase = row0 * c;
    const int n = nr * c;
    __syncthreads();  // the previous block's stores have read the tile
    // up to 16 loads per thread in flight at once (a block holds at most S
    // elements per thread: n <= R c <= R P S <= nt S).  All S at once needs
    // about 270 VGPRs at S = 32, one workgroup per CU, and measured 1.8x
    // slower; 8 at a time (four round trips at S = 32) 3-10% slower.
    constexpr int RCH = S < 16 ? S : 16;
    for (int e = t; e < n; e += RCH * nt) {
      double v[RCH];
#pragma unroll
      for (int u = 0; u < RCH; ++u) v[u] = F[gbase + min(e + u * nt, n - 1)];
#pragma unroll
      for (int u = 0; u < RCH; ++u)
        if (e + u * nt < n) tile[e + u * nt] = v[u];
    }
    __syncthreads();
    const bool active = solver && r < nr;
    double x[S];
    const double *rowp = tile + r * c + f;
#pragma unroll
    for (int q = 0; q < S; ++q) x[q] = (active && q < nload) ? rowp[q] : 0.0;
    partition_solve<S>(x, tb, f);
    if (P > 1) {
      if (solver) {
        yF[p * R + r] = x[0];
        yL[p * R + r] = pick<S>(x, nint - 1);
        Fs[p * R + r] = x[S - 1];
      }
      __syncthreads();
      if (solver && p == 0) separator_solve(tb, S, P, yF + r, yL + r, Fs + r, tt + r, R);
      __syncthreads();
      const double tl = p > 0 ? tt[(p - 1) * R + r] : 0.0;
      const double tr = p < P - 1 ? tt[p * R + r] : 0.0;
      partition_fixup<S>(x, tb, f, tl, tr, p < P - 1);
    }
    if (active) {
      double *roww = tile + r * c + f;
#pragma unroll
      for (int q = 0; q < S; ++q)
        if (q < nload) roww[q] = x[q];
    }
    __syncthreads();
    if (ep.mode == EPI_SUB_COMPACT) {
      // the stored values of the block, 16 loads at a time as above
      constexpr int RCH = S < 16 ? S : 16;
      for (int e = t; e < n; e += RCH * nt) {
        T d[RCH];
#pragma unroll
        for (int u = 0; u < RCH; ++u) d[u] = ep.dst[gbase + min(e + u * nt, n - 1)];
#pragma unroll
        for (int u = 0; u < RCH; ++u)
          if (e + u * nt < n) ep.dst[gbase + e + u * nt] = (T)((double)d[u] - tile[e + u * nt]);
      }
    } else if (ep.mode == EPI_STORE_NODAL) {
      for (int e = t; e < n; e += nt) {
        const int rr = e / c, cc = e - rr * c;
        const int64_t row = row0 + rr, i = row / c1, j = row - i * c1;
        epi_store(ep, F, gbase + e, i, j, cc, tile[e]);
      }
    } else {
      for (int e = t; e < n; e += nt) epi_store(ep, F, gbase + e, 0, 0, 0, tile[e]);
    }
  }
}

template <typename T, int S>
__global__ void __launch_bounds__(ROWS_THR) k_solve_rows(RowsArgs<T> a) {
  rows_body<T, S>(a, blockIdx.x, gridDim.x);
}
// one block per workgroup (not persistent)
template <typename T, int S>
__global__ void __launch_bounds__(ROWS_THR) k_solve_rows_group(Group<RowsArgs<T>> g) {
  int j, b;
  group_locate(g, j, b);
  rows_body<T, S>(g.job[j], b, (int64_t)1 << 62);
}

// Lines of more than kMaxBlocks partitions of 64 (up to kLongBlocks): the
// same partitioned solve.  A workgroup takes a block of LB lines; the lanes
// of a wave hold 64 / LB partition groups of those lines, and group g of
// wave w takes partitions v, v + NV, ... (v = w * 64 / LB + g, NV the groups
// of the workgroup) in turn.  The interior solutions wait
// in F between the elimination and the separator fix-up, so such a line is
// read and written twice.  LB = 64: a wave takes one partition of 64 lines
// (its solve-table reads are uniform); LB = 16 gives four times the
// workgroups, for launches that would leave most CUs idle (a 2-D field's
// lines: 4097 lines of level 0 at 8193^2 are 65 blocks of 64), at the cost
// of per-lane table reads.  Adjacent lines of a strided dimension are read
// in whole 128-byte lines; rows of the contiguous one have each lane walk
// its own row.
constexpr int LONG_WAVES = 8;
constexpr int LONG_CH = 16;  // fix-up chunk
template <typename T>
struct LongArgs {
  double *F;
  int64_t c, nk, sp, so, sk, c1;
  int P, axis;
  SolveDev tb;
  Epi<T> ep;
};

// Blocks of LB lines in (outer, k-block) order; this workgroup takes block `blk`.
template <typename T, int LB>
__device__ __forceinline__ void long_body(const LongArgs<T> &A, const int64_t blk) {
  double *F = A.F;
  const int64_t c = A.c, nk = A.nk, sp_ = A.sp, so = A.so, sk = A.sk, c1 = A.c1;
  const int P = A.P, axis = A.axis;
  const SolveDev &tb = A.tb;
  const Epi<T> &ep = A.ep;
  constexpr int S = 64;
  constexpr int NG = 64 / LB;       // partition groups per wave
  constexpr int NV = LONG_WAVES * NG;    // partition groups per workgroup
  extern __shared__ double xs[];  // yF, yL, Fs, t: [P][LB] each
  const int lane = threadIdx.x & 63;
  const int l = lane % LB;
  // this thread's partition group (LB = 64: the wave, made uniform so that
  // the table reads are scalar)
  const int v = LB == 64 ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : (threadIdx.x >> 6) * NG + lane / LB;
  const int64_t nkb = (nk + LB - 1) / LB;
  const int64_t k = (blk % nkb) * LB + l;
  const int64_t outer = blk / nkb;
  const bool active = k < nk;
  const int64_t base = outer * so + (active ? k : 0) * sk;
  double *yF = xs, *yL = xs + P * LB, *Fs = xs + 2 * P * LB, *tt = xs + 3 * P * LB;
  for (int p = v; p < P; p += NV) {
    const int64_t f = (int64_t)p * S;
    const int nload = p < P - 1 ? S : (int)(c - f);
    const int nint = p < P - 1 ? S - 1 : nload;
    double x[S];
#pragma unroll
    for (int q = 0; q < S; ++q) x[q] = (active && q < nload) ? F[base + (f + q) * sp_] : 0.0;
    partition_solve<S>(x, tb, f);
    yF[p * LB + l] = x[0];
    yL[p * LB + l] = pick<S>(x, nint - 1);
    Fs[p * LB + l] = x[S - 1];
    if (active) {
#pragma unroll
      for (int q = 0; q < S; ++q)
        if (q < nint) F[base + (f + q) * sp_] = x[q];
    }
  }
  __syncthreads();
  if (v == 0) separator_solve(tb, S, P, yF + l, yL + l, Fs + l, tt + l, LB);
  __syncthreads();
  if (!active) return;
  // fix-up in chunks of LONG_CH positions, a chunk's loads all in flight
  // before its first use
  for (int p = v; p < P; p += NV) {
    const int64_t f = (int64_t)p * S;
    const int nload = p < P - 1 ? S : (int)(c - f);
    const int nint = p < P - 1 ? S - 1 : nload;
    const double tl = p > 0 ? tt[(p - 1) * LB + l] : 0.0;
    const double tr = p < P - 1 ? tt[p * LB + l] : 0.0;
    for (int q0 = 0; q0 < nload; q0 += LONG_CH) {
      double x[LONG_CH];
#pragma unroll
      for (int u = 0; u < LONG_CH; ++u) x[u] = q0 + u < nload ? F[base + (f + q0 + u) * sp_] : 0.0;
#pragma unroll
      for (int u = 0; u < LONG_CH; ++u) {
        const int q = q0 + u;
        if (q < nload) {
          const int64_t pos = f + q;
          const double val = q < nint ? fma(-tl, tb.Ls[pos], fma(-tr, tb.Rs[pos], x[u])) : tr;
          int64_t i, j, kk;
          if (axis == 0) { i = pos; j = outer; kk = k; }
          else if (axis == 1) { i = outer; j = pos; kk = k; }
          else { i = k / c1; j = k % c1; kk = pos; }
          epi_store(ep, F, base + pos * sp_, i, j, kk, val);
        }
      }
    }
  }
}

template <typename T, int LB>
__global__ void __launch_bounds__(64 * LONG_WAVES) k_solve_long(LongArgs<T> a) {
  long_body<T, LB>(a, blockIdx.x);
}
template <typename T, int LB>
__global__ void __launch_bounds__(64 * LONG_WAVES) k_solve_long_group(Group<LongArgs<T>> g) {
  int j, b;
  group_locate(g, j, b);
  long_body<T, LB>(g.job[j], b);
}

// Sequential Thomas per line (lines longer than kLongBlocks partitions of
// 64): one thread per line, elimination in place in F.
template <typename T>
__global__ void k_solve_seq(double *F, int64_t nlines, int64_t c, int axis, int64_t c1, int64_t c2,
                            SolveDev tb, Epi<T> ep) {
  const int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (L >= nlines) return;
  int64_t base, step, o1, o2;  // o1, o2: the two fixed coordinates
  if (axis == 2) { base = L * c; step = 1; o1 = L / c1; o2 = L % c1; }
  else if (axis == 1) { o1 = L / c2; o2 = L % c2; base = o1 * c1 * c2 + o2; step = c2; }
  else { o1 = L / c2; o2 = L % c2; base = o1 * c2 + o2; step = c1 * c2; }
  double prev = F[base];
  for (int64_t q = 1; q < c; ++q) {
    double v = fma(-tb.w[q], prev, F[base + q * step]);
    F[base + q * step] = v;
    prev = v;
  }
  double nxt = 0.0;
  for (int64_t q = c - 1; q >= 0; --q) {
    double v = (q == c - 1) ? F[base + q * step] * tb.invb[q]
                            : fma(-tb.sup[q], nxt, F[base + q * step]) * tb.invb[q];
    nxt = v;
    int64_t i, j, k;
    if (axis == 2) { i = o1; j = o2; k = q; }
    else if (axis == 1) { i = o1; j = q; k = o2; }
    else { i = q; j = o1; k = o2; }
    epi_store(ep, F, base + q * step, i, j, k, v);
  }
}

// --------------------------------------------------- recomposition kernels

// Recomposition of one level: every node of the level grid gets its stored
// coefficient plus the multilinear interpolant of the coarse values
// (U_c = stored coarse grid - z).  A workgroup owns a tile of fine nodes in
// dims (1, 2) -- whole rows wherever they fit, so that each workgroup streams
// long contiguous row segments and no cache line is split between two
// workgroups except at a segment's ends -- and a chunk of coarse planes
// along dim 0.  It walks plane pairs like k_loadvec: the coarse values of the
// tile (with a one-node halo) are staged in LDS per coarse plane, the
// interpolant of each owned node stays in registers for the fine plane after
// it, and the next pair's coefficients and coarse values are prefetched into
// registers.  Each coefficient is read once and each output written once.
constexpr int RC_THR = 256;  // threads of a reconstruct workgroup
constexpr int RC_EPT = 5;    // fine nodes per thread per plane
constexpr int RC_EPC = 3;  // staged coarse nodes per thread
constexpr int RC_NE = RC_EPT * RC_THR, RC_NC = RC_EPC * RC_THR;

template <typename T>
struct ReconArgs {
  const T *coef;  // stored coefficients (level grid positions); nullptr: all zero
  Map3 cmap;
  const T *uc;    // coarse values U_c, compact next-level grid
  T *dst;         // level grid, compact
  int64_t m0, m1, m2, c0, c1, c2;
  const double *r0, *r1, *r2;
  int64_t TI;
  int TJ, TK;     // coarse rows / columns of a tile
  int gx, gy, gz;
};

template <typename T, bool NODALC, bool CO0, bool CO1, bool CO2>
__device__ __forceinline__ void reconstruct_body(const ReconArgs<T> &a, const int tile) {
  using A = Acc<T>;
  constexpr int SJ = CO1 ? 2 : 1, SK = CO2 ? 2 : 1;
  const int FJ = SJ * a.TJ, FK = SK * a.TK;  // owned fine tile (host: FJ * FK <= RC_NE)
  const int NE = FJ * FK;
  const int CK = a.TK + (CO2 ? 1 : 0);       // coarse tile with halo (host: CJ * CK <= RC_NC)
  const int NC = (a.TJ + (CO1 ? 1 : 0)) * CK;
  __shared__ A sU[2][RC_NC];  // coarse values of the current / previous coarse plane
  // interpolation weights of the tile's rows, then of its columns (FJ + FK <= RC_NE + 1)
  __shared__ A sR[RC_NE + 1];
  A *sR1 = sR, *sR2 = sR + FJ;
  // tables read inside the plane loop come from LDS or are loaded one step
  // ahead with the prefetch (see k_loadvec)
  __shared__ int64_t sPO[NODALC ? LV_MAXP : 1];  // nodal plane offsets of the coefficients
  __shared__ A sR0[2];                      // dim-0 weight of the step's fine plane

  const int tid = threadIdx.x;
  const int tx = tile % a.gx, ty = (tile / a.gx) % a.gy, tz = tile / (a.gx * a.gy);
  const int64_t J0 = (int64_t)ty * a.TJ, K0 = (int64_t)tx * a.TK;
  const int64_t I0 = (int64_t)tz * a.TI;
  const int64_t I1 = min(I0 + a.TI, a.c0);
  const bool lastJ = J0 + a.TJ >= a.c1, lastK = K0 + a.TK >= a.c2, lastI = I1 >= a.c0;
  const int64_t fj0 = SJ * J0, fje = lastJ ? a.m1 : SJ * (J0 + a.TJ);
  const int64_t fk0 = SK * K0, fke = lastK ? a.m2 : SK * (K0 + a.TK);
  const int64_t oib = (CO0 ? 2 : 1) * I0, oie = lastI ? a.m0 : (CO0 ? 2 : 1) * I1;

  enum : unsigned { F_IN = 1, F_C1 = 2, F_C2 = 4 };
  unsigned flags = 0;
  int colC[RC_EPT], colD[RC_EPT];
  int lo[RC_EPT];  // coarse-tile index of the lower corner
  int jk[RC_EPT];  // tile row << 16 | tile column
#pragma unroll
  for (int i = 0; i < RC_EPT; ++i) {
    const int e = tid + i * RC_THR;
    const int j = e / FK, k = e % FK;
    const int64_t gj = fj0 + j, gk = fk0 + k;
    unsigned f = 0;
    colC[i] = colD[i] = lo[i] = jk[i] = 0;
    if (e < NE && gj < fje && gk < fke) {
      f |= F_IN;
      const bool c1 = coarse_pos<CO1>(gj, a.m1), c2 = coarse_pos<CO2>(gk, a.m2);
      if (c1) f |= F_C1;
      if (c2) f |= F_C2;
      const int64_t a1 = c1 ? coarse_idx<CO1>(gj, a.m1, a.c1) : (gj - 1) / 2;
      const int64_t a2 = c2 ? coarse_idx<CO2>(gk, a.m2, a.c2) : (gk - 1) / 2;
      lo[i] = (int)((a1 - J0) * CK + (a2 - K0));
      colC[i] = (int)(NODALC ? a.cmap.t1[gj] + a.cmap.t2[gk] : gj * a.m2 + gk);
      colD[i] = (int)(gj * a.m2 + gk);
      jk[i] = (j << 16) | k;
    }
    flags |= f << (3 * i);
  }
  auto flag_of = [&](int i) -> unsigned { return (flags >> (3 * i)) & 7u; };
  for (int j = tid; j < FJ; j += RC_THR) {
    const int64_t gj = fj0 + j;
    sR1[j] = (CO1 && gj < a.m1 && !coarse_pos<CO1>(gj, a.m1)) ? a.r1[gj] : A(0);
  }
  for (int k = tid; k < FK; k += RC_THR) {
    const int64_t gk = fk0 + k;
    sR2[k] = (CO2 && gk < a.m2 && !coarse_pos<CO2>(gk, a.m2)) ? a.r2[gk] : A(0);
  }

  // coarse-tile elements this thread stages
  int ucol[RC_EPC];
#pragma unroll
  for (int i = 0; i < RC_EPC; ++i) {
    const int e = tid + i * RC_THR;
    const int64_t J = J0 + e / CK, K = K0 + e % CK;
    ucol[i] = (e < NC && J < a.c1 && K < a.c2) ? (int)(J * a.c2 + K) : -1;
  }
  const int64_t pw0 = CO0 ? max<int64_t>(0, 2 * I0 - 1) : I0;  // plane window (host: 2 TI + 2 <= LV_MAXP)
  if (NODALC)
    for (int q = tid; q < LV_MAXP; q += RC_THR) sPO[q] = (pw0 + q < a.m0) ? a.cmap.t0[pw0 + q] : 0;
  __syncthreads();

  // branch-free loads (invalid elements read a valid node and are never used);
  // a level whose coefficients are dropped (partial recomposition) reads none
  auto fetchC = [&](A (&v)[RC_EPT], int64_t p) {
    if (!a.coef) {
#pragma unroll
      for (int i = 0; i < RC_EPT; ++i) v[i] = A(0);
      return;
    }
    const T *base = a.coef + (NODALC ? sPO[p - pw0] : p * a.m1 * a.m2);
#pragma unroll
    for (int i = 0; i < RC_EPT; ++i) v[i] = (A)base[colC[i]];
  };
  auto fetchU = [&](A (&v)[RC_EPC], int64_t cp) {
    const T *base = a.uc + cp * a.c1 * a.c2;
#pragma unroll
    for (int i = 0; i < RC_EPC; ++i) v[i] = (A)base[ucol[i] >= 0 ? ucol[i] : 0];
  };
  double kv = 0.0;  // dim-0 weight of the fine plane of a step (thread 0), loaded a step ahead
  auto fetch_r0 = [&](int64_t pa) { kv = a.r0 ? a.r0[pa >= 0 ? pa : 0] : A(0); };
  // interpolant (dims 1, 2) of owned element i from the staged coarse tile s
  auto interp2 = [&](const A *s, int i) -> A {
    const unsigned f = flag_of(i);
    if (!(f & F_IN)) return A(0);
    const int l = lo[i];
    const bool c1 = f & F_C1, c2 = f & F_C2;
    if (c1 && c2) return s[l];
    const A rk = sR2[jk[i] & 0xffff], rj = sR1[jk[i] >> 16];
    if (c1) return lerp(s[l], s[l + 1], rk);
    if (c2) return lerp(s[l], s[l + CK], rj);
    return lerp(lerp(s[l], s[l + 1], rk), lerp(s[l + CK], s[l + CK + 1], rk), rj);
  };

  // steps: with dim 0 coarsened, step I covers (a = 2I+1, b = 2I+2) for I in
  // [I0-1, I1-1]; plane a of the first step is not owned.  Without, step I
  // is plane I.
  const int64_t sbeg = CO0 ? I0 - 1 : I0, send = I1;
  auto planes = [&](int64_t I, int64_t &pa, int64_t &pb) {
    if (!CO0) { pa = -1; pb = I; return; }
    pa = 2 * I + 1;
    pb = 2 * I + 2;
    if (!(pa >= 0 && pa < a.m0) || I < I0) pa = -1;
    if (!(pb >= 0 && pb < a.m0)) pb = -1;
    if (pa >= 0 && pb < 0) { pb = pa; pa = -1; }  // last plane of an even extent is coarse
  };

  A ca[RC_EPT], cb[RC_EPT], uv[RC_EPC];
  A piPrev[RC_EPT], piNext[RC_EPT];
#pragma unroll
  for (int i = 0; i < RC_EPT; ++i) piPrev[i] = piNext[i] = A(0);
  {
    int64_t pa, pb;
    planes(sbeg, pa, pb);
    if (pb >= 0) { fetchC(cb, pb); fetchU(uv, coarse_idx<CO0>(pb, a.m0, a.c0)); }
    if (pa >= 0) fetchC(ca, pa);
    fetch_r0(pa);
  }
  int buf = 0;
  for (int64_t I = sbeg; I < send; ++I) {
    int64_t pa, pb;
    planes(I, pa, pb);
    A *s = sU[buf];
    if (pb >= 0) {
#pragma unroll
      for (int i = 0; i < RC_EPC; ++i) {
        const int e = tid + i * RC_THR;
        if (e < NC) s[e] = ucol[i] >= 0 ? uv[i] : A(0);
      }
    }
    if (tid == 0) sR0[buf] = kv;
    A xb[RC_EPT], xa[RC_EPT];
#pragma unroll
    for (int i = 0; i < RC_EPT; ++i) {
      xb[i] = cb[i];
      xa[i] = ca[i];
    }
    if (I + 1 < send) {
      int64_t qa, qb;
      planes(I + 1, qa, qb);
      if (qb >= 0) { fetchC(cb, qb); fetchU(uv, coarse_idx<CO0>(qb, a.m0, a.c0)); }
      if (qa >= 0) fetchC(ca, qa);
      fetch_r0(qa);
    }
    __syncthreads();
    if (pb >= 0) {
      const bool own_p = pb >= oib && pb < oie;
      const int64_t po = pb * a.m1 * a.m2;
#pragma unroll
      for (int i = 0; i < RC_EPT; ++i) {
        piNext[i] = interp2(s, i);
        const unsigned f = flag_of(i);
        if (own_p && (f & F_IN)) {
          const bool coarse_all = coarse_pos<CO0>(pb, a.m0) && (f & F_C1) && (f & F_C2);
          a.dst[po + colD[i]] = (T)(coarse_all ? piNext[i] : xb[i] + piNext[i]);
        }
      }
    }
    if (pa >= 0) {
      const bool own_p = pa >= oib && pa < oie;
      const int64_t po = pa * a.m1 * a.m2;
#pragma unroll
      for (int i = 0; i < RC_EPT; ++i)
        if (own_p && (flag_of(i) & F_IN))
          a.dst[po + colD[i]] = (T)(xa[i] + lerp(piPrev[i], piNext[i], sR0[buf]));
    }
#pragma unroll
    for (int i = 0; i < RC_EPT; ++i) piPrev[i] = piNext[i];
    buf ^= 1;
  }
}

template <typename T, bool NODALC, bool CO0, bool CO1, bool CO2>
__global__ void __launch_bounds__(RC_THR) k_reconstruct(ReconArgs<T> a) {
  reconstruct_body<T, NODALC, CO0, CO1, CO2>(a, xcd_tile(blockIdx.x, a.gx * a.gy * a.gz));
}
template <typename T, bool NODALC, bool CO0, bool CO1, bool CO2>
__global__ void __launch_bounds__(RC_THR) k_reconstruct_group(Group<ReconArgs<T>> g) {
  int j, b;
  group_locate(g, j, b);
  reconstruct_body<T, NODALC, CO0, CO1, CO2>(g.job[j], b);
}

template <typename T>
__global__ void __launch_bounds__(256) k_gather(const T *src, Map3 smap, T *dst, int64_t m0, int64_t m1,
                                                int64_t m2) {
  const int64_t n = m0 * m1 * m2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e % m2, row = e / m2, j = row % m1, i = row / m1;
    dst[e] = src[moff(smap, i, j, k)];
  }
}

// ------------------------------------------------------------ 4-D levels
//
// A 4-D field is refactored as one more tensor-product dimension (Sec.
// III-D): dim 0 (time) coarsens with the same nesting rule, interpolation is
// multilinear in all four dims, and the load vector and the correction solves
// act along time as along space.  Space is processed per time slice by the
// 3-D kernels (time over launches), time by the kernels below with the three
// space dims flattened.

// Load vector along time: row J of P^T M along dim 0 applied to the per-slice
// space load vectors G (tm slices of ncs entries),
// F[J] = sum_o W[5 J + o] G[2 J - 2 + o].  A thread walks a run of TL_JC
// consecutive J for one space entry with a five-slice register window, so each
// slice of G is read about once.
constexpr int TL_JC = 8;
__global__ void __launch_bounds__(256) k_tload(const double *__restrict__ G, int64_t tm,
                                               const double *__restrict__ W, double *__restrict__ F,
                                               int64_t ct, int64_t ncs) {
  const int64_t x = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (x >= ncs) return;
  const int64_t nrun = (ct + TL_JC - 1) / TL_JC;
  for (int64_t run = blockIdx.y; run < nrun; run += gridDim.y) {
    const int64_t J0 = run * TL_JC, J1 = min(J0 + TL_JC, ct);
    auto ld = [&](int64_t p) -> double { return (p >= 0 && p < tm) ? G[p * ncs + x] : 0.0; };
    double g0 = ld(2 * J0 - 2), g1 = ld(2 * J0 - 1), g2 = ld(2 * J0), g3 = ld(2 * J0 + 1), g4 = ld(2 * J0 + 2);
    for (int64_t J = J0; J < J1; ++J) {
      const double *w = W + J * 5;
      double f = w[0] * g0;
      f = fma(w[1], g1, f);
      f = fma(w[2], g2, f);
      f = fma(w[3], g3, f);
      f = fma(w[4], g4, f);
      F[J * ncs + x] = f;
      g0 = g2;
      g1 = g3;
      g2 = g4;
      g3 = ld(2 * J + 3);
      g4 = ld(2 * J + 4);
    }
  }
}

// Neighbours of level position i along one space dim for the interpolant:
// the coarse positions on either side and the weight of the right one
// (both the node itself, weight 0, where i is coarse or the dim not
// coarsened).  Level-grid positions (LVL) or coarse-grid indices.
template <bool LVL>
__device__ __forceinline__ void nb_dim(int64_t i, int64_t m, int64_t c, bool co, const double *r, int64_t &lo,
                                       int64_t &hi, double &w) {
  if (!co) {
    lo = hi = i;
    w = 0.0;
  } else if (i % 2 == 0 || i == m - 1) {
    lo = hi = LVL ? i : (i == m - 1 ? c - 1 : i / 2);
    w = 0.0;
  } else {
    lo = LVL ? i - 1 : (i - 1) / 2;
    hi = LVL ? i + 1 : (i + 1 == m - 1 ? c - 1 : (i + 1) / 2);
    w = r[i];
  }
}

template <typename T, typename TS = T>
struct TfineArgs {
  const TS *src;         // decompose: compact level grid; recompose: stored coefficients (finest layout)
  T *dst;                // decompose: output (finest layout); recompose: compact level grid
  const TS *crs;         // coarse values: the level grid (decompose) or the compact coarse grid (recompose)
  Map3 fmap;             // space map of the finest-layout side
  const int64_t *tnod;   // finest time index of each level time position
  const double *rt;      // time interpolation weights of the level
  int64_t S0;            // nodes of a finest time slice
  int64_t tm, m0, m1, m2, c0, c1, c2;
  int co0, co1, co2;
  const double *r0, *r1, *r2;
};

// The time-fine slices of a 4-D level: every node of slice t = 2q + 1 holds a
// coefficient, and its interpolant is the space-multilinear interpolant of the
// time lerp (weight rt[t] of the later slice) of the coarse values of slices
// t - 1 and t + 1.  Decompose: coefficient = value - interpolant; recompose:
// value = coefficient + interpolant.  A workgroup takes TF_ROWS fine rows of
// TF_PI consecutive planes of one such slice, TF_CH columns at a time, and
// marches along dim 0: the time lerp of each coarse plane it needs is staged
// once in one of two LDS slots (the coarse rows and columns the fine rows
// need), and a fine plane between two coarse planes lerps the two slots along
// dim 0 before the bilinear interpolation in dims 1 and 2.  Each thread takes
// one fine column of every row.
constexpr int TF_THR = 256;
constexpr int TF_ROWS = 8;   // fine rows (dim 1) per workgroup
constexpr int TF_CH = 256;   // fine columns (dim 2) per pass, one per thread
constexpr int TF_PI = 16;    // fine planes (dim 0) per workgroup
constexpr int TF_PITCH = TF_CH + 2;
template <typename T, typename TS, bool DEC>
__global__ void __launch_bounds__(TF_THR) k_tfine(TfineArgs<T, TS> a) {
  __shared__ double sT[2][TF_ROWS * TF_PITCH];
  const int tid = threadIdx.x;
  const int64_t sm = a.m0 * a.m1 * a.m2;
  const int64_t nf = (a.tm - 1) / 2;  // odd positions below the last
  const int64_t ngr = (a.m1 + TF_ROWS - 1) / TF_ROWS;
  const int64_t npc = (a.m0 + TF_PI - 1) / TF_PI;
  // strides of the array holding the coarse values (DEC: the level grid)
  const int64_t s1 = DEC ? a.m2 : a.c2, s0 = s1 * (DEC ? a.m1 : a.c1), ss = s0 * (DEC ? a.m0 : a.c0);
  // array position of coarse index X along a dim (DEC: its level position)
  auto cpos = [](int64_t X, int64_t m, int64_t c, int co) -> int64_t {
    return (DEC && co) ? (X == c - 1 ? m - 1 : 2 * X) : X;
  };
  for (int64_t job = blockIdx.x; job < nf * npc * ngr; job += gridDim.x) {
    const int64_t q = job / (npc * ngr), rem = job - q * (npc * ngr);
    const int64_t pc = rem / ngr, g = rem - pc * ngr;
    const int64_t j0 = g * TF_ROWS, j1 = min(j0 + TF_ROWS, a.m1);
    const int64_t i0 = pc * TF_PI, i1 = min(i0 + TF_PI, a.m0);
    const int64_t t = 2 * q + 1;
    const int nr = (int)(j1 - j0);
    int64_t J0, J1, lo, hi;
    double w;
    nb_dim<false>(j0, a.m1, a.c1, a.co1, a.r1, J0, hi, w);
    nb_dim<false>(j1 - 1, a.m1, a.c1, a.co1, a.r1, lo, J1, w);
    const int nJ = (int)(J1 - J0 + 1);
    const double rt = a.rt[t];
    // the earlier and later coarse slices (level positions t -/+ 1, or coarse indices q, q + 1)
    const TS *cl = a.crs + (DEC ? t - 1 : q) * ss, *cr = a.crs + (DEC ? t + 1 : q + 1) * ss;
    const int64_t fslice = a.tnod[t] * a.S0;  // this slice in the finest layout
    for (int64_t k0 = 0; k0 < a.m2; k0 += TF_CH) {
      const int64_t k1 = min(k0 + TF_CH, a.m2);
      const int nk = (int)(k1 - k0);
      int64_t K0, K1;
      nb_dim<false>(k0, a.m2, a.c2, a.co2, a.r2, K0, hi, w);
      nb_dim<false>(k1 - 1, a.m2, a.c2, a.co2, a.r2, lo, K1, w);
      const int nK = (int)(K1 - K0 + 1);
      // this thread's column (a column past the end reads the last one and is not stored)
      const int64_t k = k0 + min(tid, nk - 1);
      const int64_t fcol = a.fmap.t0 ? a.fmap.t2[k] : k;
      int64_t kl, kh;
      double wk;
      nb_dim<false>(k, a.m2, a.c2, a.co2, a.r2, kl, kh, wk);
      const int ql = (int)(kl - K0), qh = (int)(kh - K0);
      const int64_t oc = cpos(K0 + min(tid, nK - 1), a.m2, a.c2, a.co2);  // staged coarse column
      int64_t slot[2] = {-1, -1};  // coarse plane held by each LDS slot (the same in every thread)
      // row jr of plane i in the finest layout, and in the compact level grid
      auto frow = [&](int64_t i, int jr) -> int64_t {
        const int64_t j = j0 + min(jr, nr - 1);
        return fslice + (a.fmap.t0 ? a.fmap.t0[i] + a.fmap.t1[j] : i * a.fmap.s0 + j * a.fmap.s1);
      };
      auto lrow = [&](int64_t i, int jr) -> int64_t { return t * sm + (i * a.m1 + j0 + min(jr, nr - 1)) * a.m2; };
      // fine values of a plane; the recomposition loads the next plane's
      // while this one is interpolated (measured faster there, not in the
      // decomposition, whose staging then also waits for them)
      constexpr bool PF = !DEC;
      auto loadx = [&](int64_t i, TS (&xx)[TF_ROWS]) {
#pragma unroll
        for (int jr = 0; jr < TF_ROWS; ++jr) xx[jr] = a.src[DEC ? lrow(i, jr) + k : frow(i, jr) + fcol];
      };
      TS x[TF_ROWS];
      if constexpr (PF) loadx(i0, x);
      for (int64_t i = i0; i < i1; ++i) {
        int64_t l0, h0;
        double w0;
        nb_dim<DEC>(i, a.m0, a.c0, a.co0, a.r0, l0, h0, w0);
        TS xn[TF_ROWS];
        if constexpr (PF) {
          if (i + 1 < i1) {
            loadx(i + 1, xn);
          } else {
#pragma unroll
            for (int jr = 0; jr < TF_ROWS; ++jr) xn[jr] = x[jr];
          }
        } else {
          loadx(i, x);
        }
        // coarse planes l0 and h0 into the slots (a slot is refilled only
        // after the previous plane's barrier: nothing reads it any more)
        int sl = slot[0] == l0 ? 0 : (slot[1] == l0 ? 1 : -1);
        int sh = slot[0] == h0 ? 0 : (slot[1] == h0 ? 1 : -1);
        auto stage = [&](int sidx, int64_t p) {
          if (tid < nK) {
            TS vl[TF_ROWS], vr[TF_ROWS];
#pragma unroll
            for (int jr = 0; jr < TF_ROWS; ++jr) {
              const int64_t o = p * s0 + cpos(J0 + min(jr, nJ - 1), a.m1, a.c1, a.co1) * s1 + oc;
              vl[jr] = cl[o];
              vr[jr] = cr[o];
            }
#pragma unroll
            for (int jr = 0; jr < TF_ROWS; ++jr)
              if (jr < nJ) sT[sidx][jr * TF_PITCH + tid] = lerp((double)vl[jr], (double)vr[jr], rt);
          }
          slot[sidx] = p;
        };
        if (sl < 0) {
          sl = sh == 0 ? 1 : 0;
          stage(sl, l0);
        }
        if (sh < 0) {
          if (h0 == l0) {
            sh = sl;
          } else {
            sh = 1 - sl;
            stage(sh, h0);
          }
        }
        __syncthreads();
        if (tid < nk) {
          const double *Tl = sT[sl], *Th = sT[sh];
          const bool mid = h0 != l0;  // between two coarse planes: lerp along dim 0
          auto val = [&](int jj, int qq) -> double {
            const double v = Tl[jj * TF_PITCH + qq];
            return mid ? lerp(v, Th[jj * TF_PITCH + qq], w0) : v;
          };
#pragma unroll
          for (int jr = 0; jr < TF_ROWS; ++jr) {
            if (jr >= nr) break;
            int64_t jl, jh;
            double wj;
            nb_dim<false>(j0 + jr, a.m1, a.c1, a.co1, a.r1, jl, jh, wj);
            const int rl = (int)(jl - J0), rh = (int)(jh - J0);
            const double pi = lerp(lerp(val(rl, ql), val(rl, qh), wk), lerp(val(rh, ql), val(rh, qh), wk), wj);
            if (DEC)
              a.dst[frow(i, jr) + fcol] = (T)((double)x[jr] - pi);
            else
              a.dst[lrow(i, jr) + k] = (T)((double)x[jr] + pi);
          }
        }
        __syncthreads();
        if constexpr (PF) {
#pragma unroll
          for (int jr = 0; jr < TF_ROWS; ++jr) x[jr] = xn[jr];
        }
      }
    }
  }
}

// The coarsest grid of a 4-D field between its nodal positions and a compact
// grid (TO_NODAL: compact -> nodal), converted to the destination's type.
template <typename TS, typename TD, bool TO_NODAL>
__global__ void __launch_bounds__(256) k_nodal4(const TS *src, TD *dst, Map3 nmap, const int64_t *tnod, int64_t S0,
                                                int64_t tm, int64_t m0, int64_t m1, int64_t m2) {
  const int64_t n = tm * m0 * m1 * m2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e % m2, r1 = e / m2, j = r1 % m1, r0 = r1 / m1, i = r0 % m0, t = r0 / m0;
    const int64_t o = tnod[t] * S0 + moff(nmap, i, j, k);
    if (TO_NODAL)
      dst[o] = (TD)src[e];
    else
      dst[e] = (TD)src[o];
  }
}

// Class-contiguous layout of a nodal representation: the coarsest grid's
// values, then each level's coefficient class (its nodes that are not in the
// next coarser grid) from the coarsest level to the finest, each in C order
// of its level grid.  A node's place in its class is its level-grid index
// minus the number of nodes before it that belong to the coarser grid, which
// has a closed form: coarse positions along a coarsened dimension are the
// even ones and the last, so (x + 1) / 2 of them precede position x.
// EXPORT gathers the class from the nodal array; otherwise it scatters back.
template <typename T, bool EXPORT>
__global__ void __launch_bounds__(256) k_classes(const T *__restrict__ src, T *__restrict__ dst, Map3 nmap,
                                                 int64_t m0, int64_t m1, int64_t m2, int64_t c1, int64_t c2,
                                                 int co0, int co1, int co2, int64_t class_off, int coarsest) {
  const int64_t n = m0 * m1 * m2;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e % m2, row = e / m2, j = row % m1, i = row / m1;
    int64_t pos = e;
    if (!coarsest) {
      const bool ci = !co0 || (i % 2 == 0) || i == m0 - 1;
      const bool cj = !co1 || (j % 2 == 0) || j == m1 - 1;
      const bool ck = !co2 || (k % 2 == 0) || k == m2 - 1;
      if (ci && cj && ck) continue;  // belongs to the coarser grid
      const int64_t ni = co0 ? (i + 1) / 2 : i, nj = co1 ? (j + 1) / 2 : j, nk = co2 ? (k + 1) / 2 : k;
      pos = e - (ni * c1 * c2 + (ci ? nj * c2 + (cj ? nk : 0) : 0));
    }
    const int64_t node = moff(nmap, i, j, k);
    if (EXPORT) dst[class_off + pos] = src[node];
    else dst[node] = src[class_off + pos];
  }
}

// Streaming copy of 16-byte words, one word per thread over a grid that
// covers the array, with nontemporal loads and stores (the single-pass
// bandwidth probe).  On MI355X this form measured fastest of the copies
// tried: a grid-stride loop over a few thousand workgroups reaches about 70%
// of its rate, since the waves in flight then touch addresses far apart.
typedef unsigned int probe_word __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_copy_probe(const probe_word *__restrict__ src,
                                                   probe_word *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// ------------------------------------------------------------ tail kernels
//
// The coarsest levels hold a few thousand nodes; one launch per operator
// there costs more than the work.  One workgroup of TAIL_THR threads runs all
// of them from LDS in a single launch per direction, with the same operators
// as the grid-wide kernels: coefficients (value minus multilinear
// interpolant), the load vector f = (P^T M) U per coarsened dimension from
// the plan's taps, and each coarse line solved with whole-line Thomas factors
// by one thread.  Every table of the tail levels is copied into LDS first, so
// that the serial chain of phases waits on LDS, not on global memory.  Three
// LDS grids of kTailNodes doubles rotate between the roles of level grid,
// tap-pass input and output.

constexpr int TAIL_THR = 1024;
constexpr int TAIL_PER = (kTailNodes + TAIL_THR - 1) / TAIL_THR;  // grid nodes per thread

struct TailArgs {
  const TailLevel *lv;   // [nt + 1] descriptors, level tail_start first
  const int64_t *off;    // packed nodal offsets
  const double *dbl;     // packed FP64 tables
  int noff, ndbl, nt;
  int t_drop;            // recomposition: tail levels below this one take zero coefficients
};

// LDS of a tail kernel: three level grids and the packed tables.
struct TailSmem {
  double g[3 * kTailNodes];
  double d[kTailDoubles];
  int64_t o[kTailOffsets];
};

// t / e for 0 <= t < 2^13 and 1 <= e <= 65: the single-precision quotient
// of t + 0.5 lies at least 0.5 / e from an integer, far more than its
// rounding error (a few units in 2^-22 relative), so truncation is exact.
__device__ __forceinline__ int tail_div(int t, int e) {
  return (int)(((float)t + 0.5f) * __builtin_amdgcn_rcpf((float)e));
}
__device__ __forceinline__ void tail_split(int t, int e1, int e2, int &i, int &j, int &k) {
  const int r = tail_div(t, e2);
  k = t - r * e2;
  i = tail_div(r, e1);
  j = r - i * e1;
}

__device__ __forceinline__ void tail_load_tables(TailSmem &sm, const TailArgs &a) {
  for (int t = threadIdx.x; t < a.ndbl; t += TAIL_THR) sm.d[t] = a.dbl[t];
  for (int t = threadIdx.x; t < a.noff; t += TAIL_THR) sm.o[t] = a.off[t];
}

// y = (P^T M) x along `axis` of an (e0, e1, e2) grid; y has extent c there.
__device__ __forceinline__ void tail_taps(const double *x, double *y, const int e[3], int axis, int c,
                                          const double *W) {
  int oe[3] = {e[0], e[1], e[2]};
  oe[axis] = c;
  const int n = oe[0] * oe[1] * oe[2];
  const int m = e[axis];
  const int st = axis == 0 ? e[1] * e[2] : (axis == 1 ? e[2] : 1);
  for (int t = threadIdx.x; t < n; t += TAIL_THR) {
    int i, j, k;
    tail_split(t, oe[1], oe[2], i, j, k);
    const int J = axis == 0 ? i : (axis == 1 ? j : k);
    if (axis == 0) i = 0;
    else if (axis == 1) j = 0;
    else k = 0;
    const int base = (i * e[1] + j) * e[2] + k;
    double acc = 0.0;
#pragma unroll
    for (int o = 0; o < kTaps; ++o) {
      const int q = 2 * J - 2 + o;
      if (q >= 0 && q < m) acc = fma(W[J * kTaps + o], x[base + q * st], acc);
    }
    y[t] = acc;
  }
}

// Solves M z = f along `axis` of the (c0, c1, c2) grid F in place.
__device__ __forceinline__ void tail_solve(double *F, const int ce[3], int axis, const double *sup,
                                           const double *tw, const double *tinvb) {
  const int c = ce[axis];
  const int nlines = ce[0] * ce[1] * ce[2] / c;
  const int st = axis == 0 ? ce[1] * ce[2] : (axis == 1 ? ce[2] : 1);
  for (int t = threadIdx.x; t < nlines; t += TAIL_THR) {
    int base;
    if (axis == 0) base = t;
    else if (axis == 1) {
      const int q = tail_div(t, ce[2]);
      base = q * ce[1] * ce[2] + (t - q * ce[2]);
    } else base = t * ce[2];
    double prev = F[base];
    for (int q = 1; q < c; ++q) {
      prev = fma(-tw[q], prev, F[base + q * st]);
      F[base + q * st] = prev;
    }
    double x = prev * tinvb[c - 1];
    F[base + (c - 1) * st] = x;
    for (int q = c - 2; q >= 0; --q) {
      x = fma(-sup[q], x, F[base + q * st]) * tinvb[q];
      F[base + q * st] = x;
    }
  }
}

// Load vector of the level grid x (extents L.m) along every coarsened
// dimension, then the correction solves; returns the buffer (y0 or y1) that
// holds the result (extents L.c).
__device__ __forceinline__ double *tail_project(const TailLevel &L, const double *sd, const double *x,
                                                double *y0, double *y1) {
  int e[3] = {L.m[0], L.m[1], L.m[2]};
  const double *cur = x;
  double *nxt = y0, *oth = y1;
  for (int ax = 2; ax >= 0; --ax) {
    if (!L.co[ax]) continue;
    tail_taps(cur, nxt, e, ax, L.c[ax], sd + L.W[ax]);
    __syncthreads();
    e[ax] = L.c[ax];
    cur = nxt;
    nxt = oth;
    oth = (double *)cur;
  }
  double *F = (double *)cur;
  for (int ax = 0; ax < kDims; ++ax) {
    if (!L.co[ax]) continue;
    tail_solve(F, L.c, ax, sd + L.sup[ax], sd + L.tw[ax], sd + L.tinvb[ax]);
    __syncthreads();
  }
  return F;
}

__device__ __forceinline__ bool tail_coarse_all(const TailLevel &L, int i, int j, int k) {
  auto cp = [](int g, int m, int co) { return !co || g % 2 == 0 || g == m - 1; };
  return cp(i, L.m[0], L.co[0]) && cp(j, L.m[1], L.co[1]) && cp(k, L.m[2], L.co[2]);
}

// Neighbours and right weight of level position g along one dimension, for
// the interpolant of the coarse values: in the level grid itself (dec) or in
// the compact coarse grid (rec).
template <bool COMPACT>
__device__ __forceinline__ void tail_nb(int g, int m, int c, int co, const double *r, int &lo, int &hi,
                                        double &w) {
  const bool fine = co && (g % 2 == 1) && (g != m - 1);
  w = fine ? r[g] : 0.0;
  if (!COMPACT) {
    lo = fine ? g - 1 : g;
    hi = fine ? g + 1 : g;
  } else if (!co) {
    lo = hi = g;
  } else {
    lo = fine ? (g - 1) / 2 : (g == m - 1 ? c - 1 : g / 2);
    hi = fine ? (g + 1) / 2 : lo;
  }
}

// Multilinear interpolant at (i, j, k) from the grid G (row extents g1, g2):
// dims interpolated 2, then 1, then 0.
template <bool COMPACT>
__device__ __forceinline__ double tail_interp(const TailLevel &L, const double *sd, const double *G, int i,
                                              int j, int k) {
  int lo[3], hi[3];
  double w[3];
  tail_nb<COMPACT>(i, L.m[0], L.c[0], L.co[0], sd + L.r[0], lo[0], hi[0], w[0]);
  tail_nb<COMPACT>(j, L.m[1], L.c[1], L.co[1], sd + L.r[1], lo[1], hi[1], w[1]);
  tail_nb<COMPACT>(k, L.m[2], L.c[2], L.co[2], sd + L.r[2], lo[2], hi[2], w[2]);
  const int g1 = COMPACT ? L.c[1] : L.m[1], g2 = COMPACT ? L.c[2] : L.m[2];
  auto at = [&](int a, int b, int c) { return G[(a * g1 + b) * g2 + c]; };
  auto row = [&](int a, int b) { return lerp(at(a, b, lo[2]), at(a, b, hi[2]), w[2]); };
  auto pl = [&](int a) { return lerp(row(a, lo[1]), row(a, hi[1]), w[1]); };
  return lerp(pl(lo[0]), pl(hi[0]), w[0]);
}

__device__ __forceinline__ int64_t tail_off(const TailLevel &L, const int64_t *so, int i, int j, int k) {
  return so[L.nodal[0] + i] + so[L.nodal[1] + j] + so[L.nodal[2] + k];
}

// Decomposition of levels tail_start .. nlev-1.  src: level grid of the first
// tail level, compact; out: the caller's output array (nodal positions).
template <typename T, typename TS>
struct TailDecJob {
  const TS *src;
  T *out;
  TailArgs a;
};
template <typename T, typename TS>
__device__ __forceinline__ void tail_dec_body(const TS *__restrict__ src, T *__restrict__ out, const TailArgs &a) {
  __shared__ TailSmem sm;
  auto buf = [&](int b) { return sm.g + b * kTailNodes; };
  tail_load_tables(sm, a);
  {
    const TailLevel L = a.lv[0];
    const int n = L.m[0] * L.m[1] * L.m[2];
    for (int t = threadIdx.x; t < n; t += TAIL_THR) sm.g[t] = (double)src[t];
  }
  __syncthreads();
  int ia = 0;  // buffer holding the level grid
  for (int s = 0; s < a.nt; ++s) {
    const TailLevel L = a.lv[s];
    const double *U = buf(ia);
    const int n = L.m[0] * L.m[1] * L.m[2];
    // coefficients of this level
    for (int t = threadIdx.x; t < n; t += TAIL_THR) {
      int i, j, k;
      tail_split(t, L.m[1], L.m[2], i, j, k);
      if (tail_coarse_all(L, i, j, k)) continue;
      out[tail_off(L, sm.o, i, j, k)] = (T)(U[t] - tail_interp<false>(L, sm.d, U, i, j, k));
    }
    // corrected coarse values U_c + z: the next level grid
    const double *F = tail_project(L, sm.d, U, buf((ia + 1) % 3), buf((ia + 2) % 3));
    ia = (F == buf(0)) ? 0 : (F == buf(1) ? 1 : 2);
  }
  // coarsest values to their nodal positions
  const TailLevel Lc = a.lv[a.nt];
  const int n = Lc.m[0] * Lc.m[1] * Lc.m[2];
  const double *V = buf(ia);
  for (int t = threadIdx.x; t < n; t += TAIL_THR) {
    int i, j, k;
    tail_split(t, Lc.m[1], Lc.m[2], i, j, k);
    out[tail_off(Lc, sm.o, i, j, k)] = (T)V[t];
  }
}

// Recomposition of levels nlev-1 .. tail_start.  in: the caller's input
// (nodal positions); dst: level grid of the first tail level, compact.
template <typename T, typename TS>
__global__ void __launch_bounds__(TAIL_THR) k_tail_dec(const TS *__restrict__ src, T *__restrict__ out,
                                                       TailArgs a) {
  tail_dec_body<T, TS>(src, out, a);
}
// one field's tail per workgroup
template <typename T, typename TS>
__global__ void __launch_bounds__(TAIL_THR) k_tail_dec_group(Group<TailDecJob<T, TS>> g) {
  const TailDecJob<T, TS> &q = g.job[blockIdx.x];
  tail_dec_body<T, TS>(q.src, q.out, q.a);
}

template <typename T>
struct TailRecJob {
  const T *in;
  T *dst;
  TailArgs a;
};
template <typename T>
__device__ __forceinline__ void tail_rec_body(const T *__restrict__ in, T *__restrict__ dst, const TailArgs &a) {
  __shared__ TailSmem sm;
  auto buf = [&](int b) { return sm.g + b * kTailNodes; };
  tail_load_tables(sm, a);
  __syncthreads();
  {
    const TailLevel Lc = a.lv[a.nt];
    const int n = Lc.m[0] * Lc.m[1] * Lc.m[2];
    for (int t = threadIdx.x; t < n; t += TAIL_THR) {
      int i, j, k;
      tail_split(t, Lc.m[1], Lc.m[2], i, j, k);
      sm.g[t] = (double)in[tail_off(Lc, sm.o, i, j, k)];
    }
  }
  int ia = 0;  // buffer holding the coarse values of the current step
  for (int s = a.nt - 1; s >= 0; --s) {
    const TailLevel L = a.lv[s];
    const int n = L.m[0] * L.m[1] * L.m[2];
    const bool keep = s >= a.t_drop;  // this level's coefficients are used
    // this level's coefficients (zero at the coarse nodes), all loads in flight at once
    double cf[TAIL_PER];
#pragma unroll
    for (int u = 0; u < TAIL_PER; ++u) {
      const int t = threadIdx.x + u * TAIL_THR;
      cf[u] = 0.0;
      if (keep && t < n) {
        int i, j, k;
        tail_split(t, L.m[1], L.m[2], i, j, k);
        if (!tail_coarse_all(L, i, j, k)) cf[u] = (double)in[tail_off(L, sm.o, i, j, k)];
      }
    }
    double *V = buf(ia);
    int ig = (ia + 1) % 3;
    if (keep) {
      double *Cb = buf((ia + 1) % 3);
#pragma unroll
      for (int u = 0; u < TAIL_PER; ++u) {
        const int t = threadIdx.x + u * TAIL_THR;
        if (t < n) Cb[t] = cf[u];
      }
      __syncthreads();
      const double *F = tail_project(L, sm.d, Cb, buf((ia + 2) % 3), Cb);
      // coarse values before the correction: V - z
      const int nc = L.c[0] * L.c[1] * L.c[2];
      for (int t = threadIdx.x; t < nc; t += TAIL_THR) V[t] -= F[t];
      __syncthreads();
      ig = (F == buf((ia + 1) % 3)) ? (ia + 2) % 3 : (ia + 1) % 3;
    }
    __syncthreads();  // V complete (also after the gather when the first level is dropped)
    // level grid: coefficient plus interpolant of the coarse values
    double *G = buf(ig);
#pragma unroll
    for (int u = 0; u < TAIL_PER; ++u) {
      const int t = threadIdx.x + u * TAIL_THR;
      if (t < n) {
        int i, j, k;
        tail_split(t, L.m[1], L.m[2], i, j, k);
        const double v = cf[u] + tail_interp<true>(L, sm.d, V, i, j, k);
        if (s == 0) dst[t] = (T)v;
        else G[t] = v;
      }
    }
    __syncthreads();
    ia = ig;
  }
}
template <typename T>
__global__ void __launch_bounds__(TAIL_THR) k_tail_rec(const T *__restrict__ in, T *__restrict__ dst,
                                                       TailArgs a) {
  tail_rec_body<T>(in, dst, a);
}
template <typename T>
__global__ void __launch_bounds__(TAIL_THR) k_tail_rec_group(Group<TailRecJob<T>> g) {
  const TailRecJob<T> &q = g.job[blockIdx.x];
  tail_rec_body<T>(q.in, q.dst, q.a);
}

// ------------------------------------------------------------ host launch

// One launch of a field's chain, recorded instead of launched (batched
// entry points): the batch engine launches the recorded jobs of many fields
// that share a kernel and a phase as one grouped launch.
struct RecJob {
  int phase = 0;  // a field's jobs come in increasing phase order
  // grouped launcher of this job's kernel (nullptr: launch `direct` alone)
  void (*group)(const std::vector<const struct RecJob *> &, hipStream_t, size_t, unsigned) = nullptr;
  int gmax = 1;       // jobs per grouped launch at most
  unsigned threads = 0;
  size_t lds = 0;     // dynamic LDS
  int64_t blocks = 0;
  std::vector<unsigned char> args;         // the job's argument struct
  std::function<void(hipStream_t)> direct;  // launch without grouping
  std::string label;
  double bytes = 0.0;
};
struct Rec {
  std::vector<RecJob> jobs;
  // plane-marching kernels take chunks of at least 8 coarse planes, also
  // where a field's tuned shape has shorter ones (batches: a grouped grid of
  // many fields' workgroups fills the device without the short chunks one
  // field alone needs, which re-read 1 or 2 halo planes each)
  bool long_chunks = false;
};

// Launches recorded jobs on `st`: phase by phase; within a phase, the jobs
// of one kernel share launches (in the order they first appear), each launch
// sized for its largest job (a solver workgroup of a job with fewer
// partitions leaves the extra waves idle); jobs with no grouped form run alone.
bool launch_recorded(const Rec &rec, hipStream_t st, std::string &err);
using Unit = std::function<void(hipStream_t)>;
void recorded_units(const Rec &rec, std::vector<Unit> &out);

struct Ctx {
  hipStream_t stream;
  std::string *err;
  bool ok = true;
  // per-launch requests and reports of the plane-marching launches
  int ti_req = 0;     // coarse planes per workgroup requested (0: the built-in rule)
  bool dry = false;   // compute the launch shape only, launch nothing
  int slots_out = 0;  // resident workgroups of the kernel instance chosen
  bool share = false; // the load vector runs beside other work (see launch_loadvec_t)
  int ti_out = 0;     // coarse planes per workgroup chosen
  Rec *rec = nullptr; // record the launches instead (batched entry points)
  int phase = 0;      // phase of the next recorded launch
  void check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess && ok) {
      ok = false;
      *err = std::string(what) + ": " + hipGetErrorString(e);
    }
  }
};

// Phases of a field's chain: level s of a decomposition takes 8s (load
// vector), 8s+1.. (solves); its tail comes last.  A recomposition starts with
// its tail (phase 0), then level s takes kPhaseRecLevel(s) (load vector),
// +1.. (solves) and +4 (reconstruct).
constexpr int kPhaseTail = 8 * (kMaxLevels + 1);
constexpr int phase_dec_level(int s) { return 8 * s; }
constexpr int phase_rec_level(int s) { return 8 * (kMaxLevels + 1 - s); }

// Launches up to Group<J>::N recorded jobs of kernel K as one grid.
template <typename J, void (*K)(Group<J>)>
void group_launch(const std::vector<const RecJob *> &js, hipStream_t st, size_t lds, unsigned threads) {
  Group<J> g;
  std::memset(&g, 0, sizeof(g));
  int64_t tot = 0;
  const int n = (int)js.size();
  for (int i = 0; i < n; ++i) {
    std::memcpy((void *)&g.job[i], js[i]->args.data(), sizeof(J));
    g.start[i] = (int)tot;
    tot += js[i]->blocks;
  }
  g.start[n] = (int)tot;
  g.njobs = n;
  hipLaunchKernelGGL(K, dim3((unsigned)tot), dim3(threads), lds, st, g);
}

// Launches through `direct`, or records the job when the context records.
template <typename J, void (*K)(Group<J>), typename F>
void emit(Ctx &cx, const J &job, int64_t blocks, unsigned threads, size_t lds, std::string label, double bytes,
          F &&direct) {
  if (!cx.rec) {
    direct();
    return;
  }
  RecJob r;
  r.phase = cx.phase;
  r.group = &group_launch<J, K>;
  r.gmax = Group<J>::N;
  r.threads = threads;
  r.lds = lds;
  r.blocks = blocks;
  r.args.resize(sizeof(J));
  std::memcpy(r.args.data(), (const void *)&job, sizeof(J));
  r.label = std::move(label);
  r.bytes = bytes;
  cx.rec->jobs.push_back(std::move(r));
}

// A launch with no grouped form: now, or recorded to run alone in its phase
// (`fn` must own what it uses).
inline void emit_direct(Ctx &cx, std::function<void(hipStream_t)> fn) {
  if (!cx.rec) {
    fn(cx.stream);
    return;
  }
  RecJob r;
  r.phase = cx.phase;
  r.direct = std::move(fn);
  cx.rec->jobs.push_back(std::move(r));
}

template <typename T>
const char *tname() { return sizeof(T) == 8 ? "double" : "float"; }
inline const char *bname(bool b) { return b ? "true" : "false"; }

int64_t grid_1d(int64_t n, int64_t per) {
  int64_t g = (n + per - 1) / per;
  return std::min<int64_t>(std::max<int64_t>(g, 1), 1 << 20);
}

// Compute units of the current device.
int device_cus() {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0, v = 0;
    ncu = (hipGetDevice(&dev) == hipSuccess &&
           hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
              ? v
              : 256;
  }
  return ncu;
}

// Workgroups of `kernel` (`threads` threads, static LDS) resident on the device at once.
int resident_slots(const void *kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb < 1) {
    (void)hipGetLastError();
    nb = 1;
  }
  return nb * device_cus();
}

// Coarse planes per workgroup (TI) for a plane-marching kernel over `tiles`
// tile columns: each chunk of TI planes re-reads `halo` planes, and the
// workgroups run in rounds of `slots` resident ones, so the cost is
// rounds x (TI + halo) plane steps.  The cheapest TI <= maxTI wins; ties go to
// the larger TI (fewer re-read planes).
int64_t pick_chunk(int64_t c0, int64_t tiles, int64_t slots, int halo, int64_t maxTI) {
  int64_t best = 1;
  double best_cost = 1e300;
  for (int64_t TI = 1; TI <= std::min(c0, maxTI); ++TI) {
    const int64_t nwg = tiles * ((c0 + TI - 1) / TI);
    const double cost = (double)((nwg + slots - 1) / slots) * (double)(TI + halo);
    if (cost <= best_cost) {
      best_cost = cost;
      best = TI;
    }
  }
  return best;
}

template <typename T, typename TS, bool DEC, bool NODAL, bool C0, bool C1, bool C2>
void launch_loadvec_t(LoadArgs<T, TS> a, Ctx &cx) {
  static const int slots =
      resident_slots((const void *)k_loadvec<T, TS, DEC, NODAL, C0, C1, C2>, kNTHR<T, DEC, NODAL>);
  a.gy = (int)((a.c1 + kTJ<T, DEC, NODAL> - 1) / kTJ<T, DEC, NODAL>);
  const int64_t tiles = (int64_t)a.gx * a.gy;
  // chunks short enough for the kernel's LDS plane window (2 TI + 3 planes)
  const int64_t maxti = (LV_MAXP - 3) / 2;
  a.TI = cx.ti_req > 0 ? std::min<int64_t>(std::min<int64_t>(cx.ti_req, maxti), a.c0)
                       : pick_chunk(a.c0, tiles, slots, C0 ? 2 : 0, maxti);
  if (cx.rec && cx.rec->long_chunks) a.TI = std::max<int64_t>(a.TI, std::min<int64_t>(8, a.c0));
  if (cx.share && !NODAL) {
    // Beside other work (the recomposition's finest load vector on the helper
    // stream): one round of workgroups that leaves about 5% of the resident
    // slots free, so that the coarser levels' kernels find room at once
    // instead of waiting for these long-lived workgroups to retire (measured
    // at 513^3: FP64 recomposition 1.354 -> 1.305 ms, FP32 0.886 -> 0.855).
    // The chunk length only moves work between workgroups.
    const int64_t gz = std::max<int64_t>(1, (int64_t)(0.95 * (double)slots / (double)tiles));
    a.TI = (a.c0 + gz - 1) / gz;
  }
  cx.slots_out = slots;
  cx.ti_out = (int)a.TI;
  if (cx.dry) return;
  a.gz = (int)((a.c0 + a.TI - 1) / a.TI);
  const dim3 grid((unsigned)(tiles * a.gz));
  double bytes = 0.0;
  if (timing_enabled() || cx.rec) {
    const double nl = (double)a.m0 * a.m1 * a.m2, nc = (double)a.c0 * a.c1 * a.c2;
    // recompose: read the coefficients, write f
    // decompose: read the level grid, write the coefficients and f
    if (DEC && a.out == nullptr) bytes = nl * sizeof(TS) + 8.0 * nc;
    else if (!DEC && a.keep_coarse) bytes = nl * sizeof(TS) + 8.0 * nc;
    else if (DEC) bytes = nl * sizeof(TS) + (nl - nc) * sizeof(T) + 8.0 * nc;
    else bytes = (nl - nc) * sizeof(TS) + 8.0 * nc;
  }
  std::string label = std::string("k_loadvec<") + tname<T>() + ", " + tname<TS>() + ", " + bname(DEC) + ", " +
                      bname(NODAL) + ", " + bname(C0) + ", " + bname(C1) + ", " + bname(C2) + ">";
  emit<LoadArgs<T, TS>, k_loadvec_group<T, TS, DEC, NODAL, C0, C1, C2>>(
      cx, a, (int64_t)grid.x, kNTHR<T, DEC, NODAL>, 0, label, bytes, [&] {
        TimedLaunch tl(cx.stream, label, bytes);
        hipLaunchKernelGGL((k_loadvec<T, TS, DEC, NODAL, C0, C1, C2>), grid, dim3(kNTHR<T, DEC, NODAL>), 0,
                           cx.stream, a);
      });
}

// Suffix of a solve's timing label naming what its store does (the kernel
// symbol is the same for every epilogue).
inline const char *epi_tag(int mode) {
  switch (mode) {
    case EPI_STORE_COMPACT: return " [store]";
    case EPI_STORE_NODAL: return " [nodal]";
    case EPI_SUB_COMPACT: return " [sub]";
    default: return "";
  }
}

// Algorithmic bytes of one correction solve over nc unknowns.
template <typename T>
double solve_bytes(double nc, int mode) {
  if (mode == EPI_Z) return 16.0 * nc;                          // read F, write F
  if (mode == EPI_SUB_COMPACT) return 8.0 * nc + 2.0 * sizeof(T) * nc;  // read F, read + write grid
  return 8.0 * nc + sizeof(T) * nc;                             // read F, write grid
}

// Tiles along a dimension of c coarse positions: the last tile absorbs a
// single left-over position (the ring kernel's extra row or column).
inline int ring_tiles(int64_t c, int t) { return (int)(c > t && c % t == 1 ? c / t : (c + t - 1) / t); }

template <typename T, typename TS, int TJ>
void launch_loadvec_ring(LoadArgs<T, TS> a, Ctx &cx) {
  constexpr int NTHR = kRingThr<TJ>;
  static const int slots = resident_slots((const void *)k_loadvec_ring<T, TS, true, true, true, TJ, 3>, NTHR);
  a.gx = ring_tiles(a.c2, TK);
  a.gy = ring_tiles(a.c1, TJ);
  const int64_t tiles = (int64_t)a.gx * a.gy;
  // built-in rule: long marches (the pipeline fills and drains once per
  // chunk), as many chunks as one round of resident workgroups holds
  const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(a.c0, slots / std::max<int64_t>(tiles, 1)));
  a.TI = cx.ti_req > 0 ? std::min<int64_t>(std::min<int64_t>(cx.ti_req, RING_MAXTI), a.c0)
                       : std::min<int64_t>((a.c0 + nch - 1) / nch, RING_MAXTI);
  cx.slots_out = slots;
  cx.ti_out = (int)a.TI;
  if (cx.dry) return;
  a.gz = (int)((a.c0 + a.TI - 1) / a.TI);
  const dim3 grid((unsigned)(tiles * a.gz));
  double bytes = 0.0;
  if (timing_enabled()) {
    const double nl = (double)a.m0 * a.m1 * a.m2, nc = (double)a.c0 * a.c1 * a.c2;
    // read the level grid, write the coefficients and f
    bytes = nl * sizeof(TS) + (nl - nc) * sizeof(T) + 8.0 * nc;
  }
  TimedLaunch tl(cx.stream, std::string("k_loadvec_ring<") + tname<T>() + ", " + tname<TS>() + ">", bytes);
  hipLaunchKernelGGL((k_loadvec_ring<T, TS, true, true, true, TJ, 3>), grid, dim3(NTHR), 0, cx.stream, a);
}

thread_local int g_plain_lv = 0;  // PlainLoadVector guards active on this thread

// Whether the ring kernel takes this level: a decomposition of the finest
// level grid (stored compactly in C order), FP64, coarsened along every
// dimension, not a time slice of a 4-D field.  (The recomposition keeps
// k_loadvec: its finest-level load vector runs on the helper stream beside
// the coarser levels, whose small kernels need free compute units, which a
// ring workgroup's 147 KB of LDS leaves none of; measured at 513^3 FP64 the
// ring took 0.388 ms there against 0.352, and the coarser levels' load
// vectors beside it 0.479 against 0.297.)
//
// It also needs a tiling that fills the device: one ring workgroup per CU,
// chunks of at least 32 coarse planes (the pipeline fills and drains once
// per chunk), and at least 90% of the CUs busy in one round (measured: 513^3
// FP64 fills all 256 CUs with 128 tiles x 2 chunks and gains, 0.551 -> 0.530
// ms; 400^3 gets 91 tiles x 2 chunks, 71% of the CUs, and loses, 0.65 ->
// 0.79 ms).
bool ring_fills(const Level &L) {
  const int64_t tiles = (int64_t)ring_tiles(L.c[2], TK) * ring_tiles(L.c[1], 16);
  const int64_t cus = device_cus();
  const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(L.c[0], cus / std::max<int64_t>(tiles, 1)));
  const int64_t ti = (L.c[0] + nch - 1) / nch;
  return ti >= 32 && ti <= RING_MAXTI && 10 * tiles * nch >= 9 * cus;
}
template <typename T, typename TS, bool DEC>
bool ring_applies(const Level &L, const LoadArgs<T, TS> &a) {
  return DEC && g_plain_lv == 0 && sizeof(TS) == 8 && a.omap.t0 == nullptr && L.co[0] && L.co[1] && L.co[2] &&
         a.out != nullptr && ring_fills(L);
}

template <typename T, typename TS, bool DEC>
void launch_loadvec(const Level &L, LoadArgs<T, TS> a, Ctx &cx) {
  a.m0 = L.m[0]; a.m1 = L.m[1]; a.m2 = L.m[2];
  a.c0 = L.c[0]; a.c1 = L.c[1]; a.c2 = L.c[2];
  a.r0 = L.d[0].r; a.r1 = L.d[1].r; a.r2 = L.d[2].r;
  a.W0 = L.d[0].W; a.W1 = L.d[1].W; a.W2 = L.d[2].W;
  a.gx = (int)((a.c2 + TK - 1) / TK);  // a.gy: by the kernel's tile, in launch_loadvec_t
  if constexpr (DEC && sizeof(T) == 8 && sizeof(TS) == 8) {
    // recorded launches (4-D slices, batches) take the grouped k_loadvec
    if (!cx.rec && ring_applies<T, TS, DEC>(L, a)) {
      launch_loadvec_ring<T, TS, 16>(a, cx);
      cx.check("k_loadvec_ring launch");
      return;
    }
  }
  const int key = (L.co[0] ? 4 : 0) | (L.co[1] ? 2 : 0) | (L.co[2] ? 1 : 0);
  // on coarser levels the field-side array (decompose: out; recompose: src)
  // goes through the nodal tables
  if (DEC ? a.omap.t0 != nullptr : a.smap.t0 != nullptr) {
    switch (key) {
      case 0: launch_loadvec_t<T, TS, DEC, true, false, false, false>(a, cx); break;
      case 1: launch_loadvec_t<T, TS, DEC, true, false, false, true>(a, cx); break;
      case 2: launch_loadvec_t<T, TS, DEC, true, false, true, false>(a, cx); break;
      case 3: launch_loadvec_t<T, TS, DEC, true, false, true, true>(a, cx); break;
      case 4: launch_loadvec_t<T, TS, DEC, true, true, false, false>(a, cx); break;
      case 5: launch_loadvec_t<T, TS, DEC, true, true, false, true>(a, cx); break;
      case 6: launch_loadvec_t<T, TS, DEC, true, true, true, false>(a, cx); break;
      default: launch_loadvec_t<T, TS, DEC, true, true, true, true>(a, cx); break;
    }
  } else {
    switch (key) {
      case 0: launch_loadvec_t<T, TS, DEC, false, false, false, false>(a, cx); break;
      case 1: launch_loadvec_t<T, TS, DEC, false, false, false, true>(a, cx); break;
      case 2: launch_loadvec_t<T, TS, DEC, false, false, true, false>(a, cx); break;
      case 3: launch_loadvec_t<T, TS, DEC, false, false, true, true>(a, cx); break;
      case 4: launch_loadvec_t<T, TS, DEC, false, true, false, false>(a, cx); break;
      case 5: launch_loadvec_t<T, TS, DEC, false, true, false, true>(a, cx); break;
      case 6: launch_loadvec_t<T, TS, DEC, false, true, true, false>(a, cx); break;
      default: launch_loadvec_t<T, TS, DEC, false, true, true, true>(a, cx); break;
    }
  }
  cx.check("k_loadvec launch");
}

// Persistent grid size: enough workgroups to fill the device a few times.
int64_t persistent_grid(int64_t nblocks) {
  return std::max<int64_t>(1, std::min<int64_t>(nblocks, 4 * (int64_t)device_cus()));
}

template <typename T, int S>
void launch_strided_s(double *F, const Level &L, int axis, const Epi<T> &ep, Ctx &cx) {
  const DimTabs &d = L.d[axis];
  const int64_t c0 = L.c[0], c1 = L.c[1], c2 = L.c[2];
  const int64_t c = L.c[axis];
  int64_t sp_, so, nouter;
  if (axis == 0) { sp_ = c1 * c2; so = c2; nouter = c1; }
  else { sp_ = c2; so = c1 * c2; nouter = c0; }
  dim3 grid((unsigned)(((c2 + 63) / 64) * nouter));
  const size_t lds = (size_t)4 * d.P * 64 * sizeof(double);
  const StridedArgs<T> sa{F, c, c2, sp_, so, c1, c2, d.P, axis, solve_dev(d), ep};
  std::string label = std::string("k_solve_strided<") + tname<T>() + ", " + std::to_string(S) + ">" + epi_tag(ep.mode);
  const double bytes = solve_bytes<T>((double)c0 * c1 * c2, ep.mode);
  emit<StridedArgs<T>, k_solve_strided_group<T, S>>(cx, sa, (int64_t)grid.x, 64 * d.P, lds, label, bytes, [&] {
    TimedLaunch tl(cx.stream, label, timing_enabled() ? bytes : 0.0);
    hipLaunchKernelGGL((k_solve_strided<T, S>), grid, dim3(64 * d.P), lds, cx.stream, sa);
  });
}

template <typename T, int S>
void launch_rows_s(double *F, const Level &L, const Epi<T> &ep, Ctx &cx) {
  const DimTabs &d = L.d[2];
  const int64_t c = L.c[2], nrows = L.c[0] * L.c[1];
  // about 96 KB of LDS per workgroup: larger blocks of rows measured faster
  const int budget = 96 * 1024 / (int)sizeof(double) - tables_size(d.P * S, d.P);
  int R = std::min(64, ROWS_THR / d.P);
  R = std::min<int64_t>(R, budget / (c + 4 * d.P));
  R = std::max(R, 1);
  const size_t lds = (size_t)(tables_size(d.P * S, d.P) + R * c + 4 * d.P * R) * sizeof(double);
  const int64_t nblocks = (nrows + R - 1) / R;
  dim3 grid((unsigned)persistent_grid(nblocks));
  const RowsArgs<T> ra{F, nrows, L.c[1], (int)c, d.P, R, solve_dev(d), ep};
  std::string label = std::string("k_solve_rows<") + tname<T>() + ", " + std::to_string(S) + ">" + epi_tag(ep.mode);
  const double bytes = solve_bytes<T>((double)nrows * c, ep.mode);
  emit<RowsArgs<T>, k_solve_rows_group<T, S>>(cx, ra, nblocks, R * d.P, lds, label, bytes, [&] {
    TimedLaunch tl(cx.stream, label, timing_enabled() ? bytes : 0.0);
    hipLaunchKernelGGL((k_solve_rows<T, S>), grid, dim3(R * d.P), lds, cx.stream, ra);
  });
}

template <typename T, int LB>
void launch_long_lb(double *F, const Level &L, int axis, const Epi<T> &ep, Ctx &cx) {
  const DimTabs &d = L.d[axis];
  const int64_t c0 = L.c[0], c1 = L.c[1], c2 = L.c[2];
  int64_t sp_, so, sk, nk, nouter;
  if (axis == 0) { sp_ = c1 * c2; so = c2; sk = 1; nk = c2; nouter = c1; }
  else if (axis == 1) { sp_ = c2; so = c1 * c2; sk = 1; nk = c2; nouter = c0; }
  else { sp_ = 1; so = 0; sk = c2; nk = c0 * c1; nouter = 1; }
  dim3 grid((unsigned)(((nk + LB - 1) / LB) * nouter));
  const size_t lds = (size_t)4 * d.P * LB * sizeof(double);
  const LongArgs<T> la{F, L.c[axis], nk, sp_, so, sk, c1, d.P, axis, solve_dev(d), ep};
  // the interior solutions are written and re-read once more
  std::string label = std::string("k_solve_long<") + tname<T>() + ", " + std::to_string(LB) + ">" + epi_tag(ep.mode);
  const double bytes = solve_bytes<T>((double)c0 * c1 * c2, ep.mode);
  emit<LongArgs<T>, k_solve_long_group<T, LB>>(cx, la, (int64_t)grid.x, 64 * LONG_WAVES, lds, label, bytes, [&] {
    TimedLaunch tl(cx.stream, label, timing_enabled() ? bytes : 0.0);
    hipLaunchKernelGGL((k_solve_long<T, LB>), grid, dim3(64 * LONG_WAVES), lds, cx.stream, la);
  });
}

// Blocks of 16 lines for lines of more than 32 partitions (the separator
// data of 64 lines would not fit in 64 KB of LDS) and where blocks of 64
// would not give every CU a workgroup (2-D fields: 8193^2 FP64 54 -> 258
// GB/s with the first two); 64 otherwise, also in batches, whose grouped
// launches hold many fields' blocks (the mixed 64-field batch measured 3%
// slower with 16).
template <typename T>
void launch_long(double *F, const Level &L, int axis, const Epi<T> &ep, Ctx &cx) {
  const int64_t nk = axis == 2 ? L.c[0] * L.c[1] : L.c[2];
  const int64_t nouter = axis == 0 ? L.c[1] : (axis == 1 ? L.c[0] : 1);
  const bool batch = cx.rec && cx.rec->long_chunks;
  if (L.d[axis].P > 32 || (!batch && ((nk + 63) / 64) * nouter < 256))
    launch_long_lb<T, 16>(F, L, axis, ep, cx);
  else
    launch_long_lb<T, 64>(F, L, axis, ep, cx);
}

template <typename T>
void launch_solve(double *F, const Level &L, int axis, const Epi<T> &ep, Ctx &cx) {
  const DimTabs &d = L.d[axis];
  if (d.P > kMaxBlocks || (d.S == 64 && axis != 2)) {
    // Strided lines of 64-position partitions go to the long-line solver as
    // well: beside a workgroup of up to 1024 threads a register partition of
    // 64 doubles does not fit and would spill whole (measured 1.8x slower
    // than the long-line solver's second pass over the line).
    launch_long<T>(F, L, axis, ep, cx);
  } else if (d.S == 0) {  // the plan chose one sequential partition (tables built for it)
    const int64_t nlines = L.c[0] * L.c[1] * L.c[2] / L.c[axis];
    const std::string label = std::string("k_solve_seq<") + tname<T>() + ">" + epi_tag(ep.mode);
    const double bytes = timing_enabled() ? solve_bytes<T>((double)L.c[0] * L.c[1] * L.c[2], ep.mode) : 0.0;
    const int64_t cax = L.c[axis], lc1 = L.c[1], lc2 = L.c[2];
    const SolveDev tb = solve_dev(d);
    emit_direct(cx, [=](hipStream_t st) {
      TimedLaunch tl(st, label, bytes);
      hipLaunchKernelGGL((k_solve_seq<T>), dim3((unsigned)grid_1d(nlines, 64)), dim3(64), 0, st, F, nlines, cax,
                         axis, lc1, lc2, tb, ep);
    });
  } else if (axis == 2) {
    switch (d.S) {
      case 8: launch_rows_s<T, 8>(F, L, ep, cx); break;
      case 16: launch_rows_s<T, 16>(F, L, ep, cx); break;
      case 32: launch_rows_s<T, 32>(F, L, ep, cx); break;
      default: launch_rows_s<T, 64>(F, L, ep, cx); break;
    }
  } else {
    switch (d.S) {  // 8, 16 or 32 here
      case 8: launch_strided_s<T, 8>(F, L, axis, ep, cx); break;
      case 16: launch_strided_s<T, 16>(F, L, axis, ep, cx); break;
      default: launch_strided_s<T, 32>(F, L, axis, ep, cx); break;
    }
  }
  cx.check("correction solve launch");
}

// The last coarsened dim of a level (-1: none).
int last_dim(const Level &L) {
  int lastk = -1;
  for (int k = 0; k < kDims; ++k)
    if (L.co[k]) lastk = k;
  return lastk;
}

// Solves along the coarsened dims in order 0, 1, 2; the last one applies
// `last`.  `part`: 0 all of them, 1 all but the last, 2 only the last.
// Recorded solves take phases cx.phase + 1, + 2, + 3 in order.
template <typename T>
void solve_all(double *F, const Level &L, const Epi<T> &last, Ctx &cx, int part = 0) {
  const int lastk = last_dim(L);
  const int p0 = cx.phase;
  int n = 0;
  for (int k = 0; k < kDims; ++k) {
    if (!L.co[k] || (part == 1 && k == lastk) || (part == 2 && k != lastk)) continue;
    Epi<T> ep = (k == lastk) ? last : Epi<T>{EPI_Z, nullptr, Map3{}};
    cx.phase = p0 + 1 + n++;
    launch_solve<T>(F, L, k, ep, cx);
  }
  cx.phase = p0;
}

template <typename T, bool NC, bool C0, bool C1, bool C2>
void launch_reconstruct_t(ReconArgs<T> a, Ctx &cx, const std::string &label, double bytes) {
  static const int slots = resident_slots((const void *)k_reconstruct<T, NC, C0, C1, C2>, RC_THR);
  const int64_t tiles = (int64_t)a.gx * a.gy;
  // chunks short enough for the kernel's LDS plane window (2 TI + 2 planes)
  const int64_t maxti = (LV_MAXP - 2) / 2;
  a.TI = cx.ti_req > 0 ? std::min<int64_t>(std::min<int64_t>(cx.ti_req, maxti), a.c0)
                       : pick_chunk(a.c0, tiles, slots, C0 ? 1 : 0, maxti);
  if (cx.rec && cx.rec->long_chunks) a.TI = std::max<int64_t>(a.TI, std::min<int64_t>(8, a.c0));
  cx.slots_out = slots;
  cx.ti_out = (int)a.TI;
  if (cx.dry) return;
  a.gz = (int)((a.c0 + a.TI - 1) / a.TI);
  emit<ReconArgs<T>, k_reconstruct_group<T, NC, C0, C1, C2>>(cx, a, tiles * a.gz, RC_THR, 0, label, bytes, [&] {
    TimedLaunch tl(cx.stream, label, timing_enabled() ? bytes : 0.0);
    hipLaunchKernelGGL((k_reconstruct<T, NC, C0, C1, C2>), dim3((unsigned)(tiles * a.gz)), dim3(RC_THR), 0,
                       cx.stream, a);
  });
}

// Whether a reconstruct tile of tj coarse rows and tk coarse columns fits the
// kernel's per-thread slots and its LDS coarse tile.
bool recon_tile_fits(const Level &L, int64_t tj, int64_t tk) {
  const int SJ = L.co[1] ? 2 : 1, SK = L.co[2] ? 2 : 1;
  const int HJ = L.co[1] ? 1 : 0, HK = L.co[2] ? 1 : 0;
  return tj >= 1 && tk >= 1 && tj <= L.c[1] && tk <= L.c[2] && SJ * tj * SK * tk <= RC_NE &&
         (tj + HJ) * (tk + HK) <= RC_NC;
}

// The built-in reconstruct tile: whole rows where a row fits, then as many
// coarse rows as the slots allow.
void recon_tile_rule(const Level &L, int &tj, int &tk) {
  int64_t TKc = L.c[2];
  while (TKc > 1 && !recon_tile_fits(L, 1, TKc)) TKc = (TKc + 1) / 2;
  int64_t TJc = 1;
  while (TJc < L.c[1] && recon_tile_fits(L, TJc + 1, TKc)) ++TJc;
  tj = (int)TJc;
  tk = (int)TKc;
}

template <typename T>
void launch_reconstruct(const Level &L, const T *coef, Map3 cmap, const T *uc, T *dst, Ctx &cx,
                        int tj_req = 0, int tk_req = 0) {
  ReconArgs<T> a{};
  a.coef = coef; a.cmap = cmap; a.uc = uc; a.dst = dst;
  a.m0 = L.m[0]; a.m1 = L.m[1]; a.m2 = L.m[2];
  a.c0 = L.c[0]; a.c1 = L.c[1]; a.c2 = L.c[2];
  a.r0 = L.d[0].r; a.r1 = L.d[1].r; a.r2 = L.d[2].r;
  // tile: a requested (autotuned) shape if it fits, else the built-in rule
  if (tj_req > 0 && tk_req > 0 && recon_tile_fits(L, tj_req, tk_req)) {
    a.TJ = tj_req;
    a.TK = tk_req;
  } else {
    recon_tile_rule(L, a.TJ, a.TK);
  }
  a.gx = (int)((a.c2 + a.TK - 1) / a.TK);
  a.gy = (int)((a.c1 + a.TJ - 1) / a.TJ);
  const int64_t n = L.m[0] * L.m[1] * L.m[2];
  const double nl = (double)n, nc = (double)L.c[0] * L.c[1] * L.c[2];
  // read the coefficients and the coarse grid, write the level grid
  const std::string label = std::string("k_reconstruct<") + tname<T>() + ", " + bname(cmap.t0 != nullptr) + ", " +
                            bname(L.co[0]) + ", " + bname(L.co[1]) + ", " + bname(L.co[2]) + ">";
  const double bytes = ((nl - nc) + nc + nl) * sizeof(T);
  const int key = (cmap.t0 ? 8 : 0) | (L.co[0] ? 4 : 0) | (L.co[1] ? 2 : 0) | (L.co[2] ? 1 : 0);
#define MGR_RECON(NC, C0, C1, C2) launch_reconstruct_t<T, NC, C0, C1, C2>(a, cx, label, bytes)
  switch (key) {
    case 0: MGR_RECON(false, false, false, false); break;
    case 1: MGR_RECON(false, false, false, true); break;
    case 2: MGR_RECON(false, false, true, false); break;
    case 3: MGR_RECON(false, false, true, true); break;
    case 4: MGR_RECON(false, true, false, false); break;
    case 5: MGR_RECON(false, true, false, true); break;
    case 6: MGR_RECON(false, true, true, false); break;
    case 7: MGR_RECON(false, true, true, true); break;
    case 8: MGR_RECON(true, false, false, false); break;
    case 9: MGR_RECON(true, false, false, true); break;
    case 10: MGR_RECON(true, false, true, false); break;
    case 11: MGR_RECON(true, false, true, true); break;
    case 12: MGR_RECON(true, true, false, false); break;
    case 13: MGR_RECON(true, true, false, true); break;
    case 14: MGR_RECON(true, true, true, false); break;
    default: MGR_RECON(true, true, true, true); break;
  }
#undef MGR_RECON
  cx.check("k_reconstruct launch");
}

// Levels tail_start .. nlev-1 in one workgroup.  Decompose: src is the
// compact level grid of level tail_start (FP64 from level 1 on), dst the
// caller's output.  Recompose: src is the caller's input, dst the compact
// level grid.
template <typename T, typename TS>
void launch_tail_dec(const Plan &pl, const TS *src, T *dst, Ctx &cx) {
  const Level &L = pl.lev[pl.tail_start];
  const double n = (double)L.m[0] * L.m[1] * L.m[2];
  // read the level grid, write the coefficients
  const std::string label = std::string("k_tail_dec<") + tname<T>() + ">";
  const double bytes = n * (sizeof(TS) + sizeof(T));
  const TailArgs ta{pl.dev_tail, pl.dev_tail_off, pl.dev_tail_dbl, pl.tail_noff, pl.tail_ndbl,
                    pl.nlev - pl.tail_start, 0};
  const TailDecJob<T, TS> job{src, dst, ta};
  emit<TailDecJob<T, TS>, k_tail_dec_group<T, TS>>(cx, job, 1, TAIL_THR, 0, label, bytes, [&] {
    TimedLaunch tl(cx.stream, label, timing_enabled() ? bytes : 0.0);
    hipLaunchKernelGGL((k_tail_dec<T, TS>), dim3(1), dim3(TAIL_THR), 0, cx.stream, src, dst, ta);
  });
  cx.check("k_tail_dec launch");
}

template <typename T>
void launch_tail_rec(const Plan &pl, const T *src, T *dst, Ctx &cx, int t_drop) {
  const Level &L = pl.lev[pl.tail_start];
  const double n = (double)L.m[0] * L.m[1] * L.m[2];
  // read the coefficients, write the level grid
  const std::string label = std::string("k_tail_rec<") + tname<T>() + ">";
  const double bytes = 2.0 * n * sizeof(T);
  const TailArgs ta{pl.dev_tail, pl.dev_tail_off, pl.dev_tail_dbl, pl.tail_noff, pl.tail_ndbl,
                    pl.nlev - pl.tail_start, t_drop};
  const TailRecJob<T> job{src, dst, ta};
  emit<TailRecJob<T>, k_tail_rec_group<T>>(cx, job, 1, TAIL_THR, 0, label, bytes, [&] {
    TimedLaunch tl(cx.stream, label, timing_enabled() ? bytes : 0.0);
    hipLaunchKernelGGL((k_tail_rec<T>), dim3(1), dim3(TAIL_THR), 0, cx.stream, src, dst, ta);
  });
  cx.check("k_tail_rec launch");
}

struct Workspace {
  void *buf[2];
  double *F;
  double *F2;  // coarser levels' load vector while level 0's runs beside them (nlev >= 2)
};

// The level-grid buffers hold FP64 (a decomposition keeps its coarser level
// grids in FP64 whatever the storage type) or the field's type (recomposition).
Workspace carve(const Plan &pl, void *ws) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t nb = al((size_t)pl.max_coarse * sizeof(double)), nf = nb;
  char *p = (char *)ws;
  return Workspace{{p, p + nb}, (double *)(p + 2 * nb), pl.nlev >= 2 ? (double *)(p + 2 * nb + nf) : nullptr};
}

// Decomposition.  Level 0 reads the caller's input; every coarser level grid
// is kept in FP64 in the workspace (written by the previous level's last
// solve), so that an FP32 field's coefficients at every level are rounded to
// FP32 once, when stored, and carry no rounding of the grids they came from.
template <typename T>
bool decompose_t(const Plan &pl, const T *in, T *out, void *ws, hipStream_t stream, std::string &err,
                 Rec *rec = nullptr) {
  Ctx cx{stream, &err};
  cx.rec = rec;
  const int64_t total = pl.n[0] * pl.n[1] * pl.n[2];
  if (pl.nlev == 0) {
    if (rec) {
      emit_direct(cx, [=](hipStream_t st) { (void)hipMemcpyAsync(out, in, total * sizeof(T), hipMemcpyDeviceToDevice, st); });
      return true;
    }
    if (hipMemcpyAsync(out, in, total * sizeof(T), hipMemcpyDeviceToDevice, stream) != hipSuccess) {
      err = "hipMemcpyAsync failed";
      return false;
    }
    return true;
  }
  Workspace w = carve(pl, ws);
  const double *src = nullptr;  // level grid of levels >= 1 (FP64)
  const int st = std::min(pl.tail_start, pl.nlev);
  const std::vector<LevelTune> tune = pl.tune_snapshot();
  for (int s = 0; s < st && cx.ok; ++s) {
    const Level &L = pl.lev[s];
    double *next = (double *)w.buf[s % 2];
    cx.ti_req = s < (int)tune.size() ? tune[s].lv_ti[0] : 0;
    cx.phase = phase_dec_level(s);
    if (s == 0) {
      LoadArgs<T> a{};
      a.src = in;
      a.smap = compact_map(pl.n[1], pl.n[2]);
      a.out = out;
      a.omap = compact_map(pl.n[1], pl.n[2]);
      a.F = w.F;
      launch_loadvec<T, T, true>(L, a, cx);
    } else {
      LoadArgs<T, double> a{};
      a.src = src;
      a.smap = compact_map(L.m[1], L.m[2]);
      a.out = out;
      a.omap = nodal_map(L);
      a.F = w.F;
      launch_loadvec<T, double, true>(L, a, cx);
    }
    cx.ti_req = 0;
    if (s + 1 < pl.nlev)
      solve_all<double>(w.F, L, Epi<double>{EPI_STORE_COMPACT, next, Map3{}}, cx);
    else
      solve_all<T>(w.F, L, Epi<T>{EPI_STORE_NODAL, out, nodal_map(pl.lev[s + 1])}, cx);
    src = next;
  }
  if (st < pl.nlev && cx.ok) {
    cx.phase = kPhaseTail;
    if (st == 0) launch_tail_dec<T, T>(pl, in, out, cx);
    else launch_tail_dec<T, double>(pl, src, out, cx);
  }
  return cx.ok;
}

// nkeep: coefficient classes used, coarsest first (nlev: all of them); the
// finer levels' coefficients are taken as zero, so those levels need no load
// vector and no solve (z = 0) and only interpolate.
//
// With a fork, level 0's load vector and its solves but the last -- which
// read only the stored coefficients -- run on the helper stream while the
// coarser levels recompose on `stream` (their load vectors in a second FP64
// grid); the stream then waits for them, and level 0's last solve subtracts
// z from the level-1 grid as before.  Every kernel and its arithmetic are
// those of the serial order.
template <typename T>
bool recompose_t(const Plan &pl, const T *in, T *out, void *ws, hipStream_t stream, std::string &err,
                 int nkeep, const StreamFork *fk = nullptr, Rec *rec = nullptr) {
  Ctx cx{stream, &err};
  cx.rec = rec;
  const int64_t total = pl.n[0] * pl.n[1] * pl.n[2];
  if (pl.nlev == 0) {
    if (rec) {
      emit_direct(cx, [=](hipStream_t st) { (void)hipMemcpyAsync(out, in, total * sizeof(T), hipMemcpyDeviceToDevice, st); });
      return true;
    }
    if (hipMemcpyAsync(out, in, total * sizeof(T), hipMemcpyDeviceToDevice, stream) != hipSuccess) {
      err = "hipMemcpyAsync failed";
      return false;
    }
    return true;
  }
  Workspace w = carve(pl, ws);
  const int st = std::min(pl.tail_start, pl.nlev);
  const int drop = pl.nlev - std::max(0, std::min(nkeep, pl.nlev));  // levels below take zero coefficients
  const std::vector<LevelTune> tune0 = pl.tune_snapshot();
  const bool split = fk != nullptr && rec == nullptr && w.F2 != nullptr && st >= 1 && drop == 0;
  double *Fc = split ? w.F2 : w.F;  // load vector of the levels on `stream`
  if (split) {
    hipStream_t hs = (hipStream_t)fk->helper;
    if (hipEventRecord((hipEvent_t)fk->fork, stream) != hipSuccess ||
        hipStreamWaitEvent(hs, (hipEvent_t)fk->fork, 0) != hipSuccess) {
      (void)hipGetLastError();
      err = "forking the helper stream failed";
      return false;
    }
    Ctx hx{hs, &err};
    const Level &L = pl.lev[0];
    LoadArgs<T> a{};
    a.src = in;
    a.smap = compact_map(pl.n[1], pl.n[2]);
    a.F = w.F;
    hx.share = true;
    launch_loadvec<T, T, false>(L, a, hx);
    hx.share = false;
    if (hx.ok) solve_all<T>(w.F, L, Epi<T>{EPI_Z, nullptr, Map3{}}, hx, 1);
    if (hipEventRecord((hipEvent_t)fk->join, hs) != hipSuccess) {
      (void)hipGetLastError();
      if (hx.ok) err = "joining the helper stream failed";
      hx.ok = false;
    }
    if (!hx.ok) return false;
  }
  T *V = nullptr;
  if (st < pl.nlev) {
    // the coarsest levels in one workgroup, up to the level grid of level st
    V = (st == 0) ? out : (T *)w.buf[st % 2];
    launch_tail_rec<T>(pl, in, V, cx, std::max(0, drop - st));
  } else {
    // coarsest grid values, gathered compactly
    const Level &Lc = pl.lev[pl.nlev];
    V = (T *)w.buf[pl.nlev % 2];
    const int64_t n = Lc.m[0] * Lc.m[1] * Lc.m[2];
    const Map3 nm = nodal_map(Lc);
    const int64_t g0 = Lc.m[0], g1 = Lc.m[1], g2 = Lc.m[2];
    T *Vg = V;
    emit_direct(cx, [=](hipStream_t st) {
      TimedLaunch tl(st, std::string("k_gather<") + tname<T>() + ">", 2.0 * n * sizeof(T));
      hipLaunchKernelGGL((k_gather<T>), dim3((unsigned)grid_1d(n, 256)), dim3(256), 0, st, in, nm, Vg, g0, g1, g2);
    });
    cx.check("k_gather launch");
  }
  const std::vector<LevelTune> &tune = tune0;
  for (int s = st - 1; s >= 0 && cx.ok; --s) {
    const Level &L = pl.lev[s];
    cx.phase = phase_rec_level(s);
    const LevelTune lt = s < (int)tune.size() ? tune[s] : LevelTune{};
    const Map3 cmap = (s == 0) ? compact_map(pl.n[1], pl.n[2]) : nodal_map(L);
    T *dst = (s == 0) ? out : (T *)w.buf[s % 2];
    if (s < drop) {  // dropped class: the level grid is the interpolant of U_c = V
      cx.ti_req = lt.rc_ti;
      cx.phase = phase_rec_level(s) + 4;
      launch_reconstruct<T>(L, (const T *)nullptr, cmap, V, dst, cx, lt.rc_tj, lt.rc_tk);
      cx.ti_req = 0;
      V = dst;
      continue;
    }
    Epi<T> ep{};
    ep.mode = EPI_SUB_COMPACT;
    ep.dst = V;
    if (split && s == 0) {
      // level 0's load vector and first solves ran on the helper stream
      if (hipStreamWaitEvent(stream, (hipEvent_t)fk->join, 0) != hipSuccess) {
        (void)hipGetLastError();
        err = "waiting for the helper stream failed";
        return false;
      }
      solve_all<T>(w.F, L, ep, cx, 2);
    } else {
      LoadArgs<T> a{};
      a.src = in;
      a.smap = cmap;
      a.F = Fc;
      cx.ti_req = lt.lv_ti[1];
      launch_loadvec<T, T, false>(L, a, cx);
      cx.ti_req = 0;
      solve_all<T>(Fc, L, ep, cx);
    }
    cx.ti_req = lt.rc_ti;
    cx.phase = phase_rec_level(s) + 4;
    launch_reconstruct<T>(L, in, cmap, V, dst, cx, lt.rc_tj, lt.rc_tk);
    cx.ti_req = 0;
    V = dst;
  }
  return cx.ok;
}

// ------------------------------------------------------------ 4-D fields

struct Workspace4 {
  void *buf[2];
  double *F, *G;
};

// Level-grid buffers in FP64, as in 3-D (the decomposition keeps its coarser
// level grids in FP64; the recomposition uses them in the field's type).
Workspace4 carve4(const Plan &pl, void *ws) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const int64_t cs = pl.lev[0].c[0] * pl.lev[0].c[1] * pl.lev[0].c[2];
  const int64_t c4 = pl.time->lev[0].c[2] * cs;
  const size_t nb = al((size_t)c4 * sizeof(double)), nf = nb;
  char *p = (char *)ws;
  return Workspace4{{p, p + nb}, (double *)(p + 2 * nb), (double *)(p + 2 * nb + nf)};
}

inline bool tcoarse(int64_t t, int64_t m) { return m < 3 || t % 2 == 0 || t == m - 1; }
inline int64_t tcoarse_idx(int64_t t, int64_t m, int64_t c) { return m < 3 ? t : (t == m - 1 ? c - 1 : t / 2); }

// Correction solves of a 4-D level on its compact coarse grid (ct slices of
// the space coarse grid), each run by the 3-D solvers on a rank-3 view of the
// grid: space dim 0 as dim 1 of (ct, c0, c1 c2), space dims 1 and 2 as dims 1
// and 2 of (ct c0, c1, c2), time as dim 0 of (ct, 1, c0 c1 c2).  The last
// solve applies `last`.
template <typename T>
void solve_all4(double *F, const Level &L, const Level &Lt, const Epi<T> &last, Ctx &cx) {
  const int64_t ct = Lt.c[2], c0 = L.c[0], c1 = L.c[1], c2 = L.c[2];
  struct View {
    Level v;
    int axis;
  };
  std::vector<View> views;
  for (int k = 0; k < kDims; ++k) {
    if (!L.co[k]) continue;
    View w{};
    if (k == 0) {
      w.v.c[0] = ct; w.v.c[1] = c0; w.v.c[2] = c1 * c2; w.axis = 1;
    } else {
      w.v.c[0] = ct * c0; w.v.c[1] = c1; w.v.c[2] = c2; w.axis = k;
    }
    w.v.d[w.axis] = L.d[k];
    views.push_back(w);
  }
  if (Lt.co[2]) {
    View w{};
    w.v.c[0] = ct; w.v.c[1] = 1; w.v.c[2] = c0 * c1 * c2; w.axis = 0;
    w.v.d[0] = Lt.d[2];
    views.push_back(w);
  }
  // recorded solves take phases cx.phase + 2, + 3, ... (after the load vectors
  // and the time load vector)
  const int p0 = cx.phase;
  for (size_t q = 0; q < views.size() && cx.ok; ++q) {
    const Epi<T> ep = (q + 1 == views.size()) ? last : Epi<T>{EPI_Z, nullptr, Map3{}};
    cx.phase = p0 + 2 + (int)q;
    launch_solve<T>(F, views[q].v, views[q].axis, ep, cx);
  }
  cx.phase = p0;
}

void launch_tload(const double *G, const Level &Lt, double *F, int64_t ncs, Ctx &cx) {
  const int64_t tm = Lt.m[2], ct = Lt.c[2];
  const int64_t nrun = (ct + TL_JC - 1) / TL_JC;
  const dim3 grid((unsigned)((ncs + 255) / 256), (unsigned)std::min<int64_t>(nrun, 65535));
  const double bytes = timing_enabled() ? 8.0 * (double)(tm + ct) * (double)ncs : 0.0;
  const double *W = Lt.d[2].W;
  const int p0 = cx.phase;
  cx.phase = p0 + 1;
  emit_direct(cx, [=](hipStream_t st) {
    TimedLaunch tl(st, "k_tload", bytes);
    hipLaunchKernelGGL(k_tload, grid, dim3(256), 0, st, G, tm, W, F, ct, ncs);
  });
  cx.phase = p0;
  cx.check("k_tload launch");
}

template <typename T, typename TS, bool DEC>
void launch_tfine(const Plan &pl, const Level &L, const Level &Lt, const TS *src, T *dst, const TS *crs,
                  Map3 fmap, Ctx &cx) {
  const int64_t tm = Lt.m[2], nf = (tm - 1) / 2;
  if (nf <= 0) return;
  TfineArgs<T, TS> a{};
  a.src = src; a.dst = dst; a.crs = crs; a.fmap = fmap;
  a.tnod = Lt.d[2].nodal; a.rt = Lt.d[2].r;
  a.S0 = pl.n[0] * pl.n[1] * pl.n[2];
  a.tm = tm;
  a.m0 = L.m[0]; a.m1 = L.m[1]; a.m2 = L.m[2];
  a.c0 = L.c[0]; a.c1 = L.c[1]; a.c2 = L.c[2];
  a.co0 = L.co[0]; a.co1 = L.co[1]; a.co2 = L.co[2];
  a.r0 = L.d[0].r; a.r1 = L.d[1].r; a.r2 = L.d[2].r;
  const int64_t sm = L.m[0] * L.m[1] * L.m[2];
  // (row group, plane chunk) jobs of the time-fine slices
  const int64_t jobs = nf * ((L.m[0] + TF_PI - 1) / TF_PI) * ((L.m[1] + TF_ROWS - 1) / TF_ROWS);
  const dim3 grid((unsigned)std::min<int64_t>(jobs, (int64_t)1 << 20));
  const std::string label = std::string("k_tfine<") + tname<T>() + ", " + bname(DEC) + ">";
  const double bytes = timing_enabled() ? (double)nf * (double)sm * (sizeof(T) + sizeof(TS)) : 0.0;
  emit_direct(cx, [=](hipStream_t st) {
    TimedLaunch tl(st, label, bytes);
    hipLaunchKernelGGL((k_tfine<T, TS, DEC>), grid, dim3(TF_THR), 0, st, a);
  });
  cx.check("k_tfine launch");
}

template <typename TS, typename TD, bool TO_NODAL>
void launch_nodal4(const Plan &pl, const TS *src, TD *dst, Ctx &cx) {
  const Level &L = pl.lev[pl.nlev];
  const Level &Lt = pl.time->lev[pl.nlev];
  const int64_t n = Lt.m[2] * L.m[0] * L.m[1] * L.m[2];
  const std::string label = std::string("k_nodal4<") + tname<TD>() + ", " + bname(TO_NODAL) + ">";
  const double bytes = timing_enabled() ? (double)n * (sizeof(TS) + sizeof(TD)) : 0.0;
  const Map3 nm = nodal_map(L);
  const int64_t *tnod = Lt.d[2].nodal, S0 = pl.n[0] * pl.n[1] * pl.n[2], tm = Lt.m[2];
  const int64_t m0 = L.m[0], m1 = L.m[1], m2 = L.m[2];
  emit_direct(cx, [=](hipStream_t st) {
    TimedLaunch tl(st, label, bytes);
    hipLaunchKernelGGL((k_nodal4<TS, TD, TO_NODAL>), dim3((unsigned)grid_1d(n, 256)), dim3(256), 0, st, src, dst,
                       nm, tnod, S0, tm, m0, m1, m2);
  });
  cx.check("k_nodal4 launch");
}

// One level of a 4-D decomposition: the space load vector of every time
// slice (with the coefficients of the time-coarse slices, which only space
// interpolation reaches), the load vector along time, the four solves (their
// solution is the next level's grid), then the coefficients of the time-fine
// slices.  The level grid `src` is the field at level 0 and FP64 from level 1
// on; the solves store the next level's grid in FP64 into `next`.
template <typename T, typename TS>
void decompose4_level(const Plan &pl, int s, const TS *src, T *out, double *next, const Workspace4 &w, Ctx &cx) {
  const Level &L = pl.lev[s];
  const Level &Lt = pl.time->lev[s];
  const int64_t S0 = pl.n[0] * pl.n[1] * pl.n[2];
  const int64_t tm = Lt.m[2];
  const bool cot = Lt.co[2];
  const int64_t sm = L.m[0] * L.m[1] * L.m[2], cs = L.c[0] * L.c[1] * L.c[2];
  double *G = cot ? w.G : w.F;
  const Map3 lmap = compact_map(L.m[1], L.m[2]);
  const Map3 omap = (s == 0) ? lmap : nodal_map(L);
  for (int64_t t = 0; t < tm && cx.ok; ++t) {
    const bool tc = tcoarse(t, tm) || !cot;
    LoadArgs<T, TS> a{};
    a.src = src + t * sm;
    a.smap = lmap;
    a.out = tc ? out + pl.tpos[s][t] * S0 : nullptr;
    a.omap = tc ? omap : lmap;
    a.F = G + t * cs;
    launch_loadvec<T, TS, true>(L, a, cx);
  }
  if (cot && cx.ok) launch_tload(w.G, Lt, w.F, cs, cx);
  solve_all4<double>(w.F, L, Lt, Epi<double>{EPI_STORE_COMPACT, next, Map3{}}, cx);
  const int p0 = cx.phase;
  cx.phase = p0 + 6;
  if (cot && cx.ok) launch_tfine<T, TS, true>(pl, L, Lt, src, out, src, omap, cx);
  cx.phase = p0;
}

// The 4-D drivers record their launches (per level: the time slices' space
// load vectors at phase 8s, the time load vector +1, the solves +2.., the
// time-fine slices +6; a recomposition's reconstructs +6 and time-fine
// slices +7) and launch them grouped: the slices' load vectors and
// reconstructs of one level go out as one grid each (Sec. III-D).
template <typename T>
bool decompose4_t(const Plan &pl, const T *in, T *out, void *ws, hipStream_t stream, std::string &err) {
  Rec rec;
  Ctx cx{stream, &err};
  cx.rec = &rec;
  const int64_t S0 = pl.n[0] * pl.n[1] * pl.n[2];
  if (pl.nlev == 0) {
    if (hipMemcpyAsync(out, in, pl.nt * S0 * sizeof(T), hipMemcpyDeviceToDevice, stream) != hipSuccess) {
      err = "hipMemcpyAsync failed";
      return false;
    }
    return true;
  }
  Workspace4 w = carve4(pl, ws);
  const double *src = nullptr;
  for (int s = 0; s < pl.nlev && cx.ok; ++s) {
    double *next = (double *)w.buf[s % 2];
    cx.phase = phase_dec_level(s);
    if (s == 0) decompose4_level<T, T>(pl, s, in, out, next, w, cx);
    else decompose4_level<T, double>(pl, s, src, out, next, w, cx);
    src = next;
  }
  cx.phase = kPhaseTail;
  if (cx.ok) launch_nodal4<double, T, true>(pl, src, out, cx);
  return cx.ok && launch_recorded(rec, stream, err);
}

// One level of a 4-D recomposition: the load vector of the stored
// coefficients (zero at the coarse nodes: those of the time-coarse slices
// that are coarse in space), the solves, whose solution z is subtracted from
// the stored coarse values, then the level grid: time-coarse slices by the
// space reconstruct from their coarse slice, time-fine slices by k_tfine.
template <typename T>
bool recompose4_t(const Plan &pl, const T *in, T *out, void *ws, hipStream_t stream, std::string &err) {
  Rec rec;
  Ctx cx{stream, &err};
  cx.rec = &rec;
  const int64_t S0 = pl.n[0] * pl.n[1] * pl.n[2];
  if (pl.nlev == 0) {
    if (hipMemcpyAsync(out, in, pl.nt * S0 * sizeof(T), hipMemcpyDeviceToDevice, stream) != hipSuccess) {
      err = "hipMemcpyAsync failed";
      return false;
    }
    return true;
  }
  const Plan &tp = *pl.time;
  Workspace4 w = carve4(pl, ws);
  T *V = (T *)w.buf[pl.nlev % 2];
  cx.phase = 0;
  launch_nodal4<T, T, false>(pl, in, V, cx);
  for (int s = pl.nlev - 1; s >= 0 && cx.ok; --s) {
    const Level &L = pl.lev[s];
    const Level &Lt = tp.lev[s];
    const int p0 = phase_rec_level(s);
    cx.phase = p0;
    const int64_t tm = Lt.m[2], ct = Lt.c[2];
    const bool cot = Lt.co[2];
    const int64_t sm = L.m[0] * L.m[1] * L.m[2], cs = L.c[0] * L.c[1] * L.c[2];
    T *dst = (s == 0) ? out : (T *)w.buf[s % 2];
    double *G = cot ? w.G : w.F;
    const Map3 cmap = (s == 0) ? compact_map(L.m[1], L.m[2]) : nodal_map(L);
    for (int64_t t = 0; t < tm && cx.ok; ++t) {
      LoadArgs<T> a{};
      a.src = in + pl.tpos[s][t] * S0;
      a.smap = cmap;
      a.F = G + t * cs;
      a.keep_coarse = (cot && !tcoarse(t, tm)) ? 1 : 0;
      launch_loadvec<T, T, false>(L, a, cx);
    }
    if (cot && cx.ok) launch_tload(w.G, Lt, w.F, cs, cx);
    solve_all4<T>(w.F, L, Lt, Epi<T>{EPI_SUB_COMPACT, V, Map3{}}, cx);
    cx.phase = p0 + 6;
    for (int64_t t = 0; t < tm && cx.ok; ++t) {
      if (cot && !tcoarse(t, tm)) continue;
      const int64_t J = cot ? tcoarse_idx(t, tm, ct) : t;
      launch_reconstruct<T>(L, in + pl.tpos[s][t] * S0, cmap, V + J * cs, dst + t * sm, cx);
    }
    cx.phase = p0 + 7;
    if (cot && cx.ok) launch_tfine<T, T, false>(pl, L, Lt, in, dst, V, cmap, cx);
    V = dst;
  }
  return cx.ok && launch_recorded(rec, stream, err);
}

// ------------------------------------------------------------ autotuner
//
// The paper tunes its kernels' launch shapes per problem size by ranking
// candidates with a model of their memory transactions and profiling the
// best few (Sec. III-B).  Here the tunable shapes are the dim-0 chunk length
// of the load-vector and reconstruct kernels and the reconstruct tile; the
// model counts the 128-byte lines (the CDNA4 cache line) a launch touches --
// halo planes re-read per chunk, and row segments split between tiles, are
// counted once per tile that touches them -- and adds a per-plane-step
// latency for each round of resident workgroups.  The three best candidates
// by the model run on the GPU, and the fastest is kept in the plan.  No
// candidate changes any node's arithmetic.

constexpr double kModelBytesPerSec = 4.5e12;  // streaming rate of a plain copy on MI355X
constexpr double kModelStepSec = 0.6e-6;       // one plane step of a resident workgroup

// 128-byte lines touched by the byte range [off, off + len).
inline int64_t lines128(int64_t off, int64_t len) {
  return len <= 0 ? 0 : (off + len - 1) / 128 - off / 128 + 1;
}

// Modelled seconds of a plane-marching launch over `tiles` tile columns and
// c0 coarse planes in chunks of ti (halo: extra coarse planes per chunk),
// moving bytes_per_plane per coarse plane of the whole grid.
double model_march(int64_t c0, int64_t tiles, int slots, int halo, int64_t ti, double bytes_per_plane) {
  const int64_t nch = (c0 + ti - 1) / ti, nwg = tiles * nch;
  const int64_t rounds = (nwg + slots - 1) / std::max(slots, 1);
  const double bytes = bytes_per_plane * (double)nch * (double)(ti + halo);
  return std::max(bytes / kModelBytesPerSec, (double)rounds * (double)(ti + halo) * kModelStepSec);
}

// Bytes the reconstruct moves per coarse plane for tile (tj, tk): the fine
// rows' coefficient reads and level-grid writes, line by line per tile
// (nodal coefficients use half of every line), and the coarse tiles.
double recon_bytes_per_plane(const Level &L, bool nodal, size_t es, int64_t tj, int64_t tk) {
  const int64_t SK = L.co[2] ? 2 : 1, s0 = L.co[0] ? 2 : 1;
  const int64_t gx = (L.c[2] + tk - 1) / tk, gy = (L.c[1] + tj - 1) / tj;
  int64_t fine = 0;
  for (int64_t j = 0; j < L.m[1]; ++j)
    for (int64_t tx = 0; tx < gx; ++tx) {
      const int64_t k0 = SK * tx * tk, k1 = std::min(L.m[2], SK * (tx + 1) * tk);
      const int64_t off = (j * L.m[2] + k0) * (int64_t)es, len = (k1 - k0) * (int64_t)es;
      fine += lines128(off, len) + (nodal ? 2 * (len + 127) / 128 : lines128(off, len));
    }
  int64_t coarse = 0;
  for (int64_t ty = 0; ty < gy; ++ty)
    for (int64_t tx = 0; tx < gx; ++tx) {
      const int64_t rows = std::min(tj + 1, L.c[1] - ty * tj), cols = std::min(tk + 1, L.c[2] - tx * tk);
      for (int64_t r = 0; r < rows; ++r)
        coarse += lines128(((ty * tj + r) * L.c[2] + tx * tk) * (int64_t)es, cols * (int64_t)es);
    }
  return 128.0 * ((double)fine * (double)s0 + (double)coarse);
}

template <typename T>
bool autotune_t(Plan &pl, const T *in, T *out, void *ws, hipStream_t stream, std::string &err,
                std::string &report) {
  Ctx cx{stream, &err};
  if (pl.nlev == 0) return true;
  Workspace w = carve(pl, ws);
  const int nt = std::min(pl.tail_start, pl.nlev);
  std::vector<LevelTune> tune(pl.nlev);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    (void)hipGetLastError();
    if (e0) (void)hipEventDestroy(e0);
    err = "hipEventCreate failed";
    return false;
  }
  // best of three launches, in milliseconds
  auto time_ms = [&](auto &&launch) -> double {
    double best = 1e30;
    for (int r = 0; r < 3 && cx.ok; ++r) {
      (void)hipEventRecord(e0, stream);
      launch();
      (void)hipEventRecord(e1, stream);
      if (hipEventSynchronize(e1) != hipSuccess) {
        cx.ok = false;
        err = "autotune: kernel failed";
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      best = std::min(best, (double)ms);
    }
    return best;
  };
  // times the model's three cheapest candidates and the built-in rule's
  // (`rule`), returns the fastest
  auto choose = [&](std::vector<std::pair<double, int>> cand, int rule, auto &&run, const char *what, int s) {
    std::sort(cand.begin(), cand.end());
    std::vector<int> timed;
    for (size_t q = 0; q < cand.size() && q < 3; ++q) timed.push_back(cand[q].second);
    if (std::find(timed.begin(), timed.end(), rule) == timed.end()) timed.push_back(rule);
    int best = -1;
    double best_ms = 1e30;
    for (size_t q = 0; q < timed.size() && cx.ok; ++q) {
      const int id = timed[q];
      const double ms = time_ms([&] { run(id); });
      if (ms < best_ms) {
        best_ms = ms;
        best = id;
      }
    }
    report += "level " + std::to_string(s) + " " + what + ": candidate " + std::to_string(best) + " (" +
              std::to_string(best_ms * 1e3) + " us)\n";
    return best;
  };
  const size_t es = sizeof(T);
  for (int s = 0; s < nt && cx.ok; ++s) {
    const Level &L = pl.lev[s];
    const double nl = (double)L.m[0] * L.m[1] * L.m[2];
    const int halo_lv = L.co[0] ? 2 : 0;
    for (int dec = 1; dec >= 0 && cx.ok; --dec) {
      // the finest FP64 level runs the ring kernel (its tiles absorb a single
      // left-over row or column); other levels k_loadvec, whose field-side
      // array is nodal below level 0
      const bool ring = dec && s == 0 && sizeof(T) == 8 && L.co[0] && L.co[1] && L.co[2] && g_plain_lv == 0 &&
                        ring_fills(L);
      const int tj = ring ? 16 : tile_rows<T>(dec != 0, s > 0);
      const int64_t tiles_lv = ring ? (int64_t)ring_tiles(L.c[2], TK) * ring_tiles(L.c[1], tj)
                                    : ((L.c[2] + TK - 1) / TK) * ((L.c[1] + tj - 1) / tj);
      // level s's load vector as the decomposition (FP64 level grid from
      // level 1 on) or the recomposition launches it
      auto lv = [&]() {
        const Map3 cm = compact_map(L.m[1], L.m[2]);
        if (!dec) {
          LoadArgs<T> a{};
          a.src = in;
          a.smap = s == 0 ? cm : nodal_map(L);
          a.F = w.F;
          launch_loadvec<T, T, false>(L, a, cx);
        } else if (s == 0) {
          LoadArgs<T> a{};
          a.src = in;
          a.smap = cm;
          a.out = out;
          a.omap = cm;
          a.F = w.F;
          launch_loadvec<T, T, true>(L, a, cx);
        } else {
          LoadArgs<T, double> a{};
          a.src = (const double *)w.buf[(s + 1) % 2];
          a.smap = cm;
          a.out = out;
          a.omap = nodal_map(L);
          a.F = w.F;
          launch_loadvec<T, double, true>(L, a, cx);
        }
      };
      cx.dry = true;
      cx.ti_req = 0;
      lv();
      cx.dry = false;
      const int slots = cx.slots_out, ti0 = cx.ti_out;
      const double per_plane = (dec ? 2.0 * nl * es : nl * es) / (double)L.c[0];
      std::vector<std::pair<double, int>> cand;
      const int64_t maxti = std::min<int64_t>(ring ? RING_MAXTI : (LV_MAXP - 3) / 2, L.c[0]);
      std::vector<int64_t> tis = {(int64_t)ti0, 1, 2, 4, 6, 8, 12, 16, 24, 32, 48, maxti};
      for (int64_t k = 1; k <= 8; ++k) tis.push_back((L.c[0] + k - 1) / k);  // extent split evenly
      for (int64_t ti : tis) {
        if (ti < 1 || ti > maxti) continue;
        bool dup = false;
        for (auto &c : cand) dup |= c.second == (int)ti;
        if (!dup) cand.push_back({model_march(L.c[0], tiles_lv, slots, halo_lv, ti, per_plane), (int)ti});
      }
      const int best = choose(cand, ti0, [&](int ti) {
        cx.ti_req = ti;
        lv();
        cx.ti_req = 0;
      }, dec ? "decompose load vector planes per workgroup" : "recompose load vector planes per workgroup", s);
      tune[s].lv_ti[dec ? 0 : 1] = best > 0 ? best : 0;
    }
    // reconstruct tile
    {
      const bool nodal = s > 0;
      const Map3 cmap = nodal ? nodal_map(L) : compact_map(L.m[1], L.m[2]);
      const T *uc = (const T *)w.buf[(s + 1) % 2];
      T *dst = s == 0 ? out : (T *)w.buf[s % 2];
      int tj0 = 0, tk0 = 0;
      recon_tile_rule(L, tj0, tk0);
      std::vector<std::pair<int, int>> shapes = {{tj0, tk0}};
      for (int64_t tk : {L.c[2], (L.c[2] + 1) / 2, (L.c[2] + 3) / 4, (int64_t)128, (int64_t)64, (int64_t)32,
                         (int64_t)16}) {
        if (tk < 1 || tk > L.c[2]) continue;
        int64_t tj = 1;
        if (!recon_tile_fits(L, 1, tk)) continue;
        while (tj < L.c[1] && recon_tile_fits(L, tj + 1, tk)) ++tj;
        for (int64_t t : {tj, std::max<int64_t>(1, tj / 2)}) {
          bool dup = false;
          for (auto &p : shapes) dup |= (p.first == (int)t && p.second == (int)tk);
          if (!dup) shapes.push_back({(int)t, (int)tk});
        }
      }
      std::vector<std::pair<double, int>> cand;
      for (size_t q = 0; q < shapes.size(); ++q) {
        cx.dry = true;
        launch_reconstruct<T>(L, in, cmap, uc, dst, cx, shapes[q].first, shapes[q].second);
        cx.dry = false;
        const int64_t tiles = ((L.c[2] + shapes[q].second - 1) / shapes[q].second) *
                              ((L.c[1] + shapes[q].first - 1) / shapes[q].first);
        const double bpp = recon_bytes_per_plane(L, nodal, es, shapes[q].first, shapes[q].second);
        cand.push_back({model_march(L.c[0], tiles, cx.slots_out, L.co[0] ? 1 : 0, cx.ti_out, bpp), (int)q});
      }
      const int best = choose(cand, 0, [&](int q) {
        launch_reconstruct<T>(L, in, cmap, uc, dst, cx, shapes[q].first, shapes[q].second);
      }, "reconstruct tile index", s);
      if (best >= 0) {
        tune[s].rc_tj = shapes[best].first;
        tune[s].rc_tk = shapes[best].second;
        report += "level " + std::to_string(s) + " reconstruct tile " + std::to_string(tune[s].rc_tj) + " x " +
                  std::to_string(tune[s].rc_tk) + " coarse rows x columns\n";
        // then its coarse planes per workgroup: the built-in rule against
        // the chunks that cut dim 0 into 1 to 8 pieces
        const int tj = tune[s].rc_tj, tk = tune[s].rc_tk;
        cx.dry = true;
        launch_reconstruct<T>(L, in, cmap, uc, dst, cx, tj, tk);
        cx.dry = false;
        const int ti0 = cx.ti_out, slots = cx.slots_out;
        const int64_t tiles = ((L.c[2] + tk - 1) / tk) * ((L.c[1] + tj - 1) / tj);
        const int64_t maxti = (LV_MAXP - 2) / 2;
        const double bpp = recon_bytes_per_plane(L, nodal, es, tj, tk);
        const int halo = L.co[0] ? 1 : 0;
        std::vector<std::pair<double, int>> tcand = {{model_march(L.c[0], tiles, slots, halo, ti0, bpp), ti0}};
        for (int k = 1; k <= 8; ++k) {
          const int64_t ti = (L.c[0] + k - 1) / k;
          if (ti < 1 || ti > maxti) continue;
          bool dup = false;
          for (auto &c : tcand) dup |= c.second == (int)ti;
          if (!dup) tcand.push_back({model_march(L.c[0], tiles, slots, halo, ti, bpp), (int)ti});
        }
        const int bti = choose(tcand, ti0, [&](int ti) {
          cx.ti_req = ti;
          launch_reconstruct<T>(L, in, cmap, uc, dst, cx, tj, tk);
          cx.ti_req = 0;
        }, "reconstruct planes per workgroup", s);
        tune[s].rc_ti = bti > 0 ? bti : 0;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (!cx.ok) return false;
  std::lock_guard<std::mutex> lk(pl.tune_mu);
  pl.tune = tune;
  return true;
}

template <typename T, bool EXPORT>
bool classes_t(const Plan &pl, const T *src, T *dst, hipStream_t stream, std::string &err) {
  Ctx cx{stream, &err};
  int64_t off = 0;
  for (int s = pl.nlev; s >= 0 && cx.ok; --s) {  // coarsest grid first, then classes coarse to fine
    const Level &L = pl.lev[s];
    const bool coarsest = s == pl.nlev;
    const int64_t n = L.m[0] * L.m[1] * L.m[2];
    const int64_t nc = coarsest ? 0 : L.c[0] * L.c[1] * L.c[2];
    TimedLaunch tl(stream, std::string(EXPORT ? "k_classes<" : "k_classes_import<") + tname<T>() + ">",
                   timing_enabled() ? 2.0 * (double)(n - nc) * sizeof(T) : 0.0);
    hipLaunchKernelGGL((k_classes<T, EXPORT>), dim3((unsigned)grid_1d(n, 256)), dim3(256), 0, stream, src, dst,
                       nodal_map(L), L.m[0], L.m[1], L.m[2], L.c[1], L.c[2], L.co[0] ? 1 : 0, L.co[1] ? 1 : 0,
                       L.co[2] ? 1 : 0, off, coarsest ? 1 : 0);
    cx.check("k_classes launch");
    off += n - nc;
  }
  return cx.ok;
}

}  // namespace

bool enqueue_classes(const Plan &pl, bool f64, bool export_, const void *src, void *dst, void *stream,
                     std::string &err) {
  hipStream_t st = (hipStream_t)stream;
  if (f64)
    return export_ ? classes_t<double, true>(pl, (const double *)src, (double *)dst, st, err)
                   : classes_t<double, false>(pl, (const double *)src, (double *)dst, st, err);
  return export_ ? classes_t<float, true>(pl, (const float *)src, (float *)dst, st, err)
                 : classes_t<float, false>(pl, (const float *)src, (float *)dst, st, err);
}

bool enqueue_autotune(Plan &pl, bool f64, const void *in, void *out, void *ws, void *stream, std::string &err,
                      std::string &report) {
  hipStream_t st = (hipStream_t)stream;
  return f64 ? autotune_t<double>(pl, (const double *)in, (double *)out, ws, st, err, report)
             : autotune_t<float>(pl, (const float *)in, (float *)out, ws, st, err, report);
}

bool enqueue_copy_probe(const void *src, void *dst, size_t bytes, void *stream, std::string &err) {
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = (int64_t)(bytes / 16);
  if (n == 0) return true;
  const int64_t blocks = (n + 255) / 256;
  if (blocks * 256 > (int64_t)UINT32_MAX) {  // work items of one launch dimension
    err = "copy probe larger than one launch covers (64 GiB)";
    return false;
  }
  TimedLaunch tl(st, "k_copy_probe", 2.0 * (double)bytes);
  hipLaunchKernelGGL(k_copy_probe, dim3((unsigned)blocks), dim3(256), 0, st, (const probe_word *)src,
                     (probe_word *)dst, n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    err = std::string("k_copy_probe launch: ") + hipGetErrorString(e);
    return false;
  }
  return true;
}

bool enqueue_batch(bool dec, const std::vector<std::vector<BatchItem>> &lanes, const std::vector<void *> &streams,
                   std::string &err) {
  const size_t nl = lanes.size();
  std::vector<Rec> recs(nl);
  // (64-field batch 3.5 -> 2.95 ms from a graph; the 4-D drivers' grouped
  // slices keep the single-field rule: 400^3 x 16 was 913 -> 842 GB/s with
  // the longest chunks)
  for (Rec &r : recs) r.long_chunks = true;
  {
    const PlainLoadVector plain;  // batches keep k_loadvec (see mgr_api.cpp)
    for (size_t k = 0; k < nl; ++k) {
      hipStream_t st = (hipStream_t)streams[k];
      for (const BatchItem &b : lanes[k]) {
        const bool ok =
            dec ? (b.f64 ? decompose_t<double>(*b.pl, (const double *)b.in, (double *)b.out, b.ws, st, err, &recs[k])
                         : decompose_t<float>(*b.pl, (const float *)b.in, (float *)b.out, b.ws, st, err, &recs[k]))
                : (b.f64 ? recompose_t<double>(*b.pl, (const double *)b.in, (double *)b.out, b.ws, st, err,
                                               b.pl->nlev, nullptr, &recs[k])
                         : recompose_t<float>(*b.pl, (const float *)b.in, (float *)b.out, b.ws, st, err,
                                              b.pl->nlev, nullptr, &recs[k]));
        if (!ok) return false;
      }
    }
  }
  // the lanes' launches go out interleaved, so that every stream has work
  // queued while the host is still launching
  std::vector<std::vector<Unit>> units(nl);
  size_t most = 0;
  for (size_t k = 0; k < nl; ++k) {
    recorded_units(recs[k], units[k]);
    most = std::max(most, units[k].size());
  }
  for (size_t i = 0; i < most; ++i)
    for (size_t k = 0; k < nl; ++k)
      if (i < units[k].size()) units[k][i]((hipStream_t)streams[k]);
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) {
    err = std::string("grouped batch launch: ") + hipGetErrorString(he);
    return false;
  }
  return true;
}

namespace {
// The launches of a recording in phase order, the jobs of one kernel in a
// phase merged into grouped launches.  The units refer to `rec`'s jobs.
void recorded_units(const Rec &rec, std::vector<Unit> &out) {
  std::vector<const RecJob *> js;
  js.reserve(rec.jobs.size());
  for (const RecJob &r : rec.jobs) js.push_back(&r);
  std::stable_sort(js.begin(), js.end(), [](const RecJob *a, const RecJob *b) { return a->phase < b->phase; });
  size_t i = 0;
  while (i < js.size()) {
    size_t e = i;
    while (e < js.size() && js[e]->phase == js[i]->phase) ++e;
    std::vector<bool> done(e - i, false);
    for (size_t a = i; a < e; ++a) {
      if (done[a - i]) continue;
      const RecJob *r = js[a];
      if (!r->group) {
        done[a - i] = true;
        out.push_back([r](hipStream_t st) { r->direct(st); });
        continue;
      }
      std::vector<const RecJob *> g;
      size_t lds = 0;
      unsigned thr = 0;
      double bytes = 0.0;
      auto flush = [&]() {
        out.push_back([g, lds, thr, bytes, r](hipStream_t st) {
          TimedLaunch tl(st, r->label + " [group]", timing_enabled() ? bytes : 0.0);
          r->group(g, st, lds, thr);
        });
        g.clear();
        lds = 0;
        thr = 0;
        bytes = 0.0;
      };
      for (size_t b = a; b < e; ++b) {
        const RecJob *q = js[b];
        if (done[b - i] || q->group != r->group) continue;
        done[b - i] = true;
        g.push_back(q);
        lds = std::max(lds, q->lds);
        thr = std::max(thr, q->threads);
        bytes += q->bytes;
        if ((int)g.size() == r->gmax) flush();
      }
      if (!g.empty()) flush();
    }
    i = e;
  }
}

bool launch_recorded(const Rec &rec, hipStream_t st, std::string &err) {
  std::vector<Unit> units;
  recorded_units(rec, units);
  for (const Unit &u : units) u(st);
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) {
    err = std::string("grouped launch: ") + hipGetErrorString(he);
    return false;
  }
  return true;
}
}  // namespace

PlainLoadVector::PlainLoadVector() { ++g_plain_lv; }
PlainLoadVector::~PlainLoadVector() { --g_plain_lv; }

bool enqueue_decompose(const Plan &pl, bool f64, const void *in, void *out, void *ws, void *stream,
                       std::string &err) {
  hipStream_t st = (hipStream_t)stream;
  if (pl.time)
    return f64 ? decompose4_t<double>(pl, (const double *)in, (double *)out, ws, st, err)
               : decompose4_t<float>(pl, (const float *)in, (float *)out, ws, st, err);
  return f64 ? decompose_t<double>(pl, (const double *)in, (double *)out, ws, st, err)
             : decompose_t<float>(pl, (const float *)in, (float *)out, ws, st, err);
}

bool enqueue_recompose(const Plan &pl, bool f64, const void *in, void *out, void *ws, void *stream,
                       std::string &err, int nkeep, const StreamFork *fk) {
  hipStream_t st = (hipStream_t)stream;
  if (pl.time)
    return f64 ? recompose4_t<double>(pl, (const double *)in, (double *)out, ws, st, err)
               : recompose4_t<float>(pl, (const float *)in, (float *)out, ws, st, err);
  if (nkeep < 0) nkeep = pl.nlev;
  return f64 ? recompose_t<double>(pl, (const double *)in, (double *)out, ws, st, err, nkeep, fk)
             : recompose_t<float>(pl, (const float *)in, (float *)out, ws, st, err, nkeep, fk);
}

}  // namespace mgr
