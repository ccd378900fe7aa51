// mgr_plan.cpp -- FP64 host tables for one refactoring request.
//
// Everything here is plain FP64 arithmetic on the coordinates, done once per
// (shape, coords, nlevels) and uploaded; the kernels never divide.
//
// Operators of one step along one dimension (arXiv 2105.12764, Sec. II-A.2
// and the matrices of Sec. III-A.2), on level nodes x_0 < ... < x_{m-1} with
// spacings h_i = x_{i+1} - x_i and coarse positions 0, 2, 4, ... and m-1:
//   P (prolongation): a coarse position copies its coarse value; a fine
//     position i takes (1 - r_i) v_left + r_i v_right with
//     r_i = h_{i-1} / (h_{i-1} + h_i)  (the paper's r, Sec. III-A.2);
//   M (mass matrix, scaled by 6): diagonal 2(h_{i-1} + h_i), off-diagonals
//     h_{i-1} and h_i -- the paper's printed matrix with its spacing index
//     read as the interval to the left / right of node i;
//   R = P^T, and the load vector row J is (P^T M) restricted to the fine
//     positions 2J-2 .. 2J+2 (the paper's merged "mass-trans" operator,
//     computed here as the product instead of transcribing its garbled
//     closed form);
//   the correction solve uses M (scaled by 6) on the coarse coordinates; the
//     common factor 6 cancels against the load vector.
//
// Solve factorisation (exact, not approximate): a line of c unknowns is cut
// into P partitions of S positions; the last position of each partition but
// the last is a separator.  Each partition's interior is eliminated on its
// own (block Thomas factors w, 1/b'), which expresses it as
//   x = y - t_left * Ls - t_right * Rs
// with y the interior solve of the right-hand side and Ls, Rs the interior
// responses to unit separator values.  Substituting into the separator rows
// leaves a tridiagonal system in the P-1 separators, factorised here as well.
#include "mgr_plan.hpp"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

namespace mgr {

Plan::~Plan() {
  if (dev_tables) {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != device) (void)hipSetDevice(device);
    (void)hipFree(dev_tables);
    if (cur != device && cur >= 0) (void)hipSetDevice(cur);
  }
}

int max_levels3(const int64_t n[kDims]) {
  int best = 0;
  for (int k = 0; k < kDims; ++k) {
    int steps = 0;
    for (int64_t m = n[k]; m > 2; m = coarse_count(m)) ++steps;
    if (steps > best) best = steps;
  }
  return best;
}

int max_levels4(int64_t nt, const int64_t n[kDims]) {
  int steps = 0;
  for (int64_t m = nt; m > 2; m = coarse_count(m)) ++steps;
  return std::max(steps, max_levels3(n));
}

size_t workspace_bytes4(int64_t nt, const int64_t n[kDims], int nlev, size_t elem_size) {
  if (nlev <= 0) return 0;
  int64_t cs = 1;
  for (int k = 0; k < kDims; ++k) cs *= coarse_count(n[k]);
  const int64_t c4 = coarse_count(nt) * cs;
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  (void)elem_size;  // level grids in FP64, as in 3-D
  return 3 * al((size_t)c4 * sizeof(double)) + al((size_t)(nt * cs) * sizeof(double));
}

size_t workspace_bytes(const int64_t n[kDims], int nlev, size_t elem_size) {
  if (nlev <= 0) return 0;
  int64_t c1 = 1, c2 = 1;
  for (int k = 0; k < kDims; ++k) {
    c1 *= coarse_count(n[k]);
    c2 *= coarse_count(coarse_count(n[k]));
  }
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  // two coarse level grids in FP64 (ping-pong; a decomposition keeps its
  // coarser level grids in FP64 whatever the field's type) + one FP64
  // load/correction grid, and with two or more levels one more FP64 grid of the
  // next level's size for the coarser levels while the finest level's
  // recompose load vector and solves run beside them
  (void)elem_size;
  size_t b = 3 * al((size_t)c1 * sizeof(double));
  if (nlev >= 2) b += al((size_t)c2 * sizeof(double));
  return b;
}

namespace {

// Accumulates host tables into one byte image with 16-byte aligned entries.
struct Image {
  std::vector<char> bytes;
  template <typename T>
  size_t put(const std::vector<T> &v) {
    size_t off = (bytes.size() + 15) / 16 * 16;
    bytes.resize(off + v.size() * sizeof(T) + 16);
    if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

struct HostDim {
  size_t nodal = 0, r = 0, W = 0, sub = 0, sup = 0, w = 0, invb = 0, supi = 0, Ls = 0, Rs = 0,
         sepa = 0, sepe = 0, wr = 0, invbr = 0, gam = 0, tw = 0, tinvb = 0;
  bool has_solve = false;
};

int64_t coarse_index(int64_t m, int64_t i) {
  if (m < 3) return i;
  return (i == m - 1) ? coarse_count(m) - 1 : i / 2;
}
bool is_coarse(int64_t m, int64_t i) { return m < 3 || i % 2 == 0 || i == m - 1; }

// Partition length for a line of c unknowns: the smallest of 8/16/32/64 that
// needs at most kMaxBlocks partitions, else 64 for up to kLongBlocks
// partitions (the long-line solver); 0 selects the sequential fallback.
int pick_partition(int64_t c) {
  for (int S : {8, 16, 32, 64})
    if ((c + S - 1) / S <= kMaxBlocks) return S;
  if ((c + 63) / 64 <= kLongBlocks) return 64;
  return 0;
}

struct SolveTabs {
  std::vector<double> sub, sup, w, invb, supi, Ls, Rs, sepa, sepe, wr, invbr, gam, tw, tinvb;
  int S = 0, P = 1;
};

SolveTabs solve_tables(const std::vector<double> &X) {
  const int64_t c = (int64_t)X.size();
  SolveTabs t;
  t.S = pick_partition(c);
  const int64_t S = t.S ? t.S : c;   // fallback: one partition = whole line
  t.P = (int)((c + S - 1) / S);
  const int P = t.P;
  std::vector<double> a(c), b(c), e(c);
  for (int64_t i = 0; i < c; ++i) {
    double hl = i > 0 ? X[i] - X[i - 1] : 0.0;
    double hr = i < c - 1 ? X[i + 1] - X[i] : 0.0;
    a[i] = hl;
    e[i] = hr;
    b[i] = 2.0 * (hl + hr);
  }
  t.sub = a;
  t.sup = e;
  // partition tables padded to P*S; separator and padding slots pass through
  const int64_t cp = (int64_t)P * S;
  t.w.assign(cp, 0.0);
  t.invb.assign(cp, 1.0);
  t.supi.assign(cp, 0.0);
  t.Ls.assign(cp, 0.0);
  t.Rs.assign(cp, 0.0);
  // interior [f, l] of partition p
  auto first = [&](int p) { return (int64_t)p * S; };
  auto last = [&](int p) { return p < P - 1 ? (int64_t)(p + 1) * S - 2 : c - 1; };
  for (int p = 0; p < P; ++p) {
    int64_t f = first(p), l = last(p);
    double piv = b[f];
    t.w[f] = 0.0;
    t.invb[f] = 1.0 / piv;
    for (int64_t i = f + 1; i <= l; ++i) {
      t.w[i] = a[i] / piv;
      piv = b[i] - t.w[i] * e[i - 1];
      t.invb[i] = 1.0 / piv;
    }
    for (int64_t i = f; i < l; ++i) t.supi[i] = e[i];
    // interior solve with the tables, as the kernels do it
    auto interior_solve = [&](std::vector<double> &d) {
      for (int64_t i = f + 1; i <= l; ++i) d[i] -= t.w[i] * d[i - 1];
      d[l] *= t.invb[l];
      for (int64_t i = l - 1; i >= f; --i) d[i] = (d[i] - e[i] * d[i + 1]) * t.invb[i];
    };
    if (p > 0) {  // left separator at f-1 couples through a_f
      std::vector<double> d(c, 0.0);
      d[f] = a[f];
      interior_solve(d);
      for (int64_t i = f; i <= l; ++i) t.Ls[i] = d[i];
    }
    if (p < P - 1) {  // right separator at l+1 couples through e_l
      std::vector<double> d(c, 0.0);
      d[l] = e[l];
      interior_solve(d);
      for (int64_t i = f; i <= l; ++i) t.Rs[i] = d[i];
    }
  }
  // separator system
  t.sepa.assign(std::max(P - 1, 1), 0.0);
  t.sepe.assign(std::max(P - 1, 1), 0.0);
  if (P > 1) {
    std::vector<double> al(P - 1), be(P - 1), ga(P - 1);
    for (int p = 0; p < P - 1; ++p) {
      int64_t s = last(p) + 1;
      t.sepa[p] = a[s];
      t.sepe[p] = e[s];
      al[p] = -a[s] * t.Ls[s - 1];
      be[p] = b[s] - a[s] * t.Rs[s - 1] - e[s] * t.Ls[s + 1];
      ga[p] = -e[s] * t.Rs[s + 1];
    }
    t.wr.assign(P - 1, 0.0);
    t.invbr.assign(P - 1, 0.0);
    t.gam = ga;
    double piv = be[0];
    t.invbr[0] = 1.0 / piv;
    for (int p = 1; p < P - 1; ++p) {
      t.wr[p] = al[p] / piv;
      piv = be[p] - t.wr[p] * ga[p - 1];
      t.invbr[p] = 1.0 / piv;
    }
  } else {
    t.wr.assign(1, 0.0);
    t.invbr.assign(1, 0.0);
    t.gam.assign(1, 0.0);
  }
  // whole-line Thomas factors (one partition), for the single-workgroup tail
  t.tw.assign(c, 0.0);
  t.tinvb.assign(c, 0.0);
  double piv = b[0];
  t.tinvb[0] = 1.0 / piv;
  for (int64_t i = 1; i < c; ++i) {
    t.tw[i] = a[i] / piv;
    piv = b[i] - t.tw[i] * e[i - 1];
    t.tinvb[i] = 1.0 / piv;
  }
  return t;
}

}  // namespace

std::unique_ptr<Plan> build_plan(int ndim, const int64_t n[kDims],
                                 const std::vector<std::vector<double>> &coords,
                                 int nlev, std::string &err, int &status, bool allow_tail,
                                 const TableTarget *target) {
  auto plan = std::make_unique<Plan>();
  plan->ndim = ndim;
  for (int k = 0; k < kDims; ++k) plan->n[k] = n[k];
  plan->nlev = nlev;
  plan->lev.resize(nlev + 1);

  // level coordinates and finest indices per dim
  std::vector<std::vector<double>> x(kDims);
  std::vector<std::vector<int64_t>> idx(kDims);
  for (int k = 0; k < kDims; ++k) {
    x[k] = coords[k];
    idx[k].resize(n[k]);
    for (int64_t i = 0; i < n[k]; ++i) idx[k][i] = i;
  }
  const int64_t fstride[kDims] = {n[1] * n[2], n[2], 1};

  Image img;
  std::vector<std::array<HostDim, kDims>> hd(nlev + 1);
  size_t hd_tail[3] = {0, 0, 0};
  for (int s = 0; s <= nlev; ++s) {
    Level &L = plan->lev[s];
    for (int k = 0; k < kDims; ++k) {
      const int64_t m = (int64_t)x[k].size();
      const bool co = (s < nlev) && m >= 3;
      const int64_t c = co ? coarse_count(m) : m;
      L.m[k] = m;
      L.c[k] = c;
      L.co[k] = co;
      std::vector<int64_t> nodal(m);
      for (int64_t i = 0; i < m; ++i) nodal[i] = idx[k][i] * fstride[k];
      hd[s][k].nodal = img.put(nodal);
      std::vector<double> r(m, 0.0);
      if (co)
        for (int64_t i = 0; i < m; ++i)
          if (!is_coarse(m, i))
            r[i] = (x[k][i] - x[k][i - 1]) / (x[k][i + 1] - x[k][i - 1]);
      hd[s][k].r = img.put(r);
      if (!co) continue;
      // load-vector taps: row J of P^T M on the fine positions 2J-2 .. 2J+2
      std::vector<double> W((size_t)c * kTaps, 0.0);
      auto M6 = [&](int64_t q, int64_t i) -> double {
        double hl = q > 0 ? x[k][q] - x[k][q - 1] : 0.0;
        double hr = q < m - 1 ? x[k][q + 1] - x[k][q] : 0.0;
        if (i == q) return 2.0 * (hl + hr);
        if (i == q - 1) return hl;
        if (i == q + 1) return hr;
        return 0.0;
      };
      for (int64_t q = 0; q < m; ++q) {
        // column entries P[q][J] of fine position q
        int64_t Js[2];
        double ws[2];
        int cnt = 0;
        if (is_coarse(m, q)) {
          Js[0] = coarse_index(m, q);
          ws[0] = 1.0;
          cnt = 1;
        } else {
          Js[0] = (q - 1) / 2;
          ws[0] = 1.0 - r[q];
          Js[1] = (q + 1) / 2;
          ws[1] = r[q];
          cnt = 2;
        }
        for (int a = 0; a < cnt; ++a)
          for (int64_t i = q - 1; i <= q + 1; ++i) {
            if (i < 0 || i >= m) continue;
            int64_t o = i - 2 * Js[a] + 2;
            if (o < 0 || o >= kTaps) {
              err = "internal: load-vector tap out of range";
              status = 2;
              return nullptr;
            }
            W[(size_t)Js[a] * kTaps + o] += ws[a] * M6(q, i);
          }
      }
      hd[s][k].W = img.put(W);
      // coarse coordinates and the correction solve
      std::vector<double> X;
      for (int64_t i = 0; i < m; ++i)
        if (is_coarse(m, i)) X.push_back(x[k][i]);
      SolveTabs st = solve_tables(X);
      HostDim &h = hd[s][k];
      h.has_solve = true;
      h.sub = img.put(st.sub);
      h.sup = img.put(st.sup);
      h.w = img.put(st.w);
      h.invb = img.put(st.invb);
      h.supi = img.put(st.supi);
      h.sepa = img.put(st.sepa);
      h.sepe = img.put(st.sepe);
      h.Ls = img.put(st.Ls);
      h.Rs = img.put(st.Rs);
      h.wr = img.put(st.wr);
      h.invbr = img.put(st.invbr);
      h.gam = img.put(st.gam);
      h.tw = img.put(st.tw);
      h.tinvb = img.put(st.tinvb);
      L.d[k].S = st.S;
      L.d[k].P = st.P;
    }
    // next level's coordinates and indices
    if (s < nlev)
      for (int k = 0; k < kDims; ++k) {
        const int64_t m = (int64_t)x[k].size();
        if (m < 3) continue;
        std::vector<double> nx;
        std::vector<int64_t> ni;
        for (int64_t i = 0; i < m; ++i)
          if (is_coarse(m, i)) {
            nx.push_back(x[k][i]);
            ni.push_back(idx[k][i]);
          }
        x[k] = nx;
        idx[k] = ni;
      }
  }
  plan->max_coarse = 0;
  if (nlev > 0) plan->max_coarse = plan->lev[0].c[0] * plan->lev[0].c[1] * plan->lev[0].c[2];
  // the tail runs the last levels whose grids and tables fit one workgroup's LDS
  {
    int64_t noff = 0, ndbl = 0;
    for (int k = 0; k < kDims; ++k) noff += plan->lev[nlev].m[k];
    plan->tail_start = nlev;
    for (int s = nlev - 1; allow_tail && s >= 0 && nlev - s <= kTailMaxLevels; --s) {
      const Level &L = plan->lev[s];
      if (L.m[0] * L.m[1] * L.m[2] > kTailNodes || L.m[0] > kTailMaxExtent || L.m[1] > kTailMaxExtent ||
          L.m[2] > kTailMaxExtent)
        break;
      for (int k = 0; k < kDims; ++k) {
        noff += L.m[k];
        ndbl += L.m[k] + (L.co[k] ? (kTaps + 3) * L.c[k] : 0);
      }
      if (noff > kTailOffsets || ndbl > kTailDoubles) break;
      plan->tail_start = s;
    }
  }
  const int ntail = nlev - plan->tail_start;
  if (ntail > 0) {
    // pack the tail tables from the host image
    std::vector<TailLevel> tl((size_t)ntail + 1);
    std::vector<int64_t> toff;
    std::vector<double> tdbl;
    auto copy_d = [&](size_t at, int64_t cnt) {
      const int o = (int)tdbl.size();
      const double *src = (const double *)(img.bytes.data() + at);
      tdbl.insert(tdbl.end(), src, src + cnt);
      return o;
    };
    for (int t = 0; t <= ntail; ++t) {
      const int s = plan->tail_start + t;
      const Level &L = plan->lev[s];
      TailLevel &e = tl[t];
      for (int k = 0; k < kDims; ++k) {
        const HostDim &h = hd[s][k];
        e.m[k] = (int)L.m[k];
        e.c[k] = (int)L.c[k];
        e.co[k] = L.co[k] ? 1 : 0;
        e.nodal[k] = (int)toff.size();
        const int64_t *nsrc = (const int64_t *)(img.bytes.data() + h.nodal);
        toff.insert(toff.end(), nsrc, nsrc + L.m[k]);
        if (t == ntail) continue;
        e.r[k] = copy_d(h.r, L.m[k]);
        if (!L.co[k]) continue;
        e.W[k] = copy_d(h.W, (int64_t)kTaps * L.c[k]);
        e.sup[k] = copy_d(h.sup, L.c[k]);
        e.tw[k] = copy_d(h.tw, L.c[k]);
        e.tinvb[k] = copy_d(h.tinvb, L.c[k]);
      }
    }
    plan->tail_noff = (int)toff.size();
    plan->tail_ndbl = (int)tdbl.size();
    hd_tail[0] = img.put(tl);
    hd_tail[1] = img.put(toff);
    hd_tail[2] = img.put(tdbl);
  }

  // upload
  (void)hipGetDevice(&plan->device);
  plan->table_bytes = img.bytes.size();
  char *base = nullptr;
  if (target) {
    if (plan->table_bytes > target->bytes) {
      err = "plan tables need " + std::to_string(plan->table_bytes) + " bytes, more than the " +
            std::to_string(target->bytes) + " bytes reserved for them";
      status = 3;
      return nullptr;
    }
    base = (char *)target->base;
  } else {
    if (hipMalloc(&plan->dev_tables, plan->table_bytes) != hipSuccess) {
      (void)hipGetLastError();
      plan->dev_tables = nullptr;
      err = "hipMalloc of plan tables failed";
      status = 4;
      return nullptr;
    }
    base = (char *)plan->dev_tables;
  }
  for (int s = 0; s <= nlev; ++s)
    for (int k = 0; k < kDims; ++k) {
      DimTabs &d = plan->lev[s].d[k];
      const HostDim &h = hd[s][k];
      d.nodal = (const int64_t *)(base + h.nodal);
      d.r = (const double *)(base + h.r);
      if (plan->lev[s].co[k]) {
        d.W = (const double *)(base + h.W);
        d.sub = (const double *)(base + h.sub);
        d.sup = (const double *)(base + h.sup);
        d.w = (const double *)(base + h.w);
        d.invb = (const double *)(base + h.invb);
        d.supi = (const double *)(base + h.supi);
        d.sepa = (const double *)(base + h.sepa);
        d.sepe = (const double *)(base + h.sepe);
        d.Ls = (const double *)(base + h.Ls);
        d.Rs = (const double *)(base + h.Rs);
        d.wr = (const double *)(base + h.wr);
        d.invbr = (const double *)(base + h.invbr);
        d.gam = (const double *)(base + h.gam);
        d.tw = (const double *)(base + h.tw);
        d.tinvb = (const double *)(base + h.tinvb);
      }
    }
  if (ntail > 0) {
    plan->dev_tail = (const TailLevel *)(base + hd_tail[0]);
    plan->dev_tail_off = (const int64_t *)(base + hd_tail[1]);
    plan->dev_tail_dbl = (const double *)(base + hd_tail[2]);
  }
  if (target) {
    // from pageable host memory: the image is read before the call returns;
    // the plan keeps it anyway
    plan->host_image = std::move(img.bytes);
    if (hipMemcpyAsync(base, plan->host_image.data(), plan->table_bytes, hipMemcpyHostToDevice,
                       (hipStream_t)target->stream) != hipSuccess) {
      (void)hipGetLastError();
      err = "upload of plan tables failed";
      status = 5;
      return nullptr;
    }
  } else if (hipMemcpy(plan->dev_tables, img.bytes.data(), plan->table_bytes,
                       hipMemcpyHostToDevice) != hipSuccess) {
    err = "upload of plan tables failed";
    status = 5;
    return nullptr;
  }
  status = 0;
  return plan;
}

std::unique_ptr<Plan> build_plan4(int64_t nt, const int64_t n[kDims],
                                  const std::vector<std::vector<double>> &coords, int nlev,
                                  std::string &err, int &status) {
  std::vector<std::vector<double>> cs(coords.begin() + 1, coords.end());
  auto plan = build_plan(kDims, n, cs, nlev, err, status, false);
  if (!plan) return nullptr;
  const int64_t tn[kDims] = {1, 1, nt};
  std::vector<std::vector<double>> ct = {{0.0}, {0.0}, coords[0]};
  plan->time = build_plan(1, tn, ct, nlev, err, status, false);
  if (!plan->time) return nullptr;
  plan->ndim = 4;
  plan->nt = nt;
  plan->tpos.resize(nlev + 1);
  std::vector<int64_t> idx(nt);
  for (int64_t t = 0; t < nt; ++t) idx[t] = t;
  for (int s = 0; s <= nlev; ++s) {
    plan->tpos[s] = idx;
    const int64_t m = (int64_t)idx.size();
    if (s == nlev || m < 3) continue;
    std::vector<int64_t> nx;
    for (int64_t i = 0; i < m; ++i)
      if (is_coarse(m, i)) nx.push_back(idx[i]);
    idx = nx;
  }
  return plan;
}

}  // namespace mgr
