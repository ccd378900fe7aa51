/*
 * mgr_oracle.c -- plain FP64 CPU oracle for multigrid hierarchical data
 * refactoring (decomposition and recomposition of a structured N-D field).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it, to judge the HIP library.  It shares no code,
 * header, table or helper with the HIP library.
 *
 * Method: Chen et al., "Scalable Multigrid-based Hierarchical Scientific
 * Data Refactoring on GPUs" (arXiv 2105.12764), Sec. II-A:
 *   - Eq. (1): Q_{l-1}u = Q_l u - (I - Pi_{l-1}) Q_l u + (Q_{l-1}u - Pi_{l-1} Q_l u)
 *   - Sec. II-A.1 "Compute coefficients": value minus the multilinear
 *     interpolant from the coarser grid, non-zero only on N_l \ N_{l-1}.
 *   - Sec. II-A.2 "Compute correction", Eq. (2) and the variational problem
 *     after it: M_{l-1} z_{l-1} = f_{l-1}, f_{l-1} = R_l M_l vec(C_l), with
 *     M_{l-1} the tensor product of 1-D mass matrices and R_l the transfer
 *     matrix from V_l to V_{l-1}.
 *   - Sec. II-A "Overall decomposition/recomposition process": correction
 *     dimension by dimension in a prescribed order; recomposition runs the
 *     stages in reverse, coarsest to finest.
 *   - Sec. III-A.3: the correction systems are solved with the Thomas
 *     algorithm (forward elimination, backward substitution).
 *
 * Readings where the paper is silent or garbled (each is a convention of
 * this implementation, not a fact of the paper):
 *   - Mass matrix: the Gram matrix of the piecewise-linear hat basis,
 *     M_ii = (h_{i-1} + h_i)/3, M_{i,i+1} = h_i/6 (the paper prints 6x this
 *     with its spacing indices shifted by one, Sec. III-A.2; a common scale
 *     cancels between the load vector and the solve).
 *   - Transfer matrix R = P^T, P the piecewise-linear prolongation from the
 *     coarse grid to the fine grid (forced by the variational problem: a
 *     coarse hat function is a P-weighted sum of fine hat functions).
 *   - Nesting: along a dimension with m >= 3 level nodes the coarse nodes
 *     are positions 0, 2, 4, ... and m-1; a dimension with m = 2 is not
 *     coarsened (identity factor).  For m = 2^k + 1 this is the paper's
 *     dyadic hierarchy.
 *   - Correction dimensions are processed in order 0, 1, ..., d-1 (only
 *     rounding depends on the order).
 *   - Layout: C order (dim 0 slowest).  Output is nodal: the same shape as
 *     the input; a node dropped at a level holds that level's coefficient,
 *     nodes of the final coarsest grid hold Q_coarsest u.
 *   - Coordinates default to 0, 1, ..., n-1 per dimension.
 *
 * Parallelism: outer loops carry OpenMP pragmas over independent lines; each
 * output value is computed by one thread in the same operation order, so the
 * result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXDIM 4
#define ORC_MAXLEV 64

/* ---------------------------------------------------------------- nesting */

/* Number of nodes of the next coarser grid along one dimension. */
static int64_t coarse_count(int64_t m) { return m < 3 ? m : m / 2 + 1; }

/* Is level-grid position i (of m) also a node of the next coarser grid? */
static int is_coarse(int64_t m, int64_t i) {
  if (m < 3) return 1;
  return (i % 2 == 0) || (i == m - 1);
}

/* Coarse-grid index of a coarse position i. */
static int64_t coarse_index(int64_t m, int64_t i) {
  if (m < 3) return i;
  return (i == m - 1) ? coarse_count(m) - 1 : i / 2;
}

static int64_t prod(const int64_t *m, int nd) {
  int64_t p = 1;
  for (int k = 0; k < nd; ++k) p *= m[k];
  return p;
}

/* Split a shape into (outer, len, inner) around axis k. */
static void axis_split(const int64_t *sh, int nd, int k, int64_t *outer,
                       int64_t *len, int64_t *inner) {
  *outer = prod(sh, k);
  *len = sh[k];
  *inner = prod(sh + k + 1, nd - k - 1);
}

/* ------------------------------------------------- 1-D operators along axis */

/* Prolongation P along axis k: src has c = coarse_count(m) nodes along k,
 * dst has m nodes.  Coarse positions copy; a fine position i takes the
 * linear interpolant of its coarse neighbours i-1 and i+1 (coords x). */
static void interp_axis(const double *src, double *dst, const int64_t *dst_sh,
                        int nd, int k, const double *x) {
  int64_t outer, m, inner;
  axis_split(dst_sh, nd, k, &outer, &m, &inner);
  int64_t c = coarse_count(m);
#pragma omp parallel for schedule(static)
  for (int64_t o = 0; o < outer; ++o) {
    for (int64_t i = 0; i < m; ++i) {
      double *d = dst + (o * m + i) * inner;
      if (is_coarse(m, i)) {
        const double *s = src + (o * c + coarse_index(m, i)) * inner;
        for (int64_t t = 0; t < inner; ++t) d[t] = s[t];
      } else {
        double wl = (x[i + 1] - x[i]) / (x[i + 1] - x[i - 1]);
        double wr = (x[i] - x[i - 1]) / (x[i + 1] - x[i - 1]);
        const double *sl = src + (o * c + (i - 1) / 2) * inner;
        const double *sr = src + (o * c + (i + 1) / 2) * inner;
        for (int64_t t = 0; t < inner; ++t) d[t] = wl * sl[t] + wr * sr[t];
      }
    }
  }
}

/* Mass matrix product y = M x along axis k, M the Gram matrix of the hat
 * basis on nodes x[0..m-1]. */
static void mass_axis(const double *src, double *dst, const int64_t *sh,
                      int nd, int k, const double *x) {
  int64_t outer, m, inner;
  axis_split(sh, nd, k, &outer, &m, &inner);
#pragma omp parallel for schedule(static)
  for (int64_t o = 0; o < outer; ++o) {
    for (int64_t i = 0; i < m; ++i) {
      double hl = (i > 0) ? x[i] - x[i - 1] : 0.0;
      double hr = (i < m - 1) ? x[i + 1] - x[i] : 0.0;
      double diag = (hl + hr) / 3.0, lo = hl / 6.0, up = hr / 6.0;
      double *d = dst + (o * m + i) * inner;
      const double *s0 = src + (o * m + i) * inner;
      for (int64_t t = 0; t < inner; ++t) {
        double v = diag * s0[t];
        if (i > 0) v += lo * s0[t - inner];
        if (i < m - 1) v += up * s0[t + inner];
        d[t] = v;
      }
    }
  }
}

/* Restriction R = P^T along axis k: src has m nodes along k, dst has
 * coarse_count(m).  Written as the transpose of interp_axis: every fine
 * value is scattered with the weights it was interpolated with. */
static void restrict_axis(const double *src, double *dst, const int64_t *src_sh,
                          int nd, int k, const double *x) {
  int64_t outer, m, inner;
  axis_split(src_sh, nd, k, &outer, &m, &inner);
  int64_t c = coarse_count(m);
#pragma omp parallel for schedule(static)
  for (int64_t o = 0; o < outer; ++o) {
    for (int64_t j = 0; j < c * inner; ++j) dst[o * c * inner + j] = 0.0;
    for (int64_t i = 0; i < m; ++i) {
      const double *s = src + (o * m + i) * inner;
      if (is_coarse(m, i)) {
        double *d = dst + (o * c + coarse_index(m, i)) * inner;
        for (int64_t t = 0; t < inner; ++t) d[t] += s[t];
      } else {
        double wl = (x[i + 1] - x[i]) / (x[i + 1] - x[i - 1]);
        double wr = (x[i] - x[i - 1]) / (x[i + 1] - x[i - 1]);
        double *dl = dst + (o * c + (i - 1) / 2) * inner;
        double *dr = dst + (o * c + (i + 1) / 2) * inner;
        for (int64_t t = 0; t < inner; ++t) {
          dl[t] += wl * s[t];
          dr[t] += wr * s[t];
        }
      }
    }
  }
}

/* Solve M z = f along axis k (in place), M the hat-basis mass matrix on
 * nodes x[0..m-1], by the Thomas algorithm: forward elimination then
 * backward substitution on every line. */
static void thomas_axis(double *a, const int64_t *sh, int nd, int k,
                        const double *x) {
  int64_t outer, m, inner;
  axis_split(sh, nd, k, &outer, &m, &inner);
  double *sub = malloc(sizeof(double) * m), *dia = malloc(sizeof(double) * m),
         *sup = malloc(sizeof(double) * m), *cp = malloc(sizeof(double) * m);
  for (int64_t i = 0; i < m; ++i) {
    double hl = (i > 0) ? x[i] - x[i - 1] : 0.0;
    double hr = (i < m - 1) ? x[i + 1] - x[i] : 0.0;
    sub[i] = hl / 6.0;
    dia[i] = (hl + hr) / 3.0;
    sup[i] = hr / 6.0;
  }
  /* c'_0 = c_0 / b_0 ; c'_i = c_i / (b_i - a_i c'_{i-1}) */
  cp[0] = sup[0] / dia[0];
  for (int64_t i = 1; i < m; ++i) cp[i] = sup[i] / (dia[i] - sub[i] * cp[i - 1]);
#pragma omp parallel for schedule(static)
  for (int64_t o = 0; o < outer; ++o) {
    for (int64_t t = 0; t < inner; ++t) {
      double *line = a + o * m * inner + t;
      /* d'_0 = d_0 / b_0 ; d'_i = (d_i - a_i d'_{i-1}) / (b_i - a_i c'_{i-1}) */
      line[0] = line[0] / dia[0];
      for (int64_t i = 1; i < m; ++i)
        line[i * inner] = (line[i * inner] - sub[i] * line[(i - 1) * inner]) /
                          (dia[i] - sub[i] * cp[i - 1]);
      /* z_{m-1} = d'_{m-1} ; z_i = d'_i - c'_i z_{i+1} */
      for (int64_t i = m - 2; i >= 0; --i)
        line[i * inner] = line[i * inner] - cp[i] * line[(i + 1) * inner];
    }
  }
  free(sub);
  free(dia);
  free(sup);
  free(cp);
}

/* ----------------------------------------------------------- level grids */

typedef struct {
  int nd;
  int64_t n[ORC_MAXDIM];               /* finest shape */
  int nlev;                            /* number of decomposition steps */
  int64_t m[ORC_MAXLEV + 1][ORC_MAXDIM];   /* level-grid shape per step */
  int64_t *idx[ORC_MAXLEV + 1][ORC_MAXDIM];/* finest index of each level node */
  double *x[ORC_MAXLEV + 1][ORC_MAXDIM];   /* coordinate of each level node */
} hierarchy;

static void hier_free(hierarchy *H) {
  for (int s = 0; s <= H->nlev; ++s)
    for (int k = 0; k < H->nd; ++k) {
      free(H->idx[s][k]);
      free(H->x[s][k]);
    }
}

static int hier_build(hierarchy *H, int nd, const int64_t *n,
                      const double *const *coords, int nlev) {
  memset(H, 0, sizeof(*H));
  H->nd = nd;
  H->nlev = nlev;
  for (int k = 0; k < nd; ++k) {
    H->n[k] = n[k];
    H->m[0][k] = n[k];
    H->idx[0][k] = malloc(sizeof(int64_t) * n[k]);
    H->x[0][k] = malloc(sizeof(double) * n[k]);
    for (int64_t i = 0; i < n[k]; ++i) {
      H->idx[0][k][i] = i;
      H->x[0][k][i] = (coords && coords[k]) ? coords[k][i] : (double)i;
    }
  }
  for (int s = 0; s < nlev; ++s)
    for (int k = 0; k < nd; ++k) {
      int64_t m = H->m[s][k], c = coarse_count(m);
      H->m[s + 1][k] = c;
      H->idx[s + 1][k] = malloc(sizeof(int64_t) * c);
      H->x[s + 1][k] = malloc(sizeof(double) * c);
      for (int64_t i = 0; i < m; ++i)
        if (is_coarse(m, i)) {
          H->idx[s + 1][k][coarse_index(m, i)] = H->idx[s][k][i];
          H->x[s + 1][k][coarse_index(m, i)] = H->x[s][k][i];
        }
    }
  return 0;
}

/* Flat finest-array offset of level-s node with flat level index f. */
static int64_t finest_offset(const hierarchy *H, int s, int64_t f) {
  int64_t off = 0, stride = 1, rem = f;
  int64_t mi[ORC_MAXDIM];
  for (int k = H->nd - 1; k >= 0; --k) {
    mi[k] = rem % H->m[s][k];
    rem /= H->m[s][k];
  }
  for (int k = H->nd - 1; k >= 0; --k) {
    off += H->idx[s][k][mi[k]] * stride;
    stride *= H->n[k];
  }
  return off;
}

/* Is level-s node f a node of level s+1 (coarse along every dimension)? */
static int node_is_coarse(const hierarchy *H, int s, int64_t f) {
  int64_t rem = f;
  for (int k = H->nd - 1; k >= 0; --k) {
    int64_t i = rem % H->m[s][k];
    rem /= H->m[s][k];
    if (!is_coarse(H->m[s][k], i)) return 0;
  }
  return 1;
}

/* Flat level-(s+1) index of a coarse level-s node f. */
static int64_t node_coarse_index(const hierarchy *H, int s, int64_t f) {
  int64_t rem = f, out = 0, stride = 1;
  for (int k = H->nd - 1; k >= 0; --k) {
    int64_t i = rem % H->m[s][k];
    rem /= H->m[s][k];
    out += coarse_index(H->m[s][k], i) * stride;
    stride *= H->m[s + 1][k];
  }
  return out;
}

/* Correction z_{l-1} for coefficient array C (level-s shape):
 * f = (P^T M)_0 ... (P^T M)_{d-1} C, then z = M_{l-1}^{-1} f dimension by
 * dimension.  Dimensions that are not coarsened are left alone (P = I there,
 * so the mass product and the solve cancel).  Returns a malloc'd array of the
 * level-(s+1) shape. */
static double *correction(const hierarchy *H, int s, const double *C) {
  int nd = H->nd;
  int64_t sh[ORC_MAXDIM];
  for (int k = 0; k < nd; ++k) sh[k] = H->m[s][k];
  int64_t cnt = prod(sh, nd);
  double *cur = malloc(sizeof(double) * cnt);
  memcpy(cur, C, sizeof(double) * cnt);
  for (int k = 0; k < nd; ++k) {
    if (H->m[s][k] < 3) continue;
    double *tmp = malloc(sizeof(double) * prod(sh, nd));
    mass_axis(cur, tmp, sh, nd, k, H->x[s][k]);
    int64_t sh2[ORC_MAXDIM];
    memcpy(sh2, sh, sizeof(sh2));
    sh2[k] = H->m[s + 1][k];
    double *nxt = malloc(sizeof(double) * prod(sh2, nd));
    restrict_axis(tmp, nxt, sh, nd, k, H->x[s][k]);
    free(tmp);
    free(cur);
    cur = nxt;
    sh[k] = sh2[k];
  }
  for (int k = 0; k < nd; ++k) {
    if (H->m[s][k] < 3) continue;
    thomas_axis(cur, sh, nd, k, H->x[s + 1][k]);
  }
  return cur;
}

/* Multilinear interpolant Pi_{l-1} of level-(s+1) values onto the level-s
 * grid, one dimension at a time.  Returns a malloc'd level-s array. */
static double *interpolate(const hierarchy *H, int s, const double *Uc) {
  int nd = H->nd;
  int64_t sh[ORC_MAXDIM];
  for (int k = 0; k < nd; ++k) sh[k] = H->m[s + 1][k];
  double *cur = malloc(sizeof(double) * prod(sh, nd));
  memcpy(cur, Uc, sizeof(double) * prod(sh, nd));
  for (int k = 0; k < nd; ++k) {
    int64_t sh2[ORC_MAXDIM];
    memcpy(sh2, sh, sizeof(sh2));
    sh2[k] = H->m[s][k];
    double *nxt = malloc(sizeof(double) * prod(sh2, nd));
    interp_axis(cur, nxt, sh2, nd, k, H->x[s][k]);
    free(cur);
    cur = nxt;
    sh[k] = sh2[k];
  }
  return cur;
}

/* ------------------------------------------------------------ public API */

int oracle_max_levels(int nd, const int64_t *n) {
  if (nd < 1 || nd > ORC_MAXDIM || !n) return -1;
  int best = 0;
  for (int k = 0; k < nd; ++k) {
    if (n[k] < 2) return -1;
    int steps = 0;
    for (int64_t m = n[k]; m > 2; m = coarse_count(m)) ++steps;
    if (steps > best) best = steps;
  }
  return best;
}

static int check_args(int nd, const int64_t *n, const double *const *coords,
                      int nlev) {
  int ml = oracle_max_levels(nd, n);
  if (ml < 0 || nlev < 0 || nlev > ml) return 1;
  if (coords)
    for (int k = 0; k < nd; ++k)
      if (coords[k])
        for (int64_t i = 0; i + 1 < n[k]; ++i)
          if (!(coords[k][i + 1] > coords[k][i]) || !isfinite(coords[k][i]) ||
              !isfinite(coords[k][i + 1]))
            return 1;
  return 0;
}

/* Decomposition, finest to coarsest (Eq. 1 applied nlev times).
 * in, out: finest arrays (C order, prod(n) doubles); may alias. */
int oracle_decompose(int nd, const int64_t *n, const double *const *coords,
                     int nlev, const double *in, double *out) {
  if (check_args(nd, n, coords, nlev)) return 1;
  hierarchy H;
  hier_build(&H, nd, n, coords, nlev);
  int64_t total = prod(n, nd);
  double *v = out;
  if (v != in) memcpy(v, in, sizeof(double) * total);
  for (int s = 0; s < nlev; ++s) {
    int64_t ns = prod(H.m[s], nd), nc = prod(H.m[s + 1], nd);
    /* U <- v on the level grid, U_c <- U on the coarser grid */
    double *U = malloc(sizeof(double) * ns), *Uc = malloc(sizeof(double) * nc);
    for (int64_t f = 0; f < ns; ++f) U[f] = v[finest_offset(&H, s, f)];
    for (int64_t f = 0; f < ns; ++f)
      if (node_is_coarse(&H, s, f)) Uc[node_coarse_index(&H, s, f)] = U[f];
    /* coefficients C = U - Pi U_c, exactly zero on the coarser grid */
    double *Pi = interpolate(&H, s, Uc);
    double *C = malloc(sizeof(double) * ns);
    for (int64_t f = 0; f < ns; ++f)
      C[f] = node_is_coarse(&H, s, f) ? 0.0 : U[f] - Pi[f];
    /* correction z and write-back */
    double *z = correction(&H, s, C);
    for (int64_t f = 0; f < ns; ++f) {
      int64_t off = finest_offset(&H, s, f);
      if (node_is_coarse(&H, s, f)) {
        int64_t cf = node_coarse_index(&H, s, f);
        v[off] = Uc[cf] + z[cf];
      } else {
        v[off] = C[f];
      }
    }
    free(U);
    free(Uc);
    free(Pi);
    free(C);
    free(z);
  }
  hier_free(&H);
  return 0;
}

/* Recomposition, coarsest to finest (the decomposition stages in reverse). */
int oracle_recompose(int nd, const int64_t *n, const double *const *coords,
                     int nlev, const double *in, double *out) {
  if (check_args(nd, n, coords, nlev)) return 1;
  hierarchy H;
  hier_build(&H, nd, n, coords, nlev);
  int64_t total = prod(n, nd);
  double *v = out;
  if (v != in) memcpy(v, in, sizeof(double) * total);
  for (int s = nlev - 1; s >= 0; --s) {
    int64_t ns = prod(H.m[s], nd), nc = prod(H.m[s + 1], nd);
    double *V = malloc(sizeof(double) * ns), *C = malloc(sizeof(double) * ns);
    double *Uc = malloc(sizeof(double) * nc);
    for (int64_t f = 0; f < ns; ++f) V[f] = v[finest_offset(&H, s, f)];
    for (int64_t f = 0; f < ns; ++f) C[f] = node_is_coarse(&H, s, f) ? 0.0 : V[f];
    /* the correction depends only on the level's coefficients */
    double *z = correction(&H, s, C);
    /* undo the correction on the coarser grid */
    for (int64_t f = 0; f < ns; ++f)
      if (node_is_coarse(&H, s, f)) {
        int64_t cf = node_coarse_index(&H, s, f);
        Uc[cf] = V[f] - z[cf];
      }
    /* add the interpolant back to the coefficients */
    double *Pi = interpolate(&H, s, Uc);
    for (int64_t f = 0; f < ns; ++f) {
      int64_t off = finest_offset(&H, s, f);
      v[off] = node_is_coarse(&H, s, f) ? Pi[f] : C[f] + Pi[f];
    }
    free(V);
    free(C);
    free(Uc);
    free(Pi);
    free(z);
  }
  hier_free(&H);
  return 0;
}
