"""Dense, independent characterisation of the multilevel decomposition.

Used only to pin the oracle.  It shares nothing with the oracle's operator
code: no prolongation, mass, restriction or Thomas routine is reused.  It
states what the decomposition *is* (arXiv 2105.12764, Sec. II-A, Eq. 1 and
the projection statement after Eq. 2):

* the nodes of the final coarse grid hold Q_s u, the L2 projection of the
  piecewise-multilinear interpolant u_h of the data onto V_s;
* a node dropped at step s holds (I - Pi_{s+1}) Q_s u there, i.e. the value of
  Q_s u minus its multilinear interpolant from the next coarser grid.

Building blocks, each from a definition or a library routine:

* hat-function Gram matrix by 2-point Gauss-Legendre quadrature on every
  finest interval (exact: products of two linears are quadratics);
* coarse basis functions evaluated at the finest nodes with ``np.interp``
  (the piecewise-linear interpolant in 1-D), tensorised with ``np.kron``;
* projections by a dense ``np.linalg.solve`` of the normal equations.

The nesting rule (coarse positions 0, 2, 4, ... and the last) is the
convention for sizes other than 2^k + 1; it is re-derived here.
"""
from __future__ import annotations

import numpy as np


def coarse_positions(m: int) -> np.ndarray:
    """Positions (within a level grid of m nodes) kept on the next coarser grid."""
    if m < 3:
        return np.arange(m)
    pos = list(range(0, m, 2))
    if pos[-1] != m - 1:
        pos.append(m - 1)
    return np.array(pos)


def level_coords(x: np.ndarray, nlevels: int):
    """Coordinates of every level grid, finest first (nlevels + 1 entries)."""
    out = [np.asarray(x, dtype=np.float64)]
    for _ in range(nlevels):
        out.append(out[-1][coarse_positions(len(out[-1]))])
    return out


def gram_quadrature(x: np.ndarray) -> np.ndarray:
    """Gram matrix (phi_i, phi_j) of the hat basis on nodes x (2-point Gauss)."""
    m = len(x)
    G = np.zeros((m, m))
    gp = (0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0))
    for e in range(m - 1):
        h = x[e + 1] - x[e]
        for t in gp:
            vals = {e: 1.0 - t, e + 1: t}
            for a, va in vals.items():
                for b, vb in vals.items():
                    G[a, b] += 0.5 * h * va * vb
    return G


def basis_at(x_fine: np.ndarray, x_coarse: np.ndarray) -> np.ndarray:
    """Matrix whose column J holds the coarse hat phi_J evaluated at x_fine."""
    B = np.zeros((len(x_fine), len(x_coarse)))
    for J in range(len(x_coarse)):
        e = np.zeros(len(x_coarse))
        e[J] = 1.0
        B[:, J] = np.interp(x_fine, x_coarse, e)
    return B


def kron_all(mats):
    out = mats[0]
    for A in mats[1:]:
        out = np.kron(out, A)
    return out


def dense_decompose(u: np.ndarray, coords, nlevels: int) -> np.ndarray:
    """Nodal decomposition from L2 projections (see module docstring)."""
    u = np.asarray(u, dtype=np.float64)
    shape = u.shape
    d = len(shape)
    if coords is None:
        coords = [np.arange(n, dtype=np.float64) for n in shape]
    xs = [level_coords(coords[k], nlevels) for k in range(d)]
    G0 = kron_all([gram_quadrature(xs[k][0]) for k in range(d)])
    uflat = u.reshape(-1)

    # q[s]: nodal values on level-s grid of Q_s u (q[0] = u)
    q = [u.copy()]
    for s in range(1, nlevels + 1):
        B = kron_all([basis_at(xs[k][0], xs[k][s]) for k in range(d)])
        A = B.T @ G0 @ B
        rhs = B.T @ (G0 @ uflat)
        qs = np.linalg.solve(A, rhs)
        q.append(qs.reshape([len(xs[k][s]) for k in range(d)]))

    # finest index of every level-s node, per dim
    idx = []
    for k in range(d):
        lev = [np.arange(shape[k])]
        for s in range(nlevels):
            lev.append(lev[-1][coarse_positions(len(lev[-1]))])
        idx.append(lev)

    out = np.zeros(shape)
    for s in range(nlevels):
        # (I - Pi_{s+1}) Q_s u on the level-s grid
        qs_c = q[s][np.ix_(*[coarse_positions(len(xs[k][s])) for k in range(d)])]
        interp = kron_all([basis_at(xs[k][s], xs[k][s + 1]) for k in range(d)])
        coeff = q[s].reshape(-1) - interp @ qs_c.reshape(-1)
        coeff = coeff.reshape(q[s].shape)
        out[np.ix_(*[idx[k][s] for k in range(d)])] = coeff
    out[np.ix_(*[idx[k][nlevels] for k in range(d)])] = q[nlevels]
    return out


def projection_residual(u: np.ndarray, coarse_vals: np.ndarray, coords, nlevels: int) -> float:
    """max |(u_h - Pi q, phi_J)| over coarse hats: zero iff q is the L2 projection."""
    shape = u.shape
    d = len(shape)
    if coords is None:
        coords = [np.arange(n, dtype=np.float64) for n in shape]
    xs = [level_coords(coords[k], nlevels) for k in range(d)]
    G0 = kron_all([gram_quadrature(xs[k][0]) for k in range(d)])
    B = kron_all([basis_at(xs[k][0], xs[k][nlevels]) for k in range(d)])
    r = B.T @ (G0 @ (u.reshape(-1) - B @ coarse_vals.reshape(-1)))
    return float(np.max(np.abs(r)))
