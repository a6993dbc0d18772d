"""Leaf-box Chebyshev grids of the method (test infrastructure only; see the
oracle package docstring for who may import it).

Every box carries a p x p x p grid of first-kind Chebyshev points (Sec. 3.1,
upward pass).  Two operations connect points and grids:

* anterpolation (upward pass): proxy strengths on the grid of the point's box,
  rho~(j) = sum_a rho_a l_j(x_a), with l_j the tensor-product Lagrange basis
  on the grid; the proxy field reproduces the field of the points for kernels
  that are smooth over the box;
* leaf evaluation (downward pass, last step): a potential given by its values
  on a box's grid is evaluated at the targets in the box through its
  interpolating polynomial, u(x) = sum_j U(j) l_j(x).

Grids of all boxes of an n0 x n1 x n2 tiling form one tensor of
(n0 p) x (n1 p) x (n2 p) values, index g_i = b_i p + j_i along each axis
(the layout the far field uses).  The box of a point and its wrapped
coordinate follow the binning's rules (y = x - L floor(x / L) on periodic
axes, b_i = min(n_i - 1, max(0, floor(y (n_i / L_i))))).  The Lagrange
basis is evaluated by its defining product, in float64.
"""
from __future__ import annotations

import numpy as np

from . import cheb_points


def lagrange(t, p):
    """l_j(t) for t in [-1, 1] (array of shape (N,)) -> (N, p), by the product
    prod_{k != j} (t - eta_k) / (eta_j - eta_k)."""
    eta = cheb_points(p)
    t = np.asarray(t, dtype=np.float64)
    out = np.ones((t.size, p))
    for j in range(p):
        for k in range(p):
            if k != j:
                out[:, j] *= (t - eta[k]) / (eta[j] - eta[k])
    return out


def _local(L, D, n, x):
    """(box index per axis (N, 3), box-local coordinates in [-1, 1] (N, 3))."""
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    Lv = np.asarray(L, dtype=np.float64)
    nv = np.asarray(n, dtype=np.int64)
    y = x.copy()
    for ax in range(int(D)):
        y[:, ax] = x[:, ax] - Lv[ax] * np.floor(x[:, ax] / Lv[ax])
    inv = nv.astype(np.float64) / Lv
    s = y * inv
    b = np.clip(np.floor(s), 0, nv - 1).astype(np.int64)
    return b, 2.0 * (s - b) - 1.0


def anterp(L, D, n, p, x, rho):
    """Proxy strengths rho_grid[m][n0 p][n1 p][n2 p] of points x[N][3] with
    strengths rho[N][m]."""
    rho = np.asarray(rho, dtype=np.float64).reshape(len(x), -1)
    b, t = _local(L, D, n, x)
    l0, l1, l2 = (lagrange(t[:, i], p) for i in range(3))
    out = np.zeros((rho.shape[1], n[0] * p, n[1] * p, n[2] * p))
    for a in range(len(x)):
        blk = np.einsum("i,j,k->ijk", l0[a], l1[a], l2[a])
        s0, s1, s2 = (slice(b[a, i] * p, (b[a, i] + 1) * p) for i in range(3))
        for q in range(rho.shape[1]):
            out[q, s0, s1, s2] += rho[a, q] * blk
    return out


def evaluate(L, D, n, p, x, u_grid):
    """u[N][m] at points x from grid values u_grid[m][n0 p][n1 p][n2 p]."""
    u_grid = np.asarray(u_grid, dtype=np.float64)
    b, t = _local(L, D, n, x)
    l0, l1, l2 = (lagrange(t[:, i], p) for i in range(3))
    out = np.zeros((len(b), u_grid.shape[0]))
    for a in range(len(b)):
        s0, s1, s2 = (slice(b[a, i] * p, (b[a, i] + 1) * p) for i in range(3))
        for q in range(u_grid.shape[0]):
            out[a, q] = np.einsum("ijk,i,j,k->", u_grid[q, s0, s1, s2], l0[a], l1[a], l2[a])
    return out
