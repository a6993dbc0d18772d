"""Grids whose one-workgroup-per-item launches exceed 2^32 work-items.

A dispatch holds fewer than 2^32 work-items, so the library splits the pair
kernel (one workgroup of 256 threads per tile: more than 16,777,215 tiles)
and the tile walk of the binning (one wavefront per leaf column, four
columns per 256-thread workgroup: more than 67,108,860 columns) into several
launches.  These cases cross those limits
with sparse point sets and compare targets on both sides of each split with
the oracle.
"""
import numpy as np
import pytest

import oracle
from gpu_util import HAVE_GPU, assert_parity, dev, host, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    from paper_2606_27134_amd import residual as R

TOL = {"fp64": 1e-12, "fp32c": 1e-6}
T_C = 5.042030  # erfc(t_c) = 1e-12: Gaussian window at the cutoff
TILE_LAUNCH = 0xFFFFFFFF // 256  # tiles per launch of the 256-thread variants
COL_LAUNCH = (0xFFFFFFFF // 256) * 4  # columns per launch of the tile walk


def _lattice(n, seed):
    """One point per leaf column of an n x n x 1 grid of cubes (side h = 1/n),
    jittered around the column centre; free space (D = 0)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    i = np.arange(n * n)
    b0, b1 = np.divmod(i, n)
    x = np.empty((n * n, 3))
    x[:, 0] = (b0 + 0.5 + rng.uniform(-0.3, 0.3, n * n)) * h
    x[:, 1] = (b1 + 0.5 + rng.uniform(-0.3, 0.3, n * n)) * h
    x[:, 2] = rng.uniform(0.2, 0.8, n * n) * h
    rho = rng.normal(size=(n * n, 1))
    G = rng.normal(size=(n * n, 1))
    return x, rho, G, h


def _neighbourhood(t, n):
    """Indices of the points of column t and its (up to) 8 neighbours: points
    two or more columns apart are farther than the cutoff h."""
    b0, b1 = divmod(int(t), n)
    out = [t]
    for d0 in (-1, 0, 1):
        for d1 in (-1, 0, 1):
            c0, c1 = b0 + d0, b1 + d1
            if (d0 or d1) and 0 <= c0 < n and 0 <= c1 < n:
                out.append(c0 * n + c1)
    return np.array(out)


def test_pair_kernel_in_several_launches():
    n = 4200  # 17,640,000 single-point columns, one tile each
    x, rho, G, h = _lattice(n, 77)
    L = (1.0, 1.0, h)
    rc, sigma = h, h / T_C
    print("lattice", n, "N", n * n, flush=True)
    b = R.tree_bin(L, 0, (n, n, 1), dev(x))
    assert b.ntiles == n * n > TILE_LAUNCH
    tiles = host(b.tiles())
    perm = host(b.perm())
    rng = np.random.default_rng(78)
    pick = np.concatenate([rng.integers(0, TILE_LAUNCH, 96), rng.integers(TILE_LAUNCH, b.ntiles, 96),
                           [0, TILE_LAUNCH - 1, TILE_LAUNCH, b.ntiles - 1]])
    tgt = perm[tiles[pick, 3]]  # original index of each picked tile's (only) target
    ref_u, ref_gr, ref_gx = [], [], []
    for t in tgt:
        sub = _neighbourhood(t, n)
        ref_u.append(oracle.residual("laplace", 0, L, sigma, rc, x[sub], rho[sub], targets=[0])[0])
        gr, gx = oracle.residual_vjp("laplace", 0, L, sigma, rc, x[sub], rho[sub], G[sub], targets=[0])
        ref_gr.append(gr[0])
        ref_gx.append(gx[0])
    for prec in ("fp64", "fp32c"):
        print("prec", prec, flush=True)
        u = host(R.residual_eval(b, "laplace", prec, sigma, rc, dev(rho)))
        assert_parity(u[tgt], np.array(ref_u), TOL[prec], "fwd %s" % prec)
        gr, gx = R.residual_backward(b, "laplace", prec, sigma, rc, dev(rho), dev(G))
        assert_parity(host(gr)[tgt], np.array(ref_gr), TOL[prec], "grad_rho %s" % prec)
        assert_parity(host(gx)[tgt], np.array(ref_gx), TOL[prec], "grad_x %s" % prec)


def test_tile_walk_in_several_launches():
    n = 8193  # 67,125,249 leaf columns
    ncol = n * n
    assert ncol > COL_LAUNCH
    h = 1.0 / n
    rng = np.random.default_rng(79)
    # close pairs of points in 60,000 random columns and in the last 2,000
    cols = np.unique(np.concatenate([rng.choice(COL_LAUNCH, 60000, replace=False),
                                     np.arange(ncol - 2000, ncol)]))
    b0, b1 = np.divmod(cols, n)
    first = np.stack([(b0 + rng.uniform(0.3, 0.7, cols.size)) * h, (b1 + rng.uniform(0.3, 0.7, cols.size)) * h,
                      rng.uniform(0.3, 0.7, cols.size) * h], axis=1)
    second = first + rng.uniform(-0.25, 0.25, first.shape) * h
    x = np.concatenate([first, second])
    rho = rng.normal(size=(x.shape[0], 1))
    L = (1.0, 1.0, h)
    rc, sigma = h, h / T_C
    print("columns", ncol, "N", x.shape[0], flush=True)
    b = R.tree_bin(L, 0, (n, n, 1), dev(x))
    assert b.ntiles == cols.size  # one tile per non-empty column
    u = host(R.residual_eval(b, "laplace", "fp64", sigma, rc, dev(rho)))
    # every point in the columns of the second launch, and a sample of the rest
    late = np.nonzero(np.concatenate([cols, cols]) >= COL_LAUNCH)[0]
    tgt = np.concatenate([late, rng.integers(0, x.shape[0], 500)])
    ref = oracle.residual("laplace", 0, L, sigma, rc, x, rho, targets=tgt)
    assert_parity(u[tgt], ref, TOL["fp64"], "fwd fp64 (tile walk)")
