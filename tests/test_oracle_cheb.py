"""Pins of the oracle's leaf-box Chebyshev operations (anterpolation of the
upward pass, evaluation of the downward pass at the targets), and of the
single-level periodic split built from them.

Independent routes: the Lagrange basis is the identity on its nodes and a
partition of unity; interpolation reproduces polynomials of degree < p per
axis exactly (numpy's own polynomial evaluation); anterpolation preserves
every such polynomial moment; the interpolant of a trigonometric mode
converges spectrally; and proxy strengths -> far field on the grid ->
evaluation at the points, plus residual and self term, reproduce the NaCl
Madelung constant to the tolerance of the paper's parameters (p, c, N_per
of the Laplace table)."""
import os

import numpy as np
import pytest
from numpy.polynomial import polynomial as P

import oracle
from oracle import cheb
from oracle.pswf import PswfWindow


@pytest.mark.parametrize("p", [1, 2, 7, 20, 38])
def test_lagrange_nodes_and_partition_of_unity(p):
    eta = oracle.cheb_points(p)
    np.testing.assert_allclose(cheb.lagrange(eta, p), np.eye(p), rtol=0, atol=1e-14)
    t = np.random.default_rng(1).uniform(-1, 1, 200)
    np.testing.assert_allclose(cheb.lagrange(t, p).sum(axis=1), 1.0, rtol=0, atol=1e-12)


def _poly(rng, p):
    return rng.normal(size=(p, p, p)) / np.arange(1, p + 1)[:, None, None]


def test_interpolation_reproduces_polynomials():
    rng = np.random.default_rng(2)
    p, Lv, n = 6, (2.0, 1.0, 1.5), (4, 2, 3)
    X = oracle.top_grid(Lv, n, p)
    # a polynomial of degree < p per axis in each box's local coordinates is
    # reproduced exactly; use one global polynomial of the box-local t
    c = _poly(rng, p)
    G = np.stack(np.meshgrid(*X, indexing="ij"), axis=-1).reshape(-1, 3)
    b, t = cheb._local(Lv, 3, n, G)
    vals = P.polyval3d(t[:, 0], t[:, 1], t[:, 2], c).reshape(1, *[len(a) for a in X])
    x = rng.random((300, 3)) * np.asarray(Lv)
    got = cheb.evaluate(Lv, 3, n, p, x, vals)[:, 0]
    _, tx = cheb._local(Lv, 3, n, x)
    np.testing.assert_allclose(got, P.polyval3d(tx[:, 0], tx[:, 1], tx[:, 2], c), rtol=0, atol=1e-12)


def test_anterpolation_preserves_polynomial_moments():
    rng = np.random.default_rng(3)
    p, Lv, n = 5, (1.0, 1.0, 1.0), (2, 2, 2)
    x = rng.random((80, 3))
    rho = rng.normal(size=(80, 3))
    rg = cheb.anterp(Lv, 3, n, p, x, rho)
    X = oracle.top_grid(Lv, n, p)
    G = np.stack(np.meshgrid(*X, indexing="ij"), axis=-1).reshape(-1, 3)
    _, tg = cheb._local(Lv, 3, n, G)
    _, tx = cheb._local(Lv, 3, n, x)
    for _ in range(3):
        c = _poly(rng, p)
        lhs = rg.reshape(3, -1) @ P.polyval3d(tg[:, 0], tg[:, 1], tg[:, 2], c)
        rhs = rho.T @ P.polyval3d(tx[:, 0], tx[:, 1], tx[:, 2], c)
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12 * np.abs(rhs).max())


def test_interpolant_of_a_mode_converges():
    p = 38
    X = oracle.top_grid((1, 1, 1), (1, 1, 1), p)
    f = lambda a, b, c: np.cos(2 * np.pi * 4 * a + 1.0) * np.sin(2 * np.pi * 3 * b) * np.cos(2 * np.pi * 4 * c)
    vals = f(*np.meshgrid(*X, indexing="ij"))[None]
    x = np.random.default_rng(4).random((100, 3))
    got = cheb.evaluate((1, 1, 1), 3, (1, 1, 1), p, x, vals)[:, 0]
    assert np.abs(got - f(x[:, 0], x[:, 1], x[:, 2])).max() < 1e-12


def _golden(name, key):
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                if k == key:
                    return float(v)
    raise KeyError(key)


@pytest.mark.parametrize("c,p,K,tol", [(14.5, 20, 2, 1e-6), (21.5, 30, 3, 1.5e-9), (29.0, 38, 4, 1e-12)])
def test_single_level_split_madelung(c, p, K, tol):
    # root = leaf (one cube): proxy strengths, far field on the grid,
    # evaluation at the ions, residual of support 1, self term
    M = _golden("madelung_nacl.txt", "M")
    na = [(0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)]
    cl = [(.5, 0, 0), (0, .5, 0), (0, 0, .5), (.5, .5, .5)]
    x = np.array(na + cl, dtype=np.float64) + 0.125
    q = np.array([1.0] * 4 + [-1.0] * 4).reshape(-1, 1)
    W = PswfWindow(c)
    one = (1, 1, 1)
    rg = cheb.anterp(one, 3, one, p, x, q)
    ug = oracle.far_3p_grid("laplace", one, one, p, (K, K, K), 1.0, rg, window=W)
    u = cheb.evaluate(one, 3, one, p, x, ug)
    u += oracle.residual("laplace", 3, one, 1.0, 1.0, x, q, window=W)
    u -= W.phi_at(0.0) * q / (2 * np.pi)
    expect = -M / (4 * np.pi * 0.5) * q[:, 0]
    assert np.abs(u[:, 0] - expect).max() <= tol * np.abs(expect).max()


@pytest.mark.parametrize("Lv,M", [((1.0, 1.0, 1.5), (1, 1, 2)), ((1.25, 1.0, 2.6), (2, 1, 3))])
def test_single_level_split_cut_cubes(Lv, M):
    """A cell whose sides are not multiples of the shortest one: cubes of
    side h0 = min L_i cover it (Sec. 4.1.1), the last along such an axis cut
    by the cell's face.  Proxy strengths on the cubes' grids (the cubes as
    free boxes), far field on those grids with the cell's wave numbers,
    evaluation at the points, residual of support h0 on the periodic cell
    and the self term reproduce the Gaussian Ewald total."""
    rng = np.random.default_rng(31)
    c, p = 14.5, 20
    x = rng.random((24, 3)) * np.asarray(Lv)
    q = rng.normal(size=(24, 1))
    q -= q.mean()
    h0 = min(Lv)
    cover = tuple(m * h0 for m in M)
    K = tuple(int(np.floor(c * L / (2 * np.pi * h0))) for L in Lv)
    W = PswfWindow(c)
    nu = h0 * (1 - 2.0 ** -30)
    rg = cheb.anterp(cover, 0, M, p, x, q)
    ug = oracle.far_3p_grid("laplace", Lv, M, p, K, nu, rg, window=W)
    u = cheb.evaluate(cover, 0, M, p, x, ug)
    u += oracle.residual("laplace", 3, Lv, nu, nu, x, q, window=W)
    u -= W.phi_at(0.0) * q / (2 * np.pi * nu)
    ref = oracle.full_split_3p("laplace", Lv, 0.08, x, q)
    assert np.abs(u - ref).max() <= 1e-6 * np.abs(ref).max()
