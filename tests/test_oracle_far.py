"""Pins of the oracle's root-level far field (D = 3): eq. (ewald_far_3P) over
the cube of wave numbers of eqs. (wavenumbers-3p-trunc), (kintmax), with the
structure factor of eq. (structurefacgen).

Independent routes:

* with the root-level split (sigma_0 = the cell side, PSWF bandwidth c from
  the parameter tables and their mode counts N_per = 2K + 1), far field +
  residual over all images + self term reproduces the NaCl Madelung constant
  and Hasimoto's constant to the tolerance the tables give for c;
* the far field is unchanged when a source is moved by a lattice vector;
* the grid helper places first-kind Chebyshev points (roots of T_p) in each
  top cube.
"""
import os

import numpy as np
import pytest
from numpy.polynomial import chebyshev as npcheb

import oracle
from oracle.pswf import PswfWindow

GOLD = os.path.join(os.path.dirname(__file__), "golden")
_WIN = {}


def _w(c):
    if c not in _WIN:
        _WIN[c] = PswfWindow(c)
    return _WIN[c]


def _golden(name, key):
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            if k == key:
                return float(v)
    raise KeyError(key)


def _nacl():
    na = [(0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)]
    cl = [(.5, 0, 0), (0, .5, 0), (0, 0, .5), (.5, .5, .5)]
    x = np.array(na + cl, dtype=np.float64) + 0.125
    q = np.array([1.0] * 4 + [-1.0] * 4).reshape(-1, 1)
    return x, q


def _root_split(kernel, x, rho, c, K):
    """sigma_0 = 1 (unit cell, one top cube): residual of support 1 over all
    images, far field with |n_i| <= K, self term -phi(0) rho / (2 pi sigma_0)
    for the harmonic kernel and the Stokeslet (none for stresslet and rotlet,
    Sec. 2.4)."""
    W = _w(c)
    ur = oracle.residual(kernel, 3, (1, 1, 1), 1.0, 1.0, x, rho, window=W)
    uf = oracle.far_3p(kernel, (1, 1, 1), 1.0, (K, K, K), x, rho, x, window=W)
    u = ur + uf
    if kernel in ("laplace", "stokeslet"):
        u = u - W.phi_at(0.0) * rho / (2 * np.pi)
    return u


# (c, K, tolerance): Laplace table rows 1e-6, 1e-9, 1e-12 (N_per = 5, 7, 9),
# and the larger count of eq. (kintmax) at 1e-12
@pytest.mark.parametrize("c,K,tol", [(14.5, 2, 1e-6), (21.5, 3, 1.5e-9), (29.0, 4, 1e-12), (29.0, 5, 1e-12)])
def test_root_split_madelung(c, K, tol):
    M = _golden("madelung_nacl.txt", "M")
    x, q = _nacl()
    u = _root_split("laplace", x, q, c, K)[:, 0]
    expect = -M / (4 * np.pi * 0.5) * q[:, 0]
    assert np.abs(u - expect).max() <= tol * np.abs(expect).max()


def test_root_split_hasimoto():
    # Stokeslet table row 1e-12: c = 32.46, N_per = 11
    zeta = _golden("hasimoto_simple_cubic.txt", "zeta")
    x = np.array([[0.31, 0.42, 0.53]])
    f = np.array([[0.3, -0.5, 0.8]])
    u = _root_split("stokeslet", x, f, 32.46, 5)[0]
    # zeta is known to 7 digits
    np.testing.assert_allclose(u, -zeta * f[0] / (6 * np.pi), rtol=3e-7, atol=0)


@pytest.mark.parametrize("kernel,c,K", [("stokeslet", 32.46, 5), ("rotlet", 32.46, 5), ("stresslet", 33.51, 5),
                                        ("laplace", 29.0, 4)])
def test_root_split_equals_gaussian_ewald_split(kernel, c, K):
    # another window (Gaussian, sigma = 0.08), ball truncation, generous
    # real-space cutoff: the full periodic sum does not depend on the split
    rng = np.random.default_rng(21)
    x = rng.random((10, 3))
    k = oracle.KERNELS[kernel]
    rho = rng.normal(size=(10, oracle.M_IN[k]))
    if kernel == "laplace":
        rho -= rho.mean()
    a = _root_split(kernel, x, rho, c, K)
    b = oracle.full_split_3p(kernel, (1, 1, 1), 0.08, x, rho)
    np.testing.assert_allclose(a, b, rtol=0, atol=2e-12 * np.abs(b).max())


@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "stresslet", "rotlet"])
def test_far_field_lattice_shift_invariant(kernel):
    rng = np.random.default_rng(4)
    L = (1.0, 2.0, 1.0)
    xs = rng.random((7, 3)) * L
    xt = rng.random((5, 3)) * L
    k = oracle.KERNELS[kernel]
    rho = rng.normal(size=(7, oracle.M_IN[k]))
    W = _w(14.5)
    a = oracle.far_3p(kernel, L, 1.0, (2, 4, 2), xs, rho, xt, window=W)
    shift = np.array([[1.0, -4.0, 3.0]]) * np.asarray(L)
    b = oracle.far_3p(kernel, L, 1.0, (2, 4, 2), xs + shift, rho, xt - 2 * shift, window=W)
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-12 * np.abs(a).max())


@pytest.mark.parametrize("p", [5, 12, 38])
def test_top_grid_first_kind_chebyshev(p):
    eta = oracle.cheb_points(p)
    Tp = np.zeros(p + 1)
    Tp[-1] = 1.0
    assert np.abs(npcheb.chebval(eta, Tp)).max() < 1e-13
    assert np.all(np.diff(eta) < 0) and eta[0] < 1 and eta[-1] > -1
    X = oracle.top_grid((2.0, 1.0, 3.0), (2, 1, 3), p)
    for i, Mi in enumerate((2, 1, 3)):
        g = X[i].reshape(Mi, p)
        for b in range(Mi):
            assert np.all((g[b] > b) & (g[b] < b + 1))
    with pytest.raises(ValueError):
        oracle.top_grid((2.0, 1.0, 3.0), (1, 1, 3), p)
