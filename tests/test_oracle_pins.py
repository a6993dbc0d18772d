"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these tests retypes the oracle's formulas.  Each checks the oracle
against an independent route:

* physical constants of periodic lattices (NaCl Madelung constant; Hasimoto's
  simple-cubic Stokeslet coefficient), golden values under tests/golden/;
* sigma-independence of the full Ewald-type split (residual + Fourier part +
  self term), which ties the residual formulas of App. B to the Fourier
  symbols of the mollified kernels (eqs. (Hhat_k), (moll_stokeslet),
  (moll_stresslet), (moll_rotlet));
* the unsplit limit sigma -> infinity, where the residual kernels must reduce
  to the original kernels (App. B, eqs. (stokeslet_def_deriv)-(rotlet_def_deriv));
* the pointwise split identity K_R + K_M = K for the harmonic kernel, with
  K_M from a numerical inverse radial Fourier transform (App. A, eq.
  (radial_ft_3D)) of Hhat_M;
* differential identities between kernels (rotlet = -1/2 eps grad H,
  stresslet = stress of the Stokeslet), checked by finite differences of the
  oracle's periodic sums;
* image handling: reduction of D when no pair crosses a dropped face,
  translation invariance modulo the periods, explicit replication of images;
* central finite differences of the oracle's own energy for its gradients.
"""
import os

import numpy as np
import pytest
from scipy import integrate

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


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


# --------------------------------------------------------------------------
# lattice constants
@pytest.mark.parametrize("sigma", [0.07, 0.15, 0.3])
def test_madelung_nacl(sigma):
    M = _golden("madelung_nacl.txt", "M")
    x, q = _nacl()
    u = oracle.full_split_3p("laplace", (1, 1, 1), sigma, x, q)[:, 0]
    a = 0.5  # nearest-neighbour distance
    expect = -M / (4 * np.pi * a) * q[:, 0]
    np.testing.assert_allclose(u, expect, rtol=1e-12, atol=0)


@pytest.mark.parametrize("sigma", [0.08, 0.2])
def test_hasimoto_simple_cubic(sigma):
    zeta = _golden("hasimoto_simple_cubic.txt", "zeta")
    x = np.array([[0.31, 0.42, 0.53]])
    f = np.array([[0.3, -0.5, 0.8]])
    u = oracle.full_split_3p("stokeslet", (1, 1, 1), sigma, x, f)[0]
    np.testing.assert_allclose(u, -zeta * f[0] / (6 * np.pi), rtol=2e-7)


# --------------------------------------------------------------------------
# sigma independence of the full split (D = 3)
def _random_points(seed, n, L):
    rng = np.random.default_rng(seed)
    return rng.random((n, 3)) * np.asarray(L)


@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "rotlet", "stresslet"])
def test_full_split_sigma_independent(kernel):
    L = (1.0, 1.3, 0.9)
    x = _random_points(5, 14, L)
    rng = np.random.default_rng(6)
    m_in = oracle.M_IN[oracle.KERNELS[kernel]]
    rho = rng.normal(size=(14, m_in))
    if kernel == "laplace":
        rho -= rho.mean()  # neutrality: the k = 0 term is omitted (Sec. 1, footnote)
    us = [oracle.full_split_3p(kernel, L, s, x, rho) for s in (0.06, 0.1, 0.16)]
    scale = np.abs(us[0]).max()
    for u in us[1:]:
        assert np.abs(u - us[0]).max() < 1e-11 * scale


# --------------------------------------------------------------------------
# sigma -> infinity: the residual kernels are the original kernels
@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "stresslet", "rotlet"])
def test_residual_unsplit_limit(kernel):
    x = _random_points(11, 40, (1, 1, 1))
    rng = np.random.default_rng(12)
    rho = rng.normal(size=(40, oracle.M_IN[oracle.KERNELS[kernel]]))
    rc = 0.45
    u_r = oracle.residual(kernel, 0, (1, 1, 1), 1e12, rc, x, rho)
    u_d = oracle.direct_free(kernel, x, rho, rc=rc)
    np.testing.assert_allclose(u_r, u_d, rtol=1e-10, atol=1e-10 * np.abs(u_d).max())


def test_free_kernels_textbook_values():
    # original kernels at d = (1, 2, 2), r = 3, against values worked by hand
    d = np.array([1.0, 2.0, 2.0])
    r = 3.0
    H = oracle.kernel_free_tensor("laplace", d)[0, 0]
    assert abs(H - 1 / (12 * np.pi)) < 1e-16
    S = oracle.kernel_free_tensor("stokeslet", d)
    assert abs(S[0, 0] - (1 / 3 + 1 / 27) / (8 * np.pi)) < 1e-16
    assert abs(S[1, 2] - (4 / 27) / (8 * np.pi)) < 1e-16
    T = oracle.kernel_free_tensor("stresslet", d)
    assert abs(T[1, 2 * 3 + 0] - (-3 / (4 * np.pi)) * 4 / r ** 5) < 1e-16
    O = oracle.kernel_free_tensor("rotlet", d)
    # Omega_jl = eps_jlm d_m / (8 pi r^3): Omega_01 = d_2 / (8 pi 27)
    assert abs(O[0, 1] - 2 / (8 * np.pi * 27)) < 1e-16
    assert abs(O[1, 0] + 2 / (8 * np.pi * 27)) < 1e-16


# --------------------------------------------------------------------------
# pointwise split identity for the harmonic kernel from the Fourier symbol
@pytest.mark.parametrize("r", [0.013, 0.05, 0.11])
def test_harmonic_split_identity_radial_ft(r):
    sigma = 0.04
    # H_M(r) = 1/(2 pi^2) int_0^inf sin(kr)/(kr) exp(-k^2 sigma^2/4) dk  (k^2/k^2 cancelled)
    f = lambda k: np.sinc(k * r / np.pi) * np.exp(-k * k * sigma * sigma / 4)
    HM, err = integrate.quad(f, 0, 40 / sigma, limit=400, epsabs=1e-14, epsrel=1e-13)
    HM /= 2 * np.pi ** 2
    KR = oracle.kernel_tensor("laplace", [r, 0, 0], sigma)[0][0, 0]
    np.testing.assert_allclose(KR + HM, 1 / (4 * np.pi * r), rtol=1e-11)


def test_stokeslet_split_identity_radial_ft():
    # S_M = (-delta lap + grad grad) B_M with Bhat_M = gammaB(k sigma)/k^4.
    # For a radial f: (S_M)_jl = delta_jl (-f'' - f'/r) + xhat_j xhat_l (f'' - f'/r).
    # f'(r) and f''(r) are convergent radial integrals of Bhat_M.
    sigma = 0.05
    gB = lambda k: np.exp(-(k * sigma) ** 2 / 4) * (1 + (k * sigma) ** 2 / 4)
    for r in (0.02, 0.07, 0.15):
        def d1(k):  # d/dr sin(kr)/(kr) * k^2 * Bhat = (kr cos kr - sin kr)/(k r^2) * gB/k^2
            kr = k * r
            if kr < 1e-3:
                return (-kr ** 3 / 3 + kr ** 5 / 30) / (k * r * r) * gB(k) / k ** 2
            return (kr * np.cos(kr) - np.sin(kr)) / (k * r * r) * gB(k) / k ** 2

        def d2(k):  # second radial derivative of sin(kr)/(kr), times k^2 Bhat
            kr = k * r
            if kr < 1e-3:
                val = (-1.0 / 3 + kr * kr / 10) * k * k
            else:
                val = ((2 - kr * kr) * np.sin(kr) - 2 * kr * np.cos(kr)) / (kr ** 3) * k * k
            return val * gB(k) / k ** 2
        kmax = 40 / sigma
        f1 = integrate.quad(d1, 0, kmax, limit=800, epsabs=1e-13, epsrel=1e-12)[0] / (2 * np.pi ** 2)
        f2 = integrate.quad(d2, 0, kmax, limit=800, epsabs=1e-13, epsrel=1e-12)[0] / (2 * np.pi ** 2)
        SM_diag = -f2 - f1 / r
        SM_off = f2 - f1 / r
        d = np.array([r, 0, 0])
        K = oracle.kernel_tensor("stokeslet", d, sigma)[0]
        S = oracle.kernel_free_tensor("stokeslet", d)
        # along x: xhat = e_x, so (0,0) = diag + off, (1,1) = diag
        np.testing.assert_allclose(K[1, 1] + SM_diag, S[1, 1], rtol=1e-9)
        np.testing.assert_allclose(K[0, 0] + SM_diag + SM_off, S[0, 0], rtol=1e-9)


# --------------------------------------------------------------------------
# differential identities between the periodic sums (D = 3, full split)
def _fd_grad_target(fn, xt, h=1e-4):
    """4th-order central difference of fn(target position) -> array."""
    g = []
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        g.append((-fn(xt + 2 * e) + 8 * fn(xt + e) - 8 * fn(xt - e) + fn(xt - 2 * e)) / (12 * h))
    return np.array(g)  # [k, ...]


def test_rotlet_is_half_curl_of_harmonic():
    L = (1.0, 1.0, 1.0)
    sigma = 0.12
    xa = np.array([0.2, 0.35, 0.6])
    xt = np.array([0.55, 0.5, 0.45])
    rho = np.array([0.4, -1.1, 0.7])

    def H(pt):  # periodic harmonic kernel of a unit charge at xa, evaluated at pt
        x = np.stack([xa, pt])
        q = np.array([[1.0], [0.0]])
        return oracle.full_split_3p("laplace", L, sigma, x, q, targets=[1])[0, 0]
    gH = _fd_grad_target(H, xt)  # [m]
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1
    expect = -0.5 * np.einsum("jlm,l,m->j", eps, rho, gH)
    x = np.stack([xa, xt])
    r = np.stack([rho, np.zeros(3)])
    u = oracle.full_split_3p("rotlet", L, sigma, x, r, targets=[1])[0]
    np.testing.assert_allclose(u, expect, rtol=1e-7, atol=1e-9 * np.abs(expect).max())


def test_stresslet_is_stokeslet_stress():
    # T_jlm = -delta_jm P_l + d_m S_jl + d_j S_ml with pressure P_l = -d_l H,
    # applied to the periodic sums with the k = 0 mode removed on both sides.
    L = (1.0, 1.0, 1.0)
    sigma = 0.12
    xa = np.array([0.25, 0.3, 0.7])
    xt = np.array([0.5, 0.55, 0.4])
    x = np.stack([xa, xt])
    T = np.zeros((3, 3, 3))
    for l in range(3):
        for m in range(3):
            rho = np.zeros((2, 9))
            rho[0, 3 * l + m] = 1.0
            T[:, l, m] = oracle.full_split_3p("stresslet", L, sigma, x, rho, targets=[1])[0]

    def S_col(l):
        def f(pt):
            xx = np.stack([xa, pt])
            f_ = np.zeros((2, 3))
            f_[0, l] = 1.0
            return oracle.full_split_3p("stokeslet", L, sigma, xx, f_, targets=[1])[0]
        return f
    dS = np.zeros((3, 3, 3))  # dS[m, j, l] = d_m S_jl
    for l in range(3):
        dS[:, :, l] = _fd_grad_target(S_col(l), xt)

    def H(pt):
        xx = np.stack([xa, pt])
        return oracle.full_split_3p("laplace", L, sigma, xx, np.array([[1.0], [0.0]]), targets=[1])[0, 0]
    P = -_fd_grad_target(H, xt)
    expect = np.zeros((3, 3, 3))
    for j in range(3):
        for l in range(3):
            for m in range(3):
                expect[j, l, m] = -(j == m) * P[l] + dS[m, j, l] + dS[j, m, l]
    np.testing.assert_allclose(T, expect, rtol=1e-6, atol=1e-7 * np.abs(expect).max())


# --------------------------------------------------------------------------
# image handling
@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "stresslet", "rotlet"])
def test_dimension_reduction(kernel):
    # points kept at least rc away from the faces normal to axes >= D' so no
    # image in those axes can be within the cutoff: D=3 == D=2 == D=1 == D=0.
    L = (1.0, 1.0, 1.0)
    rc = 0.2
    rng = np.random.default_rng(21)
    x = rc + rng.random((60, 3)) * (1 - 2 * rc)
    rho = rng.normal(size=(60, oracle.M_IN[oracle.KERNELS[kernel]]))
    sigma = rc / 4
    ref = oracle.residual(kernel, 0, L, sigma, rc, x, rho)
    for D in (1, 2, 3):
        np.testing.assert_array_equal(oracle.residual(kernel, D, L, sigma, rc, x, rho), ref)
    # and the cut sum equals the D=0 brute force over explicit replicas only
    # when nothing crosses a face; move points to the faces and D matters:
    x2 = x.copy()
    x2[:5, 0] = rng.random(5) * 0.05
    x2[5:10, 0] = 1 - rng.random(5) * 0.05
    assert not np.allclose(oracle.residual(kernel, 1, L, sigma, rc, x2, rho),
                           oracle.residual(kernel, 0, L, sigma, rc, x2, rho))


@pytest.mark.parametrize("kernel,D", [("laplace", 3), ("stokeslet", 2), ("stresslet", 1), ("rotlet", 1),
                                      ("rotlet", 3)])
def test_explicit_image_replication(kernel, D):
    # mode R with periodic axes == D=0 residual sum over explicit replicas
    L = (0.6, 0.5, 0.7)
    rc = 0.3
    rng = np.random.default_rng(31)
    N = 25
    x = rng.random((N, 3)) * np.asarray(L)
    rho = rng.normal(size=(N, oracle.M_IN[oracle.KERNELS[kernel]]))
    sigma = 0.07
    xs, rs = [x], [rho]
    rngs = [range(-2, 3) if i < D else range(0, 1) for i in range(3)]
    for a in rngs[0]:
        for b in rngs[1]:
            for c in rngs[2]:
                if a == b == c == 0:
                    continue
                xs.append(x + np.array([a * L[0], b * L[1], c * L[2]]))
                rs.append(rho)
    X = np.concatenate(xs)
    R = np.concatenate(rs)
    ref = oracle.residual(kernel, 0, L, sigma, rc, X, R, targets=np.arange(N))
    got = oracle.residual(kernel, D, L, sigma, rc, x, rho)
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("kernel,D", [("laplace", 3), ("stokeslet", 2), ("stresslet", 1), ("rotlet", 3)])
def test_translation_invariance(kernel, D):
    L = (1.0, 0.8, 1.2)
    rc = 0.25
    rng = np.random.default_rng(41)
    N = 80
    x = rng.random((N, 3)) * np.asarray(L)
    if D < 3:  # keep free axes away from the faces so the shift cannot move pairs out
        for ax in range(D, 3):
            x[:, ax] = 0.3 * L[ax] + 0.4 * L[ax] * rng.random(N)
    rho = rng.normal(size=(N, oracle.M_IN[oracle.KERNELS[kernel]]))
    sigma = rc / 5
    u0 = oracle.residual(kernel, D, L, sigma, rc, x, rho)
    shift = np.array([0.37, 0.61, 0.23])[:3] * np.asarray(L)
    shift[D:] = 0.0
    x1 = x + shift
    for ax in range(D):
        x1[:, ax] = np.mod(x1[:, ax], L[ax])
    u1 = oracle.residual(kernel, D, L, sigma, rc, x1, rho)
    np.testing.assert_allclose(u1, u0, rtol=1e-12, atol=1e-12 * np.abs(u0).max())


@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "rotlet"])
def test_reciprocity(kernel):
    # sum rho' . u[rho] = sum rho . u[rho'] (the Laplace kernel and Stokeslet
    # are even and symmetric; the rotlet is odd and antisymmetric)
    L = (1.0, 1.0, 1.0)
    rng = np.random.default_rng(51)
    x = rng.random((70, 3))
    m = oracle.M_IN[oracle.KERNELS[kernel]]
    r1 = rng.normal(size=(70, m))
    r2 = rng.normal(size=(70, m))
    a = np.sum(r2 * oracle.residual(kernel, 3, L, 0.05, 0.24, x, r1))
    b = np.sum(r1 * oracle.residual(kernel, 3, L, 0.05, 0.24, x, r2))
    assert abs(a - b) < 1e-12 * (abs(a) + abs(b))


@pytest.mark.parametrize("kernel", ["stokeslet", "stresslet", "rotlet"])
def test_rotation_covariance_free_space(kernel):
    # 90-degree rotation about z: R x; vectors u -> R u; stresslet rho -> R rho R^T
    R = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    rng = np.random.default_rng(61)
    x = rng.random((50, 3))
    m = oracle.M_IN[oracle.KERNELS[kernel]]
    rho = rng.normal(size=(50, m))
    if kernel == "stresslet":
        rho_r = np.einsum("ij,njk,lk->nil", R, rho.reshape(50, 3, 3), R).reshape(50, 9)
    else:
        rho_r = rho @ R.T
    u = oracle.residual(kernel, 0, (1, 1, 1), 0.08, 0.4, x, rho)
    ur = oracle.residual(kernel, 0, (1, 1, 1), 0.08, 0.4, x @ R.T, rho_r)
    np.testing.assert_allclose(ur, u @ R.T, rtol=1e-12, atol=1e-12 * np.abs(u).max())


def test_coincident_points_excluded():
    x = np.array([[0.5, 0.5, 0.5], [0.5, 0.5, 0.5], [0.55, 0.5, 0.5]])
    q = np.array([[1.0], [2.0], [4.0]])
    u = oracle.residual("laplace", 3, (1, 1, 1), 0.02, 0.1, x, q)
    # the duplicate pair (r = 0) is dropped; only the 0.05-distant point counts
    KR = oracle.kernel_tensor("laplace", [0.05, 0, 0], 0.02)[0][0, 0]
    np.testing.assert_allclose(u[:2, 0], [4 * KR, 4 * KR], rtol=1e-13)


# --------------------------------------------------------------------------
# kernel derivative and gradient pins
@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "stresslet", "rotlet"])
def test_kernel_derivative_fd(kernel):
    sigma = 0.3
    for d in ([0.2, -0.35, 0.5], [0.05, 0.1, -0.02], [0.9, 0.1, 0.3]):
        d = np.asarray(d)
        _, dK = oracle.kernel_tensor(kernel, d, sigma)
        h = 1e-5
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            fd = (-oracle.kernel_tensor(kernel, d + 2 * e, sigma)[0] + 8 * oracle.kernel_tensor(kernel, d + e, sigma)[0]
                  - 8 * oracle.kernel_tensor(kernel, d - e, sigma)[0] + oracle.kernel_tensor(kernel, d - 2 * e, sigma)[0]) / (12 * h)
            np.testing.assert_allclose(dK[k], fd, rtol=1e-7, atol=1e-8 * np.abs(fd).max())


@pytest.mark.parametrize("kernel,D", [("laplace", 3), ("stokeslet", 2), ("stresslet", 1), ("rotlet", 3),
                                      ("stokeslet", 0)])
def test_vjp_against_finite_differences(kernel, D):
    L = (1.0, 1.0, 1.0)
    rng = np.random.default_rng(71)
    N = 40
    x = rng.random((N, 3))
    k = oracle.KERNELS[kernel]
    rho = rng.normal(size=(N, oracle.M_IN[k]))
    G = rng.normal(size=(N, oracle.M_OUT[k]))
    sigma, rc = 0.06, 0.3
    gr, gx = oracle.residual_vjp(kernel, D, L, sigma, rc, x, rho, G)

    def F(xx, rr):
        return np.sum(G * oracle.residual(kernel, D, L, sigma, rc, xx, rr))
    h = 1e-6
    for c in (0, 7, 23):
        for ax in range(3):
            xp = x.copy()
            xm = x.copy()
            xp[c, ax] += h
            xm[c, ax] -= h
            fd = (F(xp, rho) - F(xm, rho)) / (2 * h)
            assert abs(fd - gx[c, ax]) < 2e-6 * (abs(fd) + 1e-3 * np.abs(gx).max())
        for q in range(oracle.M_IN[k]):
            rp = rho.copy()
            rp[c, q] += 1.0
            fdr = F(x, rp) - F(x, rho)  # F is linear in rho
            assert abs(fdr - gr[c, q]) < 1e-10 * (abs(fdr) + np.abs(gr).max())


def test_vjp_translation_invariance():
    # sum over all points of dF/dx_c vanishes for a periodic sum
    rng = np.random.default_rng(81)
    x = rng.random((60, 3))
    rho = rng.normal(size=(60, 3))
    G = rng.normal(size=(60, 3))
    _, gx = oracle.residual_vjp("stokeslet", 3, (1, 1, 1), 0.05, 0.25, x, rho, G)
    assert np.abs(gx.sum(axis=0)).max() < 1e-10 * np.abs(gx).max()
