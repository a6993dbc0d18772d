"""Leaf-box Chebyshev grids on the GPU (dmk_cheb_anterp, dmk_cheb_eval,
dmk_self_term) against the oracle, and the single-level periodic split built
from them with dmk_far3p_eval and the residual: against the oracle's
composition (FP64 bar 1e-12) and against the Madelung and Hasimoto
constants."""
import os

import numpy as np
import pytest

import oracle
from oracle import cheb as OC
from oracle.pswf import PswfWindow
from gpu_util import HAVE_GPU, assert_parity, dev, host, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    import torch
    from paper_2606_27134_amd import far as F
    from paper_2606_27134_amd import residual as R

_WIN = {}


def _w(c):
    if c not in _WIN:
        _WIN[c] = PswfWindow(c)
    return _WIN[c]


# (L, D, n, p, N)
CASES = [
    ((1.0, 1.0, 1.0), 3, (2, 2, 2), 6, 300),
    ((2.0, 1.0, 1.5), 1, (4, 2, 3), 5, 400),
    ((1.0, 1.0, 1.0), 3, (1, 1, 1), 12, 200),
    ((1.0, 1.0, 1.0), 0, (3, 3, 3), 4, 5),     # most boxes empty
    ((1.0, 1.0, 1.0), 3, (2, 1, 1), 20, 1229),  # ~600 points a box: several block groups per wavefront, ragged tail
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("m", [1, 3, 9])
def test_anterp_and_eval(case, m):
    Lv, D, n, p, N = CASES[case]
    print("cheb", case, m, flush=True)
    rng = np.random.default_rng(40 + case)
    x = rng.random((N, 3)) * np.asarray(Lv)
    rho = rng.normal(size=(N, m))
    b = R.tree_bin(Lv, D, n, dev(x))
    rg = host(F.cheb_anterp(b, p, dev(rho)))
    assert_parity(rg, OC.anterp(Lv, D, n, p, x, rho), 1e-12, "anterp")
    ug = rng.normal(size=(m, n[0] * p, n[1] * p, n[2] * p))
    got = host(F.cheb_eval(b, p, dev(ug)))
    assert_parity(got, OC.evaluate(Lv, D, n, p, x, ug), 1e-12, "eval")
    base = rng.normal(size=(N, m))
    acc = dev(base)
    F.cheb_eval(b, p, dev(ug), out=acc, accumulate=True)
    assert_parity(host(acc) - base, OC.evaluate(Lv, D, n, p, x, ug), 1e-12, "eval accumulate")


def test_degenerate_grids():
    rng = np.random.default_rng(8)
    # p = 1: one node per box, the box's total strength / a constant per box
    Lv, n = (1.0, 1.0, 1.0), (2, 3, 1)
    x = rng.random((50, 3))
    rho = rng.normal(size=(50, 3))
    b = R.tree_bin(Lv, 3, n, dev(x))
    assert_parity(host(F.cheb_anterp(b, 1, dev(rho))), OC.anterp(Lv, 3, n, 1, x, rho), 1e-12, "anterp p=1")
    ug = rng.normal(size=(3, 2, 3, 1))
    assert_parity(host(F.cheb_eval(b, 1, dev(ug))), OC.evaluate(Lv, 3, n, 1, x, ug), 1e-12, "eval p=1")
    # no points: the grids are all zero, evaluation leaves its output alone
    b0 = R.tree_bin(Lv, 3, n, dev(np.zeros((0, 3))))
    rg = F.cheb_anterp(b0, 4, dev(np.zeros((0, 1))), out=dev(np.full((1, 8, 12, 4), 7.0)))
    assert np.all(host(rg) == 0.0)
    assert host(F.cheb_eval(b0, 4, dev(np.ones((1, 8, 12, 4))))).shape == (0, 1)


def test_eval_at_grid_nodes():
    # points on (or within rounding of) grid nodes: the barycentric form near its poles
    p, Lv, n = 7, (1.0, 1.0, 1.0), (2, 1, 1)
    X = oracle.top_grid((2.0, 1.0, 1.0), (2, 1, 1), p)
    X[0] = X[0] / 2.0
    g = np.stack(np.meshgrid(X[0][[1, 9]], X[1][[0, 3]], X[2][[6]], indexing="ij"), axis=-1).reshape(-1, 3)
    ug = np.random.default_rng(5).normal(size=(1, 2 * p, p, p))
    b = R.tree_bin(Lv, 3, n, dev(g))
    got = host(F.cheb_eval(b, p, dev(ug)))[:, 0]
    np.testing.assert_allclose(got, OC.evaluate(Lv, 3, n, p, g, ug)[:, 0], rtol=0, atol=1e-14)


@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("c", [None, 29.0])
def test_self_term(kernel, c):
    k = oracle.KERNELS[kernel]
    rng = np.random.default_rng(6)
    rho = rng.normal(size=(50, oracle.M_IN[k]))
    u0 = rng.normal(size=(50, oracle.M_OUT[k]))
    u = dev(u0)
    F.self_term(kernel, 0.7, dev(rho), u, pswf_c=c)
    phi0 = (1 / np.sqrt(np.pi)) if c is None else _w(c).phi_at(0.0)
    expect = u0 - (phi0 * rho / (2 * np.pi * 0.7) if kernel in ("laplace", "stokeslet") else 0.0)
    # phi(0) of the PSWF window comes from its Chebyshev fit (~4e-15 relative)
    np.testing.assert_allclose(host(u), expect, rtol=0, atol=1e-13 * np.abs(expect).max())


def _oracle_single_level(kernel, Lv, x, rho, c, p, K):
    # the same support as the library's single-level split: a hair inside the
    # cube side, so that the points' own images (at exactly h0) lie outside.
    # Cubes of side h0 = min L_i; where they do not tile the cell they cover
    # it (M_i = ceil(L_i / h0)) and are free boxes for the proxy grids.
    h0 = min(Lv)
    nu = h0 * (1.0 - 2.0 ** -30)
    M = tuple(int(np.ceil(v / h0 * (1 - 1e-12))) for v in Lv)
    if all(abs(v / m - h0) <= 1e-12 * h0 for v, m in zip(Lv, M)):
        box, D = Lv, 3
    else:
        box, D = tuple(m * h0 for m in M), 0
    W = _w(c)
    rg = OC.anterp(box, D, M, p, x, rho)
    ug = oracle.far_3p_grid(kernel, Lv, M, p, K, nu, rg, window=W)
    u = OC.evaluate(box, D, M, p, x, ug)
    u += oracle.residual(kernel, 3, Lv, nu, nu, x, rho, window=W)
    if kernel in ("laplace", "stokeslet"):
        u -= W.phi_at(0.0) * rho / (2 * np.pi * nu)
    return u


@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("geom", [((1.0, 1.0, 1.0), 14.5, 20), ((3.0, 1.0, 1.0), 17.80, 23)])
def test_single_level_split_matches_oracle(kernel, geom):
    Lv, c, p = geom
    print("single level", kernel, Lv, flush=True)
    k = oracle.KERNELS[kernel]
    rng = np.random.default_rng(90 + k)
    N = 40
    x = rng.random((N, 3)) * np.asarray(Lv)
    rho = rng.normal(size=(N, oracle.M_IN[k]))
    K = F.table_modes(c, Lv, min(Lv))
    got = host(F.single_level_3p(dev(x), dev(rho), kernel, Lv, c, p))
    ref = _oracle_single_level(kernel, Lv, x, rho, c, p, K)
    assert_parity(got, ref, 1e-12, "single level %s" % kernel)


@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "stresslet", "rotlet"])
@pytest.mark.parametrize("Lv", [(1.0, 1.0, 1.5), (1.25, 1.0, 2.6)])
def test_single_level_split_cut_cubes(kernel, Lv):
    """Cells whose sides are not multiples of the shortest one (Sec. 4.1.1):
    the library against the oracle's composition of the same steps."""
    c, p = 14.5, 20
    print("single level cut cubes", kernel, Lv, flush=True)
    k = oracle.KERNELS[kernel]
    rng = np.random.default_rng(95 + k)
    N = 40
    x = rng.random((N, 3)) * np.asarray(Lv)
    rho = rng.normal(size=(N, oracle.M_IN[k]))
    K = F.table_modes(c, Lv, min(Lv))
    got = host(F.single_level_3p(dev(x), dev(rho), kernel, Lv, c, p))
    ref = _oracle_single_level(kernel, Lv, x, rho, c, p, K)
    assert_parity(got, ref, 1e-12, "single level cut %s" % kernel)


@pytest.mark.parametrize("Lv", [(1.0, 1.0, 1.5), (1.25, 1.0, 2.6)])
def test_single_level_cut_cubes_ewald(Lv):
    """At the Laplace table row 1e-12 (c = 29, p = 38) the split on a cut
    cover reproduces the Gaussian Ewald sum of neutral charges to 1e-12."""
    rng = np.random.default_rng(31)
    N = 24
    x = rng.random((N, 3)) * np.asarray(Lv)
    q = rng.normal(size=(N, 1))
    q -= q.mean()
    print("single level cut cubes ewald", Lv, flush=True)
    u = host(F.single_level_3p(dev(x), dev(q), "laplace", Lv, 29.0, 38))
    ref = oracle.full_split_3p("laplace", Lv, 0.08, x, q)
    assert np.abs(u - ref).max() <= 1e-12 * np.abs(ref).max()


def _golden(name, key):
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                kk, v = line.split()
                if kk == key:
                    return float(v)
    raise KeyError(key)


def test_single_level_split_madelung_on_gpu():
    # Laplace table row 1e-12: c = 29, p = 38, N_per = 9
    M = _golden("madelung_nacl.txt", "M")
    na = [(0, 0, 0), (0, .5, .5), (.5, 0, .5), (.5, .5, 0)]
    cl = [(.5, 0, 0), (0, .5, 0), (0, 0, .5), (.5, .5, .5)]
    x = np.array(na + cl, dtype=np.float64) + 0.125
    q = np.array([1.0] * 4 + [-1.0] * 4).reshape(-1, 1)
    u = host(F.single_level_3p(dev(x), dev(q), "laplace", (1.0, 1.0, 1.0), 29.0, 38))[:, 0]
    expect = -M / (4 * np.pi * 0.5) * q[:, 0]
    assert np.abs(u - expect).max() <= 1e-12 * np.abs(expect).max()


def test_single_level_split_hasimoto_on_gpu():
    # Stokeslet table row 1e-12: c = 32.46, p = 44, N_per = 11; zeta has 7 digits
    zeta = _golden("hasimoto_simple_cubic.txt", "zeta")
    x = np.array([[0.31, 0.42, 0.53]])
    f = np.array([[0.3, -0.5, 0.8]])
    u = host(F.single_level_3p(dev(x), dev(f), "stokeslet", (1.0, 1.0, 1.0), 32.46, 44))[0]
    np.testing.assert_allclose(u, -zeta * f[0] / (6 * np.pi), rtol=3e-7, atol=0)


@pytest.mark.parametrize("n,N", [((1, 1, 1), 40), ((2, 2, 2), 40)])
def test_largest_order(n, N):
    # p = 64 (the largest order the library takes), 9 components: LDS chunks
    # of a few points, 16 A fragments per matrix-core block; 40 points in one
    # box (matrix-core forms) or over 8 boxes (thread forms)
    p, m = 64, 9
    rng = np.random.default_rng(11)
    Lv = (1.0, 1.0, 1.0)
    x = rng.random((N, 3))
    rho = rng.normal(size=(N, m))
    b = R.tree_bin(Lv, 3, n, dev(x))
    print("largest order", n, N, flush=True)
    assert_parity(host(F.cheb_anterp(b, p, dev(rho))), OC.anterp(Lv, 3, n, p, x, rho), 1e-12, "anterp p=64")
    ug = rng.normal(size=(m, n[0] * p, n[1] * p, n[2] * p))
    assert_parity(host(F.cheb_eval(b, p, dev(ug))), OC.evaluate(Lv, 3, n, p, x, ug), 1e-12, "eval p=64")


@pytest.mark.parametrize("m", [1, 3])
def test_cheb_deterministic(m):
    """Repeated anterpolation and evaluation (matrix-core paths, boxes of many
    points) give bit-identical results."""
    import torch
    rng = np.random.default_rng(83)
    x = rng.random((60000, 3))
    b = R.tree_bin((1.0, 1.0, 1.0), 3, (6, 6, 6), dev(x))
    q = dev(rng.normal(size=(60000, m)))
    r1 = F.cheb_anterp(b, 20, q)
    r2 = F.cheb_anterp(b, 20, q)
    u1 = F.cheb_eval(b, 20, r1)
    u2 = F.cheb_eval(b, 20, r1)
    torch.cuda.synchronize()
    assert torch.equal(r1, r2) and torch.equal(u1, u2)
