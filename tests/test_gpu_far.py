"""dmk_far3p_eval (root-level far field, D = 3) against the oracle's direct
sums of eqs. (structurefacgen) and (ewald_far_3P) with the top-level
Chebyshev grid points as sources and targets.  FP64 bar: relative l2 <= 1e-12
(and every element within 1e-12 of the largest)."""
import numpy as np
import pytest

import oracle
from oracle.pswf import PswfWindow
from gpu_util import HAVE_GPU, assert_parity, dev, host, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    from paper_2606_27134_amd import far as F

KERNELS = ["laplace", "stokeslet", "stresslet", "rotlet"]
_WIN = {}


def _w(c):
    if c is None:
        return None
    if c not in _WIN:
        _WIN[c] = PswfWindow(c)
    return _WIN[c]


# (L, M, p, K, sigma0 for the Gaussian): small grids over one or several cubes
GEOMS = [
    ((1.0, 1.0, 1.0), (1, 1, 1), 6, (2, 2, 2), 0.3),
    ((2.0, 1.0, 3.0), (2, 1, 3), 5, (3, 1, 4), 0.4),
    ((1.0, 1.0, 1.0), (1, 1, 1), 12, (1, 1, 1), 0.5),
    ((8.0, 1.0, 1.0), (8, 1, 1), 6, (20, 2, 2), 0.35),  # long-axis contractions on the matrix cores
    # long axes of 8 or more cubes: the sums over them factor through a DFT over the cube index
    ((1.0, 12.0, 1.0), (1, 12, 1), 5, (2, 30, 2), 0.35),
    ((1.0, 1.0, 16.0), (1, 1, 16), 4, (1, 1, 40), 0.3),
    ((10.0, 1.0, 12.0), (10, 1, 12), 3, (25, 1, 30), 0.45),
]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("geom", range(len(GEOMS)))
@pytest.mark.parametrize("win", ["gauss", "pswf"])
def test_far_small_grids(kernel, geom, win):
    Lv, M, p, K, sg = GEOMS[geom]
    print("far small", kernel, geom, win, flush=True)
    k = oracle.KERNELS[kernel]
    G = [m * p for m in M]
    rng = np.random.default_rng(500 + 10 * geom + k)
    rho = rng.normal(size=(oracle.M_IN[k], *G))
    if win == "gauss":
        c, sigma0 = None, sg
    else:
        c, sigma0 = 14.5, Lv[0] / M[0]
    ref = oracle.far_3p_grid(kernel, Lv, M, p, K, sigma0, rho, window=_w(c))
    got = host(F.far3p_eval(Lv, M, p, K, kernel, sigma0, dev(rho), pswf_c=c))
    assert_parity(got, ref, 1e-12, "far %s %d %s" % (kernel, geom, win))


# cells whose sides are not multiples of the shortest one: M_i = ceil(L_i / h0)
# cubes of side h0 = min L_i, the last along such an axis cut by the face
CUT = [
    ((1.0, 1.0, 1.5), (1, 1, 2), 6, (2, 2, 3), 0.3),
    ((1.25, 1.0, 2.6), (2, 1, 3), 5, (3, 1, 5), 0.35),
    ((2.0, 3.5, 2.0), (1, 2, 1), 7, (2, 4, 2), 0.5),
]


@pytest.mark.parametrize("kernel", KERNELS)
@pytest.mark.parametrize("geom", range(len(CUT)))
@pytest.mark.parametrize("win", ["gauss", "pswf"])
def test_far_cut_cubes(kernel, geom, win):
    Lv, M, p, K, sg = CUT[geom]
    print("far cut cubes", kernel, geom, win, flush=True)
    k = oracle.KERNELS[kernel]
    G = [m * p for m in M]
    rng = np.random.default_rng(600 + 10 * geom + k)
    rho = rng.normal(size=(oracle.M_IN[k], *G))
    if win == "gauss":
        c, sigma0 = None, sg
    else:
        c, sigma0 = 14.5, min(Lv)
    ref = oracle.far_3p_grid(kernel, Lv, M, p, K, sigma0, rho, window=_w(c))
    got = host(F.far3p_eval(Lv, M, p, K, kernel, sigma0, dev(rho), pswf_c=c))
    assert_parity(got, ref, 1e-12, "far cut %s %d %s" % (kernel, geom, win))


def test_far_cube_laplace_1e12_full():
    # Laplace table row 1e-12: c = 29, p = 38, N_per = 9; sigma0 = the cube side
    Lv, M, p = (1.0, 1.0, 1.0), (1, 1, 1), 38
    K = F.table_modes(29.0, Lv, 1.0)
    assert K == (4, 4, 4)
    rng = np.random.default_rng(77)
    rho = rng.normal(size=(1, p, p, p))
    ref = oracle.far_3p_grid("laplace", Lv, M, p, K, 1.0, rho, window=_w(29.0))
    got = host(F.far3p_eval(Lv, M, p, K, "laplace", 1.0, dev(rho), pswf_c=29.0))
    assert_parity(got, ref, 1e-12, "far laplace p38")


def _sampled(kernel, Lv, M, p, K, c, nnz, ntgt, seed):
    k = oracle.KERNELS[kernel]
    G = [m * p for m in M]
    rng = np.random.default_rng(seed)
    rho = np.zeros((oracle.M_IN[k], *G))
    flat = rng.choice(G[0] * G[1] * G[2], size=nnz, replace=False)
    idx = np.unravel_index(flat, G)
    rho[(slice(None),) + idx] = rng.normal(size=(oracle.M_IN[k], nnz))
    got = host(F.far3p_eval(Lv, M, p, K, kernel, Lv[0] / M[0], dev(rho), pswf_c=c))
    X = oracle.top_grid(Lv, M, p)
    xs = np.stack([X[i][idx[i]] for i in range(3)], axis=1)
    tsel = rng.choice(G[0] * G[1] * G[2], size=ntgt, replace=False)
    tidx = np.unravel_index(tsel, G)
    xt = np.stack([X[i][tidx[i]] for i in range(3)], axis=1)
    ref = oracle.far_3p(kernel, Lv, Lv[0] / M[0], K, xs, rho[(slice(None),) + idx].T, xt, window=_w(c))
    return got[(slice(None),) + tidx].T, ref


def test_far_cube_stokeslet_1e12_sampled():
    # Stokeslet table row 1e-12: c = 32.46, p = 44, N_per = 11
    Lv, M, p = (1.0, 1.0, 1.0), (1, 1, 1), 44
    K = F.table_modes(32.46, Lv, 1.0)
    assert K == (5, 5, 5)
    got, ref = _sampled("stokeslet", Lv, M, p, K, 32.46, 4000, 256, 78)
    assert_parity(got, ref, 1e-12, "far stokeslet p44")


@pytest.mark.parametrize("kernel,c,p", [("stresslet", 33.51, 44), ("rotlet", 32.46, 44), ("laplace", 29.0, 38)])
def test_far_elongated_cell_sampled(kernel, c, p):
    # the cuboid (32, 1, 1) of 32 top cubes: 32 times the modes along x
    Lv, M = (32.0, 1.0, 1.0), (32, 1, 1)
    K = F.table_modes(c, Lv, 1.0)
    print("far elongated", kernel, K, flush=True)
    got, ref = _sampled(kernel, Lv, M, p, K, c, 1500, 128, 79)
    assert_parity(got, ref, 1e-12, "far elongated %s" % kernel)


@pytest.mark.parametrize("kernel,axis", [("laplace", 2), ("stokeslet", 1), ("rotlet", 2)])
def test_far_elongated_other_axes_sampled(kernel, axis):
    # the 32-cube cuboid along axis 1 or 2 (the contraction over the
    # innermost grid index, or the middle one, on a DFT of length 32)
    c, p = (29.0, 38) if kernel == "laplace" else (32.46, 44)
    Lv, M = [1.0, 1.0, 1.0], [1, 1, 1]
    Lv[axis], M[axis] = 32.0, 32
    Lv, M = tuple(Lv), tuple(M)
    K = F.table_modes(c, Lv, 1.0)
    print("far elongated axis", axis, kernel, K, flush=True)
    got, ref = _sampled(kernel, Lv, M, p, K, c, 1500, 128, 84 + axis)
    assert_parity(got, ref, 1e-12, "far elongated axis %d %s" % (axis, kernel))


@pytest.mark.parametrize("kernel,Lv,M,c,p", [("laplace", (128.0, 1.0, 1.0), (128, 1, 1), 29.0, 38),
                                              ("stokeslet", (1.0, 1.0, 64.0), (1, 1, 64), 32.46, 44)])
def test_far_long_cuboid_sampled(kernel, Lv, M, c, p):
    # 128 cubes (DFT of 128 terms, eight wavefronts per tile) and 64 cubes
    # along the innermost axis (64 terms, one wavefront per tile), the
    # paper's 1e-12 parameters
    K = F.table_modes(c, Lv, 1.0)
    print("far long cuboid", kernel, M, K, flush=True)
    got, ref = _sampled(kernel, Lv, M, p, K, c, 1200, 96, 88)
    assert_parity(got, ref, 1e-12, "far long cuboid %s %s" % (kernel, M))


@pytest.mark.parametrize("kernel", KERNELS)
def test_far_edge_cases(kernel):
    k = oracle.KERNELS[kernel]
    rng = np.random.default_rng(81)
    # K = 0: only k = 0, which is excluded -> exactly zero
    rho = rng.normal(size=(oracle.M_IN[k], 4, 4, 4))
    got = host(F.far3p_eval((1.0, 1.0, 1.0), (1, 1, 1), 4, (0, 0, 0), kernel, 0.3, dev(rho)))
    assert np.all(got == 0.0)
    # one grid point per cube (p = 1), modes along one axis only
    Lv, M, p, K = (3.0, 1.0, 2.0), (3, 1, 2), 1, (4, 0, 2)
    rho = rng.normal(size=(oracle.M_IN[k], 3, 1, 2))
    ref = oracle.far_3p_grid(kernel, Lv, M, p, K, 0.4, rho)
    got = host(F.far3p_eval(Lv, M, p, K, kernel, 0.4, dev(rho)))
    assert_parity(got, ref, 1e-12, "far p=1 %s" % kernel)


def test_far_largest_order():
    # p = 64 on one cube, stresslet (9 strength components)
    Lv, M, p, K = (1.0, 1.0, 1.0), (1, 1, 1), 64, (1, 2, 1)
    rng = np.random.default_rng(82)
    rho = rng.normal(size=(9, p, p, p))
    ref = oracle.far_3p_grid("stresslet", Lv, M, p, K, 0.4, rho)
    got = host(F.far3p_eval(Lv, M, p, K, "stresslet", 0.4, dev(rho)))
    assert_parity(got, ref, 1e-12, "far p=64")


def test_far_deterministic():
    """Repeated calls give bit-identical grids: every sum (the split long-axis
    contractions and their partials included) runs in a fixed order."""
    import torch
    rng = np.random.default_rng(81)
    for Lv, M in (((1.0, 1.0, 1.0), (1, 1, 1)), ((32.0, 1.0, 1.0), (32, 1, 1))):
        K = F.table_modes(29.0, Lv, 1.0)
        rho = dev(rng.normal(size=(1, 38 * M[0], 38 * M[1], 38 * M[2])))
        a = F.far3p_eval(Lv, M, 38, K, "laplace", 1.0, rho, pswf_c=29.0)
        b = F.far3p_eval(Lv, M, 38, K, "laplace", 1.0, rho, pswf_c=29.0)
        torch.cuda.synchronize()
        assert torch.equal(a, b), Lv


# Long axes of 65 or more cubes: the sums over the cube index run as FFTs
# (Stockham stages of radix 2..8, or Bluestein's chirp convolution for
# lengths with a prime factor above 8; Sec. 4, large aspect ratios).
FFT_CASES = [
    # (L, M, p, K, kernel): radix mixes along each axis, a prime length, a
    # length with a large prime factor, two long axes at once
    ((72.0, 1.0, 1.0), (72, 1, 1), 3, (150, 1, 1), "laplace"),      # 8 * 3 * 3
    ((1.0, 97.0, 1.0), (1, 97, 1), 3, (1, 160, 1), "stokeslet"),    # prime: Bluestein
    ((1.0, 1.0, 130.0), (1, 1, 130), 3, (1, 1, 200), "rotlet"),     # 2 * 5 * 13: Bluestein
    ((1.0, 1.0, 210.0), (1, 1, 210), 2, (1, 1, 300), "stresslet"),  # 2 * 3 * 5 * 7
    ((66.0, 1.0, 70.0), (66, 1, 70), 1, (60, 1, 60), "laplace"),    # two long axes, 66 = 2 * 3 * 11
]


@pytest.mark.parametrize("case", range(len(FFT_CASES)))
@pytest.mark.parametrize("win", ["gauss", "pswf"])
def test_far_fft_lengths(case, win):
    Lv, M, p, K, kernel = FFT_CASES[case]
    print("far fft", case, M, kernel, win, flush=True)
    k = oracle.KERNELS[kernel]
    G = [m * p for m in M]
    rng = np.random.default_rng(900 + case)
    rho = rng.normal(size=(oracle.M_IN[k], *G))
    c = None if win == "gauss" else 14.5
    sigma0 = 0.6 if win == "gauss" else 1.0
    ref = oracle.far_3p_grid(kernel, Lv, M, p, K, sigma0, rho, window=_w(c))
    got = host(F.far3p_eval(Lv, M, p, K, kernel, sigma0, dev(rho), pswf_c=c))
    assert_parity(got, ref, 1e-12, "far fft %d %s" % (case, win))


@pytest.mark.parametrize("kernel,Lv,M,c,p,nnz", [
    ("laplace", (256.0, 1.0, 1.0), (256, 1, 1), 29.0, 38, 400),
    ("laplace", (1024.0, 1.0, 1.0), (1024, 1, 1), 29.0, 38, 300),
    ("stokeslet", (1.0, 1.0, 256.0), (1, 1, 256), 32.46, 44, 200),
    ("rotlet", (1.0, 251.0, 1.0), (1, 251, 1), 32.46, 44, 200),
])
def test_far_fft_long_cuboid_sampled(kernel, Lv, M, c, p, nnz):
    # hundreds to a thousand cubes at the paper's 1e-12 parameters (251 is
    # prime: Bluestein); sparse proxy strengths keep the oracle's direct sums
    # over the ~1e5 - 8e5 wave numbers affordable
    K = F.table_modes(c, Lv, 1.0)
    print("far fft long cuboid", kernel, M, K, flush=True)
    got, ref = _sampled(kernel, Lv, M, p, K, c, nnz, 64, 89)
    assert_parity(got, ref, 1e-12, "far fft long cuboid %s %s" % (kernel, M))
