"""Parity of the HIP residual kernels (through the C ABI) with the CPU oracle.

Bars: FP64 path rel l2 <= 1e-12, FP32-compensated path rel l2 <= 1e-6, and
every element within 10x that bar relative to the largest reference value.
Small cases compare every output; full-size workloads (the sizes the bench
runs) compare a seeded sample of targets that the oracle evaluates one by
one.
"""
import numpy as np
import pytest

import oracle
from gpu_util import HAVE_GPU, assert_parity, dev, host, needs_gpu
from paper_2606_27134_amd import workloads as W

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    import torch
    from paper_2606_27134_amd import residual as R

TOL = {"fp64": 1e-12, "fp32c": 1e-6}
KERNELS = ["laplace", "stokeslet", "stresslet", "rotlet"]


def run_fwd(w, prec, x=None, rho=None):
    x = w.x if x is None else x
    rho = w.rho if rho is None else rho
    b = R.tree_bin(w.L, w.D, w.n, dev(x))
    u = R.residual_eval(b, w.kernel, prec, w.sigma, w.rc, dev(rho))
    return host(u), b


def run_bwd(w, prec, G):
    b = R.tree_bin(w.L, w.D, w.n, dev(w.x))
    gr, gx = R.residual_backward(b, w.kernel, prec, w.sigma, w.rc, dev(w.rho), dev(G))
    return host(gr), host(gx)


def oracle_fwd(w, targets=None):
    return oracle.residual(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, targets=targets)


# --------------------------------------------------------------------------
# small cases: all outputs compared
SMALL = []
for k in KERNELS:
    SMALL += [
        (k, 3, (1.0, 1.0, 1.0), (8, 8, 8), 3000, "uniform"),
        (k, 2, (1.0, 1.0, 2.0), (6, 6, 12), 2500, "clustered"),
        (k, 1, (4.0, 1.0, 1.0), (20, 5, 5), 3000, "uniform"),
        (k, 0, (1.0, 1.0, 1.0), (7, 5, 6), 2000, "uniform"),
        # sparse (under one point per box): stencil ranges of at most 64 slots,
        # two targets per scan step
        (k, 3, (1.0, 1.0, 1.0), (12, 12, 12), 1500, "uniform"),
        (k, 1, (4.0, 1.0, 1.0), (40, 10, 10), 2000, "uniform"),
    ]


def _case(i):
    k, D, Lv, n, N, dist = SMALL[i]
    return W.random_case(seed=500 + i, kernel=k, D=D, L=Lv, n=n, N=N, dist=dist)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("i", range(len(SMALL)))
def test_forward_small(i, prec):
    w = _case(i)
    print("case", SMALL[i], prec, flush=True)
    got, b = run_fwd(w, prec)
    assert_parity(got, oracle_fwd(w), TOL[prec], "fwd %s %s D=%d" % (w.kernel, prec, w.D))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("i", range(len(SMALL)))
def test_backward_small(i, prec):
    w = _case(i)
    print("case", SMALL[i], prec, flush=True)
    G = W.cotangent(w.seed, w.N, W.M_OUT[w.kernel])
    gr, gx = run_bwd(w, prec, G)
    rr, rx = oracle.residual_vjp(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, G)
    assert_parity(gr, rr, TOL[prec], "grad_rho %s %s D=%d" % (w.kernel, prec, w.D))
    assert_parity(gx, rx, TOL[prec], "grad_x %s %s D=%d" % (w.kernel, prec, w.D))


@pytest.mark.parametrize("prec", ["fp64"])
def test_c1_full(prec):
    w = W.make("laplace_n2k")
    got, _ = run_fwd(w, prec)
    assert_parity(got, oracle_fwd(w), TOL[prec], "laplace_n2k fwd")
    G = w.rho.copy()
    gr, gx = run_bwd(w, prec, G)
    rr, rx = oracle.residual_vjp(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, G)
    assert_parity(gr, rr, TOL[prec], "laplace_n2k grad_rho")
    assert_parity(gx, rx, TOL[prec], "laplace_n2k grad_x")


# --------------------------------------------------------------------------
# dense boxes: tiles that stream their neighbourhood through LDS in chunks
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("kernel", KERNELS)
def test_dense_boxes(kernel, prec):
    rng = np.random.default_rng(77)
    N = 6000
    x = np.concatenate([0.5 + 0.03 * rng.standard_normal((4000, 3)), rng.random((2000, 3))])
    x = np.mod(x, 1.0)
    w = W.random_case(seed=78, kernel=kernel, D=3, L=(1, 1, 1), n=(5, 5, 5), N=N)
    w.x = x
    got, b = run_fwd(w, prec)
    tiles = host(b.tiles())
    assert (tiles[:, 2] < 0).sum() >= 20, "expected dense tiles"
    # both workgroup sizes run: heavy tiles (the dense ones of the cluster
    # box) and light ones
    assert 20 <= b.nheavy < b.ntiles
    assert_parity(got, oracle_fwd(w), TOL[prec], "dense fwd %s %s" % (kernel, prec))
    G = W.cotangent(78, N, W.M_OUT[kernel])
    gr, gx = run_bwd(w, prec, G)
    rr, rx = oracle.residual_vjp(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, G)
    assert_parity(gr, rr, TOL[prec], "dense grad_rho")
    assert_parity(gx, rx, TOL[prec], "dense grad_x")


# --------------------------------------------------------------------------
# edge cases
@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_edge_cases(prec):
    rng = np.random.default_rng(11)
    # tiny periodic tilings (n_i = 1, 2): a box is its own neighbour via images
    for D, Lv, n in [(3, (0.3, 0.3, 0.3), (1, 1, 1)), (3, (0.5, 0.4, 0.6), (2, 2, 2)),
                     (2, (0.4, 0.4, 0.8), (1, 2, 3)), (1, (0.5, 1.0, 1.0), (2, 4, 3))]:
        for k in KERNELS:
            w = W.random_case(seed=12, kernel=k, D=D, L=Lv, n=n, N=150)
            got, _ = run_fwd(w, prec)
            assert_parity(got, oracle_fwd(w), TOL[prec], "tiny %s D=%d n=%s" % (k, D, n))
    # rc below the box size, points on faces and duplicates, periodic inputs outside the cell
    w = W.random_case(seed=13, kernel="stokeslet", D=3, L=(1, 1, 1), n=(6, 6, 6), N=1500, rc_frac=0.6)
    x = w.x.copy()
    x[:100] = np.round(x[:100] * 6) / 6
    x[100:110] = x[110:120]
    x[200:300, 0] += 1.0
    x[300:400, 1] -= 2.0
    x[400:405, 2] = 1.0  # exactly L on a periodic axis: the image at 0
    got, _ = run_fwd(w, prec, x=x)
    ref = oracle.residual(w.kernel, w.D, w.L, w.sigma, w.rc, x, w.rho)
    assert_parity(got, ref, TOL[prec], "faces/duplicates/outside")
    # single point, and a pair across a periodic face
    w1 = W.random_case(seed=14, kernel="laplace", D=3, L=(1, 1, 1), n=(4, 4, 4), N=1)
    got, _ = run_fwd(w1, prec)
    assert got.shape == (1, 1) and got[0, 0] == 0.0
    w2 = W.random_case(seed=15, kernel="rotlet", D=3, L=(1, 1, 1), n=(4, 4, 4), N=2)
    w2.x = np.array([[0.01, 0.5, 0.5], [0.99, 0.52, 0.49]])
    got, _ = run_fwd(w2, prec)
    assert_parity(got, oracle_fwd(w2), TOL[prec], "pair across face")


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_empty_input(prec):
    """No points: binning, both pair kernels, autograd, the leaf grids and the
    self term return empty (or zero) results without launching work."""
    import torch
    from paper_2606_27134_amd import far as F
    x = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
    b = R.tree_bin((1.0, 1.0, 1.0), 3, (4, 4, 4), x)
    assert b.ntiles == 0
    for k in KERNELS:
        mi, mo = W.M_IN[k], W.M_OUT[k]
        rho = torch.zeros((0, mi), dtype=torch.float64, device="cuda")
        u = R.residual_eval(b, k, prec, 0.05, 0.25, rho)
        assert tuple(u.shape) == (0, mo)
        gr, gx = R.residual_backward(b, k, prec, 0.05, 0.25, rho, torch.zeros((0, mo), dtype=torch.float64,
                                                                                device="cuda"))
        assert tuple(gr.shape) == (0, mi) and tuple(gx.shape) == (0, 3)
    spec = R.ResidualSpec(L=(1.0, 1.0, 1.0), D=3, n=(4, 4, 4), kernel="laplace", prec=prec, sigma=0.05, rc=0.25)
    xr = x.clone().requires_grad_(True)
    q = torch.zeros((0, 1), dtype=torch.float64, device="cuda", requires_grad=True)
    u = R.dmk_residual(xr, q, spec)
    u.sum().backward()
    assert tuple(xr.grad.shape) == (0, 3) and tuple(q.grad.shape) == (0, 1)
    rg = F.cheb_anterp(b, 6, torch.zeros((0, 1), dtype=torch.float64, device="cuda"))
    assert tuple(rg.shape) == (1, 24, 24, 24) and float(rg.abs().max()) == 0.0
    ue = F.cheb_eval(b, 6, torch.ones_like(rg))
    assert tuple(ue.shape) == (0, 1)
    us = F.self_term("laplace", 0.05, torch.zeros((0, 1), dtype=torch.float64, device="cuda"),
                     torch.zeros((0, 1), dtype=torch.float64, device="cuda"))
    assert tuple(us.shape) == (0, 1)


def test_deterministic():
    w = W.random_case(seed=21, kernel="stokeslet", D=2, L=(1, 1, 2), n=(8, 8, 16), N=20000, dist="clustered")
    for prec in ("fp64", "fp32c"):
        a, _ = run_fwd(w, prec)
        b, _ = run_fwd(w, prec)
        assert a.tobytes() == b.tobytes()


# --------------------------------------------------------------------------
# full-size workloads, sampled targets
def _sample(w, k=64, seed=0):
    rng = np.random.default_rng(seed)
    t = rng.choice(w.N, size=k, replace=False)
    return np.sort(t)


FULL = [("laplace_n1m", "laplace"), ("stokeslet_n500k_clustered", "stokeslet"), ("stokes_n2m_rod", "stresslet"), ("stokes_n2m_rod", "rotlet")]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("name,kernel", FULL)
def test_full_size_sampled(name, kernel, prec):
    w = W.make(name, kernel=kernel)
    print("full", name, kernel, prec, w.N, flush=True)
    got, b = run_fwd(w, prec)
    t = _sample(w)
    if name == "stokeslet_n500k_clustered":  # include targets of the densest boxes
        sk = host(b.skey())
        perm = host(b.perm())
        dense_box = np.bincount(sk).argmax()
        t = np.unique(np.concatenate([t, perm[sk == dense_box][:32]]))
    ref = oracle_fwd(w, targets=t)
    assert_parity(got[t], ref, TOL[prec], "%s %s %s sampled" % (name, kernel, prec))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("name,kernel", FULL)
def test_full_size_backward_sampled(name, kernel, prec):
    w = W.make(name, kernel=kernel)
    print("full bwd", name, kernel, prec, flush=True)
    G = W.cotangent(w.seed, w.N, W.M_OUT[kernel])
    gr, gx = run_bwd(w, prec, G)
    t = _sample(w, seed=1)
    rr, rx = oracle.residual_vjp(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, G, targets=t)
    assert_parity(gr[t], rr, TOL[prec], "%s grad_rho %s" % (name, prec))
    assert_parity(gx[t], rx, TOL[prec], "%s grad_x %s" % (name, prec))


# --------------------------------------------------------------------------
# seeded random small cases: kernel, periodicity, box shape, tiling, size,
# distribution and cutoff drawn at random (a 400-case sweep of this generator
# found the largest rel l2 at 4.1e-13 FP64 and 6.2e-7 FP32C, stresslet)
def _random_case(i):
    rng = np.random.default_rng(9000 + i)
    k = KERNELS[rng.integers(4)]
    D = int(rng.integers(4))
    n = tuple(int(v) for v in rng.integers(1, 14, 3))
    h = float(rng.uniform(0.05, 0.2))
    L = tuple(n[j] * h * float(rng.uniform(0.9, 1.1)) for j in range(3))
    N = int(rng.integers(20, 3000))
    dist = "clustered" if rng.random() < 0.3 else "uniform"
    rcf = float(rng.choice([1.0, 1.0, 0.7, 0.4]))
    return W.random_case(seed=int(rng.integers(1 << 30)), kernel=k, D=D, L=L, n=n, N=N, dist=dist, rc_frac=rcf)


@pytest.mark.parametrize("i", range(40))
def test_random_small_cases(i):
    w = _random_case(i)
    print("random", i, w.kernel, w.D, w.n, w.N, flush=True)
    G = W.cotangent(w.seed, w.N, W.M_OUT[w.kernel])
    ref = oracle_fwd(w)
    rr, rx = oracle.residual_vjp(w.kernel, w.D, w.L, w.sigma, w.rc, w.x, w.rho, G)
    for prec in ("fp64", "fp32c"):
        got, _ = run_fwd(w, prec)
        assert_parity(got, ref, TOL[prec], "random %d fwd %s" % (i, prec))
        gr, gx = run_bwd(w, prec, G)
        assert_parity(gr, rr, TOL[prec], "random %d grad_rho %s" % (i, prec))
        assert_parity(gx, rx, TOL[prec], "random %d grad_x %s" % (i, prec))


def test_two_streams_independent():
    """The library keeps no state between calls: binnings and evaluations
    issued on two streams (default priority), interleaved, give results
    bit-identical to the same calls made one after the other on the default
    stream, and events recorded on each stream bracket that stream's work."""
    cases = [(W.make("laplace_n2k"), "fp32c"), (W.make("laplace_n2k", kernel="stokeslet"), "fp64")]
    ref = []
    for w, prec in cases:
        b = R.tree_bin(w.L, w.D, w.n, dev(w.x))
        ref.append(host(R.residual_eval(b, w.kernel, prec, w.sigma, w.rc, dev(w.rho))))
    inputs = [(dev(w.x), dev(w.rho)) for w, _ in cases]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    bins = []
    for (w, _), (x, _), s in zip(cases, inputs, streams):
        with torch.cuda.stream(s):
            bins.append(R.tree_bin(w.L, w.D, w.n, x))
    outs = [None, None]
    events = [None, None]
    print("two streams", flush=True)
    for rep in range(3):
        for k, ((w, prec), (_, rho), s) in enumerate(zip(cases, inputs, streams)):
            with torch.cuda.stream(s):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(s)
                outs[k] = R.residual_eval(bins[k], w.kernel, prec, w.sigma, w.rc, rho)
                e1.record(s)
                events[k] = (e0, e1)
    torch.cuda.synchronize()
    for k in range(2):
        assert host(outs[k]).tobytes() == ref[k].tobytes()
        e0, e1 = events[k]
        assert e0.elapsed_time(e1) > 0.0
