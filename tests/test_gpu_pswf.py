"""Parity of the PSWF-split residual kernels (dmk_residual_eval_pswf /
dmk_residual_backward_pswf through the C ABI) with the CPU oracle evaluating
its own PSWF window (Sec. 2.2, eq. (wfunc_pswf); App. B formulas at t = r/nu).

Bars as for the Gaussian split: FP64 rel l2 <= 1e-12, FP32-compensated
<= 1e-6.  The bandwidths c are the paper's parameter-table values for the
tolerance 1e-6 (Laplace 14.5, Stokeslet and stresslet 17.80, rotlet 13.61)
and 29 (Laplace, 1e-12); the support nu is the leaf box size.
"""
import numpy as np
import pytest

import oracle
from oracle.pswf import PswfWindow
from gpu_util import HAVE_GPU, assert_parity, dev, host, needs_gpu
from paper_2606_27134_amd import workloads as W

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    from paper_2606_27134_amd import residual as R

TOL = {"fp64": 1e-12, "fp32c": 1e-6}
KERNELS = ["laplace", "stokeslet", "stresslet", "rotlet"]
C_OF = {"laplace": 14.5, "stokeslet": 17.80, "stresslet": 17.80, "rotlet": 13.61}
_OW = {}


def _ow(c):
    if c not in _OW:
        _OW[c] = PswfWindow(c)
    return _OW[c]


SMALL = []
for k in KERNELS:
    SMALL += [
        (k, 3, (1.0, 1.0, 1.0), (8, 8, 8), 3000, "uniform", C_OF[k]),
        (k, 2, (1.0, 1.0, 2.0), (6, 6, 12), 2500, "clustered", C_OF[k]),
        (k, 1, (4.0, 1.0, 1.0), (20, 5, 5), 3000, "uniform", C_OF[k]),
        (k, 0, (1.0, 1.0, 1.0), (7, 5, 6), 2000, "uniform", C_OF[k]),
    ]
SMALL += [("laplace", 3, (1.0, 1.0, 1.0), (8, 8, 8), 3000, "uniform", 29.0)]


def _case(i):
    k, D, Lv, n, N, dist, c = SMALL[i]
    return W.random_case(seed=700 + i, kernel=k, D=D, L=Lv, n=n, N=N, dist=dist), c


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("i", range(len(SMALL)))
def test_pswf_forward_small(i, prec):
    w, c = _case(i)
    print("case", SMALL[i], prec, flush=True)
    b = R.tree_bin(w.L, w.D, w.n, dev(w.x))
    got = host(R.residual_eval(b, w.kernel, prec, 0.0, w.rc, dev(w.rho), pswf_c=c))
    ref = oracle.residual(w.kernel, w.D, w.L, w.rc, w.rc, w.x, w.rho, window=_ow(c))
    assert_parity(got, ref, TOL[prec], "pswf fwd %s %s D=%d c=%g" % (w.kernel, prec, w.D, c))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("i", range(len(SMALL)))
def test_pswf_backward_small(i, prec):
    w, c = _case(i)
    print("case", SMALL[i], prec, flush=True)
    G = W.cotangent(w.seed, w.N, W.M_OUT[w.kernel])
    b = R.tree_bin(w.L, w.D, w.n, dev(w.x))
    gr, gx = R.residual_backward(b, w.kernel, prec, 0.0, w.rc, dev(w.rho), dev(G), pswf_c=c)
    rr, rx = oracle.residual_vjp(w.kernel, w.D, w.L, w.rc, w.rc, w.x, w.rho, G, window=_ow(c))
    assert_parity(host(gr), rr, TOL[prec], "pswf grad_rho %s %s D=%d" % (w.kernel, prec, w.D))
    assert_parity(host(gx), rx, TOL[prec], "pswf grad_x %s %s D=%d" % (w.kernel, prec, w.D))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
@pytest.mark.parametrize("kernel", ["laplace", "stresslet"])
def test_pswf_dense_boxes(kernel, prec):
    # a cluster much denser than a tile's staging capacity: dense tiles
    rng = np.random.default_rng(78)
    N = 6000
    x = np.vstack([rng.random((N - 2500, 3)), 0.5 + 0.01 * rng.standard_normal((2500, 3))]) % 1.0
    m_in = W.M_IN[kernel]
    rho = rng.normal(size=(N, m_in))
    c = C_OF[kernel]
    rc = 1.0 / 8
    b = R.tree_bin((1.0, 1.0, 1.0), 3, (8, 8, 8), dev(x))
    assert b.nheavy > 0  # the cluster's dense tiles lead the order as heavy tiles
    got = host(R.residual_eval(b, kernel, prec, 0.0, rc, dev(rho), pswf_c=c))
    t = np.sort(rng.choice(N, size=300, replace=False))
    t = np.unique(np.concatenate([t, np.arange(N - 2500, N - 2300)]))
    ref = oracle.residual(kernel, 3, (1, 1, 1), rc, rc, x, rho, targets=t, window=_ow(c))
    assert_parity(got[t], ref, TOL[prec], "pswf dense %s %s" % (kernel, prec))
    G = rng.normal(size=(N, W.M_OUT[kernel]))
    gr, gx = R.residual_backward(b, kernel, prec, 0.0, rc, dev(rho), dev(G), pswf_c=c)
    rr, rx = oracle.residual_vjp(kernel, 3, (1, 1, 1), rc, rc, x, rho, G, targets=t, window=_ow(c))
    assert_parity(host(gr)[t], rr, TOL[prec], "pswf dense grad_rho %s %s" % (kernel, prec))
    assert_parity(host(gx)[t], rx, TOL[prec], "pswf dense grad_x %s %s" % (kernel, prec))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_pswf_full_size_sampled_c2_geometry(prec):
    # the 1e6-point Laplace workload's geometry with the PSWF split (support = leaf box)
    w = W.make("laplace_n1m")
    c = 14.5
    b = R.tree_bin(w.L, w.D, w.n, dev(w.x))
    got = host(R.residual_eval(b, w.kernel, prec, 0.0, w.rc, dev(w.rho), pswf_c=c))
    t = np.sort(np.random.default_rng(9).choice(w.N, size=400, replace=False))
    ref = oracle.residual(w.kernel, w.D, w.L, w.rc, w.rc, w.x, w.rho, targets=t, window=_ow(c))
    assert_parity(got[t], ref, TOL[prec], "pswf laplace_n1m %s" % prec)
