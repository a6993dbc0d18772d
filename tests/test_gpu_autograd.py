"""The torch.autograd.Function around the adjoint kernel.

* torch.autograd.gradcheck on tiny FP64 inputs away from the cutoff;
* central finite differences (step h = 1e-6, fourth order, FP64 path) of the energy
  E = 1/2 sum rho . u on 64 seeded points of the full-size workloads, taken
  on the local energy of each sampled point (the terms that depend on it),
  which equals the global central difference without cancellation in E;
* translation invariance sum_b dE/dx_b = 0 and dE/drho = u for the
  symmetric kernels (Laplace, Stokeslet).
"""
import numpy as np
import pytest

from gpu_util import HAVE_GPU, dev, host, needs_gpu, rel_l2
from paper_2606_27134_amd import workloads as W

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    import torch
    from paper_2606_27134_amd import residual as R


@pytest.mark.parametrize("kernel", ["laplace", "stokeslet", "stresslet", "rotlet"])
def test_gradcheck_tiny(kernel):
    rng = np.random.default_rng(3)
    # 10 points on a coarse lattice with jitter: no pair within 0.02 of rc
    while True:
        x = rng.random((10, 3))
        d = x[:, None, :] - x[None, :, :]
        d -= np.round(d)
        r = np.sqrt((d ** 2).sum(-1))
        np.fill_diagonal(r, 1.0)
        if np.abs(r - 0.45).min() > 0.03 and r.min() > 0.05:
            break
    spec = R.ResidualSpec(L=(1, 1, 1), D=3, n=(2, 2, 2), kernel=kernel, prec="fp64", sigma=0.1, rc=0.45)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda", requires_grad=True)
    rt = torch.tensor(rng.normal(size=(10, W.M_IN[kernel])), dtype=torch.float64, device="cuda",
                      requires_grad=True)
    f = lambda a, b: R.dmk_residual(a, b, spec)
    assert torch.autograd.gradcheck(f, (xt, rt), eps=1e-6, atol=1e-7, rtol=1e-6)


def _local_energy_fd(w, prec, samples, h=1e-6):
    """Central FD (step h, 4 points) of E = 1/2 sum rho.u w.r.t. x_c, on the local energy of c."""
    L = np.asarray(w.L)
    x0 = w.x.copy()
    spec = R.ResidualSpec(L=w.L, D=w.D, n=w.n, kernel=w.kernel, prec=prec, sigma=w.sigma, rc=w.rc)
    rho_t = dev(w.rho)
    fd = np.zeros((len(samples), 3))
    for si, c in enumerate(samples):
        d = x0 - x0[c]
        for ax in range(w.D):
            d[:, ax] -= L[ax] * np.round(d[:, ax] / L[ax])
        near = np.where(np.sqrt((d ** 2).sum(1)) < 1.5 * w.rc)[0]
        for ax in range(3):
            E = {}
            for s in (+2, +1, -1, -2):
                x = x0.copy()
                x[c, ax] += s * h
                u = host(R.dmk_residual(dev(x), rho_t, spec))
                E[s] = 0.5 * np.sum(w.rho[near] * u[near])
            # fourth-order central difference: the second-order one carries a
            # relative truncation error (h/r)^2, which reaches 1e-4 for the
            # closest pairs of the clustered workload
            fd[si, ax] = (-E[2] + 8 * E[1] - 8 * E[-1] + E[-2]) / (12 * h)
    return fd


@pytest.mark.parametrize("name,kernel", [("laplace_n1m", "laplace"), ("stokeslet_n500k_clustered", "stokeslet")])
def test_fd_energy_full_size(name, kernel):
    w = W.make(name, kernel=kernel)
    rng = np.random.default_rng(5)
    samples = rng.choice(w.N, size=64, replace=False)
    # skip points with a neighbour very close or within 1e-3 rc of the cutoff
    from scipy.spatial import cKDTree
    L = np.asarray(w.L)
    box = np.array([L[i] if i < w.D else 2 * L[i] + 4 * w.rc for i in range(3)])
    tree = cKDTree(np.mod(w.x, box), boxsize=box)
    keep = []
    for c in samples:
        dd, _ = tree.query(np.mod(w.x[c], box), k=64, distance_upper_bound=1.01 * w.rc)
        dd = dd[np.isfinite(dd)][1:]
        if (np.abs(dd - w.rc) > 1e-3 * w.rc).all() and (dd > 100 * 1e-6).all():
            keep.append(c)
    samples = np.array(keep)
    assert len(samples) >= 40
    spec = R.ResidualSpec(L=w.L, D=w.D, n=w.n, kernel=w.kernel, prec="fp64", sigma=w.sigma, rc=w.rc)
    xt = dev(w.x).requires_grad_(True)
    rt = dev(w.rho).requires_grad_(True)
    u = R.dmk_residual(xt, rt, spec)
    E = 0.5 * (rt * u).sum()
    gx, gr = torch.autograd.grad(E, (xt, rt))
    gx = host(gx)
    fd = _local_energy_fd(w, "fp64", samples)
    err = rel_l2(gx[samples], fd)
    print("FD %s rel_l2 = %.3e" % (name, err), flush=True)
    assert err < 1e-6
    # dE/drho = u for the symmetric kernels, sum of forces = 0
    uu = host(u)
    assert rel_l2(host(gr), uu) < 1e-12
    assert np.abs(gx.sum(0)).max() < 1e-9 * np.abs(gx).max() * np.sqrt(w.N)


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_autograd_matches_direct_calls(prec):
    w = W.random_case(seed=31, kernel="stokeslet", D=2, L=(1, 1, 2), n=(8, 8, 16), N=8000, dist="clustered")
    spec = R.ResidualSpec(L=w.L, D=w.D, n=w.n, kernel=w.kernel, prec=prec, sigma=w.sigma, rc=w.rc)
    xt = dev(w.x).requires_grad_(True)
    rt = dev(w.rho).requires_grad_(True)
    u = R.dmk_residual(xt, rt, spec)
    G = dev(W.cotangent(31, w.N, 3))
    gx, gr = torch.autograd.grad(u, (xt, rt), G)
    b = R.tree_bin(w.L, w.D, w.n, dev(w.x))
    gr2, gx2 = R.residual_backward(b, w.kernel, prec, w.sigma, w.rc, dev(w.rho), G)
    assert host(gx).tobytes() == host(gx2).tobytes()
    assert host(gr).tobytes() == host(gr2).tobytes()


@pytest.mark.parametrize("kernel", ["laplace", "stresslet"])
def test_gradcheck_tiny_pswf(kernel):
    # the PSWF split (support nu = rc, bandwidth c) through the same autograd Function
    rng = np.random.default_rng(4)
    while True:
        x = rng.random((10, 3))
        d = x[:, None, :] - x[None, :, :]
        d -= np.round(d)
        r = np.sqrt((d ** 2).sum(-1))
        np.fill_diagonal(r, 1.0)
        if np.abs(r - 0.45).min() > 0.03 and r.min() > 0.05:
            break
    spec = R.ResidualSpec(L=(1, 1, 1), D=3, n=(2, 2, 2), kernel=kernel, prec="fp64", sigma=0.0, rc=0.45,
                          pswf_c=14.5)
    xt = torch.tensor(x, dtype=torch.float64, device="cuda", requires_grad=True)
    rt = torch.tensor(rng.normal(size=(10, W.M_IN[kernel])), dtype=torch.float64, device="cuda",
                      requires_grad=True)
    f = lambda a, b: R.dmk_residual(a, b, spec)
    assert torch.autograd.gradcheck(f, (xt, rt), eps=1e-6, atol=1e-7, rtol=1e-6)
