"""The allocation-free variant of dmk_residual_eval: its workspace is the
library's file-scope device array, so it must give exactly the results of
dmk_residual_eval with a caller-owned workspace, call after call, and refuse
sizes beyond that array."""
import numpy as np
import pytest

from paper_2606_27134_amd import _lib as L
from paper_2606_27134_amd import workloads as W


def test_noalloc_size_limit_host_only():
    # more sorted strengths than the array holds: rejected before any device work
    g = L.make_grid((1, 1, 1), 3, (4, 4, 4))
    b = L.dmk_bins()
    N = L.NOALLOC_WS_BYTES // 8 + 1
    assert L.dmk_bins_carve(g, N, 1 << 40, L.dmk_bins_bytes(g, N), b) == L.DMK_OK
    P = 1 << 41
    assert L.dmk_residual_eval_noalloc(g, b, 0, 0, 0.05, 0.1, P, P, 0) == L.DMK_ESIZE
    # Stokeslet strengths (3 per point) overflow at a third of that
    N3 = L.NOALLOC_WS_BYTES // 24 + 1
    assert L.dmk_bins_carve(g, N3, 1 << 40, L.dmk_bins_bytes(g, N3), b) == L.DMK_OK
    assert L.dmk_residual_eval_noalloc(g, b, 1, 0, 0.05, 0.1, P, P, 0) == L.DMK_ESIZE
    assert L.dmk_residual_eval_noalloc(g, b, 7, 0, 0.05, 0.1, P, P, 0) == L.DMK_EUNSUPPORTED


@pytest.mark.gpu
@pytest.mark.parametrize("kernel,prec", [("laplace", "fp32c"), ("stokeslet", "fp64"), ("stresslet", "fp32c")])
def test_noalloc_matches_eval_two_calls(kernel, prec):
    import torch
    from paper_2606_27134_amd import residual as R
    torch.cuda.set_device(0)
    k, p = L.KERNELS[kernel], L.PRECS[prec]
    stream = torch.cuda.current_stream().cuda_stream
    # two calls in a row on one device, the second with fewer points
    for N, seed in ((30000, 11), (7000, 12)):
        w = W.random_case(seed, kernel, 3, (1.0, 1.0, 1.0), (12, 12, 12), N)
        print("noalloc case", kernel, prec, N, flush=True)
        x = torch.as_tensor(w.x).cuda()
        rho = torch.as_tensor(w.rho).cuda()
        bins = R.tree_bin(w.L, w.D, w.n, x)
        ref = R.residual_eval(bins, kernel, prec, w.sigma, w.rc, rho)
        u = torch.full_like(ref, float("nan"))
        code = L.dmk_residual_eval_noalloc(bins.grid, bins.c, k, p, w.sigma, w.rc, rho.data_ptr(), u.data_ptr(),
                                           stream)
        assert code == L.DMK_OK, L.strerror(code)
        torch.cuda.synchronize()
        # same kernels on the same inputs: bit-identical results
        assert torch.equal(u, ref)
        assert np.isfinite(u.cpu().numpy()).all()
