"""Shared helpers of the GPU tests (no arithmetic of the method)."""
import sys

import numpy as np
import pytest

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    torch = None
    HAVE_GPU = False

needs_gpu = pytest.mark.skipif(not HAVE_GPU, reason="needs a GPU")


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_l2(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.linalg.norm(ref)
    return np.linalg.norm(got - ref) / (den if den > 0 else 1.0)


def assert_parity(got, ref, tol, what=""):
    """rel l2 <= tol and every element within tol * max|ref| (elementwise bar)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.isfinite(got).all(), what + ": non-finite output"
    e = rel_l2(got, ref)
    scale = np.abs(ref).max() if ref.size else 1.0
    emax = np.abs(got - ref).max() / (scale if scale > 0 else 1.0) if ref.size else 0.0
    print("%s rel_l2=%.3e max_rel=%.3e" % (what, e, emax), flush=True)
    sys.stdout.flush()
    assert e <= tol, "%s: rel l2 %.3e > %.1e" % (what, e, tol)
    assert emax <= 10 * tol, "%s: max elementwise %.3e > %.1e" % (what, emax, 10 * tol)
