"""PyTorch-facing wrappers of libdmkloc.

Tensors are used only as device memory and the current HIP stream carries
every launch.  The arithmetic is entirely in the library's kernels; there is
no host or PyTorch fallback.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import _lib as L


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _kid(kernel) -> int:
    return L.KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def _pid(prec) -> int:
    return L.PRECS[prec] if isinstance(prec, str) else int(prec)


def _require_dev_f64(t: torch.Tensor, name: str, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))


class Bins:
    """Binned point set: owns the device arena that dmk_bins_carve splits."""

    def __init__(self, L_, D: int, n, N: int, device=None):
        self.grid = L.make_grid(L_, D, n)
        self.N = int(N)
        nbytes = L.dmk_bins_bytes(self.grid, self.N)
        if nbytes == 0:
            raise L.DmkError(L.DMK_EINVAL, "dmk_bins_bytes")
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self._arena.data_ptr()
        self._off = (-base) % 256
        self.nbytes = nbytes
        self.c = L.dmk_bins()
        code = L.dmk_bins_carve(self.grid, self.N, base + self._off, nbytes, self.c)
        if code != L.DMK_OK:
            raise L.DmkError(code, "dmk_bins_carve")

    def bin(self, x: torch.Tensor):
        _require_dev_f64(x, "x", (self.N, 3))
        code = L.dmk_tree_bin(self.grid, x.data_ptr(), self.c, _stream())
        if code != L.DMK_OK:
            raise L.DmkError(code, "dmk_tree_bin")
        return self

    @property
    def ntiles(self) -> int:
        return int(self.c.ntiles)

    @property
    def nheavy(self) -> int:
        """Leading tiles that the pair kernels run with the larger workgroup."""
        return int(self.c.nheavy)

    # views into the arena (for tests and diagnostics)
    def _view(self, ptr, count, dtype):
        esz = torch.empty((), dtype=dtype).element_size()
        start = ptr - self._arena.data_ptr()
        return self._arena[start:start + count * esz].view(dtype)

    def key(self):
        return self._view(self.c.key, self.N, torch.int32)

    def perm(self):
        return self._view(self.c.perm, self.N, torch.int32)

    def skey(self):
        return self._view(self.c.skey, self.N, torch.int32)

    def box_start(self):
        return self._view(self.c.box_start, int(self.c.nbox) + 1, torch.int32)

    def ys(self):
        return self._view(self.c.ys, 3 * self.N, torch.float64).view(3, self.N)

    def axis_tables(self):
        rows = sum(int(v) for v in self.grid.n)
        nbr = self._view(self.c.axis_nbr, 3 * rows, torch.int32).view(rows, 3)
        img = self._view(self.c.axis_img, 3 * rows, torch.int8).view(rows, 3)
        return nbr, img

    def tiles(self):
        return self._view(self.c.tiles, 4 * self.ntiles, torch.int32).view(self.ntiles, 4)


def tree_bin(L_, D, n, x: torch.Tensor) -> Bins:
    return Bins(L_, D, n, x.shape[0], device=x.device).bin(x)


def workspace(bins: Bins, kernel, prec, backward: bool) -> torch.Tensor:
    nb = L.dmk_residual_ws_bytes(bins.grid, bins.c, _kid(kernel), _pid(prec), int(backward))
    return torch.empty(max(nb, 8) // 8 + 32, dtype=torch.float64, device=bins._arena.device)


_PSWF = {}


def pswf_window(c: float):
    """Host description of the PSWF window of bandwidth c (computed by the
    library, cached per c)."""
    c = float(c)
    if c not in _PSWF:
        w = L.dmk_pswf()
        code = L.dmk_pswf_window(c, w)
        if code != L.DMK_OK:
            raise L.DmkError(code, "dmk_pswf_window")
        _PSWF[c] = w
    return _PSWF[c]


def residual_eval(bins: Bins, kernel, prec, sigma: float, rc: float, rho: torch.Tensor, out=None, ws=None,
                  pswf_c: float = None):
    """Residual sum u[N, m_out].  Gaussian split of width sigma with cutoff rc,
    or, with pswf_c, the PSWF split of bandwidth pswf_c and support rc
    (sigma is then unused)."""
    k, p = _kid(kernel), _pid(prec)
    _require_dev_f64(rho, "rho", (bins.N, L.M_IN[k]))
    u = out if out is not None else torch.empty((bins.N, L.M_OUT[k]), dtype=torch.float64, device=rho.device)
    _require_dev_f64(u, "u", (bins.N, L.M_OUT[k]))
    if ws is None:
        ws = workspace(bins, k, p, False)
    if pswf_c is None:
        code = L.dmk_residual_eval(bins.grid, bins.c, k, p, sigma, rc, rho.data_ptr(), u.data_ptr(),
                                   ws.data_ptr(), ws.numel() * 8, _stream())
    else:
        code = L.dmk_residual_eval_pswf(bins.grid, bins.c, k, p, pswf_window(pswf_c), rc, rho.data_ptr(),
                                        u.data_ptr(), ws.data_ptr(), ws.numel() * 8, _stream())
    if code != L.DMK_OK:
        raise L.DmkError(code, "dmk_residual_eval")
    return u


def residual_backward(bins: Bins, kernel, prec, sigma: float, rc: float, rho: torch.Tensor, gu: torch.Tensor,
                      out=None, ws=None, pswf_c: float = None):
    """Vector-Jacobian product of :func:`residual_eval` (same split arguments)."""
    k, p = _kid(kernel), _pid(prec)
    _require_dev_f64(rho, "rho", (bins.N, L.M_IN[k]))
    _require_dev_f64(gu, "gu", (bins.N, L.M_OUT[k]))
    if out is None:
        grho = torch.empty((bins.N, L.M_IN[k]), dtype=torch.float64, device=rho.device)
        gx = torch.empty((bins.N, 3), dtype=torch.float64, device=rho.device)
    else:
        grho, gx = out
    if ws is None:
        ws = workspace(bins, k, p, True)
    if pswf_c is None:
        code = L.dmk_residual_backward(bins.grid, bins.c, k, p, sigma, rc, rho.data_ptr(), gu.data_ptr(),
                                       grho.data_ptr(), gx.data_ptr(), ws.data_ptr(), ws.numel() * 8, _stream())
    else:
        code = L.dmk_residual_backward_pswf(bins.grid, bins.c, k, p, pswf_window(pswf_c), rc, rho.data_ptr(),
                                            gu.data_ptr(), grho.data_ptr(), gx.data_ptr(), ws.data_ptr(),
                                            ws.numel() * 8, _stream())
    if code != L.DMK_OK:
        raise L.DmkError(code, "dmk_residual_backward")
    return grho, gx


def gather_sorted(bins: Bins, src: torch.Tensor, out=None) -> torch.Tensor:
    """Sorted SoA copy dst[m, N] (dst[c][j] = src[perm[j]][c]) of src[N, m]."""
    if src.dim() != 2 or src.shape[0] != bins.N:
        raise ValueError("src must be [N, m] with N = %d" % bins.N)
    _require_dev_f64(src, "src")
    m = int(src.shape[1])
    dst = out if out is not None else torch.empty((m, bins.N), dtype=torch.float64, device=src.device)
    _require_dev_f64(dst, "dst", (m, bins.N))
    code = L.dmk_gather_sorted(bins.c, m, src.data_ptr(), dst.data_ptr(), _stream())
    if code != L.DMK_OK:
        raise L.DmkError(code, "dmk_gather_sorted")
    return dst


def residual_eval_sorted(bins: Bins, kernel, prec, sigma: float, rc: float, rho_sorted: torch.Tensor, out=None,
                         pswf_c: float = None):
    """Pair kernel alone on sorted strengths rho_sorted[m_in, N]; u[N, m_out]
    in the original order."""
    k, p = _kid(kernel), _pid(prec)
    _require_dev_f64(rho_sorted, "rho_sorted", (L.M_IN[k], bins.N))
    u = out if out is not None else torch.empty((bins.N, L.M_OUT[k]), dtype=torch.float64,
                                                device=rho_sorted.device)
    _require_dev_f64(u, "u", (bins.N, L.M_OUT[k]))
    w = pswf_window(pswf_c) if pswf_c is not None else None
    code = L.dmk_residual_eval_sorted(bins.grid, bins.c, k, p, sigma, rc, w, rho_sorted.data_ptr(), u.data_ptr(),
                                      _stream())
    if code != L.DMK_OK:
        raise L.DmkError(code, "dmk_residual_eval_sorted")
    return u


def residual_backward_sorted(bins: Bins, kernel, prec, sigma: float, rc: float, rho_sorted: torch.Tensor,
                             gu_sorted: torch.Tensor, out=None, pswf_c: float = None):
    """Adjoint pair kernel alone on sorted strengths and cotangent."""
    k, p = _kid(kernel), _pid(prec)
    _require_dev_f64(rho_sorted, "rho_sorted", (L.M_IN[k], bins.N))
    _require_dev_f64(gu_sorted, "gu_sorted", (L.M_OUT[k], bins.N))
    if out is None:
        grho = torch.empty((bins.N, L.M_IN[k]), dtype=torch.float64, device=rho_sorted.device)
        gx = torch.empty((bins.N, 3), dtype=torch.float64, device=rho_sorted.device)
    else:
        grho, gx = out
    w = pswf_window(pswf_c) if pswf_c is not None else None
    code = L.dmk_residual_backward_sorted(bins.grid, bins.c, k, p, sigma, rc, w, rho_sorted.data_ptr(),
                                          gu_sorted.data_ptr(), grho.data_ptr(), gx.data_ptr(), _stream())
    if code != L.DMK_OK:
        raise L.DmkError(code, "dmk_residual_backward_sorted")
    return grho, gx


@dataclass
class ResidualSpec:
    """Problem description for :class:`DmkResidual`."""
    L: tuple
    D: int
    n: tuple
    kernel: str
    prec: str
    sigma: float
    rc: float
    pswf_c: float = None   # PSWF split of bandwidth pswf_c and support rc instead of the Gaussian


class DmkResidual(torch.autograd.Function):
    """u = residual sum of K_R over the leaf neighbourhood (HIP kernels).

    forward(x[N,3], rho[N,m_in], spec, bins=None) -> u[N,m_out]; backward
    gives (grad_x, grad_rho) from the library's adjoint kernel.  The points
    are binned on every forward call unless a Bins built from these exact
    positions is passed in (then the caller vouches that it matches x).  The
    forward keeps the strengths in the sorted order, so the backward gathers
    only the cotangent.
    """

    @staticmethod
    def forward(ctx, x, rho, spec: ResidualSpec, bins: Bins = None):
        x_ = x.detach().contiguous()
        rho_ = rho.detach().contiguous()
        if bins is None:
            bins = tree_bin(spec.L, spec.D, spec.n, x_)
        elif bins.N != x_.shape[0]:
            raise ValueError("bins were built for %d points, x has %d" % (bins.N, x_.shape[0]))
        rho_s = gather_sorted(bins, rho_)
        u = residual_eval_sorted(bins, spec.kernel, spec.prec, spec.sigma, spec.rc, rho_s, pswf_c=spec.pswf_c)
        ctx.spec = spec
        ctx.bins = bins
        ctx.save_for_backward(rho_s)
        return u

    @staticmethod
    def backward(ctx, gu):
        (rho_s,) = ctx.saved_tensors
        s = ctx.spec
        gu_s = gather_sorted(ctx.bins, gu.contiguous())
        grho, gx = residual_backward_sorted(ctx.bins, s.kernel, s.prec, s.sigma, s.rc, rho_s, gu_s,
                                            pswf_c=s.pswf_c)
        return gx, grho, None, None


def dmk_residual(x, rho, spec: ResidualSpec, bins: Bins = None):
    return DmkResidual.apply(x, rho, spec, bins)
