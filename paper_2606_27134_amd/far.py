"""Root-level far field of the triply periodic split (D = 3) on the
top-level Chebyshev grids: wrapper of ``dmk_far3p_eval``.

The cell is tiled exactly by M0 x M1 x M2 cubes (or covered by cubes of its
shortest side, the last along an axis cut by the face); every cube carries
p^3 first-kind Chebyshev points and the far field of proxy strengths on
those points is evaluated on the same points (Sec. 4, evaluation of the
far-field contribution, eqs. (structurefac), (eval_tensor)).  Long axes of an
exact tiling factor through a DFT over the cube index, an FFT from 65 cubes
on (Sec. 4, large aspect ratios).  All arithmetic is in the library's
kernels.
"""
from __future__ import annotations

import math

import torch

from . import _lib as L
from .residual import _kid, _require_dev_f64, _stream, pswf_window


def table_modes(c: float, Lv, sigma0: float):
    """Mode ranges K_i = floor(c L_i / (2 pi sigma0)): the wave numbers
    |k_i| <= c / sigma0 inside the PSWF band, which gives the mode counts
    N_per = 2 K + 1 of the parameter tables on the unit cube."""
    return tuple(int(math.floor(c * float(l) / (2.0 * math.pi * sigma0))) for l in Lv)


def far3p_eval(Lv, M, p, K, kernel, sigma0: float, rho_grid: torch.Tensor, pswf_c: float = None, out=None,
               ws=None) -> torch.Tensor:
    """u_grid[m_out, G0, G1, G2] from rho_grid[m_in, G0, G1, G2], G_i = M_i p.
    Gaussian window of width sigma0, or with pswf_c the PSWF window of
    bandwidth pswf_c and support sigma0."""
    k = _kid(kernel)
    fg = L.make_far_grid(Lv, M, p, K)
    G = tuple(int(M[i]) * int(p) for i in range(3))
    _require_dev_f64(rho_grid, "rho_grid", (L.M_IN[k],) + G)
    u = out if out is not None else torch.empty((L.M_OUT[k],) + G, dtype=torch.float64, device=rho_grid.device)
    _require_dev_f64(u, "u_grid", (L.M_OUT[k],) + G)
    nb = L.dmk_far3p_ws_bytes(fg, k)
    if nb == 0:
        raise L.DmkError(L.DMK_EINVAL, "dmk_far3p_ws_bytes")
    if ws is None:
        ws = torch.empty(nb // 8 + 32, dtype=torch.float64, device=rho_grid.device)
    w = pswf_window(pswf_c) if pswf_c is not None else None
    code = L.dmk_far3p_eval(fg, k, sigma0, w, rho_grid.data_ptr(), u.data_ptr(), ws.data_ptr(), ws.numel() * 8,
                            _stream())
    if code != L.DMK_OK:
        raise L.DmkError(code, "dmk_far3p_eval")
    return u


def cheb_workspace(bins, p: int) -> torch.Tensor:
    nb = L.dmk_cheb_ws_bytes(bins.c, p)
    if nb == 0:
        raise L.DmkError(L.DMK_EINVAL, "dmk_cheb_ws_bytes")
    return torch.empty(nb // 8 + 32, dtype=torch.float64, device=bins._arena.device)


def cheb_anterp(bins, p: int, rho: torch.Tensor, out=None, ws=None) -> torch.Tensor:
    """Proxy strengths rho_grid[m, n0 p, n1 p, n2 p] of the binned points with
    strengths rho[N, m] on the leaf boxes' Chebyshev grids."""
    m = rho.shape[1] if rho.dim() == 2 else -1
    _require_dev_f64(rho, "rho", (bins.N, m))
    G = tuple(int(bins.grid.n[i]) * int(p) for i in range(3))
    rg = out if out is not None else torch.empty((m,) + G, dtype=torch.float64, device=rho.device)
    _require_dev_f64(rg, "rho_grid", (m,) + G)
    if ws is None:
        ws = cheb_workspace(bins, p)
    code = L.dmk_cheb_anterp(bins.grid, bins.c, p, m, rho.data_ptr(), rg.data_ptr(), ws.data_ptr(),
                             ws.numel() * 8, _stream())
    if code != L.DMK_OK:
        raise L.DmkError(code, "dmk_cheb_anterp")
    return rg


def cheb_eval(bins, p: int, u_grid: torch.Tensor, out=None, accumulate: bool = False, ws=None) -> torch.Tensor:
    """u[N, m] at the binned points from grid values u_grid[m, n0 p, n1 p, n2 p]
    (added to ``out`` when accumulate)."""
    m = u_grid.shape[0]
    G = tuple(int(bins.grid.n[i]) * int(p) for i in range(3))
    _require_dev_f64(u_grid, "u_grid", (m,) + G)
    if out is None:
        if accumulate:
            raise ValueError("accumulate needs out")
        out = torch.empty((bins.N, m), dtype=torch.float64, device=u_grid.device)
    _require_dev_f64(out, "u", (bins.N, m))
    if ws is None:
        ws = cheb_workspace(bins, p)
    code = L.dmk_cheb_eval(bins.grid, bins.c, p, m, u_grid.data_ptr(), accumulate, out.data_ptr(), ws.data_ptr(),
                           ws.numel() * 8, _stream())
    if code != L.DMK_OK:
        raise L.DmkError(code, "dmk_cheb_eval")
    return out


def self_term(kernel, sigma0: float, rho: torch.Tensor, u: torch.Tensor, pswf_c: float = None) -> torch.Tensor:
    """u += self-interaction correction of the split (in place)."""
    k = _kid(kernel)
    _require_dev_f64(rho, "rho", (rho.shape[0], L.M_IN[k]))
    _require_dev_f64(u, "u", (rho.shape[0], L.M_OUT[k]))
    w = pswf_window(pswf_c) if pswf_c is not None else None
    code = L.dmk_self_term(k, sigma0, w, rho.shape[0], rho.data_ptr(), u.data_ptr(), _stream())
    if code != L.DMK_OK:
        raise L.DmkError(code, "dmk_self_term")
    return u


def single_level_3p(x: torch.Tensor, rho: torch.Tensor, kernel, Lv, c: float, p: int, K=None,
                    prec="fp64") -> torch.Tensor:
    """Triply periodic sum with the PSWF split at the root level only: the
    top cubes (side h0 = min L_i) are the leaf boxes.
    u = residual (support nu) + far field (proxy strengths on the cubes'
    grids -> far field on the grids -> evaluation at the points) + self term.
    K defaults to the mode ranges of the parameter tables (table_modes).

    When the cubes tile the cell exactly they are also the residual's boxes.
    Otherwise (Sec. 4.1.1) M_i = ceil(L_i / h0) cubes cover it, the last one
    along such an axis reaching past the cell's face: the residual then bins
    the periodic cell in floor(L_i / h0) boxes per axis (sides >= h0), and the
    proxy grids bin the same points on the cubes as free boxes of the cover;
    the points must then lie in [0, L_i).

    The support is nu = h0 (1 - 2^-30), a hair inside the cube side: a
    point's own periodic images lie at distance exactly h0 along the axes of
    side h0, and the PSWF residual kernels jump by O(phi(1)) (of the order of
    the tolerance) at the edge of their support, so such ties are kept
    clearly outside it instead of being left to the rounding of the image
    shift."""
    import math
    from .residual import residual_eval, tree_bin
    h0 = min(float(v) for v in Lv)
    nu = h0 * (1.0 - 2.0 ** -30)
    M = tuple(int(math.ceil(float(v) / h0 * (1.0 - 1e-12))) for v in Lv)
    exact = all(abs(float(v) / m - h0) <= 1e-12 * h0 for v, m in zip(Lv, M))
    if K is None:
        K = table_modes(c, Lv, h0)
    if exact:
        bins = grid_bins = tree_bin(Lv, 3, M, x)
    else:
        nres = tuple(max(1, int(math.floor(float(v) / h0 * (1.0 + 1e-12)))) for v in Lv)
        bins = tree_bin(Lv, 3, nres, x)
        grid_bins = tree_bin(tuple(m * h0 for m in M), 0, M, x)
    u = residual_eval(bins, kernel, prec, nu, nu, rho, pswf_c=c)
    ws = cheb_workspace(grid_bins, p)
    rg = cheb_anterp(grid_bins, p, rho, ws=ws)
    ug = far3p_eval(Lv, M, p, K, kernel, nu, rg, pswf_c=c)
    cheb_eval(grid_bins, p, ug, out=u, accumulate=True, ws=ws)
    return self_term(kernel, nu, rho, u, pswf_c=c)
