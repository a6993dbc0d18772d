"""Root-level far field of the triply periodic split (D = 3) on the
top-level Chebyshev grids: wrapper of ``dmk_far3p_eval``.

The cell is tiled exactly by M0 x M1 x M2 cubes; every cube carries p^3
first-kind Chebyshev points and the far field of proxy strengths on those
points is evaluated on the same points (Sec. 4, evaluation of the far-field
contribution, eqs. (structurefac), (eval_tensor)).  All arithmetic is in the
library's kernels.
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
