"""ctypes binding of libdmkloc (include/dmk.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of the library.  PyTorch supplies device memory (tensors) and the
current HIP stream.  There is no fallback: if the library cannot be loaded
the call raises.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdmkloc.so")

DMK_OK, DMK_EINVAL, DMK_EDOMAIN, DMK_ECUTOFF, DMK_EUNSUPPORTED, DMK_EHIP, DMK_ESIZE = range(7)
KERNELS = {"laplace": 0, "stokeslet": 1, "stresslet": 2, "rotlet": 3}
PRECS = {"fp64": 0, "fp32c": 1}
M_IN = {0: 1, 1: 3, 2: 9, 3: 3}
M_OUT = {0: 1, 1: 3, 2: 3, 3: 3}


class dmk_grid(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("D", ctypes.c_int32), ("n", ctypes.c_int32 * 3)]


class dmk_bins(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int64), ("nbox", ctypes.c_int64), ("ntiles", ctypes.c_int64), ("nheavy", ctypes.c_int64),
        ("max_tiles", ctypes.c_int64),
        ("key", ctypes.c_void_p), ("perm", ctypes.c_void_p), ("skey", ctypes.c_void_p),
        ("box_start", ctypes.c_void_p), ("ys", ctypes.c_void_p), ("axis_nbr", ctypes.c_void_p),
        ("axis_img", ctypes.c_void_p), ("tiles", ctypes.c_void_p), ("status", ctypes.c_void_p),
        ("tmp", ctypes.c_void_p), ("tmp_ints", ctypes.c_int64),
    ]


PSWF_MAXTERMS = 32


class dmk_pswf(ctypes.Structure):
    _fields_ = [("c", ctypes.c_double), ("nterms64", ctypes.c_int32), ("nterms32", ctypes.c_int32),
                ("cheb", (ctypes.c_double * PSWF_MAXTERMS) * 4)]


class dmk_far_grid(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double * 3), ("M", ctypes.c_int32 * 3), ("p", ctypes.c_int32),
                ("K", ctypes.c_int32 * 3)]


FAR_PMAX = 64
FAR_MMAX = 4096
FAR_KMAX = 65536
GATHER_MMAX = 12
NOALLOC_WS_BYTES = 64 << 20


class DmkError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s failed: %s (status %d)" % (where, strerror(code), code))


_lib = None


def load():
    """Load libdmkloc.so; build it first only when no built library exists."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        from . import build as _build
        _build.build()
    # PyTorch's HIP libraries load their own HIP runtime by the unversioned
    # name; loaded first, it also serves this library (same soname), so
    # streams and device memory from torch are valid here.  Loaded after this
    # library, torch would bring a second runtime into the process.
    try:
        import torch  # noqa: F401
    except ImportError:  # pragma: no cover - binding used without torch
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    G = ctypes.POINTER(dmk_grid)
    B = ctypes.POINTER(dmk_bins)
    lib.dmk_bins_bytes.argtypes = [G, ctypes.c_int64]
    lib.dmk_bins_bytes.restype = ctypes.c_size_t
    lib.dmk_bins_carve.argtypes = [G, ctypes.c_int64, P, ctypes.c_size_t, B]
    lib.dmk_bins_carve.restype = ctypes.c_int
    lib.dmk_tree_bin.argtypes = [G, P, B, P]
    lib.dmk_tree_bin.restype = ctypes.c_int
    lib.dmk_residual_ws_bytes.argtypes = [G, B, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.dmk_residual_ws_bytes.restype = ctypes.c_size_t
    lib.dmk_residual_eval.argtypes = [G, B, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P, P,
                                      ctypes.c_size_t, P]
    lib.dmk_residual_eval.restype = ctypes.c_int
    lib.dmk_residual_backward.argtypes = [G, B, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P,
                                          P, P, P, ctypes.c_size_t, P]
    lib.dmk_residual_backward.restype = ctypes.c_int
    W = ctypes.POINTER(dmk_pswf)
    lib.dmk_pswf_window.argtypes = [ctypes.c_double, W]
    lib.dmk_pswf_window.restype = ctypes.c_int
    lib.dmk_residual_eval_pswf.argtypes = [G, B, ctypes.c_int, ctypes.c_int, W, ctypes.c_double, P, P, P,
                                           ctypes.c_size_t, P]
    lib.dmk_residual_eval_pswf.restype = ctypes.c_int
    lib.dmk_residual_backward_pswf.argtypes = [G, B, ctypes.c_int, ctypes.c_int, W, ctypes.c_double, P, P, P, P,
                                               P, ctypes.c_size_t, P]
    lib.dmk_residual_backward_pswf.restype = ctypes.c_int
    lib.dmk_gather_sorted.argtypes = [B, ctypes.c_int, P, P, P]
    lib.dmk_gather_sorted.restype = ctypes.c_int
    lib.dmk_residual_eval_sorted.argtypes = [G, B, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, W,
                                             P, P, P]
    lib.dmk_residual_eval_sorted.restype = ctypes.c_int
    lib.dmk_residual_backward_sorted.argtypes = [G, B, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                                 ctypes.c_double, W, P, P, P, P, P]
    lib.dmk_residual_backward_sorted.restype = ctypes.c_int
    lib.dmk_residual_eval_noalloc.argtypes = [G, B, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              P, P, P]
    lib.dmk_residual_eval_noalloc.restype = ctypes.c_int
    F = ctypes.POINTER(dmk_far_grid)
    lib.dmk_far3p_ws_bytes.argtypes = [F, ctypes.c_int]
    lib.dmk_far3p_ws_bytes.restype = ctypes.c_size_t
    lib.dmk_far3p_eval.argtypes = [F, ctypes.c_int, ctypes.c_double, P, P, P, P, ctypes.c_size_t, P]
    lib.dmk_far3p_eval.restype = ctypes.c_int
    lib.dmk_cheb_ws_bytes.argtypes = [B, ctypes.c_int]
    lib.dmk_cheb_ws_bytes.restype = ctypes.c_size_t
    lib.dmk_cheb_anterp.argtypes = [G, B, ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_size_t, P]
    lib.dmk_cheb_anterp.restype = ctypes.c_int
    lib.dmk_cheb_eval.argtypes = [G, B, ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, P, ctypes.c_size_t, P]
    lib.dmk_cheb_eval.restype = ctypes.c_int
    lib.dmk_self_term.argtypes = [ctypes.c_int, ctypes.c_double, P, ctypes.c_int64, P, P, P]
    lib.dmk_self_term.restype = ctypes.c_int
    lib.dmk_strerror.argtypes = [ctypes.c_int]
    lib.dmk_strerror.restype = ctypes.c_char_p
    lib.dmk_version.argtypes = []
    lib.dmk_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().dmk_strerror(int(code)).decode()


def make_grid(L, D, n) -> dmk_grid:
    g = dmk_grid()
    for i in range(3):
        g.L[i] = float(L[i])
        g.n[i] = int(n[i])
    g.D = int(D)
    return g


def _check(code, where):
    if code != DMK_OK:
        raise DmkError(code, where)


# ---- thin wrappers with the C names -------------------------------------
def dmk_bins_bytes(grid: dmk_grid, N: int) -> int:
    return int(load().dmk_bins_bytes(ctypes.byref(grid), int(N)))


def dmk_bins_carve(grid: dmk_grid, N: int, arena_ptr: int, nbytes: int, bins: dmk_bins) -> int:
    return int(load().dmk_bins_carve(ctypes.byref(grid), int(N), ctypes.c_void_p(arena_ptr), int(nbytes),
                                     ctypes.byref(bins)))


def dmk_tree_bin(grid: dmk_grid, x_ptr: int, bins: dmk_bins, stream: int) -> int:
    return int(load().dmk_tree_bin(ctypes.byref(grid), ctypes.c_void_p(x_ptr), ctypes.byref(bins),
                                   ctypes.c_void_p(stream)))


def dmk_residual_ws_bytes(grid: dmk_grid, bins: dmk_bins, kernel: int, prec: int, backward: int) -> int:
    return int(load().dmk_residual_ws_bytes(ctypes.byref(grid), ctypes.byref(bins), int(kernel), int(prec),
                                            int(backward)))


def dmk_residual_eval(grid, bins, kernel, prec, sigma, rc, rho_ptr, u_ptr, ws_ptr, ws_bytes, stream) -> int:
    return int(load().dmk_residual_eval(ctypes.byref(grid), ctypes.byref(bins), int(kernel), int(prec),
                                        float(sigma), float(rc), ctypes.c_void_p(rho_ptr), ctypes.c_void_p(u_ptr),
                                        ctypes.c_void_p(ws_ptr), int(ws_bytes), ctypes.c_void_p(stream)))


def dmk_residual_backward(grid, bins, kernel, prec, sigma, rc, rho_ptr, gu_ptr, grho_ptr, gx_ptr, ws_ptr, ws_bytes,
                          stream) -> int:
    return int(load().dmk_residual_backward(ctypes.byref(grid), ctypes.byref(bins), int(kernel), int(prec),
                                            float(sigma), float(rc), ctypes.c_void_p(rho_ptr),
                                            ctypes.c_void_p(gu_ptr), ctypes.c_void_p(grho_ptr),
                                            ctypes.c_void_p(gx_ptr), ctypes.c_void_p(ws_ptr), int(ws_bytes),
                                            ctypes.c_void_p(stream)))


def dmk_pswf_window(c: float, w: dmk_pswf) -> int:
    return int(load().dmk_pswf_window(float(c), ctypes.byref(w)))


def dmk_residual_eval_pswf(grid, bins, kernel, prec, w, nu, rho_ptr, u_ptr, ws_ptr, ws_bytes, stream) -> int:
    return int(load().dmk_residual_eval_pswf(ctypes.byref(grid), ctypes.byref(bins), int(kernel), int(prec),
                                             ctypes.byref(w), float(nu), ctypes.c_void_p(rho_ptr),
                                             ctypes.c_void_p(u_ptr), ctypes.c_void_p(ws_ptr), int(ws_bytes),
                                             ctypes.c_void_p(stream)))


def dmk_residual_backward_pswf(grid, bins, kernel, prec, w, nu, rho_ptr, gu_ptr, grho_ptr, gx_ptr, ws_ptr,
                               ws_bytes, stream) -> int:
    return int(load().dmk_residual_backward_pswf(ctypes.byref(grid), ctypes.byref(bins), int(kernel), int(prec),
                                                 ctypes.byref(w), float(nu), ctypes.c_void_p(rho_ptr),
                                                 ctypes.c_void_p(gu_ptr), ctypes.c_void_p(grho_ptr),
                                                 ctypes.c_void_p(gx_ptr), ctypes.c_void_p(ws_ptr), int(ws_bytes),
                                                 ctypes.c_void_p(stream)))


def dmk_gather_sorted(bins, m, src_ptr, dst_ptr, stream) -> int:
    return int(load().dmk_gather_sorted(ctypes.byref(bins), int(m), ctypes.c_void_p(src_ptr),
                                        ctypes.c_void_p(dst_ptr), ctypes.c_void_p(stream)))


def dmk_residual_eval_sorted(grid, bins, kernel, prec, sigma, rc, w, rho_s_ptr, u_ptr, stream) -> int:
    """w: a dmk_pswf (PSWF split of support rc) or None (Gaussian of width sigma, cutoff rc)."""
    return int(load().dmk_residual_eval_sorted(ctypes.byref(grid), ctypes.byref(bins), int(kernel), int(prec),
                                               float(sigma), float(rc), ctypes.byref(w) if w is not None else None,
                                               ctypes.c_void_p(rho_s_ptr), ctypes.c_void_p(u_ptr),
                                               ctypes.c_void_p(stream)))


def dmk_residual_backward_sorted(grid, bins, kernel, prec, sigma, rc, w, rho_s_ptr, gu_s_ptr, grho_ptr, gx_ptr,
                                 stream) -> int:
    return int(load().dmk_residual_backward_sorted(ctypes.byref(grid), ctypes.byref(bins), int(kernel), int(prec),
                                                   float(sigma), float(rc),
                                                   ctypes.byref(w) if w is not None else None,
                                                   ctypes.c_void_p(rho_s_ptr), ctypes.c_void_p(gu_s_ptr),
                                                   ctypes.c_void_p(grho_ptr), ctypes.c_void_p(gx_ptr),
                                                   ctypes.c_void_p(stream)))


def dmk_residual_eval_noalloc(grid, bins, kernel, prec, sigma, rc, rho_ptr, u_ptr, stream) -> int:
    return int(load().dmk_residual_eval_noalloc(ctypes.byref(grid), ctypes.byref(bins), int(kernel), int(prec),
                                                float(sigma), float(rc), ctypes.c_void_p(rho_ptr),
                                                ctypes.c_void_p(u_ptr), ctypes.c_void_p(stream)))


def make_far_grid(L, M, p, K) -> dmk_far_grid:
    g = dmk_far_grid()
    for i in range(3):
        g.L[i] = float(L[i])
        g.M[i] = int(M[i])
        g.K[i] = int(K[i])
    g.p = int(p)
    return g


def dmk_far3p_ws_bytes(fg: dmk_far_grid, kernel: int) -> int:
    return int(load().dmk_far3p_ws_bytes(ctypes.byref(fg), int(kernel)))


def dmk_far3p_eval(fg, kernel, sigma0, w, rho_ptr, u_ptr, ws_ptr, ws_bytes, stream) -> int:
    """w: a dmk_pswf (PSWF window of support sigma0) or None (Gaussian of width sigma0)."""
    return int(load().dmk_far3p_eval(ctypes.byref(fg), int(kernel), float(sigma0),
                                     ctypes.byref(w) if w is not None else None, ctypes.c_void_p(rho_ptr),
                                     ctypes.c_void_p(u_ptr), ctypes.c_void_p(ws_ptr), int(ws_bytes),
                                     ctypes.c_void_p(stream)))


def dmk_cheb_ws_bytes(bins: dmk_bins, p: int) -> int:
    return int(load().dmk_cheb_ws_bytes(ctypes.byref(bins), int(p)))


def dmk_cheb_anterp(grid, bins, p, m, rho_ptr, rg_ptr, ws_ptr, ws_bytes, stream) -> int:
    return int(load().dmk_cheb_anterp(ctypes.byref(grid), ctypes.byref(bins), int(p), int(m),
                                      ctypes.c_void_p(rho_ptr), ctypes.c_void_p(rg_ptr), ctypes.c_void_p(ws_ptr),
                                      int(ws_bytes), ctypes.c_void_p(stream)))


def dmk_cheb_eval(grid, bins, p, m, ug_ptr, accumulate, u_ptr, ws_ptr, ws_bytes, stream) -> int:
    return int(load().dmk_cheb_eval(ctypes.byref(grid), ctypes.byref(bins), int(p), int(m), ctypes.c_void_p(ug_ptr),
                                    int(bool(accumulate)), ctypes.c_void_p(u_ptr), ctypes.c_void_p(ws_ptr),
                                    int(ws_bytes), ctypes.c_void_p(stream)))


def dmk_self_term(kernel, sigma0, w, N, rho_ptr, u_ptr, stream) -> int:
    return int(load().dmk_self_term(int(kernel), float(sigma0), ctypes.byref(w) if w is not None else None, int(N),
                                    ctypes.c_void_p(rho_ptr), ctypes.c_void_p(u_ptr), ctypes.c_void_p(stream)))


def dmk_version() -> str:
    return load().dmk_version().decode()
