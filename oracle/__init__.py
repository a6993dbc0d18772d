"""CPU oracle for the residual sums (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it and shares no code with it.

The arithmetic lives in ``dmk_oracle.c`` (long-double brute force, one
OpenMP thread per target batch); this module only marshals numpy arrays.

Functions follow the paper's notation:

* :func:`residual` -- mode R, eq. (u_local) of Sec. 2.3 over the image set of
  eq. (periodic-images), Sec. 1, with the residual kernels of eq.
  (Hhatsplit_wfunc) and App. B (eqs. (res_stokeslet), (res_stresslet),
  (res_rotlet)) for the Gaussian window.
* :func:`residual_vjp` -- its exact vector-Jacobian product.
* :func:`direct_free` -- D = 0 direct sum of the original kernels (App. B).
* :func:`full_split_3p` -- mode F for D = 3 (eq. (ewald_far_3P) plus the
  self-interaction correction of Sec. 2.4).
* :func:`far_3p` -- the far-field part of eq. (ewald_far_3P) alone, from given
  sources to given targets, over the cube of wave numbers of eqs.
  (wavenumbers-3p-trunc), (kintmax); :func:`far_3p_grid` applies it to the
  root-level Chebyshev grids of the top cubes (Sec. 4, evaluation of the
  far-field contribution, eqs. (structurefac), (eval_tensor)).

Every function takes ``window=None`` (the Gaussian split of width sigma) or a
:class:`oracle.pswf.PswfWindow` (the PSWF split of Sec. 2.2, eq.
(wfunc_pswf)); for the latter ``sigma`` is the support radius nu.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dmk_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

KERNELS = {"laplace": 0, "stokeslet": 1, "stresslet": 2, "rotlet": 3}
M_IN = {0: 1, 1: 3, 2: 9, 3: 3}
M_OUT = {0: 1, 1: 3, 2: 3, 3: 3}

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        D = ctypes.c_double
        C = ctypes.c_int
        lib.oracle_residual.argtypes = [C, C, P, D, D, I64, P, P, I64, P, P]
        lib.oracle_residual_vjp.argtypes = [C, C, P, D, D, I64, P, P, P, I64, P, P, P]
        lib.oracle_direct_free.argtypes = [C, I64, P, P, D, I64, P, P]
        lib.oracle_full_split_3p.argtypes = [C, P, D, I64, P, P, D, D, I64, P, P]
        lib.oracle_kernel_tensor.argtypes = [C, P, D, P, P]
        lib.oracle_kernel_free_tensor.argtypes = [C, P, P]
        lib.oracle_set_window.argtypes = [C, C, P, C, P, P, P]
        lib.oracle_set_window.restype = C
        lib.oracle_far_3p.argtypes = [C, P, D, P, I64, P, P, I64, P, P]
        lib.oracle_far_3p.restype = C
        for f in (lib.oracle_residual, lib.oracle_residual_vjp, lib.oracle_direct_free,
                  lib.oracle_full_split_3p, lib.oracle_kernel_tensor, lib.oracle_kernel_free_tensor):
            f.restype = C
        _lib = lib
    return _lib


def _set_window(window):
    lib = _load()
    if window is None:
        lib.oracle_set_window(0, 0, None, 0, None, None, None)
        return
    n, ser, qs, qw, qf = window.packed()
    ser = np.ascontiguousarray(ser, dtype=np.float64)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (qs, qw, qf)]
    if lib.oracle_set_window(1, int(n), _ptr(ser), len(qs), *[_ptr(a) for a in arrs]) != 0:
        raise ValueError("oracle_set_window: bad window")


def _kid(kernel) -> int:
    return KERNELS[kernel] if isinstance(kernel, str) else int(kernel)


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _targets(targets, n):
    if targets is None:
        return None, n
    t = np.ascontiguousarray(np.asarray(targets, dtype=np.int64).ravel())
    if t.size and (t.min() < 0 or t.max() >= n):
        raise IndexError("target index out of range")
    return t, t.size


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def residual(kernel, D, L, sigma, rc, x, rho, targets=None, window=None):
    """Mode R residual sum; returns u[ntgt, m_out] (float64)."""
    _set_window(window)
    k = _kid(kernel)
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    rho = _f64(rho, (n, M_IN[k]))
    Lv = _f64(L, (3,))
    t, nt = _targets(targets, n)
    u = np.zeros((nt, M_OUT[k]), dtype=np.float64)
    rc_ = _load().oracle_residual(k, int(D), _ptr(Lv), float(sigma), float(rc), n, _ptr(x), _ptr(rho),
                                  nt, _ptr(t), _ptr(u))
    if rc_ != 0:
        raise ValueError("oracle_residual: bad arguments")
    return u


def residual_vjp(kernel, D, L, sigma, rc, x, rho, G, targets=None, window=None):
    """Gradients of F = sum_b G_b . u_b; returns (grad_rho[ntgt, m_in], grad_x[ntgt, 3])."""
    _set_window(window)
    k = _kid(kernel)
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    rho = _f64(rho, (n, M_IN[k]))
    G = _f64(G, (n, M_OUT[k]))
    Lv = _f64(L, (3,))
    t, nt = _targets(targets, n)
    gr = np.zeros((nt, M_IN[k]), dtype=np.float64)
    gx = np.zeros((nt, 3), dtype=np.float64)
    rc_ = _load().oracle_residual_vjp(k, int(D), _ptr(Lv), float(sigma), float(rc), n, _ptr(x), _ptr(rho),
                                      _ptr(G), nt, _ptr(t), _ptr(gr), _ptr(gx))
    if rc_ != 0:
        raise ValueError("oracle_residual_vjp: bad arguments")
    return gr, gx


def direct_free(kernel, x, rho, rc=np.inf, targets=None):
    """D = 0 direct sum of the original kernels over pairs with 0 < r < rc."""
    k = _kid(kernel)
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    rho = _f64(rho, (n, M_IN[k]))
    t, nt = _targets(targets, n)
    u = np.zeros((nt, M_OUT[k]), dtype=np.float64)
    rc_ = _load().oracle_direct_free(k, n, _ptr(x), _ptr(rho), float(rc), nt, _ptr(t), _ptr(u))
    if rc_ != 0:
        raise ValueError("oracle_direct_free: bad arguments")
    return u


def full_split_3p(kernel, L, sigma, x, rho, rcut_real=None, kmax=None, targets=None, window=None):
    """Mode F (D = 3): residual over all images + Fourier part (k != 0) + self term.

    Defaults: Gaussian window: real-space cutoff 7 sigma and |k| sigma <= 14,
    so both neglected tails are below 1e-17 relative to the leading terms;
    PSWF window: the support nu = sigma and the band |k| nu <= c.
    """
    _set_window(window)
    k = _kid(kernel)
    x = _f64(x, (-1, 3))
    n = x.shape[0]
    rho = _f64(rho, (n, M_IN[k]))
    Lv = _f64(L, (3,))
    if rcut_real is None:
        rcut_real = 7.0 * sigma if window is None else sigma
    if kmax is None:
        kmax = 14.0 / sigma if window is None else window.c / sigma
    t, nt = _targets(targets, n)
    u = np.zeros((nt, M_OUT[k]), dtype=np.float64)
    rc_ = _load().oracle_full_split_3p(k, _ptr(Lv), float(sigma), n, _ptr(x), _ptr(rho), float(rcut_real),
                                       float(kmax), nt, _ptr(t), _ptr(u))
    if rc_ != 0:
        raise ValueError("oracle_full_split_3p: bad arguments")
    return u


def kernel_tensor(kernel, d, sigma, window=None):
    """Residual kernel K[j, L] and derivative dK[k, j, L] at one displacement."""
    _set_window(window)
    k = _kid(kernel)
    d = _f64(d, (3,))
    K = np.zeros((3, 9))
    dK = np.zeros((3, 3, 9))
    _load().oracle_kernel_tensor(k, _ptr(d), float(sigma), _ptr(K), _ptr(dK))
    return K[:M_OUT[k], :M_IN[k]], dK[:, :M_OUT[k], :M_IN[k]]


def kernel_free_tensor(kernel, d):
    """Original (unsplit) kernel K[j, L] at one displacement."""
    k = _kid(kernel)
    d = _f64(d, (3,))
    K = np.zeros((3, 9))
    _load().oracle_kernel_free_tensor(k, _ptr(d), _ptr(K))
    return K[:M_OUT[k], :M_IN[k]]


def far_3p(kernel, L, sigma, K, xs, rho, xt, window=None):
    """u[nt, m_out] = far-field part (eq. (ewald_far_3P)) at targets xt from
    sources xs with strengths rho, wave numbers 2 pi n_i / L_i with
    |n_i| <= K_i, n != 0."""
    _set_window(window)
    k = _kid(kernel)
    xs = _f64(xs, (-1, 3))
    xt = _f64(xt, (-1, 3))
    rho = _f64(rho, (xs.shape[0], M_IN[k]))
    Lv = _f64(L, (3,))
    Kv = np.ascontiguousarray(np.asarray(K, dtype=np.int32).reshape(3))
    u = np.zeros((xt.shape[0], M_OUT[k]), dtype=np.float64)
    rc_ = _load().oracle_far_3p(k, _ptr(Lv), float(sigma), _ptr(Kv), xs.shape[0], _ptr(xs), _ptr(rho),
                                xt.shape[0], _ptr(xt), _ptr(u))
    if rc_ != 0:
        raise ValueError("oracle_far_3p: bad arguments")
    return u


def cheb_points(p):
    """First-kind Chebyshev points cos((2j - 1) pi / (2p)), j = 1..p, on [-1, 1]
    (the proxy grid of every box, Sec. 3.1, upward pass)."""
    j = np.arange(1, p + 1, dtype=np.float64)
    return np.cos((2 * j - 1) * np.pi / (2 * p))


def top_grid(L, M, p):
    """Per-axis coordinates of the root-level (or leaf-box) Chebyshev grids:
    M0 x M1 x M2 cubes of side h0, grid index g = b p + (j - 1) on each axis,
    coordinate (b + 1/2) h0 + (h0/2) eta_j.  Either the cubes tile the cell
    [0,L0)x[0,L1)x[0,L2) exactly (h0 = L_i / M_i on every axis), or they are
    the smallest union of cubes of side h0 = min_i L_i that covers it (Sec.
    4.1.1, cube tiling): M_i = ceil(L_i / h0), the last cube along an axis
    whose length is not a multiple of h0 cut by the cell's face."""
    L = np.asarray(L, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    h = L / M
    if np.allclose(h, h[0], rtol=0, atol=1e-14 * h[0]):
        h0 = float(h[0])
    else:
        h0 = float(L.min())
        need = np.ceil(L / h0 * (1.0 - 1e-12)).astype(np.int64)
        if not np.array_equal(M, need):
            raise ValueError("the cubes neither tile the cell nor are the ceil(L_i / min L) cover: %s" % (need,))
    eta = cheb_points(p)
    return [((np.arange(M[i])[:, None] + 0.5) * h0 + 0.5 * h0 * eta[None, :]).ravel() for i in range(3)]


def far_3p_grid(kernel, L, M, p, K, sigma, rho_grid, window=None):
    """Far field on the root-level Chebyshev grids from proxy strengths on the
    same grids: rho_grid[m_in][G0][G1][G2] -> u[m_out][G0][G1][G2], G_i = M_i p,
    by the direct sums of :func:`far_3p` with every grid point a source and a
    target."""
    k = _kid(kernel)
    X = top_grid(L, M, p)
    G = [len(a) for a in X]
    pts = np.stack(np.meshgrid(*X, indexing="ij"), axis=-1).reshape(-1, 3)
    rho = np.asarray(rho_grid, dtype=np.float64).reshape(M_IN[k], -1).T
    u = far_3p(kernel, L, sigma, K, pts, rho, pts, window=window)
    return u.T.reshape(M_OUT[k], *G)
