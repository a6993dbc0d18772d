"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/dmk.h, sizes its arena, and rejects bad arguments on the
host before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2606_27134_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "dmk.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dmk_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = L.load()
    names = _declared_functions()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name
        assert getattr(lib, name) is not None


def test_version_and_strerror():
    assert "gfx950" in L.dmk_version()
    for code in range(7):
        assert L.strerror(code)
    assert L.strerror(DMK_UNKNOWN := 99) == "unknown status"


def test_bins_bytes_and_carve_host_only():
    g = L.make_grid((1, 1, 1), 3, (64, 64, 64))
    nb = L.dmk_bins_bytes(g, 1_000_000)
    assert nb > 1_000_000 * (4 * 3 + 24)
    b = L.dmk_bins()
    fake = 1 << 40  # carve only computes pointers
    assert L.dmk_bins_carve(g, 1_000_000, fake, nb, b) == L.DMK_OK
    assert b.N == 1_000_000 and b.nbox == 64 ** 3 and b.ntiles == 0
    ptrs = [b.key, b.perm, b.skey, b.box_start, b.ys, b.axis_nbr, b.axis_img, b.tiles, b.status, b.tmp]
    assert all(p % 256 == 0 for p in ptrs)
    assert max(ptrs) < fake + nb
    assert L.dmk_bins_carve(g, 1_000_000, fake, nb - 1, b) == L.DMK_ESIZE
    assert L.dmk_bins_carve(g, 1_000_000, fake + 8, nb, b) == L.DMK_EINVAL


@pytest.mark.parametrize("L_,D,n", [((1, 1, 1), 4, (4, 4, 4)), ((1, 1, 1), 3, (0, 4, 4)),
                                    ((0, 1, 1), 3, (4, 4, 4)), ((1, -1, 1), 1, (4, 4, 4))])
def test_bad_grid_rejected(L_, D, n):
    g = L.make_grid(L_, D, n)
    assert L.dmk_bins_bytes(g, 10) == 0
    b = L.dmk_bins()
    assert L.dmk_bins_carve(g, 10, 1 << 40, 1 << 30, b) == L.DMK_EINVAL
    assert L.dmk_tree_bin(g, 0, b, 0) == L.DMK_EINVAL


def _carved(N=100):
    g = L.make_grid((1, 1, 1), 3, (4, 4, 4))
    b = L.dmk_bins()
    assert L.dmk_bins_carve(g, N, 1 << 40, L.dmk_bins_bytes(g, N), b) == L.DMK_OK
    return g, b


def test_eval_argument_errors_before_launch():
    g, b = _carved()
    P = 1 << 41
    ws = L.dmk_residual_ws_bytes(g, b, 0, 0, 0)
    assert ws >= 100 * 8
    # cutoff larger than the leaf box, non-positive cutoff, bad sigma
    assert L.dmk_residual_eval(g, b, 0, 0, 0.05, 0.3, P, P, P, ws, 0) == L.DMK_ECUTOFF
    assert L.dmk_residual_eval(g, b, 0, 0, 0.05, 0.0, P, P, P, ws, 0) == L.DMK_ECUTOFF
    assert L.dmk_residual_eval(g, b, 0, 0, -1.0, 0.1, P, P, P, ws, 0) == L.DMK_ECUTOFF
    assert L.dmk_residual_eval(g, b, 0, 0, float("nan"), 0.1, P, P, P, ws, 0) == L.DMK_ECUTOFF
    # unsupported kernel / precision
    assert L.dmk_residual_eval(g, b, 7, 0, 0.05, 0.1, P, P, P, ws, 0) == L.DMK_EUNSUPPORTED
    assert L.dmk_residual_eval(g, b, 0, 5, 0.05, 0.1, P, P, P, ws, 0) == L.DMK_EUNSUPPORTED
    # null pointers and small workspace
    assert L.dmk_residual_eval(g, b, 0, 0, 0.05, 0.1, 0, P, P, ws, 0) == L.DMK_EINVAL
    assert L.dmk_residual_eval(g, b, 0, 0, 0.05, 0.1, P, P, P, ws - 8, 0) == L.DMK_ESIZE
    wsb = L.dmk_residual_ws_bytes(g, b, 1, 1, 1)
    assert L.dmk_residual_backward(g, b, 1, 1, 0.05, 0.1, P, 0, P, P, P, wsb, 0) == L.DMK_EINVAL
    assert L.dmk_residual_backward(g, b, 1, 1, 0.05, 0.1, P, P, P, P, P, wsb - 8, 0) == L.DMK_ESIZE
    # grid / bins mismatch
    g2 = L.make_grid((1, 1, 1), 3, (5, 4, 4))
    assert L.dmk_residual_eval(g2, b, 0, 0, 0.05, 0.1, P, P, P, ws, 0) == L.DMK_EINVAL


def test_workspace_sizes_grow_with_components():
    g, b = _carved(1000)
    sizes = [L.dmk_residual_ws_bytes(g, b, k, 0, bw) for k in range(4) for bw in (0, 1)]
    assert all(s >= 1000 * 8 for s in sizes)
    assert L.dmk_residual_ws_bytes(g, b, 2, 0, 1) > L.dmk_residual_ws_bytes(g, b, 0, 0, 0)


def test_library_keeps_no_timing_hook():
    # the library records no events of its own: a caller times a pair kernel
    # with its own events around dmk_residual_eval_sorted / _backward_sorted
    assert not hasattr(L.load(), "dmk_residual_set_kernel_events")


def test_sorted_entry_points_argument_errors_before_launch():
    g, b = _carved()
    P = 1 << 41
    assert L.dmk_gather_sorted(b, 0, P, P, 0) == L.DMK_EINVAL
    assert L.dmk_gather_sorted(b, L.GATHER_MMAX + 1, P, P, 0) == L.DMK_EINVAL
    assert L.dmk_gather_sorted(b, 3, 0, P, 0) == L.DMK_EINVAL
    assert L.dmk_gather_sorted(b, 3, P, 0, 0) == L.DMK_EINVAL
    big = L.dmk_bins()
    big.N, big.perm = 1 << 30, P
    assert L.dmk_gather_sorted(big, 1, P, P, 0) == L.DMK_ESIZE
    # split arguments as in dmk_residual_eval
    assert L.dmk_residual_eval_sorted(g, b, 0, 0, 0.05, 0.3, None, P, P, 0) == L.DMK_ECUTOFF
    assert L.dmk_residual_eval_sorted(g, b, 0, 0, -1.0, 0.1, None, P, P, 0) == L.DMK_ECUTOFF
    assert L.dmk_residual_eval_sorted(g, b, 7, 0, 0.05, 0.1, None, P, P, 0) == L.DMK_EUNSUPPORTED
    assert L.dmk_residual_eval_sorted(g, b, 0, 0, 0.05, 0.1, None, 0, P, 0) == L.DMK_EINVAL
    assert L.dmk_residual_eval_sorted(g, b, 0, 0, 0.05, 0.1, None, P, 0, 0) == L.DMK_EINVAL
    assert L.dmk_residual_backward_sorted(g, b, 1, 1, 0.05, 0.1, None, P, 0, P, P, 0) == L.DMK_EINVAL
    assert L.dmk_residual_backward_sorted(g, b, 1, 1, 0.05, 0.1, None, P, P, 0, P, 0) == L.DMK_EINVAL
    # with a PSWF window sigma is not used, the support rc still is
    w = L.dmk_pswf()
    assert L.dmk_pswf_window(14.5, w) == L.DMK_OK
    assert L.dmk_residual_eval_sorted(g, b, 0, 0, -1.0, 0.1, w, 0, P, 0) == L.DMK_EINVAL
    assert L.dmk_residual_eval_sorted(g, b, 0, 0, -1.0, 0.3, w, P, P, 0) == L.DMK_ECUTOFF
    assert L.dmk_residual_eval_sorted(g, b, 0, 0, 0.05, 0.1, L.dmk_pswf(), P, P, 0) == L.DMK_EUNSUPPORTED


def test_pswf_window_host_matches_oracle_window():
    # the library's host-side PSWF (its own eigen-solve and Chebyshev fit)
    # against the oracle's PSWF window, at many points of the support
    from numpy.polynomial import chebyshev as C
    from oracle.pswf import PswfWindow
    for c in (7.0, 14.5, 29.0, 40.0):
        w = L.dmk_pswf()
        assert L.dmk_pswf_window(c, w) == L.DMK_OK
        assert 1 <= w.nterms32 <= 24 and 1 <= w.nterms64 <= L.PSWF_MAXTERMS
        O = PswfWindow(c)
        t = np.linspace(1e-3, 1 - 1e-3, 997)
        u = 2 * t * t - 1
        cf = [np.array([w.cheb[q][k] for k in range(w.nterms64)]) for q in range(4)]
        np.testing.assert_allclose(C.chebval(u, cf[0]), O.phi_at(t), rtol=0, atol=1e-13)
        np.testing.assert_allclose(1 - t * C.chebval(u, cf[1]), O.Phi_at(t), rtol=0, atol=1e-13)
        np.testing.assert_allclose(t * C.chebval(u, cf[2]), O.dphi_at(t), rtol=0, atol=2e-14 * c)
        np.testing.assert_allclose(C.chebval(u, cf[3]), O.d2phi_at(t), rtol=0, atol=2e-14 * c * c)


def test_pswf_window_argument_errors():
    w = L.dmk_pswf()
    assert L.dmk_pswf_window(0.0, w) == L.DMK_EUNSUPPORTED
    assert L.dmk_pswf_window(41.0, w) == L.DMK_EUNSUPPORTED
    assert L.dmk_pswf_window(float("nan"), w) == L.DMK_EUNSUPPORTED
    g = L.make_grid((1, 1, 1), 3, (8, 8, 8))
    b = L.dmk_bins()
    P = 1 << 40
    bad = L.dmk_pswf()  # c = 0: not a window
    assert L.dmk_residual_eval_pswf(g, b, 0, 0, bad, 0.1, P, P, P, 1 << 30, 0) == L.DMK_EUNSUPPORTED


def test_far3p_host_argument_checks():
    fg = L.make_far_grid((1, 1, 1), (1, 1, 1), 8, (2, 2, 2))
    nb = L.dmk_far3p_ws_bytes(fg, 1)
    assert nb >= 16 * (3 * 8 * 5) and nb % 256 == 0
    fake = 1 << 40  # never dereferenced: every check below fails before a launch
    assert L.dmk_far3p_eval(fg, 1, 1.0, None, fake, fake, fake, nb - 1, 0) == L.DMK_ESIZE
    assert L.dmk_far3p_eval(fg, 1, 0.0, None, fake, fake, fake, nb, 0) == L.DMK_ECUTOFF
    assert L.dmk_far3p_eval(fg, 4, 1.0, None, fake, fake, fake, nb, 0) == L.DMK_EINVAL
    assert L.dmk_far3p_eval(fg, 1, 1.0, None, 0, fake, fake, nb, 0) == L.DMK_EINVAL
    bad = L.dmk_pswf()  # c = 0: not a window
    assert L.dmk_far3p_eval(fg, 1, 1.0, bad, fake, fake, fake, nb, 0) == L.DMK_EUNSUPPORTED
    # the largest mode ranges on every axis: more wave numbers than one launch covers
    huge = L.make_far_grid((1, 1, 1), (1, 1, 1), 2, (L.FAR_KMAX,) * 3)
    assert L.dmk_far3p_eval(huge, 0, 1.0, None, fake, fake, fake, 1 << 62, 0) == L.DMK_ESIZE
    # 6.8e7 wave numbers with n_i >= 0 (a wavefront each: 4.4e9 work-items in
    # one launch), though only 5.4e8 in all
    wide = L.make_far_grid((1, 1, 1), (1, 1, 1), 2, (1024, 1024, 64))
    assert L.dmk_far3p_eval(wide, 0, 1.0, None, fake, fake, fake, 1 << 62, 0) == L.DMK_ESIZE
    # cubes of the shortest side covering the cell, the last cut by its face
    for Lv, M in (((1, 1, 1.5), (1, 1, 2)), ((1.25, 1, 2.6), (2, 1, 3)), ((2, 3.5, 2), (1, 2, 1))):
        assert L.dmk_far3p_ws_bytes(L.make_far_grid(Lv, M, 8, (2, 2, 2)), 0) > 0
    for args in [((1, 1, 1), (1, 1, 2), 8, (2, 2, 2)),      # cubes do not tile the cell
                 ((1, 1, 1.5), (1, 1, 1), 8, (2, 2, 2)),    # cubes do not cover it
                 ((1, 1, 1.5), (1, 1, 3), 8, (2, 2, 2)),    # more cubes than the cover
                 ((2, 3.5, 2), (1, 2, 2), 8, (2, 2, 2)),
                 ((1, 1, 1), (1, 1, 1), 0, (2, 2, 2)),      # p < 1
                 ((1, 1, 1), (1, 1, 1), L.FAR_PMAX + 1, (2, 2, 2)),
                 ((1, 1, 1), (1, 1, 1), 8, (2, -1, 2)),
                 ((1, 1, 1), (1, 1, 1), 8, (2, L.FAR_KMAX + 1, 2)),
                 ((0, 1, 1), (1, 1, 1), 8, (2, 2, 2))]:
        g = L.make_far_grid(*args)
        assert L.dmk_far3p_ws_bytes(g, 0) == 0
        assert L.dmk_far3p_eval(g, 0, 1.0, None, fake, fake, fake, 1 << 30, 0) == L.DMK_EINVAL


def test_cheb_and_self_term_host_argument_checks():
    g = L.make_grid((1, 1, 1), 3, (2, 2, 2))
    b = L.dmk_bins()
    nb = L.dmk_bins_bytes(g, 100)
    fake = 1 << 40  # never dereferenced: every check below fails before a launch
    assert L.dmk_bins_carve(g, 100, fake, nb, b) == L.DMK_OK
    ws = L.dmk_cheb_ws_bytes(b, 8)
    assert ws >= 100 * 3 * 8 * 8
    assert L.dmk_cheb_ws_bytes(b, 0) == 0 and L.dmk_cheb_ws_bytes(b, L.FAR_PMAX + 1) == 0
    assert L.dmk_cheb_anterp(g, b, 8, 1, fake, fake, fake, ws - 1, 0) == L.DMK_ESIZE
    assert L.dmk_cheb_anterp(g, b, 8, 2, fake, fake, fake, ws, 0) == L.DMK_EINVAL
    assert L.dmk_cheb_eval(g, b, 8, 3, fake, 0, fake, fake, ws - 1, 0) == L.DMK_ESIZE
    assert L.dmk_cheb_eval(g, b, 0, 3, fake, 0, fake, fake, ws, 0) == L.DMK_EINVAL
    other = L.make_grid((1, 1, 1), 3, (3, 2, 2))  # bins of another tiling
    assert L.dmk_cheb_eval(other, b, 8, 1, fake, 0, fake, fake, ws, 0) == L.DMK_EINVAL
    assert L.dmk_self_term(4, 1.0, None, 10, fake, fake, 0) == L.DMK_EINVAL
    assert L.dmk_self_term(0, 0.0, None, 10, fake, fake, 0) == L.DMK_ECUTOFF
    assert L.dmk_self_term(0, 1.0, L.dmk_pswf(), 10, fake, fake, 0) == L.DMK_EUNSUPPORTED
    assert L.dmk_self_term(0, 1.0, None, 10, 0, fake, 0) == L.DMK_EINVAL
    assert L.dmk_self_term(2, 1.0, None, 10, 0, 0, 0) == L.DMK_OK  # stresslet: nothing to add
