"""PSWF window of the kernel split (test infrastructure only; see the oracle
package docstring for who may import it).

The zeroth-order prolate spheroidal wave function psi_0^c is the leading
eigenfunction of the band-limited Fourier transform on [-1, 1] (Sec. 2.2,
eq. (PSWFeig)).  It is also the eigenfunction of the smallest eigenvalue chi
of the prolate differential operator

    -((1 - x^2) psi')' + c^2 x^2 psi = chi psi ,

which commutes with that transform.  In the orthonormal Legendre basis
Pn_k = sqrt(k + 1/2) P_k the operator is a symmetric tridiagonal matrix that
couples k with k +- 2 (the Legendre three-term recurrence applied twice to
x^2 P_k); psi_0^c is even, so only even k appear.  Its eigenvector is found
with a dense symmetric eigen-solver (a library step).

The window is phi(x) = psi_0^c(x) / int_{-1}^{1} psi_0^c, supported on
|x| <= 1 (eq. (wfunc_pswf)), and Phi(r) = 1 - 2 int_0^r phi (eq.
(def_erfc_like_fcn)); both vanish for r >= 1 (remark on compact support).
Everything is kept as Legendre series so that the C oracle can evaluate
phi, Phi, phi' and phi'' in long double at any point.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import legendre as npleg


def pswf_legendre(c: float, nterms: int | None = None) -> np.ndarray:
    """Standard-Legendre coefficients a_k (P_k, not normalised) of psi_0^c,
    scaled so that psi_0^c(0) > 0; the overall scale is arbitrary."""
    c = float(c)
    if nterms is None:
        nterms = int(c) + 40          # even terms kept; the series decays super-exponentially past ~c
    k = 2.0 * np.arange(nterms)
    # x^2 P_k = A_k P_{k+2} + B_k P_k + C_k P_{k-2}
    B = (k + 1) ** 2 / ((2 * k + 1) * (2 * k + 3)) + np.where(k > 0, k ** 2 / ((2 * k + 1) * (2 * k - 1)), 0.0)
    diag = k * (k + 1) + c * c * B
    kk = k[:-1]
    off = c * c * (kk + 1) * (kk + 2) / ((2 * kk + 3) * np.sqrt((2 * kk + 1) * (2 * kk + 5)))
    A = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    w, V = np.linalg.eigh(A)
    v = V[:, 0]                                   # smallest chi: psi_0
    a = np.zeros(2 * nterms)
    a[0::2] = v * np.sqrt(k + 0.5)                # orthonormal -> standard Legendre
    if npleg.legval(0.0, a) < 0:
        a = -a
    return a


class PswfWindow:
    """Window phi, Phi, phi', phi'' of the PSWF split with bandwidth c, as
    Legendre series on [-1, 1] (functions of t = r / nu)."""

    def __init__(self, c: float):
        self.c = float(c)
        a = pswf_legendre(c)
        self.psi = a
        # int_{-1}^{1} P_k = 2 delta_k0
        self.phi = a / (2.0 * a[0])
        self.integral = npleg.legint(self.phi, m=1, lbnd=0)   # int_0^t phi
        self.dphi = npleg.legder(self.phi, 1)
        self.d2phi = npleg.legder(self.phi, 2)

    # evaluation (float64; zero outside the support)
    def _ev(self, coef, t):
        t = np.asarray(t, dtype=np.float64)
        return np.where(np.abs(t) < 1.0, npleg.legval(t, coef), 0.0)

    def phi_at(self, t):
        return self._ev(self.phi, t)

    def Phi_at(self, t):
        t = np.asarray(t, dtype=np.float64)
        return np.where(np.abs(t) < 1.0, 1.0 - 2.0 * npleg.legval(t, self.integral), 0.0)

    def dphi_at(self, t):
        return self._ev(self.dphi, t)

    def d2phi_at(self, t):
        return self._ev(self.d2phi, t)

    def psi_at(self, x):
        return npleg.legval(np.asarray(x, dtype=np.float64), self.psi)

    def fourier(self, q, nquad: int = 200):
        """phihat(q) = int_{-1}^{1} phi(s) e^{i q s} ds and its q-derivative, by
        Gauss-Legendre quadrature of the (even) window."""
        s, wq = npleg.leggauss(nquad)
        q = np.asarray(q, dtype=np.float64)[..., None]
        f = npleg.legval(s, self.phi)
        ph = np.sum(wq * f * np.cos(q * s), axis=-1)
        dph = -np.sum(wq * f * s * np.sin(q * s), axis=-1)
        return ph, dph

    def packed(self, nquad: int = 200):
        """Arrays handed to the C oracle: the four Legendre series (padded to a
        common length n) and quadrature nodes, weights and phi values on [0, 1]
        for its Fourier transforms."""
        n = max(len(self.phi), len(self.integral), len(self.dphi), len(self.d2phi))
        ser = np.zeros((4, n))
        for i, c_ in enumerate((self.phi, self.integral, self.dphi, self.d2phi)):
            ser[i, :len(c_)] = c_
        s, wq = npleg.leggauss(nquad)
        return n, ser, s, wq, npleg.legval(s, self.phi)
