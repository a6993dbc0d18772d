// dmk_pswf.cpp -- host-side construction of the PSWF window of the kernel
// split (Sec. 2.2, eqs. (PSWFeig), (wfunc_pswf)) as short Chebyshev series
// that the residual kernels evaluate per pair.
//
// psi_0^c is the eigenfunction of the smallest eigenvalue of the prolate
// operator -((1-x^2) psi')' + c^2 x^2 psi, which commutes with the
// band-limited Fourier transform on [-1, 1].  On even orthonormal Legendre
// polynomials the operator is a symmetric tridiagonal matrix (x^2 couples
// degree k with k +- 2).  Its smallest eigenvalue is bracketed by bisection
// on Sturm sequence counts and the eigenvector found by inverse iteration.
//
// The window phi = psi / int psi lives on |t| < 1, t = r / nu; with
// Phi = 1 - 2 int_0^t phi the residual kernels need phi, Phi, phi' and phi''.
// In u = 2 t^2 - 1 the even functions phi, (1 - Phi)/t, phi'/t and phi'' are
// smooth on [-1, 1]; each is interpolated at Chebyshev points of u.
#include <math.h>
#include <string.h>

#include <vector>

#include "../../include/dmk.h"

namespace {

// number of eigenvalues of the symmetric tridiagonal (d, e) below x
int sturm_count(const std::vector<double> &d, const std::vector<double> &e, double x)
{
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < d.size(); ++i) {
        const double e2 = i > 0 ? e[i - 1] * e[i - 1] : 0.0;
        q = d[i] - x - (i > 0 ? e2 / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// solve (T - s I) y = b for tridiagonal T = (d, e), Gaussian elimination with
// partial pivoting (one extra super-diagonal of fill)
void tridiag_solve(const std::vector<double> &d, const std::vector<double> &e, double s, std::vector<double> &b)
{
    const int n = (int)d.size();
    std::vector<double> a0(n), a1(n), a2(n), sub(n);  // rows: diag, super, super2; sub-diagonal
    for (int i = 0; i < n; ++i) {
        a0[i] = d[i] - s;
        a1[i] = i + 1 < n ? e[i] : 0.0;
        a2[i] = 0.0;
        sub[i] = i > 0 ? e[i - 1] : 0.0;
    }
    for (int i = 0; i + 1 < n; ++i) {
        // candidate pivot rows i (a0[i], a1[i], a2[i]) and i+1 (sub[i+1], a0[i+1], a1[i+1])
        if (fabs(sub[i + 1]) > fabs(a0[i])) {
            double t0 = a0[i], t1 = a1[i], t2 = a2[i], tb = b[i];
            a0[i] = sub[i + 1];
            a1[i] = a0[i + 1];
            a2[i] = a1[i + 1];
            b[i] = b[i + 1];
            sub[i + 1] = t0;
            a0[i + 1] = t1;
            a1[i + 1] = t2;
            b[i + 1] = tb;
        }
        if (a0[i] == 0.0) a0[i] = 1e-300;
        const double m = sub[i + 1] / a0[i];
        a0[i + 1] -= m * a1[i];
        a1[i + 1] -= m * a2[i];
        b[i + 1] -= m * b[i];
    }
    if (a0[n - 1] == 0.0) a0[n - 1] = 1e-300;
    for (int i = n - 1; i >= 0; --i) {
        double v = b[i];
        if (i + 1 < n) v -= a1[i] * b[i + 1];
        if (i + 2 < n) v -= a2[i] * b[i + 2];
        b[i] = v / a0[i];
    }
}

}  // namespace

extern "C" int dmk_pswf_window(double c, dmk_pswf *w)
{
    if (!w) return DMK_EINVAL;
    if (!(c > 0.0) || !(c <= DMK_PSWF_CMAX)) return DMK_EUNSUPPORTED;
    memset(w, 0, sizeof(*w));
    w->c = c;

    // even orthonormal Legendre basis Pn_k = sqrt(k + 1/2) P_k, k = 2i
    const int M = (int)c + 40;
    std::vector<double> d(M), e(M > 1 ? M - 1 : 1);
    for (int i = 0; i < M; ++i) {
        const double k = 2.0 * i;
        // x^2 P_k = A P_{k+2} + B P_k + C P_{k-2}, three-term recurrence twice
        double B = (k + 1) * (k + 1) / ((2 * k + 1) * (2 * k + 3));
        if (i > 0) B += k * k / ((2 * k + 1) * (2 * k - 1));
        d[i] = k * (k + 1) + c * c * B;
        if (i + 1 < M) e[i] = c * c * (k + 1) * (k + 2) / ((2 * k + 3) * sqrt((2 * k + 1) * (2 * k + 5)));
    }
    // smallest eigenvalue: Gershgorin bracket, then bisection on Sturm counts
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < M; ++i) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < M ? fabs(e[i]) : 0.0);
        lo = fmin(lo, d[i] - r);
        hi = fmax(hi, d[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(1.0, fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(d, e, mid) >= 1)
            hi = mid;
        else
            lo = mid;
    }
    const double chi = 0.5 * (lo + hi);
    // inverse iteration from a flat start
    std::vector<double> v(M, 1.0);
    for (int it = 0; it < 4; ++it) {
        tridiag_solve(d, e, chi - 1e-10 * fmax(1.0, fabs(chi)), v);
        double nrm = 0.0;
        for (int i = 0; i < M; ++i) nrm += v[i] * v[i];
        nrm = sqrt(nrm);
        for (int i = 0; i < M; ++i) v[i] /= nrm;
    }
    // standard Legendre coefficients of psi (degree 2i), phi = psi / int psi,
    // int_{-1}^{1} P_k = 2 delta_k0
    const int K = 2 * M + 2;  // degrees 0 .. K-1
    std::vector<double> a(K, 0.0);
    for (int i = 0; i < M; ++i) a[2 * i] = v[i] * sqrt(2.0 * i + 0.5);
    const double a0 = a[0];
    if (!(fabs(a0) > 0.0)) return DMK_EUNSUPPORTED;
    for (int k = 0; k < K; ++k) a[k] /= 2.0 * a0;  // psi(0) > 0 follows from int psi > 0

    // the four functions at Chebyshev points of u = 2 t^2 - 1
    const int NP = 2 * DMK_PSWF_MAXTERMS;
    std::vector<double> f[4];
    for (int q = 0; q < 4; ++q) f[q].assign(NP, 0.0);
    std::vector<double> P(K + 1), dP(K + 1), d2P(K + 1);
    for (int j = 0; j < NP; ++j) {
        const double u = cos(M_PI * (j + 0.5) / NP);
        const double t = sqrt(0.5 * (u + 1.0));
        P[0] = 1.0;
        P[1] = t;
        dP[0] = 0.0;
        dP[1] = 1.0;
        d2P[0] = 0.0;
        d2P[1] = 0.0;
        for (int k = 1; k < K; ++k) {
            P[k + 1] = ((2.0 * k + 1.0) * t * P[k] - k * P[k - 1]) / (k + 1.0);
            dP[k + 1] = dP[k - 1] + (2.0 * k + 1.0) * P[k];
            d2P[k + 1] = d2P[k - 1] + (2.0 * k + 1.0) * dP[k];
        }
        double phi = 0.0, I = 0.0, dphi = 0.0, d2phi = 0.0;
        for (int k = 0; k < K; k += 2) {
            if (a[k] == 0.0) continue;
            phi += a[k] * P[k];
            dphi += a[k] * dP[k];
            d2phi += a[k] * d2P[k];
            // int_0^t P_k = (P_{k+1} - P_{k-1}) / (2k + 1), int_0^t P_0 = t
            I += a[k] * (k == 0 ? t : (P[k + 1] - P[k - 1]) / (2.0 * k + 1.0));
        }
        f[0][j] = phi;
        f[1][j] = 2.0 * I / t;  // (1 - Phi) / t
        f[2][j] = dphi / t;
        f[3][j] = d2phi;
    }
    // Chebyshev coefficients (discrete cosine transform of the point values)
    for (int q = 0; q < 4; ++q)
        for (int m = 0; m < DMK_PSWF_MAXTERMS; ++m) {
            double s = 0.0;
            for (int j = 0; j < NP; ++j) s += f[q][j] * cos(M_PI * m * (j + 0.5) / NP);
            w->cheb[q][m] = (m == 0 ? 1.0 : 2.0) * s / NP;
        }
    // terms kept: the tail below the precision of each path
    for (int pass = 0; pass < 2; ++pass) {
        // (the FP64 threshold sits just above the rounding floor of the fit)
        const double tol = pass == 0 ? 5e-14 : 2e-9;
        int n = 1;
        for (int q = 0; q < 4; ++q) {
            double sc = 0.0;
            for (int m = 0; m < DMK_PSWF_MAXTERMS; ++m) sc = fmax(sc, fabs(w->cheb[q][m]));
            for (int m = 0; m < DMK_PSWF_MAXTERMS; ++m)
                if (fabs(w->cheb[q][m]) > tol * sc && m + 1 > n) n = m + 1;
        }
        if (pass == 0)
            w->nterms64 = n;
        else
            w->nterms32 = n;
    }
    if (w->nterms32 > DMK_PSWF_MAXTERMS32) return DMK_EUNSUPPORTED;
    return DMK_OK;
}
