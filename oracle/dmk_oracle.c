/*
 * dmk_oracle.c -- plain, slow CPU oracle for the residual (short-range) part
 * of the periodic kernel sums in "Fast summation on rectangular cuboids with
 * arbitrary periodicity in the DMK framework" (Krantz, af Klinteberg,
 * Tornberg).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU library; both only see the same seeded
 * input arrays.
 *
 * Inputs are FP64; every pair term and every accumulation is done in long
 * double (x87 80-bit) so that the oracle is at least as accurate as FP64.
 *
 * What is computed (all brute force, no cell lists, no sorting):
 *
 *  oracle_residual       Mode R.  u_b = sum_a sum_{p in P_D}^* [0<|d|<rc] K_R(d) rho_a
 *                        with d = x_b - x_a + p  (eq. (u_local), Sec. 2.3, with
 *                        the image set P_D of eq. (periodic-images), Sec. 1).
 *  oracle_residual_vjp   Analytic vector-Jacobian product of mode R
 *                        (gradients w.r.t. positions and strengths).
 *  oracle_direct_free    D = 0 direct sum of the ORIGINAL kernels (App. B
 *                        eqs. (stokeslet_def_deriv)-(rotlet_def_deriv),
 *                        H = 1/(4 pi r) from eq. (ewald-split)); optional cutoff.
 *  oracle_full_split_3p  Mode F for D = 3: residual part over all images with a
 *                        generous real-space cutoff + Fourier part of the
 *                        mollified kernel over k != 0 (eq. (ewald_far_3P),
 *                        structure factor eq. (structurefacgen)) + the
 *                        self-interaction correction (Sec. 2.4, App. B).
 *  oracle_far_3p         The far-field part alone (eq. (ewald_far_3P)) from
 *                        given sources to given targets, over the cube of
 *                        wave numbers |kbar_i| <= K_i, kbar != 0 (eqs.
 *                        (wavenumbers-3p-trunc), (kintmax)); used with the
 *                        root-level Chebyshev grids as sources and targets.
 *
 * Kernel ids: 0 Laplace (harmonic), 1 Stokeslet, 2 stresslet, 3 rotlet.
 * Strength sizes m_in = 1, 3, 9, 3; potential sizes m_out = 1, 3, 3, 3.
 * Stresslet strengths are row-major rho[l*3+m] and u_j = T_jlm rho_lm.
 *
 * Window (Sec. 2.2), selected with oracle_set_window:
 *  - the Gaussian (default), phi(t) = exp(-t^2)/sqrt(pi), whose Fourier
 *    transform is exp(-k^2/4) (remark after eq. (Hhatsplit_wfunc)); then
 *    Phi(t) = 1 - 2 int_0^t phi = erfc(t)  (eq. (def_erfc_like_fcn));
 *  - the PSWF window of eq. (wfunc_pswf), supported on |t| < 1, given as
 *    Legendre series of phi, int_0^t phi, phi' and phi'' (computed by the
 *    Python side of the oracle from its own eigen-solve), with quadrature
 *    nodes for its Fourier transform.
 * All real-space functions are evaluated at t = r/sigma, sigma being the
 * split length (nu for the PSWF window; remark scaling_stokes_split, App. B).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <complex.h>

#define PI_L 3.141592653589793238462643383279502884L

/* ------------------------------------------------------------------------ */
/* window and its integral (Sec. 2.2)                                       */
#define WIN_MAXN 256
#define WIN_MAXQ 512
static int g_win = 0;                      /* 0 Gaussian, 1 Legendre-series window on |t| < 1 */
static int g_win_n = 0;
static long double g_win_ser[4][WIN_MAXN]; /* phi, int_0^t phi, phi', phi'' */
static int g_win_nq = 0;
static long double g_win_qs[WIN_MAXQ], g_win_qw[WIN_MAXQ], g_win_qf[WIN_MAXQ];

/* sum_k a_k P_k(t), Legendre polynomials by their three-term recurrence */
static long double leg_sum(const long double *a, int n, long double t)
{
    long double p0 = 1.0L, p1 = t, s = a[0];
    if (n > 1) s += a[1] * t;
    for (int k = 1; k + 1 < n; k++) {
        const long double p2 = ((2.0L * k + 1.0L) * t * p1 - (long double)k * p0) / (long double)(k + 1);
        s += a[k + 1] * p2;
        p0 = p1;
        p1 = p2;
    }
    return s;
}

static long double win_phi(long double t)
{
    if (g_win == 0) return expl(-t * t) / sqrtl(PI_L);
    return fabsl(t) < 1.0L ? leg_sum(g_win_ser[0], g_win_n, t) : 0.0L;
}
static long double win_Phi(long double t)
{
    if (g_win == 0) return erfcl(t);
    return fabsl(t) < 1.0L ? 1.0L - 2.0L * leg_sum(g_win_ser[1], g_win_n, t) : 0.0L;
}
static long double win_dphi(long double t)
{
    if (g_win == 0) return -2.0L * t * win_phi(t);
    return fabsl(t) < 1.0L ? leg_sum(g_win_ser[2], g_win_n, t) : 0.0L;
}
static long double win_ddphi(long double t)
{
    if (g_win == 0) return (4.0L * t * t - 2.0L) * win_phi(t);
    return fabsl(t) < 1.0L ? leg_sum(g_win_ser[3], g_win_n, t) : 0.0L;
}
/* phihat(q) = int phi(s) e^{iqs} ds and d phihat / dq */
static void win_hat(long double q, long double *ph, long double *dph)
{
    if (g_win == 0) {
        *ph = expl(-q * q / 4.0L);
        *dph = -(q / 2.0L) * *ph;
        return;
    }
    long double a = 0.0L, b = 0.0L;
    for (int i = 0; i < g_win_nq; i++) {
        a += g_win_qw[i] * g_win_qf[i] * cosl(q * g_win_qs[i]);
        b -= g_win_qw[i] * g_win_qf[i] * g_win_qs[i] * sinl(q * g_win_qs[i]);
    }
    *ph = a;
    *dph = b;
}

/* Select the window: type 0 Gaussian; type 1 Legendre-series window with
 * ser[4][n] (row-major) and nq quadrature nodes qs / weights qw / phi values
 * qf on [-1, 1].  Not thread-safe; set before a computation. */
int oracle_set_window(int type, int n, const double *ser, int nq, const double *qs, const double *qw,
                      const double *qf)
{
    if (type == 0) {
        g_win = 0;
        return 0;
    }
    if (type != 1 || n < 1 || n > WIN_MAXN || nq < 1 || nq > WIN_MAXQ) return 1;
    for (int i = 0; i < 4; i++)
        for (int k = 0; k < n; k++) g_win_ser[i][k] = ser[i * n + k];
    for (int i = 0; i < nq; i++) {
        g_win_qs[i] = qs[i];
        g_win_qw[i] = qw[i];
        g_win_qf[i] = qf[i];
    }
    g_win_n = n;
    g_win_nq = nq;
    g_win = 1;
    return 0;
}

static int m_in_of(int k) { return k == 0 ? 1 : (k == 2 ? 9 : 3); }
static int m_out_of(int k) { return k == 0 ? 1 : 3; }

static long double levi(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0.0L;
    /* even permutations of (0,1,2) */
    if ((a == 0 && b == 1 && c == 2) || (a == 1 && b == 2 && c == 0) || (a == 2 && b == 0 && c == 1))
        return 1.0L;
    return -1.0L;
}

/*
 * Residual kernel tensor K[j][L] (j < m_out, L < m_in) at displacement d, and
 * optionally its derivative dK[k][j][L] = d K[j][L] / d d_k.
 *
 *  Laplace   K = Phi(t)/(4 pi r)                          eq. (Hhatsplit_wfunc)
 *  Stokeslet K_jl = Sd(t) delta_jl/(8 pi r) + So(t) d_j d_l/(8 pi r^3)
 *            Sd = Phi - 2 t phi,  So = Phi + 2 t phi      eqs. (res_stokeslet),(Soffdiag)
 *  Stresslet K_j(lm) = (delta_jl d_m + delta_lm d_j + delta_mj d_l) Td(t)/(8 pi r^3)
 *                      - 3/(4 pi) d_j d_l d_m To(t)/r^5
 *            Td = -2 t^2 phi',  To = Phi + 2 t phi - (2/3) t^2 phi'
 *                                                          eqs. (res_stresslet),(T-offd)
 *  Rotlet    K_jl = eps_jlm d_m Oo(t)/(8 pi r^3), Oo = Phi + 2 t phi
 *                                                          eqs. (res_rotlet),(ROoffd)
 *
 * The derivative follows from the product rule: every term is a radial factor
 * a(r) times a polynomial in d, and d a/d d_k = a'(r) d_k / r with
 * a'(r) = (da/dt)/sigma (explicit partials below).
 */
static void kernel_tensor(int kern, const long double d[3], long double sigma,
                          long double K[3][9], long double dK[3][3][9])
{
    const long double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const long double r = sqrtl(r2);
    const long double t = r / sigma;
    const long double Ph = win_Phi(t), ph = win_phi(t), dph = win_dphi(t), ddph = win_ddphi(t);
    /* d/dt of Phi, phi */
    const long double dPh = -2.0L * ph;
    int j, l, m, k;
    memset(K, 0, sizeof(long double) * 3 * 9);
    if (dK) memset(dK, 0, sizeof(long double) * 3 * 3 * 9);

    if (kern == 0) {
        /* a(r) = Phi(r/sigma) / (4 pi r) */
        long double a = Ph / (4.0L * PI_L * r);
        long double da = (dPh / sigma) / (4.0L * PI_L * r) - Ph / (4.0L * PI_L * r2);
        K[0][0] = a;
        if (dK)
            for (k = 0; k < 3; k++) dK[k][0][0] = da * d[k] / r;
    } else if (kern == 1) {
        long double Sd = Ph - 2.0L * t * ph;
        long double So = Ph + 2.0L * t * ph;
        long double dSd = dPh - 2.0L * ph - 2.0L * t * dph;   /* d/dt */
        long double dSo = dPh + 2.0L * ph + 2.0L * t * dph;
        long double A = Sd / (8.0L * PI_L * r);
        long double B = So / (8.0L * PI_L * r * r2);
        long double dA = (dSd / sigma) / (8.0L * PI_L * r) - Sd / (8.0L * PI_L * r2);
        long double dB = (dSo / sigma) / (8.0L * PI_L * r * r2) - 3.0L * So / (8.0L * PI_L * r2 * r2);
        for (j = 0; j < 3; j++)
            for (l = 0; l < 3; l++) {
                K[j][l] = A * (j == l) + B * d[j] * d[l];
                if (dK)
                    for (k = 0; k < 3; k++)
                        dK[k][j][l] = dA * d[k] / r * (j == l) + dB * d[k] / r * d[j] * d[l] +
                                      B * ((j == k) * d[l] + d[j] * (l == k));
            }
    } else if (kern == 2) {
        long double Td = -2.0L * t * t * dph;
        long double To = Ph + 2.0L * t * ph - (2.0L / 3.0L) * t * t * dph;
        long double dTd = -4.0L * t * dph - 2.0L * t * t * ddph;
        long double dTo = dPh + 2.0L * ph + 2.0L * t * dph - (4.0L / 3.0L) * t * dph - (2.0L / 3.0L) * t * t * ddph;
        long double P = Td / (8.0L * PI_L * r * r2);
        long double Q = -3.0L / (4.0L * PI_L) * To / (r2 * r2 * r);
        long double dP = (dTd / sigma) / (8.0L * PI_L * r * r2) - 3.0L * Td / (8.0L * PI_L * r2 * r2);
        long double dQ = -3.0L / (4.0L * PI_L) * ((dTo / sigma) / (r2 * r2 * r) - 5.0L * To / (r2 * r2 * r2));
        for (j = 0; j < 3; j++)
            for (l = 0; l < 3; l++)
                for (m = 0; m < 3; m++) {
                    long double poly = (j == l) * d[m] + (l == m) * d[j] + (m == j) * d[l];
                    long double cub = d[j] * d[l] * d[m];
                    K[j][l * 3 + m] = P * poly + Q * cub;
                    if (dK)
                        for (k = 0; k < 3; k++) {
                            long double dpoly = (j == l) * (m == k) + (l == m) * (j == k) + (m == j) * (l == k);
                            long double dcub = (j == k) * d[l] * d[m] + d[j] * (l == k) * d[m] + d[j] * d[l] * (m == k);
                            dK[k][j][l * 3 + m] = dP * d[k] / r * poly + P * dpoly + dQ * d[k] / r * cub + Q * dcub;
                        }
                }
    } else {
        long double Oo = Ph + 2.0L * t * ph;
        long double dOo = dPh + 2.0L * ph + 2.0L * t * dph;
        long double f = Oo / (8.0L * PI_L * r * r2);
        long double df = (dOo / sigma) / (8.0L * PI_L * r * r2) - 3.0L * Oo / (8.0L * PI_L * r2 * r2);
        for (j = 0; j < 3; j++)
            for (l = 0; l < 3; l++) {
                long double s = 0.0L;
                for (m = 0; m < 3; m++) s += levi(j, l, m) * d[m];
                K[j][l] = f * s;
                if (dK)
                    for (k = 0; k < 3; k++) dK[k][j][l] = df * d[k] / r * s + f * levi(j, l, k);
            }
    }
}

/* Original (unsplit) kernels, App. B eqs. (stokeslet_def_deriv)-(rotlet_def_deriv)
 * and H = 1/(4 pi r) from eq. (ewald-split). */
static void kernel_free_tensor(int kern, const long double d[3], long double K[3][9])
{
    const long double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    const long double r = sqrtl(r2);
    int j, l, m;
    memset(K, 0, sizeof(long double) * 3 * 9);
    if (kern == 0) {
        K[0][0] = 1.0L / (4.0L * PI_L * r);
    } else if (kern == 1) {
        for (j = 0; j < 3; j++)
            for (l = 0; l < 3; l++) K[j][l] = ((j == l) / r + d[j] * d[l] / (r * r2)) / (8.0L * PI_L);
    } else if (kern == 2) {
        for (j = 0; j < 3; j++)
            for (l = 0; l < 3; l++)
                for (m = 0; m < 3; m++) K[j][l * 3 + m] = -3.0L / (4.0L * PI_L) * d[j] * d[l] * d[m] / (r2 * r2 * r);
    } else {
        for (j = 0; j < 3; j++)
            for (l = 0; l < 3; l++) {
                long double s = 0.0L;
                for (m = 0; m < 3; m++) s += levi(j, l, m) * d[m];
                K[j][l] = s / (8.0L * PI_L * r * r2);
            }
    }
}

/* ------------------------------------------------------------------------ */
/* image enumeration for P_D (eq. (periodic-images)): the first D axes are    */
/* periodic.  For a displacement component dd along a periodic axis, the     */
/* images n with |dd + n L| < rc are n in [ceil((-rc-dd)/L), floor((rc-dd)/L)].*/
static void image_range(int axis, int D, const double L[3], long double dd, long double rc,
                        long n_lo_hi[2])
{
    if (axis >= D) {
        n_lo_hi[0] = 0;
        n_lo_hi[1] = 0;
        return;
    }
    n_lo_hi[0] = (long)ceill((-rc - dd) / (long double)L[axis]);
    n_lo_hi[1] = (long)floorl((rc - dd) / (long double)L[axis]);
}

static int check_common(int kern, int D, const double L[3], double sigma, double rc, int64_t N)
{
    if (kern < 0 || kern > 3) return 1;
    if (D < 0 || D > 3) return 1;
    if (!(sigma > 0.0) || !(rc > 0.0) || N < 0) return 1;
    for (int i = 0; i < 3; i++)
        if (!(L[i] > 0.0)) return 1;
    return 0;
}

/*
 * Mode R: residual sum over every source and every image inside the cutoff.
 *   u[b] = sum_a sum_{p in P_D, 0 < |d| < rc} K_R(d) rho_a,  d = x_tb - x_a + p.
 * Targets are the points tgt[0..ntgt) (indices into x), or all points when
 * tgt == NULL (then ntgt must equal N).  The term with |d| == 0 is the one the
 * star in eq. (periodic_sum) removes.
 */
int oracle_residual(int kern, int D, const double L[3], double sigma, double rc, int64_t N,
                    const double *x, const double *rho, int64_t ntgt, const int64_t *tgt,
                    double *u)
{
    if (check_common(kern, D, L, sigma, rc, N)) return 1;
    const int mi = m_in_of(kern), mo = m_out_of(kern);
    const long double rcl = rc;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ib = 0; ib < ntgt; ib++) {
        const int64_t b = tgt ? tgt[ib] : ib;
        long double acc[3] = {0.0L, 0.0L, 0.0L};
        long double K[3][9];
        for (int64_t a = 0; a < N; a++) {
            long double d0[3];
            long rng[3][2];
            int i;
            for (i = 0; i < 3; i++) {
                d0[i] = (long double)x[3 * b + i] - (long double)x[3 * a + i];
                image_range(i, D, L, d0[i], rcl, rng[i]);
            }
            for (long n0 = rng[0][0]; n0 <= rng[0][1]; n0++)
                for (long n1 = rng[1][0]; n1 <= rng[1][1]; n1++)
                    for (long n2 = rng[2][0]; n2 <= rng[2][1]; n2++) {
                        long double d[3] = {d0[0] + n0 * (long double)L[0], d0[1] + n1 * (long double)L[1],
                                            d0[2] + n2 * (long double)L[2]};
                        long double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (!(r2 > 0.0L) || !(r2 < rcl * rcl)) continue;
                        kernel_tensor(kern, d, sigma, K, NULL);
                        for (int j = 0; j < mo; j++)
                            for (int q = 0; q < mi; q++) acc[j] += K[j][q] * (long double)rho[mi * a + q];
                    }
        }
        for (int j = 0; j < mo; j++) u[mo * ib + j] = (double)acc[j];
    }
    return 0;
}

/*
 * Vector-Jacobian product of mode R with cotangent G[N][m_out] (sources are
 * the targets, so every point is both).  With F = sum_b G_b . u_b:
 *   dF/drho_c = sum_b sum_p K(x_b - x_c + p)^T G_b
 *   dF/dx_c   = sum_a sum_p dK(x_c - x_a + p)[G_c, rho_a]
 *             - sum_b sum_p dK(x_b - x_c + p)[G_b, rho_c]
 * Both sums run over the same cutoff set (the mask is piecewise constant and
 * contributes nothing).  The oracle evaluates K and dK at the displacement it
 * needs, with no use of kernel parity.
 */
int oracle_residual_vjp(int kern, int D, const double L[3], double sigma, double rc, int64_t N,
                        const double *x, const double *rho, const double *G, int64_t ntgt,
                        const int64_t *tgt, double *grad_rho, double *grad_x)
{
    if (check_common(kern, D, L, sigma, rc, N)) return 1;
    const int mi = m_in_of(kern), mo = m_out_of(kern);
    const long double rcl = rc;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ic = 0; ic < ntgt; ic++) {
        const int64_t c = tgt ? tgt[ic] : ic;
        long double gr[9] = {0}, gx[3] = {0};
        long double K[3][9], dK[3][3][9];
        for (int64_t a = 0; a < N; a++) {
            long double d0[3];
            long rng[3][2];
            int i;
            for (i = 0; i < 3; i++) {
                d0[i] = (long double)x[3 * c + i] - (long double)x[3 * a + i];
                image_range(i, D, L, d0[i], rcl, rng[i]);
            }
            for (long n0 = rng[0][0]; n0 <= rng[0][1]; n0++)
                for (long n1 = rng[1][0]; n1 <= rng[1][1]; n1++)
                    for (long n2 = rng[2][0]; n2 <= rng[2][1]; n2++) {
                        /* e = x_c - x_a + p : c is the target, a the source */
                        long double e[3] = {d0[0] + n0 * (long double)L[0], d0[1] + n1 * (long double)L[1],
                                            d0[2] + n2 * (long double)L[2]};
                        long double r2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
                        if (!(r2 > 0.0L) || !(r2 < rcl * rcl)) continue;
                        /* term 1: c as target of source a */
                        kernel_tensor(kern, e, sigma, K, dK);
                        for (int k = 0; k < 3; k++)
                            for (int j = 0; j < mo; j++)
                                for (int q = 0; q < mi; q++)
                                    gx[k] += dK[k][j][q] * (long double)G[mo * c + j] * (long double)rho[mi * a + q];
                        /* c as source of target a, image -p: displacement
                         * x_a - x_c - p = -e */
                        long double me[3] = {-e[0], -e[1], -e[2]};
                        kernel_tensor(kern, me, sigma, K, dK);
                        for (int q = 0; q < mi; q++)
                            for (int j = 0; j < mo; j++) gr[q] += K[j][q] * (long double)G[mo * a + j];
                        /* d/dx_c of K(x_a - x_c - p) = -dK(-e) */
                        for (int k = 0; k < 3; k++)
                            for (int j = 0; j < mo; j++)
                                for (int q = 0; q < mi; q++)
                                    gx[k] -= dK[k][j][q] * (long double)G[mo * a + j] * (long double)rho[mi * c + q];
                    }
        }
        for (int q = 0; q < mi; q++) grad_rho[mi * ic + q] = (double)gr[q];
        for (int k = 0; k < 3; k++) grad_x[3 * ic + k] = (double)gx[k];
    }
    return 0;
}

/* D = 0 direct sum of the original kernels over all pairs with 0 < r < rc
 * (pass rc = INFINITY for the plain N-body sum). */
int oracle_direct_free(int kern, int64_t N, const double *x, const double *rho, double rc, int64_t ntgt,
                       const int64_t *tgt, double *u)
{
    if (kern < 0 || kern > 3 || N < 0) return 1;
    const int mi = m_in_of(kern), mo = m_out_of(kern);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t ib = 0; ib < ntgt; ib++) {
        const int64_t b = tgt ? tgt[ib] : ib;
        long double acc[3] = {0, 0, 0};
        long double K[3][9];
        for (int64_t a = 0; a < N; a++) {
            long double d[3];
            for (int i = 0; i < 3; i++) d[i] = (long double)x[3 * b + i] - (long double)x[3 * a + i];
            long double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 > 0.0L)) continue;
            if (isfinite(rc) && !(r2 < (long double)rc * (long double)rc)) continue;
            kernel_free_tensor(kern, d, K);
            for (int j = 0; j < mo; j++)
                for (int q = 0; q < mi; q++) acc[j] += K[j][q] * (long double)rho[mi * a + q];
        }
        for (int j = 0; j < mo; j++) u[mo * ib + j] = (double)acc[j];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Mode F, D = 3 (Ewald-type full split).                                     */
/*                                                                            */
/* Fourier transform of the mollified kernels (App. A convention            */
/* fhat(k) = int f(x) exp(-i k.x) dx):                                       */
/*   harmonic   Hhat_M = phihat(k sigma)/k^2,  phihat(q) = exp(-q^2/4)        */
/*              eqs. (Hhat_k), (Hhatsplit_wfunc)                            */
/*   biharmonic Bhat_M = gammaB(k sigma)/k^4, gammaB(q) = phihat - q phihat'/2 */
/*              eqs. (gammaB_in_phi), (Bmollhat)                            */
/*   Stokeslet  (k^2 delta_jl - k_j k_l) Bhat_M             eq. (moll_stokeslet)*/
/*   stresslet  i[(k_m d_jl + k_j d_lm + k_l d_mj) k^2 - 2 k_j k_l k_m] Bhat_M */
/*              eq. (moll_stresslet)                                         */
/*   rotlet     -(i/2) eps_jlm k_m Hhat_M                   eq. (moll_rotlet) */
/* Self term  -lim_{r->0} K_M rho_b = -phi(0) rho_b / (2 pi sigma) for the   */
/* harmonic kernel and the Stokeslet; 0 for stresslet and rotlet (Sec. 2.4,  */
/* eq. (S_self) and the remark on scaling, App. B).                          */
/* The stresslet's extra k = 0 compensation term of the paper's footnote in  */
/* Sec. 1 is NOT included (the paper does not state it).                    */
static void khat_tensor(int kern, const long double k[3], long double sigma,
                        long double complex Kh[3][9])
{
    const long double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const long double q = sqrtl(k2) * sigma;
    long double ph, dph;
    win_hat(q, &ph, &dph);
    const long double gB = ph - 0.5L * q * dph;
    const long double Hh = ph / k2;
    const long double Bh = gB / (k2 * k2);
    int j, l, m;
    for (j = 0; j < 3; j++)
        for (l = 0; l < 9; l++) Kh[j][l] = 0;
    if (kern == 0) {
        Kh[0][0] = Hh;
    } else if (kern == 1) {
        for (j = 0; j < 3; j++)
            for (l = 0; l < 3; l++) Kh[j][l] = (k2 * (j == l) - k[j] * k[l]) * Bh;
    } else if (kern == 2) {
        for (j = 0; j < 3; j++)
            for (l = 0; l < 3; l++)
                for (m = 0; m < 3; m++)
                    Kh[j][l * 3 + m] =
                        I * ((k[m] * (j == l) + k[j] * (l == m) + k[l] * (m == j)) * k2 -
                             2.0L * k[j] * k[l] * k[m]) * Bh;
    } else {
        for (j = 0; j < 3; j++)
            for (l = 0; l < 3; l++) {
                long double s = 0.0L;
                for (m = 0; m < 3; m++) s += levi(j, l, m) * k[m];
                Kh[j][l] = -0.5L * I * s * Hh;
            }
    }
}

/*
 * u = u_R (all images, |d| < rcut_real) + u_F (k != 0, |k| <= kmax) + u_self
 * for the triply periodic cell [0,L1)x[0,L2)x[0,L3).
 */
int oracle_full_split_3p(int kern, const double L[3], double sigma, int64_t N, const double *x,
                         const double *rho, double rcut_real, double kmax, int64_t ntgt,
                         const int64_t *tgt, double *u)
{
    if (check_common(kern, 3, L, sigma, rcut_real, N)) return 1;
    const int mi = m_in_of(kern), mo = m_out_of(kern);
    /* real-space part */
    double *ur = (double *)calloc((size_t)(ntgt > 0 ? ntgt : 1) * mo, sizeof(double));
    if (!ur) return 2;
    oracle_residual(kern, 3, L, sigma, rcut_real, N, x, rho, ntgt, tgt, ur);

    /* Fourier part: wave numbers 2 pi (n1/L1, n2/L2, n3/L3) (eq. (wavenumbers-3p)) */
    long nmax[3];
    for (int i = 0; i < 3; i++) nmax[i] = (long)ceil(kmax * L[i] / (2.0 * M_PI));
    const long double V = (long double)L[0] * L[1] * L[2];
    long double *uf = (long double *)calloc((size_t)(ntgt > 0 ? ntgt : 1) * 3, sizeof(long double));
    if (!uf) {
        free(ur);
        return 2;
    }
    for (long n0 = -nmax[0]; n0 <= nmax[0]; n0++)
        for (long n1 = -nmax[1]; n1 <= nmax[1]; n1++)
            for (long n2 = -nmax[2]; n2 <= nmax[2]; n2++) {
                if (n0 == 0 && n1 == 0 && n2 == 0) continue;
                long double k[3] = {2.0L * PI_L * n0 / L[0], 2.0L * PI_L * n1 / L[1], 2.0L * PI_L * n2 / L[2]};
                long double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                if (k2 > (long double)kmax * kmax) continue;
                long double complex Kh[3][9];
                khat_tensor(kern, k, sigma, Kh);
                /* structure factor per strength component: sum_a rho_a,q exp(-i k.x_a) / |Omega| */
                long double complex chi[9];
                for (int q = 0; q < mi; q++) chi[q] = 0;
                for (int64_t a = 0; a < N; a++) {
                    long double ph = k[0] * x[3 * a] + k[1] * x[3 * a + 1] + k[2] * x[3 * a + 2];
                    long double complex e = cosl(ph) - I * sinl(ph);
                    for (int q = 0; q < mi; q++) chi[q] += e * (long double)rho[mi * a + q];
                }
                for (int q = 0; q < mi; q++) chi[q] /= V;
                long double complex w[3];
                for (int j = 0; j < mo; j++) {
                    w[j] = 0;
                    for (int q = 0; q < mi; q++) w[j] += Kh[j][q] * chi[q];
                }
                for (int64_t ib = 0; ib < ntgt; ib++) {
                    const int64_t b = tgt ? tgt[ib] : ib;
                    long double ph = k[0] * x[3 * b] + k[1] * x[3 * b + 1] + k[2] * x[3 * b + 2];
                    long double complex e = cosl(ph) + I * sinl(ph);
                    for (int j = 0; j < mo; j++) uf[3 * ib + j] += creall(w[j] * e);
                }
            }
    const long double phi0 = win_phi(0.0L);
    for (int64_t ib = 0; ib < ntgt; ib++) {
        const int64_t b = tgt ? tgt[ib] : ib;
        for (int j = 0; j < mo; j++) {
            long double self = 0.0L;
            if (kern == 0 || kern == 1) self = -phi0 * (long double)rho[mi * b + j] / (2.0L * PI_L * sigma);
            u[mo * ib + j] = (double)((long double)ur[mo * ib + j] + uf[3 * ib + j] + self);
        }
    }
    free(ur);
    free(uf);
    return 0;
}

/*
 * Far-field part of the D = 3 split (eq. (ewald_far_3P)) truncated to the
 * cube of wave numbers 2 pi (n0/L0, n1/L1, n2/L2), |n_i| <= K_i, n != 0
 * (eq. (wavenumbers-3p-trunc)): for every target x_t
 *   u_j(x_t) = sum_k Re[ sum_q Khat_jq(k) chi_q(k) e^{i k.x_t} ],
 *   chi_q(k) = (1/|Omega|) sum_s rho_{s,q} e^{-i k.x_s}   (eq. (structurefacgen)).
 */
int oracle_far_3p(int kern, const double L[3], double sigma, const int32_t K[3], int64_t ns, const double *xs,
                  const double *rho, int64_t nt, const double *xt, double *u)
{
    if (kern < 0 || kern > 3 || !(sigma > 0.0) || ns < 0 || nt < 0) return 1;
    for (int i = 0; i < 3; i++)
        if (!(L[i] > 0.0) || K[i] < 0 || K[i] > 65536) return 1;
    const int mi = m_in_of(kern), mo = m_out_of(kern);
    const long double V = (long double)L[0] * L[1] * L[2];
    const int64_t w0 = 2 * K[0] + 1, w1 = 2 * K[1] + 1, w2 = 2 * K[2] + 1;
    const int64_t nm = w0 * w1 * w2;
    /* per mode: wave vector and w_j = sum_q Khat_jq chi_q */
    long double(*kv)[3] = malloc(sizeof(long double[3]) * (size_t)nm);
    long double complex(*wm)[3] = malloc(sizeof(long double complex[3]) * (size_t)nm);
    if (!kv || !wm) {
        free(kv);
        free(wm);
        return 2;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t m = 0; m < nm; m++) {
        const long n0 = (long)(m / (w1 * w2)) - K[0];
        const long n1 = (long)((m / w2) % w1) - K[1];
        const long n2 = (long)(m % w2) - K[2];
        kv[m][0] = 2.0L * PI_L * n0 / L[0];
        kv[m][1] = 2.0L * PI_L * n1 / L[1];
        kv[m][2] = 2.0L * PI_L * n2 / L[2];
        for (int j = 0; j < 3; j++) wm[m][j] = 0;
        if (n0 == 0 && n1 == 0 && n2 == 0) continue; /* k = 0 omitted */
        long double complex Kh[3][9];
        khat_tensor(kern, kv[m], sigma, Kh);
        long double complex chi[9];
        for (int q = 0; q < mi; q++) chi[q] = 0;
        for (int64_t a = 0; a < ns; a++) {
            long double ph = kv[m][0] * xs[3 * a] + kv[m][1] * xs[3 * a + 1] + kv[m][2] * xs[3 * a + 2];
            long double complex e = cosl(ph) - I * sinl(ph);
            for (int q = 0; q < mi; q++) chi[q] += e * (long double)rho[mi * a + q];
        }
        for (int j = 0; j < mo; j++)
            for (int q = 0; q < mi; q++) wm[m][j] += Kh[j][q] * chi[q] / V;
    }
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nt; b++) {
        long double acc[3] = {0, 0, 0};
        for (int64_t m = 0; m < nm; m++) {
            long double ph = kv[m][0] * xt[3 * b] + kv[m][1] * xt[3 * b + 1] + kv[m][2] * xt[3 * b + 2];
            long double complex e = cosl(ph) + I * sinl(ph);
            for (int j = 0; j < mo; j++) acc[j] += creall(wm[m][j] * e);
        }
        for (int j = 0; j < mo; j++) u[mo * b + j] = (double)acc[j];
    }
    free(kv);
    free(wm);
    return 0;
}

/* Point-pair kernel evaluation for tests of the formulas themselves. */
int oracle_kernel_tensor(int kern, const double d[3], double sigma, double *K /*[3*9]*/, double *dK /*[3*3*9]*/)
{
    long double dl[3] = {d[0], d[1], d[2]};
    long double Kl[3][9], dKl[3][3][9];
    if (kern < 0 || kern > 3) return 1;
    kernel_tensor(kern, dl, sigma, Kl, dKl);
    for (int j = 0; j < 3; j++)
        for (int q = 0; q < 9; q++) {
            K[9 * j + q] = (double)Kl[j][q];
            for (int k = 0; k < 3; k++) dK[27 * k + 9 * j + q] = (double)dKl[k][j][q];
        }
    return 0;
}

int oracle_kernel_free_tensor(int kern, const double d[3], double *K)
{
    long double dl[3] = {d[0], d[1], d[2]};
    long double Kl[3][9];
    if (kern < 0 || kern > 3) return 1;
    kernel_free_tensor(kern, dl, Kl);
    for (int j = 0; j < 3; j++)
        for (int q = 0; q < 9; q++) K[9 * j + q] = (double)Kl[j][q];
    return 0;
}
