// dmk_far.hip -- root-level far field of the triply periodic split on gfx950.
//
// At the top level the cell is tiled exactly by M0 x M1 x M2 cubes of side h0,
// each carrying a p^3 grid of first-kind Chebyshev points (Sec. 4,
// evaluation of the far-field contribution).  With proxy strengths rho on the
// grids, the far field on the same grids is
//
//   chi_q(k) = (1/|Omega|) sum_x e^{-i k.x} rho_q(x)          eq. (structurefac)
//   u_j(x)   = sum_{k != 0} Re[ e^{i k.x} sum_q Khat_jq(k) chi_q(k) ]   eq. (eval_tensor)
//
// over the wave numbers k = 2 pi (n0/L0, n1/L1, n2/L2), |n_i| <= K_i.  Along
// axis i the grid points of all cubes form one coordinate list X_i[g],
// g = b p + j (G_i = M_i p entries), and e^{i k.x} = prod_i E_i[g_i][n_i] with
// E_i[g][n] = exp(2 pi i n X_i[g] / L_i).  Both sums therefore factor into
// three one-axis contractions each (sum factorization); every contraction is
// one launch of a complex "mode product"
//
//   Y[a][o][c] = s * sum_i coef(i, o) X[a][i][c]
//
// with coef a view of one of the E_i tables (grids with no axis factored
// over the cube index run all of this in three fused launches, k_far_c1..3).
// On a cover of the cell by cut cubes every contraction is such a direct sum.  On an exact tiling, an axis
// of 8 or more cubes factors through a DFT over the cube index (Sec. 4, large
// aspect ratios): a dense product on the matrix cores up to 64 cubes, an FFT
// (mixed-radix Stockham stages, or Bluestein's chirp convolution for lengths
// with a prime factor above 8) beyond, O(M_i log M_i) per column.
//
// The mollified kernels in Fourier space (App. A convention) are
//   harmonic   Hhat = phihat(|k| sigma) / k^2                 eq. (Hhatsplit_wfunc)
//   biharmonic Bhat = gammaB(|k| sigma) / k^4, gammaB(q) = phihat(q) - q phihat'(q)/2
//   Stokeslet  (k^2 delta_jl - k_j k_l) Bhat                  eq. (moll_stokeslet)
//   stresslet  i [(k_m d_jl + k_j d_lm + k_l d_mj) k^2 - 2 k_j k_l k_m] Bhat
//   rotlet     -(i/2) eps_jlm k_m Hhat
// with phihat(q) = exp(-q^2/4) for the Gaussian window and, for the PSWF
// window of support sigma, phihat(q) = phi(q/c) / phi(0) inside the band
// |q| <= c and 2 int_0^1 phi(t) cos(q t) dt by composite Gauss-Legendre
// quadrature of the window's Chebyshev series beyond it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <type_traits>

#include "dmk_internal.h"

namespace dmk {
namespace {

constexpr int GL_N = 16;  // Gauss-Legendre nodes per quadrature panel

constexpr int FFT_MAXST = 24;   // radix stages of one FFT (lengths up to 2^24)
constexpr int FFT_MIN = 65;     // cube-index DFTs of this length or more run as FFTs

// A length-N FFT as Stockham stages of radix 2 .. 8, or (N with a prime
// factor above 8) Bluestein's convolution through FFTs of length N2, the
// power of two >= 2 N - 1.
struct FftPlan {
    int n;                  // transform length (the axis' cube count)
    int n2;                 // Bluestein: padded length (0: plain Stockham)
    int nst, rad[FFT_MAXST];  // stages of the length-n (or n2) FFT
    int64_t twoff;          // w^k = exp(2 pi i k / len), k < len (len = n, or n2)
    int64_t choff, hoff;    // Bluestein: chirp c_k = exp(-pi i k^2 / n), k < n; H = FFT(h), n2 entries
};

struct FarGeom {
    int G[3], W[3], K[3], M[3], p;
    double L[3];
    int cover;        // 1: cubes of side h0 = min L_i cover the cell, the last cut by a face
    double hr[3];     // h0 / L_i (cover)
    int rows[3];      // grid points with phase-table rows: G_i, or p (the first cube, fac)
    int64_t eoff[3];  // offset of E_i in the table array (double2 entries)
    int fac[3];       // 1: the sums along axis i factor through a length-M_i DFT over the cube index
    int fft[3];       // 1: that DFT runs as an FFT (M_i >= FFT_MIN), else as a dense product
    int64_t doff[3];  // offset of D_i[b][r] = exp(2 pi i r b / M_i) in the table array (dense DFT)
    int64_t foff[3];  // offset of FT_i[n][j] = E_i[j][n], j < p: the first cube's rows transposed (fac)
    FftPlan pl[3];    // FFT of the cube index (fft)
    int64_t nE, nD;   // set-up entries of the phase tables (one per n >= 0) and of the other tables
    int64_t ntab;     // double2 entries of all tables
};

struct FarWin {
    int pswf;      // 0 Gaussian, 1 PSWF series
    int nterms;
    double sigma;
    double c;                        // bandwidth
    double cheb[DMK_PSWF_MAXTERMS];  // phi(t) = sum_m cheb[m] T_m(2 t^2 - 1), t in [0, 1]
    double dcheb[DMK_PSWF_MAXTERMS]; // phi'(t) / t in the same form
    double gx[GL_N], gw[GL_N];       // Gauss-Legendre nodes / weights on [0, 1]
};

// E_i[g][n] = exp(2 pi i n X_i[g] / L_i), X_i[g] / L_i = (b + 1/2 + cos((2j+1) pi/(2p))/2) / M_i
// entries t = 0 .. sum_i G_i (K_i + 1) - 1: one per axis, grid point and
// n >= 0, which also writes n's mirror -n (the complex conjugate)
__device__ inline void far_table_entry(const FarGeom &g, double2 *__restrict__ E, int64_t t)
{
    if (t >= g.nE) {
        // tables of the factored axes: D (dense DFT) or the FFT's twiddles,
        // and for Bluestein the chirp and h (transformed into H after set-up);
        // every phase is reduced mod its period exactly in integers
        int64_t r = t - g.nE;
        for (int ax = 0; ax < 3; ++ax) {
            if (!g.fac[ax]) continue;
            const int64_t m = g.M[ax];
            if (!g.fft[ax]) {
                if (r < m * m) {
                    const int64_t q = ((r / m) * (r % m)) % m;
                    double s, c;
                    sincospi(2.0 * (double)q / (double)m, &s, &c);
                    E[g.doff[ax] + r] = make_double2(c, s);
                    return;
                }
                r -= m * m;
                continue;
            }
            const FftPlan &pl = g.pl[ax];
            const int64_t len = pl.n2 ? pl.n2 : pl.n;
            if (r < len) {  // w^r = exp(2 pi i r / len)
                double s, c;
                sincospi(2.0 * (double)r / (double)len, &s, &c);
                E[pl.twoff + r] = make_double2(c, s);
                return;
            }
            r -= len;
            if (!pl.n2) continue;
            if (r < pl.n2) {
                // chirp c_k = exp(-pi i k^2 / n) (k < n) and h_k = conj(c_|k|) on
                // the circle of length n2 (zero between n and n2 - n)
                const int64_t k = r;
                const int64_t kk = k < pl.n ? k : (pl.n2 - k < pl.n ? pl.n2 - k : -1);
                double s = 0.0, c = 0.0;
                if (kk >= 0) sincospi((double)((kk * kk) % (2 * m)) / (double)m, &s, &c);
                if (k < pl.n) E[pl.choff + k] = make_double2(c, -s);
                E[pl.hoff + k] = kk >= 0 ? make_double2(c, s) : make_double2(0.0, 0.0);
                return;
            }
            r -= pl.n2;
        }
        return;
    }
    int ax = 0;
    int64_t r = t;
    while (ax < 3 && r >= (int64_t)g.rows[ax] * (g.K[ax] + 1)) {
        r -= (int64_t)g.rows[ax] * (g.K[ax] + 1);
        ++ax;
    }
    if (ax >= 3) return;
    const int gi = (int)(r / (g.K[ax] + 1));
    const int n = (int)(r % (g.K[ax] + 1));
    const int b = gi / g.p, j = gi % g.p;
    // node coordinate over the cell length: ((b + 1/2) h0 + (h0/2) eta_j) / L_i
    const double v = (double)b + 0.5 + 0.5 * cospi((double)(2 * j + 1) / (double)(2 * g.p));
    const double xr = g.cover ? v * g.hr[ax] : v / (double)g.M[ax];
    double s, c;
    sincospi(2.0 * (double)n * xr, &s, &c);
    double2 *row = E + g.eoff[ax] + (int64_t)gi * g.W[ax] + g.K[ax];  // entry n = 0 of this grid point
    row[n] = make_double2(c, s);
    if (n > 0) row[-n] = make_double2(c, -s);
    if (g.fac[ax] && gi < g.p) {
        double2 *ft = E + g.foff[ax] + (int64_t)(g.K[ax] + n) * g.p + gi;
        ft[0] = make_double2(c, s);
        if (n > 0) ft[-(int64_t)2 * n * g.p] = make_double2(c, -s);
    }
}

// Y[a][o][c] = s * sum_i coef(i, o) X[a][i][c], coef(i, o) = E[i*si + o*so]
// (conjugated when CONJ); RIN: X real; ROUT: only Re(Y) is stored (real Y)
template <bool RIN, bool ROUT, bool CONJ>
__global__ void k_mode(const void *__restrict__ Xv, const double2 *__restrict__ E, int64_t A, int I, int O, int C,
                       int64_t si, int64_t so, double s, void *__restrict__ Yv)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A * O * C) return;
    const int c = (int)(t % C);
    const int o = (int)((t / C) % O);
    const int64_t a = t / ((int64_t)C * O);
    double re = 0.0, im = 0.0;
    const int64_t xb = a * I * C + c;
#pragma unroll 4
    for (int i = 0; i < I; ++i) {
        const double2 e = E[i * si + o * so];
        const double ei = CONJ ? -e.y : e.y;
        if constexpr (RIN) {
            const double x = ((const double *)Xv)[xb + (int64_t)i * C];
            re = fma(e.x, x, re);
            im = fma(ei, x, im);
        } else {
            const double2 x = ((const double2 *)Xv)[xb + (int64_t)i * C];
            re = fma(e.x, x.x, fma(-ei, x.y, re));
            im = fma(e.x, x.y, fma(ei, x.x, im));
        }
    }
    const int64_t yi = (a * O + o) * C + c;
    if constexpr (ROUT)
        ((double *)Yv)[yi] = s * re;
    else
        ((double2 *)Yv)[yi] = make_double2(s * re, s * im);
}

// The same mode product with its operands staged in LDS (few terms i, a small
// coefficient table): a workgroup takes AB consecutive a and CB consecutive
// c, copies coef(i, o) for all (i, o) and its block of X (AB x I x CB, rows of
// CB contiguous values) into LDS with coalesced loads, and evaluates its
// AB x O x CB outputs from there in the order of k_mode (same terms, same
// fused multiply-adds), so the results are identical.
constexpr int ML_T = 256;
constexpr int ML_LDS = 48 * 1024;

struct ModeBlock {
    int ab, cb;   // a and c per workgroup
    int64_t nwg;  // workgroups
    size_t lds;   // bytes of LDS
};

template <bool RIN, bool ROUT, bool CONJ>
__global__ __launch_bounds__(ML_T) void k_mode_lds(const void *__restrict__ Xv, const double2 *__restrict__ E,
                                                   int64_t A, int I, int O, int C, int64_t si, int64_t so, double s,
                                                   int ab, int cb, void *__restrict__ Yv)
{
    extern __shared__ double2 ml[];
    double2 *es = ml;                         // coef(i, o) at es[i * O + o]
    double *xr = (double *)(ml + (int64_t)I * O);  // X block (RIN)
    double2 *xc = ml + (int64_t)I * O;        // X block (complex)
    const int ncb = (C + cb - 1) / cb;
    const int64_t a0 = (int64_t)(blockIdx.x / ncb) * ab;
    const int c0 = (int)(blockIdx.x % ncb) * cb;
    const int na = (int)min((int64_t)ab, A - a0), nc = min(cb, C - c0);
    // staging, ML_U loads of a thread in flight before its stores
    constexpr int ML_U = 8;
    const int ne = I * O;
    for (int k0 = threadIdx.x; k0 < ne; k0 += ML_U * ML_T) {
        double2 v[ML_U];
#pragma unroll
        for (int u = 0; u < ML_U; ++u) {
            const int k = k0 + u * ML_T;
            if (k < ne) v[u] = E[(k / O) * si + (k % O) * so];
        }
#pragma unroll
        for (int u = 0; u < ML_U; ++u)
            if (k0 + u * ML_T < ne) es[k0 + u * ML_T] = v[u];
    }
    // block element (al, i, cl) at (al * I + i) * nc + cl
    const int nx = na * I * nc;
    for (int k0 = threadIdx.x; k0 < nx; k0 += ML_U * ML_T) {
        typename std::conditional<RIN, double, double2>::type v[ML_U];
#pragma unroll
        for (int u = 0; u < ML_U; ++u) {
            const int k = k0 + u * ML_T;
            if (k < nx) {
                const int row = k / nc, cl = k - row * nc;
                const int64_t g = (a0 + row / I) * I * C + (int64_t)(row % I) * C + c0 + cl;
                if constexpr (RIN)
                    v[u] = ((const double *)Xv)[g];
                else
                    v[u] = ((const double2 *)Xv)[g];
            }
        }
#pragma unroll
        for (int u = 0; u < ML_U; ++u) {
            const int k = k0 + u * ML_T;
            if (k < nx) {
                if constexpr (RIN)
                    xr[k] = v[u];
                else
                    xc[k] = v[u];
            }
        }
    }
    __syncthreads();
    const int ny = na * O * nc;
    for (int k = threadIdx.x; k < ny; k += ML_T) {
        const int cl = k % nc, o = (k / nc) % O, al = k / (nc * O);
        double re = 0.0, im = 0.0;
        const int xb = al * I * nc + cl;
#pragma unroll 4
        for (int i = 0; i < I; ++i) {
            const double2 e = es[i * O + o];
            const double ei = CONJ ? -e.y : e.y;
            if constexpr (RIN) {
                const double x = xr[xb + i * nc];
                re = fma(e.x, x, re);
                im = fma(ei, x, im);
            } else {
                const double2 x = xc[xb + i * nc];
                re = fma(e.x, x.x, fma(-ei, x.y, re));
                im = fma(e.x, x.y, fma(ei, x.x, im));
            }
        }
        const int64_t yi = ((a0 + al) * O + o) * C + c0 + cl;
        if constexpr (ROUT)
            ((double *)Yv)[yi] = s * re;
        else
            ((double2 *)Yv)[yi] = make_double2(s * re, s * im);
    }
}

// The same mode product on the FP64 matrix cores, for contractions large
// enough to fill 16 x 16 tiles (the long axis of an elongated cell): one
// workgroup per (a, 16 outputs o, 16 outputs c); its MM_W wavefronts take
// every MM_W-th group of 4 terms i, one v_mfma_f64_16x16x4 per group (A: lane l
// holds A[l % 16][l / 16], B: B[l / 16][l % 16], D: D[4 r + l / 16][l % 16]),
// and the partial tiles are summed through LDS in a fixed order.  (8
// wavefronts per tile measured best for the long axis of a 32-cube cell: 4 and
// 16 were slower.)  Real and
// imaginary parts accumulate in two tiles:
//   Re += Re(coef) Re(x) - Im(coef) Im(x),  Im += Re(coef) Im(x) + Im(coef) Re(x).
typedef double dbl4m __attribute__((ext_vector_type(4)));
constexpr int MM_W = 8;  // wavefronts per tile

template <bool RIN, bool ROUT, bool CONJ, int NW = MM_W>
__global__ __launch_bounds__(NW * WAVE) void k_mode_mfma(const void *__restrict__ Xv,
                                                           const double2 *__restrict__ E, int64_t A, int I, int O,
                                                           int C, int64_t si, int64_t so, double s, int nsplit,
                                                           double2 *__restrict__ part, void *__restrict__ Yv)
{
    __shared__ double red[NW > 1 ? NW - 1 : 1][8][WAVE];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int to = (O + 15) / 16, tc = (C + 15) / 16;
    const int64_t tile = blockIdx.x / nsplit;
    const int sp = (int)(blockIdx.x - tile * nsplit);
    // this workgroup's groups of 4 terms: [g0, g1) of the split's share
    const int ng = (I + 3) / 4;
    const int g0 = (int)((int64_t)ng * sp / nsplit), g1 = (int)((int64_t)ng * (sp + 1) / nsplit);
    const int64_t a = tile / ((int64_t)to * tc);
    const int rem = (int)(tile - a * to * tc);
    const int ot = rem / tc, ct = rem - (rem / tc) * tc;
    const int li = lane & 15, lk = lane >> 4;
    const int oa = ot * 16 + li, cb = ct * 16 + li;
    const bool ook = oa < O, cok = cb < C;
    dbl4m dre = {0.0, 0.0, 0.0, 0.0}, dim = {0.0, 0.0, 0.0, 0.0};
    for (int gq = g0 + wv; gq < g1; gq += NW) {
        const int k = 4 * gq + lk;
        const bool kok = k < I;
        double er = 0.0, ei = 0.0, xr = 0.0, xi = 0.0;
        if (kok && ook) {
            const double2 e = E[(int64_t)k * si + (int64_t)oa * so];
            er = e.x;
            ei = CONJ ? -e.y : e.y;
        }
        if (kok && cok) {
            const int64_t xo = (a * I + k) * C + cb;
            if constexpr (RIN) {
                xr = ((const double *)Xv)[xo];
            } else {
                const double2 x = ((const double2 *)Xv)[xo];
                xr = x.x;
                xi = x.y;
            }
        }
        dre = __builtin_amdgcn_mfma_f64_16x16x4f64(er, xr, dre, 0, 0, 0);
        if constexpr (!RIN) dre = __builtin_amdgcn_mfma_f64_16x16x4f64(-ei, xi, dre, 0, 0, 0);
        if constexpr (!ROUT) {
            dim = __builtin_amdgcn_mfma_f64_16x16x4f64(ei, xr, dim, 0, 0, 0);
            if constexpr (!RIN) dim = __builtin_amdgcn_mfma_f64_16x16x4f64(er, xi, dim, 0, 0, 0);
        }
    }
    if (wv > 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            red[wv - 1][r][lane] = dre[r];
            red[wv - 1][4 + r][lane] = dim[r];
        }
    }
    __syncthreads();
    if (wv > 0 || !cok) return;
#pragma unroll
    for (int w = 0; w < NW - 1; ++w)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            dre[r] += red[w][r][lane];
            dim[r] += red[w][4 + r][lane];
        }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int o = ot * 16 + 4 * r + lk;
        if (o < O) {
            const int64_t yi = (a * O + o) * C + cb;
            if (nsplit > 1) {
                part[(int64_t)sp * A * O * C + yi] = make_double2(dre[r], dim[r]);
            } else if constexpr (ROUT) {
                ((double *)Yv)[yi] = s * dre[r];
            } else {
                ((double2 *)Yv)[yi] = make_double2(s * dre[r], s * dim[r]);
            }
        }
    }
}

// Y = s * (sum of the nsplit partial results, in split order)
template <bool ROUT>
__global__ void k_mode_sum(const double2 *__restrict__ part, int64_t n, int nsplit, double s, void *__restrict__ Yv)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    double re = 0.0, im = 0.0;
    for (int q = 0; q < nsplit; ++q) {
        const double2 v = part[q * n + t];
        re += v.x;
        im += v.y;
    }
    if constexpr (ROUT)
        ((double *)Yv)[t] = s * re;
    else
        ((double2 *)Yv)[t] = make_double2(s * re, s * im);
}

// Long axes of an exact tiling: the grid index is g = b p + j and the phase
// factors as E[b p + j][n] = w^(n b) F[j][n], w = exp(2 pi i / M), F the
// rows of the first cube (b = 0).  A sum over g is then a length-M DFT over
// the cube index b (a mode product with D[b][r] = w^(r b)) followed by a sum
// over j for each n, which only reads the DFT at r = n mod M (k_fold); the
// evaluation runs the transposed steps (k_unfold, then the DFT).

// Y[a][n][c] = s * sum_j F(j, n) Z[a][n mod M][j][c], n = -K..K, F conjugated when CONJ
template <bool CONJ>
__global__ void k_fold(const double2 *__restrict__ Z, const double2 *__restrict__ E, int64_t A, int M, int p, int W,
                       int K, int C, double s, double2 *__restrict__ Y)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A * W * C) return;
    const int c = (int)(t % C);
    const int o = (int)((t / C) % W);
    const int64_t a = t / ((int64_t)C * W);
    const int r = ((o - K) % M + M) % M;
    const double2 *z = Z + ((a * M + r) * p) * (int64_t)C + c;
    double re = 0.0, im = 0.0;
    for (int j = 0; j < p; ++j) {
        const double2 e = E[(int64_t)j * W + o];
        const double ei = CONJ ? -e.y : e.y;
        const double2 x = z[(int64_t)j * C];
        re = fma(e.x, x.x, fma(-ei, x.y, re));
        im = fma(e.x, x.y, fma(ei, x.x, im));
    }
    Y[t] = make_double2(s * re, s * im);
}

// k_fold for one column (C = 1), one workgroup per a: the slice Z[a] (M p
// values, read by about W / M outputs each) is staged in LDS with coalesced
// loads; same terms and order as k_fold
constexpr int FL_T = 256;
constexpr int FL_LDS = 48 * 1024;

template <bool CONJ>
__global__ __launch_bounds__(FL_T) void k_fold_lds(const double2 *__restrict__ Z, const double2 *__restrict__ E, int M,
                                                   int p, int W, int K, double s, double2 *__restrict__ Y)
{
    extern __shared__ double2 zs[];
    const int64_t a = blockIdx.x;
    const int n = M * p;
    const double2 *za = Z + a * n;
    for (int i = threadIdx.x; i < n; i += FL_T) zs[i] = za[i];
    __syncthreads();
    for (int o = threadIdx.x; o < W; o += FL_T) {
        const int r = ((o - K) % M + M) % M;
        const double2 *z = zs + r * p;
        double re = 0.0, im = 0.0;
        for (int j = 0; j < p; ++j) {
            const double2 e = E[(int64_t)j * W + o];
            const double ei = CONJ ? -e.y : e.y;
            const double2 x = z[j];
            re = fma(e.x, x.x, fma(-ei, x.y, re));
            im = fma(e.x, x.y, fma(ei, x.x, im));
        }
        Y[a * W + o] = make_double2(s * re, s * im);
    }
}

// U[a][r][j][c] = sum over n = -K..K with n = r (mod M) of F(j, n) X[a][n][c],
// F read from its transpose FT[n][j] (coalesced across j)
__global__ void k_unfold(const double2 *__restrict__ X, const double2 *__restrict__ FT, int64_t A, int M, int p, int W,
                         int K, int C, double2 *__restrict__ U)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A * M * p * C) return;
    const int c = (int)(t % C);
    const int j = (int)((t / C) % p);
    const int r = (int)((t / ((int64_t)C * p)) % M);
    const int64_t a = t / ((int64_t)C * p * M);
    double re = 0.0, im = 0.0;
    // o = n + K runs over the class of r: the first o >= 0 with o = r + K (mod M)
    for (int o = (r + K) % M; o < W; o += M) {
        const double2 e = FT[(int64_t)o * p + j];
        const double2 x = X[(a * W + o) * C + c];
        re = fma(e.x, x.x, fma(-e.y, x.y, re));
        im = fma(e.x, x.y, fma(e.y, x.x, im));
    }
    U[t] = make_double2(re, im);
}

// ---- FFT over the cube index (Sec. 4, large aspect ratios): data [A][N][ncol],
// the transform along the middle index.

// One radix-R Stockham stage.  With S the product of the radices of the
// stages before, the sub-transforms have length n = N / S; a thread takes the
// butterfly (s, b2) of one (a, column), s < S, b2 < m = n / R:
//   x_b1 = in[a][(m b1 + b2) S + s],  b1 < R,
//   out[a][b2 S R + s + S r1] = w_n^(sg r1 b2) sum_b1 w_R^(sg r1 b1) x_b1,
// with w_len = exp(2 pi i / len) from the twiddle table tw of the length-N
// transform (w_n = w_N^S, w_R = w_N^(N/R)) and sg = -1 or +1.  After the
// last stage (S R = N) the outputs are in natural order.  INM: real input;
// OUTM: only the real part is stored; the output is scaled by `scale`.
template <int R, bool INM, bool OUTM>
__global__ void k_fft_stage(const void *__restrict__ in, void *__restrict__ out, int64_t A, int N, int ncol, int S,
                            int sg, const double2 *__restrict__ tw, double scale)
{
    const int nbf = N / R;
    const int64_t per = (int64_t)nbf * ncol;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A * per) return;
    const int col = (int)(t % ncol);
    const int u = (int)((t / ncol) % nbf);
    const int64_t a = t / per;
    const int m = nbf / S;
    const int sb = u % S, b2 = u / S;
    const int64_t base = a * N;
    double2 x[R];
#pragma unroll
    for (int b1 = 0; b1 < R; ++b1) {
        const int64_t idx = (base + (int64_t)(m * b1 + b2) * S + sb) * ncol + col;
        if constexpr (INM)
            x[b1] = make_double2(((const double *)in)[idx], 0.0);
        else
            x[b1] = ((const double2 *)in)[idx];
    }
    const double sgn = sg < 0 ? -1.0 : 1.0;
    double2 wr[R];  // w_R^k with the transform's sign
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const double2 w = tw[(int64_t)k * nbf];
        wr[k] = make_double2(w.x, sgn * w.y);
    }
#pragma unroll
    for (int r1 = 0; r1 < R; ++r1) {
        double re = 0.0, im = 0.0;
#pragma unroll
        for (int b1 = 0; b1 < R; ++b1) {
            const double2 w = wr[(r1 * b1) % R];
            re = fma(w.x, x[b1].x, fma(-w.y, x[b1].y, re));
            im = fma(w.x, x[b1].y, fma(w.y, x[b1].x, im));
        }
        const double2 tv = tw[(int64_t)S * r1 * b2];  // w_n^(r1 b2), S r1 b2 < N
        const double ti = sgn * tv.y;
        const double yr = scale * (tv.x * re - ti * im), yi = scale * (tv.x * im + ti * re);
        const int64_t o = (base + (int64_t)b2 * S * R + sb + (int64_t)S * r1) * ncol + col;
        if constexpr (OUTM)
            ((double *)out)[o] = yr;
        else
            ((double2 *)out)[o] = make_double2(yr, yi);
    }
}

// Bluestein: sum_b w^(sg r b) X_b = c_r sum_b (X_b c_b) conj(c_(r-b)), c_k =
// exp(sg pi i k^2 / n); the sum is a circular convolution of length n2 >=
// 2n - 1 with h_k = conj(c_|k|), done as IFFT(FFT(a) H), H = FFT(h).  The
// tables hold the sg = -1 chirp; sg = +1 runs the same steps on conj(X) and
// conjugates the result.
template <bool RIN>
__global__ void k_blue_in(const void *__restrict__ in, double2 *__restrict__ P, int64_t A, int n, int n2, int ncol,
                          int sg, const double2 *__restrict__ ch)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A * n2 * (int64_t)ncol) return;
    const int col = (int)(t % ncol);
    const int k = (int)((t / ncol) % n2);
    const int64_t a = t / ((int64_t)ncol * n2);
    double2 v = make_double2(0.0, 0.0);
    if (k < n) {
        const int64_t idx = (a * n + k) * ncol + col;
        double2 x;
        if constexpr (RIN)
            x = make_double2(((const double *)in)[idx], 0.0);
        else
            x = ((const double2 *)in)[idx];
        if (sg > 0) x.y = -x.y;
        const double2 c = ch[k];
        v = make_double2(x.x * c.x - x.y * c.y, x.x * c.y + x.y * c.x);
    }
    P[t] = v;
}

__global__ void k_blue_mul(double2 *__restrict__ P, int64_t A, int n2, int ncol, const double2 *__restrict__ H)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A * n2 * (int64_t)ncol) return;
    const int k = (int)((t / ncol) % n2);
    const double2 h = H[k], x = P[t];
    P[t] = make_double2(x.x * h.x - x.y * h.y, x.x * h.y + x.y * h.x);
}

template <bool ROUT>
__global__ void k_blue_out(const double2 *__restrict__ P, void *__restrict__ out, int64_t A, int n, int n2, int ncol,
                           int sg, const double2 *__restrict__ ch, double scale)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A * n * (int64_t)ncol) return;
    const int col = (int)(t % ncol);
    const int r = (int)((t / ncol) % n);
    const int64_t a = t / ((int64_t)ncol * n);
    const double2 x = P[(a * n2 + r) * ncol + col], c = ch[r];
    double yr = scale * (x.x * c.x - x.y * c.y), yi = scale * (x.x * c.y + x.y * c.x);
    if (sg > 0) yi = -yi;
    if constexpr (ROUT)
        ((double *)out)[t] = yr;
    else
        ((double2 *)out)[t] = make_double2(yr, yi);
}

// a Chebyshev series of the PSWF window in u = 2 t^2 - 1 (Clenshaw), over
// all DMK_PSWF_MAXTERMS coefficients (zero past the window's nterms64, where
// the recurrence stays exactly zero): a fixed length lets the coefficient
// loads be issued ahead of the dependent steps
__device__ inline double win_series(const FarWin &w, const double *cf, double t)
{
    const double u = 2.0 * t * t - 1.0;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int m = DMK_PSWF_MAXTERMS - 1; m >= 1; --m) {
        const double b0 = fma(2.0 * u, b1, cf[m] - b2);
        b2 = b1;
        b1 = b0;
    }
    (void)w;
    return fma(u, b1, cf[0] - b2);
}

__device__ inline double win_phi(const FarWin &w, double t) { return win_series(w, w.cheb, t); }

// phihat(q) and phihat'(q), the same on every lane of the wavefront.  Beyond
// the band the quadrature nodes are split over the 64 lanes and the partial
// sums combined with shuffles in a fixed order.
__device__ inline void win_hat(const FarWin &w, double q, int lane, double &ph, double &dph)
{
    if (!w.pswf) {
        ph = exp(-0.25 * q * q);
        dph = -0.5 * q * ph;
        return;
    }
    if (q <= w.c) {
        // in the band the window's transform is the window rescaled (the
        // eigen-relation of psi_0^c, Sec. 2.2): phihat(q) = phi(q/c) / phi(0)
        const double t = q / w.c, phi0 = win_phi(w, 0.0);
        ph = win_phi(w, t) / phi0;
        dph = t * win_series(w, w.dcheb, t) / (w.c * phi0);
        return;
    }
    // beyond it: 2 int_0^1 phi(t) cos(q t) dt and -2 int_0^1 t phi(t) sin(q t) dt on
    // panels over which q t varies by at most 4; at least two panels, as phi is
    // a polynomial of degree up to ~60 in t
    const int np = 2 + (int)(q * 0.25);
    const double hw = 1.0 / np;
    double a = 0.0, b = 0.0;
    for (int i = lane; i < np * GL_N; i += WAVE) {
        const int k = i / GL_N, nd = i - k * GL_N;
        const double t = (k + w.gx[nd]) * hw;
        const double f = w.gw[nd] * win_phi(w, t);
        double sn, cs;
        sincos(q * t, &sn, &cs);
        a = fma(f, cs, a);
        b = fma(f * t, sn, b);
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off);
        b += __shfl_xor(b, off);
    }
    ph = 2.0 * hw * a;
    dph = -2.0 * hw * b;
}

// phihat(q) and phihat'(q) at q = |k| sigma for the wave numbers of one
// octant, n_i = 0 .. K_i: the mode weights depend on the sign of each n_i only
// through k itself, so the window's transform (a quadrature beyond the band)
// is evaluated once per octant mode m, by one wavefront.  k^2 is formed as in
// the weights kernel, so both see the same q.
__device__ inline void far_phihat_mode(const FarGeom &g, const FarWin &w, double2 *__restrict__ PH, int64_t m,
                                       int lane)
{
    const int64_t o1 = g.K[1] + 1, o2 = g.K[2] + 1;
    if (m >= (int64_t)(g.K[0] + 1) * o1 * o2) return;
    const int a0 = (int)(m / (o1 * o2)), a1 = (int)((m / o2) % o1), a2 = (int)(m % o2);
    double ph = 0.0, dph = 0.0;
    if (a0 != 0 || a1 != 0 || a2 != 0) {
        const double k[3] = {2.0 * M_PI * a0 / g.L[0], 2.0 * M_PI * a1 / g.L[1], 2.0 * M_PI * a2 / g.L[2]};
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        win_hat(w, sqrt(k2) * w.sigma, lane, ph, dph);
    }
    if (lane == 0) PH[m] = make_double2(ph, dph);
}

// One launch for the two independent set-up tables: workgroups below nbt
// write the phase tables E (one entry per thread), the rest the window's
// transform per octant mode (one mode per wavefront).
constexpr int PREP_T = 256;

__global__ __launch_bounds__(PREP_T) void k_far_prep(FarGeom g, FarWin w, double2 *__restrict__ E,
                                                     double2 *__restrict__ PH, unsigned nbt)
{
    if (blockIdx.x < nbt) {
        far_table_entry(g, E, (int64_t)blockIdx.x * PREP_T + threadIdx.x);
        return;
    }
    const int64_t m = (int64_t)(blockIdx.x - nbt) * (PREP_T / WAVE) + threadIdx.x / WAVE;
    far_phihat_mode(g, w, PH, m, threadIdx.x & (WAVE - 1));
}

// sum_q Khat_jq(k) x[q] for the kernel's mollified Fourier symbol at wave
// vector k (k2 = |k|^2, q = |k| sigma, ph / dph = phihat and phihat' at q)
template <int KERN>
__device__ inline void mode_weight(const double k[3], double k2, double q, double ph, double dph, const double2 *x,
                                   double2 *out)
{
    const double Hh = ph / k2;
    const double Bh = (ph - 0.5 * q * dph) / (k2 * k2);
    if constexpr (KERN == 0) {
        out[0] = make_double2(Hh * x[0].x, Hh * x[0].y);
    } else if constexpr (KERN == 1) {
        for (int j = 0; j < 3; ++j) {
            double re = 0.0, im = 0.0;
            for (int l = 0; l < 3; ++l) {
                const double K = ((j == l ? k2 : 0.0) - k[j] * k[l]) * Bh;
                re += K * x[l].x;
                im += K * x[l].y;
            }
            out[j] = make_double2(re, im);
        }
    } else if constexpr (KERN == 2) {
        // i * T: multiplying by i maps (re, im) to (-im, re)
        for (int j = 0; j < 3; ++j) {
            double re = 0.0, im = 0.0;
            for (int l = 0; l < 3; ++l)
                for (int mm = 0; mm < 3; ++mm) {
                    const double T = ((j == l ? k[mm] : 0.0) + (l == mm ? k[j] : 0.0) + (mm == j ? k[l] : 0.0)) * k2 -
                                     2.0 * k[j] * k[l] * k[mm];
                    const double K = T * Bh;
                    re += K * x[3 * l + mm].x;
                    im += K * x[3 * l + mm].y;
                }
            out[j] = make_double2(-im, re);
        }
    } else {
        // sum_l -(i/2) eps_jlm k_m Hhat chi_l = (i/2) Hhat (k x chi)_j
        const double h = 0.5 * Hh;
        const double cr[3] = {k[1] * x[2].x - k[2] * x[1].x, k[2] * x[0].x - k[0] * x[2].x,
                              k[0] * x[1].x - k[1] * x[0].x};
        const double ci[3] = {k[1] * x[2].y - k[2] * x[1].y, k[2] * x[0].y - k[0] * x[2].y,
                              k[0] * x[1].y - k[1] * x[0].y};
        // i h (cr + i ci) = (-h ci, h cr)
        for (int j = 0; j < 3; ++j) out[j] = make_double2(-h * ci[j], h * cr[j]);
    }
    (void)Bh;
    (void)Hh;
}

// W[j][m] = sum_q Khat_jq(k_m) chi[q][m] for every mode m (0 at k = 0), one
// thread per mode, with phihat and phihat' from the octant table
constexpr int FW_T = 256;

template <int KERN>
__global__ __launch_bounds__(FW_T) void k_far_weights(FarGeom g, double sigma, const double2 *__restrict__ PH,
                                                      const double2 *__restrict__ chi, const double2 *__restrict__ part,
                                                      int nsplit, double chi_scale, double2 *__restrict__ Wt)
{
    constexpr int MI = KERN == 0 ? 1 : (KERN == 2 ? 9 : 3);
    constexpr int MO = KERN == 0 ? 1 : 3;
    const int64_t nm = (int64_t)g.W[0] * g.W[1] * g.W[2];
    const int64_t m = (int64_t)blockIdx.x * FW_T + threadIdx.x;
    if (m >= nm) return;
    const int n0 = (int)(m / ((int64_t)g.W[1] * g.W[2])) - g.K[0];
    const int n1 = (int)((m / g.W[2]) % g.W[1]) - g.K[1];
    const int n2 = (int)(m % g.W[2]) - g.K[2];
    double2 out[MO];
    for (int j = 0; j < MO; ++j) out[j] = make_double2(0.0, 0.0);
    if (n0 != 0 || n1 != 0 || n2 != 0) {
        const double k[3] = {2.0 * M_PI * n0 / g.L[0], 2.0 * M_PI * n1 / g.L[1], 2.0 * M_PI * n2 / g.L[2]};
        const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        const double q = sqrt(k2) * sigma;
        const int64_t o =
            ((int64_t)abs(n0) * (g.K[1] + 1) + abs(n1)) * (int64_t)(g.K[2] + 1) + abs(n2);
        const double2 pd = PH[o];
        const double ph = pd.x, dph = pd.y;
        double2 x[MI];
        if (nsplit > 1) {
            // chi from the split partial results of its contraction, added in
            // split order and scaled as k_mode_sum would
            for (int c = 0; c < MI; ++c) {
                double re = 0.0, im = 0.0;
                for (int q = 0; q < nsplit; ++q) {
                    const double2 v = part[(int64_t)q * MI * nm + c * nm + m];
                    re += v.x;
                    im += v.y;
                }
                x[c] = make_double2(chi_scale * re, chi_scale * im);
            }
        } else {
            for (int c = 0; c < MI; ++c) x[c] = chi[c * nm + m];
        }
        mode_weight<KERN>(k, k2, q, ph, dph, x, out);
    }
    for (int j = 0; j < MO; ++j) Wt[j * nm + m] = out[j];
}

// ---------------------------------------------------------------------------
// Small grids (no axis factored over the cube index): the whole far field in
// three launches.  Each workgroup keeps its share in LDS and computes the
// phase factors it needs itself (as the table entries above); the slab
// kernels run 1024-thread workgroups (few workgroups, so each thread's serial
// share of a sum is what costs), the pencil kernel 256:
//   k_far_c1, one (component, g0) slab:  T2[q][g0][n1][n2] = sum_g1 conj(E1)
//             sum_g2 conj(E2) rho[q][g0][g1][g2]; further workgroups beside
//             the slabs write the window's transform per octant mode (PH);
//   k_far_c2, one (n1, n2) pencil: chi over g0 (scaled by 1/|Omega|), the
//             mode weights (the window's transform from PH), and back over
//             n0: V1[j][g0][n1][n2];
//   k_far_c3, one (component, g0) slab: u[j][g0][g1][g2] = Re sum_n2 E2
//             sum_n1 E1 V1[j][g0][n1][n2].
// Every sum takes the fused multiply-adds of k_mode, split over the lanes in a
// fixed order (wg_sums).
constexpr int FC_TS = 1024;  // threads of the slab kernels (k_far_c1, k_far_c3)
constexpr int FC_TP = 256;   // threads of the pencil kernel (k_far_c2)
constexpr size_t FC_LDS = 64 * 1024;
constexpr int FC_PRE = 8;   // slab values per thread loaded ahead (doubles)
constexpr int FC_PRE2 = 4;  // pencil / slab values per thread loaded ahead (complex)

// Sums of a workgroup: out o (o < nout) = sum over i < nin of the terms that
// acc(o, i, re, im) adds.  Each output takes L lanes of one wavefront (L a
// power of two, as many as the NT threads allow, at most 64); lane r of the
// group adds the terms i = r, r + L, ... in order, and the L partial sums are
// combined by xor shuffles, so the order of every sum is fixed.  st(o, re,
// im) stores the result (called by the group's first lane).
template <int NT, class Acc, class Store>
__device__ inline void wg_sums(int nout, int nin, int tid, Acc acc, Store st)
{
    int L = 1;
    while (L < WAVE && 2 * L * nout <= NT && 2 * L <= nin) L *= 2;
    const int per = NT / L;  // outputs per round
    for (int o0 = 0; o0 < nout; o0 += per) {
        const int o = o0 + tid / L, r = tid & (L - 1);
        double re = 0.0, im = 0.0;
        if (o < nout) {
#pragma unroll 4
            for (int i = r; i < nin; i += L) acc(o, i, re, im);
        }
        for (int off = L / 2; off > 0; off >>= 1) {
            re += __shfl_xor(re, off);
            im += __shfl_xor(im, off);
        }
        if (o < nout && r == 0) st(o, re, im);
    }
}

// E_i[gi][n], n >= 0 (the table entry far_table_entry writes)
__device__ inline double2 far_phase(const FarGeom &g, int ax, int gi, int n)
{
    const int b = gi / g.p, j = gi % g.p;
    const double v = (double)b + 0.5 + 0.5 * cospi((double)(2 * j + 1) / (double)(2 * g.p));
    const double xr = g.cover ? v * g.hr[ax] : v / (double)g.M[ax];
    double sn, cs;
    sincospi(2.0 * (double)n * xr, &sn, &cs);
    return make_double2(cs, sn);
}

// the imaginary part of E_i[.][n] (n of either sign) from the row of n >= 0
__device__ inline double phase_im(const double2 e, int n) { return n < 0 ? -e.y : e.y; }

template <int NT>
__device__ inline void fill_phases(const FarGeom &g, int ax, double2 *e, int tid)
{
    const int kk = g.K[ax] + 1;
    for (int t = tid; t < g.G[ax] * kk; t += NT) e[t] = far_phase(g, ax, t / kk, t % kk);
}

__global__ __launch_bounds__(FC_TS) void k_far_c1(FarGeom g, const double *__restrict__ rho, double2 *__restrict__ T2,
                                                 FarWin w, double2 *__restrict__ PH, unsigned nslab)
{
    if (blockIdx.x >= nslab) {  // the window's transform per octant mode, one per wavefront
        const int64_t m = (int64_t)(blockIdx.x - nslab) * (FC_TS / WAVE) + threadIdx.x / WAVE;
        far_phihat_mode(g, w, PH, m, threadIdx.x & (WAVE - 1));
        return;
    }
    extern __shared__ double2 fc_lds[];
    const int G1 = g.G[1], G2 = g.G[2], W1 = g.W[1], W2 = g.W[2], K1 = g.K[1], K2 = g.K[2];
    double2 *e2 = fc_lds;
    double2 *e1 = e2 + G2 * (K2 + 1);
    double2 *t1 = e1 + G1 * (K1 + 1);
    double *x = (double *)(t1 + G1 * W2);
    const int64_t a = blockIdx.x;  // q * G0 + g0
    const int tid = threadIdx.x;
    // the slab's first FC_PRE values per thread are loaded before the phase
    // factors are computed, so that the two overlap
    const double *xs = rho + a * G1 * G2;
    double xr[FC_PRE];
#pragma unroll
    for (int u = 0; u < FC_PRE; ++u) {
        const int t = tid + u * FC_TS;
        xr[u] = t < G1 * G2 ? xs[t] : 0.0;
    }
    fill_phases<FC_TS>(g, 2, e2, tid);
    fill_phases<FC_TS>(g, 1, e1, tid);
#pragma unroll
    for (int u = 0; u < FC_PRE; ++u) {
        const int t = tid + u * FC_TS;
        if (t < G1 * G2) x[t] = xr[u];
    }
    for (int t = tid + FC_PRE * FC_TS; t < G1 * G2; t += FC_TS) x[t] = xs[t];
    __syncthreads();
    wg_sums<FC_TS>(
        G1 * W2, G2, tid,
        [&](int t, int i, double &re, double &im) {
            const int g1 = t / W2, n = t % W2 - K2;
            const double2 e = e2[i * (K2 + 1) + (n < 0 ? -n : n)];
            const double ei = -phase_im(e, n);
            const double xv = x[g1 * G2 + i];
            re = fma(e.x, xv, re);
            im = fma(ei, xv, im);
        },
        [&](int t, double re, double im) { t1[t] = make_double2(re, im); });
    __syncthreads();
    double2 *out = T2 + a * W1 * W2;
    wg_sums<FC_TS>(
        W1 * W2, G1, tid,
        [&](int t, int i, double &re, double &im) {
            const int n = t / W2 - K1, c = t % W2;
            const double2 e = e1[i * (K1 + 1) + (n < 0 ? -n : n)];
            const double ei = -phase_im(e, n);
            const double2 xv = t1[i * W2 + c];
            re = fma(e.x, xv.x, fma(-ei, xv.y, re));
            im = fma(e.x, xv.y, fma(ei, xv.x, im));
        },
        [&](int t, double re, double im) { out[t] = make_double2(re, im); });
}

template <int KERN>
__global__ __launch_bounds__(FC_TP) void k_far_c2(FarGeom g, double sigma, double invV, const double2 *__restrict__ PH,
                                                 const double2 *__restrict__ T2, double2 *__restrict__ V1)
{
    constexpr int MI = KERN == 0 ? 1 : (KERN == 2 ? 9 : 3);
    constexpr int MO = KERN == 0 ? 1 : 3;
    extern __shared__ double2 fc_lds[];
    const int G0 = g.G[0], W0 = g.W[0], W1 = g.W[1], W2 = g.W[2], K0 = g.K[0];
    double2 *e0 = fc_lds;
    double2 *xp = e0 + G0 * (K0 + 1);  // [MI][G0]
    double2 *ch = xp + MI * G0;        // [MI][W0]
    double2 *ph = ch + MI * W0;        // [K0 + 1]
    double2 *wo = ph + (K0 + 1);       // [MO][W0]
    const int n1i = (int)blockIdx.x / W2, n2i = (int)blockIdx.x % W2;
    const int n1 = n1i - g.K[1], n2 = n2i - g.K[2];
    const int tid = threadIdx.x;
    double2 xr[FC_PRE2];  // the pencil's first values, loaded before the phase factors
#pragma unroll
    for (int u = 0; u < FC_PRE2; ++u) {
        const int t = tid + u * FC_TP;
        xr[u] = t < MI * G0 ? T2[((int64_t)t * W1 + n1i) * W2 + n2i] : make_double2(0.0, 0.0);
    }
    fill_phases<FC_TP>(g, 0, e0, tid);
#pragma unroll
    for (int u = 0; u < FC_PRE2; ++u) {
        const int t = tid + u * FC_TP;
        if (t < MI * G0) xp[t] = xr[u];
    }
    for (int t = tid + FC_PRE2 * FC_TP; t < MI * G0; t += FC_TP) xp[t] = T2[((int64_t)t * W1 + n1i) * W2 + n2i];
    // phihat and phihat' of the octant modes (|n0|, |n1|, |n2|), from k_far_c1
    {
        const int a1 = n1 < 0 ? -n1 : n1, a2 = n2 < 0 ? -n2 : n2;
        for (int a0 = tid; a0 <= K0; a0 += FC_TP) ph[a0] = PH[((int64_t)a0 * (g.K[1] + 1) + a1) * (g.K[2] + 1) + a2];
    }
    __syncthreads();
    wg_sums<FC_TP>(
        MI * W0, G0, tid,
        [&](int t, int i, double &re, double &im) {
            const int q = t / W0, n = t % W0 - K0;
            const double2 e = e0[i * (K0 + 1) + (n < 0 ? -n : n)];
            const double ei = -phase_im(e, n);
            const double2 xv = xp[q * G0 + i];
            re = fma(e.x, xv.x, fma(-ei, xv.y, re));
            im = fma(e.x, xv.y, fma(ei, xv.x, im));
        },
        [&](int t, double re, double im) { ch[t] = make_double2(invV * re, invV * im); });
    __syncthreads();
    // mode weights (as k_far_weights)
    for (int i = tid; i < W0; i += FC_TP) {
        const int n0 = i - K0;
        double2 out[MO];
        for (int j = 0; j < MO; ++j) out[j] = make_double2(0.0, 0.0);
        if (n0 != 0 || n1 != 0 || n2 != 0) {
            const double k[3] = {2.0 * M_PI * n0 / g.L[0], 2.0 * M_PI * n1 / g.L[1], 2.0 * M_PI * n2 / g.L[2]};
            const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            const double q = sqrt(k2) * sigma;
            const double2 pd = ph[n0 < 0 ? -n0 : n0];
            double2 x[MI];
            for (int c = 0; c < MI; ++c) x[c] = ch[c * W0 + i];
            mode_weight<KERN>(k, k2, q, pd.x, pd.y, x, out);
        }
        for (int j = 0; j < MO; ++j) wo[j * W0 + i] = out[j];
    }
    __syncthreads();
    wg_sums<FC_TP>(
        MO * G0, W0, tid,
        [&](int t, int i, double &re, double &im) {
            const int j = t / G0, g0 = t % G0, n = i - K0;
            const double2 e = e0[g0 * (K0 + 1) + (n < 0 ? -n : n)];
            const double ei = phase_im(e, n);
            const double2 xv = wo[j * W0 + i];
            re = fma(e.x, xv.x, fma(-ei, xv.y, re));
            im = fma(e.x, xv.y, fma(ei, xv.x, im));
        },
        [&](int t, double re, double im) { V1[((int64_t)t * W1 + n1i) * W2 + n2i] = make_double2(re, im); });
}

__global__ __launch_bounds__(FC_TS) void k_far_c3(FarGeom g, const double2 *__restrict__ V1, double *__restrict__ u)
{
    extern __shared__ double2 fc_lds[];
    const int G1 = g.G[1], G2 = g.G[2], W1 = g.W[1], W2 = g.W[2], K1 = g.K[1], K2 = g.K[2];
    double2 *e1 = fc_lds;
    double2 *e2 = e1 + G1 * (K1 + 1);
    double2 *v1 = e2 + G2 * (K2 + 1);  // [W1][W2]
    double2 *v2 = v1 + W1 * W2;        // [G1][W2]
    const int64_t a = blockIdx.x;      // j * G0 + g0
    const int tid = threadIdx.x;
    const double2 *vs = V1 + a * W1 * W2;
    double2 xr[FC_PRE2];  // the slab's first values, loaded before the phase factors
#pragma unroll
    for (int u = 0; u < FC_PRE2; ++u) {
        const int t = tid + u * FC_TS;
        xr[u] = t < W1 * W2 ? vs[t] : make_double2(0.0, 0.0);
    }
    fill_phases<FC_TS>(g, 1, e1, tid);
    fill_phases<FC_TS>(g, 2, e2, tid);
#pragma unroll
    for (int u = 0; u < FC_PRE2; ++u) {
        const int t = tid + u * FC_TS;
        if (t < W1 * W2) v1[t] = xr[u];
    }
    for (int t = tid + FC_PRE2 * FC_TS; t < W1 * W2; t += FC_TS) v1[t] = vs[t];
    __syncthreads();
    wg_sums<FC_TS>(
        G1 * W2, W1, tid,
        [&](int t, int i, double &re, double &im) {
            const int g1 = t / W2, c = t % W2, n = i - K1;
            const double2 e = e1[g1 * (K1 + 1) + (n < 0 ? -n : n)];
            const double ei = phase_im(e, n);
            const double2 xv = v1[i * W2 + c];
            re = fma(e.x, xv.x, fma(-ei, xv.y, re));
            im = fma(e.x, xv.y, fma(ei, xv.x, im));
        },
        [&](int t, double re, double im) { v2[t] = make_double2(re, im); });
    __syncthreads();
    double *out = u + a * G1 * G2;
    wg_sums<FC_TS>(
        G1 * G2, W2, tid,
        [&](int t, int i, double &re, double &im) {
            const int g1 = t / G2, g2 = t % G2, n = i - K2;
            const double2 e = e2[g2 * (K2 + 1) + (n < 0 ? -n : n)];
            const double ei = phase_im(e, n);
            const double2 xv = v2[g1 * W2 + i];
            re = fma(e.x, xv.x, fma(-ei, xv.y, re));
            (void)im;
        },
        [&](int t, double re, double im) {
            (void)im;
            out[t] = re;
        });
}

int m_in_k(int k) { return k == 0 ? 1 : (k == 2 ? 9 : 3); }
int m_out_k(int k) { return k == 0 ? 1 : 3; }

// radices 8, 4, 2, 3, 5, 7 of n into the plan's stages; n keeps the rest
void fft_factor(int &n, FftPlan &pl)
{
    static const int rads[6] = {8, 4, 2, 3, 5, 7};
    for (int k = 0; k < 6; ++k)
        while (n % rads[k] == 0 && n > 1 && pl.nst < FFT_MAXST) {
            pl.rad[pl.nst++] = rads[k];
            n /= rads[k];
        }
}

int far_geom(const dmk_far_grid *fg, FarGeom &g)
{
    if (!fg) return DMK_EINVAL;
    if (fg->p < 1 || fg->p > DMK_FAR_PMAX) return DMK_EINVAL;
    for (int i = 0; i < 3; ++i) {
        if (!(fg->L[i] > 0.0) || !isfinite(fg->L[i])) return DMK_EINVAL;
        if (fg->M[i] < 1 || fg->M[i] > DMK_FAR_MMAX) return DMK_EINVAL;
        if (fg->K[i] < 0 || fg->K[i] > DMK_FAR_KMAX) return DMK_EINVAL;
    }
    // the top cubes either tile the cell (L_i / M_i equal) or are the smallest
    // cover by cubes of the shortest side (Sec. 4.1.1): M_i = ceil(L_i / h0)
    const double h0t = fg->L[0] / fg->M[0];
    bool tiles = true;
    for (int i = 1; i < 3; ++i)
        if (fabs(fg->L[i] / fg->M[i] - h0t) > 1e-12 * h0t) tiles = false;
    const double h0 = fmin(fg->L[0], fmin(fg->L[1], fg->L[2]));
    if (!tiles)
        for (int i = 0; i < 3; ++i)
            if ((double)fg->M[i] != ceil(fg->L[i] / h0 * (1.0 - 1e-12))) return DMK_EINVAL;
    memset(&g, 0, sizeof(g));
    g.cover = tiles ? 0 : 1;
    for (int i = 0; i < 3; ++i) g.hr[i] = h0 / fg->L[i];
    g.p = fg->p;
    // The cube-index DFT on the cube grid of an exact tiling (the cubes'
    // centres at multiples of L_i / M_i), for 8 or more cubes: as an FFT from
    // FFT_MIN cubes on, below that as a dense product where it at least
    // halves the terms of the direct sums ((M^2 + W) p against W M p per
    // output column).  A factored axis keeps the phase-table rows of the first
    // cube only.
    for (int i = 0; i < 3; ++i) {
        const int64_t m = fg->M[i], w = 2 * (int64_t)fg->K[i] + 1;
        g.fac[i] = !g.cover && m >= 8 && (m >= FFT_MIN || 2 * (m * m + w) <= w * m);
        g.fft[i] = g.fac[i] && m >= FFT_MIN;
    }
    int64_t off = 0;
    for (int i = 0; i < 3; ++i) {
        g.L[i] = fg->L[i];
        g.M[i] = fg->M[i];
        g.K[i] = fg->K[i];
        g.G[i] = fg->M[i] * fg->p;
        g.W[i] = 2 * fg->K[i] + 1;
        g.rows[i] = g.fac[i] ? g.p : g.G[i];
        g.eoff[i] = off;
        off += (int64_t)g.rows[i] * g.W[i];
        g.nE += (int64_t)g.rows[i] * (g.K[i] + 1);
    }
    for (int i = 0; i < 3; ++i) {
        if (!g.fac[i]) continue;
        const int64_t m = g.M[i];
        if (!g.fft[i]) {
            g.doff[i] = off;
            off += m * m;
            g.nD += m * m;
            continue;
        }
        FftPlan &pl = g.pl[i];
        pl.n = (int)m;
        int rest = (int)m;
        fft_factor(rest, pl);
        if (rest > 1) {  // a prime factor above 8: Bluestein with a power-of-two length
            pl.n2 = 1;
            while (pl.n2 < 2 * pl.n - 1) pl.n2 *= 2;
            pl.nst = 0;
            int r2 = pl.n2;
            fft_factor(r2, pl);
        }
        const int64_t len = pl.n2 ? pl.n2 : pl.n;
        pl.twoff = off;
        off += len;
        g.nD += len;
        if (pl.n2) {
            pl.choff = off;
            off += pl.n;
            pl.hoff = off;  // h, then H = FFT(h) after it
            off += 2 * (int64_t)pl.n2;
            g.nD += pl.n2;
        }
    }
    for (int i = 0; i < 3; ++i)
        if (g.fac[i]) {
            g.foff[i] = off;
            off += (int64_t)g.p * g.W[i];
        }
    g.ntab = off;
    return DMK_OK;
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton on P_n)
void gauss_legendre01(double *x, double *w)
{
    const int n = GL_N;
    for (int k = 0; k < n; ++k) {
        double z = cos(M_PI * (k + 0.75) / (n + 0.5));
        double dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) {
                const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int m = 2; m <= n; ++m) {
            const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[k] = 0.5 * (1.0 - z);
        w[k] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2 / ((1 - z^2) P'^2) halved for [0, 1]
    }
}

inline int64_t nblk(int64_t n, int t) { return (n + t - 1) / t; }

// a dispatch holds fewer than 2^32 work-items
inline bool grid_fits(int64_t blocks, int threads) { return blocks * threads <= (int64_t)0xffffffff; }

// Workgroups per 16 x 16 output tile on the matrix cores: with fewer tiles
// than CUs the terms are split over several workgroups (partial tiles summed
// by k_mode_sum) up to about 512 workgroups, each split keeping two groups of
// 4 terms per wavefront (the 32-cube cuboid's first long-axis contraction: 114
// tiles, 31 us in one workgroup each, 24 us in five with the sum)
inline int mode_nsplit(int64_t A, int I, int O, int C)
{
    const int64_t tiles = A * ((O + 15) / 16) * ((C + 15) / 16);
    if (tiles >= 256) return 1;
    const int64_t ns = std::min<int64_t>((512 + tiles - 1) / tiles, ((I + 3) / 4) / (2 * MM_W));
    return (int)std::max<int64_t>(1, std::min<int64_t>(ns, 16));
}

// the contraction runs on the matrix cores (16 x 16 output tiles) when every
// dimension fills a tile and the grid fits
inline bool mode_on_mfma(int64_t A, int I, int O, int C)
{
    return O >= 16 && C >= 16 && I >= 16 &&
           grid_fits(A * ((O + 15) / 16) * ((C + 15) / 16) * mode_nsplit(A, I, O, C), MM_W * WAVE) &&
           grid_fits(nblk(A * O * C, 256), 256);
}

// Few terms (at most two groups of 4 per wavefront of the 8-wave form) over
// many tiles: one wavefront per tile takes all groups in order, without the
// reduction through LDS (the cube-index DFTs of short axes)
inline bool mode_one_wave(int I, int64_t tiles) { return I <= 64 && tiles >= 1024; }

// doubles2 of partial results a contraction needs (0 without a split)
inline int64_t mode_part(int64_t A, int I, int O, int C)
{
    if (!mode_on_mfma(A, I, O, C)) return 0;
    const int ns = mode_nsplit(A, I, O, C);
    return ns > 1 ? (int64_t)ns * A * O * C : 0;
}

// Blocks of the LDS form, used for the contractions along the last axis
// (C = 1), where the direct form reads X and coef with strides across the
// lanes: AB consecutive a per workgroup, up to 8 outputs per thread while the
// grid keeps 512 workgroups or more and the staged tiles stay within 16 KiB
// (more resident workgroups), so that each copy of coef serves many outputs.
inline ModeBlock mode_block(int64_t A, int I, int O, int C, bool rin)
{
    ModeBlock b;
    b.cb = 1;
    for (int64_t r = std::max<int64_t>(1, std::min<int64_t>(8, A * O / (512 * ML_T)));; --r) {
        b.ab = (int)std::min<int64_t>(A, std::max<int64_t>(1, (r * ML_T + O - 1) / O));
        b.nwg = nblk(A, b.ab);
        b.lds = sizeof(double2) * (size_t)I * O + (rin ? sizeof(double) : sizeof(double2)) * (size_t)b.ab * I;
        if (r == 1 || b.lds <= 16 * 1024) break;
    }
    (void)C;
    return b;
}

// used for C = 1 when its tiles fit and give at least one workgroup per CU
// (smaller grids are latency-bound, where the direct form does better)
inline bool mode_on_lds(int64_t A, int I, int O, int C, bool rin)
{
    if (C != 1) return false;
    const ModeBlock b = mode_block(A, I, O, C, rin);
    return b.lds <= (size_t)ML_LDS && b.nwg >= 256 && grid_fits(b.nwg, ML_T);
}

inline bool mode_fits(int64_t A, int I, int O, int C)
{
    return mode_on_mfma(A, I, O, C) || mode_on_lds(A, I, O, C, false) || grid_fits(nblk(A * O * C, 256), 256);
}

// Returns 1, or (defer_sum) the number of split partial results left in part
// for the consumer to add up (k_mode_sum's order and scale) instead of Y.
template <bool RIN, bool ROUT, bool CONJ>
int mode(const void *X, const double2 *E, int64_t A, int I, int O, int C, int64_t si, int64_t so, double s, void *Y,
         double2 *part, hipStream_t st, bool defer_sum = false)
{
    const int64_t n = A * O * C;
    if (n <= 0) return 1;
    if (mode_on_mfma(A, I, O, C)) {
        // 16 x 16 output tiles on the matrix cores, nsplit workgroups each
        const int64_t tiles = A * ((O + 15) / 16) * ((C + 15) / 16);
        const int ns = mode_nsplit(A, I, O, C);
        if (ns == 1 && mode_one_wave(I, tiles)) {
            hipLaunchKernelGGL((k_mode_mfma<RIN, ROUT, CONJ, 1>), dim3((unsigned)tiles), dim3(WAVE), 0, st, X, E, A, I,
                               O, C, si, so, s, 1, part, Y);
            return 1;
        }
        hipLaunchKernelGGL((k_mode_mfma<RIN, ROUT, CONJ>), dim3((unsigned)(tiles * ns)), dim3(MM_W * WAVE), 0, st, X,
                           E, A, I, O, C, si, so, s, ns, part, Y);
        if (ns > 1 && defer_sum) return ns;
        if (ns > 1)
            hipLaunchKernelGGL((k_mode_sum<ROUT>), dim3((unsigned)nblk(n, 256)), dim3(256), 0, st, part, n, ns, s, Y);
        return 1;
    }
    if (mode_on_lds(A, I, O, C, RIN)) {
        const ModeBlock b = mode_block(A, I, O, C, RIN);
        hipLaunchKernelGGL((k_mode_lds<RIN, ROUT, CONJ>), dim3((unsigned)b.nwg), dim3(ML_T), b.lds, st, X, E, A, I, O,
                           C, si, so, s, b.ab, b.cb, Y);
        return 1;
    }
    hipLaunchKernelGGL((k_mode<RIN, ROUT, CONJ>), dim3((unsigned)nblk(n, 256)), dim3(256), 0, st, X, E, A, I, O, C, si, so, s,
                       Y);
    return 1;
}

// ---- FFT launches
template <bool INM, bool OUTM>
void fft_stage_launch(int R, const void *in, void *out, int64_t A, int N, int ncol, int S, int sg,
                      const double2 *tw, double scale, hipStream_t st)
{
    const dim3 grid((unsigned)nblk(A * (N / R) * (int64_t)ncol, 256)), blk(256);
    switch (R) {
    case 2: hipLaunchKernelGGL((k_fft_stage<2, INM, OUTM>), grid, blk, 0, st, in, out, A, N, ncol, S, sg, tw, scale); break;
    case 3: hipLaunchKernelGGL((k_fft_stage<3, INM, OUTM>), grid, blk, 0, st, in, out, A, N, ncol, S, sg, tw, scale); break;
    case 4: hipLaunchKernelGGL((k_fft_stage<4, INM, OUTM>), grid, blk, 0, st, in, out, A, N, ncol, S, sg, tw, scale); break;
    case 5: hipLaunchKernelGGL((k_fft_stage<5, INM, OUTM>), grid, blk, 0, st, in, out, A, N, ncol, S, sg, tw, scale); break;
    case 7: hipLaunchKernelGGL((k_fft_stage<7, INM, OUTM>), grid, blk, 0, st, in, out, A, N, ncol, S, sg, tw, scale); break;
    default: hipLaunchKernelGGL((k_fft_stage<8, INM, OUTM>), grid, blk, 0, st, in, out, A, N, ncol, S, sg, tw, scale); break;
    }
}

// The stages of a length-N transform (stages rad[0 .. nst)) on [A][N][ncol]:
// stage 0 reads `in` (real if rin), the last writes `out` (real part if rout;
// when out is null, the result stays in a scratch buffer), the ones between
// alternate between bufA and bufB (never the buffer they read).  Returns the
// buffer that holds the result.
void *fft_stages(const FftPlan &pl, int N, const double2 *tw, const void *in, bool rin, void *out, bool rout,
                 int64_t A, int ncol, int sg, double scale, double2 *bufA, double2 *bufB, hipStream_t st)
{
    const void *cur = in;
    int S = 1;
    for (int k = 0; k < pl.nst; ++k) {
        const bool last = k == pl.nst - 1;
        void *dst = (last && out) ? out : (cur == (const void *)bufA ? (void *)bufB : (void *)bufA);
        const bool ri = k == 0 && rin, ro = last && rout && out;
        const double sc = last ? scale : 1.0;
        if (ri && ro) fft_stage_launch<true, true>(pl.rad[k], cur, dst, A, N, ncol, S, sg, tw, sc, st);
        else if (ri) fft_stage_launch<true, false>(pl.rad[k], cur, dst, A, N, ncol, S, sg, tw, sc, st);
        else if (ro) fft_stage_launch<false, true>(pl.rad[k], cur, dst, A, N, ncol, S, sg, tw, sc, st);
        else fft_stage_launch<false, false>(pl.rad[k], cur, dst, A, N, ncol, S, sg, tw, sc, st);
        S *= pl.rad[k];
        cur = dst;
    }
    return (void *)cur;
}

// Y[a][r][c] = sum_b exp(sg 2 pi i r b / M) X[a][b][c] over the cube index of
// axis ax (X real if RIN; only Re(Y) stored if ROUT), via the axis' plan
template <bool RIN, bool ROUT>
void fft_cube(const FarGeom &g, int ax, const double2 *E, const void *X, void *Y, int64_t A, int ncol, int sg,
              double2 *bufA, double2 *bufB, hipStream_t st)
{
    const FftPlan &pl = g.pl[ax];
    const double2 *tw = E + pl.twoff;
    if (!pl.n2) {
        fft_stages(pl, pl.n, tw, X, RIN, Y, ROUT, A, ncol, sg, 1.0, bufA, bufB, st);
        return;
    }
    const double2 *ch = E + pl.choff, *H = E + pl.hoff + pl.n2;
    const int64_t n2c = A * pl.n2 * (int64_t)ncol;
    hipLaunchKernelGGL((k_blue_in<RIN>), dim3((unsigned)nblk(n2c, 256)), dim3(256), 0, st, X, bufA, A, pl.n, pl.n2,
                       ncol, sg, ch);
    double2 *P = (double2 *)fft_stages(pl, pl.n2, tw, bufA, false, nullptr, false, A, ncol, -1, 1.0, bufA, bufB, st);
    hipLaunchKernelGGL(k_blue_mul, dim3((unsigned)nblk(n2c, 256)), dim3(256), 0, st, P, A, pl.n2, ncol, H);
    double2 *Q = (double2 *)fft_stages(pl, pl.n2, tw, P, false, nullptr, false, A, ncol, 1, 1.0, bufA, bufB, st);
    hipLaunchKernelGGL((k_blue_out<ROUT>), dim3((unsigned)nblk(A * pl.n * (int64_t)ncol, 256)), dim3(256), 0, st, Q,
                       Y, A, pl.n, pl.n2, ncol, sg, ch, 1.0 / pl.n2);
}

// H = FFT(h) (sign -1) of every Bluestein axis, after the set-up kernel
void fft_bluestein_tables(const FarGeom &g, double2 *E, double2 *bufA, double2 *bufB, hipStream_t st)
{
    for (int ax = 0; ax < 3; ++ax) {
        if (!g.fft[ax] || !g.pl[ax].n2) continue;
        const FftPlan &pl = g.pl[ax];
        fft_stages(pl, pl.n2, E + pl.twoff, E + pl.hoff, false, E + pl.hoff + pl.n2, false, 1, 1, -1, 1.0, bufA, bufB,
                   st);
    }
}

// launch sizes of the FFT of axis ax on [A][M][ncol]
inline bool fft_fits(const FarGeom &g, int ax, int64_t A, int64_t ncol)
{
    const FftPlan &pl = g.pl[ax];
    const int64_t len = pl.n2 ? pl.n2 : pl.n;
    return grid_fits(nblk(A * len * ncol, 256), 256);
}

// complex scratch of the FFT of axis ax on [A][M][ncol] (each of two buffers)
inline int64_t fft_scratch(const FarGeom &g, int ax, int64_t A, int64_t ncol)
{
    if (!g.fft[ax]) return 0;
    const FftPlan &pl = g.pl[ax];
    return A * (int64_t)(pl.n2 ? pl.n2 : pl.n) * ncol;
}

// The three contractions of each side, axis ax: A leading and C trailing
// columns around the contracted index, input Q (forward) or J (evaluation)
// components.
struct AxisCols {
    int64_t A;
    int C;
};

inline AxisCols axis_cols(const FarGeom &g, int ax, int64_t comps)
{
    // forward: axis 2 on [q][g0][g1][g2], axis 1 on [q][g0][g1][n2], axis 0 on [q][g0][n1][n2];
    // evaluation: axis 0 on [j][n0][n1][n2], axis 1 on [j][g0][n1][n2], axis 2 on [j][g0][g1][n2]
    const int64_t G0 = g.G[0], G1 = g.G[1];
    const int W1 = g.W[1], W2 = g.W[2];
    if (ax == 2) return {comps * G0 * G1, 1};
    if (ax == 1) return {comps * G0, W2};
    return {comps, W1 * W2};
}

// Launch sizes of one contraction (direct, or the DFT and the fold / unfold)
inline bool axis_fits(const FarGeom &g, int ax, int64_t comps, bool fwd)
{
    const AxisCols ac = axis_cols(g, ax, comps);
    const int G = g.G[ax], W = g.W[ax], M = g.M[ax];
    if (!g.fac[ax]) return fwd ? mode_fits(ac.A, G, W, ac.C) : mode_fits(ac.A, W, G, ac.C);
    const int64_t pc = (int64_t)g.p * ac.C;
    if (pc > INT32_MAX) return false;
    const bool dft = g.fft[ax] ? fft_fits(g, ax, ac.A, pc) : mode_fits(ac.A, M, M, (int)pc);
    return dft && grid_fits(nblk(ac.A * W * ac.C, 256), 256) && grid_fits(nblk(ac.A * G * ac.C, 256), 256);
}

// doubles2 of split partials and of the DFT's output a contraction needs
inline int64_t axis_part(const FarGeom &g, int ax, int64_t comps, bool fwd)
{
    const AxisCols ac = axis_cols(g, ax, comps);
    if (!g.fac[ax]) return fwd ? mode_part(ac.A, g.G[ax], g.W[ax], ac.C) : mode_part(ac.A, g.W[ax], g.G[ax], ac.C);
    if (g.fft[ax]) return 0;
    return mode_part(ac.A, g.M[ax], g.M[ax], g.p * ac.C);
}

inline int64_t axis_z(const FarGeom &g, int ax, int64_t comps)
{
    const AxisCols ac = axis_cols(g, ax, comps);
    return g.fac[ax] ? ac.A * g.G[ax] * ac.C : 0;
}

// the fold of one column (C = 1) stages Z[a] in LDS when it fits
inline bool fold_on_lds(const FarGeom &g, int ax, const AxisCols &ac)
{
    return ac.C == 1 && (int64_t)g.M[ax] * g.p * (int64_t)sizeof(double2) <= FL_LDS && grid_fits(ac.A, FL_T);
}

// One contraction of the structure factor along axis ax (conj(E)), scaled by s.
// Returns mode()'s count of deferred partial results (1 when written to Y).
template <bool RIN>
int contract_fwd(const FarGeom &g, int ax, int64_t comps, const void *X, const double2 *E, double s, double2 *Y,
                 double2 *Z, double2 *part, double2 *fa, double2 *fb, hipStream_t st, bool defer_sum = false)
{
    const AxisCols ac = axis_cols(g, ax, comps);
    const int W = g.W[ax];
    if (!g.fac[ax])
        return mode<RIN, false, true>(X, E + g.eoff[ax], ac.A, g.G[ax], W, ac.C, W, 1, s, Y, part, st, defer_sum);
    const int M = g.M[ax];
    if (g.fft[ax])
        fft_cube<RIN, false>(g, ax, E, X, Z, ac.A, g.p * ac.C, -1, fa, fb, st);
    else
        mode<RIN, false, true>(X, E + g.doff[ax], ac.A, M, M, g.p * ac.C, M, 1, 1.0, Z, part, st);
    if (fold_on_lds(g, ax, ac))
        hipLaunchKernelGGL(k_fold_lds<true>, dim3((unsigned)ac.A), dim3(FL_T), (size_t)M * g.p * sizeof(double2), st, Z,
                           E + g.eoff[ax], M, g.p, W, g.K[ax], s, Y);
    else
        hipLaunchKernelGGL(k_fold<true>, dim3((unsigned)nblk(ac.A * W * ac.C, 256)), dim3(256), 0, st, Z,
                           E + g.eoff[ax], ac.A, M, g.p, W, g.K[ax], ac.C, s, Y);
    return 1;
}

// One contraction of the evaluation along axis ax (E); ROUT: real part only
template <bool ROUT>
void contract_eval(const FarGeom &g, int ax, int64_t comps, const double2 *X, const double2 *E, void *Y, double2 *Z,
                   double2 *part, double2 *fa, double2 *fb, hipStream_t st)
{
    const AxisCols ac = axis_cols(g, ax, comps);
    const int W = g.W[ax];
    if (!g.fac[ax]) {
        mode<false, ROUT, false>(X, E + g.eoff[ax], ac.A, W, g.G[ax], ac.C, 1, W, 1.0, Y, part, st);
        return;
    }
    const int M = g.M[ax];
    hipLaunchKernelGGL(k_unfold, dim3((unsigned)nblk(ac.A * g.G[ax] * ac.C, 256)), dim3(256), 0, st, X,
                       E + g.foff[ax], ac.A, M, g.p, W, g.K[ax], ac.C, Z);
    if (g.fft[ax])
        fft_cube<false, ROUT>(g, ax, E, Z, Y, ac.A, g.p * ac.C, 1, fa, fb, st);
    else
        mode<false, ROUT, false>(Z, E + g.doff[ax], ac.A, M, M, g.p * ac.C, M, 1, 1.0, Y, part, st);
}

// LDS bytes of the three compact kernels, or 0 where the compact form does
// not apply (an axis factored over the cube index)
struct FarCompact {
    size_t l1, l2, l3;
};

inline FarCompact far_compact(const FarGeom &g, int64_t Q, int64_t J)
{
    FarCompact c{0, 0, 0};
    for (int ax = 0; ax < 3; ++ax)
        if (g.fac[ax]) return c;
    const size_t z = sizeof(double2);
    const size_t G0 = g.G[0], G1 = g.G[1], G2 = g.G[2], W0 = g.W[0], W1 = g.W[1], W2 = g.W[2];
    const size_t k0 = g.K[0] + 1, k1 = g.K[1] + 1, k2 = g.K[2] + 1;
    const size_t l1 = z * (G2 * k2 + G1 * k1 + G1 * W2) + sizeof(double) * G1 * G2;
    const size_t l2 = z * (G0 * k0 + Q * G0 + Q * W0 + k0 + J * W0);
    const size_t l3 = z * (G1 * k1 + G2 * k2 + W1 * W2 + G1 * W2);
    if (l1 > FC_LDS || l2 > FC_LDS || l3 > FC_LDS) return c;
    const int64_t nom = (int64_t)k0 * k1 * k2;  // octant modes, one wavefront each beside the slabs
    if (!grid_fits(Q * (int64_t)G0 + nblk(nom, FC_TS / WAVE), FC_TS) || !grid_fits((int64_t)W1 * W2, FC_TP) ||
        !grid_fits(J * (int64_t)G0, FC_TS))
        return c;
    c.l1 = l1;
    c.l2 = l2;
    c.l3 = l3;
    return c;
}

struct FarLayout {
    int64_t E, T1, T2, CHI, WT, V1, V2, PH, PART, Z, FA, FB, total;  // byte offsets
};

FarLayout far_layout(const FarGeom &g, int kernel)
{
    const int64_t Q = m_in_k(kernel), J = m_out_k(kernel);
    const int64_t G0 = g.G[0], G1 = g.G[1], W0 = g.W[0], W1 = g.W[1], W2 = g.W[2];
    auto al = [](int64_t v) { return (v + 255) & ~(int64_t)255; };
    FarLayout l{};
    int64_t off = 0;
    const int64_t z = (int64_t)sizeof(double2);
    l.E = off;
    // phase tables, DFT / FFT tables (Bluestein's H included), transposed first-cube rows
    off = al(off + z * g.ntab);
    l.T1 = off;
    off = al(off + z * Q * G0 * G1 * W2);
    l.T2 = off;
    off = al(off + z * Q * G0 * W1 * W2);
    l.CHI = off;
    off = al(off + z * Q * W0 * W1 * W2);
    l.WT = off;
    off = al(off + z * J * W0 * W1 * W2);
    l.V1 = off;
    off = al(off + z * J * G0 * W1 * W2);
    l.V2 = off;
    off = al(off + z * J * G0 * G1 * W2);
    l.PH = off;
    off = al(off + z * (int64_t)(g.K[0] + 1) * (g.K[1] + 1) * (g.K[2] + 1));
    // partial results of the split contractions (the six of dmk_far3p_eval)
    // and the cube-index DFTs' outputs
    int64_t np = 0, nz = 0, nf = 0;
    for (int ax = 0; ax < 3; ++ax) {
        np = std::max({np, axis_part(g, ax, Q, true), axis_part(g, ax, J, false)});
        nz = std::max({nz, axis_z(g, ax, Q), axis_z(g, ax, J)});
        if (g.fft[ax]) {
            const AxisCols aq = axis_cols(g, ax, Q), aj = axis_cols(g, ax, J);
            nf = std::max({nf, fft_scratch(g, ax, aq.A, (int64_t)g.p * aq.C), fft_scratch(g, ax, aj.A, (int64_t)g.p * aj.C)});
            if (g.pl[ax].n2) nf = std::max<int64_t>(nf, g.pl[ax].n2);
        }
    }
    l.PART = off;
    off = al(off + z * np);
    l.Z = off;
    off = al(off + z * nz);
    l.FA = off;
    off = al(off + z * nf);
    l.FB = off;
    off = al(off + z * nf);
    l.total = off;
    return l;
}

}  // namespace
}  // namespace dmk

using namespace dmk;

extern "C" size_t dmk_far3p_ws_bytes(const dmk_far_grid *fg, int kernel)
{
    FarGeom g;
    if (far_geom(fg, g) != DMK_OK || kernel < 0 || kernel > 3) return 0;
    return (size_t)far_layout(g, kernel).total;
}

extern "C" int dmk_far3p_eval(const dmk_far_grid *fg, int kernel, double sigma0, const dmk_pswf *win,
                              const double *rho_grid, double *u_grid, void *ws, size_t ws_bytes, hipStream_t stream)
{
    FarGeom g;
    int st = far_geom(fg, g);
    if (st != DMK_OK) return st;
    if (kernel < 0 || kernel > 3) return DMK_EINVAL;
    if (!(sigma0 > 0.0) || !isfinite(sigma0)) return DMK_ECUTOFF;
    if (!rho_grid || !u_grid || !ws) return DMK_EINVAL;
    FarWin w;
    memset(&w, 0, sizeof(w));
    w.sigma = sigma0;
    if (win) {
        if (!(win->c > 0.0) || !(win->c <= DMK_PSWF_CMAX) || win->nterms64 < 1 ||
            win->nterms64 > DMK_PSWF_MAXTERMS)
            return DMK_EUNSUPPORTED;
        w.pswf = 1;
        w.nterms = win->nterms64;
        w.c = win->c;
        // the terms past nterms64 are zero here, so that the kernels' fixed-
        // length recurrence equals the nterms64-term sum exactly
        for (int m = 0; m < DMK_PSWF_MAXTERMS; ++m) {
            w.cheb[m] = m < w.nterms ? win->cheb[0][m] : 0.0;
            w.dcheb[m] = m < w.nterms ? win->cheb[2][m] : 0.0;
        }
        gauss_legendre01(w.gx, w.gw);
        // the quadrature grows with |k| sigma: bound it
        double kk = 0.0;
        for (int i = 0; i < 3; ++i) {
            const double ki = 2.0 * M_PI * g.K[i] / g.L[i];
            kk += ki * ki;
        }
        if (sqrt(kk) * sigma0 > 4096.0) return DMK_EUNSUPPORTED;
    }
    // launch sizes: every dispatch of the evaluation below holds fewer than 2^32 work-items
    {
        const int64_t Q = m_in_k(kernel), J = m_out_k(kernel);
        const int64_t W1 = g.W[1], W2 = g.W[2];
        const int64_t ne = g.nE + g.nD;
        const int64_t no = (int64_t)(g.K[0] + 1) * (g.K[1] + 1) * (g.K[2] + 1);
        const int64_t nm = (int64_t)g.W[0] * W1 * W2;
        if (!grid_fits((int64_t)nblk(ne, PREP_T) + (int64_t)nblk(no, PREP_T / WAVE), PREP_T) ||
            !grid_fits(nblk(nm, FW_T), FW_T))
            return DMK_ESIZE;
        for (int ax = 0; ax < 3; ++ax)
            if (!axis_fits(g, ax, Q, true) || !axis_fits(g, ax, J, false)) return DMK_ESIZE;
    }
    const FarLayout l = far_layout(g, kernel);
    if (ws_bytes < (size_t)l.total) return DMK_ESIZE;
    char *b = (char *)ws;
    double2 *E = (double2 *)(b + l.E);
    double2 *T1 = (double2 *)(b + l.T1), *T2 = (double2 *)(b + l.T2), *CHI = (double2 *)(b + l.CHI);
    double2 *WT = (double2 *)(b + l.WT), *V1 = (double2 *)(b + l.V1), *V2 = (double2 *)(b + l.V2);
    double2 *PH = (double2 *)(b + l.PH), *PART = (double2 *)(b + l.PART), *Z = (double2 *)(b + l.Z);
    double2 *FA = (double2 *)(b + l.FA), *FB = (double2 *)(b + l.FB);
    const int64_t Q = m_in_k(kernel), J = m_out_k(kernel);
    const int W0 = g.W[0], W1 = g.W[1], W2 = g.W[2];
    const double invV = 1.0 / (g.L[0] * g.L[1] * g.L[2]);

    // small grids: three launches, each workgroup holding its share in LDS
    const FarCompact fc = far_compact(g, Q, J);
    if (fc.l1) {
        // the slabs, and beside them the octant table of the window's transform
        const unsigned nslab = (unsigned)(Q * g.G[0]);
        const int64_t nom = (int64_t)(g.K[0] + 1) * (g.K[1] + 1) * (g.K[2] + 1);
        hipLaunchKernelGGL(k_far_c1, dim3(nslab + (unsigned)nblk(nom, FC_TS / WAVE)), dim3(FC_TS), fc.l1, stream, g,
                           rho_grid, T2, w, PH, nslab);
        const dim3 gp((unsigned)((int64_t)W1 * W2));
        switch (kernel) {
        case 0: hipLaunchKernelGGL(k_far_c2<0>, gp, dim3(FC_TP), fc.l2, stream, g, sigma0, invV, PH, T2, V1); break;
        case 1: hipLaunchKernelGGL(k_far_c2<1>, gp, dim3(FC_TP), fc.l2, stream, g, sigma0, invV, PH, T2, V1); break;
        case 2: hipLaunchKernelGGL(k_far_c2<2>, gp, dim3(FC_TP), fc.l2, stream, g, sigma0, invV, PH, T2, V1); break;
        default: hipLaunchKernelGGL(k_far_c2<3>, gp, dim3(FC_TP), fc.l2, stream, g, sigma0, invV, PH, T2, V1); break;
        }
        hipLaunchKernelGGL(k_far_c3, dim3((unsigned)(J * g.G[0])), dim3(FC_TS), fc.l3, stream, g, V1, u_grid);
        DMK_HIP_CHECK(hipGetLastError());
        return DMK_OK;
    }
    const int64_t ne = g.nE + g.nD;
    const int64_t no = (int64_t)(g.K[0] + 1) * (g.K[1] + 1) * (g.K[2] + 1);
    const unsigned nbt = (unsigned)nblk(ne, PREP_T);
    hipLaunchKernelGGL(k_far_prep, dim3(nbt + (unsigned)nblk(no, PREP_T / WAVE)), dim3(PREP_T), 0, stream, g, w, E, PH, nbt);
    fft_bluestein_tables(g, E, FA, FB, stream);
    // structure factor (eq. (structurefac)): contract g2, g1, g0 with conj(E)
    contract_fwd<true>(g, 2, Q, rho_grid, E, 1.0, T1, Z, PART, FA, FB, stream);
    contract_fwd<false>(g, 1, Q, T1, E, 1.0, T2, Z, PART, FA, FB, stream);
    const int ns_chi = contract_fwd<false>(g, 0, Q, T2, E, invV, CHI, Z, PART, FA, FB, stream, true);
    // mode weights (with the window's transform per octant mode from k_far_prep)
    const int64_t nm = (int64_t)W0 * W1 * W2;
    const dim3 gw((unsigned)nblk(nm, FW_T));
    switch (kernel) {
    case 0: hipLaunchKernelGGL(k_far_weights<0>, gw, dim3(FW_T), 0, stream, g, sigma0, PH, CHI, PART, ns_chi, invV, WT); break;
    case 1: hipLaunchKernelGGL(k_far_weights<1>, gw, dim3(FW_T), 0, stream, g, sigma0, PH, CHI, PART, ns_chi, invV, WT); break;
    case 2: hipLaunchKernelGGL(k_far_weights<2>, gw, dim3(FW_T), 0, stream, g, sigma0, PH, CHI, PART, ns_chi, invV, WT); break;
    default: hipLaunchKernelGGL(k_far_weights<3>, gw, dim3(FW_T), 0, stream, g, sigma0, PH, CHI, PART, ns_chi, invV, WT); break;
    }
    // evaluation on the grids (eq. (eval_tensor)): contract n0, n1, n2 with E
    contract_eval<false>(g, 0, J, WT, E, V1, Z, PART, FA, FB, stream);
    contract_eval<false>(g, 1, J, V1, E, V2, Z, PART, FA, FB, stream);
    contract_eval<true>(g, 2, J, V2, E, u_grid, Z, PART, FA, FB, stream);
    DMK_HIP_CHECK(hipGetLastError());
    return DMK_OK;
}
