// dmk_cheb.hip -- leaf-box Chebyshev grids on gfx950.
//
// Every box of the tiling carries a p x p x p grid of first-kind Chebyshev
// points (Sec. 3.1, upward pass).  This file provides
//   * anterpolation (upward pass): proxy strengths on the grid of each box,
//     rho~_q(j) = sum_{a in box} rho_{a,q} l_j(x_a);
//   * leaf evaluation (downward pass, last step): u_q(x) = sum_j U_q(j) l_j(x)
//     for the targets x of each box;
//   * the self-interaction correction of the split (Sec. 2.4): the far field
//     includes the k-space image of a point's own mollified kernel, removed by
//     u -= phi(0) rho / (2 pi sigma0) for the harmonic kernel and the
//     Stokeslet.
// l_j is the tensor-product Lagrange basis of the box's grid in box-local
// coordinates t = 2 (y n / L - b) - 1, evaluated with the barycentric formula
// for first-kind Chebyshev points (weights (-1)^k sin((2k+1) pi / (2p))).
// Grid values of all boxes form one tensor [m][n0 p][n1 p][n2 p] (index
// g_i = b_i p + j_i), the layout of the root-level far field.
//
// Points are taken in the binning's sorted order (box ranges from box_start),
// so a box's points are contiguous; results go to the original order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>

#include "dmk_internal.h"

namespace dmk {
namespace {

struct ChebGeom {
    double inv[3];  // n_i / L_i, as in the binning
    int n[3];
    int p;
    int64_t N;
    int64_t G[3];   // n_i p
    int64_t wg0;    // first workgroup of this launch (per-box kernels, launched in chunks)
};

constexpr int CB_T = 256;
// workgroups of one launch (fewer than 2^32 work-items)
constexpr int64_t MAX_WG = 0xffffffffu / CB_T;

// accumulator tile of v_mfma_f64_16x16x4 (4 doubles per lane)
typedef double dbl4 __attribute__((ext_vector_type(4)));

// LDS stores of a wavefront made visible to all its lanes, in order (no
// other wavefront touches the same region)
__device__ inline void wave_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// l_j(t_ax(s)) for the sorted points s, stored node-fastest lag[s][ax][j]
// (anterpolation: the lanes of a wavefront are consecutive nodes of one point)
// or point-fastest lag[ax][j][s] (PT; evaluation: the lanes are consecutive
// points)
template <bool PT>
__global__ __launch_bounds__(CB_T) void k_cheb_lagrange(ChebGeom g, const double *__restrict__ ys,
                                                        const int32_t *__restrict__ skey, double *__restrict__ lag)
{
    __shared__ double eta[DMK_FAR_PMAX], wb[DMK_FAR_PMAX];
    const int p = g.p;
    for (int k = threadIdx.x; k < p; k += CB_T) {
        const double a = (double)(2 * k + 1) / (double)(2 * p);
        eta[k] = cospi(a);
        wb[k] = (k & 1) ? -sinpi(a) : sinpi(a);
    }
    __syncthreads();
    const int64_t e = (int64_t)blockIdx.x * CB_T + threadIdx.x;
    if (e >= 3 * g.N) return;
    const int64_t s = e / 3;
    const int ax = (int)(e % 3);
    const int key = skey[s];
    const int b = ax == 0 ? key / (g.n[1] * g.n[2]) : (ax == 1 ? (key / g.n[2]) % g.n[1] : key % g.n[2]);
    const double t = 2.0 * (ys[(int64_t)ax * g.N + s] * g.inv[ax] - (double)b) - 1.0;
    double *out = PT ? lag + (int64_t)ax * p * g.N + s : lag + (s * 3 + ax) * p;
    const int64_t st = PT ? g.N : 1;
    int hit = -1;
    double S = 0.0;
    for (int k = 0; k < p; ++k) {
        const double d = t - eta[k];
        if (d == 0.0) hit = k;
        S += wb[k] / (d == 0.0 ? 1.0 : d);
    }
    if (hit >= 0) {
        for (int k = 0; k < p; ++k) out[k * st] = k == hit ? 1.0 : 0.0;
        return;
    }
    const double iS = 1.0 / S;
    for (int k = 0; k < p; ++k) out[k * st] = wb[k] / (t - eta[k]) * iS;
}

// rho_grid[q][g0][g1][g2] = sum over the points s of box (g0/p, g1/p, g2/p)
// of rho[perm[s]][q] l_{g0%p} l_{g1%p} l_{g2%p}.  A workgroup takes CB_NODES
// nodes of one box; the box's points are staged in LDS in chunks of `ch`
// (l0, l1 and l2 * rho per point), and every thread sums over a chunk for its
// nodes.  More than one chunk: the first writes, later ones add (the same
// thread owns a node throughout, so there are no races).
constexpr int CB_NODES = 2048;

template <int M>
__global__ __launch_bounds__(CB_T) void k_cheb_anterp(ChebGeom g, int ch, int nsplit, const int32_t *__restrict__ bs,
                                                      const int32_t *__restrict__ perm,
                                                      const double *__restrict__ lag, const double *__restrict__ rho,
                                                      double *__restrict__ rg)
{
    extern __shared__ double sm[];
    const int p = g.p;
    const int64_t wg = g.wg0 + blockIdx.x;
    const int64_t box = wg / nsplit;
    const int part = (int)(wg - box * nsplit);
    const int64_t b0 = box / ((int64_t)g.n[1] * g.n[2]), b1 = (box / g.n[2]) % g.n[1], b2 = box % g.n[2];
    const int64_t tot = g.G[0] * g.G[1] * g.G[2];
    const int nn = p * p * p;
    const int e0 = part * CB_NODES, e1 = min(nn, e0 + CB_NODES);
    double *L0 = sm, *L1 = sm + ch * p, *Cq = sm + 2 * ch * p;
    const int sb = bs[box], se = bs[box + 1];
    const int npass = max(1, (se - sb + ch - 1) / ch);
    for (int ps = 0; ps < npass; ++ps) {
        const int c0 = sb + ps * ch;
        const int nc = max(0, min(ch, se - c0));
        __syncthreads();  // the previous chunk is no longer read
        for (int e = threadIdx.x; e < nc * p; e += CB_T) {
            const int si = e / p, j = e - si * p;
            const int64_t s = c0 + si;
            const double *l = lag + s * 3 * p;
            L0[si * p + j] = l[j];
            L1[si * p + j] = l[p + j];
            const double l2 = l[2 * p + j];
            const int64_t i = perm[s];
#pragma unroll
            for (int q = 0; q < M; ++q) Cq[(q * ch + si) * p + j] = l2 * rho[i * M + q];
        }
        __syncthreads();
        for (int e = e0 + threadIdx.x; e < e1; e += CB_T) {
            const int j0 = e / (p * p), j1 = (e / p) % p, j2 = e % p;
            double acc[M];
#pragma unroll
            for (int q = 0; q < M; ++q) acc[q] = 0.0;
            for (int si = 0; si < nc; ++si) {
                const double w = L0[si * p + j0] * L1[si * p + j1];
#pragma unroll
                for (int q = 0; q < M; ++q) acc[q] = fma(w, Cq[(q * ch + si) * p + j2], acc[q]);
            }
            const int64_t idx = ((b0 * p + j0) * g.G[1] + (b1 * p + j1)) * g.G[2] + b2 * p + j2;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                if (ps == 0)
                    rg[q * tot + idx] = acc[q];
                else
                    rg[q * tot + idx] += acc[q];
            }
        }
    }
}

// The same anterpolation as a dense contraction on the FP64 matrix cores,
// for boxes holding many points: per box,
//   rho~_q[j0][(j1, j2)] = sum_s l0(s, j0) * (l1(s, j1) l2(s, j2) rho_q(s)),
// a (p x N_b) by (N_b x p^2) product.  Each wavefront owns NT 16 x 16 tiles
// of (j0, (j1, j2)) in one row of tiles (sharing the A fragment) and adds 4
// points per v_mfma_f64_16x16x4 from the LDS chunk (lane layout as in
// k_cheb_eval_mfma); the workgroups of a box share its tiles.

template <int M>
struct AnterpTiles {
    static constexpr int NT = M == 1 ? 4 : (M == 3 ? 2 : 1);  // tiles per wavefront
};

template <int M>
__global__ __launch_bounds__(CB_T) void k_cheb_anterp_mfma(ChebGeom g, int ch, int nsplit,
                                                           const int32_t *__restrict__ bs,
                                                           const int32_t *__restrict__ perm,
                                                           const double *__restrict__ lag,
                                                           const double *__restrict__ rho, double *__restrict__ rg)
{
    constexpr int NT = AnterpTiles<M>::NT;
    extern __shared__ double sm[];
    const int p = g.p;
    const int64_t wg = g.wg0 + blockIdx.x;
    const int64_t box = wg / nsplit;
    const int part = (int)(wg - box * nsplit);
    const int64_t b0 = box / ((int64_t)g.n[1] * g.n[2]), b1 = (box / g.n[2]) % g.n[1], b2 = box % g.n[2];
    const int64_t tot = g.G[0] * g.G[1] * g.G[2];
    const int pp = p * p;
    const int ntn = (pp + 15) / 16;            // column tiles
    const int ngn = (ntn + NT - 1) / NT;       // groups of NT column tiles
    const int ngroup = ((p + 15) / 16) * ngn;
    const int lane = threadIdx.x & (WAVE - 1);
    const int grp = part * (CB_T / WAVE) + threadIdx.x / WAVE;
    const bool active = grp < ngroup;  // uniform per wavefront
    const int tj = active ? grp / ngn : 0, tn0 = active ? (grp - (grp / ngn) * ngn) * NT : 0;
    const int li = lane & 15, lk = lane >> 4;
    const int j0a = tj * 16 + li;  // A row of this lane
    int j1[NT], j2[NT];
    bool nok[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int n = (tn0 + t) * 16 + li;  // B / D column of this lane in tile t
        nok[t] = n < pp;
        j1[t] = nok[t] ? n / p : 0;
        j2[t] = nok[t] ? n - (n / p) * p : 0;
    }
    double *L0 = sm, *L1 = sm + ch * p, *Cq = sm + 2 * ch * p;
    const int sb = bs[box], se = bs[box + 1];
    const int npass = max(1, (se - sb + ch - 1) / ch);
    for (int ps = 0; ps < npass; ++ps) {
        const int c0 = sb + ps * ch;
        const int nc = max(0, min(ch, se - c0));
        __syncthreads();  // the previous chunk is no longer read
        for (int e = threadIdx.x; e < nc * p; e += CB_T) {
            const int si = e / p, j = e - si * p;
            const int64_t s = c0 + si;
            const double *l = lag + s * 3 * p;
            L0[si * p + j] = l[j];
            L1[si * p + j] = l[p + j];
            const double l2 = l[2 * p + j];
            const int64_t i = perm[s];
#pragma unroll
            for (int q = 0; q < M; ++q) Cq[(q * ch + si) * p + j] = l2 * rho[i * M + q];
        }
        __syncthreads();
        if (!active) continue;
        dbl4 d[NT][M];
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int q = 0; q < M; ++q) d[t][q] = (dbl4){0.0, 0.0, 0.0, 0.0};
        // straight-line body: every LDS read at an index clamped into the
        // staged chunk, the unused values replaced by zero with selects (so
        // that the accumulators stay in the matrix-core registers)
        const int j0c = j0a < p ? j0a : 0;
        for (int k0 = 0; k0 < nc; k0 += 4) {
            const int k = k0 + lk;
            const bool kok = k < nc;
            const int kc = kok ? k : 0;
            const double a0 = L0[kc * p + j0c];
            const double a = (kok && j0a < p) ? a0 : 0.0;
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const bool ok = kok && nok[t];
                const double w1 = L1[kc * p + j1[t]];
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    const double c = Cq[(q * ch + kc) * p + j2[t]];
                    const double b = ok ? w1 * c : 0.0;
                    d[t][q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d[t][q], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j0 = tj * 16 + 4 * r + lk;
                if (j0 < p && nok[t]) {
                    const int64_t idx = ((b0 * p + j0) * g.G[1] + (b1 * p + j1[t])) * g.G[2] + b2 * p + j2[t];
#pragma unroll
                    for (int q = 0; q < M; ++q) {
                        if (ps == 0)
                            rg[q * tot + idx] = d[t][q][r];
                        else
                            rg[q * tot + idx] += d[t][q][r];
                    }
                }
            }
    }
}

// u[perm[s]][q] (+)= sum_j U[q][grid of the box of s](j) l_j(s)
template <int M, bool ACC>
__global__ __launch_bounds__(CB_T) void k_cheb_eval(ChebGeom g, const int32_t *__restrict__ skey,
                                                    const int32_t *__restrict__ perm, const double *__restrict__ lag,
                                                    const double *__restrict__ U, double *__restrict__ u)
{
    const int64_t s = (int64_t)blockIdx.x * CB_T + threadIdx.x;
    if (s >= g.N) return;
    const int p = g.p;
    const int key = skey[s];
    const int64_t b0 = key / (g.n[1] * g.n[2]), b1 = (key / g.n[2]) % g.n[1], b2 = key % g.n[2];
    const int64_t tot = g.G[0] * g.G[1] * g.G[2];
    const int64_t N = g.N;
    const double *l0 = lag + s, *l1 = lag + (int64_t)p * N + s, *l2 = lag + 2 * (int64_t)p * N + s;
    double acc[M];
#pragma unroll
    for (int q = 0; q < M; ++q) acc[q] = 0.0;
    for (int j0 = 0; j0 < p; ++j0) {
        double a1[M];
#pragma unroll
        for (int q = 0; q < M; ++q) a1[q] = 0.0;
        for (int j1 = 0; j1 < p; ++j1) {
            const int64_t row = ((b0 * p + j0) * g.G[1] + (b1 * p + j1)) * g.G[2] + b2 * p;
            double a2[M];
#pragma unroll
            for (int q = 0; q < M; ++q) a2[q] = 0.0;
#pragma unroll 4
            for (int j2 = 0; j2 < p; ++j2) {
                const double w = l2[j2 * N];
#pragma unroll
                for (int q = 0; q < M; ++q) a2[q] = fma(w, U[q * tot + row + j2], a2[q]);
            }
            const double w1 = l1[j1 * N];
#pragma unroll
            for (int q = 0; q < M; ++q) a1[q] = fma(w1, a2[q], a1[q]);
        }
        const double w0 = l0[j0 * N];
#pragma unroll
        for (int q = 0; q < M; ++q) acc[q] = fma(w0, a1[q], acc[q]);
    }
    const int64_t i = perm[s];
#pragma unroll
    for (int q = 0; q < M; ++q) {
        if constexpr (ACC)
            u[i * M + q] += acc[q];
        else
            u[i * M + q] = acc[q];
    }
}

// The same evaluation as a dense contraction on the FP64 matrix cores, for
// boxes holding many points.  For a block of 16 points of one box,
//   V[i][n] = sum_{j2} l2(s_i, j2) U[n][j2],   n = (j0, j1),
// is a (16 x p) by (p x p^2) product, done with v_mfma_f64_16x16x4 (A: lane l
// holds A[l % 16][l / 16], B: B[l / 16][l % 16], D: D[4 r + l / 16][l % 16]);
// each D element is then weighted by l0(s_i, j0) l1(s_i, j1) (the blocks'
// l0 and l1 rows staged in the wavefront's LDS) and the 16 lanes that hold a
// point's row are summed with shuffles.  One workgroup per box; its
// wavefronts take groups of NB consecutive 16-point blocks in turn, so that
// every B fragment (4 x 16 values of the box's grid) feeds NB independent
// products, and (one component) the fragments of the next column tile are
// loaded before the products of the current one.  Each lane takes the contiguous run
// j2 = lk nkk .. lk nkk + nkk - 1 (nkk = ceil(p / 4)); KM >= nkk is a
// compile-time bound and loads are clamped into the row, so none is
// conditional.
constexpr int KMAX = DMK_FAR_PMAX / 4;

template <int M, bool ACC, int KM, int NB>
__global__ __launch_bounds__(CB_T) void k_cheb_eval_mfma(ChebGeom g, const int32_t *__restrict__ bs,
                                                         const int32_t *__restrict__ perm,
                                                         const double *__restrict__ lag,
                                                         const double *__restrict__ U, double *__restrict__ u)
{
    extern __shared__ double sm[];
    constexpr bool PF = M == 1;  // prefetch the next tile's B fragments
    const int p = g.p;
    const int64_t N = g.N;
    const int64_t box = g.wg0 + blockIdx.x;
    const int64_t b0 = box / ((int64_t)g.n[1] * g.n[2]), b1 = (box / g.n[2]) % g.n[1], b2 = box % g.n[2];
    const int64_t tot = g.G[0] * g.G[1] * g.G[2];
    const int lane = threadIdx.x & (WAVE - 1);
    const int wv = threadIdx.x / WAVE;
    const int li = lane & 15, lk = lane >> 4;  // A row / B column, A column / B row
    const int sb = bs[box], se = bs[box + 1];
    const int ngrp = (se - sb + 16 * NB - 1) / (16 * NB);
    const int pp = p * p;
    const int nkk = (p + 3) / 4;
    const int64_t g12 = g.G[1] * g.G[2];
    const int64_t rb = ((b0 * p) * g.G[1] + b1 * p) * g.G[2] + b2 * p;  // the box's first grid value
    // this wavefront's copy of the group's l0 and l1: W0[b][j][i], W1[b][j][i]
    double *W0 = sm + (size_t)wv * 32 * NB * p, *W1 = W0 + 16 * NB * p;
    // B fragments of the column (j0, j1): this lane's run of j2 of every component
    auto load_b = [&](int j0, int j1, double (&bv)[M][KM]) {
        const int64_t row = rb + (int64_t)j0 * g12 + (int64_t)j1 * g.G[2];
#pragma unroll
        for (int q = 0; q < M; ++q)
#pragma unroll
            for (int kk = 0; kk < KM; ++kk) bv[q][kk] = U[q * tot + row + min(lk * nkk + kk, p - 1)];
    };
    for (int grp = wv; grp < ngrp; grp += CB_T / WAVE) {
        const int s0 = sb + grp * 16 * NB;
        const int nv = min(16 * NB, se - s0);  // points of the group
        wave_barrier();  // the previous group's weights are no longer read
        for (int e = lane; e < 16 * NB * p; e += WAVE) {
            const int b = e / (16 * p), r = e - b * (16 * p);
            const int j = r >> 4, i = b * 16 + (r & 15);
            W0[e] = i < nv ? lag[(int64_t)j * N + s0 + i] : 0.0;
            W1[e] = i < nv ? lag[(int64_t)(p + j) * N + s0 + i] : 0.0;
        }
        wave_barrier();
        // A fragments: l2 of point li of block b at j2 = lk nkk + kk
        double afr[NB][KM];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int kk = 0; kk < KM; ++kk) {
                const int k = lk * nkk + kk, i = b * 16 + li;
                afr[b][kk] = (kk < nkk && k < p && i < nv) ? lag[(int64_t)(2 * p + k) * N + s0 + i] : 0.0;
            }
        double part[NB][M][4];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r) part[b][q][r] = 0.0;
        // this lane's B / D column n = n0 + li = j0 p + j1, advanced by 16 per
        // tile without a division
        int jn0 = li / p, jn1 = li - (li / p) * p;
        double bv[M][KM], bn[M][KM];
        if constexpr (PF) load_b(jn0 < p ? jn0 : 0, jn0 < p ? jn1 : 0, bv);
        for (int n0 = 0; n0 < pp; n0 += 16) {
            const bool nok = jn0 < p;
            const int j0 = nok ? jn0 : 0, j1 = nok ? jn1 : 0;
            // the next tile's column
            int kn0 = jn0, kn1 = jn1 + 16;
            while (kn1 >= p) {
                kn1 -= p;
                ++kn0;
            }
            // one component: the next tile's fragments are loaded now (past
            // the last tile: the clamped column 0, loaded and not used);
            // several: this tile's, all before its products
            if constexpr (PF)
                load_b(kn0 < p ? kn0 : 0, kn0 < p ? kn1 : 0, bn);
            else
                load_b(j0, j1, bv);
            // no select on B: A is zero for j2 >= p, and the columns past p^2
            // (finite values of the box) get the weight 0 below
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                dbl4 d[M];
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    d[q] = (dbl4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int kk = 0; kk < KM; ++kk)
                        if (kk < nkk) d[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(afr[b][kk], bv[q][kk], d[q], 0, 0, 0);
                }
                // weights of the four D rows this lane holds (points 4 r + lk of block b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = 4 * r + lk;
                    const double w = nok ? W0[(b * p + j0) * 16 + i] * W1[(b * p + j1) * 16 + i] : 0.0;
#pragma unroll
                    for (int q = 0; q < M; ++q) part[b][q][r] = fma(w, d[q][r], part[b][q][r]);
                }
            }
            if constexpr (PF)
#pragma unroll
                for (int q = 0; q < M; ++q)
#pragma unroll
                    for (int kk = 0; kk < KM; ++kk) bv[q][kk] = bn[q][kk];
            jn0 = kn0;
            jn1 = kn1;
        }
        // sum over the 16 lanes of a row group, in a fixed order
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int q = 0; q < M; ++q)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    for (int off = 8; off > 0; off >>= 1) part[b][q][r] += __shfl_xor(part[b][q][r], off);
        if (li == 0) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = b * 16 + 4 * r + lk;
                    if (i < nv) {
                        const int64_t pi = perm[s0 + i];
#pragma unroll
                        for (int q = 0; q < M; ++q) {
                            if constexpr (ACC)
                                u[pi * M + q] += part[b][q][r];
                            else
                                u[pi * M + q] = part[b][q][r];
                        }
                    }
                }
        }
    }
}

// u[i][j] += -phi(0) / (2 pi sigma0) rho[i][j] (harmonic kernel: 1 component,
// Stokeslet: 3); phi(0) = 1/sqrt(pi) for the Gaussian, or the PSWF series at
// t = 0, i.e. u = -1: sum_m (-1)^m c_m
struct SelfWin {
    double cheb[DMK_PSWF_MAXTERMS];
};

__global__ void k_self_term_w(int ncomp, int64_t N, int pswf, int nterms, SelfWin w, double sigma0,
                              const double *__restrict__ rho, double *__restrict__ u)
{
    double phi0;
    if (pswf) {
        phi0 = 0.0;
        for (int m = nterms - 1; m >= 0; --m) phi0 += (m & 1) ? -w.cheb[m] : w.cheb[m];
    } else {
        phi0 = 1.0 / sqrt(M_PI);
    }
    const double f = -phi0 / (2.0 * M_PI * sigma0);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < N * ncomp; e += (int64_t)gridDim.x * blockDim.x)
        u[e] += f * rho[e];
}

inline unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

int cheb_geom(const dmk_grid *grid, const dmk_bins *bins, int p, int m, ChebGeom &g)
{
    if (!grid || !bins) return DMK_EINVAL;
    if (grid->D < 0 || grid->D > 3) return DMK_EINVAL;
    if (p < 1 || p > DMK_FAR_PMAX) return DMK_EINVAL;
    if (m != 1 && m != 3 && m != 9) return DMK_EINVAL;
    const int64_t nbox = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    if (bins->nbox != nbox || bins->N < 0) return DMK_EINVAL;
    memset(&g, 0, sizeof(g));
    for (int i = 0; i < 3; ++i) {
        if (grid->n[i] < 1 || !(grid->L[i] > 0.0)) return DMK_EINVAL;
        g.n[i] = grid->n[i];
        g.inv[i] = (double)grid->n[i] / grid->L[i];  // the binning's factor
        g.G[i] = (int64_t)grid->n[i] * p;
    }
    if ((double)g.G[0] * (double)g.G[1] * (double)g.G[2] * m > 9.0e15) return DMK_ESIZE;
    g.p = p;
    g.N = bins->N;
    return DMK_OK;
}

size_t lag_bytes(int64_t N, int p) { return (size_t)(sizeof(double) * 3 * p * (N > 0 ? N : 1) + 256); }

}  // namespace
}  // namespace dmk

using namespace dmk;

extern "C" size_t dmk_cheb_ws_bytes(const dmk_bins *bins, int p)
{
    if (!bins || bins->N < 0 || p < 1 || p > DMK_FAR_PMAX) return 0;
    return lag_bytes(bins->N, p);
}

extern "C" int dmk_cheb_anterp(const dmk_grid *grid, const dmk_bins *bins, int p, int m, const double *rho,
                               double *rho_grid, void *ws, size_t ws_bytes, hipStream_t stream)
{
    ChebGeom g;
    const int st = cheb_geom(grid, bins, p, m, g);
    if (st != DMK_OK) return st;
    if (!rho_grid || !ws || (g.N > 0 && !rho)) return DMK_EINVAL;
    if (ws_bytes < lag_bytes(g.N, p)) return DMK_ESIZE;
    double *lag = (double *)ws;
    if (g.N > 0)
        hipLaunchKernelGGL(k_cheb_lagrange<false>, dim3(nblk(3 * g.N, CB_T)), dim3(CB_T), 0, stream, g, bins->ys,
                           bins->skey, lag);
    // points per LDS chunk: (2 + m) p doubles each, within 48 KB
    const int ch = max(1, min(256, 49152 / ((2 + m) * p * 8)));
    const int64_t nbox = (g.G[0] / p) * (g.G[1] / p) * (g.G[2] / p);
    const size_t lds = sizeof(double) * (size_t)(2 + m) * ch * p;
    const int32_t *bsp = bins->box_start, *pm = bins->perm;
    if (g.N >= 16 * nbox) {
        // boxes of 16 or more points on average: matrix-core contraction,
        // one group of 16 x 16 output tiles per wavefront
        const int nt = m == 1 ? AnterpTiles<1>::NT : (m == 3 ? AnterpTiles<3>::NT : AnterpTiles<9>::NT);
        const int ngroup = ((p + 15) / 16) * (((p * p + 15) / 16 + nt - 1) / nt);
        const int nsplit = (ngroup + CB_T / WAVE - 1) / (CB_T / WAVE);
        const int64_t nwg = nbox * nsplit;
        for (g.wg0 = 0; g.wg0 < nwg; g.wg0 += MAX_WG) {
            const dim3 grd((unsigned)std::min(MAX_WG, nwg - g.wg0));
            switch (m) {
            case 1: hipLaunchKernelGGL(k_cheb_anterp_mfma<1>, grd, dim3(CB_T), lds, stream, g, ch, nsplit, bsp, pm, lag, rho, rho_grid); break;
            case 3: hipLaunchKernelGGL(k_cheb_anterp_mfma<3>, grd, dim3(CB_T), lds, stream, g, ch, nsplit, bsp, pm, lag, rho, rho_grid); break;
            default: hipLaunchKernelGGL(k_cheb_anterp_mfma<9>, grd, dim3(CB_T), lds, stream, g, ch, nsplit, bsp, pm, lag, rho, rho_grid); break;
            }
        }
        DMK_HIP_CHECK(hipGetLastError());
        return DMK_OK;
    }
    const int nsplit = (p * p * p + CB_NODES - 1) / CB_NODES;
    const int64_t nwg = nbox * nsplit;
    for (g.wg0 = 0; g.wg0 < nwg; g.wg0 += MAX_WG) {
        const dim3 grd((unsigned)std::min(MAX_WG, nwg - g.wg0));
        switch (m) {
        case 1: hipLaunchKernelGGL(k_cheb_anterp<1>, grd, dim3(CB_T), lds, stream, g, ch, nsplit, bsp, pm, lag, rho, rho_grid); break;
        case 3: hipLaunchKernelGGL(k_cheb_anterp<3>, grd, dim3(CB_T), lds, stream, g, ch, nsplit, bsp, pm, lag, rho, rho_grid); break;
        default: hipLaunchKernelGGL(k_cheb_anterp<9>, grd, dim3(CB_T), lds, stream, g, ch, nsplit, bsp, pm, lag, rho, rho_grid); break;
        }
    }
    DMK_HIP_CHECK(hipGetLastError());
    return DMK_OK;
}

namespace dmk {
namespace {
// one launch of k_cheb_eval_mfma; the LDS holds each wavefront's l0 and l1
// rows of a group of NB blocks (32 NB p doubles)
template <int M, int KM, int NB>
void launch_em(bool acc, dim3 grd, hipStream_t st, const ChebGeom &g, const int32_t *bsp, const int32_t *pm,
               const double *lag, const double *U, double *u)
{
    const size_t lds = sizeof(double) * (size_t)(CB_T / WAVE) * 32 * NB * g.p;
    if (acc)
        hipLaunchKernelGGL((k_cheb_eval_mfma<M, true, KM, NB>), grd, dim3(CB_T), lds, st, g, bsp, pm, lag, U, u);
    else
        hipLaunchKernelGGL((k_cheb_eval_mfma<M, false, KM, NB>), grd, dim3(CB_T), lds, st, g, bsp, pm, lag, U, u);
}
// NB1: blocks per group for one component (several components keep one
// block per group: their B fragments and sums already fill the registers)
template <int KM, int NB1>
void launch_eval_mfma(int m, bool acc, dim3 grd, hipStream_t st, const ChebGeom &g, const int32_t *bsp,
                      const int32_t *pm, const double *lag, const double *U, double *u)
{
    switch (m) {
    case 1: launch_em<1, KM, NB1>(acc, grd, st, g, bsp, pm, lag, U, u); break;
    case 3: launch_em<3, KM, 1>(acc, grd, st, g, bsp, pm, lag, U, u); break;
    default: launch_em<9, KM, 1>(acc, grd, st, g, bsp, pm, lag, U, u); break;
    }
}
}  // namespace
}  // namespace dmk

extern "C" int dmk_cheb_eval(const dmk_grid *grid, const dmk_bins *bins, int p, int m, const double *u_grid,
                             int accumulate, double *u, void *ws, size_t ws_bytes, hipStream_t stream)
{
    ChebGeom g;
    const int st = cheb_geom(grid, bins, p, m, g);
    if (st != DMK_OK) return st;
    if (!u_grid || !ws || (g.N > 0 && !u)) return DMK_EINVAL;
    if (ws_bytes < lag_bytes(g.N, p)) return DMK_ESIZE;
    if (g.N == 0) return DMK_OK;
    double *lag = (double *)ws;
    hipLaunchKernelGGL(k_cheb_lagrange<true>, dim3(nblk(3 * g.N, CB_T)), dim3(CB_T), 0, stream, g, bins->ys,
                       bins->skey, lag);
    const int32_t *sk = bins->skey, *pm = bins->perm, *bsp = bins->box_start;
    const int64_t nbox = (g.G[0] / p) * (g.G[1] / p) * (g.G[2] / p);
    if (g.N >= 16 * nbox) {
        // boxes of 16 or more points on average: matrix-core contraction per box
        // groups of 2 blocks for one component while p <= 32 (LDS <= 64 KiB)
        const bool acc = accumulate != 0;
        for (g.wg0 = 0; g.wg0 < nbox; g.wg0 += MAX_WG) {
            const dim3 grd((unsigned)std::min(MAX_WG, nbox - g.wg0));
            const int nkk = (p + 3) / 4;
            if (nkk <= 4)
                launch_eval_mfma<4, 2>(m, acc, grd, stream, g, bsp, pm, lag, u_grid, u);
            else if (nkk <= 5)
                launch_eval_mfma<5, 2>(m, acc, grd, stream, g, bsp, pm, lag, u_grid, u);
            else if (nkk <= 8)
                launch_eval_mfma<8, 2>(m, acc, grd, stream, g, bsp, pm, lag, u_grid, u);
            else
                launch_eval_mfma<KMAX, 1>(m, acc, grd, stream, g, bsp, pm, lag, u_grid, u);
        }
        DMK_HIP_CHECK(hipGetLastError());
        return DMK_OK;
    }
    const dim3 grd(nblk(g.N, CB_T));
    if (accumulate) {
        switch (m) {
        case 1: hipLaunchKernelGGL((k_cheb_eval<1, true>), grd, dim3(CB_T), 0, stream, g, sk, pm, lag, u_grid, u); break;
        case 3: hipLaunchKernelGGL((k_cheb_eval<3, true>), grd, dim3(CB_T), 0, stream, g, sk, pm, lag, u_grid, u); break;
        default: hipLaunchKernelGGL((k_cheb_eval<9, true>), grd, dim3(CB_T), 0, stream, g, sk, pm, lag, u_grid, u); break;
        }
    } else {
        switch (m) {
        case 1: hipLaunchKernelGGL((k_cheb_eval<1, false>), grd, dim3(CB_T), 0, stream, g, sk, pm, lag, u_grid, u); break;
        case 3: hipLaunchKernelGGL((k_cheb_eval<3, false>), grd, dim3(CB_T), 0, stream, g, sk, pm, lag, u_grid, u); break;
        default: hipLaunchKernelGGL((k_cheb_eval<9, false>), grd, dim3(CB_T), 0, stream, g, sk, pm, lag, u_grid, u); break;
        }
    }
    DMK_HIP_CHECK(hipGetLastError());
    return DMK_OK;
}

extern "C" int dmk_self_term(int kernel, double sigma0, const dmk_pswf *win, int64_t N, const double *rho, double *u,
                             hipStream_t stream)
{
    if (kernel < 0 || kernel > 3 || N < 0) return DMK_EINVAL;
    if (!(sigma0 > 0.0) || !isfinite(sigma0)) return DMK_ECUTOFF;
    SelfWin w;
    memset(&w, 0, sizeof(w));
    int nterms = 0;
    if (win) {
        if (!(win->c > 0.0) || !(win->c <= DMK_PSWF_CMAX) || win->nterms64 < 1 ||
            win->nterms64 > DMK_PSWF_MAXTERMS)
            return DMK_EUNSUPPORTED;
        nterms = win->nterms64;
        for (int m = 0; m < DMK_PSWF_MAXTERMS; ++m) w.cheb[m] = win->cheb[0][m];
    }
    if (kernel == 2 || kernel == 3 || N == 0) return DMK_OK;  // no self term for stresslet and rotlet
    if (!rho || !u) return DMK_EINVAL;
    const int nc = kernel == 0 ? 1 : 3;
    // grid-stride over the N m elements (at most 65536 workgroups)
    const unsigned nb = (unsigned)std::min<int64_t>(65536, (N + 255) / 256 * nc);
    hipLaunchKernelGGL(k_self_term_w, dim3(nb), dim3(256), 0, stream, nc, N,
                       win ? 1 : 0, nterms, w,
                       sigma0, rho, u);
    DMK_HIP_CHECK(hipGetLastError());
    return DMK_OK;
}
