// dmk_residual.hip -- leaf-level residual interaction of the periodized DMK
// method (Sec. 2.3, eq. (u_local); Sec. 3.1.5) and its adjoint, for gfx950.
//
// Per target x_b the kernels sum K_R(x_b - x_a + p) rho_a over the sources of
// the target's leaf box and its 26 neighbours (periodic images across the
// faces of the first D axes), keeping pairs with 0 < |d| < rc.
//
// Work decomposition (one 64-lane wavefront per workgroup):
//  * a tile is <= 64 consecutive sorted targets of one leaf column (b0, b1)
//    in z-boxes [z0, z1];
//  * its neighbour sources (9 neighbour columns x z-slabs z0-1 .. z1+1) are
//    staged in LDS in slab-major order, so the 27-box stencil of a target in
//    box z is ONE contiguous LDS range (slabs z-1, z, z+1).  Coordinates are
//    formed in FP64 relative to the tile's reference box centre, with the
//    periodic image shift applied, and kept as FP64 (FP64 path) or as an
//    FP32 hi/lo pair (FP32 path);
//  * all 64 lanes scan one target's range at a time with a cheap FP32
//    distance test; in-cutoff pairs are compacted into an LDS queue
//    (ballot + mbcnt), so the transcendental pair math runs on full
//    wavefronts;
//  * queued pairs are evaluated 64 at a time into an LDS contribution array;
//    then each target's lane sums its own contiguous run (fixed order: the
//    result is deterministic; Kahan-compensated in the FP32 path).
//  * tiles of very dense boxes stream their neighbourhood through LDS in
//    chunks.
//
// Kernels (Gaussian window phi(t) = exp(-t^2)/sqrt(pi), Phi = erfc,
// t = r/sigma; App. B and eq. (Hhatsplit_wfunc)):
//   Laplace   erfc(t)/(4 pi r) q
//   Stokeslet [Sd f/(8 pi r)] + [So (d.f) d/(8 pi r^3)], Sd = Phi - 2t phi, So = Phi + 2t phi
//   stresslet Td/(8 pi r^3) (rho d + rho^T d + tr(rho) d) - 3/(4 pi) To (d.rho.d) d / r^5,
//             Td = 4 t^3 phi (= -2 t^2 phi'), To = Phi + 2t phi + (4/3) t^3 phi
//   rotlet    Oo/(8 pi r^3) (rho x d), Oo = Phi + 2t phi
#include <hip/hip_runtime.h>
#include <math.h>

#include "dmk_internal.h"

namespace dmk {

template <int K>
struct KDim {
    static constexpr int MIN = (K == 0) ? 1 : ((K == 2) ? 9 : 3);
    static constexpr int MOUT = (K == 0) ? 1 : 3;
};

template <int KERN, typename FP, bool BWD>
struct Cfg {
    static constexpr int MIN = KDim<KERN>::MIN;
    static constexpr int MOUT = KDim<KERN>::MOUT;
    static constexpr int NPL = BWD ? MIN + MOUT : MIN;   // payload per source
    static constexpr int NTP = BWD ? MIN + MOUT : 0;     // payload per target
    static constexpr int NC = BWD ? MIN + 3 : MOUT;      // sums per target
    static constexpr bool F32 = sizeof(FP) == 4;
    static constexpr int CAPP = TILE_CAP + TILE_PAD;
    static constexpr int QB = NC * (int)sizeof(FP);
    static constexpr int QCAP = (QB <= 16) ? 512 : (QB <= 48 ? 256 : 128);
};

struct ResParams {
    double L[3], h[3];
    int n[3], D;
    double sigma, rc;
    int64_t N;
    int ntiles;
    const double *ys;
    const int32_t *skey, *bs, *perm, *nbr;
    const int8_t *img;
    const int4 *tiles;
    const double *pl;
    double *out0, *out1;
};

struct Seg {
    int gstart, glen, k, vshift, so, pad;
    double offx, offy, offz;
};

template <class C>
struct Smem {
    static constexpr int S32 = C::F32 ? C::CAPP : 1;
    static constexpr int S64 = C::F32 ? 1 : C::CAPP;
    static constexpr int NX32 = (C::F32 && C::NPL > 2) ? C::NPL - 2 : 1;
    static constexpr int NX64 = C::F32 ? 1 : C::NPL;
    static constexpr int TX32 = (C::F32 && C::NTP > 2) ? C::NTP - 2 : 1;
    static constexpr int TX64 = (!C::F32 && C::NTP > 0) ? C::NTP : 1;
    float4 sc[C::CAPP];          // FP32 hi coords (scan), w = payload 0 (FP32 path)
    float4 sl[S32];              // FP32 lo coords, w = payload 1
    float sp[NX32][(C::F32 && C::NPL > 2) ? C::CAPP : 1];  // FP32 payload 2..
    double sx[S64], sy[S64], sz[S64];
    double spd[NX64][S64];
    float4 tc[TILE_T];
    float4 tl[C::F32 ? TILE_T : 1];
    float tp[TX32][(C::F32 && C::NTP > 2) ? TILE_T : 1];
    double tx[C::F32 ? 1 : TILE_T], ty[C::F32 ? 1 : TILE_T], tz[C::F32 ? 1 : TILE_T];
    double tpd[TX64][(!C::F32 && C::NTP > 0) ? TILE_T : 1];
    uint32_t queue[C::QCAP];
    typename std::conditional<C::F32, float, double>::type contrib[C::NC][C::QCAP];
    int dtab[(TILE_ZMAX + 2) * 9];
    int soff[TILE_ZMAX + 4];
    int ccol[9];
    int qtot;
    Seg seg[27];
};

// --------------------------------------------------------------------------
// scalar helpers
__device__ inline float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsqrt_(double x) { return rsqrt(x); }
__device__ inline float erfc_(float x) { return erfcf(x); }
__device__ inline double erfc_(double x) { return erfc(x); }
__device__ inline float expneg_(float x) { return __expf(-x); }
__device__ inline double expneg_(double x) { return exp(-x); }

__device__ inline int wave_incl_scan(int v)
{
    const int lane = threadIdx.x & 63;
    for (int off = 1; off < 64; off <<= 1) {
        int w = __shfl_up(v, off, 64);
        if (lane >= off) v += w;
    }
    return v;
}

template <typename T>
struct Rad {
    T ri, r, t, t2, phi, Phi;
};

template <typename T>
__device__ inline Rad<T> radial(T r2, T isig, T isig2)
{
    Rad<T> R;
    R.ri = rsqrt_(r2);
    R.r = r2 * R.ri;
    R.t = R.r * isig;
    R.t2 = r2 * isig2;
    R.phi = expneg_(R.t2) * (T)0.56418958354775628695;  // 1/sqrt(pi)
    R.Phi = erfc_(R.t);
    return R;
}

#define INV4PI 0.079577471545947667884
#define INV8PI 0.039788735772973833942
#define C34PI 0.23873241463784300365

// forward pair contribution v[MOUT]; ps = source strengths
template <int KERN, typename T>
__device__ inline void pair_fwd(const T d[3], T r2, T isig, T isig2, const T *ps, T *v)
{
    const Rad<T> R = radial(r2, isig, isig2);
    const T tphi2 = (T)2 * R.t * R.phi;
    if constexpr (KERN == 0) {
        v[0] = R.Phi * R.ri * (T)INV4PI * ps[0];
    } else if constexpr (KERN == 1) {
        const T ri3 = R.ri * R.ri * R.ri;
        const T A = (R.Phi - tphi2) * R.ri * (T)INV8PI;
        const T B = (R.Phi + tphi2) * ri3 * (T)INV8PI;
        const T df = d[0] * ps[0] + d[1] * ps[1] + d[2] * ps[2];
        const T Bdf = B * df;
        for (int c = 0; c < 3; ++c) v[c] = A * ps[c] + Bdf * d[c];
    } else if constexpr (KERN == 2) {
        const T ri2 = R.ri * R.ri;
        const T ri3 = ri2 * R.ri;
        const T t3phi = R.t2 * R.t * R.phi;
        const T P = (T)4 * t3phi * ri3 * (T)INV8PI;
        const T Qc = -(T)C34PI * (R.Phi + tphi2 + (T)(4.0 / 3.0) * t3phi) * ri3 * ri2;
        T rd[3], rtd[3];
        for (int l = 0; l < 3; ++l) {
            rd[l] = ps[3 * l + 0] * d[0] + ps[3 * l + 1] * d[1] + ps[3 * l + 2] * d[2];
            rtd[l] = ps[0 * 3 + l] * d[0] + ps[1 * 3 + l] * d[1] + ps[2 * 3 + l] * d[2];
        }
        const T tr = ps[0] + ps[4] + ps[8];
        const T drd = d[0] * rd[0] + d[1] * rd[1] + d[2] * rd[2];
        for (int c = 0; c < 3; ++c) v[c] = P * (rd[c] + rtd[c] + tr * d[c]) + Qc * drd * d[c];
    } else {
        const T ri3 = R.ri * R.ri * R.ri;
        const T f = (R.Phi + tphi2) * ri3 * (T)INV8PI;
        v[0] = f * (ps[1] * d[2] - ps[2] * d[1]);
        v[1] = f * (ps[2] * d[0] - ps[0] * d[2]);
        v[2] = f * (ps[0] * d[1] - ps[1] * d[0]);
    }
}

// adjoint pair contribution v[MIN + 3] = (d grad_rho_t, d grad_x_t);
// ps = (rho_s, G_s), pt = (rho_t, G_t); d = x_t - x_s (+ image).
template <int KERN, typename T>
__device__ inline void pair_bwd(const T d[3], T r2, T isig, T isig2, const T *ps, const T *pt, T *v)
{
    constexpr int MIN = KDim<KERN>::MIN;
    const T *rs = ps, *Gs = ps + MIN, *rt = pt, *Gt = pt + MIN;
    const Rad<T> R = radial(r2, isig, isig2);
    const T tphi2 = (T)2 * R.t * R.phi;
    const T ri2 = R.ri * R.ri;
    const T ri3 = ri2 * R.ri;
    if constexpr (KERN == 0) {
        const T K = R.Phi * R.ri * (T)INV4PI;
        const T g = -(R.Phi + tphi2) * ri3 * (T)INV4PI;
        v[0] = K * Gs[0];
        const T s = g * (Gt[0] * rs[0] + Gs[0] * rt[0]);
        for (int c = 0; c < 3; ++c) v[1 + c] = s * d[c];
    } else if constexpr (KERN == 1) {
        const T Sd = R.Phi - tphi2, So = R.Phi + tphi2;
        const T A = Sd * R.ri * (T)INV8PI;
        const T B = So * ri3 * (T)INV8PI;
        const T dSd = (T)4 * R.phi * (R.t2 - (T)1);
        const T dSo = -(T)4 * R.t2 * R.phi;
        const T Ar = (dSd * isig * ri2 - Sd * ri3) * (T)INV8PI;             // A'(r)/r
        const T Br = (dSo * isig * ri2 * ri2 - (T)3 * So * ri3 * ri2) * (T)INV8PI;  // B'(r)/r
        const T dGs = d[0] * Gs[0] + d[1] * Gs[1] + d[2] * Gs[2];
        const T dGt = d[0] * Gt[0] + d[1] * Gt[1] + d[2] * Gt[2];
        const T drs = d[0] * rs[0] + d[1] * rs[1] + d[2] * rs[2];
        const T drt = d[0] * rt[0] + d[1] * rt[1] + d[2] * rt[2];
        const T GtRs = Gt[0] * rs[0] + Gt[1] * rs[1] + Gt[2] * rs[2];
        const T GsRt = Gs[0] * rt[0] + Gs[1] * rt[1] + Gs[2] * rt[2];
        const T sd = Ar * (GtRs + GsRt) + Br * (dGt * drs + dGs * drt);
        for (int c = 0; c < 3; ++c) {
            v[c] = A * Gs[c] + B * dGs * d[c];
            v[3 + c] = sd * d[c] + B * (Gt[c] * drs + rs[c] * dGt + Gs[c] * drt + rt[c] * dGs);
        }
    } else if constexpr (KERN == 2) {
        const T t3phi = R.t2 * R.t * R.phi;
        const T Td = (T)4 * t3phi;
        const T To = R.Phi + tphi2 + (T)(4.0 / 3.0) * t3phi;
        const T P = Td * ri3 * (T)INV8PI;
        const T ri5 = ri3 * ri2;
        const T Qc = -(T)C34PI * To * ri5;
        const T dTd = (T)4 * R.t2 * R.phi * ((T)3 - (T)2 * R.t2);
        const T dTo = -(T)(8.0 / 3.0) * R.t2 * R.t2 * R.phi;
        const T Pr = (dTd * isig * ri2 * ri2 - (T)3 * Td * ri5) * (T)INV8PI;
        const T Qr = -(T)C34PI * (dTo * isig * ri3 * ri3 - (T)5 * To * ri5 * ri2);
        const T dGs = d[0] * Gs[0] + d[1] * Gs[1] + d[2] * Gs[2];
        // grad_rho_t[l][m] = -T_jlm(d) Gs_j
        for (int l = 0; l < 3; ++l)
            for (int m = 0; m < 3; ++m)
                v[3 * l + m] = -(P * (Gs[l] * d[m] + (l == m ? dGs : (T)0) + d[l] * Gs[m]) + Qc * dGs * d[l] * d[m]);
        // grad_x_t = dF(Gt, rho_s) - dF(Gs, rho_t)
        T gx[3] = {0, 0, 0};
        for (int side = 0; side < 2; ++side) {
            const T *a = side ? Gs : Gt;
            const T *rho = side ? rt : rs;
            const T sgn = side ? (T)-1 : (T)1;
            T rd[3], rtd[3], ra[3], rta[3];
            for (int l = 0; l < 3; ++l) {
                rd[l] = rho[3 * l] * d[0] + rho[3 * l + 1] * d[1] + rho[3 * l + 2] * d[2];
                rtd[l] = rho[l] * d[0] + rho[3 + l] * d[1] + rho[6 + l] * d[2];
                ra[l] = rho[3 * l] * a[0] + rho[3 * l + 1] * a[1] + rho[3 * l + 2] * a[2];
                rta[l] = rho[l] * a[0] + rho[3 + l] * a[1] + rho[6 + l] * a[2];
            }
            const T tr = rho[0] + rho[4] + rho[8];
            const T ad = a[0] * d[0] + a[1] * d[1] + a[2] * d[2];
            const T drd = d[0] * rd[0] + d[1] * rd[1] + d[2] * rd[2];
            const T aRd = a[0] * rd[0] + a[1] * rd[1] + a[2] * rd[2];
            const T dRa = d[0] * ra[0] + d[1] * ra[1] + d[2] * ra[2];
            const T sd = Pr * (aRd + dRa + ad * tr) + Qr * ad * drd;
            for (int k = 0; k < 3; ++k)
                gx[k] += sgn * (sd * d[k] + P * (rta[k] + ra[k] + a[k] * tr) + Qc * (a[k] * drd + ad * (rd[k] + rtd[k])));
        }
        for (int k = 0; k < 3; ++k) v[9 + k] = gx[k];
    } else {
        const T Oo = R.Phi + tphi2;
        const T f = Oo * ri3 * (T)INV8PI;
        const T dOo = -(T)4 * R.t2 * R.phi;
        const T fr = (dOo * isig * ri2 * ri2 - (T)3 * Oo * ri3 * ri2) * (T)INV8PI;
        // grad_rho_t = f (Gs x d)
        v[0] = f * (Gs[1] * d[2] - Gs[2] * d[1]);
        v[1] = f * (Gs[2] * d[0] - Gs[0] * d[2]);
        v[2] = f * (Gs[0] * d[1] - Gs[1] * d[0]);
        T w[3];
        w[0] = (Gt[1] * rs[2] - Gt[2] * rs[1]) - (Gs[1] * rt[2] - Gs[2] * rt[1]);
        w[1] = (Gt[2] * rs[0] - Gt[0] * rs[2]) - (Gs[2] * rt[0] - Gs[0] * rt[2]);
        w[2] = (Gt[0] * rs[1] - Gt[1] * rs[0]) - (Gs[0] * rt[1] - Gs[1] * rt[0]);
        const T dw = d[0] * w[0] + d[1] * w[1] + d[2] * w[2];
        for (int c = 0; c < 3; ++c) v[3 + c] = fr * dw * d[c] + f * w[c];
    }
}

// --------------------------------------------------------------------------
template <class C>
__device__ inline void stage_source(Smem<C> &S, const ResParams &P, int dest, int64_t j, double ox, double oy,
                                    double oz)
{
    const int64_t N = P.N;
    const double X = P.ys[j] + ox;
    const double Y = P.ys[N + j] + oy;
    const double Z = P.ys[2 * N + j] + oz;
    if constexpr (C::F32) {
        const float hx = (float)X, hy = (float)Y, hz = (float)Z;
        const float lx = (float)(X - (double)hx), ly = (float)(Y - (double)hy), lz = (float)(Z - (double)hz);
        const float p0 = (float)P.pl[j];
        const float p1 = (C::NPL > 1) ? (float)P.pl[N + j] : 0.0f;
        S.sc[dest] = make_float4(hx, hy, hz, p0);
        S.sl[dest] = make_float4(lx, ly, lz, p1);
        for (int c = 2; c < C::NPL; ++c) S.sp[c - 2][dest] = (float)P.pl[c * N + j];
    } else {
        S.sc[dest] = make_float4((float)X, (float)Y, (float)Z, 0.0f);
        S.sx[dest] = X;
        S.sy[dest] = Y;
        S.sz[dest] = Z;
        for (int c = 0; c < C::NPL; ++c) S.spd[c][dest] = P.pl[c * N + j];
    }
}

template <int KERN, typename FP, bool BWD>
__global__ __launch_bounds__(64) void k_residual(ResParams P)
{
    using C = Cfg<KERN, FP, BWD>;
    using T = FP;
    __shared__ Smem<C> S;
    const int lane = threadIdx.x;
    const int per = (P.ntiles + 7) >> 3;
    const int tile = (blockIdx.x & 7) * per + (blockIdx.x >> 3);  // XCD-contiguous tile runs
    if (tile >= P.ntiles) return;

    const int4 TD = P.tiles[tile];
    const int n0 = P.n[0], n1 = P.n[1], n2 = P.n[2];
    const int col = TD.x, z0 = TD.y;
    const bool dense = TD.z < 0;
    const int z1 = dense ? z0 : TD.z;
    const int tstart = TD.w;
    const int64_t colb = (int64_t)col * n2;
    const int ntgt = dense ? min(TILE_T, P.bs[colb + z0 + 1] - tstart) : (P.bs[colb + z1 + 1] - tstart);
    const int b0 = col / n1, b1 = col - (col / n1) * n1;
    const double crx = (b0 + 0.5) * P.h[0], cry = (b1 + 0.5) * P.h[1], crz = (z0 + 0.5) * P.h[2];
    const int za = z0 - 1, zb = z1 + 1, nslab = z1 - z0 + 3;
    const int r0 = n0 + n1;

    // ---- neighbour columns and their contiguous source pieces (<= 3 each)
    if (lane < 27) S.seg[lane].glen = 0;
    if (lane < 9) S.ccol[lane] = -1;
    __syncthreads();
    if (lane < 9) {
        const int k = lane, c0 = k / 3, c1 = k % 3;
        const int nb0 = P.nbr[3 * b0 + c0], nb1 = P.nbr[3 * (n0 + b1) + c1];
        if (nb0 >= 0 && nb1 >= 0) {
            const int s0 = P.img[3 * b0 + c0], s1 = P.img[3 * (n0 + b1) + c1];
            const int cc = nb0 * n1 + nb1;
            const int64_t cb = (int64_t)cc * n2;
            S.ccol[k] = cc;
            const double ox = s0 * P.L[0] - crx, oy = s1 * P.L[1] - cry;
            // piece 0: virtual z = -1
            if (za == -1) {
                const int zp = P.nbr[3 * r0 + 0];
                if (zp >= 0) {
                    Seg &g = S.seg[3 * k + 0];
                    g.gstart = P.bs[cb + zp];
                    g.glen = P.bs[cb + zp + 1] - g.gstart;
                    g.k = k;
                    g.vshift = -1 - zp;
                    g.offx = ox;
                    g.offy = oy;
                    g.offz = P.img[3 * r0 + 0] * P.L[2] - crz;
                }
            }
            // piece 1: virtual z in [max(za,0), min(zb,n2-1)], no z image
            {
                const int lo = za < 0 ? 0 : za, hi = zb > n2 - 1 ? n2 - 1 : zb;
                if (lo <= hi) {
                    Seg &g = S.seg[3 * k + 1];
                    g.gstart = P.bs[cb + lo];
                    g.glen = P.bs[cb + hi + 1] - g.gstart;
                    g.k = k;
                    g.vshift = 0;
                    g.offx = ox;
                    g.offy = oy;
                    g.offz = -crz;
                }
            }
            // piece 2: virtual z = n2
            if (zb == n2) {
                const int zp = P.nbr[3 * (r0 + n2 - 1) + 2];
                if (zp >= 0) {
                    Seg &g = S.seg[3 * k + 2];
                    g.gstart = P.bs[cb + zp];
                    g.glen = P.bs[cb + zp + 1] - g.gstart;
                    g.k = k;
                    g.vshift = n2 - zp;
                    g.offx = ox;
                    g.offy = oy;
                    g.offz = P.img[3 * (r0 + n2 - 1) + 2] * P.L[2] - crz;
                }
            }
        }
    }
    __syncthreads();
    if (lane == 0) {
        int so = 0;
        for (int s = 0; s < 27; ++s) {
            S.seg[s].so = so;
            so += S.seg[s].glen;
        }
        S.qtot = so;
    }
    // ---- slab-major offsets for multi-box tiles
    if (!dense) {
        const int M = nslab * 9;
        int carry = 0;
        for (int base = 0; base < M; base += 64) {
            const int idx = base + lane;
            int cnt = 0, gs = 0;
            if (idx < M) {
                const int s = idx / 9, k = idx - (idx / 9) * 9;
                const int cc = S.ccol[k];
                const int zv = za + s;
                int zp = zv;
                if (zv < 0)
                    zp = P.nbr[3 * r0 + 0];
                else if (zv >= n2)
                    zp = P.nbr[3 * (r0 + n2 - 1) + 2];
                if (cc >= 0 && zp >= 0) {
                    const int64_t b = (int64_t)cc * n2 + zp;
                    gs = P.bs[b];
                    cnt = P.bs[b + 1] - gs;
                }
            }
            const int incl = wave_incl_scan(cnt);
            if (idx < M) {
                const int off = carry + incl - cnt;
                S.dtab[idx] = off - gs;
                if (idx % 9 == 0) S.soff[idx / 9] = off;
            }
            carry += __shfl(incl, 63, 64);
        }
        if (lane == 0) S.soff[nslab] = carry;
    }
    __syncthreads();

    // ---- targets: tile-relative coordinates, payload, stencil range
    const T isig = (T)(1.0 / P.sigma);
    const T isig2 = isig * isig;
    const T rc2 = (T)(P.rc * P.rc);
    const float rc2s = (float)(P.rc * P.rc * (1.0 + 4e-4));  // scan margin; exact test in the pair step
    float thx = 0.f, thy = 0.f, thz = 0.f;
    int my_a = 0, my_b = 0;
    if (lane < ntgt) {
        const int64_t j = tstart + lane;
        const double X = P.ys[j] - crx, Y = P.ys[P.N + j] - cry, Z = P.ys[2 * P.N + j] - crz;
        thx = (float)X;
        thy = (float)Y;
        thz = (float)Z;
        if constexpr (C::F32) {
            const float t0 = (C::NTP > 0) ? (float)P.pl[j] : 0.0f;
            const float t1 = (C::NTP > 1) ? (float)P.pl[P.N + j] : 0.0f;
            S.tc[lane] = make_float4(thx, thy, thz, t0);
            S.tl[lane] = make_float4((float)(X - (double)thx), (float)(Y - (double)thy), (float)(Z - (double)thz), t1);
            for (int c = 2; c < C::NTP; ++c) S.tp[c - 2][lane] = (float)P.pl[c * P.N + j];
        } else {
            S.tx[lane] = X;
            S.ty[lane] = Y;
            S.tz[lane] = Z;
            for (int c = 0; c < C::NTP; ++c) S.tpd[c][lane] = P.pl[c * P.N + j];
        }
        if (!dense) {
            const int zt = P.skey[j] - (int)colb;
            my_a = S.soff[zt - z0];
            my_b = S.soff[zt - z0 + 3];
        }
    }

    T acc[C::NC], cmp[C::NC];
    for (int c = 0; c < C::NC; ++c) {
        acc[c] = 0;
        cmp[c] = 0;
    }
    int qn = 0;
    int rs = 0, re = 0;

    auto flush = [&]() {
        __syncthreads();
        for (int base = 0; base < qn; base += 64) {
            const int i = base + lane;
            if (i < qn) {
                const uint32_t e = S.queue[i];
                const int t = (int)(e >> 16), q = (int)(e & 0xffffu);
                T d[3], ps[C::NPL], pt[C::NTP > 0 ? C::NTP : 1];
                if constexpr (C::F32) {
                    const float4 sh = S.sc[q], sl = S.sl[q], th = S.tc[t], tl = S.tl[t];
                    d[0] = (th.x - sh.x) + (tl.x - sl.x);
                    d[1] = (th.y - sh.y) + (tl.y - sl.y);
                    d[2] = (th.z - sh.z) + (tl.z - sl.z);
                    ps[0] = sh.w;
                    if (C::NPL > 1) ps[1] = sl.w;
                    for (int c = 2; c < C::NPL; ++c) ps[c] = S.sp[c - 2][q];
                    if constexpr (C::NTP > 0) {
                        pt[0] = th.w;
                        pt[1] = tl.w;
                        for (int c = 2; c < C::NTP; ++c) pt[c] = S.tp[c - 2][t];
                    }
                } else {
                    d[0] = S.tx[t] - S.sx[q];
                    d[1] = S.ty[t] - S.sy[q];
                    d[2] = S.tz[t] - S.sz[q];
                    for (int c = 0; c < C::NPL; ++c) ps[c] = S.spd[c][q];
                    for (int c = 0; c < C::NTP; ++c) pt[c] = S.tpd[c][t];
                }
                T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                const bool ok = (r2 > (T)0) && (r2 < rc2);
                if (!ok) r2 = rc2;  // keeps the math finite; result discarded
                T v[C::NC];
                if constexpr (BWD)
                    pair_bwd<KERN, T>(d, r2, isig, isig2, ps, pt, v);
                else
                    pair_fwd<KERN, T>(d, r2, isig, isig2, ps, v);
                for (int c = 0; c < C::NC; ++c) S.contrib[c][i] = ok ? v[c] : (T)0;
            }
        }
        __syncthreads();
        // each target lane sums its own run, in queue order
        for (int i = rs; i < re; ++i) {
            for (int c = 0; c < C::NC; ++c) {
                const T x = S.contrib[c][i];
                if constexpr (C::F32) {
                    const T y = x - cmp[c];
                    const T s = acc[c] + y;
                    cmp[c] = (s - acc[c]) - y;
                    acc[c] = s;
                } else {
                    acc[c] += x;
                }
            }
        }
        __syncthreads();
        qn = 0;
        rs = 0;
        re = 0;
    };

    const int qtot = dense ? S.qtot : S.soff[nslab];
    for (int c0 = 0; c0 < qtot || c0 == 0; c0 += TILE_CAP) {
        const int clen = dense ? min(TILE_CAP, qtot - c0) : qtot;
        // ---- stage sources of this chunk
        for (int sg = 0; sg < 27; ++sg) {
            const Seg g = S.seg[sg];
            if (g.glen == 0) continue;
            if (dense) {
                const int lo = max(g.so, c0), hi = min(g.so + g.glen, c0 + clen);
                for (int p = lo + lane; p < hi; p += 64)
                    stage_source<C>(S, P, p - c0, (int64_t)g.gstart + (p - g.so), g.offx, g.offy, g.offz);
            } else {
                const int cb = S.ccol[g.k] * n2;
                for (int j = g.gstart + lane; j < g.gstart + g.glen; j += 64) {
                    const int s = (P.skey[j] - cb) + g.vshift - za;
                    stage_source<C>(S, P, S.dtab[s * 9 + g.k] + j, (int64_t)j, g.offx, g.offy, g.offz);
                }
            }
        }
        if (clen + lane < C::CAPP) S.sc[clen + lane] = make_float4(1e18f, 1e18f, 1e18f, 0.0f);
        __syncthreads();

        // ---- scan: one target at a time over its contiguous stencil range
        for (int t = 0; t < ntgt; ++t) {
            const float tx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(thx), t));
            const float ty = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(thy), t));
            const float tz = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(thz), t));
            const int a = dense ? 0 : __builtin_amdgcn_readlane(my_a, t);
            const int b = dense ? clen : __builtin_amdgcn_readlane(my_b, t);
            if (lane == t) rs = qn;
            for (int p = a; p < b; p += 64) {
                if (qn + 64 > C::QCAP) {
                    if (lane == t) re = qn;
                    flush();
                }
                const int q = p + lane;
                const float4 s = S.sc[q];
                const float dx = s.x - tx, dy = s.y - ty, dz = s.z - tz;
                const float r2 = dx * dx + dy * dy + dz * dz;
                const bool hit = r2 < rc2s;
                const uint64_t m = __ballot(hit);
                if (hit) {
                    const int pos = qn + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    S.queue[pos] = ((uint32_t)t << 16) | (uint32_t)q;
                }
                qn += __popcll(m);
            }
            if (lane == t) re = qn;
        }
        flush();
        if (!dense) break;
    }

    // ---- write back in the original order
    if (lane < ntgt) {
        const int64_t orig = P.perm[tstart + lane];
        double res[C::NC];
        for (int c = 0; c < C::NC; ++c) res[c] = C::F32 ? (double)acc[c] - (double)cmp[c] : (double)acc[c];
        if constexpr (BWD) {
            for (int c = 0; c < C::MIN; ++c) P.out0[orig * C::MIN + c] = res[c];
            for (int c = 0; c < 3; ++c) P.out1[orig * 3 + c] = res[C::MIN + c];
        } else {
            for (int c = 0; c < C::MOUT; ++c) P.out0[orig * C::MOUT + c] = res[c];
        }
    }
}

// sorted SoA payload: pl[c][j] = rho[perm[j]][c] (c < m_in), then gu
__global__ void k_gather_payload(const double *__restrict__ rho, const double *__restrict__ gu,
                                 const int32_t *__restrict__ perm, int64_t N, int min_, int mout,
                                 double *__restrict__ pl)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int64_t i = perm[j];
    for (int c = 0; c < min_; ++c) pl[c * N + j] = rho[i * min_ + c];
    if (gu)
        for (int c = 0; c < mout; ++c) pl[(min_ + c) * N + j] = gu[i * mout + c];
}

}  // namespace dmk

using namespace dmk;

namespace {

int m_in_of(int k) { return k == 0 ? 1 : (k == 2 ? 9 : 3); }
int m_out_of(int k) { return k == 0 ? 1 : 3; }

int check_call(const dmk_grid *g, const dmk_bins *b, int kernel, int prec, double sigma, double rc)
{
    if (!g || !b) return DMK_EINVAL;
    if (g->D < 0 || g->D > 3) return DMK_EINVAL;
    double hmin = 1e308;
    for (int i = 0; i < 3; ++i) {
        if (g->n[i] < 1 || !(g->L[i] > 0.0) || !isfinite(g->L[i])) return DMK_EINVAL;
        const double h = g->L[i] / g->n[i];
        hmin = h < hmin ? h : hmin;
    }
    if (b->nbox != (int64_t)g->n[0] * g->n[1] * g->n[2]) return DMK_EINVAL;
    if (kernel < 0 || kernel > 3 || prec < 0 || prec > 1) return DMK_EUNSUPPORTED;
    if (!(sigma > 0.0) || !isfinite(sigma)) return DMK_ECUTOFF;
    if (!(rc > 0.0) || !(rc <= hmin)) return DMK_ECUTOFF;
    if (b->N > 0 && (!b->perm || !b->skey || !b->box_start || !b->ys || !b->tiles || !b->axis_nbr || !b->axis_img))
        return DMK_EINVAL;
    return DMK_OK;
}

size_t ws_need(int64_t N, int kernel, int backward)
{
    const int64_t ncomp = m_in_of(kernel) + (backward ? m_out_of(kernel) : 0);
    return (size_t)(sizeof(double) * ncomp * (N > 0 ? N : 1) + 256);
}

template <int KERN, typename FP, bool BWD>
void launch_one(const ResParams &P, hipStream_t s)
{
    const unsigned per = (unsigned)((P.ntiles + 7) / 8);
    hipLaunchKernelGGL((k_residual<KERN, FP, BWD>), dim3(8 * per), dim3(64), 0, s, P);
}

template <bool BWD>
int dispatch(int kernel, int prec, const ResParams &P, hipStream_t s)
{
    if (prec == DMK_FP64) {
        switch (kernel) {
        case 0: launch_one<0, double, BWD>(P, s); break;
        case 1: launch_one<1, double, BWD>(P, s); break;
        case 2: launch_one<2, double, BWD>(P, s); break;
        default: launch_one<3, double, BWD>(P, s); break;
        }
    } else {
        switch (kernel) {
        case 0: launch_one<0, float, BWD>(P, s); break;
        case 1: launch_one<1, float, BWD>(P, s); break;
        case 2: launch_one<2, float, BWD>(P, s); break;
        default: launch_one<3, float, BWD>(P, s); break;
        }
    }
    return hipGetLastError() == hipSuccess ? DMK_OK : DMK_EHIP;
}

ResParams make_params(const dmk_grid *g, const dmk_bins *b, double sigma, double rc, const double *pl)
{
    ResParams P{};
    for (int i = 0; i < 3; ++i) {
        P.L[i] = g->L[i];
        P.h[i] = g->L[i] / g->n[i];
        P.n[i] = g->n[i];
    }
    P.D = g->D;
    P.sigma = sigma;
    P.rc = rc;
    P.N = b->N;
    P.ntiles = (int)b->ntiles;
    P.ys = b->ys;
    P.skey = b->skey;
    P.bs = b->box_start;
    P.perm = b->perm;
    P.nbr = b->axis_nbr;
    P.img = b->axis_img;
    P.tiles = (const int4 *)b->tiles;
    P.pl = pl;
    return P;
}

}  // namespace

extern "C" size_t dmk_residual_ws_bytes(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec,
                                        int backward)
{
    (void)grid;
    (void)prec;
    if (!bins || kernel < 0 || kernel > 3) return 0;
    return ws_need(bins->N, kernel, backward);
}

extern "C" int dmk_residual_eval(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma,
                                 double rc, const double *rho, double *u, void *ws, size_t ws_bytes,
                                 hipStream_t stream)
{
    int rc_ = check_call(grid, bins, kernel, prec, sigma, rc);
    if (rc_ != DMK_OK) return rc_;
    const int64_t N = bins->N;
    if (N == 0) return DMK_OK;
    if (!rho || !u || !ws) return DMK_EINVAL;
    if (ws_bytes < ws_need(N, kernel, 0)) return DMK_ESIZE;
    double *pl = (double *)ws;
    hipLaunchKernelGGL(k_gather_payload, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream, rho,
                       (const double *)nullptr, bins->perm, N, m_in_of(kernel), m_out_of(kernel), pl);
    if (bins->ntiles == 0) return hipGetLastError() == hipSuccess ? DMK_OK : DMK_EHIP;
    ResParams P = make_params(grid, bins, sigma, rc, pl);
    P.out0 = u;
    return dispatch<false>(kernel, prec, P, stream);
}

extern "C" int dmk_residual_backward(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec,
                                     double sigma, double rc, const double *rho, const double *gu, double *grad_rho,
                                     double *grad_x, void *ws, size_t ws_bytes, hipStream_t stream)
{
    int rc_ = check_call(grid, bins, kernel, prec, sigma, rc);
    if (rc_ != DMK_OK) return rc_;
    const int64_t N = bins->N;
    if (N == 0) return DMK_OK;
    if (!rho || !gu || !grad_rho || !grad_x || !ws) return DMK_EINVAL;
    if (ws_bytes < ws_need(N, kernel, 1)) return DMK_ESIZE;
    double *pl = (double *)ws;
    hipLaunchKernelGGL(k_gather_payload, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, stream, rho, gu,
                       bins->perm, N, m_in_of(kernel), m_out_of(kernel), pl);
    ResParams P = make_params(grid, bins, sigma, rc, pl);
    P.out0 = grad_rho;
    P.out1 = grad_x;
    return dispatch<true>(kernel, prec, P, stream);
}
