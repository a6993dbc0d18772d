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
//  * queued pairs are evaluated 64 at a time, one per lane; a segmented sum
//    over the lanes (DPP moves) gives each target's run its total, which the
//    run's last lane adds to the target's FP64 sum in LDS.  Only the
//    wavefront that owns a target adds to its sum, in program order, so the
//    result is deterministic;
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

#include "dmk_dpp.h"
#include "dmk_internal.h"
#include "erfcx_f32.h"
#include "erfcx_f64.h"

namespace dmk {

template <int K>
struct KDim {
    static constexpr int MIN = (K == 0) ? 1 : ((K == 2) ? 9 : 3);
    static constexpr int MOUT = (K == 0) ? 1 : 3;
};

// a scan step reads a window of 128 staged slots
static_assert(TILE_CAP >= 2 * WAVE && TILE_CAP < 65536, "staged slots per tile");

template <int KERN, typename FP, bool BWD, bool HEAVY>
struct Cfg {
    static constexpr int K = KERN;
    static constexpr int MIN = KDim<KERN>::MIN;
    static constexpr int MOUT = KDim<KERN>::MOUT;
    static constexpr int NPL = BWD ? MIN + MOUT : MIN;   // payload per source
    static constexpr int NTP = BWD ? MIN + MOUT : 0;     // payload per target
    static constexpr int NC = BWD ? MIN + 3 : MOUT;      // sums per target
    static constexpr bool F32 = sizeof(FP) == 4;
    // A scan step tests 128 sources.  Full batches of the queue are evaluated
    // after each half of a step, or after the whole step for the FP64 adjoints
    // of the Stokes-flow kernels, whose long pair code is better inlined at
    // one call site; fewer than WAVE entries wait in between, so the queue
    // holds 2 or 3 WAVE entries.
    static constexpr bool DRAIN_HALF = F32 || !BWD || KERN == 0;
    static constexpr int QCAP = DRAIN_HALF ? 2 * WAVE : 3 * WAVE;
    // LDS bytes of the staged sources and of one wavefront's queue; tiles use
    // TILE_NW wavefronts, 8 when only one workgroup fits in the 160 KiB of a
    // CU (more resident waves for the same staged tile; the rest of the
    // workgroup's LDS is below 16 KiB), and 2 if TILE_NW would not fit at all.
    // The heavy-tile variant has HEAVY_NW instead of TILE_NW where that fits
    // in LDS (whether it runs is decided at launch, heavy_pays).
    static constexpr int STAGE_B = TILE_CAP * (16 + (F32 ? 16 + 4 * (NPL - 1) : 8 * (3 + NPL))) + 64;
    static constexpr int WAVE_B = QCAP * 4;
    static constexpr int NW0 = (STAGE_B + TILE_NW * WAVE_B > 150 * 1024) ? 2
                               : (STAGE_B + TILE_NW * WAVE_B + 16 * 1024 > 80 * 1024) ? 8
                                                                                        : TILE_NW;
    static constexpr int NW =
        (HEAVY && NW0 == TILE_NW && STAGE_B + HEAVY_NW * WAVE_B <= 150 * 1024) ? HEAVY_NW : NW0;
};

struct ResParams {
    double L[3], h[3];
    int n[3], D;
    double sigma, rc;
    int64_t N;
    int ntiles, tile0;  // end of this launch's tile range; its first tile
    int nheavy;         // leading tiles run with the heavy-tile workgroup
    const double *ys;
    const int32_t *skey, *bs, *perm, *nbr;
    const int8_t *img;
    const int4 *tiles;
    const double *pl;   // sorted strengths [MIN][N]
    const double *pg;   // sorted cotangent [MOUT][N] (adjoint)
    double *out0, *out1;
};

// payload component c of sorted point j: strengths, then (adjoint) cotangent
template <int MIN>
__device__ inline double payload(const ResParams &P, int c, int64_t j)
{
    return c < MIN ? P.pl[(int64_t)c * P.N + j] : P.pg[(int64_t)(c - MIN) * P.N + j];
}

// one source piece: a z-range of one neighbour column (piece 0: the image
// box below the domain, 1: boxes inside, 2: the image box above)
struct Seg {
    int gstart, glen, so;               // first sorted index, length, offset in the concatenation
    signed char k, vshift, piece, pad;  // column 0..8, virtual-z shift of an image box
};

template <class C>
struct Smem {
    static constexpr int S32 = C::F32 ? TILE_CAP : 1;
    static constexpr int S64 = C::F32 ? 1 : TILE_CAP;
    static constexpr int NX32 = (C::F32 && C::NPL > 1) ? C::NPL - 1 : 1;
    static constexpr int NX64 = C::F32 ? 1 : C::NPL;
    static constexpr int TX32 = (C::F32 && C::NTP > 1) ? C::NTP - 1 : 1;
    static constexpr int TX64 = (!C::F32 && C::NTP > 0) ? C::NTP : 1;
    // FP32 (hi) coords s and |s|^2 / 2 (scan test); the slot after the last
    // staged one holds a sentinel that no scan test accepts
    float4 sc[TILE_CAP + 4];
    float4 sl[S32];              // FP32 lo coords, w = payload 0 (FP32 path)
    float sp[NX32][(C::F32 && C::NPL > 1) ? TILE_CAP : 1];  // FP32 payload 1..
    double sx[S64], sy[S64], sz[S64];
    double spd[NX64][S64];
    float4 tc[TILE_T];           // target (hi) coords t, w = scan threshold (rc2s - |t|^2) / 2
    float4 tl[C::F32 ? TILE_T : 1];  // FP32 lo coords, w = target payload 0
    float tp[TX32][(C::F32 && C::NTP > 1) ? TILE_T : 1];  // FP32 target payload 1..
    double tx[C::F32 ? 1 : TILE_T], ty[C::F32 ? 1 : TILE_T], tz[C::F32 ? 1 : TILE_T];
    double tpd[TX64][(!C::F32 && C::NTP > 0) ? TILE_T : 1];
    int trange[TILE_T];          // stencil range [a, b) of each target in the staged order: a | b << 16
    union {
        uint32_t queue[C::NW][C::QCAP];   // pair queue of each wavefront (scan / pair step)
        struct {
            // per (slab, column) box: count | (start - start of its piece) << 16,
            // then slab-major offset - (start - start of its piece)
            int dtab[(TILE_ZMAX + 2) * 9];
        } st;                               // set-up and staging only
    };
    double tacc[C::NC][TILE_T];  // per-target sums (FP64 in both paths)
    int soff[TILE_ZMAX + 4];        // slab offsets in the staged order
    int ccol[9];
    int qtot;
    int segso[32];                  // piece offsets in the concatenated order (padded)
    Seg seg[27];
    double2 coff[9];                // tile-frame offset (x, y) of each neighbour column's points
    double zoff[3];                 // tile-frame z offset of each piece's points
};

// --------------------------------------------------------------------------
// scalar helpers
__device__ inline float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsqrt_(double x) { return rsqrt(x); }
__device__ inline double expneg_(double x) { return exp(-x); }


#define INV4PI 0.079577471545947667884
#define INV8PI 0.039788735772973833942
#define INV_SQRT_PI 0.56418958354775628695

// normalisation of each kernel: 1/(4 pi) for Laplace, 1/(8 pi) for the
// Stokes-flow kernels (the stresslet's 3/(4 pi) is 6 of those).  Every pair
// term is linear in exactly one source payload (rho_s or G_s), so the
// constant is applied to the source payloads, in FP64, when they are staged.
template <int KERN>
struct KNorm {
    static constexpr double c = KERN == 0 ? INV4PI : INV8PI;
};

// Window of the split: WIN_GAUSS (sigma = width) or WIN_PSWF (sigma = support
// radius nu), the latter as Chebyshev series in u = 2 t^2 - 1 of phi,
// (1 - Phi)/t, phi'/t and phi'' with WIN - 1 terms (WIN > 1; zero-padded by
// the host past the terms the window needs).
constexpr int WIN_GAUSS = 0;
template <int NT, typename T>
struct WinCoef {
    T c[4][NT];
};
struct NoWin {
    int unused;
};
template <int WIN, typename T>
using WinArg = typename std::conditional<(WIN > 1), WinCoef<(WIN > 1 ? WIN - 1 : 1), T>, NoWin>::type;

template <typename T>
struct Rad {
    T ri, r, t, t2, phi, Phi, dphi, d2phi;  // window values at t: phi, Phi, phi', phi''
};

// radial quantities of a pair at squared distance r2 (isig = 1/sigma,
// kexp = -log2(e)/sigma^2 for the FP32 exponential of the Gaussian window)
template <int WIN, typename T, typename W>
__device__ inline Rad<T> radial(T r2, T isig, T isig2, T kexp, const W &wc)
{
    Rad<T> R;
    R.ri = rsqrt_(r2);
    R.r = r2 * R.ri;
    R.t = R.r * isig;
    R.t2 = r2 * isig2;
    if constexpr (WIN > 1) {
        // Chebyshev polynomials T_k(u) by their recurrence, one sum per function
        constexpr int NT = WIN - 1;
        const T u = (T)2 * R.t2 - (T)1;
        T g[4];
        for (int q = 0; q < 4; ++q) g[q] = wc.c[q][0] + wc.c[q][1] * u;
        T tkm1 = (T)1, tk = u;
#pragma unroll
        for (int k = 2; k < NT; ++k) {
            const T tk1 = (T)2 * u * tk - tkm1;
            for (int q = 0; q < 4; ++q) g[q] += wc.c[q][k] * tk1;
            tkm1 = tk;
            tk = tk1;
        }
        (void)kexp;
        R.phi = g[0];
        R.Phi = (T)1 - R.t * g[1];
        R.dphi = R.t * g[2];
        R.d2phi = g[3];
        return R;
    } else if constexpr (sizeof(T) == 4) {
        // one exponential serves both the window phi(t) = e^{-t^2}/sqrt(pi) and
        // Phi(t) = erfc(t) = e^{-t^2} erfcx(t); erfcx from the fitted polynomial
        const float e = __builtin_amdgcn_exp2f(r2 * kexp);
        const float u = __builtin_amdgcn_rcpf(1.0f + ERFCX_F32_SHIFT * R.t);
        float pol = ERFCX_F32_C[ERFCX_F32_DEG];
#pragma unroll
        for (int k = ERFCX_F32_DEG - 1; k >= 0; --k) pol = pol * u + ERFCX_F32_C[k];
        R.phi = e * (float)INV_SQRT_PI;
        R.Phi = e * (u * pol);
    } else {
        // the same for FP64: erfcx(t) = u S(x), u = 1/(1 + t/2), S a fitted
        // Chebyshev series in x = A u + B (Clenshaw); branch-free, unlike a
        // library erfc whose argument ranges split the lanes of a wavefront
        (void)kexp;
        const double e = expneg_(R.t2);
        const double u = 1.0 / (1.0 + ERFCX_F64_SHIFT * R.t);
        const double x = fma(ERFCX_F64_A, u, ERFCX_F64_B);
        double b1 = 0.0, b2 = 0.0;
#pragma unroll
        for (int k = ERFCX_F64_DEG; k >= 1; --k) {
            const double b0 = fma(2.0 * x, b1, ERFCX_F64_C[k] - b2);
            b2 = b1;
            b1 = b0;
        }
        R.phi = e * INV_SQRT_PI;
        R.Phi = e * (u * fma(x, b1, ERFCX_F64_C[0] - b2));
    }
    (void)wc;
    R.dphi = (T)-2 * R.t * R.phi;                  // phi' = -2 t phi
    R.d2phi = ((T)4 * R.t2 - (T)2) * R.phi;         // phi'' = (4 t^2 - 2) phi
    return R;
}

// forward pair contribution v[MOUT]; ps = source strengths
template <int KERN, int WIN, typename T, typename W>
__device__ inline void pair_fwd(const T d[3], T r2, T isig, T isig2, T kexp, const W &wc, const T *ps, T *v)
{
    const Rad<T> R = radial<WIN, T>(r2, isig, isig2, kexp, wc);
    const T tphi2 = (T)2 * R.t * R.phi;
    if constexpr (KERN == 0) {
        v[0] = R.Phi * R.ri * ps[0];
    } else if constexpr (KERN == 1) {
        const T ri3 = R.ri * R.ri * R.ri;
        const T A = (R.Phi - tphi2) * R.ri;
        const T B = (R.Phi + tphi2) * ri3;
        const T df = d[0] * ps[0] + d[1] * ps[1] + d[2] * ps[2];
        const T Bdf = B * df;
        for (int c = 0; c < 3; ++c) v[c] = A * ps[c] + Bdf * d[c];
    } else if constexpr (KERN == 2) {
        const T ri2 = R.ri * R.ri;
        const T ri3 = ri2 * R.ri;
        const T t2dphi = R.t2 * R.dphi;
        const T P = (T)-2 * t2dphi * ri3;                                       // Td = -2 t^2 phi'
        const T Qc = -(T)6 * (R.Phi + tphi2 - (T)(2.0 / 3.0) * t2dphi) * ri3 * ri2;  // To
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
        const T f = (R.Phi + tphi2) * ri3;
        v[0] = f * (ps[1] * d[2] - ps[2] * d[1]);
        v[1] = f * (ps[2] * d[0] - ps[0] * d[2]);
        v[2] = f * (ps[0] * d[1] - ps[1] * d[0]);
    }
}

// adjoint pair contribution v[MIN + 3] = (d grad_rho_t, d grad_x_t);
// ps = (rho_s, G_s), pt = (rho_t, G_t); d = x_t - x_s (+ image).  Radial
// derivatives d/dt of the window parts: Sd' = -4 phi - 2 t phi',
// So' = 2 t phi', Td' = -4 t phi' - 2 t^2 phi'', To' = (2/3)(t phi' - t^2 phi''),
// Oo' = 2 t phi' (with Phi' = -2 phi); d/dr = (1/sigma) d/dt.
template <int KERN, int WIN, typename T, typename W>
__device__ inline void pair_bwd(const T d[3], T r2, T isig, T isig2, T kexp, const W &wc, const T *ps, const T *pt,
                                T *v)
{
    constexpr int MIN = KDim<KERN>::MIN;
    const T *rs = ps, *Gs = ps + MIN, *rt = pt, *Gt = pt + MIN;
    const Rad<T> R = radial<WIN, T>(r2, isig, isig2, kexp, wc);
    const T tphi2 = (T)2 * R.t * R.phi;
    const T ri2 = R.ri * R.ri;
    const T ri3 = ri2 * R.ri;
    if constexpr (KERN == 0) {
        const T K = R.Phi * R.ri;
        const T g = -(R.Phi + tphi2) * ri3;
        v[0] = K * Gs[0];
        const T s = g * (Gt[0] * rs[0] + Gs[0] * rt[0]);
        for (int c = 0; c < 3; ++c) v[1 + c] = s * d[c];
    } else if constexpr (KERN == 1) {
        const T Sd = R.Phi - tphi2, So = R.Phi + tphi2;
        const T A = Sd * R.ri;
        const T B = So * ri3;
        const T tdphi = R.t * R.dphi;
        const T dSd = (T)-4 * R.phi - (T)2 * tdphi;
        const T dSo = (T)2 * tdphi;
        const T Ar = dSd * isig * ri2 - Sd * ri3;                      // A'(r)/r
        const T Br = dSo * isig * ri2 * ri2 - (T)3 * So * ri3 * ri2;   // B'(r)/r
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
        const T t2dphi = R.t2 * R.dphi, tdphi = R.t * R.dphi, t2d2phi = R.t2 * R.d2phi;
        const T Td = (T)-2 * t2dphi;
        const T To = R.Phi + tphi2 - (T)(2.0 / 3.0) * t2dphi;
        const T P = Td * ri3;
        const T ri5 = ri3 * ri2;
        const T Qc = -(T)6 * To * ri5;
        const T dTd = (T)-4 * tdphi - (T)2 * t2d2phi;
        const T dTo = (T)(2.0 / 3.0) * (tdphi - t2d2phi);
        const T Pr = dTd * isig * ri2 * ri2 - (T)3 * Td * ri5;
        const T Qr = -(T)6 * (dTo * isig * ri3 * ri3 - (T)5 * To * ri5 * ri2);
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
        const T f = Oo * ri3;
        const T dOo = (T)2 * R.t * R.dphi;
        const T fr = dOo * isig * ri2 * ri2 - (T)3 * Oo * ri3 * ri2;
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
__device__ inline void store_source(Smem<C> &S, int dest, double X, double Y, double Z, const double *pl)
{
    if constexpr (C::F32) {
        const float hx = (float)X, hy = (float)Y, hz = (float)Z;
        const float lx = (float)(X - (double)hx), ly = (float)(Y - (double)hy), lz = (float)(Z - (double)hz);
        S.sc[dest] = make_float4(hx, hy, hz, 0.5f * (hx * hx + hy * hy + hz * hz));
        S.sl[dest] = make_float4(lx, ly, lz, (float)pl[0]);
        for (int c = 1; c < C::NPL; ++c) S.sp[c - 1][dest] = (float)pl[c];
    } else {
        const float fx = (float)X, fy = (float)Y, fz = (float)Z;
        S.sc[dest] = make_float4(fx, fy, fz, 0.5f * (fx * fx + fy * fy + fz * fz));
        S.sx[dest] = X;
        S.sy[dest] = Y;
        S.sz[dest] = Z;
        for (int c = 0; c < C::NPL; ++c) S.spd[c][dest] = pl[c];
    }
}

// Stage the sources of one chunk [c0, c0+clen) of the tile's concatenated
// pieces.  Multi-box tiles (dense == false, one chunk) place every source at
// its slab-major slot dtab[slab*9 + column] + rank in its piece; dense tiles keep the
// concatenated order.  Each thread handles up to PER sources and issues all
// of their global loads before its first LDS store.
template <class C>
__device__ inline void stage_chunk(Smem<C> &S, const ResParams &P, bool dense, int c0, int clen, int za, int n2,
                                   int tid)
{
    constexpr int NT = C::NW * WAVE;
    constexpr int PER = (TILE_CAP + NT - 1) / NT;
    const int64_t N = P.N;
    int sgi[PER], sk[PER], rk[PER];
    int64_t jj[PER];
    double X[PER], Y[PER], Z[PER], pl[PER][C::NPL];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int q = tid + u * NT;
        const int qc = (dense ? c0 : 0) + (q < clen ? q : 0);
        int lo = 0;  // last piece whose offset is <= qc
#pragma unroll
        for (int step = 16; step > 0; step >>= 1)
            if (S.segso[lo + step] <= qc) lo += step;
        sgi[u] = lo;
        rk[u] = qc - S.seg[lo].so;  // rank within the piece
        jj[u] = (int64_t)S.seg[lo].gstart + rk[u];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        if (tid + u * NT < clen) {
            const int64_t j = jj[u];
            const Seg &g = S.seg[sgi[u]];
            const double2 co = S.coff[g.k];
            X[u] = P.ys[j] + co.x;
            Y[u] = P.ys[N + j] + co.y;
            Z[u] = P.ys[2 * N + j] + S.zoff[g.piece];
            for (int c = 0; c < C::NPL; ++c) pl[u][c] = payload<C::MIN>(P, c, j) * KNorm<C::K>::c;  // normalised
            sk[u] = dense ? 0 : P.skey[j];
        }
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int q = tid + u * NT;
        if (q < clen) {
            int dest = q;
            if (!dense) {
                const Seg &g = S.seg[sgi[u]];
                const int slab = (sk[u] - S.ccol[g.k] * n2) + g.vshift - za;
                dest = S.st.dtab[slab * 9 + g.k] + rk[u];
            }
            store_source<C>(S, dest, X[u], Y[u], Z[u], pl[u]);
        }
    }
}

// neighbour box index along one axis for offset off in {-1,0,1}, with the
// image index of the neighbour's points (periodic axes wrap, free axes end);
// the same definition as the binning's axis tables, evaluated in registers
__device__ inline int axis_nb(const ResParams &P, int ax, int b, int off, int &img)
{
    const int n = P.n[ax];
    int nb = b + off;
    img = 0;
    if (ax < P.D) {
        if (nb < 0) {
            nb += n;
            img = -1;
        } else if (nb >= n) {
            nb -= n;
            img = 1;
        }
    } else if (nb < 0 || nb >= n) {
        nb = -1;
    }
    return nb;
}

// wavefront-local ordering of LDS accesses (the LDS unit serves one
// wavefront's instructions in order; this stops compiler reordering)
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Segmented inclusive sum over the 64 lanes.  Lanes hold values v[NC] whose
// tags (>= 1) are non-decreasing along the lanes; afterwards the last lane
// of each run of equal tags holds the run's total.  Shifts by 1, 2, 4, 8
// within each row of 16 lanes, then the row totals are carried into rows 1
// and 3 (from lanes 15, 47) and into rows 2 and 3 (from lane 31), the usual
// wavefront scan pattern.  In a shift step lane l passes its partial sum to
// lane l + s when that lane carries the same tag (tested at the sender, as
// the tags are sorted); in a carry step the receiver tests the sender's tag.
// Returns whether lane l is the last of its run.
template <int S, int NC, typename T>
__device__ inline bool seg_shift(int tag, T *v)
{
    // tag of lane l + S (0 past the end of the row, or of the wavefront for
    // S = 1, so the result also marks the last lane of each run)
    const int tn = dpp_int<S == 1 ? DPP_WAVE_SHL1 : DPP_ROW_SHL + S, 0xf>(tag, 0);
    const bool pass = tn == tag;
    for (int c = 0; c < NC; ++c) {
        const T w = pass ? v[c] : (T)0;
        v[c] += dpp_val<DPP_ROW_SHR + S, 0xf>(w);
    }
    return !pass;
}
template <int CTRL, int RM, int NC, typename T>
__device__ inline void seg_carry(int tag, T *v)
{
    const bool same = dpp_int<CTRL, RM>(tag, 0) == tag;  // false in rows not written
    for (int c = 0; c < NC; ++c) {
        const T x = dpp_any<CTRL, RM>(v[c]);
        v[c] += same ? x : (T)0;
    }
}
template <int NC, typename T>
__device__ inline bool seg_sum(int tag, T *v)
{
    const bool last = seg_shift<1, NC>(tag, v);
    seg_shift<2, NC>(tag, v);
    seg_shift<4, NC>(tag, v);
    seg_shift<8, NC>(tag, v);
    seg_carry<DPP_ROW_BCAST15, 0xa, NC>(tag, v);
    seg_carry<DPP_ROW_BCAST31, 0xc, NC>(tag, v);
    return last;
}

template <int KERN, typename FP, bool BWD, int WIN, bool HEAVY>
__global__ __launch_bounds__((Cfg<KERN, FP, BWD, HEAVY>::NW * WAVE)) void k_residual(ResParams P,
                                                                                     WinArg<WIN, FP> WC)
{
    using C = Cfg<KERN, FP, BWD, HEAVY>;
    using T = FP;
    __shared__ Smem<C> S;
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    // wavefront index, uniform across the wavefront (readfirstlane tells the
    // compiler so: loops bounded by it then keep their control in scalar regs)
    const int w = __builtin_amdgcn_readfirstlane(tid / WAVE);
    // tiles are ordered heavy-first by the binning; consecutive workgroups go
    // to different XCDs, which spreads the heavy tiles over all of them
    const int tile = P.tile0 + (int)blockIdx.x;
    if (tile >= P.ntiles) return;

    const int4 TD = P.tiles[tile];
    const int n1 = P.n[1], n2 = P.n[2];
    const int col = TD.x, z0 = TD.y;
    const bool dense = TD.z < 0;
    const int z1 = dense ? z0 : TD.z;
    const int tstart = TD.w;
    const int64_t colb = (int64_t)col * n2;
    const int ntgt = dense ? min(TILE_T, P.bs[colb + z0 + 1] - tstart) : (P.bs[colb + z1 + 1] - tstart);
    const int b0 = col / n1, b1 = col - (col / n1) * n1;
    // tile frame: origin at the centre of the column's middle z-box range
    const double crx = (b0 + 0.5) * P.h[0], cry = (b1 + 0.5) * P.h[1], crz = ((z0 + z1) * 0.5 + 0.5) * P.h[2];
    const int za = z0 - 1, zb = z1 + 1, nslab = z1 - z0 + 3;

    const T isig = (T)(1.0 / P.sigma);
    const T isig2 = isig * isig;
    const T kexp = (T)(-1.4426950408889634 / (P.sigma * P.sigma));  // -log2(e) / sigma^2
    const T rc2 = (T)(P.rc * P.rc);
    // Scan test (FP32, conservative): source s is queued for target t when
    // |s|^2 - 2 s.t < rc2s - |t|^2 (both sides halved in the code).  The
    // rounding error of that expansion and of the FP32 coordinates is a few
    // ulp of (|s| + |t|)^2 <= 4 R^2, with R the largest coordinate norm in
    // the tile frame; the margin exceeds it twentyfold.  The pair step then
    // applies the exact test.
    const double ext_z = (z1 - z0) * 0.5 + 1.5;
    const double R2 = 2.25 * (P.h[0] * P.h[0] + P.h[1] * P.h[1]) + ext_z * ext_z * P.h[2] * P.h[2];
    const float rc2s = (float)(P.rc * P.rc * (1.0 + 4e-4) + 4.2e-5 * R2);

    // ---- phase A: every global load of the tile set-up issued before any
    // of them is used, so that the set-up waits on memory once after the
    // tile descriptor.  A load whose piece, box or target does not exist
    // reads index 0 (the box starts and the sorted arrays are never empty
    // here) and its value is dropped: a load behind a branch would be waited
    // for inside that branch.
    //  * tid < 27: source piece (neighbour column k = tid/3, z piece tid%3)
    //  * tid < 9 * nslab: box count of the slab-major table (multi-box
    //    tiles; the entries past the workgroup size, tall tiles only, are
    //    loaded afterwards)
    //  * tid < TILE_T: target coordinates, payload, box and original index
    Seg g;
    g.glen = 0;
    g.gstart = 0;
    g.k = 0;
    g.vshift = 0;
    g.piece = 0;
    g.pad = 0;
    int64_t sga = 0, sgb = 0;  // box starts of the piece (when it has boxes)
    bool sgok = false;
    if (tid < 27) {
        const int k = tid / 3, piece = tid % 3, c0 = k / 3, c1 = k % 3;
        g.k = (signed char)k;
        g.piece = (signed char)piece;
        int i0, i1;
        const int nb0 = axis_nb(P, 0, b0, c0 - 1, i0), nb1 = axis_nb(P, 1, b1, c1 - 1, i1);
        if (piece == 1) S.coff[k] = make_double2(i0 * P.L[0] - crx, i1 * P.L[1] - cry);
        if (k == 0) {
            // z image of each piece: -1 below, +1 above (periodic z), 0 inside
            int zi = 0;
            if (piece == 0) axis_nb(P, 2, 0, -1, zi);
            if (piece == 2) axis_nb(P, 2, n2 - 1, 1, zi);
            S.zoff[piece] = zi * P.L[2] - crz;
        }
        if (nb0 >= 0 && nb1 >= 0) {
            const int cc = nb0 * n1 + nb1;
            const int64_t cb = (int64_t)cc * n2;
            int lo = 1, hi = 0, zimg = 0;
            if (piece == 0 && za == -1) {  // virtual z = -1
                lo = hi = axis_nb(P, 2, 0, -1, zimg);
                g.vshift = -1 - lo;
            } else if (piece == 1) {       // virtual z in [max(za,0), min(zb,n2-1)]
                lo = za < 0 ? 0 : za;
                hi = zb > n2 - 1 ? n2 - 1 : zb;
            } else if (piece == 2 && zb == n2) {  // virtual z = n2
                lo = hi = axis_nb(P, 2, n2 - 1, 1, zimg);
                g.vshift = n2 - lo;
            }
            if (lo >= 0 && lo <= hi) {
                sgok = true;
                sga = cb + lo;
                sgb = cb + hi + 1;
            }
            (void)zimg;
            if (piece == 1) S.ccol[k] = cc;
        } else if (piece == 1) {
            S.ccol[k] = -1;
        }
    }
    const int M = dense ? 0 : nslab * 9;
    int64_t dta = 0, dtc = 0;  // box start of the entry's box, and of the first box of its piece
    bool dtok = false, dtpre = false;
    if (tid < M) {
        const int sl = tid / 9, k = tid - (tid / 9) * 9;
        int i0, i1, iz;
        const int nb0 = axis_nb(P, 0, b0, k / 3 - 1, i0), nb1 = axis_nb(P, 1, b1, k % 3 - 1, i1);
        const int zv = za + sl;
        const int zp = (zv < 0) ? axis_nb(P, 2, 0, -1, iz) : (zv >= n2 ? axis_nb(P, 2, n2 - 1, 1, iz) : zv);
        if (nb0 >= 0 && nb1 >= 0 && zp >= 0) {
            const int64_t cb = (int64_t)(nb0 * n1 + nb1) * n2;
            dtok = true;
            dta = cb + zp;
            // boxes inside the domain form one piece starting at max(za, 0)
            dtpre = zv >= 0 && zv < n2;
            dtc = cb + (za < 0 ? 0 : za);
        }
    }
    const bool tgok = tid < TILE_T && tstart + tid < P.N;  // all 64 slots; ones past ntgt are never used
    const int64_t j = tgok ? tstart + tid : 0;
    // the loads
    const int sgv0 = P.bs[sga], sgv1 = P.bs[sgb];
    const int dtv0 = P.bs[dta], dtv1 = P.bs[dta + 1], dtv2 = P.bs[dtc];
    const double ysx = P.ys[j], ysy = P.ys[P.N + j], ysz = P.ys[2 * P.N + j];
    double tpl[C::NTP > 0 ? C::NTP : 1];
    for (int c = 0; c < C::NTP; ++c) tpl[c] = payload<C::MIN>(P, c, j);
    const int skj = P.skey[j], pmj = P.perm[j];
    // their uses
    if (tid < 27) {
        if (sgok) {
            g.gstart = sgv0;
            g.glen = sgv1 - sgv0;
        }
        S.seg[tid] = g;
    }
    if (tid < M) S.st.dtab[tid] = dtok ? (dtv1 - dtv0) | ((dtpre ? dtv0 - dtv2 : 0) << 16) : 0;
    for (int idx = tid + C::NW * WAVE; idx < M; idx += C::NW * WAVE) {
        const int sl = idx / 9, k = idx - (idx / 9) * 9;
        int i0, i1, iz;
        const int nb0 = axis_nb(P, 0, b0, k / 3 - 1, i0), nb1 = axis_nb(P, 1, b1, k % 3 - 1, i1);
        const int zv = za + sl;
        const int zp = (zv < 0) ? axis_nb(P, 2, 0, -1, iz) : (zv >= n2 ? axis_nb(P, 2, n2 - 1, 1, iz) : zv);
        int cnt = 0, pre = 0;
        if (nb0 >= 0 && nb1 >= 0 && zp >= 0) {
            const int64_t cb = (int64_t)(nb0 * n1 + nb1) * n2;
            const int gs = P.bs[cb + zp];
            cnt = P.bs[cb + zp + 1] - gs;
            if (zv >= 0 && zv < n2) pre = gs - P.bs[cb + (za < 0 ? 0 : za)];
        }
        S.st.dtab[idx] = cnt | (pre << 16);
    }
    for (int idx = tid; idx < C::NC * TILE_T; idx += C::NW * WAVE) (&S.tacc[0][0])[idx] = 0.0;
    int my_zt = 0, my_orig = 0;
    if (tgok) {
        const double X = ysx - crx, Y = ysy - cry, Z = ysz - crz;
        const float hx = (float)X, hy = (float)Y, hz = (float)Z;
        S.tc[tid] = make_float4(hx, hy, hz, 0.5f * (rc2s - (hx * hx + hy * hy + hz * hz)));
        if constexpr (C::F32) {
            const float t0 = (C::NTP > 0) ? (float)tpl[0] : 0.0f;
            S.tl[tid] = make_float4((float)(X - (double)hx), (float)(Y - (double)hy), (float)(Z - (double)hz), t0);
            for (int c = 1; c < C::NTP; ++c) S.tp[c - 1][tid] = (float)tpl[c];
        } else {
            S.tx[tid] = X;
            S.ty[tid] = Y;
            S.tz[tid] = Z;
            for (int c = 0; c < C::NTP; ++c) S.tpd[c][tid] = tpl[c];
        }
        if (!dense) my_zt = skj - (int)colb;
        my_orig = pmj;
    }
    __syncthreads();

    // ---- phase B (LDS only): piece offsets in the concatenated order, and the
    // slab-major offsets dtab[s*9+k] (multi-box tiles)
    if (w == 0) {
        // inclusive scan of the 27 piece lengths
        const int gl = lane < 27 ? S.seg[lane].glen : 0;
        const int incl = wave_incl_scan(gl);
        if (lane < 27) S.seg[lane].so = incl - gl;
        if (lane < 32) S.segso[lane] = lane < 27 ? incl - gl : 0x7fffffff;
        if (lane == 26) S.qtot = incl;
    }
    if (!dense && w == 1) {
        int carry = 0;
        for (int base = 0; base < M; base += WAVE) {
            const int idx = base + lane;
            const int e = idx < M ? S.st.dtab[idx] : 0;
            const int cnt = e & 0xffff;
            const int incl = wave_incl_scan(cnt);
            if (idx < M) {
                const int off = carry + incl - cnt;
                S.st.dtab[idx] = off - (e >> 16);
                if (idx % 9 == 0) S.soff[idx / 9] = off;
            }
            carry += __builtin_amdgcn_readlane(incl, WAVE - 1);
        }
        if (lane == 0) S.soff[nslab] = carry;
    }
    __syncthreads();
    if (!dense && tid < ntgt) S.trange[tid] = S.soff[my_zt - z0] | (S.soff[my_zt - z0 + 3] << 16);

    int qn = 0;  // entries in this wavefront's queue (uniform)
    uint32_t *queue = S.queue[w];

    // pair step for queue entry e = (t << 16) | source slot: contribution
    // v[NC] (zero when the exact test rejects the pair: self / coincident, or
    // outside the cutoff)
    auto pair_value = [&](uint32_t e, T *v) {
        const int t = (int)(e >> 16), q = (int)(e & 0xffffu);
        T d[3], ps[C::NPL], pt[C::NTP > 0 ? C::NTP : 1];
        if constexpr (C::F32) {
            const float4 sh = S.sc[q], sl = S.sl[q], th = S.tc[t], tl = S.tl[t];
            d[0] = (th.x - sh.x) + (tl.x - sl.x);
            d[1] = (th.y - sh.y) + (tl.y - sl.y);
            d[2] = (th.z - sh.z) + (tl.z - sl.z);
            ps[0] = sl.w;
            for (int c = 1; c < C::NPL; ++c) ps[c] = S.sp[c - 1][q];
            if constexpr (C::NTP > 0) {
                pt[0] = tl.w;
                for (int c = 1; c < C::NTP; ++c) pt[c] = S.tp[c - 1][t];
            }
        } else {
            d[0] = S.tx[t] - S.sx[q];
            d[1] = S.ty[t] - S.sy[q];
            d[2] = S.tz[t] - S.sz[q];
            for (int c = 0; c < C::NPL; ++c) ps[c] = S.spd[c][q];
            for (int c = 0; c < C::NTP; ++c) pt[c] = S.tpd[c][t];
        }
        // a rejected pair (coincident points, or outside the cutoff) may give
        // non-finite intermediates; its result is replaced by zero
        const T r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const bool ok = (r2 > (T)0) && (r2 < rc2);
        if constexpr (BWD)
            pair_bwd<KERN, WIN, T>(d, r2, isig, isig2, kexp, WC, ps, pt, v);
        else
            pair_fwd<KERN, WIN, T>(d, r2, isig, isig2, kexp, WC, ps, v);
        for (int c = 0; c < C::NC; ++c) v[c] = ok ? v[c] : (T)0;
    };

    // Pair step over queue entries [base, base + cnt), cnt <= 64, one per lane.
    //  * multi-box tiles: a batch holds the pairs of several targets, each
    //    target's entries one run of consecutive lanes; a segmented sum over
    //    the lanes leaves each run's total in its last lane, which adds it to
    //    the target's FP64 sum (only this wavefront touches that sum, one
    //    batch after another, so the order is fixed);
    //  * dense tiles: a batch holds one target's pairs; each lane keeps a
    //    running FP32 sum part[] of at most TILE_CAP / 64 terms, reduced when
    //    the target's range in the chunk is done and added to its FP64 sum.
    T part[C::NC];
    for (int c = 0; c < C::NC; ++c) part[c] = 0;
    auto batch = [&](int base, int cnt) {
        T v[C::NC];
        for (int c = 0; c < C::NC; ++c) v[c] = 0;
        int tag = 127;  // lanes past cnt: a run of their own, never added
        if (lane < cnt) {
            const uint32_t e = queue[base + lane];
            pair_value(e, v);
            tag = (int)(e >> 16) + 1;
        }
        if (dense) {
            for (int c = 0; c < C::NC; ++c) part[c] += v[c];
        } else {
            // a target's entries are one run of the batch: its total goes to
            // the run's last lane, the only lane that adds to that target
            const bool last = seg_sum<C::NC>(tag, v);
            if (lane < cnt && last)
                for (int c = 0; c < C::NC; ++c) S.tacc[c][tag - 1] += (double)v[c];
        }
    };

    // evaluate full batches from the top of the queue (its last 64 entries,
    // in target order like the whole queue) until fewer than 64 are left;
    // the entries below stay where they are
    auto drain = [&]() {
        wave_sync();
        for (; qn >= WAVE; qn -= WAVE) batch(qn - WAVE, WAVE);
        wave_sync();
    };

    const int qtot = dense ? S.qtot : S.soff[nslab];
    for (int c0 = 0; c0 < qtot || c0 == 0; c0 += TILE_CAP) {
        const int clen = dense ? min(TILE_CAP, qtot - c0) : qtot;
        // ---- stage sources of this chunk: flat over the concatenated pieces,
        // all loads of a thread issued before any of its LDS stores; the slot
        // after the last one gets the sentinel (|s|^2 / 2 = +inf)
        stage_chunk<C>(S, P, dense, c0, clen, za, n2, tid);
        if (tid == 0) S.sc[clen] = make_float4(0.0f, 0.0f, 0.0f, INFINITY);
        __syncthreads();

        // ---- scan: one target at a time over its contiguous stencil range;
        // wavefront w takes the consecutive targets [t0, t1) (an even share),
        // so that consecutive targets mostly lie in one box and share their
        // range: a one-step range already held in s0, s1 is not read again.
        // The target's coordinates and threshold are read from LDS at a
        // uniform address (a broadcast).
        const int t0 = (w * ntgt) / C::NW, t1 = ((w + 1) * ntgt) / C::NW;
        int pa = -1;  // first slot of the one-step window held in s0, s1 (-1: none)
        float4 s0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), s1 = s0;
        for (int t = t0; t < t1; ++t) {
            const float4 ts = S.tc[t];
            const float tx = ts.x, ty = ts.y, tz = ts.z, thr = ts.w;
            int a = 0, b = clen;
            if (!dense) {
                const int rg = __builtin_amdgcn_readfirstlane(S.trange[t]);
                a = rg & 0xffff;
                b = rg >> 16;
            }
            const uint32_t tag = (uint32_t)t << 16;
            // Each step tests sources [p, p + 128).  Slots past b belong to
            // other slabs, farther than the cutoff (the pair step's exact test
            // rejects any that pass the conservative scan test); a lane whose
            // slot is at or past clen reads the sentinel slot clen instead,
            // which fails the test.  The hit test is one compare and its ballot
            // is the compare's lane mask.  Hits are appended at queue[qn ..) in
            // lane order, those of the first half first; entry = (t << 16) |
            // source slot.
            const bool one = b - a <= 2 * WAVE;
            for (int p = a; p < b; p += 2 * WAVE) {
                if (p != pa) {
                    s0 = S.sc[min(p + lane, clen)];
                    s1 = S.sc[min(p + WAVE + lane, clen)];
                    pa = one ? p : -1;
                }
                // (|s|^2 - 2 s.t) / 2 against (rc2s - |t|^2) / 2
                const float ra = fmaf(-s0.x, tx, fmaf(-s0.y, ty, fmaf(-s0.z, tz, s0.w)));
                const float rb = fmaf(-s1.x, tx, fmaf(-s1.y, ty, fmaf(-s1.z, tz, s1.w)));
                const bool ha = ra < thr, hb = rb < thr;
                const uint64_t ma = __builtin_amdgcn_ballot_w64(ha), mb = __builtin_amdgcn_ballot_w64(hb);
                const uint32_t ea = (tag | (uint32_t)p) + (uint32_t)lane;
                const uint32_t ra_ = __builtin_amdgcn_mbcnt_hi((uint32_t)(ma >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ma, 0u));
                const uint32_t rb_ = __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
                if constexpr (C::DRAIN_HALF) {
                    if (ha) queue[qn + ra_] = ea;
                    qn += __popcll(ma);
                    if (qn >= WAVE) drain();
                    if (hb) queue[qn + rb_] = ea + (uint32_t)WAVE;
                    qn += __popcll(mb);
                    if (qn >= WAVE) drain();
                } else {
                    const int na = __popcll(ma);
                    if (ha) queue[qn + ra_] = ea;
                    if (hb) queue[qn + na + rb_] = ea + (uint32_t)WAVE;
                    qn += na + __popcll(mb);
                    if (qn >= WAVE) drain();
                }
            }
            if (dense) {
                // the rest of this target's pairs, then its total
                wave_sync();
                if (qn > 0) batch(0, qn);
                qn = 0;
                wave_sum<C::NC>(part);
                if (lane == WAVE - 1)
                    for (int c = 0; c < C::NC; ++c) S.tacc[c][t] += (double)part[c];
                for (int c = 0; c < C::NC; ++c) part[c] = 0;
                wave_sync();
            }
        }
        if (!dense && qn > 0) {
            wave_sync();
            batch(0, qn);
            qn = 0;
        }
        __syncthreads();
        if (!dense) break;
    }

    // ---- each target's FP64 sums, written back in the original order
    if (tid < ntgt) {
        const int64_t orig = my_orig;
        double res[C::NC];
        for (int c = 0; c < C::NC; ++c) res[c] = S.tacc[c][tid];
        if constexpr (BWD) {
            for (int c = 0; c < C::MIN; ++c) P.out0[orig * C::MIN + c] = res[c];
            for (int c = 0; c < 3; ++c) P.out1[orig * 3 + c] = res[C::MIN + c];
        } else {
            for (int c = 0; c < C::MOUT; ++c) P.out0[orig * C::MOUT + c] = res[c];
        }
    }
}

// Sorted SoA copy of a per-point array: dst[c][j] = src[perm[j]][c].  Each
// thread reads one record of M doubles at a random position (perm) and
// writes M coalesced values; all of its loads are issued before its stores.
template <int M>
__global__ void k_gather_sorted(const double *__restrict__ src, const int32_t *__restrict__ perm, int64_t N,
                                double *__restrict__ dst)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= N) return;
    const int64_t i = perm[j];
    double v[M];
    if constexpr (M % 2 == 0) {
        const double2 *r2 = (const double2 *)(src + i * M);
#pragma unroll
        for (int c = 0; c < M / 2; ++c) {
            const double2 t = r2[c];
            v[2 * c] = t.x;
            v[2 * c + 1] = t.y;
        }
    } else {
#pragma unroll
        for (int c = 0; c < M; ++c) v[c] = src[i * M + c];
    }
#pragma unroll
    for (int c = 0; c < M; ++c) dst[c * N + j] = v[c];
}

}  // namespace dmk

using namespace dmk;

namespace {

int m_in_of(int k) { return k == 0 ? 1 : (k == 2 ? 9 : 3); }
int m_out_of(int k) { return k == 0 ? 1 : 3; }

// sorted SoA copy of m components (1 <= m <= DMK_GATHER_MMAX)
int gather_m(int m, const double *src, const int32_t *perm, int64_t N, double *dst, hipStream_t s)
{
    if (N <= 0) return DMK_OK;
    if (N > (int64_t)0x3fffffff) return DMK_ESIZE;
    // one launch of 256-thread workgroups: below 2^32 work-items for the
    // at most 2^30 - 1 points a binning holds
    const dim3 grid((unsigned)((N + 255) / 256)), blk(256);
    switch (m) {
#define DMK_G(M) \
    case M: hipLaunchKernelGGL((k_gather_sorted<M>), grid, blk, 0, s, src, perm, N, dst); break;
        DMK_G(1) DMK_G(2) DMK_G(3) DMK_G(4) DMK_G(5) DMK_G(6) DMK_G(7) DMK_G(8) DMK_G(9) DMK_G(10) DMK_G(11)
        DMK_G(12)
#undef DMK_G
    default: return DMK_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? DMK_OK : DMK_EHIP;
}

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
    if (b->nheavy < 0 || b->nheavy > b->ntiles) return DMK_EINVAL;
    return DMK_OK;
}

int check_window(const dmk_pswf *w)
{
    if (!w) return DMK_EINVAL;
    if (!(w->c > 0.0) || !(w->c <= DMK_PSWF_CMAX) || w->nterms64 < 1 || w->nterms64 > DMK_PSWF_MAXTERMS ||
        w->nterms32 < 1 || w->nterms32 > DMK_PSWF_MAXTERMS32)
        return DMK_EUNSUPPORTED;
    return DMK_OK;
}

// split arguments of a call: the Gaussian of width sigma with cutoff rc
// (w null), or the PSWF window w of support rc (sigma unused)
int check_split(const dmk_grid *g, const dmk_bins *b, int kernel, int prec, double sigma, double rc,
                const dmk_pswf *w)
{
    if (w) {
        const int st = check_window(w);
        if (st != DMK_OK) return st;
        sigma = rc;
    }
    return check_call(g, b, kernel, prec, sigma, rc);
}

// workspace of dmk_residual_eval / _backward: the sorted strengths, and for
// the adjoint the sorted cotangent after them (256-byte aligned)
size_t ws_part(int64_t N, int m) { return ((size_t)sizeof(double) * m * (size_t)(N > 0 ? N : 1) + 255) & ~(size_t)255; }
size_t ws_need(int64_t N, int kernel, int backward)
{
    return ws_part(N, m_in_of(kernel)) + (backward ? ws_part(N, m_out_of(kernel)) : 0) + 256;
}

// tiles [t0, t1), one workgroup per tile, in launches of fewer than 2^32
// work-items
template <int KERN, typename FP, bool BWD, int WIN, bool HEAVY>
void launch_range(const ResParams &P, int t0, int t1, const WinArg<WIN, FP> &wc, hipStream_t s)
{
    constexpr int NT = Cfg<KERN, FP, BWD, HEAVY>::NW * WAVE;
    constexpr int MAXB = (int)(0xffffffffu / NT);
    for (int a = t0; a < t1; a += MAXB) {
        ResParams Q = P;
        Q.tile0 = a;
        Q.ntiles = t1;
        hipLaunchKernelGGL((k_residual<KERN, FP, BWD, WIN, HEAVY>), dim3((unsigned)min(MAXB, t1 - a)), dim3(NT), 0,
                           s, Q, wc);
        if (t1 - a <= MAXB) break;
    }
}

// Whether heavy tiles run with the larger workgroup: only where it keeps
// more wavefronts resident per CU than the smaller one, given each variant's
// LDS and register use.  A tile's waves split its long scans between them,
// so on a heavy tile more waves hide more of the latency of each; where the
// registers or LDS allow no more resident waves, the larger workgroup only
// adds waiting at its barriers (measured slower on clustered inputs).  Asked
// on every call that has heavy tiles (a host-side query of the current
// device; nothing is cached); a failed query leaves its error for the
// launch check.
template <int KERN, typename FP, bool BWD, int WIN>
bool heavy_pays()
{
    constexpr int NL = Cfg<KERN, FP, BWD, false>::NW * WAVE;
    constexpr int NH = Cfg<KERN, FP, BWD, true>::NW * WAVE;
    if (NL == NH) return false;
    int bl = 0, bh = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bl, k_residual<KERN, FP, BWD, WIN, false>, NL, 0) !=
            hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&bh, k_residual<KERN, FP, BWD, WIN, true>, NH, 0) != hipSuccess)
        return false;
    return bh * NH > bl * NL;
}

template <int KERN, typename FP, bool BWD, int WIN>
void launch_one(const ResParams &P, const dmk_pswf *w, hipStream_t s)
{
    WinArg<WIN, FP> wc{};
    if constexpr (WIN > 1) {
        // the series of the precision's path, zero past the terms it keeps
        const int nt = sizeof(FP) == 4 ? w->nterms32 : w->nterms64;
        for (int q = 0; q < 4; ++q)
            for (int k = 0; k < WIN - 1; ++k) wc.c[q][k] = k < nt ? (FP)w->cheb[q][k] : (FP)0;
    } else {
        (void)w;
    }
    // the heavy tiles [0, nheavy) with the larger workgroup where it pays,
    // then the others (all tiles in one range otherwise)
    const int nh = (P.nheavy > 0 && heavy_pays<KERN, FP, BWD, WIN>()) ? P.nheavy : 0;
    if (nh > 0) launch_range<KERN, FP, BWD, WIN, true>(P, 0, nh, wc, s);
    launch_range<KERN, FP, BWD, WIN, false>(P, nh, P.ntiles, wc, s);
}

template <bool BWD, int WIN>
int dispatch(int kernel, int prec, const ResParams &P, const dmk_pswf *w, hipStream_t s)
{
    if (prec == DMK_FP64) {
        switch (kernel) {
        case 0: launch_one<0, double, BWD, WIN>(P, w, s); break;
        case 1: launch_one<1, double, BWD, WIN>(P, w, s); break;
        case 2: launch_one<2, double, BWD, WIN>(P, w, s); break;
        default: launch_one<3, double, BWD, WIN>(P, w, s); break;
        }
    } else {
        switch (kernel) {
        case 0: launch_one<0, float, BWD, WIN>(P, w, s); break;
        case 1: launch_one<1, float, BWD, WIN>(P, w, s); break;
        case 2: launch_one<2, float, BWD, WIN>(P, w, s); break;
        default: launch_one<3, float, BWD, WIN>(P, w, s); break;
        }
    }
    return hipGetLastError() == hipSuccess ? DMK_OK : DMK_EHIP;
}

ResParams make_params(const dmk_grid *g, const dmk_bins *b, double sigma, double rc)
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
    P.nheavy = (int)b->nheavy;
    P.ys = b->ys;
    P.skey = b->skey;
    P.bs = b->box_start;
    P.perm = b->perm;
    P.nbr = b->axis_nbr;
    P.img = b->axis_img;
    P.tiles = (const int4 *)b->tiles;
    return P;
}

// the pair kernel alone; w selects the PSWF window (null: Gaussian)
template <bool BWD>
int launch_pairs(int kernel, int prec, const ResParams &P, const dmk_pswf *w, hipStream_t s)
{
    if (P.ntiles <= 0) return DMK_OK;
    if (!w) return dispatch<BWD, WIN_GAUSS>(kernel, prec, P, w, s);
    // PSWF: Chebyshev series of 16 / 24 terms (FP32) or 24 / 32 (FP64), the
    // shortest that holds the window's terms; WIN = terms + 1
    if (prec == DMK_FP32C)
        return w->nterms32 <= 16 ? dispatch<BWD, 17>(kernel, prec, P, w, s) : dispatch<BWD, 25>(kernel, prec, P, w, s);
    return w->nterms64 <= 24 ? dispatch<BWD, 25>(kernel, prec, P, w, s) : dispatch<BWD, 33>(kernel, prec, P, w, s);
}

int eval_sorted_impl(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma, double rc,
                     const dmk_pswf *w, const double *rho_s, double *u, hipStream_t stream)
{
    const int st = check_split(grid, bins, kernel, prec, sigma, rc, w);
    if (st != DMK_OK) return st;
    if (bins->N == 0) return DMK_OK;
    if (!rho_s || !u) return DMK_EINVAL;
    ResParams P = make_params(grid, bins, w ? rc : sigma, rc);
    P.pl = rho_s;
    P.out0 = u;
    return launch_pairs<false>(kernel, prec, P, w, stream);
}

int backward_sorted_impl(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma, double rc,
                         const dmk_pswf *w, const double *rho_s, const double *gu_s, double *grad_rho,
                         double *grad_x, hipStream_t stream)
{
    const int st = check_split(grid, bins, kernel, prec, sigma, rc, w);
    if (st != DMK_OK) return st;
    if (bins->N == 0) return DMK_OK;
    if (!rho_s || !gu_s || !grad_rho || !grad_x) return DMK_EINVAL;
    ResParams P = make_params(grid, bins, w ? rc : sigma, rc);
    P.pl = rho_s;
    P.pg = gu_s;
    P.out0 = grad_rho;
    P.out1 = grad_x;
    return launch_pairs<true>(kernel, prec, P, w, stream);
}

// gather + pair kernel, the workspace holding the sorted payload
int eval_impl(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma, double rc,
              const dmk_pswf *w, const double *rho, double *u, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const int st = check_split(grid, bins, kernel, prec, sigma, rc, w);
    if (st != DMK_OK) return st;
    const int64_t N = bins->N;
    if (N == 0) return DMK_OK;
    if (!rho || !u || !ws) return DMK_EINVAL;
    if (ws_bytes < ws_need(N, kernel, 0)) return DMK_ESIZE;
    double *pl = (double *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    const int g = gather_m(m_in_of(kernel), rho, bins->perm, N, pl, stream);
    if (g != DMK_OK) return g;
    return eval_sorted_impl(grid, bins, kernel, prec, sigma, rc, w, pl, u, stream);
}

int backward_impl(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma, double rc,
                  const dmk_pswf *w, const double *rho, const double *gu, double *grad_rho, double *grad_x,
                  void *ws, size_t ws_bytes, hipStream_t stream)
{
    const int st = check_split(grid, bins, kernel, prec, sigma, rc, w);
    if (st != DMK_OK) return st;
    const int64_t N = bins->N;
    if (N == 0) return DMK_OK;
    if (!rho || !gu || !grad_rho || !grad_x || !ws) return DMK_EINVAL;
    if (ws_bytes < ws_need(N, kernel, 1)) return DMK_ESIZE;
    double *pl = (double *)(((uintptr_t)ws + 255) & ~(uintptr_t)255);
    double *pg = (double *)((char *)pl + ws_part(N, m_in_of(kernel)));
    int g = gather_m(m_in_of(kernel), rho, bins->perm, N, pl, stream);
    if (g == DMK_OK) g = gather_m(m_out_of(kernel), gu, bins->perm, N, pg, stream);
    if (g != DMK_OK) return g;
    return backward_sorted_impl(grid, bins, kernel, prec, sigma, rc, w, pl, pg, grad_rho, grad_x, stream);
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

extern "C" int dmk_gather_sorted(const dmk_bins *bins, int m, const double *src, double *dst, hipStream_t stream)
{
    if (!bins || m < 1 || m > DMK_GATHER_MMAX) return DMK_EINVAL;
    if (bins->N == 0) return DMK_OK;
    if (!bins->perm || !src || !dst) return DMK_EINVAL;
    return gather_m(m, src, bins->perm, bins->N, dst, stream);
}

extern "C" int dmk_residual_eval(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma,
                                 double rc, const double *rho, double *u, void *ws, size_t ws_bytes,
                                 hipStream_t stream)
{
    return eval_impl(grid, bins, kernel, prec, sigma, rc, nullptr, rho, u, ws, ws_bytes, stream);
}

extern "C" int dmk_residual_backward(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec,
                                     double sigma, double rc, const double *rho, const double *gu, double *grad_rho,
                                     double *grad_x, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return backward_impl(grid, bins, kernel, prec, sigma, rc, nullptr, rho, gu, grad_rho, grad_x, ws, ws_bytes,
                         stream);
}

extern "C" int dmk_residual_eval_pswf(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec,
                                      const dmk_pswf *w, double nu, const double *rho, double *u, void *ws,
                                      size_t ws_bytes, hipStream_t stream)
{
    if (!w) return DMK_EINVAL;
    return eval_impl(grid, bins, kernel, prec, nu, nu, w, rho, u, ws, ws_bytes, stream);
}

extern "C" int dmk_residual_backward_pswf(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec,
                                          const dmk_pswf *w, double nu, const double *rho, const double *gu,
                                          double *grad_rho, double *grad_x, void *ws, size_t ws_bytes,
                                          hipStream_t stream)
{
    if (!w) return DMK_EINVAL;
    return backward_impl(grid, bins, kernel, prec, nu, nu, w, rho, gu, grad_rho, grad_x, ws, ws_bytes, stream);
}

extern "C" int dmk_residual_eval_sorted(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec,
                                        double sigma, double rc, const dmk_pswf *w, const double *rho_sorted,
                                        double *u, hipStream_t stream)
{
    return eval_sorted_impl(grid, bins, kernel, prec, sigma, rc, w, rho_sorted, u, stream);
}

extern "C" int dmk_residual_backward_sorted(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec,
                                            double sigma, double rc, const dmk_pswf *w, const double *rho_sorted,
                                            const double *gu_sorted, double *grad_rho, double *grad_x,
                                            hipStream_t stream)
{
    return backward_sorted_impl(grid, bins, kernel, prec, sigma, rc, w, rho_sorted, gu_sorted, grad_rho, grad_x,
                                stream);
}
