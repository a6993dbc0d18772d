/*
 * dmk.h -- C ABI of libdmkloc: the leaf-level residual (short-range) kernel
 * interaction of the periodized DMK method on one AMD MI355X (gfx950), with
 * the binning it runs on and, further down, the root-level far field of the
 * triply periodic split, the leaf boxes' Chebyshev grids (proxy strengths,
 * evaluation at targets) and the self-interaction correction.
 *
 * Operation (Sec. 2.3, eq. (u_local); image set P_D of eq. (periodic-images),
 * Sec. 1): for every point x_b of the cell [0,L1)x[0,L2)x[0,L3), whose first
 * D axes are periodic,
 *
 *     u_b = sum_a sum_{p in P_D} [0 < |d| < rc] K_R(d; sigma) rho_a,
 *     d   = x_b - x_a + p,
 *
 * where sources and targets are the same N points.  The term |d| = 0 is the
 * excluded self/coincident term of eq. (periodic_sum).  K_R is the residual
 * kernel of the Gaussian split (window phi(t) = exp(-t^2)/sqrt(pi),
 * Phi = erfc, functions evaluated at t = r/sigma):
 *
 *     DMK_LAPLACE    erfc(t)/(4 pi r) q                     eq. (Hhatsplit_wfunc)
 *     DMK_STOKESLET  residual Stokeslet S_R f               App. B eq. (res_stokeslet)
 *     DMK_STRESSLET  residual stresslet T_R : rho (rho 3x3) App. B eq. (res_stresslet)
 *     DMK_ROTLET     residual rotlet Omega_R rho            App. B eq. (res_rotlet)
 *
 * The cell is tiled by n1 x n2 x n3 leaf boxes of side h_i = L_i/n_i (the
 * exact cube tiling of Sec. 4.1.1 at the leaf level).  With rc <= min_i h_i
 * every interaction of a target lies in its own leaf box and its 26
 * neighbours (colleagues, Sec. 3.1.1 and 3.1.5); neighbours across a
 * periodic face are the image-shifted boxes (Sec. 4.1.2-4.1.3).
 *
 * Conventions
 *  - All pointers named "dev" are device pointers on the current HIP device.
 *    The caller owns every byte: the library allocates nothing and keeps no
 *    global state, so calls on different streams with different arenas are
 *    independent.  The one exception is dmk_residual_eval_noalloc (below),
 *    whose workspace is a device array of the library itself.
 *  - User-facing arrays are row-major in the ORIGINAL point order and FP64:
 *      x[N][3], rho[N][m_in], u[N][m_out], grad_rho[N][m_in], grad_x[N][3]
 *    with (m_in, m_out) = (1,1) Laplace, (3,3) Stokeslet, (9,3) stresslet
 *    (rho_lm row-major, u_j = T_jlm rho_lm), (3,3) rotlet.
 *  - prec selects only the internal pair arithmetic: DMK_FP64, or DMK_FP32C
 *    (FP32 pair arithmetic on hi/lo FP32 coordinates formed in FP64; the
 *    FP32 pair terms are summed per target in FP64).
 *  - Return value: a dmk_status.  Argument errors are detected on the host
 *    before any launch.  dmk_residual_eval / _backward return right after
 *    their launches (asynchronous on `stream`).  dmk_tree_bin synchronises
 *    `stream` once to read back its data checks.
 */
#ifndef DMK_H
#define DMK_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DMK_OK = 0,
    DMK_EINVAL = 1,       /* bad argument (null pointer, size, enum)                 */
    DMK_EDOMAIN = 2,      /* non-finite coordinate, or free-axis coordinate outside [0,L) */
    DMK_ECUTOFF = 3,      /* rc not in (0, min h_i], or sigma <= 0                   */
    DMK_EUNSUPPORTED = 4, /* combination not supported by the library               */
    DMK_EHIP = 5,         /* a HIP runtime call failed                               */
    DMK_ESIZE = 6         /* arena / workspace too small, or N / box count too large */
} dmk_status;

typedef enum { DMK_LAPLACE = 0, DMK_STOKESLET = 1, DMK_STRESSLET = 2, DMK_ROTLET = 3 } dmk_kernel;
typedef enum { DMK_FP64 = 0, DMK_FP32C = 1 } dmk_prec;

/* Cell and leaf tiling: cell [0,L[0])x[0,L[1])x[0,L[2]); axes 0..D-1 are
 * periodic (eq. (periodic-images)), the others free; n[i] >= 1 leaf boxes
 * along axis i. */
typedef struct {
    double L[3];
    int32_t D;
    int32_t n[3];
} dmk_grid;

/*
 * Binned point set.  All pointers are device pointers carved by
 * dmk_bins_carve from ONE caller-owned device arena; the scalar fields are
 * host values.  Box id of leaf (b0,b1,b2) is (b0*n1 + b1)*n2 + b2.
 * "Sorted order" is the stable counting-sort order by box id (points of a box
 * keep their original relative order).
 */
typedef struct {
    int64_t N;           /* number of points                                   */
    int64_t nbox;        /* n0*n1*n2                                           */
    int64_t ntiles;      /* target tiles built by dmk_tree_bin (host value)    */
    int64_t nheavy;      /* leading tiles of high cost, run with more           */
                         /*          wavefronts per workgroup (host value;     */
                         /*          residual calls reject it outside          */
                         /*          [0, ntiles] with DMK_EINVAL)              */
    int64_t max_tiles;   /* capacity of `tiles`                                */
    int32_t *key;        /* [N]      box id of each point, original order       */
    int32_t *perm;       /* [N]      sorted position -> original index          */
    int32_t *skey;       /* [N]      box id in sorted order                     */
    int32_t *box_start;  /* [nbox+1] first sorted position of each box          */
    double *ys;          /* [3][N]   wrapped coordinates, sorted order (SoA)    */
    int32_t *axis_nbr;   /* [n0+n1+n2][3] neighbour box index along each axis    */
                         /*          for offsets -1,0,+1, or -1 if none (free)  */
    int8_t *axis_img;    /* [n0+n1+n2][3] image index s in {-1,0,1}: the        */
                         /*          neighbour's points sit at x + s*L_i         */
    int32_t *tiles;      /* [max_tiles][4] target tiles {leaf column, z0, z1 or  */
                         /*          -(z0+1) for one dense box, first target}  */
    int32_t *status;     /* [4] device error word, tile count, heavy tiles      */
    int32_t *tmp;        /* sort / tile scratch                                  */
    int64_t tmp_ints;    /* size of tmp in int32                                 */
} dmk_bins;

/* Bytes of device arena dmk_bins_carve needs for N points on `grid`
 * (0 on invalid arguments). */
size_t dmk_bins_bytes(const dmk_grid *grid, int64_t N);

/* Carve the arena (device pointer, >= dmk_bins_bytes bytes, 256-byte
 * aligned) into `bins`.  No device work.  DMK_EINVAL / DMK_ESIZE on bad
 * input. */
int dmk_bins_carve(const dmk_grid *grid, int64_t N, void *dev_arena, size_t arena_bytes, dmk_bins *bins);

/*
 * Bin the points x[N][3] (dev, FP64, original order) into the leaf tiling:
 *  - periodic axis: y = x - L floor(x/L); free axis: 0 <= x < L required;
 *  - box index b_i = min(n_i - 1, floor(y_i * (n_i / L_i))), IEEE FP64 ops
 *    without contraction, so the result is bit-exact;
 *  - stable counting sort by box id (perm, skey, box_start), the sorted
 *    wrapped coordinates ys, the per-axis neighbour/image tables and the
 *    target tiles used by the residual kernels.
 * Runs on `stream`, then synchronises it once to read the error word:
 * DMK_EDOMAIN if any coordinate is non-finite or a free-axis coordinate is
 * outside [0, L).  Sets bins->ntiles and bins->nheavy (tiles are ordered by
 * descending power-of-two cost class; the first nheavy are the costly ones).
 */
int dmk_tree_bin(const dmk_grid *grid, const double *x, dmk_bins *bins, hipStream_t stream);

/* Workspace bytes for dmk_residual_eval (backward = 0) or
 * dmk_residual_backward (backward = 1). */
size_t dmk_residual_ws_bytes(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, int backward);

/*
 * u[N][m_out] (dev, FP64, original order) = residual sum above with strengths
 * rho[N][m_in] (dev, FP64, original order).  Requires 0 < sigma and
 * 0 < rc <= min_i h_i (DMK_ECUTOFF otherwise).  `ws` is a device workspace of
 * >= dmk_residual_ws_bytes(.., 0) bytes.  Asynchronous on `stream`; u is
 * fully overwritten.  Summation order is fixed, so results are bit-identical
 * between runs.
 */
int dmk_residual_eval(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma, double rc,
                      const double *rho, double *u, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Vector-Jacobian product of dmk_residual_eval: with cotangent
 * gu[N][m_out] (dev) and F = sum_b gu_b . u_b,
 *     grad_rho[N][m_in] = dF/drho,   grad_x[N][3] = dF/dx
 * (both dev, FP64, original order, fully overwritten).  The cutoff mask is
 * treated as locally constant.  Same argument rules as dmk_residual_eval;
 * workspace of >= dmk_residual_ws_bytes(.., 1) bytes.  Asynchronous.
 */
int dmk_residual_backward(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma,
                          double rc, const double *rho, const double *gu, double *grad_rho, double *grad_x,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * PSWF window (Sec. 2.2, eq. (wfunc_pswf)): phi(t) = psi_0^c(t) / int psi_0^c
 * on |t| < 1 and Phi(t) = 1 - 2 int_0^t phi, with psi_0^c the zeroth-order
 * prolate spheroidal wave function of bandwidth c (eq. (PSWFeig)).  The
 * residual kernels of the split at length nu are the formulas of App. B
 * (eqs. (Hhatsplit_wfunc), (Soffdiag), (T-offd), (ROoffd)) at t = r/nu, and
 * vanish for r >= nu (remark on compact support).
 *
 * dmk_pswf_window fills w (host memory, computed on the host) for
 * 0 < c <= DMK_PSWF_CMAX: Chebyshev coefficients, in u = 2 t^2 - 1, of
 * phi(t), (1 - Phi(t))/t, phi'(t)/t and phi''(t), and the number of terms
 * the FP64 / FP32 paths use.  Returns DMK_EINVAL (null w) or
 * DMK_EUNSUPPORTED (c out of range).
 */
#define DMK_PSWF_MAXTERMS 32   /* terms per function, FP64 path */
#define DMK_PSWF_MAXTERMS32 24 /* terms per function, FP32 path */
#define DMK_PSWF_CMAX 40.0
typedef struct {
    double c;
    int32_t nterms64, nterms32;
    double cheb[4][DMK_PSWF_MAXTERMS];
} dmk_pswf;
int dmk_pswf_window(double c, dmk_pswf *w);

/*
 * dmk_residual_eval / dmk_residual_backward with the PSWF split of support
 * radius nu instead of the Gaussian: same arguments, layouts, workspace and
 * error rules, with `w` (host pointer, from dmk_pswf_window, read during the
 * call) and 0 < nu <= min_i h_i in place of (sigma, rc).
 */
int dmk_residual_eval_pswf(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, const dmk_pswf *w,
                           double nu, const double *rho, double *u, void *ws, size_t ws_bytes, hipStream_t stream);
int dmk_residual_backward_pswf(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, const dmk_pswf *w,
                               double nu, const double *rho, const double *gu, double *grad_rho, double *grad_x,
                               void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * The residual sums of dmk_residual_eval / dmk_residual_backward split into
 * their two steps, for callers that keep strengths in the sorted order (an
 * adjoint that reuses the forward's sorted strengths, or a caller that times
 * the pair kernel alone with its own events around the call).
 *
 * dmk_gather_sorted: dst[c][j] = src[perm[j]][c] for the N points of `bins`
 * and c < m: src[N][m] (dev, FP64, original order), dst[m][N] (dev, FP64,
 * sorted order, rows N apart).  1 <= m <= DMK_GATHER_MMAX.  Asynchronous.
 * DMK_EINVAL on a bad m or null pointer, DMK_ESIZE for more than 2^30 - 1
 * points.
 *
 * dmk_residual_eval_sorted: u[N][m_out] (dev, original order) from the sorted
 * strengths rho_sorted[m_in][N] (as dmk_gather_sorted writes them).
 * dmk_residual_backward_sorted: grad_rho[N][m_in], grad_x[N][3] (dev,
 * original order) from rho_sorted[m_in][N] and the sorted cotangent
 * gu_sorted[m_out][N].  Both launch the pair kernel only, asynchronously on
 * `stream`, and need no workspace.  With w == NULL the split is the Gaussian
 * of width sigma with cutoff rc; with a PSWF window w (dmk_pswf_window) it is
 * the PSWF split of support nu = rc, and sigma is not used.  Argument rules
 * and results are those of the calls above (bit-identical output).
 */
#define DMK_GATHER_MMAX 12
int dmk_gather_sorted(const dmk_bins *bins, int m, const double *src, double *dst, hipStream_t stream);
int dmk_residual_eval_sorted(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma,
                             double rc, const dmk_pswf *w, const double *rho_sorted, double *u, hipStream_t stream);
int dmk_residual_backward_sorted(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma,
                                 double rc, const dmk_pswf *w, const double *rho_sorted, const double *gu_sorted,
                                 double *grad_rho, double *grad_x, hipStream_t stream);

/*
 * dmk_residual_eval for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments and results as dmk_residual_eval (the same
 * kernels, bit-identical u), without a workspace argument.  The sorted
 * strengths go to a device array of the library, DMK_NOALLOC_WS_BYTES bytes
 * that each GPU the library runs on holds from its first such call (the
 * array's address is looked up then, once per device) until the process
 * ends.  The call allocates nothing.  Errors: those of dmk_residual_eval, and
 * DMK_ESIZE when dmk_residual_ws_bytes(.., 0) exceeds the array, i.e. for
 * N > 8,388,576 Laplace, > 2,796,192 Stokeslet or rotlet, > 932,064 stresslet
 * points.  All calls on one GPU share its array: calls that overlap
 * on one GPU (other streams, other host threads) race and must not be issued.
 * Asynchronous on `stream`.
 */
#define DMK_NOALLOC_WS_BYTES (64 << 20)
int dmk_residual_eval_noalloc(const dmk_grid *grid, const dmk_bins *bins, int kernel, int prec, double sigma,
                              double rc, const double *rho, double *u, hipStream_t stream);

/* Static description of a status code. */
const char *dmk_strerror(int status);

/* Library version string. */
const char *dmk_version(void);

/*
 * Root-level far field of the triply periodic split (D = 3; Sec. 4,
 * evaluation of the far-field contribution, eqs. (structurefac),
 * (eval_tensor), wave numbers of eqs. (wavenumbers-3p-trunc), (kintmax)).
 *
 * The cell [0,L0)x[0,L1)x[0,L2) is covered by M0 x M1 x M2 top-level cubes of
 * side h0: either they tile it exactly (h0 = L_i / M_i, equal on the three
 * axes), or they are the smallest cover by cubes of the shortest side
 * (Sec. 4.1.1), h0 = min_i L_i and M_i = ceil(L_i / h0), the last cube along
 * an axis whose length is not a multiple of h0 reaching past the cell's face
 * (its proxy strengths then come from the points inside the cell, as for any
 * cube; the wave numbers are those of the cell).  Each cube carries a
 * p x p x p grid of first-kind Chebyshev points, (h0/2) cos((2j-1) pi/(2p)),
 * j = 1..p, about its centre.  Along axis i the grid coordinates of all cubes
 * form one list of G_i = M_i p entries, index g = b p + (j - 1) (cube b),
 * coordinate (b + 1/2) h0 + (h0/2) cos((2j-1) pi/(2p)).
 *
 * Given proxy strengths rho on those grid points, dmk_far3p_eval computes
 * on the same points
 *
 *   u_j(x) = sum_{k != 0} Re[ e^{i k.x} sum_q Khat_jq(k; sigma0) chi_q(k) ],
 *   chi_q(k) = (1/(L0 L1 L2)) sum_y e^{-i k.y} rho_q(y),
 *   k = 2 pi (n0/L0, n1/L1, n2/L2), |n_i| <= K_i,
 *
 * with Khat the Fourier transform of the mollified kernel (harmonic,
 * Stokeslet, stresslet, rotlet; App. A) for the Gaussian window of width
 * sigma0 (win = NULL, phihat(q) = exp(-q^2/4)) or the PSWF window of support
 * sigma0 (win from dmk_pswf_window).  The stresslet's extra k = 0
 * compensation term is not included.
 *
 * Both sums factor over the axes (sum factorization).  On an exact tiling,
 * an axis of 8 or more cubes factors further through a DFT over the cube
 * index (Sec. 4, large aspect ratios): a dense product up to 64 cubes, an
 * FFT (O(M_i log M_i) per column) from 65 cubes on, for any M_i up to
 * DMK_FAR_MMAX (Bluestein's convolution when M_i has a prime factor above
 * 8).  Such an axis needs only the first cube's phase table, so the
 * workspace grows linearly in M_i.
 *
 * Layout (dev, FP64): rho_grid[m_in][G0][G1][G2], u_grid[m_out][G0][G1][G2]
 * (last index fastest).  `ws` is a device workspace of >= dmk_far3p_ws_bytes
 * bytes.  Asynchronous on `stream`; u_grid is fully overwritten.  Errors:
 * DMK_EINVAL (null pointer, p outside [1, DMK_FAR_PMAX], M_i outside
 * [1, DMK_FAR_MMAX], K_i outside [0, DMK_FAR_KMAX], M that is neither an exact
 * tiling nor the cover above), DMK_ECUTOFF (sigma0 <= 0), DMK_EUNSUPPORTED (bad window, or
 * |k|max sigma0 > 4096 with the PSWF window), DMK_ESIZE (workspace too small,
 * or sizes for which one kernel launch would hold 2^32 or more work-items:
 * about 6.7e7 wave numbers with all n_i >= 0, 4.3e9 in all, or grid
 * contractions of that order).
 */
#define DMK_FAR_PMAX 64
#define DMK_FAR_MMAX 4096
#define DMK_FAR_KMAX 65536

typedef struct {
    double L[3];
    int32_t M[3];
    int32_t p;
    int32_t K[3];
} dmk_far_grid;

/* Workspace bytes for dmk_far3p_eval, or 0 for invalid arguments. */
size_t dmk_far3p_ws_bytes(const dmk_far_grid *fg, int kernel);

int dmk_far3p_eval(const dmk_far_grid *fg, int kernel, double sigma0, const dmk_pswf *win, const double *rho_grid,
                   double *u_grid, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Leaf-box Chebyshev grids (Sec. 3.1: every box carries a p x p x p grid of
 * first-kind Chebyshev points; upward pass: proxy charges by anterpolation;
 * leaf level: the smooth potential's expansion evaluated at the targets).
 *
 * The boxes are the leaf boxes of `grid` as binned in `bins` (dmk_tree_bin).
 * Grid values of all boxes form one tensor [m][n0 p][n1 p][n2 p] (index
 * g_i = b_i p + (j - 1) for node j of box b_i; dev, FP64), the layout of
 * dmk_far3p_eval when the leaf boxes are the top cubes.  In a box of side
 * h_i the node j sits at (b_i + 1/2) h_i + (h_i/2) cos((2j-1) pi/(2p)); l_j is
 * the tensor-product Lagrange basis on the nodes, in the box-local coordinate
 * of the point's wrapped position (the binning's box).  m in {1, 3, 9};
 * p in [1, DMK_FAR_PMAX].  `ws` is a device workspace of >= dmk_cheb_ws_bytes
 * bytes.  Asynchronous on `stream`.  Errors: DMK_EINVAL (bad p, m, pointer,
 * or bins not of this grid), DMK_ESIZE (workspace too small or tensor too
 * large).
 *
 * dmk_cheb_anterp: rho_grid[q](g) = sum over the points a of the box of g of
 *   rho[a][q] l_j(x_a)  (rho[N][m] in the original order; rho_grid fully
 *   overwritten).
 * dmk_cheb_eval: u[a][q] = sum_j u_grid[q](box of a, j) l_j(x_a), stored to
 *   u[N][m] (original order), or added to it when accumulate != 0.
 */
size_t dmk_cheb_ws_bytes(const dmk_bins *bins, int p);
int dmk_cheb_anterp(const dmk_grid *grid, const dmk_bins *bins, int p, int m, const double *rho, double *rho_grid,
                    void *ws, size_t ws_bytes, hipStream_t stream);
int dmk_cheb_eval(const dmk_grid *grid, const dmk_bins *bins, int p, int m, const double *u_grid, int accumulate,
                  double *u, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Self-interaction correction of the split (Sec. 2.4, eq. (S_self)): the far
 * field contains the k-space image of each point's own mollified kernel; for
 * the harmonic kernel and the Stokeslet it is removed by
 *   u[i][j] += -phi(0) rho[i][j] / (2 pi sigma0)
 * (phi the window: Gaussian of width sigma0 when win = NULL, else the PSWF
 * window of support sigma0).  The stresslet and rotlet have none (no-op).
 * u[N][m_out], rho[N][m_in] dev FP64, original order.  Asynchronous.
 */
int dmk_self_term(int kernel, double sigma0, const dmk_pswf *win, int64_t N, const double *rho, double *u,
                  hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* DMK_H */
