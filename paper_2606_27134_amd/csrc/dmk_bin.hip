// dmk_bin.hip -- leaf binning for libdmkloc on gfx950.
//
// The leaf level of the method is an exact tiling of the cell by n0 x n1 x n2
// boxes (Sec. 4.1.1 at the leaf level); the residual interaction of a target
// involves its own box and the 26 colleagues (Sec. 3.1.1, 3.1.5), with
// periodic neighbours across the faces of the first D axes (Sec. 4.1.2,
// 4.1.3).  This file builds, all with integer or contraction-free IEEE FP64
// arithmetic so that the output is bit-exact:
//   1. the wrapped coordinate y and the box id of every point;
//   2. a stable LSD radix sort (digits of up to 9 bits) of the box ids ->
//      perm, skey;
//   3. box_start from the key changes of the sorted ids (or by binary search
//      when there are fewer points than boxes);
//   4. the sorted wrapped coordinates ys (SoA);
//   5. the per-axis neighbour / image tables;
//   6. the target tiles walked by the residual kernels.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>

#include "dmk_dpp.h"
#include "dmk_internal.h"

#pragma clang fp contract(off)

namespace dmk {

struct BinGeom {
    double L[3];
    double inv[3];  // n_i / L_i, formed on the host
    int n[3];
    int D;
};

// ---------------------------------------------------------------------------
// 1. wrap + box id
__device__ inline bool wrap_coord(double xc, int ax, const BinGeom &g, double &y)
{
    if (!isfinite(xc)) return false;
    if (ax < g.D) {
        y = xc - g.L[ax] * floor(xc / g.L[ax]);
        return true;
    }
    if (!(xc >= 0.0 && xc < g.L[ax])) return false;
    y = xc;
    return true;
}

__device__ inline int box_coord(double y, int ax, const BinGeom &g)
{
    double f = floor(y * g.inv[ax]);
    int b = (f < 0.0) ? 0 : (f >= (double)g.n[ax] ? g.n[ax] - 1 : (int)f);
    return b;
}


// ---------------------------------------------------------------------------
// 2. stable LSD radix sort of (key, original index), digits of up to 9 bits
//    (RS_BINS buckets): as few passes as the key width allows.
constexpr int RS_THREADS = 256;
constexpr int RS_ITEMS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
constexpr int RS_MAXBITS = 9;
constexpr int RS_BINS = 1 << RS_MAXBITS;
constexpr int RS_BPT = RS_BINS / RS_THREADS;  // buckets per thread

// Workgroup barrier that orders LDS only: waits for this wavefront's LDS
// operations, not for its global stores (__syncthreads also waits for those,
// which costs a memory round trip where no thread reads them back).
__device__ inline void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Order of LDS accesses within one wavefront (which the LDS unit serves in
// order): a compiler fence only.
__device__ inline void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Key tile of radix workgroup i (histogram and scatter).  Workgroup i runs on
// XCD i mod 8; the workgroups of one XCD take one contiguous run of tiles, so
// that what consecutive tiles write for one digit (adjacent counts of the
// histogram, adjacent runs of the output) mostly meets in the L2 of one XCD,
// which merges their partial memory lines.
__device__ inline int rs_tile(int i, int nblk)
{
    const int q = i % XCDS;
    int s = 0;
    for (int p = 0; p < q; ++p) s += (nblk - p + XCDS - 1) / XCDS;  // tiles of XCD p (none when p >= nblk)
    return s + i / XCDS;
}

// per-tile bucket counts, hist[d * nblk + tile] for every bucket d < 2^nbits
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const int32_t *__restrict__ keys, int64_t N, int shift,
                                                        int nbits, int32_t *__restrict__ hist, int nblk)
{
    __shared__ int h[RS_BINS];
    const int tid = threadIdx.x;
    const int nb = 1 << nbits, mask = nb - 1;
    for (int q = 0; q < RS_BPT; ++q) h[q * RS_THREADS + tid] = 0;
    __syncthreads();
    const int tile = rs_tile((int)blockIdx.x, nblk);
    const int64_t base = (int64_t)tile * RS_TILE;
    // all keys of the thread loaded before the first count (an index past
    // the end reads the last key, not counted)
    int kv[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int64_t i = base + r * RS_THREADS + tid;
        kv[r] = keys[i < N ? i : N - 1];
    }
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r)
        if (base + r * RS_THREADS + tid < N) atomicAdd(&h[(kv[r] >> shift) & mask], 1);
    __syncthreads();
    for (int q = 0; q < RS_BPT; ++q) {
        const int d = q * RS_THREADS + tid;
        if (d < nb) hist[(int64_t)d * nblk + tile] = h[d];
    }
}

// Exclusive scan of a[0..n) in place.  A chunk of NT x 16 values goes
// through LDS: coalesced loads, each thread scans 16 consecutive values
// serially, the per-thread totals are scanned with wave shuffles and the
// wave totals, and the chunk is written back coalesced.  The LDS index is
// padded by one word in 32 so that the per-thread reads (stride 16 words)
// spread over the banks.  Short arrays take one workgroup that walks the
// chunks; longer ones are split into 4096-value blocks: block sums, a scan of
// those, then every block scans its values from its offset.
constexpr int SCAN_I = 16;
constexpr int SCAN_T = 1024;           // single-workgroup scan
constexpr int SCAN_BT = 256;           // per-block scan
constexpr int SCAN_B = SCAN_BT * SCAN_I;

__device__ inline int scan_pad(int i) { return i + (i >> 5); }

// scans a[base, base + m) (m <= NT * SCAN_I) adding `carry`; returns the
// chunk total.  buf holds NT * SCAN_I padded words, wsum NT / WAVE words.
template <int NT>
__device__ int scan_chunk(int32_t *__restrict__ a, int64_t base, int m, int carry, int *buf, int *wsum)
{
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int w = tid / WAVE;
    for (int r = 0; r < SCAN_I; ++r) {
        const int i = r * NT + tid;
        buf[scan_pad(i)] = i < m ? a[base + i] : 0;
    }
    lds_barrier();
    int v[SCAN_I];
    int tsum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_I; ++i) {
        v[i] = buf[scan_pad(tid * SCAN_I + i)];
        tsum += v[i];
    }
    int x = tsum;  // inclusive scan of the thread totals within the wave
#pragma unroll
    for (int off = 1; off < WAVE; off <<= 1) {
        const int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == WAVE - 1) wsum[w] = x;
    lds_barrier();
    int wpre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < NT / WAVE; ++q) {
        const int t = wsum[q];
        wpre += q < w ? t : 0;
        tot += t;
    }
    int run = carry + wpre + x - tsum;
#pragma unroll
    for (int i = 0; i < SCAN_I; ++i) {
        buf[scan_pad(tid * SCAN_I + i)] = run;
        run += v[i];
    }
    lds_barrier();
    for (int r = 0; r < SCAN_I; ++r) {
        const int i = r * NT + tid;
        if (i < m) a[base + i] = buf[scan_pad(i)];
    }
    lds_barrier();  // buf and wsum are rewritten by the next chunk
    return tot;
}

__global__ __launch_bounds__(SCAN_T) void k_scan_excl(int32_t *__restrict__ a, int64_t n)
{
    __shared__ int buf[SCAN_T * SCAN_I + SCAN_T * SCAN_I / 32];
    __shared__ int wsum[SCAN_T / WAVE];
    int carry = 0;
    for (int64_t base = 0; base < n; base += SCAN_T * SCAN_I) {
        const int64_t rem = n - base;
        const int m = rem < SCAN_T * SCAN_I ? (int)rem : SCAN_T * SCAN_I;
        carry += scan_chunk<SCAN_T>(a, base, m, carry, buf, wsum);
    }
}

// part[blk] = sum of block blk's values
__global__ __launch_bounds__(SCAN_BT) void k_scan_reduce(const int32_t *__restrict__ a, int64_t n,
                                                         int32_t *__restrict__ part)
{
    __shared__ int wsum[SCAN_BT / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B;
    int t = 0;
    for (int r = 0; r < SCAN_I; ++r) {
        const int64_t i = base + r * SCAN_BT + threadIdx.x;
        t += i < n ? a[i] : 0;
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if ((threadIdx.x & (WAVE - 1)) == 0) wsum[threadIdx.x / WAVE] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        int s = 0;
        for (int q = 0; q < SCAN_BT / WAVE; ++q) s += wsum[q];
        part[blockIdx.x] = s;
    }
}

// block blk scans its values from offset part[blk] (already scanned)
__global__ __launch_bounds__(SCAN_BT) void k_scan_apply(int32_t *__restrict__ a, int64_t n,
                                                        const int32_t *__restrict__ part)
{
    __shared__ int buf[SCAN_B + SCAN_B / 32];
    __shared__ int wsum[SCAN_BT / WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_B;
    const int64_t rem = n - base;
    const int m = rem < SCAN_B ? (int)rem : SCAN_B;
    scan_chunk<SCAN_BT>(a, base, m, part[blockIdx.x], buf, wsum);
}

// block blk scans its values from the sum of the block sums before it
// (part[b], b < blk, as k_scan_reduce wrote them): used up to SCAN_PRE_MAX
// blocks, where adding them in every block costs less than a launch
constexpr int64_t SCAN_PRE_MAX = 4096;
__global__ __launch_bounds__(SCAN_BT) void k_scan_apply_sum(int32_t *__restrict__ a, int64_t n,
                                                            const int32_t *__restrict__ part)
{
    __shared__ int buf[SCAN_B + SCAN_B / 32];
    __shared__ int wsum[SCAN_BT / WAVE];
    const int blk = (int)blockIdx.x;
    int t = 0;
    for (int b = threadIdx.x; b < blk; b += SCAN_BT) t += part[b];
    for (int off = WAVE / 2; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if ((threadIdx.x & (WAVE - 1)) == 0) wsum[threadIdx.x / WAVE] = t;
    lds_barrier();
    int pre = 0;
    for (int q = 0; q < SCAN_BT / WAVE; ++q) pre += wsum[q];
    lds_barrier();  // wsum is scan_chunk's scratch next
    const int64_t base = (int64_t)blk * SCAN_B;
    const int64_t rem = n - base;
    const int m = rem < SCAN_B ? (int)rem : SCAN_B;
    scan_chunk<SCAN_BT>(a, base, m, pre, buf, wsum);
}

// scratch ints that scan_excl needs for n values
inline int64_t scan_part_ints(int64_t n) { return (n + SCAN_B - 1) / SCAN_B + 1; }

// exclusive scan of a[0, n) on the stream; part holds scan_part_ints(n) ints
void scan_excl(int32_t *a, int64_t n, int32_t *part, hipStream_t s)
{
    if (n <= 0) return;
    if (n <= 4 * SCAN_B) {
        hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(SCAN_T), 0, s, a, n);
        return;
    }
    const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(SCAN_BT), 0, s, (const int32_t *)a, n, part);
    if (nb <= SCAN_PRE_MAX) {
        hipLaunchKernelGGL(k_scan_apply_sum, dim3((unsigned)nb), dim3(SCAN_BT), 0, s, a, n, (const int32_t *)part);
        return;
    }
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(SCAN_T), 0, s, part, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(SCAN_BT), 0, s, a, n, (const int32_t *)part);
}

// Stable scatter of one pass.  Each block ranks its elements within their
// bucket (wavefront match over the digit bits, then the wavefronts in order,
// then the rounds in order), places them in bucket order in LDS, and writes
// them out by consecutive threads, so that the elements of one bucket (about
// RS_TILE / RS_BINS of them) leave as one contiguous run instead of one
// store per element.  Every thread loads its RS_ITEMS keys and values before
// the first round.  wcnt[w][d] holds wavefront w's count of digit d in the
// current round and is zero otherwise: the lane that writes an entry clears
// it once the round's ranks are read.  run[d] counts the block's elements of
// digit d so far (the last wavefront holding d in a round advances it); its
// exclusive scan over the digits then gives each digit's first place in LDS.
static_assert(RS_BINS == 2 * RS_THREADS, "two digits per thread in the local scan");
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const int32_t *__restrict__ kin,
                                                           const int32_t *__restrict__ vin, int64_t N,
                                                           int shift, int nbits,
                                                           const int32_t *__restrict__ hist, int nblk,
                                                           int32_t *__restrict__ kout, int32_t *__restrict__ vout)
{
    constexpr int NWV = RS_THREADS / WAVE;
    __shared__ int base[RS_BINS];  // the block's first output of each digit
    __shared__ int run[RS_BINS];
    __shared__ int wcnt[NWV][RS_BINS];
    __shared__ int wtot[NWV];
    __shared__ int sk[RS_TILE], sv[RS_TILE];
    const int tid = threadIdx.x;
    const int lane = tid & (WAVE - 1);
    const int w = tid / WAVE;
    const int nb = 1 << nbits, mask = nb - 1;
    const int tile = rs_tile((int)blockIdx.x, nblk);
    const int64_t b0 = (int64_t)tile * RS_TILE;
    int kk[RS_ITEMS], vv[RS_ITEMS], lr[RS_ITEMS];
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const int64_t i = b0 + r * RS_THREADS + tid;
        kk[r] = i < N ? kin[i] : 0;
        vv[r] = i < N ? (vin ? vin[i] : (int)i) : 0;
        lr[r] = 0;
    }
    for (int q = 0; q < RS_BPT; ++q) {
        const int d = q * RS_THREADS + tid;
        base[d] = d < nb ? hist[(int64_t)d * nblk + tile] : 0;
        run[d] = 0;
        for (int u = 0; u < NWV; ++u) wcnt[u][d] = 0;
    }
    lds_barrier();
    const uint64_t below = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    // ranks within the block
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        const bool valid = b0 + r * RS_THREADS + tid < N;
        const int d = (kk[r] >> shift) & mask;
        uint64_t m = __ballot(valid);
        for (int bit = 0; bit < nbits; ++bit) {
            const bool on = (d >> bit) & 1;
            const uint64_t bb = __ballot(valid && on);
            m &= on ? bb : ~bb;
        }
        if (!valid) m = 0;
        const int rank = __popcll(m & below);
        const bool last = valid && ((m >> lane) == 1ull);
        const int cnt = __popcll(m);
        if (last) wcnt[w][d] = cnt;
        lds_barrier();
        int nrun = -1;  // new count of d, set by the last wavefront holding d
        if (valid) {
            int off = run[d];
            for (int q = 0; q < w; ++q) off += wcnt[q][d];
            lr[r] = off + rank;
            if (last) {
                bool final = true;
                for (int q = w + 1; q < NWV; ++q) final = final && wcnt[q][d] == 0;
                if (final) nrun = off + cnt;
            }
        }
        lds_barrier();
        if (last) {
            if (nrun >= 0) run[d] = nrun;
            wcnt[w][d] = 0;
        }
    }
    lds_barrier();
    // run[d] becomes the first LDS place of digit d (thread t owns 2t, 2t+1)
    {
        const int c0 = run[2 * tid], c1 = run[2 * tid + 1];
        int x = c0 + c1;
        for (int off = 1; off < WAVE; off <<= 1) {
            const int y = __shfl_up(x, off);
            if (lane >= off) x += y;
        }
        if (lane == WAVE - 1) wtot[w] = x;
        lds_barrier();
        int pre = 0;
        for (int q = 0; q < w; ++q) pre += wtot[q];
        const int ex = pre + x - (c0 + c1);
        run[2 * tid] = ex;
        run[2 * tid + 1] = ex + c0;
    }
    lds_barrier();
#pragma unroll
    for (int r = 0; r < RS_ITEMS; ++r) {
        if (b0 + r * RS_THREADS + tid < N) {
            const int lp = run[(kk[r] >> shift) & mask] + lr[r];
            sk[lp] = kk[r];
            sv[lp] = vv[r];
        }
    }
    lds_barrier();
    const int nvalid = N - b0 < RS_TILE ? (int)(N - b0) : RS_TILE;
    for (int q = tid; q < nvalid; q += RS_THREADS) {
        const int k = sk[q];
        const int d = (k >> shift) & mask;
        const int64_t o = (int64_t)base[d] + (q - run[d]);
        kout[o] = k;
        vout[o] = sv[q];
    }
}

// ---------------------------------------------------------------------------
// 3.-5. sorted coordinates, box_start, axis tables

// ys[ax][j] = wrapped x[perm[j]][ax]: a workgroup of nt threads takes GY * nt
// consecutive sorted points from j0, thread t the points j0 + u * nt + t
// (u < GY), so that every load of perm and every store of ys covers
// consecutive addresses across the lanes (whole memory lines); each thread
// issues all of its loads before its stores
constexpr int GY = 4;
__device__ inline void gather_ys_at(const double *__restrict__ x, const int32_t *__restrict__ perm, int64_t N,
                                    const BinGeom &g, double *__restrict__ ys, int64_t j0, int nt, int t)
{
    int64_t i[GY];
    double v[GY][3];
    // (indices past the end read the last point: no branch around a load,
    // so that all GY loads are in flight at once)
#pragma unroll
    for (int u = 0; u < GY; ++u) {
        const int64_t j = j0 + (int64_t)u * nt + t;
        i[u] = perm[j < N ? j : N - 1];
    }
#pragma unroll
    for (int u = 0; u < GY; ++u)
        for (int ax = 0; ax < 3; ++ax) v[u][ax] = x[3 * i[u] + ax];
#pragma unroll
    for (int u = 0; u < GY; ++u) {
        const int64_t j = j0 + (int64_t)u * nt + t;
        if (j < N)
            for (int ax = 0; ax < 3; ++ax) {
                double y = 0.0;
                wrap_coord(v[u][ax], ax, g, y);
                ys[(int64_t)ax * N + j] = y;
            }
    }
}

// box_start from the key changes of the sorted keys: sorted position j is
// the start of every box b with skey[j-1] < b <= skey[j] (skey[-1] = -1,
// skey[N] = nbox), so each b in [0, nbox] is written exactly once.  Used when
// there are at least as many points as boxes (short gaps); otherwise the
// binary search below.
__global__ void k_box_start_fill(const int32_t *__restrict__ skey, int64_t N, int64_t nbox,
                                 int32_t *__restrict__ bs)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > N) return;
    // both keys loaded together (indices clamped into [0, N); N >= 1 here)
    const int32_t sa = skey[j > 0 ? j - 1 : 0], sc = skey[j < N ? j : N - 1];
    const int64_t kp = j > 0 ? sa : -1;
    const int64_t kc = j < N ? sc : nbox;
    for (int64_t b = kp + 1; b <= kc; ++b) bs[b] = (int32_t)j;
}

__global__ void k_box_start(const int32_t *__restrict__ skey, int64_t N, int64_t nbox, int32_t *__restrict__ bs)
{
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nbox) return;
    // first sorted position with skey >= b
    int64_t lo = 0, hi = N;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (skey[mid] < b)
            lo = mid + 1;
        else
            hi = mid;
    }
    bs[b] = (int32_t)lo;
}

// row r of the table (axes stacked: rows [0,n0) axis 0, [n0,n0+n1) axis 1, rest axis 2),
// column c = offset + 1 for offsets -1, 0, +1.
__device__ inline void axis_table_entry(const BinGeom &g, int e, int32_t *__restrict__ nbr,
                                        int8_t *__restrict__ img)
{
    const int row = e / 3, c = e % 3;
    int ax = 0, b = row;
    if (b >= g.n[0]) {
        b -= g.n[0];
        ax = 1;
        if (b >= g.n[1]) {
            b -= g.n[1];
            ax = 2;
        }
    }
    const int n = g.n[ax];
    int nb = b + (c - 1);
    int s = 0;
    if (ax < g.D) {
        if (nb < 0) {
            nb += n;
            s = -1;
        } else if (nb >= n) {
            nb -= n;
            s = 1;
        }
    } else if (nb < 0 || nb >= n) {
        nb = -1;
    }
    nbr[e] = nb;
    img[e] = (int8_t)s;
}

// wrap + box id of point i (i < N), and entry e = i of the axis tables (e <
// 3 * (n0 + n1 + n2))
__global__ void k_bin_keys(const double *__restrict__ x, int64_t N, BinGeom g, int32_t *__restrict__ key,
                           int32_t *__restrict__ err, int32_t *__restrict__ nbr, int8_t *__restrict__ img)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 3 * (int64_t)(g.n[0] + g.n[1] + g.n[2])) axis_table_entry(g, (int)i, nbr, img);
    if (i >= N) return;
    const double xv[3] = {x[3 * i], x[3 * i + 1], x[3 * i + 2]};  // loaded together
    int b[3];
    bool ok = true;
    for (int ax = 0; ax < 3; ++ax) {
        double y = 0.0;
        ok = wrap_coord(xv[ax], ax, g, y) && ok;
        b[ax] = ok ? box_coord(y, ax, g) : 0;
    }
    if (!ok) atomicOr(err, 1);
    key[i] = ok ? (b[0] * g.n[1] + b[1]) * g.n[2] + b[2] : 0;
}

// ---------------------------------------------------------------------------
// 6. target tiles, one leaf column (b0, b1) at a time.
struct TileGeom {
    int n[3];
    int D;
    const int32_t *bs;
};

// neighbour index along axis ax of coordinate b at offset off in {-1, 0, 1}:
// wrapped on a periodic axis, -1 past the end of a free one (the same
// definition as the axis tables)
__device__ inline int nb_of(const TileGeom &g, int ax, int b, int off)
{
    const int n = g.n[ax];
    int nb = b + off;
    if (ax < g.D) {
        if (nb < 0) nb += n;
        if (nb >= n) nb -= n;
    } else if (nb < 0 || nb >= n) {
        nb = -1;
    }
    return nb;
}

__device__ inline int box_count(const TileGeom &g, int col, int zp)
{
    if (col < 0 || zp < 0) return 0;
    const int64_t b = (int64_t)col * g.n[2] + zp;
    return g.bs[b + 1] - g.bs[b];
}

// physical z of virtual z in [-1, n2], or -1 if it does not exist (free axis)
__device__ inline int phys_z(const TileGeom &g, int zv)
{
    if (zv >= 0 && zv < g.n[2]) return zv;
    if (zv == -1) return nb_of(g, 2, 0, -1);
    return nb_of(g, 2, g.n[2] - 1, 1);
}

__device__ inline int slab_count(const TileGeom &g, const int ccol[9], int zv)
{
    const int zp = phys_z(g, zv);
    if (zp < 0) return 0;
    int s = 0;
    for (int k = 0; k < 9; ++k) s += box_count(g, ccol[k], zp);
    return s;
}

// Cost of a tile = sum over its targets of the size of their stencil ranges.
// Tiles are ordered heavy-first by power-of-two cost class: class 0 holds the
// costs of bit length TK_CLASSES and more, class TK_CLASSES - 1 those of bit
// length 1.  A tile's cost is below 2^37 (at most 64 targets times a
// three-slab neighbourhood of fewer than 2^30 points), so no two bit lengths
// share a class.
constexpr int TK_CLASSES = 40;
static_assert(TILE_HEAVY_LOG >= 1 && TILE_HEAVY_LOG <= TK_CLASSES, "heavy tile threshold");
__device__ inline int tile_class(int64_t cost)
{
    const int len = 64 - __clzll((unsigned long long)(cost + 1));
    return TK_CLASSES - (len < TK_CLASSES ? len : TK_CLASSES);
}

// Final position of the tile of stable rank r in a class of B tiles at
// offset o.  Workgroup i of the pair kernels runs on XCD i mod 8; within the
// class the positions o + k with k mod 8 = q (one XCD) take the q-th
// contiguous run of the class's tiles, so every XCD works on a spatially
// compact share of every class (tiles that stage the same neighbour columns
// meet in one L2) and the heavy classes stay spread over all XCDs.  o, B
// and r come from the int32 count table, so 32-bit arithmetic holds them.
__device__ inline int64_t xcd_position(int o, int B, int r)
{
    int start = 0;
    int q = 0;
    for (; q < XCDS - 1; ++q) {
        const int len = q < B ? (B - q + XCDS - 1) / XCDS : 0;  // run of XCD q
        if (r < start + len) break;
        start += len;
    }
    return (int64_t)o + (int64_t)XCDS * (r - start) + q;
}

// One wavefront per leaf column (b0, b1).  The lanes first stage, for the
// column's z range, the first target and the target count of each box and
// the slab count (sources in the 9 stencil columns at that z) in LDS
// (dynamic: three ints per box, for the first TW_ZST boxes, and four per
// cost class); the column is then walked in z, each tile growing while its
// targets, its staged sources and its z extent fit.  Columns taller than
// TW_ZST boxes read the rest from the box starts.  A workgroup holds up to
// TW_WPB wavefronts, each walking a column of its own in an LDS region of its
// own (TW_WPB where the regions total at most TW_WPB_LDS bytes, else one):
// the walks use no workgroup barrier, and larger workgroups leave
// workgroup slots on the CUs for the coordinate gather that shares the
// counting walk's launch.
constexpr int TW_ZST = 2048;
constexpr int TW_WPB = 4;
constexpr int TW_WPB_LDS = 32768;
__host__ __device__ inline int tw_wave_ints(int n2)
{
    return 3 * (n2 < TW_ZST ? n2 : TW_ZST) + 2 + 4 * TK_CLASSES;
}

// The staged column.  sslp[zv + 1] is the slab count at virtual z zv: the
// staged boxes at 1 .. zst, and (columns of at most TW_ZST boxes) the slabs
// across the z faces at 0 and n2 + 1, so that those reads take no branch;
// taller columns (TALL) read what is not staged from the box starts.
template <bool TALL>
struct ColView {
    const TileGeom *g;
    const int *ccol;
    const int *snt;
    const int *sslp;
    const int *sbs;
    int col;
    __device__ int nt(int z) const
    {
        if (!TALL) return snt[z];
        return z < TW_ZST ? snt[z] : box_count(*g, col, z);
    }
    __device__ int first(int z) const
    {
        if (!TALL) return sbs[z];
        return z < TW_ZST ? sbs[z] : g->bs[(int64_t)col * g->n[2] + z];
    }
    // slab count at virtual z in [-1, n2]
    __device__ int sl(int zv) const
    {
        if (!TALL) return sslp[zv + 1];
        const int zp = phys_z(*g, zv);
        if (zp < 0) return 0;
        return zp < TW_ZST ? sslp[zp + 1] : slab_count(*g, ccol, zp);
    }
};

// lane total of the tile walk's cost: a DPP sum over the wavefront, read
// from lane 63
__device__ inline int tw_total(int v) { return __builtin_amdgcn_readlane(wave_incl_scan(v), WAVE - 1); }

// Counting pass (WRITE false): the column's tiles per cost class, into
// table[c * ncol + col] (class-major, so that the exclusive scan of the table
// gives every (class, column) its first rank in the stable heavy-first
// order); the last column also zeroes the sentinel table[TK_CLASSES * ncol],
// which the scan turns into the number of tiles.  Writing pass: each tile at
// its final position (xcd_position), the number of tiles in st[1] and the
// number of heavy tiles (cost + 1 of bit length above TILE_HEAVY_LOG) in st[2].
template <bool WRITE, bool TALL>
__device__ void tile_walk(const TileGeom &g, int col, int32_t *__restrict__ table, int4 *__restrict__ tiles,
                          int64_t cap, int32_t *__restrict__ st)
{
    extern __shared__ int tw_lds_all[];
    const int n2 = g.n[2];
    const int zst = n2 < TW_ZST ? n2 : TW_ZST;
    int *tw_lds = tw_lds_all + (threadIdx.x / WAVE) * tw_wave_ints(n2);
    int *snt = tw_lds, *sslp = tw_lds + zst, *sbs = tw_lds + 2 * zst + 2;
    int *run = tw_lds + 3 * zst + 2;    // tiles of each class so far in this column
    int *cbase = run + TK_CLASSES;      // rank of this column's first tile within each class
    int *cofs = cbase + TK_CLASSES;     // first position of each class
    int *clen = cofs + TK_CLASSES;      // tiles in each class
    const int64_t ncol = (int64_t)g.n[0] * g.n[1];
    const int lane = threadIdx.x & (WAVE - 1);
    const int b0 = col / g.n[1], b1 = col % g.n[1];
    int ccol[9];
    for (int k = 0; k < 9; ++k) {
        const int nb0 = nb_of(g, 0, b0, k / 3 - 1);
        const int nb1 = nb_of(g, 1, b1, k % 3 - 1);
        ccol[k] = (nb0 < 0 || nb1 < 0) ? -1 : nb0 * g.n[1] + nb1;
    }
    // the class offsets and this column's ranks (writing pass) are loaded
    // first, so that their latency overlaps the staging loads
    int tb0 = 0, tb1 = 0, tb2 = 0;
    if (WRITE && lane < TK_CLASSES) {
        tb0 = table[(int64_t)lane * ncol];
        tb1 = table[(int64_t)lane * ncol + col];
        tb2 = table[(int64_t)(lane + 1) * ncol];
    }
    // all ten box-start pairs of a lane are loaded before any is used (a
    // missing neighbour column, past a free face, reads column 0 and counts
    // nothing), so that they cost one memory round trip, not ten
    const int32_t *pcol[10];  // uniform: each column's box starts
#pragma unroll
    for (int k = 0; k < 10; ++k) pcol[k] = g.bs + (int64_t)(k == 9 ? col : (ccol[k] < 0 ? 0 : ccol[k])) * n2;
    for (int z = lane; z < zst; z += WAVE) {
        int lo[10], hi[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            lo[k] = pcol[k][z];
            hi[k] = pcol[k][z + 1];
        }
        int sc = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) sc += ccol[k] < 0 ? 0 : hi[k] - lo[k];
        snt[z] = hi[9] - lo[9];
        sbs[z] = lo[9];
        sslp[z + 1] = sc;
    }
    if (!TALL) {
        // the slabs across the z faces: wrapped (periodic z) or empty
        wave_fence();
        if (lane == 0) {
            const int lo = phys_z(g, -1), hi = phys_z(g, n2);
            sslp[0] = lo < 0 ? 0 : sslp[lo + 1];
            sslp[n2 + 1] = hi < 0 ? 0 : sslp[hi + 1];
        }
    }
    if (lane < TK_CLASSES) {
        run[lane] = 0;
        if (WRITE) {
            cbase[lane] = tb1 - tb0;
            cofs[lane] = tb0;
            clen[lane] = tb2 - tb0;
        }
    }
    wave_fence();
    // The wavefront's own LDS region: from here on, the staged boxes and the
    // counters are read by all lanes, and the counters updated by lane 0, in
    // program order (LDS operations of a wavefront complete in order;
    // wave_fence keeps the compiler from moving them).
    // final position of the next tile of class c (uniform c)
    auto place = [&](int c, int ahead) -> int64_t {
        return xcd_position(cofs[c], clen[c], cbase[c] + run[c] + ahead);
    };
    // The walk, with the whole wavefront on every step (z stays uniform).  A
    // tile starting at z may end at z + l for the l whose extent, targets and
    // staged sources all fit; each of these only grows with l, so the lanes
    // that fit form a prefix and one ballot gives the end.
    const ColView<TALL> cv{&g, ccol, snt, sslp, sbs, col};
    int z = 0;
    while (z < n2) {
        {  // next box with targets
            const int zz = z + lane;
            const uint64_t m = __ballot(zz < n2 && cv.nt(zz) > 0);
            if (m == 0) {
                z += WAVE;
                continue;
            }
            z += __ffsll((unsigned long long)m) - 1;
        }
        const int nt = cv.nt(z);
        const int q1 = cv.sl(z - 1) + cv.sl(z) + cv.sl(z + 1);
        const int first = cv.first(z);
        if (nt > TILE_T || q1 > TILE_CAP) {
            // dense: nd tiles of TILE_T targets, the last one of the rest;
            // all but possibly the last share one class
            const int nd = (nt + TILE_T - 1) / TILE_T;
            const int cf = tile_class((int64_t)TILE_T * q1);
            const int cl = tile_class((int64_t)(nt - (nd - 1) * TILE_T) * q1);
            const int nf = cl == cf ? nd : nd - 1;  // tiles of class cf
            if (WRITE) {
                for (int c = lane; c < nd; c += WAVE) {
                    const bool lastc = c == nd - 1 && cl != cf;
                    const int64_t pos = lastc ? place(cl, 0) : place(cf, c);
                    if (pos < cap)
                        tiles[pos] = make_int4(col, z, -(z + 1), first + c * TILE_T);
                }
            }
            wave_fence();
            if (lane == 0) {
                run[cf] += nf;
                if (cl != cf) run[cl] += 1;
            }
            wave_fence();
            ++z;
            continue;
        }
        // candidate end ze = z + lane: targets of boxes z..ze, sources of
        // slabs z-1..ze+1, by inclusive scans over the lanes
        const int ze = z + lane;
        const bool inr = ze < n2 && lane < TILE_ZMAX;
        const int ntl = inr ? cv.nt(ze) : 0;
        const int T = wave_incl_scan(ntl);
        const int Q = wave_incl_scan(inr ? cv.sl(ze + 1) : 0) + cv.sl(z - 1) + cv.sl(z);
        const int len = __popcll(__ballot(inr && T <= TILE_T && Q <= TILE_CAP));
        const int z1 = z + len - 1;
        // cost: sum over the tile's boxes of targets x the three slabs (at
        // most TILE_T targets, each with at most TILE_CAP sources: below 2^22)
        const int cost = tw_total(lane < len ? ntl * (cv.sl(ze - 1) + cv.sl(ze) + cv.sl(ze + 1)) : 0);
        const int c = tile_class((int64_t)cost);
        if (WRITE && lane == 0) {
            const int64_t pos = place(c, 0);
            if (pos < cap) tiles[pos] = make_int4(col, z, z1, first);
        }
        wave_fence();
        if (lane == 0) run[c] += 1;
        wave_fence();
        z = z1 + 1;
    }
    if (!WRITE) {
        if (lane < TK_CLASSES) table[(int64_t)lane * ncol + col] = run[lane];
        if (lane == 0 && col == ncol - 1) table[(int64_t)TK_CLASSES * ncol] = 0;
    } else if (lane == 0 && col == ncol - 1) {
        st[1] = table[(int64_t)TK_CLASSES * ncol];
        st[2] = table[(int64_t)(TK_CLASSES - TILE_HEAVY_LOG) * ncol];  // tiles of the classes before
    }
}

template <bool WRITE, bool TALL>
__global__ __launch_bounds__(TW_WPB *WAVE) void k_tiles(TileGeom g, int64_t col0, int32_t *__restrict__ table,
                                                         int4 *__restrict__ tiles, int64_t cap,
                                                         int32_t *__restrict__ st)
{
    const int64_t col = col0 + (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    if (col >= (int64_t)g.n[0] * g.n[1]) return;  // whole wavefronts
    tile_walk<WRITE, TALL>(g, (int)col, table, tiles, cap, st);
}

// The counting walk (blocks below nwb, one column per wavefront) and the
// sorted coordinates (the blocks after them, GY points per thread) in one launch:
// both wait mostly on memory and do not depend on each other, so their
// wavefronts overlap on the device.
template <bool TALL>
__global__ __launch_bounds__(TW_WPB *WAVE) void k_ys_count(TileGeom tg, unsigned nwb, int32_t *__restrict__ table,
                                                            int64_t cap, int32_t *__restrict__ st,
                                                            const double *__restrict__ x,
                                                            const int32_t *__restrict__ perm, int64_t N, BinGeom g,
                                                            double *__restrict__ ys)
{
    if (blockIdx.x < nwb) {
        const int64_t col = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
        if (col < (int64_t)tg.n[0] * tg.n[1]) tile_walk<false, TALL>(tg, (int)col, table, nullptr, cap, st);
        return;
    }
    gather_ys_at(x, perm, N, g, ys, (int64_t)(blockIdx.x - nwb) * blockDim.x * GY, (int)blockDim.x, (int)threadIdx.x);
}

}  // namespace dmk

using namespace dmk;

// ---------------------------------------------------------------------------
// host side
namespace {

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int check_grid(const dmk_grid *g)
{
    if (!g) return DMK_EINVAL;
    if (g->D < 0 || g->D > 3) return DMK_EINVAL;
    for (int i = 0; i < 3; ++i) {
        if (g->n[i] < 1) return DMK_EINVAL;
        if (!(g->L[i] > 0.0) || !isfinite(g->L[i])) return DMK_EINVAL;
    }
    const int64_t nbox = (int64_t)g->n[0] * g->n[1] * g->n[2];
    if (nbox > (int64_t)0x3fffffff) return DMK_ESIZE;
    return DMK_OK;
}

struct Layout {
    size_t key, perm, skey, bs, ys, nbr, img, tiles, status, tmp, total;
    int64_t max_tiles, tmp_ints;
};

Layout layout_for(const dmk_grid *g, int64_t N)
{
    Layout l{};
    const int64_t nbox = (int64_t)g->n[0] * g->n[1] * g->n[2];
    const int64_t rows = (int64_t)g->n[0] + g->n[1] + g->n[2];
    const int64_t ncol = (int64_t)g->n[0] * g->n[1];
    const int64_t nblk = (N + RS_TILE - 1) / RS_TILE;
    l.max_tiles = max_tiles_for(N, nbox);
    const int64_t nh = (int64_t)RS_BINS * (nblk > 0 ? nblk : 1);
    const int64_t phase1 = 2 * N + nh + scan_part_ints(nh) + 64;
    const int64_t ntab = (int64_t)TK_CLASSES * ncol;  // tile count table, then its scan's partials
    const int64_t phase2 = ((ntab + 1 + 63) & ~(int64_t)63) + scan_part_ints(ntab + 1) + 64;
    l.tmp_ints = phase1 > phase2 ? phase1 : phase2;
    size_t off = 0;
    l.key = off;
    off = align256(off + sizeof(int32_t) * N);
    l.perm = off;
    off = align256(off + sizeof(int32_t) * N);
    l.skey = off;
    off = align256(off + sizeof(int32_t) * N);
    l.bs = off;
    off = align256(off + sizeof(int32_t) * (nbox + 1));
    l.ys = off;
    off = align256(off + sizeof(double) * 3 * N);
    l.nbr = off;
    off = align256(off + sizeof(int32_t) * 3 * rows);
    l.img = off;
    off = align256(off + sizeof(int8_t) * 3 * rows);
    l.tiles = off;
    off = align256(off + sizeof(int32_t) * 4 * l.max_tiles);
    l.status = off;
    off = align256(off + sizeof(int32_t) * 64);
    l.tmp = off;
    off = align256(off + sizeof(int32_t) * l.tmp_ints);
    l.total = off;
    return l;
}

BinGeom make_geom(const dmk_grid *g)
{
    BinGeom b{};
    for (int i = 0; i < 3; ++i) {
        b.L[i] = g->L[i];
        b.inv[i] = (double)g->n[i] / g->L[i];
        b.n[i] = g->n[i];
    }
    b.D = g->D;
    return b;
}

inline unsigned nblocks(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

extern "C" size_t dmk_bins_bytes(const dmk_grid *grid, int64_t N)
{
    if (check_grid(grid) != DMK_OK || N < 0 || N > (int64_t)0x3fffffff) return 0;
    return layout_for(grid, N).total;
}

extern "C" int dmk_bins_carve(const dmk_grid *grid, int64_t N, void *arena, size_t bytes, dmk_bins *bins)
{
    int rc = check_grid(grid);
    if (rc != DMK_OK) return rc;
    if (!bins || N < 0) return DMK_EINVAL;
    if (N > (int64_t)0x3fffffff) return DMK_ESIZE;
    if (!arena || ((uintptr_t)arena & 255)) return DMK_EINVAL;
    Layout l = layout_for(grid, N);
    if (bytes < l.total) return DMK_ESIZE;
    char *a = (char *)arena;
    memset(bins, 0, sizeof(*bins));
    bins->N = N;
    bins->nbox = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    bins->ntiles = 0;
    bins->max_tiles = l.max_tiles;
    bins->key = (int32_t *)(a + l.key);
    bins->perm = (int32_t *)(a + l.perm);
    bins->skey = (int32_t *)(a + l.skey);
    bins->box_start = (int32_t *)(a + l.bs);
    bins->ys = (double *)(a + l.ys);
    bins->axis_nbr = (int32_t *)(a + l.nbr);
    bins->axis_img = (int8_t *)(a + l.img);
    bins->tiles = (int32_t *)(a + l.tiles);
    bins->status = (int32_t *)(a + l.status);
    bins->tmp = (int32_t *)(a + l.tmp);
    bins->tmp_ints = l.tmp_ints;
    return DMK_OK;
}

// The tile walks and the coordinate gather: the counting walk beside the
// gather, the scan of the count table, the writing walk (columns of more than
// TW_ZST boxes: TALL)
template <bool TALL>
void walks(const TileGeom &tg, int wpb, int64_t bt, int64_t maxb, int64_t nwb, int64_t nyb,
           size_t tw_lds, int32_t *table, int32_t *tpart, int64_t ntab, dmk_bins *bins, const double *x, int64_t N,
           const BinGeom &g, hipStream_t stream)
{
    if (nwb + nyb <= maxb) {
        hipLaunchKernelGGL(k_ys_count<TALL>, dim3((unsigned)(nwb + nyb)), dim3((unsigned)bt), tw_lds, stream, tg,
                           (unsigned)nwb, table, bins->max_tiles, bins->status, x, (const int32_t *)bins->perm, N, g,
                           bins->ys);
    } else {
        for (int64_t b0 = 0; b0 < nwb; b0 += maxb)
            hipLaunchKernelGGL((k_tiles<false, TALL>), dim3((unsigned)std::min(maxb, nwb - b0)), dim3((unsigned)bt),
                               tw_lds, stream, tg, b0 * wpb, table, (int4 *)bins->tiles, bins->max_tiles,
                               bins->status);
        // (N < 2^30 points: one launch of fewer than 2^28 threads)
        if (nyb > 0)
            hipLaunchKernelGGL(k_ys_count<TALL>, dim3((unsigned)nyb), dim3((unsigned)bt), 0, stream, tg, 0u, table,
                               bins->max_tiles, bins->status, x, (const int32_t *)bins->perm, N, g, bins->ys);
    }
    // first rank of every (class, column) in the heavy-first order, and the
    // number of tiles in the sentinel; then every tile at its place
    scan_excl(table, ntab + 1, tpart, stream);
    for (int64_t b0 = 0; b0 < nwb; b0 += maxb)
        hipLaunchKernelGGL((k_tiles<true, TALL>), dim3((unsigned)std::min(maxb, nwb - b0)), dim3((unsigned)bt),
                           tw_lds, stream, tg, b0 * wpb, table, (int4 *)bins->tiles, bins->max_tiles, bins->status);
}

extern "C" int dmk_tree_bin(const dmk_grid *grid, const double *x, dmk_bins *bins, hipStream_t stream)
{
    int rc = check_grid(grid);
    if (rc != DMK_OK) return rc;
    if (!bins || !bins->key || !bins->status || !bins->tmp) return DMK_EINVAL;
    const int64_t N = bins->N;
    const int64_t nbox = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
    if (bins->nbox != nbox) return DMK_EINVAL;
    if (N > 0 && !x) return DMK_EINVAL;
    Layout l = layout_for(grid, N);
    if (bins->tmp_ints < l.tmp_ints || bins->max_tiles < l.max_tiles) return DMK_ESIZE;

    const BinGeom g = make_geom(grid);
    const int64_t nblk = (N + RS_TILE - 1) / RS_TILE;
    const int64_t ncol = (int64_t)grid->n[0] * grid->n[1];
    int32_t *altk = bins->tmp;
    int32_t *altv = bins->tmp + N;
    int32_t *hist = bins->tmp + 2 * N;

    DMK_HIP_CHECK(hipMemsetAsync(bins->status, 0, sizeof(int32_t) * 4, stream));
    // box ids, and the axis tables
    const int rows = grid->n[0] + grid->n[1] + grid->n[2];
    hipLaunchKernelGGL(k_bin_keys, dim3(nblocks(std::max(N, (int64_t)3 * rows), 256)), dim3(256), 0, stream, x, N, g,
                       bins->key, bins->status, bins->axis_nbr, bins->axis_img);
    if (N > 0) {
        // radix passes over ceil(log2(nbox)) bits, digits of at most 9 bits
        int bits = 0;
        while (bits < 31 && ((int64_t)1 << bits) < nbox) ++bits;
        const int passes = bits > 0 ? (bits + RS_MAXBITS - 1) / RS_MAXBITS : 1;
        const int width = bits > 0 ? (bits + passes - 1) / passes : 1;
        const int32_t *kin = bins->key;
        const int32_t *vin = nullptr;
        for (int p = 0; p < passes; ++p) {
            const bool to_final = ((passes - 1 - p) % 2) == 0;
            int32_t *kout = to_final ? bins->skey : altk;
            int32_t *vout = to_final ? bins->perm : altv;
            const int64_t nh = ((int64_t)1 << width) * nblk;
            hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblk), dim3(RS_THREADS), 0, stream, kin, N, width * p,
                               width, hist, (int)nblk);
            scan_excl(hist, nh, hist + nh, stream);
            hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblk), dim3(RS_THREADS), 0, stream, kin, vin, N,
                               width * p, width, (const int32_t *)hist, (int)nblk, kout, vout);
            kin = kout;
            vin = vout;
        }
    }
    if (N >= nbox)
        hipLaunchKernelGGL(k_box_start_fill, dim3(nblocks(N + 1, 256)), dim3(256), 0, stream, bins->skey, N, nbox,
                           bins->box_start);
    else
        hipLaunchKernelGGL(k_box_start, dim3(nblocks(nbox + 1, 256)), dim3(256), 0, stream, bins->skey, N, nbox,
                           bins->box_start);
    TileGeom tg{};
    for (int i = 0; i < 3; ++i) tg.n[i] = grid->n[i];
    tg.D = grid->D;
    tg.bs = bins->box_start;
    // tile scratch (the point sort is done with tmp by now): the class x
    // column count table with its sentinel, then the scan's partial sums
    const int64_t ntab = (int64_t)TK_CLASSES * ncol;
    int32_t *table = bins->tmp;
    int32_t *tpart = bins->tmp + ((ntab + 1 + 63) & ~(int64_t)63);
    // one wavefront per column, wpb columns per workgroup, in launches of
    // fewer than 2^32 work-items; LDS per wavefront: first target, target
    // count and slab count of each staged box, and four ints per cost class
    const size_t tw_wave = sizeof(int) * (size_t)tw_wave_ints(grid->n[2]);
    const int wpb = tw_wave * TW_WPB <= (size_t)TW_WPB_LDS ? TW_WPB : 1;
    const size_t tw_lds = tw_wave * wpb;
    const int64_t bt = (int64_t)wpb * WAVE;          // threads per workgroup
    const int64_t maxb = 0xffffffffu / bt;           // workgroups per launch
    const int64_t nwb = (ncol + wpb - 1) / wpb;      // workgroups of the walks
    // the counting walk and the sorted coordinates in one launch (the walk's
    // workgroups first, then workgroups of bt threads taking GY points each)
    const int64_t nyb = N > 0 ? ((N + GY - 1) / GY + bt - 1) / bt : 0;
    if (grid->n[2] > TW_ZST)
        walks<true>(tg, wpb, bt, maxb, nwb, nyb, tw_lds, table, tpart, ntab, bins, x, N, g, stream);
    else
        walks<false>(tg, wpb, bt, maxb, nwb, nyb, tw_lds, table, tpart, ntab, bins, x, N, g, stream);
    DMK_HIP_CHECK(hipGetLastError());
    int32_t st[4] = {0, 0, 0, 0};
    DMK_HIP_CHECK(hipMemcpyAsync(st, bins->status, sizeof(st), hipMemcpyDeviceToHost, stream));
    DMK_HIP_CHECK(hipStreamSynchronize(stream));
    if (st[0] != 0) return DMK_EDOMAIN;
    if (st[1] < 0 || st[1] > bins->max_tiles) return DMK_ESIZE;
    if (st[2] < 0 || st[2] > st[1]) return DMK_EHIP;
    bins->ntiles = st[1];
    bins->nheavy = st[2];
    return DMK_OK;
}

extern "C" const char *dmk_strerror(int s)
{
    switch (s) {
    case DMK_OK: return "ok";
    case DMK_EINVAL: return "invalid argument";
    case DMK_EDOMAIN: return "coordinate not finite or outside [0,L) along a free axis";
    case DMK_ECUTOFF: return "cutoff must satisfy 0 < rc <= min_i L_i/n_i and sigma > 0";
    case DMK_EUNSUPPORTED: return "unsupported kernel / precision combination";
    case DMK_EHIP: return "HIP runtime error";
    case DMK_ESIZE: return "arena or workspace too small, or size limit exceeded";
    default: return "unknown status";
    }
}

extern "C" const char *dmk_version(void) { return "libdmkloc 0.1 (gfx950)"; }
