// dmk_internal.h -- constants and helpers shared by the binning and residual
// translation units of libdmkloc (gfx950).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dmk.h"

namespace dmk {

// A target tile is worked on by one wavefront (64 lanes): at most TILE_T
// targets, all in one leaf column (b0, b1) and in consecutive z-boxes
// [z0, z1].  A multi-box tile stages at most TILE_CAP neighbour sources in
// LDS at once; a box whose targets or neighbourhood exceed that becomes
// "dense" tiles of up to TILE_T targets that stream their neighbourhood
// through LDS in chunks of TILE_CAP sources.
#ifndef DMK_TILE_CAP
#define DMK_TILE_CAP 512
#endif
#ifndef DMK_WAVES_PER_TILE
#define DMK_WAVES_PER_TILE 4
#endif
#ifndef DMK_TILE_T
#define DMK_TILE_T 64
#endif
constexpr int WAVE = 64;
constexpr int XCDS = 8;  // accelerator complex dies: workgroup i runs on XCD i mod 8
constexpr int TILE_T = DMK_TILE_T;
constexpr int TILE_CAP = DMK_TILE_CAP;
constexpr int TILE_NW = DMK_WAVES_PER_TILE;  // wavefronts per tile workgroup
// Tiles of cost (targets times the sources of their stencil ranges, summed
// over the tile's boxes) 2^TILE_HEAVY_LOG - 1 or more are "heavy": they come
// first in the tile order, and the pair kernels give them HEAVY_NW
// wavefronts per workgroup where a workgroup of that size fits in LDS
#ifndef DMK_TILE_HEAVY_LOG
#define DMK_TILE_HEAVY_LOG 16
#endif
#ifndef DMK_WAVES_PER_HEAVY_TILE
#define DMK_WAVES_PER_HEAVY_TILE 8
#endif
constexpr int TILE_HEAVY_LOG = DMK_TILE_HEAVY_LOG;
constexpr int HEAVY_NW = DMK_WAVES_PER_HEAVY_TILE;
#ifndef DMK_TILE_ZMAX
#define DMK_TILE_ZMAX 46
#endif
constexpr int TILE_ZMAX = DMK_TILE_ZMAX;  // z-boxes per multi-box tile (<= 64 slabs)

// tiles[t] = {col, z0, z1 or -(z+1) for a dense tile, first target}
struct TileDesc {
    int col, z0, z1, tstart;
};

inline int64_t max_tiles_for(int64_t N, int64_t nbox)
{
    int64_t m = N < nbox ? N : nbox;
    return 2 * m + N / TILE_T + 2;
}

#define DMK_HIP_CHECK(call)                         \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return DMK_EHIP;      \
    } while (0)

}  // namespace dmk
