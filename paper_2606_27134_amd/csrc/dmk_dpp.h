// dmk_dpp.h -- cross-lane sums of one wavefront with DPP moves (GFX9
// data-parallel primitives) for the libdmkloc kernels (gfx950).  Not part of
// the public ABI.
#pragma once

#include <hip/hip_runtime.h>

namespace dmk {

// DPP_* are dpp_ctrl codes.  With bound_ctrl set, a lane whose source lane
// lies outside its row (or the wavefront) reads 0; a lane of a row masked
// out by row_mask is not written and keeps the `old` operand.
constexpr int DPP_ROW_SHL = 0x100, DPP_ROW_SHR = 0x110;  // + shift 1..15
constexpr int DPP_WAVE_SHL1 = 0x130, DPP_ROW_BCAST15 = 0x142, DPP_ROW_BCAST31 = 0x143;

template <int CTRL, int RM>
__device__ inline int dpp_int(int x, int old)
{
    return __builtin_amdgcn_update_dpp(old, x, CTRL, RM, 0xf, true);
}
template <int CTRL, int RM>
__device__ inline float dpp_val(float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, RM, 0xf, true));
}
template <int CTRL, int RM>
__device__ inline double dpp_val(double x)
{
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, RM, 0xf, true);
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, RM, 0xf, true);
    return __hiloint2double(hi, lo);
}

// the same move where lanes that are not written may hold any value
template <int CTRL, int RM>
__device__ inline float dpp_any(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, RM, 0xf, true));
}
template <int CTRL, int RM>
__device__ inline double dpp_any(double x)
{
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, RM, 0xf, true);
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, RM, 0xf, true);
    return __hiloint2double(hi, lo);
}

// inclusive prefix sum over the 64 lanes (shifts within rows, then carries
// into the following rows)
__device__ inline int wave_incl_scan(int v)
{
    v += dpp_int<DPP_ROW_SHR + 1, 0xf>(v, 0);
    v += dpp_int<DPP_ROW_SHR + 2, 0xf>(v, 0);
    v += dpp_int<DPP_ROW_SHR + 4, 0xf>(v, 0);
    v += dpp_int<DPP_ROW_SHR + 8, 0xf>(v, 0);
    v += dpp_int<DPP_ROW_BCAST15, 0xa>(v, 0);
    v += dpp_int<DPP_ROW_BCAST31, 0xc>(v, 0);
    return v;
}

// plain wavefront sum by the same pattern; lane 63 holds the total
template <int NC, typename T>
__device__ inline void wave_sum(T *v)
{
    for (int c = 0; c < NC; ++c) {
        T x = v[c];
        x += dpp_val<DPP_ROW_SHR + 1, 0xf>(x);
        x += dpp_val<DPP_ROW_SHR + 2, 0xf>(x);
        x += dpp_val<DPP_ROW_SHR + 4, 0xf>(x);
        x += dpp_val<DPP_ROW_SHR + 8, 0xf>(x);
        x += dpp_val<DPP_ROW_BCAST15, 0xa>(x);
        x += dpp_val<DPP_ROW_BCAST31, 0xc>(x);
        v[c] = x;
    }
}

}  // namespace dmk
