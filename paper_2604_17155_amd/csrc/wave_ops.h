// Wavefront helpers shared by the tile kernels (wave64, gfx950).
#pragma once

#include "gsc_internal.h"

namespace gsc {

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// Sum over the 64 lanes; the result is uniform.  All lanes must be active.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_mov<0x141>(v);  // row_half_mirror
    v += dpp_mov<0x140>(v);  // row_mirror: every lane holds its row's sum
    float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16));
    float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 48));
    return (r0 + r1) + (r2 + r3);
}

// Sums four per-lane values over the wave at once.  Quad exchanges split the
// four values between lanes (lane bit 0 picks the pair, bit 1 the member),
// rotations sum the four quads of a row, and two shuffles sum the rows.
// On return lane L < 4 holds the total of value 2*(L&1) + (L>>1).
__device__ __forceinline__ float wave_sum4_transposed(float v0, float v1, float v2, float v3,
                                                      uint32_t lane) {
    const bool b0 = lane & 1u, b1 = lane & 2u;
    const float x0 = (b0 ? v2 : v0) + dpp_mov<0xB1>(b0 ? v0 : v2);
    const float x1 = (b0 ? v3 : v1) + dpp_mov<0xB1>(b0 ? v1 : v3);
    float y = (b1 ? x1 : x0) + dpp_mov<0x4E>(b1 ? x0 : x1);
    y += dpp_mov<0x124>(y);  // row_ror:4
    y += dpp_mov<0x128>(y);  // row_ror:8
    y += __shfl_xor(y, 16, 64);
    y += __shfl_xor(y, 32, 64);
    return y;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

__device__ __forceinline__ float bcast(float v, uint32_t lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)lane));
}
__device__ __forceinline__ uint32_t bcast_u(uint32_t v, uint32_t lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)lane);
}

__device__ __forceinline__ int find_view(const ViewInfo* __restrict__ views, int n_views, uint32_t tile) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_base <= tile) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <bool BF16>
__device__ __forceinline__ float load_target(const void* __restrict__ t, int64_t idx) {
    if constexpr (BF16) {
        uint32_t b = ((const uint16_t*)t)[idx];
        return __uint_as_float(b << 16);
    } else {
        return ((const float*)t)[idx];
    }
}


}  // namespace gsc
