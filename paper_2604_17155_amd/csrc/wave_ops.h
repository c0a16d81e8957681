// Wavefront helpers shared by the tile kernels (wave64, gfx950).
#pragma once

#include "gsc_internal.h"

namespace gsc {

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}

// DPP controls (GFX9 encoding).
constexpr int kQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]
constexpr int kRowShl4 = 0x104;   // lane L <- L + 4 within its row of 16
constexpr int kRowShr4 = 0x114;   // lane L <- L - 4 within its row
constexpr int kRowRor4 = 0x124;
constexpr int kRowRor8 = 0x128;   // lane L <- L xor 8 within its row

// x + (x from the lane 16 apart within each half-wave) and likewise 32 apart,
// with the gfx950 lane-swap instructions (no LDS round trip).
__device__ __forceinline__ float sum_xor16(float x) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float sum_xor32(float x) {
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Sum over the 64 lanes; the result is uniform.  All lanes must be active.
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_mov<kQuadXor1>(v);
    v += dpp_mov<kQuadXor2>(v);
    v += dpp_mov<kRowRor4>(v);
    v += dpp_mov<kRowRor8>(v);  // every lane holds its row's sum
    v = sum_xor32(sum_xor16(v));
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Value of the partner at lane distance 2^S (every lane takes part in each
// exchange: a lane-permuting read inside a divergent branch would see its
// disabled partners as 0).
template <int S>
__device__ __forceinline__ float partner(float send, bool hi) {
    if constexpr (S == 0) {
        return dpp_mov<kQuadXor1>(send);
    } else if constexpr (S == 1) {
        return dpp_mov<kQuadXor2>(send);
    } else if constexpr (S == 2) {
        const float from_above = dpp_mov<kRowShl4>(send);  // lane L + 4
        const float from_below = dpp_mov<kRowShr4>(send);  // lane L - 4
        return hi ? from_below : from_above;
    } else {
        return dpp_mov<kRowRor8>(send);
    }
}

// One halving step at lane distance 2^S over 2H values (indices fixed at
// compile time, so the values stay in registers).
template <int H, int S>
__device__ __forceinline__ void halve(float* a, uint32_t lane) {
    const bool hi = (lane >> S) & 1u;
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const float keep = hi ? a[i + H] : a[i];
        const float send = hi ? a[i] : a[i + H];
        a[i] = keep + partner<S>(send, hi);
    }
}

// Sums NV per-lane values (NV = 4, 8 or 16) over the wave at once.  Each
// exchange step at lane distance d = 1, 2, 4, 8 halves the values a lane
// holds: the lane with bit d clear keeps the lower half and adds its
// partner's lower half, the other keeps the upper half.  Once one value is
// left, the remaining lane bits are summed without halving.  On return lane
// L < NV holds the total of value bitrev(L) = sum_s bit_s(L) NV / 2^(s+1)
// (e.g. NV = 4: 2*(L&1) + (L>>1)&1).  All lanes must be active.
template <int NV>
__device__ __forceinline__ float wave_sum_transposed(const float (&v)[NV], uint32_t lane) {
    static_assert(NV == 4 || NV == 8 || NV == 16, "NV must be 4, 8 or 16");
    float a[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) a[i] = v[i];
    halve<NV / 2, 0>(a, lane);
    halve<NV / 4, 1>(a, lane);
    if constexpr (NV >= 8) halve<NV / 8, 2>(a, lane);
    if constexpr (NV >= 16) halve<1, 3>(a, lane);
    float y = a[0];
    if constexpr (NV == 4) {
        y += dpp_mov<kRowRor4>(y);
        y += dpp_mov<kRowRor8>(y);
    } else if constexpr (NV == 8) {
        y += dpp_mov<kRowRor8>(y);
    }
    return sum_xor32(sum_xor16(y));
}

// Value index held by lane L < NV after wave_sum_transposed<NV>.
template <int NV>
__device__ __forceinline__ int transposed_index(uint32_t lane) {
    int idx = 0, w = NV / 2;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        if (w == 0) break;
        idx += ((lane >> s) & 1u) ? w : 0;
        w /= 2;
    }
    return idx;
}

// Four values at once (NV = 4); lane L < 4 holds value 2*(L&1) + ((L>>1)&1).
__device__ __forceinline__ float wave_sum4_transposed(float v0, float v1, float v2, float v3,
                                                      uint32_t lane) {
    const float v[4] = {v0, v1, v2, v3};
    return wave_sum_transposed<4>(v, lane);
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

// The 16x16 tile a wave works on.  A launch over bins of BIN pixels runs
// (BIN / 16)^2 waves per bin; wave tile vt is tile `quad` (bit 0: column
// half, bit 1: row half) of bin vt / (BIN / 16)^2.
struct TileGeom {
    uint32_t bin;   // global bin id within the batch
    uint32_t quad;  // tile within the bin (0 for 16-pixel bins)
    int vloc;       // view of the bin within the batch table
    int x0, y0;     // pixel origin of the tile
};

template <int BIN>
__device__ __forceinline__ TileGeom tile_geom(uint32_t vt, const ViewInfo* __restrict__ views,
                                              int n_views) {
    TileGeom t;
    vt = (uint32_t)__builtin_amdgcn_readfirstlane((int)vt);  // wave-uniform
    t.bin = BIN == 32 ? vt >> 2 : vt;
    t.quad = BIN == 32 ? (vt & 3u) : 0u;
    t.vloc = __builtin_amdgcn_readfirstlane(find_view(views, n_views, t.bin));
    const ViewInfo& V = views[t.vloc];
    const uint32_t local = t.bin - V.tile_base;
    const int bx = (int)(local % (uint32_t)V.tiles_x), by = (int)(local / (uint32_t)V.tiles_x);
    t.x0 = bx * BIN + (int)(t.quad & 1u) * kTile;
    t.y0 = by * BIN + (int)(t.quad >> 1) * kTile;
    return t;
}

// Logical block of a grid block.  The dispatcher deals a grid's blocks to
// the 8 XCDs in turn (block b runs on XCD b % 8), and each XCD has an L2 of
// its own.  The grid is cut into groups of 8 kXcdRun blocks; within a group,
// XCD x takes the logical blocks x kXcdRun .. x kXcdRun + kXcdRun - 1, so
// that consecutive logical blocks (neighbouring tiles of the launch order,
// which read the same Gaussian records, and the quadrant waves of one
// 32-pixel bin) share an L2, while the groups still start in order.  Blocks
// of a last, incomplete group keep their index.  A bijection on [0, G).
constexpr uint32_t kXcds = 8, kXcdRun = 32;
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) {
    constexpr uint32_t group = kXcds * kXcdRun;
    if (b >= G - G % group) return b;
    const uint32_t x = b % kXcds, r = b / kXcds;
    return (r / kXcdRun) * group + x * kXcdRun + r % kXcdRun;
}

// The wave tile taken t-th from a persistent launch's queue.  With `order`
// (bins by decreasing octave of list length) the longest lists start first,
// so that no long tile is left to run alone at the end of the launch.
template <int BIN>
__device__ __forceinline__ uint32_t queued_tile(uint32_t t, const uint32_t* __restrict__ order) {
    if (order == nullptr) return t;
    if constexpr (BIN == 32) return order[t >> 2] * 4u + (t & 3u);
    else return order[t];
}

// Bands (rows y0 + 4k .. y0 + 4k + 3 of the tile) a list entry can reach:
// the pair's band mask for 16-pixel bins; for 32-pixel bins, none unless the
// pair marks this tile, else the bands met by the footprint's rows
// [ext & 0xFFFF, ext >> 16].
template <int BIN>
__device__ __forceinline__ uint32_t entry_bands(uint32_t pc, uint32_t quad, uint32_t ext, int y0) {
    const uint32_t m = pc >> kItemBits;
    if constexpr (BIN == 16) {
        return m;
    } else {
        if (!((m >> quad) & 1u)) return 0u;
        const int ylo = (int)(ext & 0xFFFFu), yhi = (int)(ext >> 16);
        uint32_t b = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) b |= (ylo <= y0 + 4 * k + 3 && yhi >= y0 + 4 * k) ? (1u << k) : 0u;
        return b;
    }
}

// Whether a list entry can reach a live band of this tile judging by its
// pair value alone: for 16-pixel bins the pair's band bits; for 32-pixel
// bins only whether the pair marks this tile (its rows come with the record).
template <int BIN>
__device__ __forceinline__ bool pair_reaches(uint32_t pc, uint32_t quad, uint32_t alive) {
    const uint32_t m = pc >> kItemBits;
    if constexpr (BIN == 16) return (m & alive) != 0u;
    else return ((m >> quad) & 1u) != 0u;
}

// Pixel offsets d = pixel centre - projected centre within a 16x16 tile are
// formed against the tile's centre point x0 + 8 (between its two middle pixel
// columns): an entry's offset of that point, (x0 + 8 - u_hi) - u_lo, is
// formed once and broadcast, and a lane adds its pixel's offset from the
// point, column - 7.5 (exact).  Every binary32 step then rounds a quantity of
// at most |d| + 7.5 pixels, so |error of d| <= u (3 |d| + 15) per axis.  The
// blend, render and adjoint kernels all form d this way, so they take the
// same pixel decisions.
__device__ __forceinline__ float tile_centre(int x0) { return (float)x0 + 8.0f; }
__device__ __forceinline__ float tile_offset_col(uint32_t lane) { return (float)(lane & 15) - 7.5f; }
__device__ __forceinline__ float tile_offset_row(uint32_t lane, int k) {
    return (float)((lane >> 4) + 4 * k) - 7.5f;
}

// A wave-uniform loop constant held in a vector register: the identity DPP
// move makes the compiler treat it as a per-lane value, so it takes one VGPR
// instead of a scalar register that the inner loops, short of scalar
// registers, would otherwise spill to vector lanes and reload every iteration.
__device__ __forceinline__ float uniform_in_vgpr(float x) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xE4, 0xF, 0xF, true));
}

// One front-to-back step of one pixel (eq. 2).  alpha = min(alpha_max, o 2^q2)
// is used when the pixel lies inside the cut-off ellipse (q2 >= qlim) and
// alpha >= alpha_min (effective alpha 0 otherwise).  T takes T (1 - alpha)
// (one fma); when that falls below t_min the pixel stops: this Gaussian
// contributes nothing, and since T keeps the value below t_min, every later
// step fails the same test (T (1 - alpha) never exceeds T for T >= 0), so
// the pixel takes no more weight.  A live pixel has T >= t_min, so an unused
// Gaussian leaves T as it is through the same test.  Returns the weight
// alpha T (0 unless used); `taken` gets the wave's lanes that contributed,
// built from one ballot per condition (each a compare the step makes
// anyway); `kept` the lanes still live after the step (empty: every pixel of
// the band has stopped and the band can be retired).
// Pixels outside the image start at kOutsideT (negative): T (1 - alpha)
// stays negative and fails the test for any t_min >= 0.
constexpr float kOutsideT = -1.0f;

__device__ __forceinline__ float pixel_step(float q2, float opac, float& T, float qlim, float amin,
                                            float amax, float tmin, uint64_t& taken, uint64_t& kept) {
    const float al = __builtin_amdgcn_fmed3f(opac * __builtin_amdgcn_exp2f(q2), 0.0f, amax);
    const bool inq = q2 >= qlim, ina = al >= amin;
    const float ae = (inq & ina) ? al : 0.0f;
    const float wt = T * ae;
    T = fmaf(-T, ae, T);  // in place: the product above is the last read of the old T
    const bool keep = T >= tmin;
    kept = __builtin_amdgcn_ballot_w64(keep);
    taken = __builtin_amdgcn_ballot_w64(inq) & __builtin_amdgcn_ballot_w64(ina) & kept;
    return keep ? wt : 0.0f;
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
