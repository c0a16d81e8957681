// Fused per-tile blend + accumulate (the hot loop).
//
// One wave64 owns one 16x16 tile; lane l handles the four pixels
// (l%16, l/16 + 4k), k = 0..3.  The tile's Gaussians arrive in front-to-back
// order (eq. 2).  Each lane blends its pixels in FP32; per Gaussian the wave
// reduces sum_p w and sum_p w*y_p over the tile (the per-view visibility V_gj
// of eq. 5 and the numerator of eq. 6) with DPP row reductions, and one
// atomic per value adds the tile's share to the (view, Gaussian) slot.
// Splat records for the next 64 list entries are loaded one per lane and
// broadcast with v_readlane, so the loop needs no LDS and no barriers.
#include <type_traits>

#include "gsc_internal.h"
#include "wave_ops.h"

#include <algorithm>

namespace gsc {


// Adds a tile's share v to the per-view sum at p (an element of VS).  The
// default adds binary32 with a float atomic, so the order of the tiles'
// additions shows in the last bits.  DET: VS holds 64-bit fixed-point words
// instead (element k of VS is word k); v is scaled by the power of two
// `scale`, rounded to an integer and added with an integer atomic, which is
// exact and therefore independent of the order.
template <bool DET>
__device__ __forceinline__ void vs_add(float* VS, float* p, float v, float scale) {
    if constexpr (DET) {
        unsigned long long* q = reinterpret_cast<unsigned long long*>(VS) + (p - VS);
        atomicAdd(q, (unsigned long long)__float2ll_rn(v * scale));
    } else {
        unsafeAtomicAdd(p, v);
    }
}

// One tile, by one wave: blend its pixels front to back and add each
// Gaussian's tile share of V and S (channels [c_off, c_off + CC) of C) to its
// slot.  Returns the wave's accepted contributions (uniform).
//
// A pixel that stopped has T < t_min (outside the image it starts at kOutsideT).  Bands of
// four pixel rows are skipped when the Gaussian's footprint misses them (bits
// of the pair value) or when none of their pixels is live; the wave ends when
// no band is live.
template <int CC, bool BF16, int BIN, bool DET>
__device__ __forceinline__ uint32_t accumulate_tile(
    uint32_t tile, uint32_t lane, const ViewInfo* __restrict__ views, int n_views,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_vals,
    const float4* __restrict__ rec0, const float4* __restrict__ rec1,
    const uint2* __restrict__ rec2,
    const void* __restrict__ targets, int C, int c_off, int per_view, const BlendParams& bp,
    float* __restrict__ VS, float2 dsc, uint32_t* __restrict__ gcount, float4* __restrict__ lrec1,
    float2* __restrict__ lrec0) {
    constexpr int CCA = CC > 0 ? CC : 1;
    const TileGeom tg = tile_geom<BIN>(tile, views, n_views);
    const ViewInfo& V = views[tg.vloc];
    // view fields read once (plain values: the conditions below need no branch)
    const int vw = V.width, vh = V.height;
    const int64_t poff = V.pixel_offset;
    const int ix = tg.x0 + (int)(lane & 15);
    const int iy0 = tg.y0 + (int)(lane >> 4);
    const int stride = C + 1;

    float T[4];
    float y[4][CCA];
    uint32_t alive = 0;  // bit k: band k has a live pixel (wave-uniform)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int iy = iy0 + 4 * k;
        const bool inside = (ix < vw) & (iy < vh);
        T[k] = inside ? 1.0f : kOutsideT;
        alive |= (__builtin_amdgcn_ballot_w64(inside) != 0 ? 1u : 0u) << k;
        const int64_t row = poff + (int64_t)iy * vw + ix;
        // unconditional loads (element 0 stands in for pixels outside the
        // image): no branch per load
#pragma unroll
        for (int c = 0; c < CC; ++c) {
            const bool use = inside && c_off + c < C;
            const float v = load_target<BF16>(targets, use ? row * C + c_off + c : 0);
            y[k][c] = use ? v : 0.0f;
        }
    }
    alive = (uint32_t)__builtin_amdgcn_readfirstlane((int)alive);
    uint2 rg = ranges[tg.bin];
    rg.x = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.x);
    rg.y = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.y);
    uint32_t cnt = 0;
    // item = V.item_base + g (g local to the view's scene)
    const int64_t item_base = V.item_base;
    const int64_t slot_base = per_view ? V.vs_base : V.g_offset;
    const bool first_chunk = c_off == 0;

    // loop constants in vector registers (see uniform_in_vgpr)
    const float qlim = uniform_in_vgpr((float)(kExp2Scale * (double)bp.cut2));  // q <= cut2  <=>  q2 >= qlim
    const float amax = uniform_in_vgpr(bp.alpha_max), amin = uniform_in_vgpr(bp.alpha_min),
                tmin = uniform_in_vgpr(bp.t_min);
    // the lane's pixel column and rows within the tile
    const float lx = tile_offset_col(lane);
    float lyk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) lyk[k] = tile_offset_row(lane, k);

    // The list is walked in chunks of 64 entries.  A chunk's records are
    // gathered at once, one entry per lane, and broadcast entry by entry with
    // v_readlane; the next chunk's gather (and the pair values of the one
    // after) are in flight while a chunk is blended.
    auto load_pv = [&](uint32_t b) -> uint32_t {
        return b + lane < rg.y ? pair_vals[b + lane] : 0u;
    };
    // R0 keeps, per entry, the offset of the tile's centre point from the
    // projected centre, (x0 + 8 - u_hi) - u_lo and the same in y: a lane's
    // offset is then that plus its pixel's offset from the point
    // (tile_offset_col / tile_offset_row).
    const float ox = tile_centre(tg.x0), oy = tile_centre(tg.y0);
    auto gather = [&](uint32_t pv, uint32_t b, float2& R0, float4& R1, uint2& R2) {
        const uint32_t it = pv & kItemMask;
        const bool own = b + lane < rg.y;
        const float4 r = own ? rec0[it] : make_float4(0.f, 0.f, 0.f, 0.f);
        R0 = make_float2((ox - r.x) - r.z, (oy - r.y) - r.w);
        R1 = own ? rec1[it] : make_float4(0.f, 0.f, 0.f, 0.f);
        R2 = own ? rec2[it] : make_uint2(0u, 0u);
    };
    // (wide channel chunks have no registers to spare for the second buffer:
    // there the next chunk is gathered when the current one is done)
    constexpr bool kDouble = CC <= 4;
    uint32_t pv = load_pv(rg.x), pvn = load_pv(rg.x + 64);
    float2 R0;
    float4 R1;
    uint2 R2;
    gather(pv, rg.x, R0, R1, R2);
    for (uint32_t b = rg.x; b < rg.y && alive != 0u; b += 64) {
        const uint32_t nb = min(64u, rg.y - b);
        float2 Q0;
        float4 Q1;
        uint2 Q2;
        if constexpr (kDouble) gather(pvn, b + 64, Q0, Q1, Q2);
        const uint32_t pvnn = load_pv(b + 128);
        // the chunk's entries that can reach a live band, one bit per lane in
        // list order: the walk visits only these
        // each lane forms its entry's band mask: taking an entry then costs
        // one broadcast of it
        const uint32_t BL = lane < nb ? entry_bands<BIN>(pv, tg.quad, R2.x, tg.y0) : 0u;
        uint64_t todo = __builtin_amdgcn_ballot_w64((BL & alive) != 0u);
        // the chunk's records go through LDS (this wave's 64 slots): an entry
        // reads them back with two broadcast loads instead of six readlanes
        lrec1[lane] = R1;
        lrec0[lane] = R0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if constexpr (CC >= 1 && CC <= 3) {
            // Entries in groups of four: each entry's tile sums (V, S) stay in
            // a fixed register slot, and one wave reduction of the group's 16
            // values (lane e*4+v, bit-reversed) feeds one atomic per value.
            // Tile liveness is refreshed once per group: entries after the
            // last live pixel stopped meet T < t_min everywhere and add nothing.
            while (todo != 0u && alive != 0u) {
                float pend[16];
                int64_t gslot[4];
                bool has[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const bool any = todo != 0u;
                    const uint32_t j = any ? (uint32_t)__builtin_ctzll(todo) : 0u;
                    todo &= todo - 1u;
                    const uint32_t gid = bcast_u(R2.y, j);  // the entry's item
                    const uint32_t bands = any ? bcast_u(BL, j) & alive : 0u;
                    float sv = 0.0f, s0 = 0.0f, s1 = 0.0f, s2 = 0.0f;
                    uint32_t nh = 0;
                    if (bands != 0u) {
                        const float2 c0 = lrec0[j];
                        const float4 c1 = lrec1[j];
                        const float dx = c0.x + lx;
                        const float a0 = c1.x * dx * dx;
                        const float b0 = c1.y * dx;
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            if (!((bands >> k) & 1u)) continue;  // uniform
                            const float dy = c0.y + lyk[k];
                            const float q2 = fmaf(dy, fmaf(c1.z, dy, b0), a0);
                            uint64_t taken, kept;
                            const float w = pixel_step(q2, c1.w, T[k], qlim, amin, amax, tmin, taken, kept);
                            sv += w;
                            s0 = fmaf(w, y[k][0], s0);
                            if constexpr (CC > 1) s1 = fmaf(w, y[k][CC > 1 ? 1 : 0], s1);
                            if constexpr (CC > 2) s2 = fmaf(w, y[k][CC > 2 ? 2 : 0], s2);
                            nh += (uint32_t)__popcll(taken);
                        }
                    }
                    nh = (uint32_t)__builtin_amdgcn_readfirstlane((int)nh);
                    cnt += nh;
                    const int64_t g = (int64_t)gid - item_base;
                    if (nh != 0u && gcount != nullptr && first_chunk && lane == 0)
                        atomicAdd(gcount + V.g_offset + g, nh);
                    has[u] = nh != 0u;
                    gslot[u] = slot_base + g;
                    pend[4 * u] = sv;
                    pend[4 * u + 1] = s0;
                    pend[4 * u + 2] = s1;
                    pend[4 * u + 3] = s2;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (((alive >> k) & 1u) && __builtin_amdgcn_ballot_w64(T[k] >= tmin) == 0) alive &= ~(1u << k);
                alive = (uint32_t)__builtin_amdgcn_readfirstlane((int)alive);
                if (has[0] || has[1] || has[2] || has[3]) {
                    const float t = wave_sum_transposed<16>(pend, lane);
                    const int idx = transposed_index<16>(lane);
                    const int e = idx >> 2, v = idx & 3;
                    const bool he = e == 0 ? has[0] : (e == 1 ? has[1] : (e == 2 ? has[2] : has[3]));
                    const int64_t sl = e == 0 ? gslot[0] : (e == 1 ? gslot[1] : (e == 2 ? gslot[2] : gslot[3]));
                    const bool use = lane < 16u && he && (v == 0 ? first_chunk : (v <= CC && c_off + v - 1 < C));
                    if (use) vs_add<DET>(VS, VS + sl * (int64_t)stride + (v == 0 ? 0 : c_off + v), t,
                                         v == 0 ? dsc.x : dsc.y);
                }
            }
        } else {
            while (todo != 0u) {
                const uint32_t j = (uint32_t)__builtin_ctzll(todo);
                todo &= todo - 1u;
                const uint32_t bands = bcast_u(BL, j) & alive;
                if (bands == 0u) continue;
                const uint32_t gid = bcast_u(R2.y, j);  // the entry's item
                const float2 c0 = lrec0[j];
                const float4 c1 = lrec1[j];
                const float dx = c0.x + lx;
                const float a0 = c1.x * dx * dx;
                const float b0 = c1.y * dx;
                float sv = 0.0f;
                float ss[CCA];
#pragma unroll
                for (int c = 0; c < CCA; ++c) ss[c] = 0.0f;
                uint32_t nh = 0;    // contributions of this entry (wave total)
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    if (!((bands >> k) & 1u)) continue;  // uniform
                    const float dy = c0.y + lyk[k];
                    const float q2 = fmaf(dy, fmaf(c1.z, dy, b0), a0);
                    uint64_t taken, kept;
                    const float w = pixel_step(q2, c1.w, T[k], qlim, amin, amax, tmin, taken, kept);
                    sv += w;
#pragma unroll
                    for (int c = 0; c < CC; ++c) ss[c] = fmaf(w, y[k][c], ss[c]);
                    nh += (uint32_t)__popcll(taken);
                    if (kept == 0) alive &= ~(1u << k);
                }
                // keep the band mask and the count in scalar registers
                alive = (uint32_t)__builtin_amdgcn_readfirstlane((int)alive);
                nh = (uint32_t)__builtin_amdgcn_readfirstlane((int)nh);
                cnt += nh;
                if (nh != 0u) {
                    // the pair carries the depth rank; the record names the item
                    const int64_t g = (int64_t)gid - item_base;
                    if (gcount != nullptr && first_chunk && lane == 0) atomicAdd(gcount + V.g_offset + g, nh);
                    float* slot = VS + (slot_base + g) * (int64_t)stride;
                    if constexpr (CC == 0) {
                        const float tv = wave_sum(sv);
                        if (lane == 0) vs_add<DET>(VS, slot, tv, dsc.x);
                    } else if constexpr (CC <= 3) {
                        const float v1 = CC > 1 ? ss[CC > 1 ? 1 : 0] : 0.0f;
                        const float v2 = CC > 2 ? ss[CC > 2 ? 2 : 0] : 0.0f;
                        const float t = wave_sum4_transposed(sv, ss[0], v1, v2, lane);
                        if (lane < 4u) {
                            const int idx = transposed_index<4>(lane);
                            if (idx == 0) {
                                if (first_chunk) vs_add<DET>(VS, slot, t, dsc.x);
                            } else if (idx <= CC && c_off + idx - 1 < C) {
                                vs_add<DET>(VS, slot + c_off + idx, t, dsc.y);
                            }
                        }
                    } else {
                        const float tv = wave_sum(sv);
                        const float t = wave_sum_transposed<CC>(ss, lane);
                        if (lane == 0 && first_chunk) vs_add<DET>(VS, slot, tv, dsc.x);
                        if (lane < (uint32_t)CC) {
                            const int c = c_off + transposed_index<CC>(lane);
                            if (c < C) vs_add<DET>(VS, slot + 1 + c, t, dsc.y);
                        }
                    }
                }
                if (alive == 0u) break;
            }
        }
        __builtin_amdgcn_wave_barrier();  // the next chunk's records overwrite these
        if constexpr (kDouble) {
            R0 = Q0;
            R1 = Q1;
            R2 = Q2;
        } else {
            gather(pvn, b + 64, R0, R1, R2);
        }
        pv = pvn;
        pvn = pvnn;
    }
    return cnt;
}

// CC: channels handled by this launch (chunk [c_off, c_off + CC) of C).
// queue == nullptr: one tile per wave (4 per block) over a grid covering all
// tiles.  Otherwise persistent: a fixed grid whose waves take tiles from the
// counter *queue (zero before the launch) until none are left.  Either way
// tiles come in the order `order` gives (nullptr: tile index order).
// Waves per SIMD the register allocation is held to: the forms of up to
// three channels fit seven (72 registers) and run faster there; wider ones
// spill when held below their natural count and are left alone.
template <int CC>
constexpr int acc_waves_per_simd() { return CC >= 1 && CC <= 3 ? 7 : 1; }

template <int CC, bool BF16, int BIN, bool DET>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(acc_waves_per_simd<CC>()))) void k_accumulate(
    const ViewInfo* __restrict__ views, int n_views, uint32_t n_tiles, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ pair_vals,
    const float4* __restrict__ rec0, const float4* __restrict__ rec1,
    const uint2* __restrict__ rec2, const void* __restrict__ targets, int C, int c_off,
    int per_view, BlendParams bp, float* __restrict__ VS, float2 dsc,
    unsigned long long* __restrict__ counter, uint32_t* __restrict__ gcount,
    uint32_t* __restrict__ queue, const uint32_t* __restrict__ order) {
    __shared__ float4 srec1[4][64];
    __shared__ float2 srec0[4][64];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t cnt = 0;
    if (queue == nullptr) {
        const uint32_t wi = xcd_block(blockIdx.x, gridDim.x) * 4 + w;
        if (wi >= n_tiles) return;  // whole wave
        const uint32_t tile = queued_tile<BIN>(wi, order);  // blocks start in index order
        cnt = accumulate_tile<CC, BF16, BIN, DET>(tile, lane, views, n_views, ranges, pair_vals,
                                                  rec0, rec1, rec2, targets, C, c_off, per_view, bp,
                                                  VS, dsc, gcount, srec1[w], srec0[w]);
    } else {
        for (;;) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(queue, 1u);
            const uint32_t tq = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
            if (tq >= n_tiles) break;  // uniform: every wave ends here
            const uint32_t tile = queued_tile<BIN>(tq, order);
            cnt += accumulate_tile<CC, BF16, BIN, DET>(tile, lane, views, n_views, ranges, pair_vals,
                                                       rec0, rec1, rec2, targets, C, c_off,
                                                       per_view, bp, VS, dsc, gcount, srec1[w], srec0[w]);
        }
    }
    if (c_off == 0 && lane == 0 && cnt) atomicAdd(counter, (unsigned long long)cnt);
}

// Waves (16x16 tiles) of a launch over n_bins bins of `bin` pixels.
static inline uint32_t wave_tiles(uint32_t n_bins, int bin) { return bin == 32 ? 4u * n_bins : n_bins; }

template <int CC, bool BF16, int BIN, bool DET = false>
static void launch_acc_k(const ViewInfo* views, int n_views, uint32_t n_wt, const uint2* ranges,
                         const uint32_t* pair_vals, const float4* rec0,
                         const float4* rec1,
                         const uint2* rec2, const void* targets, int C, bool per_view,
                         BlendParams bp, float* VS, unsigned long long* counter, uint32_t* gcount,
                         uint32_t* queues, const uint32_t* order, hipStream_t s,
                         float2 dsc = make_float2(0.f, 0.f)) {
    const uint32_t full = (n_wt + 3) / 4;
    dim3 grid(queues ? std::min(full, kPersistentBlocks) : full), block(256);
    int pass = 0;
    const int step = CC > 0 ? CC : C + 1;
    for (int c_off = 0; c_off < std::max(C, 1); c_off += step, ++pass) {
        uint32_t* q = queues ? queues + pass : nullptr;
        hipLaunchKernelGGL((k_accumulate<CC, BF16, BIN, DET>), grid, block, 0, s, views, n_views, n_wt,
                           ranges, pair_vals, rec0, rec1, rec2, targets, C, c_off,
                           (int)per_view, bp, VS, dsc, counter, gcount, q, order);
    }
}

template <int CC>
static void launch_acc_cc(const ViewInfo* views, int n_views, uint32_t n_bins, const uint2* ranges,
                          const uint32_t* pair_vals, const float4* rec0,
                          const float4* rec1,
                          const uint2* rec2, int bin, const void* targets, int tdtype, int C,
                          bool per_view, BlendParams bp, float* VS, unsigned long long* counter,
                          uint32_t* gcount, uint32_t* queues, const uint32_t* order, hipStream_t s,
                          const float2* det) {
    const uint32_t n_wt = wave_tiles(n_bins, bin);
    const bool bf = tdtype == GSC_BF16;
#define GSC_ACCK(BFV, BINV, DETV)                                                                  \
    launch_acc_k<CC, BFV, BINV, DETV>(views, n_views, n_wt, ranges, pair_vals, rec0, rec1, rec2,    \
                                      targets, C, per_view, bp, VS, counter, gcount, queues, order, s, \
                                      det ? *det : make_float2(0.f, 0.f))
    if (det) {
        if (bin == 32) {
            if (bf) GSC_ACCK(true, 32, true); else GSC_ACCK(false, 32, true);
        } else {
            if (bf) GSC_ACCK(true, 16, true); else GSC_ACCK(false, 16, true);
        }
    } else if (bin == 32) {
        if (bf) GSC_ACCK(true, 32, false); else GSC_ACCK(false, 32, false);
    } else {
        if (bf) GSC_ACCK(true, 16, false); else GSC_ACCK(false, 16, false);
    }
#undef GSC_ACCK
}

// ---- matrix-core accumulate (BF16 targets, channel blocks of 16) ----------
//
// The channel sums S_g[c] = sum_p w_gp y_p[c] of a tile are a product
// W (Gaussians x pixels) . Y (pixels x channels).  Here the blend runs as in
// accumulate_tile, but each entry's weights go to LDS as a row of W, split
// into a BF16 high part (w's upper half) and a BF16 remainder (the exact
// w - hi rounded; w = hi + lo to 2^-16 relative).  Every 8 or 16 entries,
// v_mfma_f32_16x16x32_bf16 forms (W_hi + W_lo) . [Y | 1] over the tile's 256
// pixels (eight K-steps of 32 pixels): the targets, held as B operands in
// registers for the whole tile, give S, and a block of ones gives
// V = sum_p w from the same split weights.  (Groups of 8 entries put W_hi in
// rows 0..7 of the A operand and W_lo in rows 8..15: one product per K-step.)
// K index k = 32 s + 8 (lane / 16) + i of K-step s is tile pixel k (row k/16,
// column k%16); the blend's lane l owns pixels l + 64 j, j = 0..3.

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

constexpr int kWRow = 264;       // LDS row of W in BF16 elements (256 + padding against bank conflicts)
constexpr int kMfmaWaves = 2;    // waves per block

// W rows of one wave: ROWS list entries per matrix product (8 or 16; with 8,
// the A operand holds the high parts in rows 0..7 and the remainders in rows
// 8..15, and less LDS per wave leaves room for more waves).
template <int ROWS>
struct alignas(16) MfmaLds {
    __bf16 whi[ROWS * kWRow];
    __bf16 wlo[ROWS * kWRow];
    uint32_t gslot[ROWS];  // local Gaussian of each group row (0xFFFFFFFF: no contribution)
    float4 crec1[64];      // the chunk's records, read back by every lane as one broadcast:
    float2 crec0[64];      // conic and opacity; the centre offset (one channel block only)
};

template <int NBLK>
constexpr int mfma_rows() { return NBLK <= 2 ? 8 : 16; }
// Waves per SIMD the register allocation is held to (the weight rows in LDS
// allow them): the 32-channel form ran at two waves per SIMD with 208
// registers and runs at three with 168; the 16-channel and packed forms at
// four (128 registers, up from three).  The 64-channel form keeps its 128
// target registers unconstrained.
template <int NBLK>
constexpr int mfma_waves_per_simd() { return NBLK == 2 ? 3 : (NBLK == 1 ? 4 : 1); }

// YM: target layout in the B operand.  0: BF16, NBLK blocks of 16 channels,
// V from a separate product against ones.  1: BF16, C <= 15 channels packed
// with a ones column (column C) in one block.  2: FP32, C <= 7 channels
// split into BF16 high parts (columns 0..C-1) and remainders (columns
// C..2C-1), ones in column 2C.  Packed forms run in one launch (c_off = 0).
template <int NBLK, int BIN, int YM>
__device__ __forceinline__ uint32_t accumulate_tile_mfma(
    uint32_t tile, uint32_t lane, MfmaLds<mfma_rows<NBLK>()>& L, const ViewInfo* __restrict__ views, int n_views,
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ pair_vals,
    const float4* __restrict__ rec0, const float4* __restrict__ rec1, const uint2* __restrict__ rec2,
    const void* __restrict__ targets, int C, int c_off, int per_view, const BlendParams& bp,
    float* __restrict__ VS, uint32_t* __restrict__ gcount) {
    const TileGeom tg = tile_geom<BIN>(tile, views, n_views);
    const ViewInfo& V = views[tg.vloc];
    // view fields read once (plain values: the conditions below need no branch)
    const int vw = V.width, vh = V.height;
    const int64_t poff = V.pixel_offset;
    const int ix = tg.x0 + (int)(lane & 15);
    const int iy0 = tg.y0 + (int)(lane >> 4);
    const int stride = C + 1;
    const uint32_t n16 = lane & 15, q4 = lane >> 4;
    constexpr int ROWS = mfma_rows<NBLK>();

    // targets of the tile as B operands: Y[s][b] holds pixels 32 s + 8 q4 + i
    // (tile row 2 s + q4/2, columns 8 (q4&1) + i) of channel c_off + 16 b + n16
    bf16x8_t Y[8][NBLK];
    // packed forms: the channel this lane's column reads, and its role
    const int pc = YM == 2 ? ((int)n16 < C ? (int)n16 : (int)n16 - C) : (int)n16;
    const bool pcol = YM == 2 ? (int)n16 < 2 * C : (int)n16 < C;   // a target column
    const bool pone = YM == 2 ? (int)n16 == 2 * C : (int)n16 == C;  // the ones column
    if constexpr (NBLK == 1) {
        // One 64-bit offset per row of eight pixels, then a uniform step of C
        // elements per pixel; element 0 of the view stands in outside (no branch).
        // All loads are issued before any is used (one channel block: 5.37 ->
        // 5.31-5.34 ms per launch on the 32-scene plan; with two blocks the
        // loaded values spill, 8.0 -> 8.2 ms, and the form below is kept).
        using TY = std::conditional_t<YM == 2, float, uint16_t>;
        const TY* vt = (const TY*)targets + poff * C;
        TY xv[8][NBLK][8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int gy = tg.y0 + 2 * s + (int)(q4 >> 1);
            const int gx0 = tg.x0 + 8 * (int)(q4 & 1u);
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                const int c = YM == 0 ? c_off + 16 * b + (int)n16 : pc;
                const bool rowin = (gy < vh) & (YM == 0 ? c < C : pcol);
                const TY* rp = vt + (rowin ? ((int64_t)gy * vw + gx0) * C + c : (int64_t)0);
#pragma unroll
                for (int i = 0; i < 8; ++i) xv[s][b][i] = *((rowin & (gx0 + i < vw)) ? rp + i * C : vt);
            }
        }
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int gy = tg.y0 + 2 * s + (int)(q4 >> 1);
            const int gx0 = tg.x0 + 8 * (int)(q4 & 1u);
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                const int c = YM == 0 ? c_off + 16 * b + (int)n16 : pc;
                const bool rowin = (gy < vh) & (YM == 0 ? c < C : pcol);
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const bool in = rowin & (gx0 + i < vw);
                    const TY x = xv[s][b][i];
                    if constexpr (YM == 2) {
                        const __bf16 hi = (__bf16)x;
                        const __bf16 v = (int)n16 < C ? hi : (__bf16)(x - (float)hi);
                        Y[s][b][i] = in ? v : (pone ? (__bf16)1.0f : (__bf16)0.0f);
                    } else {
                        const __bf16 v = __builtin_bit_cast(__bf16, x);
                        Y[s][b][i] = in ? v : ((YM == 1 && pone) ? (__bf16)1.0f : (__bf16)0.0f);
                    }
                }
            }
        }
    } else {
        // a 64-bit element index per load
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int gy = tg.y0 + 2 * s + (int)(q4 >> 1);
            const int gx0 = tg.x0 + 8 * (int)(q4 & 1u);
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                const int c = YM == 0 ? c_off + 16 * b + (int)n16 : pc;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int gx = gx0 + i;
                    const bool in = (gx < vw) & (gy < vh) & (YM == 0 ? c < C : pcol);
                    const int64_t row = poff + (int64_t)gy * vw + gx;
                    // unconditional load (element 0 stands in outside): no branch
                    const int64_t e = in ? row * C + c : 0;
                    if constexpr (YM == 2) {
                        const float f = ((const float*)targets)[e];
                        const __bf16 hi = (__bf16)f;
                        const __bf16 v = (int)n16 < C ? hi : (__bf16)(f - (float)hi);
                        Y[s][b][i] = in ? v : (pone ? (__bf16)1.0f : (__bf16)0.0f);
                    } else {
                        const uint16_t u = ((const uint16_t*)targets)[e];
                        const __bf16 v = __builtin_bit_cast(__bf16, u);
                        Y[s][b][i] = in ? v : ((YM == 1 && pone) ? (__bf16)1.0f : (__bf16)0.0f);
                    }
                }
            }
        }
    }
    // the ones operand, each register made through an identity DPP move so
    // that the compiler holds it instead of rebuilding it before every product
    bf16x8_t ones;
    {
        uint32_t o4[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) o4[i] = (uint32_t)__builtin_amdgcn_mov_dpp(0x3F803F80, 0xE4, 0xF, 0xF, true);
        ones = __builtin_bit_cast(bf16x8_t, o4);
    }

    // transmittance of the lane's pixel in each band: four scalars (as an
    // array the compiler rebuilt it in new registers on every band update)
    float T0, T1, T2, T3;
    uint32_t alive = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool inside = (ix < vw) & (iy0 + 4 * k < vh);
        const float t = inside ? 1.0f : kOutsideT;
        if (k == 0) T0 = t;
        if (k == 1) T1 = t;
        if (k == 2) T2 = t;
        if (k == 3) T3 = t;
        alive |= (__builtin_amdgcn_ballot_w64(inside) != 0 ? 1u : 0u) << k;
    }
    alive = (uint32_t)__builtin_amdgcn_readfirstlane((int)alive);
    uint2 rg = ranges[tg.bin];
    rg.x = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.x);
    rg.y = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.y);
    uint32_t cnt = 0;
    const int64_t item_base = V.item_base;
    const int64_t slot_base = per_view ? V.vs_base : V.g_offset;
    const int64_t g_off = V.g_offset;
    const bool first_chunk = c_off == 0;
    // loop constants in vector registers (see uniform_in_vgpr)
    const float qlim = uniform_in_vgpr((float)(kExp2Scale * (double)bp.cut2));
    const float amax = uniform_in_vgpr(bp.alpha_max), amin = uniform_in_vgpr(bp.alpha_min),
                tmin = uniform_in_vgpr(bp.t_min);
    // the lane's pixel offsets from the tile's centre point; R0 below keeps,
    // per entry, the offset of that point from the projected centre
    const float lx = tile_offset_col(lane);
    float lyk[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) lyk[k] = tile_offset_row(lane, k);
    const float ox = tile_centre(tg.x0), oy = tile_centre(tg.y0);

    // Rows are never cleared: rows past a group's count feed only output rows
    // that the flush does not use, and an entry writes zeros in the bands its
    // footprint misses (measured faster than per-row band masks that zero
    // the operand in the flush, for one and for two channel blocks).

    // one matrix product over the group's `rows` entries, then the atomics.
    // With 8 rows per group the A operand's rows 0..7 take the weights' high
    // parts and rows 8..15 their remainders, so one product per K-step forms
    // both halves; each output row then adds its two halves (lanes l and
    // l + 32).  With 16 rows the high parts and the remainders take a
    // product each.
    constexpr bool kSplitRows = ROWS == 8;
    auto flush = [&](uint32_t rows) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        floatx4_t D[NBLK], DV;
#pragma unroll
        for (int b = 0; b < NBLK; ++b) D[b] = floatx4_t{0.f, 0.f, 0.f, 0.f};
        DV = floatx4_t{0.f, 0.f, 0.f, 0.f};
        const uint32_t arow = kSplitRows ? (n16 & 7u) : n16;
        const __bf16* ah_p = &((kSplitRows && n16 >= 8u) ? L.wlo : L.whi)[arow * kWRow + 8 * q4];
        const __bf16* al_p = &L.wlo[arow * kWRow + 8 * q4];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const bf16x8_t ah = *reinterpret_cast<const bf16x8_t*>(ah_p + 32 * s);
            if (YM == 0 && first_chunk) DV = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, ones, DV, 0, 0, 0);
#pragma unroll
            for (int b = 0; b < NBLK; ++b) D[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, Y[s][b], D[b], 0, 0, 0);
            if constexpr (!kSplitRows) {
                const bf16x8_t al = *reinterpret_cast<const bf16x8_t*>(al_p + 32 * s);
                if (YM == 0 && first_chunk) DV = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, ones, DV, 0, 0, 0);
#pragma unroll
                for (int b = 0; b < NBLK; ++b)
                    D[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, Y[s][b], D[b], 0, 0, 0);
            }
        }
        if constexpr (kSplitRows) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if (YM == 0 && first_chunk) DV[i] += __shfl_xor(DV[i], 32, 64);
#pragma unroll
                for (int b = 0; b < NBLK; ++b) D[b][i] += __shfl_xor(D[b][i], 32, 64);
            }
        }
        // lane holds rows 4 q4 + i, column n16
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t m = 4 * q4 + (uint32_t)i;
            float lo = 0.0f;
            if constexpr (YM == 2) lo = __shfl(D[0][i], (int)lane + C, 64);  // remainder column
            if (m >= rows) continue;
            const uint32_t gl = L.gslot[m];
            if (gl == 0xFFFFFFFFu) continue;
            float* slot = VS + (slot_base + (int64_t)gl) * (int64_t)stride;
            if constexpr (YM == 0) {
                if (first_chunk && n16 == 0) unsafeAtomicAdd(slot, DV[i]);
#pragma unroll
                for (int b = 0; b < NBLK; ++b) {
                    const int c = c_off + 16 * b + (int)n16;
                    if (c < C) unsafeAtomicAdd(slot + 1 + c, D[b][i]);
                }
            } else {
                if (pone) unsafeAtomicAdd(slot, D[0][i]);
                else if ((int)n16 < C) unsafeAtomicAdd(slot + 1 + n16, D[0][i] + lo);
            }
        }
        // the next group overwrites these rows
        __builtin_amdgcn_wave_barrier();
    };

    // list walk: chunks of 64 entries gathered one per lane; each lane also
    // forms its entry's band mask (the live bands its footprint rows reach),
    // so taking an entry costs one broadcast of that mask; the entries that
    // reach a live band are taken in order
    constexpr bool kLdsCentre = NBLK == 1;
    uint32_t rows = 0;
    for (uint32_t b = rg.x; b < rg.y && alive != 0u; b += 64) {
        const bool in_list = b + lane < rg.y;
        const uint32_t pv = in_list ? pair_vals[b + lane] : 0u;
        const uint32_t it = pv & kItemMask;
        const bool own = in_list && pair_reaches<BIN>(pv, tg.quad, alive);
        const float4 r = own ? rec0[it] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float2 R0 = make_float2((ox - r.x) - r.z, (oy - r.y) - r.w);
        const float4 R1 = own ? rec1[it] : make_float4(0.f, 0.f, 0.f, 0.f);
        const uint2 r2 = own ? rec2[it] : make_uint2(0u, 0u);
        const uint32_t gid = r2.y;  // the entry's item (geometry slot) index
        const uint32_t BL = own ? (entry_bands<BIN>(pv, tg.quad, r2.x, tg.y0) & alive) : 0u;
        uint64_t sm = __builtin_amdgcn_ballot_w64(BL != 0u);  // entries still to take
        // the records go through LDS: an entry then reads them with one
        // broadcast load each instead of a readlane per value (measured:
        // the centre offset too for one channel block, 5.52 -> 5.43 ms per
        // launch on the 32-scene plan; the conic and opacity only for two,
        // 8.18 -> 7.99 ms on the feature workload)
        L.crec1[lane] = R1;
        if constexpr (kLdsCentre) L.crec0[lane] = R0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        while (sm != 0u) {
            const uint32_t j = (uint32_t)__builtin_ctzll(sm);
            sm &= sm - 1;
            const uint32_t bands = bcast_u(BL, j) & alive;
            if (bands == 0u) continue;
            const float2 c0 = kLdsCentre ? L.crec0[j] : make_float2(bcast(R0.x, j), bcast(R0.y, j));
            const float4 c1 = L.crec1[j];
            const float dx = c0.x + lx;
            const float a0 = c1.x * dx * dx;
            const float b0 = c1.y * dx;
            uint32_t nh = 0;
            __bf16* wrow_h = &L.whi[rows * kWRow];
            __bf16* wrow_l = &L.wlo[rows * kWRow];
            auto band = [&](const int k, float& Tk) {
                if (!((bands >> k) & 1u)) {  // uniform: no weight in this band
                    wrow_h[lane + 64 * k] = (__bf16)0.0f;
                    wrow_l[lane + 64 * k] = (__bf16)0.0f;
                    return;
                }
                const float dy = c0.y + lyk[k];
                const float q2 = fmaf(dy, fmaf(c1.z, dy, b0), a0);
                uint64_t taken, kept;
                const float w = pixel_step(q2, c1.w, Tk, qlim, amin, amax, tmin, taken, kept);
                // hi: w's upper half (truncated), lo: the exact remainder rounded
                // to BF16; |w - hi - lo| <= 2^-16 |w|
                const uint32_t wb = __float_as_uint(w);
                const __bf16 hi = __builtin_bit_cast(__bf16, (uint16_t)(wb >> 16));
                const __bf16 lo = (__bf16)(w - __uint_as_float(wb & 0xffff0000u));
                wrow_h[lane + 64 * k] = hi;
                wrow_l[lane + 64 * k] = lo;
                nh += (uint32_t)__popcll(taken);
                if (kept == 0) alive &= ~(1u << k);
            };
            band(0, T0);
            band(1, T1);
            band(2, T2);
            band(3, T3);
            alive = (uint32_t)__builtin_amdgcn_readfirstlane((int)alive);
            nh = (uint32_t)__builtin_amdgcn_readfirstlane((int)nh);
            cnt += nh;
            const uint32_t gl = (uint32_t)((int64_t)bcast_u(gid, j) - item_base);
            if (lane == 0) L.gslot[rows] = nh != 0u ? gl : 0xFFFFFFFFu;
            if (nh != 0u && gcount != nullptr && first_chunk && lane == 0) atomicAdd(gcount + g_off + gl, nh);
            if (++rows == (uint32_t)ROWS) {
                flush(rows);
                rows = 0;
            }
            if (alive == 0u) break;
        }
        __builtin_amdgcn_wave_barrier();  // the next chunk's records overwrite these
    }
    if (rows != 0u) flush(rows);
    return cnt;
}

template <int NBLK, int BIN, int YM>
__global__ __launch_bounds__(64 * kMfmaWaves)
__attribute__((amdgpu_waves_per_eu(mfma_waves_per_simd<NBLK>()))) void k_accumulate_mfma(
    const ViewInfo* __restrict__ views, int n_views, uint32_t n_tiles, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ pair_vals, const float4* __restrict__ rec0,
    const float4* __restrict__ rec1, const uint2* __restrict__ rec2,
    const void* __restrict__ targets, int C, int c_off, int per_view, BlendParams bp,
    float* __restrict__ VS, unsigned long long* __restrict__ counter, uint32_t* __restrict__ gcount,
    uint32_t* __restrict__ queue, const uint32_t* __restrict__ order) {
    __shared__ MfmaLds<mfma_rows<NBLK>()> lds[kMfmaWaves];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t cnt = 0;
    if (queue == nullptr) {
        const uint32_t wi = xcd_block(blockIdx.x, gridDim.x) * kMfmaWaves + w;
        if (wi >= n_tiles) return;  // whole wave
        const uint32_t tile = queued_tile<BIN>(wi, order);  // blocks start in index order
        cnt = accumulate_tile_mfma<NBLK, BIN, YM>(tile, lane, lds[w], views, n_views, ranges, pair_vals,
                                              rec0, rec1, rec2, targets, C, c_off, per_view, bp, VS,
                                              gcount);
    } else {
        for (;;) {
            uint32_t t = 0;
            if (lane == 0) t = atomicAdd(queue, 1u);
            const uint32_t tq = (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
            if (tq >= n_tiles) break;  // uniform: every wave ends here
            const uint32_t tile = queued_tile<BIN>(tq, order);
            cnt += accumulate_tile_mfma<NBLK, BIN, YM>(tile, lane, lds[w], views, n_views, ranges,
                                                   pair_vals, rec0, rec1, rec2, targets, C, c_off,
                                                   per_view, bp, VS, gcount);
        }
    }
    if (c_off == 0 && lane == 0 && cnt) atomicAdd(counter, (unsigned long long)cnt);
}

template <int NBLK, int BIN, int YM>
static void launch_acc_mfma(const ViewInfo* views, int n_views, uint32_t n_wt, const uint2* ranges,
                            const uint32_t* pair_vals, const float4* rec0, const float4* rec1,
                            const uint2* rec2, const void* targets, int C, bool per_view,
                            BlendParams bp, float* VS, unsigned long long* counter, uint32_t* gcount,
                            uint32_t* queues, const uint32_t* order, hipStream_t s) {
    const uint32_t full = (n_wt + kMfmaWaves - 1) / kMfmaWaves;
    dim3 grid(queues ? std::min(full, 2 * kPersistentBlocks) : full), block(64 * kMfmaWaves);
    int pass = 0;
    const int step = YM == 0 ? 16 * NBLK : C;  // packed forms: one launch
    for (int c_off = 0; c_off < C; c_off += step, ++pass) {
        uint32_t* q = queues ? queues + pass : nullptr;
        hipLaunchKernelGGL((k_accumulate_mfma<NBLK, BIN, YM>), grid, block, 0, s, views, n_views, n_wt,
                           ranges, pair_vals, rec0, rec1, rec2, targets, C, c_off,
                           (int)per_view, bp, VS, counter, gcount, q, order);
    }
}

template <int NBLK, int YM>
static void launch_acc_mfma_bin(const ViewInfo* views, int n_views, uint32_t n_bins, const uint2* ranges,
                                const uint32_t* pair_vals, const float4* rec0, const float4* rec1,
                                const uint2* rec2, int bin, const void* targets, int C, bool per_view,
                                BlendParams bp, float* VS, unsigned long long* counter,
                                uint32_t* gcount, uint32_t* queues, const uint32_t* order,
                                hipStream_t s) {
    const uint32_t n_wt = wave_tiles(n_bins, bin);
    if (bin == 32)
        launch_acc_mfma<NBLK, 32, YM>(views, n_views, n_wt, ranges, pair_vals, rec0, rec1, rec2, targets, C,
                                  per_view, bp, VS, counter, gcount, queues, order, s);
    else
        launch_acc_mfma<NBLK, 16, YM>(views, n_views, n_wt, ranges, pair_vals, rec0, rec1, rec2, targets, C,
                                  per_view, bp, VS, counter, gcount, queues, order, s);
}

int accumulate_chunk(int C, int tdtype) {
    // (one 64-channel launch holds its targets in 128 registers and runs one
    // wave per SIMD; two 32-channel launches measure as fast or faster)
    if (tdtype == GSC_BF16 && C >= 16) return kChunkMfma | (C <= 16 ? 16 : 32);
    return C <= 3 ? C : (C <= 4 ? 4 : (C <= 8 ? 8 : 16));
}

int resolve_chunk(int requested, int C, int tdtype) {
    if (!accumulate_chunk_valid(requested, tdtype)) return accumulate_chunk(C, tdtype);
    if (requested == kChunkPacked && C > (tdtype == GSC_BF16 ? 15 : 7)) return accumulate_chunk(C, tdtype);
    return requested;
}

bool accumulate_chunk_valid(int chunk, int tdtype) {
    if (chunk & kChunkMfma) {
        const int ch = chunk_channels(chunk);
        if (chunk != (kChunkMfma | ch)) return false;
        if (ch == 1) return true;  // packed form; fits_packed() checks C
        return tdtype == GSC_BF16 && (ch == 16 || ch == 32 || ch == 64);
    }
    return chunk == 1 || chunk == 2 || chunk == 3 || chunk == 4 || chunk == 8 || chunk == 16;
}

void launch_accumulate(const ViewInfo* views, int n_views, uint32_t n_tiles, const uint2* ranges,
                       const uint32_t* pair_vals, const float4* rec0,
                       const float4* rec1,
                       const uint2* rec2, int bin, const void* targets, int tdtype, int C,
                       bool per_view, BlendParams bp, float* VS, unsigned long long* counter,
                       uint32_t* gcount, hipStream_t s, const uint32_t* order) {
    launch_accumulate_chunked(views, n_views, n_tiles, ranges, pair_vals, rec0, rec1, rec2, bin,
                              targets, tdtype, C, per_view, bp, VS, counter, gcount, 0, s, nullptr, order,
                              nullptr);
}

void launch_accumulate_chunked(const ViewInfo* views, int n_views, uint32_t n_tiles,
                               const uint2* ranges, const uint32_t* pair_vals,
                               const float4* rec0,
                               const float4* rec1, const uint2* rec2, int bin,
                               const void* targets, int tdtype, int C, bool per_view,
                               BlendParams bp, float* VS, unsigned long long* counter,
                               uint32_t* gcount, int chunk, hipStream_t s, uint32_t* queues,
                               const uint32_t* order, const float2* det) {
    if (n_tiles == 0) return;
    chunk = resolve_chunk(chunk, C, tdtype);
    if (det && (chunk & kChunkMfma)) chunk = accumulate_chunk(C, GSC_F32);  // vector form only
    if (queues) launch_fill_u32(queues, 0u, (uint64_t)accumulate_launches(C, chunk), s);
    if (chunk & kChunkMfma) {
#define GSC_ACCM(NB, YMV)                                                                          \
    launch_acc_mfma_bin<NB, YMV>(views, n_views, n_tiles, ranges, pair_vals, rec0, rec1, rec2, bin, \
                                 targets, C, per_view, bp, VS, counter, gcount, queues, order, s)
        switch (chunk_channels(chunk)) {
            case 1:
                if (tdtype == GSC_BF16) GSC_ACCM(1, 1); else GSC_ACCM(1, 2);
                break;
            case 16: GSC_ACCM(1, 0); break;
            case 32: GSC_ACCM(2, 0); break;
            default: GSC_ACCM(4, 0); break;
        }
#undef GSC_ACCM
        return;
    }
#define GSC_ACC(CCV)                                                                                \
    launch_acc_cc<CCV>(views, n_views, n_tiles, ranges, pair_vals, rec0, rec1, rec2, bin, targets, \
                       tdtype, C, per_view, bp, VS, counter, gcount, queues, order, s, det)
    switch (chunk) {
        case 1: GSC_ACC(1); break;
        case 2: GSC_ACC(2); break;
        case 3: GSC_ACC(3); break;
        case 4: GSC_ACC(4); break;
        case 8: GSC_ACC(8); break;
        default: GSC_ACC(16); break;
    }
#undef GSC_ACC
}

void launch_accumulate_weights(const ViewInfo* views, int n_views, uint32_t n_tiles,
                               const uint2* ranges, const uint32_t* pair_vals,
                               const float4* rec0,
                               const float4* rec1, const uint2* rec2, int bin, bool per_view,
                               BlendParams bp, float* V, unsigned long long* counter, hipStream_t s,
                               const uint32_t* order) {
    if (n_tiles == 0) return;
    const uint32_t n_wt = wave_tiles(n_tiles, bin);
    if (bin == 32)
        launch_acc_k<0, false, 32>(views, n_views, n_wt, ranges, pair_vals, rec0, rec1, rec2, nullptr,
                                   0, per_view, bp, V, counter, nullptr, nullptr, order, s);
    else
        launch_acc_k<0, false, 16>(views, n_views, n_wt, ranges, pair_vals, rec0, rec1, rec2, nullptr,
                                   0, per_view, bp, V, counter, nullptr, nullptr, order, s);
}

}  // namespace gsc
