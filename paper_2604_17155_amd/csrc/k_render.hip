// Render: per-item view colours from SH coefficients, then the same
// front-to-back tile blend as the accumulate pass, writing each pixel's
// blended colour (eq. 2 with the colours of eq. 3).
#include "gsc_internal.h"
#include "sh.h"
#include "wave_ops.h"

namespace gsc {

static inline uint32_t wave_tiles(uint32_t n_bins, int bin) { return bin == 32 ? 4u * n_bins : n_bins; }

// 64 x 64 tiles through LDS: rows read and columns written as contiguous
// runs (the padded row keeps the column reads free of bank conflicts).
__global__ __launch_bounds__(256) void k_transpose(const float* __restrict__ in, int64_t rows, int K,
                                                   float* __restrict__ out) {
    __shared__ float t[64][65];
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int k0 = (int)blockIdx.y * 64;
    const int tx = (int)(threadIdx.x & 63), ty = (int)(threadIdx.x >> 6);
    for (int j = ty; j < 64; j += 4) {
        const int64_t r = r0 + j;
        const int k = k0 + tx;
        t[j][tx] = (r < rows && k < K) ? in[r * K + k] : 0.0f;
    }
    __syncthreads();
    for (int j = ty; j < 64; j += 4) {
        const int k = k0 + j;
        const int64_t r = r0 + tx;
        if (k < K && r < rows) out[(int64_t)k * rows + r] = t[tx][j];
    }
}

void launch_transpose(const float* in, int64_t rows, int K, float* out, hipStream_t s) {
    if (rows <= 0 || K <= 0) return;
    dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((K + 63) / 64)), block(256);
    hipLaunchKernelGGL(k_transpose, grid, block, 0, s, in, rows, K, out);
}

// gamma[i*C + c] = sum_m coeffs[g][m][c] * phi_m(dir_gv) for batch item i
// (view v, Gaussian g): items in their own order, reading the transposed
// coefficients, so that consecutive threads read consecutive floats.
template <int L>
__global__ void k_view_colors(const ViewInfo* __restrict__ views, int n_views, uint32_t n_items,
                              const float* __restrict__ means, const float* __restrict__ coeffs_t,
                              int64_t ldn, int C, float* __restrict__ gamma) {
    constexpr int NB = (L + 1) * (L + 1);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const ViewInfo& V = views[find_view_item(views, n_views, i)];
    const int64_t g = V.g_offset + (int64_t)(i - V.item_base);
    double dx = (double)means[3 * g] - V.centre[0];
    double dy = (double)means[3 * g + 1] - V.centre[1];
    double dz = (double)means[3 * g + 2] - V.centre[2];
    double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    float phi[NB];
    sh_eval<float, L>((float)(dx * inv), (float)(dy * inv), (float)(dz * inv), phi);
    const float* cg = coeffs_t + g;
    float* out = gamma + (int64_t)i * C;
    for (int c = 0; c < C; ++c) {
        float a = 0.0f;
#pragma unroll
        for (int m = 0; m < NB; ++m) a += cg[(int64_t)(m * C + c) * ldn] * phi[m];
        out[c] = a;
    }
}

void launch_view_colors(const ViewInfo* views, int n_views, uint32_t n_items, const float* means,
                        const float* coeffs_t, int64_t ldn, int C, int sh_deg, float* gamma,
                        hipStream_t s) {
    if (n_items == 0 || n_views <= 0) return;
    dim3 grid((n_items + 255) / 256), block(256);
#define GSC_VC(LL)                                                                                   \
    hipLaunchKernelGGL(k_view_colors<LL>, grid, block, 0, s, views, n_views, n_items, means, coeffs_t, \
                       ldn, C, gamma)
    switch (sh_deg) {
        case 0: GSC_VC(0); break;
        case 1: GSC_VC(1); break;
        case 2: GSC_VC(2); break;
        default: GSC_VC(3); break;
    }
#undef GSC_VC
}

// images[row][c] = sum_g w_gp * gamma_gv[c]; every pixel of every tile is
// written.  Same tile walk and blend decisions as accumulate_tile.
template <int CC, int BIN>
__global__ __launch_bounds__(256) void k_render(
    const ViewInfo* __restrict__ views, int n_views, uint32_t n_wt, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ pair_vals, const float4* __restrict__ rec0,
    const float4* __restrict__ rec1, const uint2* __restrict__ rec2,
    const float* __restrict__ gamma, int C, int c_off, BlendParams bp, float* __restrict__ images,
    unsigned long long* __restrict__ counter, const uint32_t* __restrict__ order) {
    static_assert(CC <= 4, "one float4 of colours per entry");
    // the chunk's records and colours, read back by every lane as broadcasts
    __shared__ float4 srec1[4][64];
    __shared__ float4 scol[4][64];
    __shared__ float2 srec0[4][64];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t wi = xcd_block(blockIdx.x, gridDim.x) * 4 + w;
    if (wi >= n_wt) return;
    const uint32_t wt = queued_tile<BIN>(wi, order);  // blocks start in index order
    const TileGeom tg = tile_geom<BIN>(wt, views, n_views);
    const ViewInfo& V = views[tg.vloc];
    const int ix = tg.x0 + (int)(lane & 15);
    const int iy0 = tg.y0 + (int)(lane >> 4);
    float T[4];
    bool inside[4];
    float img[4][CC];
    uint32_t alive = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        inside[k] = ix < V.width && iy0 + 4 * k < V.height;
        T[k] = inside[k] ? 1.0f : kOutsideT;
        alive |= (__builtin_amdgcn_ballot_w64(inside[k]) != 0 ? 1u : 0u) << k;
#pragma unroll
        for (int c = 0; c < CC; ++c) img[k][c] = 0.0f;
    }
    alive = (uint32_t)__builtin_amdgcn_readfirstlane((int)alive);
    uint2 rg = ranges[tg.bin];
    rg.x = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.x);
    rg.y = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.y);
    uint32_t cnt = 0;
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
    // A chunk of 64 entries is gathered at once, one entry per lane (records
    // and the item's colours), and staged in LDS, from which an entry reads
    // them back with broadcast loads; each lane forms its entry's band mask,
    // and only entries reaching a band with a live pixel are visited.
    for (uint32_t b = rg.x; b < rg.y && alive != 0u; b += 64) {
        const uint32_t nb = min(64u, rg.y - b);
        const bool own = lane < nb;
        const uint32_t pv = own ? pair_vals[b + lane] : 0u;
        const uint32_t it = pv & kItemMask;
        const float4 r = own ? rec0[it] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float2 R0 = make_float2((ox - r.x) - r.z, (oy - r.y) - r.w);
        const float4 R1 = own ? rec1[it] : make_float4(0.f, 0.f, 0.f, 0.f);
        const uint2 R2 = own ? rec2[it] : make_uint2(0u, 0u);
        const float* gl = gamma + (int64_t)R2.y * C + c_off;  // the record names the item
        float RC[CC];
#pragma unroll
        for (int c = 0; c < CC; ++c) RC[c] = (own && c_off + c < C) ? gl[c] : 0.0f;
        const uint32_t BL = own ? (entry_bands<BIN>(pv, tg.quad, R2.x, tg.y0) & alive) : 0u;
        uint64_t todo = __builtin_amdgcn_ballot_w64(BL != 0u);
        srec1[w][lane] = R1;
        srec0[w][lane] = R0;
        scol[w][lane] = make_float4(RC[0], CC > 1 ? RC[CC > 1 ? 1 : 0] : 0.0f, CC > 2 ? RC[CC > 2 ? 2 : 0] : 0.0f,
                                    CC > 3 ? RC[CC > 3 ? 3 : 0] : 0.0f);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        while (todo != 0u) {
            const uint32_t j = (uint32_t)__builtin_ctzll(todo);
            todo &= todo - 1u;
            const uint32_t bands = bcast_u(BL, j) & alive;
            if (bands == 0u) continue;
            const float2 c0 = srec0[w][j];
            const float4 c1 = srec1[w][j];
            const float4 c4 = scol[w][j];
            const float col[4] = {c4.x, c4.y, c4.z, c4.w};
            const float dx = c0.x + lx;
            const float a0 = c1.x * dx * dx;
            const float b0 = c1.y * dx;
            uint32_t nh = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (!((bands >> k) & 1u)) continue;
                const float dy = c0.y + lyk[k];
                const float q2 = fmaf(dy, fmaf(c1.z, dy, b0), a0);
                uint64_t taken, kept;
                const float w = pixel_step(q2, c1.w, T[k], qlim, amin, amax, tmin, taken, kept);
#pragma unroll
                for (int c = 0; c < CC; ++c) img[k][c] = fmaf(w, col[c], img[k][c]);
                nh += (uint32_t)__popcll(taken);
                if (kept == 0) alive &= ~(1u << k);
            }
            alive = (uint32_t)__builtin_amdgcn_readfirstlane((int)alive);
            cnt += (uint32_t)__builtin_amdgcn_readfirstlane((int)nh);
            if (alive == 0u) break;
        }
        __builtin_amdgcn_wave_barrier();  // the next chunk overwrites the records
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!inside[k]) continue;
        int64_t row = V.pixel_offset + (int64_t)(iy0 + 4 * k) * V.width + ix;
#pragma unroll
        for (int c = 0; c < CC; ++c)
            if (c_off + c < C) images[row * C + c_off + c] = img[k][c];
    }
    if (c_off == 0 && lane == 0 && cnt) atomicAdd(counter, (unsigned long long)cnt);
}

void launch_render(const ViewInfo* views, int n_views, uint32_t n_tiles, const uint2* ranges,
                   const uint32_t* pair_vals, const float4* rec0, const float4* rec1,
                   const uint2* rec2, int bin, const float* gamma, int C, BlendParams bp,
                   float* images, unsigned long long* counter, hipStream_t s, const uint32_t* order) {
    if (n_tiles == 0) return;
    const uint32_t n_wt = wave_tiles(n_tiles, bin);
    dim3 grid((n_wt + 3) / 4), block(256);
#define GSC_RENDER(CCV, BINV)                                                                     \
    hipLaunchKernelGGL((k_render<CCV, BINV>), grid, block, 0, s, views, n_views, n_wt, ranges,    \
                       pair_vals, rec0, rec1, rec2, gamma, C, c_off, bp, images, counter, order)
    for (int c_off = 0; c_off < C; c_off += 4) {
        const bool three = C <= 3 && c_off == 0;
        if (bin == 32) {
            if (three) GSC_RENDER(3, 32); else GSC_RENDER(4, 32);
        } else {
            if (three) GSC_RENDER(3, 16); else GSC_RENDER(4, 16);
        }
    }
#undef GSC_RENDER
}

}  // namespace gsc
