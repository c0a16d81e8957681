// Backward pass: hand-written adjoints of colorize and render with respect to
// the target pixels and the opacities.
//
// Colorize.  The coefficients solve (A_g + w_g Lambda) c_g = B_g (eq. 14), so
// for an upstream gradient dL/dc_g and Bbar_g = (A_g + w_g Lambda)^{-1} dL/dc_g
//   dL = sum_g <Bbar_g, dB_g - dA_g c_g - dw_g Lambda c_g>.
// B_g, A_g and w_g are sums over contributions of w*phi*y^T, w*phi*phi^T and w
// (eqs. 10-13), hence
//   dL/dy_p  = sum_g w_gp beta_gj            beta_gj  = Bbar_g^T phi_gj
//   dL/dw_gp = beta^T y_p - delta_gj        delta_gj = beta^T gamma + rho_g
// with gamma_gj = c_g^T phi_gj and rho_g = sum_{m,c} lambda_m Bbar[m][c] c[m][c].
// Render (eqs. 1-3).  images_p = sum_g w_gp gamma_gj, so for dL/dimages_p
//   dL/dc_g  = sum_{j,p} phi_gj w_gp (dL/dimages_p)^T
//   dL/dw_gp = gamma^T (dL/dimages_p)        (beta = gamma, delta = 0).
// Both then go through the adjoint of the front-to-back blend (eq. 2):
// w_k = alpha_k T_k with T_k = prod_{i<k} (1 - alpha_i) over accepted entries, so
//   dL/dalpha_k = u_k T_k - (1 - alpha_k)^{-1} sum_{i>k} u_i w_i,  u = dL/dw,
// and alpha = min(alpha_max, o G) gives dalpha/do = G unless clamped.  The
// skip, footprint and stop decisions are piecewise constant and carry no
// derivative.
//
// The weights are recomputed, never stored: one tile pass forms per pixel the
// total S = sum_k u_k w_k (and dL/dy), a second identical pass forms the
// running prefix P_k, so that the suffix sum is S - P_k.  S and P are kept in
// FP64, which keeps the suffix accurate deep into the pixel where it is many
// orders below S.
#include "gsc_internal.h"
#include "sh.h"
#include "wave_ops.h"

namespace gsc {

// beta[i*(C+1) + c] = beta_gj[c] and [.. + C] = delta_gj for batch item i
// (view v, Gaussian g), items in their own order; the coefficient arrays are
// transposed ([m * C + c][g], rows of ldn floats) so that consecutive threads
// read consecutive floats.
template <int L, bool RENDER>
__global__ void k_view_adjoint(const ViewInfo* __restrict__ views, int n_views, uint32_t n_items,
                               const float* __restrict__ means, const float* __restrict__ coeffs_t,
                               const float* __restrict__ bbar_t, int64_t ldn,
                               const float* __restrict__ rho, int C, float* __restrict__ beta) {
    constexpr int NB = (L + 1) * (L + 1);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const ViewInfo& V = views[find_view_item(views, n_views, i)];
    const int64_t g = V.g_offset + (int64_t)(i - V.item_base);
    const double dx = (double)means[3 * g] - V.centre[0];
    const double dy = (double)means[3 * g + 1] - V.centre[1];
    const double dz = (double)means[3 * g + 2] - V.centre[2];
    const double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    float phi[NB];
    sh_eval<float, L>((float)(dx * inv), (float)(dy * inv), (float)(dz * inv), phi);
    const float* cg = coeffs_t + g;
    float* out = beta + (int64_t)i * (C + 1);
    if constexpr (RENDER) {
        for (int c = 0; c < C; ++c) {
            float a = 0.0f;
#pragma unroll
            for (int m = 0; m < NB; ++m) a = fmaf(cg[(int64_t)(m * C + c) * ldn], phi[m], a);
            out[c] = a;
        }
        out[C] = 0.0f;
    } else {
        const float* bg = bbar_t + g;
        double delta = (double)rho[g];
        for (int c = 0; c < C; ++c) {
            float a = 0.0f, b = 0.0f;
#pragma unroll
            for (int m = 0; m < NB; ++m) {
                const int64_t k = (int64_t)(m * C + c) * ldn;
                a = fmaf(cg[k], phi[m], a);
                b = fmaf(bg[k], phi[m], b);
            }
            out[c] = b;
            delta += (double)a * (double)b;
        }
        out[C] = (float)delta;
    }
}

void launch_view_adjoint(const ViewInfo* views, int n_views, uint32_t n_items, const float* means,
                         const float* coeffs_t, const float* bbar_t, int64_t ldn, const float* rho,
                         int C, int sh_deg, bool render, float* beta, hipStream_t s) {
    if (n_items == 0 || n_views <= 0) return;
    dim3 grid((n_items + 255) / 256), block(256);
#define GSC_VA(LL)                                                                                   \
    do {                                                                                             \
        if (render)                                                                                  \
            hipLaunchKernelGGL((k_view_adjoint<LL, true>), grid, block, 0, s, views, n_views,        \
                               n_items, means, coeffs_t, bbar_t, ldn, rho, C, beta);                 \
        else                                                                                         \
            hipLaunchKernelGGL((k_view_adjoint<LL, false>), grid, block, 0, s, views, n_views,       \
                               n_items, means, coeffs_t, bbar_t, ldn, rho, C, beta);                 \
    } while (0)
    switch (sh_deg) {
        case 0: GSC_VA(0); break;
        case 1: GSC_VA(1); break;
        case 2: GSC_VA(2); break;
        default: GSC_VA(3); break;
    }
#undef GSC_VA
}

namespace {

// One front-to-back step of one pixel (the decisions of the forward blend).
struct Step {
    float w;      // accepted weight alpha*T (0 if not accepted)
    float alpha;  // alpha of the entry
    float G;      // exp(-q/2)
    float Tb;     // transmittance before the entry
    bool take;
};

__device__ __forceinline__ Step blend_step(float& T, bool& live, float q2, float opac,
                                           float qlim, const BlendParams& bp) {
    Step st;
    st.G = __builtin_amdgcn_exp2f(q2);
    st.alpha = fminf(bp.alpha_max, opac * st.G);
    const float test = fmaf(-T, st.alpha, T);
    const bool cand = live && q2 >= qlim && st.alpha >= bp.alpha_min;
    const bool stop = cand && test < bp.t_min;
    st.take = cand && !stop;
    live = live && !stop;
    st.Tb = T;
    st.w = st.take ? st.alpha * T : 0.0f;
    T = st.take ? test : T;
    return st;
}

}  // namespace

// CC: channels of this launch (chunk [c_off, c_off + CC) of C).  dL/dw is
// linear in the channels, so chunk launches add their shares of dL/do; the
// first chunk also carries -delta.
// The forms of up to three channels are held to seven waves per SIMD (72
// registers), as the forward accumulate.
template <int CC>
constexpr int adj_waves_per_simd() { return CC >= 1 && CC <= 3 ? 7 : 1; }

template <int CC, bool BF16, bool GY, int BIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(adj_waves_per_simd<CC>()))) void k_blend_adjoint(
    const ViewInfo* __restrict__ views, int n_views, uint32_t n_wt, const uint2* __restrict__ ranges,
    const uint32_t* __restrict__ pair_vals,
    const float4* __restrict__ rec0, const float4* __restrict__ rec1,
    const uint2* __restrict__ rec2, const void* __restrict__ ypix, int C, int c_off,
    const float* __restrict__ beta, BlendParams bp, float* __restrict__ grad_y,
    float* __restrict__ grad_o, const uint32_t* __restrict__ order) {
    // the chunk's records and, for up to three channels, the entry's adjoint
    // colours and offset, read back by every lane as broadcasts
    constexpr bool kLdsB = CC <= 3;
    __shared__ float4 srec1[4][64];
    __shared__ float4 sbet[4][kLdsB ? 64 : 1];
    __shared__ float2 srec0[4][64];
    const uint32_t lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t wi = xcd_block(blockIdx.x, gridDim.x) * 4 + w;
    if (wi >= n_wt) return;  // whole wave
    const uint32_t wt = queued_tile<BIN>(wi, order);  // blocks start in index order
    const TileGeom tg = tile_geom<BIN>(wt, views, n_views);
    const ViewInfo& V = views[tg.vloc];
    const int ix = tg.x0 + (int)(lane & 15);
    const int iy0 = tg.y0 + (int)(lane >> 4);
    const int stride = C + 1;
    const bool first_chunk = c_off == 0;
    // dL/do of an entry goes to Gaussian g_offset + (item - item_base), the
    // item being named by the entry's record
    const int64_t g_shift = V.g_offset - (int64_t)V.item_base;
    // loop constants in vector registers (see uniform_in_vgpr)
    const float qlim = uniform_in_vgpr((float)(kExp2Scale * (double)bp.cut2));
    BlendParams bpv = bp;
    bpv.alpha_max = uniform_in_vgpr(bp.alpha_max);
    bpv.alpha_min = uniform_in_vgpr(bp.alpha_min);
    bpv.t_min = uniform_in_vgpr(bp.t_min);

    bool inside[4];
    float yv[4][CC];  // pixel values (read only when dL/do is wanted)
    // the lane's pixel offsets from the tile's centre point; R0 below keeps,
    // per entry, the offset of that point from the projected centre
    const float lx = tile_offset_col(lane);
    float lyk[4];
    const float ox = tile_centre(tg.x0), oy = tile_centre(tg.y0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int iy = iy0 + 4 * k;
        inside[k] = ix < V.width && iy < V.height;
        lyk[k] = tile_offset_row(lane, k);
        const int64_t row = V.pixel_offset + (int64_t)iy * V.width + ix;
#pragma unroll
        for (int c = 0; c < CC; ++c)
            yv[k][c] = (inside[k] && grad_o && c_off + c < C) ? load_target<BF16>(ypix, row * C + c_off + c) : 0.0f;
    }
    uint2 rg = ranges[tg.bin];
    rg.x = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.x);
    rg.y = (uint32_t)__builtin_amdgcn_readfirstlane((int)rg.y);

    // Both passes walk the list the same way, so that they take the same
    // decisions.  A chunk of 64 entries is gathered at once, one entry per
    // lane (records and the entry's adjoint colours), and staged in LDS, from
    // which an entry reads them back with broadcast loads (adjoint colours of
    // wider chunks by readlane); each lane forms its entry's band mask, and
    // only entries reaching a band with a live pixel are visited.  A
    // pixel that stopped adds nothing in either pass, so the skipped entries
    // and bands change no sum.
    uint32_t alive0 = 0;  // bands holding a pixel of the image
#pragma unroll
    for (int k = 0; k < 4; ++k) alive0 |= (__builtin_amdgcn_ballot_w64(inside[k]) != 0 ? 1u : 0u) << k;
    alive0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)alive0);
    float T[4];
    bool live[4];
    auto walk = [&](auto&& body) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            T[k] = 1.0f;
            live[k] = inside[k];
        }
        uint32_t alive = alive0;
        for (uint32_t b = rg.x; b < rg.y && alive != 0u; b += 64) {
            const uint32_t nb = min(64u, rg.y - b);
            const bool own = lane < nb;
            const uint32_t pv = own ? pair_vals[b + lane] : 0u;
            const uint32_t it = pv & kItemMask;
            const float4 r = own ? rec0[it] : make_float4(0.f, 0.f, 0.f, 0.f);
            const float2 R0 = make_float2((ox - r.x) - r.z, (oy - r.y) - r.w);
            const float4 R1 = own ? rec1[it] : make_float4(0.f, 0.f, 0.f, 0.f);
            const uint2 R2 = own ? rec2[it] : make_uint2(0u, 0u);
            const float* bl = beta + (int64_t)R2.y * stride;  // the record names the item
            float RB[CC];
#pragma unroll
            for (int c = 0; c < CC; ++c) RB[c] = (own && c_off + c < C) ? bl[c_off + c] : 0.0f;
            const float RD = (own && first_chunk) ? bl[C] : 0.0f;
            const uint32_t BL = own ? (entry_bands<BIN>(pv, tg.quad, R2.x, tg.y0) & alive) : 0u;
            uint64_t todo = __builtin_amdgcn_ballot_w64(BL != 0u);
            srec1[w][lane] = R1;
            srec0[w][lane] = R0;
            if constexpr (kLdsB)
                sbet[w][lane] = make_float4(RB[0], CC > 1 ? RB[CC > 1 ? 1 : 0] : 0.0f,
                                            CC > 2 ? RB[CC > 2 ? 2 : 0] : 0.0f, RD);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            while (todo != 0u) {
                const uint32_t j = (uint32_t)__builtin_ctzll(todo);
                todo &= todo - 1u;
                const uint32_t bands = bcast_u(BL, j) & alive;
                if (bands == 0u) continue;
                const uint2 e2 = make_uint2(0u, bcast_u(R2.y, j));  // the item
                const float2 c0 = srec0[w][j];
                const float4 c1 = srec1[w][j];
                float bet[CC];
                float del;
                if constexpr (kLdsB) {
                    const float4 b4 = sbet[w][kLdsB ? j : 0];
                    const float bb[3] = {b4.x, b4.y, b4.z};
#pragma unroll
                    for (int c = 0; c < CC; ++c) bet[c] = bb[c < 3 ? c : 0];
                    del = b4.w;
                } else {
#pragma unroll
                    for (int c = 0; c < CC; ++c) bet[c] = bcast(RB[c], j);
                    del = bcast(RD, j);
                }
                body(bands, c0, c1, e2, bet, del);
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if (((bands >> k) & 1u) && __builtin_amdgcn_ballot_w64(live[k]) == 0) alive &= ~(1u << k);
                alive = (uint32_t)__builtin_amdgcn_readfirstlane((int)alive);
                if (alive == 0u) break;
            }
            __builtin_amdgcn_wave_barrier();  // the next chunk overwrites the records
        }
    };

    // ---- pass 1: S = sum_k u_k w_k per pixel, and dL/dy -------------------
    double S[4];
    float gy[4][GY ? CC : 1];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        S[k] = 0.0;
#pragma unroll
        for (int c = 0; c < (GY ? CC : 1); ++c) gy[k][c] = 0.0f;
    }
    walk([&](uint32_t bands, const float2& c0, const float4& c1, const uint2& e2, const float (&bet)[CC],
             float del) {
        const float dx = c0.x + lx;
        const float a0 = c1.x * dx * dx;
        const float b0 = c1.y * dx;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!((bands >> k) & 1u)) continue;  // uniform
            const float dy = c0.y + lyk[k];
            const float q2 = fmaf(dy, fmaf(c1.z, dy, b0), a0);
            const Step st = blend_step(T[k], live[k], q2, c1.w, qlim, bpv);
            float u = -del;
#pragma unroll
            for (int c = 0; c < CC; ++c) u = fmaf(bet[c], yv[k][c], u);
            S[k] += (double)(st.w * u);
            if constexpr (GY) {
#pragma unroll
                for (int c = 0; c < CC; ++c) gy[k][c] = fmaf(st.w, bet[c], gy[k][c]);
            }
        }
    });
    if constexpr (GY) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!inside[k]) continue;
            const int64_t row = V.pixel_offset + (int64_t)(iy0 + 4 * k) * V.width + ix;
#pragma unroll
            for (int c = 0; c < CC; ++c)
                if (c_off + c < C) grad_y[row * C + c_off + c] = gy[k][c];
        }
    }
    if (grad_o == nullptr) return;

    // ---- pass 2: dL/dalpha per entry, reduced to dL/do per Gaussian -------
    double P[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) P[k] = 0.0;
    walk([&](uint32_t bands, const float2& c0, const float4& c1, const uint2& e2, const float (&bet)[CC],
             float del) {
        const float dx = c0.x + lx;
        const float a0 = c1.x * dx * dx;
        const float b0 = c1.y * dx;
        float go = 0.0f;
        uint32_t any = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (!((bands >> k) & 1u)) continue;  // uniform
            const float dy = c0.y + lyk[k];
            const float q2 = fmaf(dy, fmaf(c1.z, dy, b0), a0);
            const Step st = blend_step(T[k], live[k], q2, c1.w, qlim, bpv);
            float u = -del;
#pragma unroll
            for (int c = 0; c < CC; ++c) u = fmaf(bet[c], yv[k][c], u);
            P[k] += (double)(st.w * u);
            const float suffix = (float)(S[k] - P[k]);
            const float dal = u * st.Tb - suffix / (1.0f - st.alpha);
            const bool clamped = c1.w * st.G >= bp.alpha_max;
            go += (st.take && !clamped) ? dal * st.G : 0.0f;
            any |= st.take ? 1u : 0u;
        }
        if (__ballot(any != 0) != 0) {
            const float t = wave_sum(go);
            if (lane == 0) unsafeAtomicAdd(grad_o + ((int64_t)e2.y + g_shift), t);
        }
    });
}

template <int CC, bool GY>
static void launch_badj_cc(const ViewInfo* views, int n_views, uint32_t n_bins, const uint2* ranges,
                           const uint32_t* pair_vals, const float4* rec0,
                           const float4* rec1, const uint2* rec2, int bin, const void* ypix,
                           int ydtype, int C, const float* beta, BlendParams bp, float* grad_y,
                           float* grad_o, const uint32_t* order, hipStream_t s) {
    const uint32_t n_wt = bin == 32 ? 4u * n_bins : n_bins;
    dim3 grid((n_wt + 3) / 4), block(256);
#define GSC_BADJ(BFV, BINV)                                                                         \
    hipLaunchKernelGGL((k_blend_adjoint<CC, BFV, GY, BINV>), grid, block, 0, s, views, n_views, n_wt, \
                       ranges, pair_vals, rec0, rec1, rec2, ypix, C, c_off, beta, bp, grad_y, grad_o, order)
    for (int c_off = 0; c_off < C; c_off += CC) {
        const bool bf = ydtype == GSC_BF16;
        if (bin == 32) {
            if (bf) GSC_BADJ(true, 32); else GSC_BADJ(false, 32);
        } else {
            if (bf) GSC_BADJ(true, 16); else GSC_BADJ(false, 16);
        }
    }
#undef GSC_BADJ
}

template <bool GY>
static void launch_badj(const ViewInfo* views, int n_views, uint32_t n_tiles, const uint2* ranges,
                        const uint32_t* pair_vals, const float4* rec0,
                        const float4* rec1,
                        const uint2* rec2, int bin, const void* ypix, int ydtype, int C,
                        const float* beta, BlendParams bp, float* grad_y, float* grad_o,
                        const uint32_t* order, hipStream_t s) {
#define GSC_BA(CCV)                                                                                \
    launch_badj_cc<CCV, GY>(views, n_views, n_tiles, ranges, pair_vals, rec0, rec1, rec2, bin, ypix, \
                            ydtype, C, beta, bp, grad_y, grad_o, order, s)
    switch (accumulate_chunk(C, GSC_F32)) {  // vector-lane channel chunks
        case 1: GSC_BA(1); break;
        case 2: GSC_BA(2); break;
        case 3: GSC_BA(3); break;
        case 4: GSC_BA(4); break;
        case 8: GSC_BA(8); break;
        default: GSC_BA(16); break;
    }
#undef GSC_BA
}

void launch_blend_adjoint(const ViewInfo* views, int n_views, uint32_t n_tiles, const uint2* ranges,
                          const uint32_t* pair_vals, const float4* rec0,
                          const float4* rec1,
                          const uint2* rec2, int bin, const void* ypix, int ydtype, int C,
                          const float* beta, BlendParams bp, float* grad_y, float* grad_o,
                          hipStream_t s, const uint32_t* order) {
    if (n_tiles == 0 || (!grad_y && !grad_o)) return;
    if (grad_y)
        launch_badj<true>(views, n_views, n_tiles, ranges, pair_vals, rec0, rec1, rec2, bin, ypix,
                          ydtype, C, beta, bp, grad_y, grad_o, order, s);
    else
        launch_badj<false>(views, n_views, n_tiles, ranges, pair_vals, rec0, rec1, rec2, bin, ypix,
                           ydtype, C, beta, bp, grad_y, grad_o, order, s);
}

// grad_coeffs[g][m][c] = sum_j phi_gj[m] S_gj[c] from the per-view sums
// VS[j][g] = (V_gj, S_gj[0..C)) (per_view), or phi = Y0 and one summed slot
// per Gaussian (L = 0).  One thread per (Gaussian, CH channels); FP64 sums.
template <int L>
constexpr int fold_rhs_channels() { return L >= 3 ? 2 : 4; }

template <int L>
__global__ void k_fold_rhs(const ViewInfo* __restrict__ views, int n_views,
                           const float* __restrict__ means, const float* __restrict__ VS,
                           int per_view, int64_t N, int C, float* __restrict__ out) {
    constexpr int NB = (L + 1) * (L + 1);
    constexpr int CH = fold_rhs_channels<L>();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c0 = blockIdx.y * CH;
    if (g >= N) return;
    const int stride = C + 1;
    double acc[NB][CH];
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
        for (int c = 0; c < CH; ++c) acc[m][c] = 0.0;
    const int nv = per_view ? n_views : 1;
    const float mx = means[3 * g], my = means[3 * g + 1], mz = means[3 * g + 2];
    for (int v = 0; v < nv; ++v) {
        const float* slot = VS + ((per_view ? views[v].vs_base : 0) + g) * stride;
        if (slot[0] == 0.0f) continue;  // no contribution in this view
        float phi[NB];
        if (per_view) {
            const ViewInfo& Vw = views[v];
            const float dx = mx - (float)Vw.centre[0], dy = my - (float)Vw.centre[1],
                        dz = mz - (float)Vw.centre[2];
            const float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
            sh_eval<float, L>(dx * inv, dy * inv, dz * inv, phi);
        } else {
            sh_eval<float, L>(0.0f, 0.0f, 1.0f, phi);
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const double sc = (c0 + c < C) ? (double)slot[1 + c0 + c] : 0.0;
#pragma unroll
            for (int m = 0; m < NB; ++m) acc[m][c] = fma((double)phi[m], sc, acc[m][c]);
        }
    }
#pragma unroll
    for (int m = 0; m < NB; ++m)
#pragma unroll
        for (int c = 0; c < CH; ++c)
            if (c0 + c < C) out[(g * NB + m) * C + c0 + c] = (float)acc[m][c];
}

template <int L>
static void launch_fold_rhs_l(const ViewInfo* views, int n_views, const float* means, const float* VS,
                              bool per_view, int64_t N, int C, float* out, hipStream_t s) {
    constexpr int CH = fold_rhs_channels<L>();
    dim3 grid((unsigned)((N + 127) / 128), (unsigned)((C + CH - 1) / CH)), block(128);
    hipLaunchKernelGGL(k_fold_rhs<L>, grid, block, 0, s, views, n_views, means, VS, (int)per_view, N, C, out);
}

void launch_fold_rhs(const ViewInfo* views, int n_views, const float* means, const float* VS,
                     bool per_view, int64_t N, int C, int sh_deg, float* out, hipStream_t s) {
    if (N <= 0) return;
    switch (sh_deg) {
        case 0: launch_fold_rhs_l<0>(views, n_views, means, VS, per_view, N, C, out, s); break;
        case 1: launch_fold_rhs_l<1>(views, n_views, means, VS, per_view, N, C, out, s); break;
        case 2: launch_fold_rhs_l<2>(views, n_views, means, VS, per_view, N, C, out, s); break;
        default: launch_fold_rhs_l<3>(views, n_views, means, VS, per_view, N, C, out, s); break;
    }
}

}  // namespace gsc
