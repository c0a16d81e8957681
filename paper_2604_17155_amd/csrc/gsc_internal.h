// Internal declarations shared by the HIP translation units of libgsc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gsc.h"

namespace gsc {

constexpr int kTile = 16;           // tile edge in pixels (16x16 = one wave, 4 pixels per lane)
constexpr int kTileShift = 4;
// Binning granularity: 16 (a bin is one tile) or 32 (a bin is 2x2 tiles).
constexpr int kMinBin = 16;
constexpr int kMaxBin = 32;
constexpr int kMaxNb = 16;          // (L+1)^2 for L <= 3
constexpr int kMaxC = 64;

// One view as the kernels see it.  A batch of views may mix scenes: each view
// names its scene's Gaussians [g_offset, g_offset + n_gauss) in the
// concatenated arrays.  The (view, Gaussian) items of a batch are numbered
// view by view: item = item_base + local Gaussian index.
struct ViewInfo {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    double centre[3];      // camera centre -R^T t, for the SH view direction
    int32_t width, height;
    int32_t tiles_x, tiles_y;  // bins per row and column
    uint32_t tile_base;    // first global bin id of this view within its batch
    uint32_t item_base;    // first item of this view within its batch
    int64_t pixel_offset;  // first target row
    int64_t g_offset;      // first Gaussian of the view's scene
    int64_t vs_base;       // first per-view sum slot of this view (per-view layouts)
    uint32_t n_gauss;      // Gaussians of the view's scene
    uint32_t scene;        // scene index
    uint32_t uniform_n;    // n_gauss when every view of the batch has the same
                           // count (item = view * n + g), else 0
};

// View of a batch item: a division when every view has the same count,
// else a binary search on item_base (n_views >= 1).
__device__ inline int find_view_item(const ViewInfo* __restrict__ views, int n_views, uint32_t item) {
    const uint32_t un = views[0].uniform_n;
    if (un != 0u) return min((int)(item / un), n_views - 1);
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].item_base <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The same lookup on the views' first items staged in LDS by the block:
// stage_view_bases fills sbase (kViewLds words) when the batch's views differ
// in size and fit, and ends with a block barrier (every thread must call it);
// view_of then searches LDS instead of the view records in global memory.
constexpr int kViewLds = 512;
__device__ inline bool stage_view_bases(const ViewInfo* __restrict__ views, int n_views, uint32_t* sbase) {
    const bool use = views[0].uniform_n == 0u && n_views <= kViewLds;
    if (use)
        for (int v = (int)threadIdx.x; v < n_views; v += (int)blockDim.x) sbase[v] = views[v].item_base;
    __syncthreads();
    return use;
}
__device__ inline int view_of(const ViewInfo* __restrict__ views, int n_views, const uint32_t* sbase,
                              bool staged, uint32_t item) {
    if (!staged) return find_view_item(views, n_views, item);
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sbase[mid] <= item) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Blend constants in the form the kernels use.
struct BlendParams {
    float alpha_min, alpha_max, t_min, cut2, dilation, znear;
};

// Splat record of one (view, Gaussian) item i = v * N + g, two float4:
//   r0 = (u_hi, v_hi, u_lo, v_lo)   projected mean as FP32 hi/lo pairs
//   r1 = (K*cxx, 2*K*cxy, K*cyy, opacity) with the conic (cxx, cxy, cyy) =
//        Sigma_2D^{-1} pre-scaled by K = -log2(e)/2, so that
//        q2 = K*q = r1.x dx^2 + r1.y dx dy + r1.z dy^2 and exp(-q/2) = exp2(q2).
constexpr double kExp2Scale = -0.72134752044448170368;  // -0.5 * log2(e)

// Bin pairs carry the item index in the low 26 bits and a 4-bit mask above:
// 16-pixel bins: which 16x4 pixel bands (rows 4k..4k+3 of the tile) the
// footprint reaches; 32-pixel bins: which of the bin's four 16x16 tiles
// (bit 2 * row half + column half).  The tile kernels run one wave per
// 16x16 tile: (bin / 16)^2 waves per bin.
constexpr uint32_t kItemBits = 26;
constexpr uint32_t kItemMask = (1u << kItemBits) - 1u;

// ---- kernels launched from gsc_api.hip ----------------------------------
// Per-Gaussian geometry packed for the projection's gathers: one 64-byte
// record geo[g] = float (mean x, y, z, opacity), then double (Sigma xx, xy,
// xz, yy, yz, zz) with Sigma = R(q) diag(s^2) R(q)^T.
constexpr int kGeoStride = 16;  // floats per record
void launch_cov3d(const float* means, const float* opac, const float* scales, const float* quats,
                  float* geo, int64_t N, hipStream_t s);

// out[0] = sum_g mean axis scale, out[1..3] = sum_g mean (device doubles).
void launch_geometry_stats(const float* means, const float* scales, int64_t N, double* out,
                           hipStream_t s);

// Depth keys of the batch items (n_items = sum of n_gauss over the batch's
// views): keys[i] = binary32 depth bits or 0xFFFFFFFF (culled), vals[i] = i.
void launch_depth_keys(const ViewInfo* views, int n_views, uint32_t n_items, const float* means,
                       const float* opac, BlendParams bp, uint32_t* keys, uint32_t* vals,
                       hipStream_t s);

// Projection in depth order: position k handles item i = order[k] (k if order
// is null) and writes counts[k] and, when counts[k] > 0, rec0/rec1[k] and
// rec2[k] = (first | last << 16, i): the pixel rows of the footprint and the
// item (records are only ever read through tile pairs).
void launch_project(const ViewInfo* views, int n_views, uint32_t n_items, const uint32_t* order,
                    const float* geo, BlendParams bp, uint32_t* counts, float4* rec0, float4* rec1,
                    uint2* rec2, int bin, hipStream_t s);

// Pairs of the depth-ordered records: pair values carry the depth rank k.
// Pairs at offsets >= cap are dropped and counted in *overflow (if given).
void launch_emit(const ViewInfo* views, int n_views, const uint32_t* sorted_vals,
                 const uint32_t* offsets, const uint32_t* counts, const float4* rec0,
                 const float4* rec1, BlendParams bp, uint32_t n_items, uint32_t n_tiles,
                 uint32_t* pair_keys, uint32_t* pair_vals, int bin, hipStream_t s,
                 uint32_t cap = 0xFFFFFFFFu, uint32_t* overflow = nullptr);

// Sum of n uint32 counts into *out (u64, must be zeroed).
void launch_sum_u64(const uint32_t* counts, uint32_t n, unsigned long long* out, hipStream_t s);

// Pairs whose key is >= n_tiles are ignored.  n_dev (optional, device): live
// pair count, clamped to n_pairs.
void launch_tile_ranges(const uint32_t* sorted_keys, uint32_t n_pairs, uint32_t n_tiles,
                        uint2* ranges, hipStream_t s, const uint32_t* n_dev = nullptr);

void launch_fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);

// Exclusive scan of n uint32 values; total written to *total (device). Scratch
// must hold scan_scratch_words(n) words.
size_t scan_scratch_words(uint64_t n);
void launch_scan(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* total, uint32_t* scratch,
                 hipStream_t s);

// Stable LSD radix sort of (key, val) on the low `bits` bits of key. The
// result ends in (keys, vals); alt buffers are scratch of the same size.
// n_dev (optional, device): the live count, clamped to n (the capacity the
// launches are sized for); no host synchronisation is needed.
size_t radix_scratch_words(uint32_t n);
// Bins by decreasing octave of their list length (floor log2 of
// ranges[b].y - ranges[b].x + 1; bin order within an octave) at
// work + n_bins.  work holds tile_order_words(n_bins) words.
size_t tile_order_words(uint32_t n_bins);
const uint32_t* launch_tile_order(const uint2* ranges, uint32_t n_bins, uint32_t* work, hipStream_t s);
// Stable LSD radix sort of (key, value) by the low `bits` key bits, 8 per
// pass.  The result lands in keys/vals, except with result_in_alt: then an odd
// pass count leaves it in keys_alt/vals_alt (*result_in_alt = true) instead of
// copying it back.
void radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                uint32_t n, int bits, uint32_t* scratch, hipStream_t s,
                const uint32_t* n_dev = nullptr, bool* result_in_alt = nullptr);

// Accumulate variants ("chunks"): the channels per launch (launches =
// ceil(C / channels)), plus kChunkMfma for the matrix-core forms: BF16
// targets in blocks of 16, 32 or 64 channels per launch, or (kChunkMfma | 1)
// all channels and a ones column packed into one block of 16 (C <= 15 for
// BF16 targets, C <= 7 for FP32 targets, split into BF16 high and low parts).
constexpr int kChunkMfma = 128;
constexpr int kChunkPacked = kChunkMfma | 1;
inline int chunk_channels(int chunk) { return chunk & (kChunkMfma - 1); }
inline int accumulate_launches(int C, int chunk) {
    if (chunk == kChunkPacked) return 1;
    const int ch = chunk_channels(chunk);
    return (C + ch - 1) / ch;
}
// Default variant for C channels of targets of type tdtype.
int accumulate_chunk(int C, int tdtype);
// `requested` if it is a valid variant that applies to C channels of type
// tdtype, else the default.
int resolve_chunk(int requested, int C, int tdtype);

// Accumulate V_gj and S_gj into slot (view.vs_base + g) when per_view, else
// into slot (view.g_offset + g), summed over views; slots hold C+1 floats.
void launch_accumulate(const ViewInfo* views, int n_views, uint32_t n_tiles, const uint2* ranges,
                       const uint32_t* pair_vals, const float4* rec0, const float4* rec1, const uint2* rec2, int bin,
                       const void* targets, int tdtype, int C, bool per_view, BlendParams bp,
                       float* VS, unsigned long long* counter, uint32_t* gcount, hipStream_t s,
                       const uint32_t* order = nullptr);

// As launch_accumulate with accumulate variant `chunk` (1, 2, 3, 4, 8 or 16
// channels per launch, or kChunkMfma | 16, 32 or 64 for BF16 targets;
// anything else picks accumulate_chunk(C, tdtype)).  queues (device, one word per
// channel pass, zeroed here by a fill kernel): persistent launches of
// kPersistentBlocks blocks that take tiles from a counter; nullptr: one
// block per four tiles.  order (device, optional, with queues): the bins in
// the order their tiles are taken (launch_tile_order).
constexpr uint32_t kPersistentBlocks = 2048;  // 8 blocks of 4 waves per CU
bool accumulate_chunk_valid(int chunk, int tdtype);
void launch_accumulate_chunked(const ViewInfo* views, int n_views, uint32_t n_tiles,
                               const uint2* ranges, const uint32_t* pair_vals, const float4* rec0,
                               const float4* rec1, const uint2* rec2, int bin, const void* targets, int tdtype, int C,
                               bool per_view, BlendParams bp, float* VS,
                               unsigned long long* counter, uint32_t* gcount, int chunk,
                               hipStream_t s, uint32_t* queues = nullptr,
                               const uint32_t* order = nullptr, const float2* det = nullptr);
// det (non-null): deterministic form.  VS holds 64-bit fixed-point words
// (zero before the first launch); each tile's share is scaled by det->x
// (visibility column) or det->y (channel columns), powers of two, and added
// with integer atomics.  Vector form only (a matrix-core chunk falls back).

// out[k][r] = in[r][k] (rows x K row-major in, K x rows row-major out).
void launch_transpose(const float* in, int64_t rows, int K, float* out, hipStream_t s);

// Colour of batch item i (view v, Gaussian g):
// gamma[i][c] = sum_m coeffs[g][m][c] phi_m(dir_gv), from the coefficients
// transposed: coeffs_t[m * C + c][g], rows of ldn floats (consecutive items
// read consecutive floats).
void launch_view_colors(const ViewInfo* views, int n_views, uint32_t n_items, const float* means,
                        const float* coeffs_t, int64_t ldn, int C, int sh_deg, float* gamma,
                        hipStream_t s);

void launch_render(const ViewInfo* views, int n_views, uint32_t n_tiles, const uint2* ranges,
                   const uint32_t* pair_vals, const float4* rec0, const float4* rec1, const uint2* rec2, int bin,
                   const float* gamma, int C, BlendParams bp, float* images,
                   unsigned long long* counter, hipStream_t s,
                       const uint32_t* order = nullptr);

// Fold the per-view sums into the regularised normal equations and solve.
// per_view: VS holds [n_views][N][C+1] (else [N][C+1] summed over views).
// wout (optional): w_g = sum_j V_gj.  dc_scratch: N*(C+1) floats, used when
// sh_deg == 0 and per_view.
// factor (optional, sh_deg >= 1): per Gaussian the Cholesky factor of
// A_g + w_g Lambda, packed by rows (row i at i (i + 1) / 2, 1/L_ii on the
// diagonal), then w_g: refine_factor_words(sh_deg) doubles.
// obs_scratch (optional, sh_deg >= 1): fold_obs_words(N) words; then the
// unobserved Gaussians (no view saw them) are written directly and the fold
// runs over an ordered list of the observed ones only.
void launch_fold_solve(const ViewInfo* views, int n_views, const float* means, const float* VS,
                       bool per_view, int64_t N, int C, int sh_deg, const double* lam_nb /*host, nb*/,
                       float kappa_max, float* coeffs, uint8_t* status, float* wout,
                       float* dc_scratch, unsigned int* ill_count, hipStream_t s,
                       double* factor = nullptr, uint32_t* obs_scratch = nullptr);
inline int64_t fold_obs_words(int64_t N) {  // list, block counts, int64 total, flag bytes
    return N + (N + 1023) / 1024 + 4 + (N + 3) / 4;
}
inline int refine_factor_words(int sh_deg) {
    const int nb = (sh_deg + 1) * (sh_deg + 1);
    return nb * (nb + 1) / 2 + 1;
}

// One refinement update (Algorithm 1, step 10): with the per-view sums VS of
// the residual targets (as for launch_fold_solve; per_view when sh_deg >= 1),
//   c_g += (A_g + w_g Lambda)^{-1} (sum_j phi_gj S_gj^T - w_g Lambda c_g)
// using the stored factor (sh_deg >= 1) or w (sh_deg == 0, where the matrix is
// w_g (Y0^2 + lambda_0)).  Gaussians whose status has UNOBSERVED or FAILED
// are left alone.
void launch_refine_update(const ViewInfo* views, int n_views, const float* means, const float* VS,
                          int64_t N, int C, int sh_deg, const double* lam_nb, const double* factor,
                          const float* w, const uint8_t* status, float* coeffs, hipStream_t s);

// Residual targets of the views of a batch, in place: img[row][c] =
// y[row][c] - img[row][c] for every pixel of the n_views views (y float32
// or bfloat16).
void launch_residual(const ViewInfo* views, int n_views, int max_pixels, const void* y, int ydtype,
                     int C, float* img, hipStream_t s);

// Weights-only accumulate: V[slot] += sum_p w (stride 1; slots as in launch_accumulate).
void launch_accumulate_weights(const ViewInfo* views, int n_views, uint32_t n_tiles,
                               const uint2* ranges, const uint32_t* pair_vals, const float4* rec0,
                               const float4* rec1, const uint2* rec2, int bin, bool per_view, BlendParams bp, float* V,
                               unsigned long long* counter, hipStream_t s,
                       const uint32_t* order = nullptr);

// Adjoint solve: bbar = (A_g + w_g Lambda)^{-1} grad_coeffs and
// rho_g = sum lambda_m bbar[m][c] coeffs[m][c].  V holds per-view
// visibilities [n_views][N] (per_view) or their sums [N].  w_scratch: N floats
// (sh_deg == 0 with per_view).
void launch_adjoint_solve(const ViewInfo* views, int n_views, const float* means, const float* V,
                          bool per_view, int64_t N, int C, int sh_deg, const double* lam_nb,
                          const float* grad_coeffs, const float* coeffs, float* bbar, float* rho,
                          float* w_scratch, hipStream_t s);

// Adjoint colours of batch item i: beta [i][C+1] = (beta_gj, delta_gj).
// render: beta = c^T phi, delta = 0.  Otherwise beta = bbar^T phi and
// delta = beta^T (c^T phi) + rho_g.  coeffs_t and bbar_t are transposed as
// for launch_view_colors (rows of ldn floats).
void launch_view_adjoint(const ViewInfo* views, int n_views, uint32_t n_items, const float* means,
                         const float* coeffs_t, const float* bbar_t, int64_t ldn, const float* rho,
                         int C, int sh_deg, bool render, float* beta, hipStream_t s);

// Blend adjoint over the binned tiles: grad_y[row][c] = sum_g w beta (every
// pixel of every view written, if grad_y) and grad_o[g] += dL/do (atomics, if grad_o).
void launch_blend_adjoint(const ViewInfo* views, int n_views, uint32_t n_tiles, const uint2* ranges,
                          const uint32_t* pair_vals, const float4* rec0, const float4* rec1, const uint2* rec2, int bin,
                          const void* ypix, int ydtype, int C, const float* beta, BlendParams bp,
                          float* grad_y, float* grad_o, hipStream_t s,
                       const uint32_t* order = nullptr);

// grad_coeffs[g][m][c] = sum_j phi_gj[m] S_gj[c] from per-view sums [n_views][N][C+1].
void launch_fold_rhs(const ViewInfo* views, int n_views, const float* means, const float* VS,
                     bool per_view, int64_t N, int C, int sh_deg, float* out, hipStream_t s);

// Input checks and the deterministic sums.
// Over n values of dtype GSC_F32 or GSC_BF16 at p: the smallest index of a
// non-finite value (atomicMin into *first_bad, which the caller sets to
// UINT64_MAX) and the largest |value| as binary32 bits (atomicMax into
// *absmax, set to 0 by the caller; NaN counts as larger than infinity).
void launch_scan_values(const void* p, int dtype, int64_t n, unsigned long long* first_bad,
                        uint32_t* absmax, hipStream_t s);
// out[i] = in[i] / scale, scale = 1/inv_v for column 0 of every row of
// `stride` words and 1/inv_s for the others (powers of two).
void launch_det_to_float(const unsigned long long* in, int64_t n, int stride, double inv_v,
                         double inv_s, float* out, hipStream_t s);

// View selection: one bitset per view of the Gaussians it observed
// (bits[v][w], (N + 63) / 64 words per view) from per-view weights V [n_views][N].
void launch_seen_bits(const float* V, int n_views, int64_t N, unsigned long long* bits, hipStream_t s);

// Post-processing.  Linear combination of up to kCombineSets coefficient sets
// per launch: out = filter * sum_k w_k p_k elementwise (filter by channel,
// i mod C, applied when `filter`); with `accumulate` the sum continues from
// out.
constexpr int kCombineSets = 16;
struct CombineArgs {
    const float* p[kCombineSets];
    float w[kCombineSets];
    float f[kMaxC];
    int n;
    int accumulate;
    int filter;
};
void launch_combine(const CombineArgs& a, int64_t n, int C, bool vec4, float* out, hipStream_t s);

// Segmentation filter over coeffs rows of `row` floats: keep[g] (optional),
// the kept indices in increasing order (optional) and their number (device
// int64, optional).  block_scratch: mask_blocks(N) words.
int mask_blocks(int64_t N);
// Exclusive scan in place of n_blocks counts (one block of 1024 threads);
// *total (if non-null) receives the sum.
void launch_block_scan(uint32_t* counts, int n_blocks, int64_t* total, hipStream_t s);
void launch_mask_filter(const float* coeffs, int64_t N, int64_t row, int channel, float thr,
                        const uint8_t* status, uint8_t* keep, int64_t* indices, int64_t* n_kept,
                        uint32_t* block_scratch, hipStream_t s);

}  // namespace gsc
