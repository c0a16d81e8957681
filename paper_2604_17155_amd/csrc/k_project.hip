// Projection, binning and tile ranges (per view x Gaussian).
//
// Gaussian geometry follows the 3DGS renderer the paper builds on (Sec. 3,
// "Differentiable renderer"): Sigma = R(q) diag(s^2) R(q)^T, EWA projection
// Sigma_2D = J W Sigma W^T J^T + dilation*I, a 3-sigma footprint, and the
// front-to-back order of eq. 2 keyed on the camera-space depth of the mean.
#include <algorithm>

#include "gsc_internal.h"

namespace gsc {

// a1: 3D covariance Sigma = R(q) diag(s^2) R(q)^T, evaluated in FP64 (a few
// dozen operations per Gaussian): the projection that consumes it is FP64,
// and a binary32 covariance would be the largest error in the blend's
// footprint and alpha decisions (a thin Gaussian's rounded rotation moves q by
// up to ~1e-5 relative at its 3-sigma edge).  Record layout: float4 (mean,
// opacity), then the six terms xx xy xz yy yz zz as doubles (64 bytes).
__global__ void k_cov3d(const float* __restrict__ means, const float* __restrict__ opac,
                        const float* __restrict__ scales, const float* __restrict__ quats,
                        float* __restrict__ geo, int64_t N) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    double w = quats[4 * g], x = quats[4 * g + 1], y = quats[4 * g + 2], z = quats[4 * g + 3];
    const double inv = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    w *= inv; x *= inv; y *= inv; z *= inv;
    const double R[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                            {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                            {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
    const double s0 = scales[3 * g], s1 = scales[3 * g + 1], s2 = scales[3 * g + 2];
    const double d[3] = {s0 * s0, s1 * s1, s2 * s2};
    double S[6];
    int k = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j)
            S[k++] = R[i][0] * d[0] * R[j][0] + R[i][1] * d[1] * R[j][1] + R[i][2] * d[2] * R[j][2];
    float4* o = reinterpret_cast<float4*>(geo + kGeoStride * g);
    o[0] = make_float4(means[3 * g], means[3 * g + 1], means[3 * g + 2], opac[g]);
    double2* od = reinterpret_cast<double2*>(o + 1);
    od[0] = make_double2(S[0], S[1]);
    od[1] = make_double2(S[2], S[3]);
    od[2] = make_double2(S[4], S[5]);
}

void launch_cov3d(const float* means, const float* opac, const float* scales, const float* quats,
                  float* geo, int64_t N, hipStream_t s) {
    if (N <= 0) return;
    hipLaunchKernelGGL(k_cov3d, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, means, opac,
                       scales, quats, geo, N);
}

// Sums over the Gaussians of the mean axis scale and of the mean position
// (out: 4 doubles, zeroed by the caller), for the automatic bin size.
__global__ __launch_bounds__(256) void k_geometry_stats(const float* __restrict__ means,
                                                        const float* __restrict__ scales, int64_t N,
                                                        double* __restrict__ out) {
    __shared__ double part[4][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < N;
         g += (int64_t)gridDim.x * blockDim.x) {
        acc[0] += (double)(scales[3 * g] + scales[3 * g + 1] + scales[3 * g + 2]) * (1.0 / 3.0);
        for (int k = 0; k < 3; ++k) acc[1 + k] += (double)means[3 * g + k];
    }
    for (int k = 0; k < 4; ++k)
        for (int d = 32; d >= 1; d >>= 1) acc[k] += __shfl_xor(acc[k], d, 64);
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 4; ++k) part[threadIdx.x >> 6][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        unsafeAtomicAdd(out + k, part[0][k] + part[1][k] + part[2][k] + part[3][k]);
    }
}

void launch_geometry_stats(const float* means, const float* scales, int64_t N, double* out,
                           hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t*>(out), 0u, 8, s);
    if (N <= 0) return;
    const int64_t blocks = std::min<int64_t>((N + 255) / 256, 1024);
    hipLaunchKernelGGL(k_geometry_stats, dim3((unsigned)blocks), dim3(256), 0, s, means, scales, N, out);
}

// Largest q at which a pixel can still pass both the footprint test
// (q <= cut2) and the alpha floor (o exp(-q/2) >= alpha_min), with a margin
// covering the FP32 evaluation in the blend; negative when nothing passes.
__device__ inline float reach_q(float o, const BlendParams& bp) {
    if (!(o >= bp.alpha_min)) return -1.0f;
    const float qa = 2.0f * __logf(o / bp.alpha_min);
    const float q = fminf(bp.cut2, qa);
    return q * (1.0f + 1e-4f) + 1e-3f;
}

// Walks a record's footprint {q <= qmax} band by band (four pixel rows) and
// calls visit(ty, lo, hi) once per 16-row tile row, where [lo[k], hi[k]] is a
// range of 16-column blocks covering every pixel centre of band k (rows
// 4k..4k+3 of the tile row) inside the footprint (lo > hi: none).  The x
// extent of a band is taken over the continuous span of its row centres: the
// left edge of the ellipse is convex and the right edge concave in y, so the
// extremes lie at the span's ends or at the ellipse's leftmost / rightmost
// point when that falls inside the span.  Extents are widened by 0.01 pixel
// (and 1e-4 relative), so the walk is conservative with respect to the
// blend's FP32 test (and cover the ~1 ulp of the hardware square root used
// here).  *rows (optional) receives the first and last pixel row walked.
// Used identically for counting and emitting.
// STEP = 16 walks whole tile rows instead of bands (only [lo[0], hi[0]] is
// then set): the extent over a tile row's span is the union of its bands'.
template <int STEP = 4, typename Visit>
__device__ inline void footprint_rows(float4 r0, float4 r1, float qmax, int W, int H,
                                      Visit&& visit, int* rows = nullptr) {
    static_assert(STEP == 4 || STEP == 16, "steps of a band or of a tile row");
    constexpr float kInvK = (float)(1.0 / kExp2Scale);
    const float a = r1.x * kInvK, b = 0.5f * r1.y * kInvK, c = r1.z * kInvK;
    const float det = a * c - b * b;
    if (!(a > 0.0f && det > 0.0f && qmax > 0.0f)) return;
    const float ia = 1.0f / a, cq = det * ia;  // q = a (dx + b dy / a)^2 + cq dy^2
    const float ry = __builtin_amdgcn_sqrtf(qmax / cq) * 1.0001f + 0.01f;
    const float vc = r0.y - 0.5f + r0.w;  // row index whose centre is the mean
    const float fy0 = fmaxf(ceilf(vc - ry), 0.0f);
    const float fy1 = fminf(floorf(vc + ry), (float)(H - 1));
    if (!(fy0 <= fy1)) return;
    const int y0 = (int)fy0, y1 = (int)fy1;
    if (rows) {
        rows[0] = y0;
        rows[1] = y1;
    }
    const float cx = r0.x - 0.5f + r0.z;  // column index whose centre is the mean
    // leftmost / rightmost point of the ellipse: dx = -+ sqrt(qmax Sxx) at
    // dy = -+ sqrt(qmax / Sxx) Sxy, with Sxx = c / det, Sxy = -b / det
    const float sxx = c / det, sxy = -b / det;
    const float xr = __builtin_amdgcn_sqrtf(qmax * sxx) * 1.0001f + 0.01f;
    const float dyl = -__builtin_amdgcn_sqrtf(qmax / sxx) * sxy;  // row offset of the leftmost point (rightmost: -dyl)
    auto edges = [&](int y, float& l, float& r) {
        const float dy = ((float)y + 0.5f - r0.y) - r0.w;
        const float disc = fmaxf(qmax - cq * dy * dy, 0.0f);
        const float half = __builtin_amdgcn_sqrtf(disc * ia) * 1.0001f + 0.01f;
        const float mid = cx - b * dy * ia;
        l = mid - half;
        r = mid + half;
    };
    int lo[4], hi[4];
    int cur = y0 >> kTileShift;
    for (int k = 0; k < 4; ++k) { lo[k] = 1 << 30; hi[k] = -1; }
    for (int ya = y0; ya <= y1; ya = (ya | (STEP - 1)) + 1) {
        const int yb = min(ya | (STEP - 1), y1);  // rows [ya, yb] of one band (tile row)
        const int ty = ya >> kTileShift;
        if (ty != cur) {
            visit(cur, lo, hi);
            for (int k = 0; k < 4; ++k) { lo[k] = 1 << 30; hi[k] = -1; }
            cur = ty;
        }
        float la, ra, lb, rb;
        edges(ya, la, ra);
        edges(yb, lb, rb);
        float l = fminf(la, lb), r = fmaxf(ra, rb);
        const float sa = ((float)ya + 0.5f - r0.y) - r0.w, sb = ((float)yb + 0.5f - r0.y) - r0.w;
        if (sa <= dyl && dyl <= sb) l = cx - xr;
        if (sa <= -dyl && -dyl <= sb) r = cx + xr;
        const float xf = fmaxf(ceilf(l), 0.0f);
        const float xl = fminf(floorf(r), (float)(W - 1));
        if (!(xf <= xl)) continue;
        const int band = STEP == 4 ? (ya >> 2) & 3 : 0;
        const int t0 = (int)xf >> kTileShift, t1 = (int)xl >> kTileShift;
        for (int k = 0; k < 4; ++k)
            if (k == band) {
                lo[k] = min(lo[k], t0);
                hi[k] = max(hi[k], t1);
            }
    }
    visit(cur, lo, hi);
}

// Footprint per bin row.  BIN = 16: the bin is the 16x16 tile and its 4-bit
// mask marks the bands (rows 4k..4k+3) the footprint reaches.  BIN = 32: the
// bin is a 32x32 block of four 16x16 tiles and bit 2h + c marks the tile in
// row half h and column half c.  visit(bin_row, t0, t1, mask_of, n, h) is
// called per bin row with the bin columns [t0, t1], a function giving a bin
// column's mask (0: not reached), n, the number of columns in [t0, t1] whose
// mask is not 0, and (BIN = 32) h = the first and last 16-pixel tile column
// reached in each row half (lo0, hi0, lo1, hi1; lo > hi: none).
template <int BIN, typename Visit>
__device__ inline void footprint_bins(float4 r0, float4 r1, float qmax, int W, int H,
                                      Visit&& visit, int* rows = nullptr) {
    if constexpr (BIN == 16) {
        footprint_rows(r0, r1, qmax, W, H, [&](int ty, const int* lo, const int* hi) {
            int t0 = 1 << 30, t1 = -1;
            for (int k = 0; k < 4; ++k) {
                t0 = min(t0, lo[k]);
                t1 = max(t1, hi[k]);
            }
            auto mask_of = [&](int t) {
                uint32_t m = 0;
                for (int k = 0; k < 4; ++k) m |= (lo[k] <= t && t <= hi[k]) ? (1u << k) : 0u;
                return m;
            };
            int n = 0;
            for (int t = t0; t <= t1; ++t) n += mask_of(t) != 0u;
            visit(ty, t0, t1, mask_of, n, make_int4(0, -1, 0, -1));
        }, rows);
    } else {
        static_assert(BIN == 32, "bins are 16 or 32 pixels");
        // 16-column block ranges of the two tile rows of the current bin row
        int cur = -1, lo[2] = {1 << 30, 1 << 30}, hi[2] = {-1, -1};
        auto flush = [&]() {
            if (cur < 0) return;
            const int b0 = min(lo[0], lo[1]), b1 = max(hi[0], hi[1]);
            if (b0 <= b1) {
                // a bin column t has a tile of row half h reached exactly when
                // lo[h] >> 1 <= t <= hi[h] >> 1 (tile columns are >= 0; an
                // unreached half has lo > hi and gives an empty range), so the
                // reached columns are the union of two ranges
                const int a0 = lo[0] >> 1, a1 = hi[0] >> 1, c0 = lo[1] >> 1, c1 = hi[1] >> 1;
                const int na = max(a1 - a0 + 1, 0), nc = max(c1 - c0 + 1, 0);
                const int nboth = max(min(a1, c1) - max(a0, c0) + 1, 0);
                visit(cur, b0 >> 1, b1 >> 1, [&](int t) {
                    uint32_t m = 0;
                    for (int h = 0; h < 2; ++h)
                        for (int c = 0; c < 2; ++c)
                            m |= (lo[h] <= 2 * t + c && 2 * t + c <= hi[h]) ? (1u << (2 * h + c)) : 0u;
                    return m;
                }, na + nc - nboth, make_int4(lo[0], hi[0], lo[1], hi[1]));
            }
        };
        footprint_rows<16>(r0, r1, qmax, W, H, [&](int ty, const int* l4, const int* h4) {
            const int br = ty >> 1, h = ty & 1;
            if (br != cur) {
                flush();
                cur = br;
                lo[0] = lo[1] = 1 << 30;
                hi[0] = hi[1] = -1;
            }
            for (int k = 0; k < 4; ++k) {
                lo[h] = min(lo[h], l4[k]);
                hi[h] = max(hi[h], h4[k]);
            }
        }, rows);
        flush();
    }
}

// a2, first step: the depth key of every (view, Gaussian) item of the batch,
// keys[i] = bits of the camera-space depth of the mean computed in binary32
// (positive floats order like their bit patterns), 0xFFFFFFFF for items culled
// by the near plane or too faint to pass the alpha floor anywhere; vals[i] = i.
__global__ __launch_bounds__(256) void k_depth_keys(const ViewInfo* __restrict__ views, int n_views,
                                                    uint32_t n_items, const float* __restrict__ means,
                                                    const float* __restrict__ opac, BlendParams bp,
                                                    uint32_t* __restrict__ keys,
                                                    uint32_t* __restrict__ vals) {
    __shared__ uint32_t sbase[kViewLds];
    const bool vlds = stage_view_bases(views, n_views, sbase);
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_items) return;
    const ViewInfo& V = views[view_of(views, n_views, sbase, vlds, i)];
    const int64_t g = V.g_offset + (int64_t)(i - V.item_base);
    const float key = __fmaf_rn(V.R[6], means[3 * g],
                                __fmaf_rn(V.R[7], means[3 * g + 1], __fmaf_rn(V.R[8], means[3 * g + 2], V.t[2])));
    keys[i] = (key > bp.znear && reach_q(opac[g], bp) > 0.0f) ? __float_as_uint(key) : 0xFFFFFFFFu;
    vals[i] = i;
}

void launch_depth_keys(const ViewInfo* views, int n_views, uint32_t n_items, const float* means,
                       const float* opac, BlendParams bp, uint32_t* keys, uint32_t* vals,
                       hipStream_t s) {
    if (n_items == 0 || n_views <= 0) return;
    hipLaunchKernelGGL(k_depth_keys, dim3((n_items + 255) / 256), dim3(256), 0, s, views, n_views,
                       n_items, means, opac, bp, keys, vals);
}

// a2: projection of the items in depth order: thread k handles item
// order[k] (k itself when order is null) and writes its record and tile-pair
// count at position k, so that binning reads them contiguously; the random
// reads go to the per-Gaussian geometry, which caches across views.
// The projection is evaluated in FP64 (a few dozen operations per item) and
// the pixel position is stored as an FP32 hi/lo pair, so that the blend can
// form pixel offsets d = (p - u_hi) - u_lo exactly to one FP32 ulp of d; a
// single FP32 coordinate of a 512-pixel image is only good to ~3e-5 pixel,
// enough to move alpha by ~1e-4 relative at the footprint edge.
// A tile is binned only if its pixel centres come within the footprint
// reach (3-sigma ellipse, shrunk by the alpha floor for faint splats).
// rec2[k] = (first | last << 16, i): the pixel rows the footprint walk covers
// and the item.
template <int BIN>
__global__ __launch_bounds__(256) void k_project(const ViewInfo* __restrict__ views, int n_views,
                                                 uint32_t n_items, const uint32_t* __restrict__ order,
                                                 const float* __restrict__ geo,
                                                 BlendParams bp, uint32_t* __restrict__ counts,
                                                 float4* __restrict__ rec0, float4* __restrict__ rec1,
                                                 uint2* __restrict__ rec2) {
    __shared__ uint32_t sbase[kViewLds];
    const bool vlds = stage_view_bases(views, n_views, sbase);
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_items) return;
    const uint32_t i = order ? order[k] : k;
    const ViewInfo& V = views[view_of(views, n_views, sbase, vlds, i)];
    const int64_t g = V.g_offset + (int64_t)(i - V.item_base);
    // one 64-byte record per Gaussian: a single cache line per random gather
    const float4* gr = reinterpret_cast<const float4*>(geo + kGeoStride * g);
    const double2* gd = reinterpret_cast<const double2*>(gr + 1);
    const float4 ga = gr[0];
    const double2 s01 = gd[0], s23 = gd[1], s45 = gd[2];  // xx xy | xz yy | yz zz
    float mx = ga.x, my = ga.y, mz = ga.z;
    float key = __fmaf_rn(V.R[6], mx, __fmaf_rn(V.R[7], my, __fmaf_rn(V.R[8], mz, V.t[2])));
    uint32_t cnt = 0;
    int rows[2] = {1, 0};
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
    const float og = ga.w;
    const float qmax = reach_q(og, bp);
    if (key > bp.znear && qmax > 0.0f) {
        double R[9];
        for (int k = 0; k < 9; ++k) R[k] = V.R[k];
        const double dmx = mx, dmy = my, dmz = mz;
        const double tx = R[0] * dmx + R[1] * dmy + R[2] * dmz + (double)V.t[0];
        const double ty = R[3] * dmx + R[4] * dmy + R[5] * dmz + (double)V.t[1];
        const double tz = R[6] * dmx + R[7] * dmy + R[8] * dmz + (double)V.t[2];
        const double iz = 1.0 / tz;
        const double fx = V.fx, fy = V.fy;
        const double j00 = fx * iz, j02 = -fx * tx * iz * iz;
        const double j11 = fy * iz, j12 = -fy * ty * iz * iz;
        const double S[3][3] = {{s01.x, s01.y, s23.x}, {s01.y, s23.y, s45.x}, {s23.x, s45.x, s45.y}};
        // Sc = W S W^T
        double M[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                M[a][b] = R[3 * a] * S[0][b] + R[3 * a + 1] * S[1][b] + R[3 * a + 2] * S[2][b];
        double Sc[3][3];
        for (int a = 0; a < 3; ++a)
            for (int b = a; b < 3; ++b)
                Sc[a][b] = M[a][0] * R[3 * b] + M[a][1] * R[3 * b + 1] + M[a][2] * R[3 * b + 2];
        const double dil = bp.dilation;
        const double sxx = j00 * j00 * Sc[0][0] + 2.0 * j00 * j02 * Sc[0][2] + j02 * j02 * Sc[2][2] + dil;
        const double sxy = j00 * j11 * Sc[0][1] + j00 * j12 * Sc[0][2] + j02 * j11 * Sc[1][2] + j02 * j12 * Sc[2][2];
        const double syy = j11 * j11 * Sc[1][1] + 2.0 * j11 * j12 * Sc[1][2] + j12 * j12 * Sc[2][2] + dil;
        const double det = sxx * syy - sxy * sxy;
        const double u = fx * tx * iz + (double)V.cx;
        const double vv = fy * ty * iz + (double)V.cy;
        if (det > 0.0 && isfinite(u) && isfinite(vv)) {
            const double inv = 1.0 / det;
            const float uh = (float)u, vh = (float)vv;
            r0 = make_float4(uh, vh, (float)(u - (double)uh), (float)(vv - (double)vh));
            r1 = make_float4((float)(kExp2Scale * syy * inv), (float)(-2.0 * kExp2Scale * sxy * inv),
                             (float)(kExp2Scale * sxx * inv), og);
            footprint_bins<BIN>(r0, r1, qmax, V.width, V.height, [&](int, int, int, auto&&, int n, int4) {
                cnt += (uint32_t)n;
            }, rows);
        }
    }
    counts[k] = cnt;
    // records are read only through tile pairs: an item with none keeps its
    // slot unwritten
    if (cnt != 0) {
        rec0[k] = r0;
        rec1[k] = r1;
        rec2[k] = make_uint2((uint32_t)(rows[0] & 0xFFFF) | ((uint32_t)(rows[1] & 0xFFFF) << 16), i);
    }
}

void launch_project(const ViewInfo* views, int n_views, uint32_t n_items, const uint32_t* order,
                    const float* geo, BlendParams bp, uint32_t* counts, float4* rec0, float4* rec1,
                    uint2* rec2, int bin, hipStream_t s) {
    if (n_items == 0 || n_views <= 0) return;
    if (bin == 32)
        hipLaunchKernelGGL(k_project<32>, dim3((n_items + 255) / 256), dim3(256), 0, s, views, n_views,
                           n_items, order, geo, bp, counts, rec0, rec1, rec2);
    else
        hipLaunchKernelGGL(k_project<16>, dim3((n_items + 255) / 256), dim3(256), 0, s, views, n_views,
                           n_items, order, geo, bp, counts, rec0, rec1, rec2);
}

// a3: emit (global bin id, k | mask) pairs in depth order, k being the depth
// rank of the item (records, counts and offsets are in that order); a stable
// sort by bin id then yields every bin's list in front-to-back order.
constexpr uint32_t kEmitStage = 2048;  // pairs a block stages in LDS (16 KB: eight resident blocks per CU)

template <int BIN>
__global__ __launch_bounds__(256) void k_emit(const ViewInfo* __restrict__ views, int n_views,
                                              const uint32_t* __restrict__ sorted_vals,
                                              const uint32_t* __restrict__ offsets,
                                              const uint32_t* __restrict__ counts,
                                              const float4* __restrict__ rec0,
                                              const float4* __restrict__ rec1, BlendParams bp,
                                              uint32_t n_items, uint32_t sentinel, uint32_t cap,
                                              uint32_t* __restrict__ overflow,
                                              uint32_t* __restrict__ pair_keys,
                                              uint32_t* __restrict__ pair_vals) {
    // The block's items are consecutive depth ranks, so their pairs form one
    // contiguous range [base, end_all): when it fits, the pairs are assembled
    // in LDS and stored with full-width coalesced writes.
    __shared__ uint32_t skey[kEmitStage];
    __shared__ uint32_t sval[kEmitStage];
    const uint32_t k0 = blockIdx.x * blockDim.x;
    const uint32_t klast = min(k0 + blockDim.x, n_items) - 1;
    const uint32_t base = offsets[k0];
    const uint32_t end_all = offsets[klast] + counts[klast];
    const bool staged = end_all - base <= kEmitStage;
    const uint32_t k = k0 + threadIdx.x;
    if (k < n_items) {
        const uint32_t cnt = counts[k];
        if (cnt != 0) {
            const ViewInfo& V = views[find_view_item(views, n_views, sorted_vals[k])];
            const float4 r0 = rec0[k], r1 = rec1[k];
            uint32_t off = offsets[k];
            uint32_t end = off + cnt;
            if (end > cap || end < off) {  // capacity exceeded: keep what fits, report the rest
                if (overflow) atomicAdd(overflow, 1u);
                end = off < cap ? cap : off;
            }
            auto put = [&](uint32_t o, uint32_t key, uint32_t val) {
                if (staged) {
                    skey[o - base] = key;
                    sval[o - base] = val;
                } else {
                    pair_keys[o] = key;
                    pair_vals[o] = val;
                }
            };
            footprint_bins<BIN>(r0, r1, reach_q(r1.w, bp), V.width, V.height,
                                [&](int ty, int t0, int t1, auto&& mask_of, int, int4) {
                for (int t = t0; t <= t1; ++t) {
                    const uint32_t m = mask_of(t);
                    if (m == 0u || off >= end) continue;
                    put(off, V.tile_base + (uint32_t)ty * (uint32_t)V.tiles_x + (uint32_t)t,
                        k | (m << kItemBits));
                    ++off;
                }
            });
            // The walk above and the one that counted are the same code on the
            // same record; should they ever disagree, unused slots get a tile
            // id past the last tile, which sorts last and is ignored by the
            // range kernel.
            for (; off < end; ++off) put(off, sentinel, 0u);
        }
    }
    if (!staged) return;  // uniform over the block
    __syncthreads();
    const uint32_t lim = min(end_all, max(cap, base));
    for (uint32_t o = base + threadIdx.x; o < lim; o += blockDim.x) {
        pair_keys[o] = skey[o - base];
        pair_vals[o] = sval[o - base];
    }
}

// 32-pixel bins, emitted by the block together.  Each lane walks its item's
// footprint as above, but records every bin row it reaches as one segment
// in LDS (the row's first output slot, the lane, and the two tile-row
// halves' column ranges, whose union is the row's reached bin columns);
// the first slot of each segment is marked.  A max-scan over the block's
// output slots then names each slot's segment, and every thread writes one
// pair per step: the pair's bin column is found by rank within its segment,
// so an item's pair count no longer holds the other 63 lanes of its wave,
// and the stores are coalesced.  Pairs come out in the order the per-lane
// walk writes them.  Blocks whose range exceeds kEmitStage slots, or whose
// rows exceed kEmitSegs segments, fall back to that walk.
constexpr uint32_t kEmitSegs = 1024;  // bin-row segments a block collects (16 KB)

// A tile-column range packed as lo | hi << 16; no columns: (0x7FFF, 0).
__device__ inline uint32_t pack_cols(int lo, int hi) {
    return lo <= hi ? ((uint32_t)lo | ((uint32_t)hi << 16)) : 0x7FFFu;
}

__global__ __launch_bounds__(256) void k_emit32(const ViewInfo* __restrict__ views, int n_views,
                                                const uint32_t* __restrict__ sorted_vals,
                                                const uint32_t* __restrict__ offsets,
                                                const uint32_t* __restrict__ counts,
                                                const float4* __restrict__ rec0,
                                                const float4* __restrict__ rec1, BlendParams bp,
                                                uint32_t n_items, uint32_t sentinel, uint32_t cap,
                                                uint32_t* __restrict__ overflow,
                                                uint32_t* __restrict__ pair_keys,
                                                uint32_t* __restrict__ pair_vals) {
    __shared__ uint4 sseg[kEmitSegs];        // (first slot | lane << 16 | sentinel << 31, bin row, half 0, half 1)
    __shared__ uint16_t sslot[kEmitStage];   // segment marks, then each slot's segment
    __shared__ uint32_t sitem[256], stbase[256], stx[256];
    __shared__ uint32_t wtop[4];
    __shared__ uint32_t nseg;
    __shared__ uint32_t sbase[kViewLds];
    static_assert(kEmitStage == 8 * 256, "eight slots per thread");
    const bool vlds = stage_view_bases(views, n_views, sbase);
    const uint32_t tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t k0 = blockIdx.x * blockDim.x;
    const uint32_t klast = min(k0 + blockDim.x, n_items) - 1;
    const uint32_t base = offsets[k0];
    const uint32_t end_all = offsets[klast] + counts[klast];
    const bool staged = end_all - base <= kEmitStage;  // uniform over the block
    const uint32_t k = k0 + tid;
    uint32_t cnt = 0, off = 0, end = 0;
    const ViewInfo* V = nullptr;
    float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
    if (k < n_items) {
        cnt = counts[k];
        if (cnt != 0) {
            V = &views[view_of(views, n_views, sbase, vlds, sorted_vals[k])];
            r0 = rec0[k];
            r1 = rec1[k];
            off = offsets[k];
            end = off + cnt;
            if (end > cap || end < off) {  // capacity exceeded: keep what fits, report the rest
                if (overflow) atomicAdd(overflow, 1u);
                end = off < cap ? cap : off;
            }
        }
    }
    if (staged) {
        reinterpret_cast<uint4*>(sslot)[tid] = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
        if (tid == 0) nseg = 0u;
        __syncthreads();
        if (cnt != 0) {
            sitem[tid] = k;
            stbase[tid] = V->tile_base;
            stx[tid] = V->tiles_x;
            uint32_t o = off;
            auto add_seg = [&](uint32_t x, uint32_t y, uint32_t z, uint32_t ww) {
                const uint32_t si = atomicAdd(&nseg, 1u);
                if (si < kEmitSegs) {
                    sseg[si] = make_uint4(x, y, z, ww);
                    sslot[o - base] = (uint16_t)si;
                }
            };
            footprint_bins<32>(r0, r1, reach_q(r1.w, bp), V->width, V->height,
                               [&](int ty, int, int, auto&&, int n, int4 h) {
                if (n <= 0) return;
                if (o < end)
                    add_seg((o - base) | (tid << 16), (uint32_t)ty, pack_cols(h.x, h.y), pack_cols(h.z, h.w));
                o += (uint32_t)n;
            });
            // The walk above and the one that counted are the same code on the
            // same record; should they ever disagree, unused slots get a tile
            // id past the last tile, which sorts last and is ignored by the
            // range kernel.
            if (o < end) add_seg((o - base) | (tid << 16) | 0x80000000u, 0u, 0x7FFFu, 0x7FFFu);
        }
        __syncthreads();
        if (nseg <= kEmitSegs) {  // uniform over the block
            // each slot's segment: the last mark at or before it, by a max-scan
            // of (slot + 1) << 16 | segment over the marked slots
            const uint4 raw = reinterpret_cast<const uint4*>(sslot)[tid];
            const uint32_t words[4] = {raw.x, raw.y, raw.z, raw.w};
            uint32_t inc[8], run = 0u;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t mk = (words[j >> 1] >> (16 * (j & 1))) & 0xFFFFu;
                if (mk != 0xFFFFu) run = ((8u * tid + (uint32_t)j + 1u) << 16) | mk;
                inc[j] = run;
            }
            uint32_t sc = run;  // wave inclusive max-scan of the threads' last marks
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o2 = __shfl_up(sc, d, 64);
                if ((int)lane >= d) sc = max(sc, o2);
            }
            if (lane == 63) wtop[w] = sc;
            uint32_t carry = __shfl_up(sc, 1, 64);
            if (lane == 0) carry = 0u;
            __syncthreads();
            for (uint32_t q = 0; q < w; ++q) carry = max(carry, wtop[q]);
            uint32_t outw[4];
#pragma unroll
            for (int j = 0; j < 8; j += 2)
                outw[j >> 1] = (max(carry, inc[j]) & 0xFFFFu) | ((max(carry, inc[j + 1]) & 0xFFFFu) << 16);
            reinterpret_cast<uint4*>(sslot)[tid] = make_uint4(outw[0], outw[1], outw[2], outw[3]);
            __syncthreads();
            const uint32_t lim = min(end_all, max(cap, base));
            for (uint32_t i = tid; base + i < lim; i += blockDim.x) {
                const uint4 sg = sseg[sslot[i]];
                uint32_t key = sentinel, val = 0u;
                if (!(sg.x & 0x80000000u)) {
                    const uint32_t l = (sg.x >> 16) & 0xFFu;
                    const int r = (int)(i - (sg.x & 0xFFFFu));
                    const int lo0 = (int)(sg.z & 0xFFFFu), hi0 = (int)(sg.z >> 16);
                    const int lo1 = (int)(sg.w & 0xFFFFu), hi1 = (int)(sg.w >> 16);
                    // the row's reached bin columns, [a0, a1] u [c0, c1], in
                    // increasing order
                    const int a0 = lo0 >> 1, a1 = hi0 >> 1, c0 = lo1 >> 1, c1 = hi1 >> 1;
                    int t;
                    if (a1 < a0) {
                        t = c0 + r;
                    } else if (c1 < c0) {
                        t = a0 + r;
                    } else {
                        const bool af = a0 <= c0;
                        const int f0 = af ? a0 : c0, f1 = af ? a1 : c1, s0 = af ? c0 : a0;
                        const int nf = f1 - f0 + 1;
                        t = (s0 <= f1 + 1 || r < nf) ? f0 + r : s0 + (r - nf);
                    }
                    uint32_t m = 0u;
#pragma unroll
                    for (int c = 0; c < 2; ++c) {
                        m |= (lo0 <= 2 * t + c && 2 * t + c <= hi0) ? (1u << c) : 0u;
                        m |= (lo1 <= 2 * t + c && 2 * t + c <= hi1) ? (1u << (2 + c)) : 0u;
                    }
                    key = stbase[l] + sg.y * stx[l] + (uint32_t)t;
                    val = sitem[l] | (m << kItemBits);
                }
                pair_keys[base + i] = key;
                pair_vals[base + i] = val;
            }
            return;
        }
    }
    // each lane writes its own pairs
    if (cnt == 0) return;
    footprint_bins<32>(r0, r1, reach_q(r1.w, bp), V->width, V->height,
                       [&](int ty, int t0, int t1, auto&& mask_of, int, int4) {
        for (int t = t0; t <= t1; ++t) {
            const uint32_t m = mask_of(t);
            if (m == 0u || off >= end) continue;
            pair_keys[off] = V->tile_base + (uint32_t)ty * (uint32_t)V->tiles_x + (uint32_t)t;
            pair_vals[off] = k | (m << kItemBits);
            ++off;
        }
    });
    for (; off < end; ++off) {
        pair_keys[off] = sentinel;
        pair_vals[off] = 0u;
    }
}

void launch_emit(const ViewInfo* views, int n_views, const uint32_t* sorted_vals,
                 const uint32_t* offsets, const uint32_t* counts, const float4* rec0,
                 const float4* rec1, BlendParams bp, uint32_t n_items, uint32_t n_tiles,
                 uint32_t* pair_keys, uint32_t* pair_vals, int bin, hipStream_t s, uint32_t cap,
                 uint32_t* overflow) {
    if (n_items == 0) return;
    if (bin == 32)
        hipLaunchKernelGGL(k_emit32, dim3((n_items + 255) / 256), dim3(256), 0, s, views, n_views,
                           sorted_vals, offsets, counts, rec0, rec1, bp, n_items, n_tiles, cap,
                           overflow, pair_keys, pair_vals);
    else
        hipLaunchKernelGGL(k_emit<16>, dim3((n_items + 255) / 256), dim3(256), 0, s, views, n_views,
                           sorted_vals, offsets, counts, rec0, rec1, bp, n_items, n_tiles, cap,
                           overflow, pair_keys, pair_vals);
}

// A modest grid (one 64-bit atomic per block on the same word) reading 16
// bytes per thread and step; counts is 16-byte aligned.
__global__ __launch_bounds__(256) void k_sum_u64(const uint32_t* __restrict__ counts, uint32_t n,
                                                unsigned long long* __restrict__ out) {
    __shared__ unsigned long long part[4];
    unsigned long long acc = 0;
    const uint4* c4 = reinterpret_cast<const uint4*>(counts);
    const uint32_t n4 = n / 4;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += gridDim.x * blockDim.x) {
        const uint4 v = c4[i];
        acc += (unsigned long long)v.x + v.y + v.z + v.w;
    }
    if (blockIdx.x == 0 && threadIdx.x < n - 4 * n4) acc += counts[4 * n4 + threadIdx.x];
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

void launch_sum_u64(const uint32_t* counts, uint32_t n, unsigned long long* out, hipStream_t s) {
    if (n == 0) return;
    // about eight 16-byte loads per thread, at most 1024 atomics
    uint32_t blocks = (n / 4 + 2047) / 2048;
    blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
    hipLaunchKernelGGL(k_sum_u64, dim3(blocks), dim3(256), 0, s, counts, n, out);
}

// Thread q owns keys 4q .. 4q + 3 (one 16-byte load where all four are
// live); neighbours across threads come from the adjacent lanes, with loads
// only at the wave's edges.
__global__ __launch_bounds__(256) void k_tile_ranges(const uint32_t* __restrict__ keys, uint32_t n,
                                                     const uint32_t* __restrict__ n_dev, uint32_t n_tiles,
                                                     uint2* __restrict__ ranges) {
    if (n_dev) n = min(n, *n_dev);
    const uint32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    const uint64_t k0 = 4ull * q;
    uint32_t t[4];
    if (k0 + 3 < n) {
        const uint4 v = reinterpret_cast<const uint4*>(keys)[q];
        t[0] = v.x; t[1] = v.y; t[2] = v.z; t[3] = v.w;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = k0 + e < n ? keys[k0 + e] : 0xFFFFFFFFu;
    }
    uint32_t prev = (uint32_t)__shfl_up((int)t[3], 1, 64);
    uint32_t next = (uint32_t)__shfl_down((int)t[0], 1, 64);
    if (lane == 0) prev = (k0 > 0 && k0 - 1 < n) ? keys[k0 - 1] : 0xFFFFFFFFu;
    if (lane == 63) next = k0 + 4 < n ? keys[k0 + 4] : 0xFFFFFFFFu;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const uint64_t k = k0 + e;
        if (k >= n || t[e] >= n_tiles) continue;
        const uint32_t p = e == 0 ? prev : t[e > 0 ? e - 1 : 0];
        const uint32_t x = e == 3 ? next : t[e < 3 ? e + 1 : 3];
        if (k == 0 || p != t[e]) ranges[t[e]].x = (uint32_t)k;
        if (k + 1 == n || x != t[e]) ranges[t[e]].y = (uint32_t)(k + 1);
    }
}

void launch_tile_ranges(const uint32_t* sorted_keys, uint32_t n_pairs, uint32_t n_tiles,
                        uint2* ranges, hipStream_t s, const uint32_t* n_dev) {
    if (n_pairs == 0) return;
    const uint32_t quads = (uint32_t)(((uint64_t)n_pairs + 3) / 4);
    hipLaunchKernelGGL(k_tile_ranges, dim3((quads + 255) / 256), dim3(256), 0, s, sorted_keys,
                       n_pairs, n_dev, n_tiles, ranges);
}

}  // namespace gsc
