// C ABI: argument validation, context and scratch management, and the
// per-call pipeline  project -> depth sort -> scan -> emit -> tile sort ->
// tile ranges -> accumulate (per view batch) -> fold + solve.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gsc_internal.h"

using namespace gsc;

namespace {

thread_local std::string g_last_error;

gsc_status fail(gsc_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define GSC_HIP(call)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(GSC_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_));       \
    } while (0)

#define GSC_LAUNCHED(what)                                                                  \
    do {                                                                                    \
        hipError_t e_ = hipGetLastError();                                                  \
        if (e_ != hipSuccess)                                                               \
            return fail(GSC_ERR_HIP, "%s launch failed: %s", what, hipGetErrorString(e_)); \
    } while (0)

// A fixed region of device memory that buffers are carved from instead of
// being allocated (the allocation-free entry point).  Carving only moves a
// cursor; nothing carved is ever freed.
struct Arena {
    char* base = nullptr;
    size_t cap = 0;
    size_t used = 0;
    size_t need = 0;  // bytes the first request that did not fit would have needed
};

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    Arena* arena = nullptr;  // non-null: carve from the arena, never allocate
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap && p) return hipSuccess;
        if (arena) {
            const size_t off = (arena->used + 255) & ~(size_t)255;
            if (off + bytes > arena->cap) {
                if (arena->need == 0) arena->need = off + bytes;
                return hipErrorOutOfMemory;
            }
            p = arena->base + off;
            cap = bytes;
            arena->used = off + bytes;
            return hipSuccess;
        }
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            cap = 0;
        }
        size_t want = std::max<size_t>(bytes + bytes / 8, 4096);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        return e;
    }
    void release() {
        if (p && !arena) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T* as() const { return reinterpret_cast<T*>(p); }
};

// Upper bound on (view, Gaussian) items per batch.
constexpr uint64_t kMaxItemsPerBatch = 1ull << 26;
// Upper bound on (tile, item) pairs per batch (uint32 offsets).
constexpr uint64_t kMaxPairsPerBatch = 1ull << 31;

// The batch bounds of a set of options (gsc_options.batch_items / batch_pairs).
inline uint64_t batch_item_limit(const gsc_options& o) {
    return o.batch_items ? (uint64_t)o.batch_items : kMaxItemsPerBatch;
}
// A plan's default batch: 2^24 items, whose depth-sort keys, values and
// their alternates (16 bytes per item) about fill the 256 MB last-level
// cache.  Measured on the 32-scene plan (8 to 49 batches): 2^24 items per
// batch 281 ms per run, 2^26 296 ms; the accumulate itself is 3% slower in
// the smaller batches, the sorts gain more.
constexpr uint64_t kPlanItemsPerBatch = 1ull << 24;
inline uint64_t plan_item_limit(const gsc_options& o) {
    return o.batch_items ? (uint64_t)o.batch_items : kPlanItemsPerBatch;
}
inline uint64_t batch_pair_limit(const gsc_options& o) {
    return o.batch_pairs ? (uint64_t)o.batch_pairs : kMaxPairsPerBatch - 1;
}

}  // namespace

// What a binning depends on: the geometry arrays (by address; their contents
// are the caller's promise under GSC_FLAG_REUSE_BINNING), the cameras, the
// blend constants and the requested bin size.
struct BinKey {
    const float *means = nullptr, *scales = nullptr, *quats = nullptr, *opac = nullptr;
    int64_t N = 0;
    std::vector<gsc_camera> cams;
    BlendParams bp{};
    int bin_opt = 0;
    bool same(const BinKey& o) const {
        return means == o.means && scales == o.scales && quats == o.quats && opac == o.opac && N == o.N &&
               bin_opt == o.bin_opt && cams.size() == o.cams.size() &&
               (cams.empty() || memcmp(cams.data(), o.cams.data(), sizeof(gsc_camera) * cams.size()) == 0) &&
               memcmp(&bp, &o.bp, sizeof(bp)) == 0;
    }
};

struct gsc_ctx {
    gsc_options opt;
    int bin = 16;  // bin size of the current call
    // The automatic bin size of the last call and what it was chosen for
    // (geometry buffers, size, cameras): a call on the same ones reuses it
    // without reading statistics back.  The choice only steers performance.
    BinKey bin_choice_key;
    int bin_choice = 0;
    // the single-batch binning left in the buffers by the last call
    bool cache_valid = false;
    BinKey cache_key;
    int cache_bin = 16;
    uint32_t cache_tiles = 0, cache_pairs = 0;
    uint64_t cache_items = 0;
    // device scratch
    DevBuf views, views_all, cov, keys, vals, keys_alt, vals_alt, counts, offsets, rec0, rec1, rec2,
        sort_scratch, pkeys, pvals, pkeys_alt, pvals_alt, ranges, vs, gamma, bbar, misc, order, queues,
        coef_t, factor, img, stat, wbuf, post, vsdet, chk, obs;
    bool order_valid = false;  // `order` holds the tile order of the current binning
    // host staging
    ViewInfo* h_views = nullptr;  // staging of one batch's table
    size_t h_views_cap = 0;
    ViewInfo* h_all = nullptr;    // staging of the full camera table
    size_t h_all_cap = 0;
    uint32_t* h_total = nullptr;
    // allocation-free working context: buffers carved from an arena, host
    // staging in static arrays (never freed here), no host allocation
    bool no_alloc = false;
    gsc_stats stats;
    bool stats_pending = false;
    // device words the pending statistics are read from (the misc layout
    // below); null: misc
    const void* stats_dev = nullptr;
    // GSC_FLAG_PROFILE: event pairs recorded during the last call
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    struct Mark { int stage; hipEvent_t a, b; uint32_t launches; };
    std::vector<Mark> marks;
    std::array<DevBuf*, 33> bufs() {
        return {&views, &views_all, &cov, &keys, &vals, &keys_alt, &vals_alt, &counts,
                &offsets, &rec0, &rec1, &rec2, &sort_scratch, &pkeys, &pvals, &pkeys_alt,
                &pvals_alt, &ranges, &vs, &gamma, &bbar, &misc, &order, &queues, &coef_t,
                &factor, &img, &stat, &wbuf, &post, &vsdet, &chk, &obs};
    }
    ~gsc_ctx() {
        for (DevBuf* b : bufs()) b->release();
        if (!no_alloc) {
            if (h_views) (void)hipHostFree(h_views);
            if (h_all) (void)hipHostFree(h_all);
            if (h_total) (void)hipHostFree(h_total);
        }
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    }
};

namespace {
constexpr size_t kMaxEvents = 1 << 14;
// Records an event pair around a stage when profiling is on.  Pairs pile up
// until gsc_get_stats() sums them.  Under stream capture each event becomes an
// event-record node of the graph, added after the capture's current nodes
// (which it then replaces), so every replay re-records it and gsc_get_stats()
// reads the last replay's times.  (The runtime torch loads rejects
// hipEventRecordExternal under capture, so the node is added directly.)  If
// that fails the stage is not timed and the error is cleared: profiling never
// breaks a capture.
struct StageTimer {
    gsc_ctx* ctx;
    hipStream_t s;
    int stage;
    uint32_t launches;
    hipEvent_t a = nullptr;
    bool capturing = false;
    StageTimer(gsc_ctx* c, hipStream_t st, int stg, uint32_t n = 1) : ctx(c), s(st), stage(stg), launches(n) {
        if (!(ctx->opt.flags & GSC_FLAG_PROFILE)) return;
        if (ctx->opt.profile_stages != 0u && !((ctx->opt.profile_stages >> (stg & 31)) & 1u)) return;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        capturing = hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive;
        a = take();
        if (a && record(a) != hipSuccess) {
            (void)hipGetLastError();
            a = nullptr;
        }
    }
    hipError_t record(hipEvent_t e) {
        if (!capturing) return hipEventRecord(e, s);
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        unsigned long long id = 0;
        hipGraph_t g = nullptr;
        const hipGraphNode_t* deps = nullptr;
        size_t nd = 0;
        hipError_t err = hipStreamGetCaptureInfo_v2(s, &cs, &id, &g, &deps, &nd);
        if (err != hipSuccess) return err;
        hipGraphNode_t node = nullptr;
        if ((err = hipGraphAddEventRecordNode(&node, g, deps, nd, e)) != hipSuccess) return err;
        return hipStreamUpdateCaptureDependencies(s, &node, 1, hipStreamSetCaptureDependencies);
    }
    hipEvent_t take() {
        if (ctx->ev_used >= kMaxEvents) return nullptr;  // stats not drained: stop recording
        if (ctx->ev_used == ctx->ev_pool.size()) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            ctx->ev_pool.push_back(e);
        }
        return ctx->ev_pool[ctx->ev_used++];
    }
    ~StageTimer() {
        if (!a) return;
        hipEvent_t b = take();
        if (!b) return;
        if (record(b) != hipSuccess) {
            (void)hipGetLastError();
            return;
        }
        ctx->marks.push_back({stage, a, b, launches});
    }
};
}  // namespace

// misc buffer layout (device): [0] u64 contributions, [8] u32 pair total, [12] u32 ill count,
// [16] u64 pair total (overflow check)
namespace {
constexpr size_t kMiscBytes = 64;  // [32..63]: geometry statistics (4 doubles)
// bin_views result asking the caller to retry with fewer views per batch
constexpr gsc_status kSplit = (gsc_status)1;

// Entry points that read a count back cannot run under stream capture.
gsc_status refuse_capture(hipStream_t s, const char* what) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return fail(GSC_ERR_NOT_CAPTURABLE,
                    "%s reads the tile-pair count back and cannot be captured into a graph; "
                    "create a plan (gsc_plan_create) and capture gsc_colorize_batched", what);
    return GSC_OK;
}

gsc_status validate_options(const gsc_options* o) {
    if (!(o->alpha_min >= 0.0f && o->alpha_min < 1.0f)) return fail(GSC_ERR_INVALID_ARG, "alpha_min must be in [0,1)");
    if (!(o->alpha_max > 0.0f && o->alpha_max < 1.0f)) return fail(GSC_ERR_INVALID_ARG, "alpha_max must be in (0,1)");
    if (!(o->t_min >= 0.0f && o->t_min < 1.0f)) return fail(GSC_ERR_INVALID_ARG, "t_min must be in [0,1)");
    if (!(o->sigma_cut > 0.0f && o->sigma_cut < 16.0f)) return fail(GSC_ERR_INVALID_ARG, "sigma_cut must be in (0,16)");
    if (!(o->dilation >= 0.0f)) return fail(GSC_ERR_INVALID_ARG, "dilation must be >= 0");
    if (!(o->znear > 0.0f)) return fail(GSC_ERR_INVALID_ARG, "znear must be > 0");
    if (!(o->kappa_max > 0.0f)) return fail(GSC_ERR_INVALID_ARG, "kappa_max must be > 0");
    if (!(o->bin_size == 0 || o->bin_size == 16 || o->bin_size == 32))
        return fail(GSC_ERR_INVALID_ARG, "bin_size must be 0, 16 or 32");
    if (o->accumulate_variant != 0 && !accumulate_chunk_valid(o->accumulate_variant, GSC_F32) &&
        !accumulate_chunk_valid(o->accumulate_variant, GSC_BF16))
        return fail(GSC_ERR_INVALID_ARG, "accumulate_variant %d is not a variant code", o->accumulate_variant);
    if (!(o->schedule >= GSC_SCHEDULE_AUTO && o->schedule <= GSC_SCHEDULE_LONGEST_FIRST))
        return fail(GSC_ERR_INVALID_ARG, "schedule must be 0, 1 or 2");
    if ((uint64_t)o->batch_items > kMaxItemsPerBatch)
        return fail(GSC_ERR_INVALID_ARG, "batch_items must be at most 2^26 (got %u)", o->batch_items);
    if ((uint64_t)o->batch_pairs >= kMaxPairsPerBatch)
        return fail(GSC_ERR_INVALID_ARG, "batch_pairs must be below 2^31 (got %u)", o->batch_pairs);
    return GSC_OK;
}

// Automatic bin size.  32-pixel bins cut the (bin, Gaussian) pairs to sort
// by ~2.5x once footprints span several 16-pixel tiles, at the price of a
// coarser band cull in the blend; 16-pixel bins win for small footprints.
// The estimate of the footprint diameter is 6 sigma with sigma the mean axis
// scale projected at the distance from each camera to the centroid.
constexpr double kBin32Diameter = 24.0;  // pixels

int choose_bin(const double* stats /* host: sum scale, sum means */, int64_t N,
               const gsc_camera* cams, int n_cams) {
    if (N <= 0 || n_cams <= 0) return 16;
    const double sbar = stats[0] / (double)N;
    const double cx = stats[1] / N, cy = stats[2] / N, cz = stats[3] / N;
    double acc = 0.0;
    int n = 0;
    for (int j = 0; j < n_cams; ++j) {
        const gsc_camera& c = cams[j];
        // camera-space depth of the centroid
        const double z = c.R[6] * cx + c.R[7] * cy + c.R[8] * cz + c.t[2];
        if (!(z > 1e-6)) continue;
        acc += 6.0 * sbar * 0.5 * ((double)c.fx + (double)c.fy) / z;
        ++n;
    }
    return (n > 0 && acc / n > kBin32Diameter) ? 32 : 16;
}

gsc_status validate_geometry(const float* means, const float* scales, const float* quats,
                             const float* opac, int64_t N, const gsc_camera* cams, int32_t n_cams,
                             int64_t* rows_needed) {
    if (N < 0) return fail(GSC_ERR_INVALID_ARG, "N must be >= 0 (got %lld)", (long long)N);
    if (N > (int64_t)kItemMask) return fail(GSC_ERR_UNSUPPORTED, "N must be < 2^26 (got %lld)", (long long)N);
    if (N > 0 && (!means || !scales || !quats || !opac))
        return fail(GSC_ERR_INVALID_ARG, "null Gaussian array with N > 0");
    if (n_cams < 0) return fail(GSC_ERR_INVALID_ARG, "n_cams must be >= 0");
    if (n_cams > 0 && !cams) return fail(GSC_ERR_INVALID_ARG, "cams is null with n_cams > 0");
    int64_t rows = 0;
    for (int j = 0; j < n_cams; ++j) {
        const gsc_camera& c = cams[j];
        if (c.width <= 0 || c.height <= 0 || c.width > 32768 || c.height > 32768)
            return fail(GSC_ERR_INVALID_ARG, "camera %d: size %dx%d out of range", j, c.width, c.height);
        if (c.pixel_offset < 0) return fail(GSC_ERR_INVALID_ARG, "camera %d: negative pixel_offset", j);
        if (!(c.fx > 0.0f && c.fy > 0.0f) || !isfinite(c.cx) || !isfinite(c.cy))
            return fail(GSC_ERR_INVALID_ARG, "camera %d: bad intrinsics", j);
        for (int k = 0; k < 9; ++k)
            if (!isfinite(c.R[k])) return fail(GSC_ERR_INVALID_ARG, "camera %d: non-finite R", j);
        for (int k = 0; k < 3; ++k)
            if (!isfinite(c.t[k])) return fail(GSC_ERR_INVALID_ARG, "camera %d: non-finite t", j);
        rows = std::max<int64_t>(rows, c.pixel_offset + (int64_t)c.width * c.height);
    }
    *rows_needed = rows;
    return GSC_OK;
}

gsc_status validate_channels(int32_t C, int32_t sh_deg) {
    if (C < 1 || C > kMaxC) return fail(GSC_ERR_INVALID_ARG, "C must be in [1,64] (got %d)", C);
    if (sh_deg < 0 || sh_deg > 3) return fail(GSC_ERR_INVALID_ARG, "sh_deg must be in [0,3] (got %d)", sh_deg);
    return GSC_OK;
}

gsc_status expand_lambda(const float* lambda, int32_t n_lambda, int sh_deg, double* out) {
    int nb = (sh_deg + 1) * (sh_deg + 1);
    if (!lambda) return fail(GSC_ERR_INVALID_ARG, "lambda is null");
    if (!(n_lambda == 1 || n_lambda == sh_deg + 1 || n_lambda == nb))
        return fail(GSC_ERR_INVALID_ARG, "n_lambda must be 1, L+1 or (L+1)^2 (got %d)", n_lambda);
    for (int i = 0; i < n_lambda; ++i)
        if (!(lambda[i] >= 0.0f) || !isfinite(lambda[i]))
            return fail(GSC_ERR_INVALID_ARG, "lambda[%d] must be finite and >= 0", i);
    for (int l = 0; l <= sh_deg; ++l)
        for (int m = -l; m <= l; ++m) {
            int i = l * l + l + m;
            out[i] = n_lambda == 1 ? lambda[0] : (n_lambda == sh_deg + 1 ? lambda[l] : lambda[i]);
        }
    return GSC_OK;
}

BlendParams blend_params(const gsc_options& o) {
    BlendParams bp;
    bp.alpha_min = o.alpha_min;
    bp.alpha_max = o.alpha_max;
    bp.t_min = o.t_min;
    bp.cut2 = o.sigma_cut * o.sigma_cut;
    bp.dilation = o.dilation;
    bp.znear = o.znear;
    return bp;
}

// View j of a single scene of N Gaussians (per-view sums at slots j*N + g),
// binned at `bin` pixels.
ViewInfo make_view(const gsc_camera& c, int j, int64_t N, int bin) {
    ViewInfo v;
    memset(&v, 0, sizeof(v));
    memcpy(v.R, c.R, sizeof(v.R));
    memcpy(v.t, c.t, sizeof(v.t));
    v.fx = c.fx; v.fy = c.fy; v.cx = c.cx; v.cy = c.cy;
    for (int i = 0; i < 3; ++i)
        v.centre[i] = -((double)c.R[i] * c.t[0] + (double)c.R[3 + i] * c.t[1] + (double)c.R[6 + i] * c.t[2]);
    v.width = c.width;
    v.height = c.height;
    v.tiles_x = (c.width + bin - 1) / bin;
    v.tiles_y = (c.height + bin - 1) / bin;
    v.pixel_offset = c.pixel_offset;
    v.g_offset = 0;
    v.vs_base = (int64_t)j * N;
    v.n_gauss = (uint32_t)N;
    v.scene = 0;
    return v;
}

int bits_for(uint64_t n) {
    int b = 0;
    while (b < 32 && (1ull << b) < n) ++b;
    return b;
}

// Result of binning one view batch.
struct Binned {
    uint32_t n_tiles = 0;
    uint32_t n_pairs = 0;
    uint64_t n_items = 0;
};

// The tile order of the current binning for launches that take it, or
// nullptr (tile index order) under GSC_SCHEDULE_GRID.
const uint32_t* tile_order(const gsc_ctx* ctx, uint32_t n_tiles) {
    if (ctx->opt.schedule == GSC_SCHEDULE_GRID || !ctx->order_valid) return nullptr;
    return ctx->order.as<uint32_t>() + n_tiles;
}

// Project, depth-sort, emit and tile-sort the views [v0, v0+nv) of `all`.
// The batch's ViewInfo table is uploaded to ctx->views (tile_base local to
// the batch).  Synchronises `s` once to read the pair count.
gsc_status bin_views(gsc_ctx* ctx, const ViewInfo* all, int v0, int nv,
                     const float* means, const float* opac, int64_t N, const BlendParams& bp,
                     hipStream_t s, Binned* out) {
    ctx->order_valid = false;  // until this binning's order is built
    // tile numbering local to the batch
    if ((size_t)nv > ctx->h_views_cap) {
        if (ctx->h_views) GSC_HIP(hipHostFree(ctx->h_views));
        ctx->h_views = nullptr;
        GSC_HIP(hipHostMalloc((void**)&ctx->h_views, sizeof(ViewInfo) * (size_t)nv));
        ctx->h_views_cap = (size_t)nv;
    }
    uint64_t tiles = 0, items = 0;
    bool uniform = true;
    for (int k = 0; k < nv; ++k) {
        ViewInfo v = all[v0 + k];
        v.tile_base = (uint32_t)tiles;
        v.item_base = (uint32_t)items;
        tiles += (uint64_t)v.tiles_x * v.tiles_y;
        items += v.n_gauss;
        uniform = uniform && v.n_gauss == all[v0].n_gauss;
        ctx->h_views[k] = v;
    }
    for (int k = 0; k < nv; ++k) ctx->h_views[k].uniform_n = uniform ? all[v0].n_gauss : 0u;
    if (tiles >= 0xffffffffull) return fail(GSC_ERR_CAPACITY, "too many tiles in one batch");
    if (items > kMaxItemsPerBatch) return fail(GSC_ERR_CAPACITY, "too many items in one batch");
    GSC_HIP(ctx->views.ensure(sizeof(ViewInfo) * (size_t)nv));
    GSC_HIP(hipMemcpyAsync(ctx->views.p, ctx->h_views, sizeof(ViewInfo) * (size_t)nv,
                           hipMemcpyHostToDevice, s));
    out->n_items = items;
    out->n_tiles = (uint32_t)tiles;
    const uint32_t ni = (uint32_t)items;
    GSC_HIP(ctx->keys.ensure(4 * items + 4));
    GSC_HIP(ctx->vals.ensure(4 * items + 4));
    GSC_HIP(ctx->keys_alt.ensure(4 * items + 4));
    GSC_HIP(ctx->vals_alt.ensure(4 * items + 4));
    GSC_HIP(ctx->counts.ensure(4 * items + 4));
    GSC_HIP(ctx->offsets.ensure(4 * items + 4));
    GSC_HIP(ctx->rec0.ensure(16 * items + 16));
    GSC_HIP(ctx->rec1.ensure(16 * items + 16));
    GSC_HIP(ctx->rec2.ensure(8 * items + 8));
    GSC_HIP(ctx->ranges.ensure(sizeof(uint2) * (tiles + 1)));
    const ViewInfo* dviews = ctx->views.as<ViewInfo>();
    {
        StageTimer t(ctx, s, GSC_STAGE_PROJECT);
        launch_depth_keys(dviews, nv, ni, means, opac, bp, ctx->keys.as<uint32_t>(),
                          ctx->vals.as<uint32_t>(), s);
        GSC_LAUNCHED("depth keys");
    }
    size_t scr = std::max(radix_scratch_words(ni), scan_scratch_words(ni));
    GSC_HIP(ctx->sort_scratch.ensure(4 * scr + 256));
    {
        StageTimer t(ctx, s, GSC_STAGE_DEPTH_SORT);
        radix_sort(ctx->keys.as<uint32_t>(), ctx->vals.as<uint32_t>(), ctx->keys_alt.as<uint32_t>(),
                   ctx->vals_alt.as<uint32_t>(), ni, 32, ctx->sort_scratch.as<uint32_t>(), s);
        GSC_LAUNCHED("depth sort");
    }
    {
        // projection in depth order: records and counts land at the depth rank
        StageTimer t(ctx, s, GSC_STAGE_PROJECT);
        launch_project(dviews, nv, ni, ctx->vals.as<uint32_t>(), ctx->cov.as<float>(), bp,
                       ctx->counts.as<uint32_t>(), ctx->rec0.as<float4>(), ctx->rec1.as<float4>(),
                       ctx->rec2.as<uint2>(), ctx->bin, s);
        GSC_LAUNCHED("project");
    }
    StageTimer* scan_t = new StageTimer(ctx, s, GSC_STAGE_SCAN);
    uint32_t* d_total = reinterpret_cast<uint32_t*>(ctx->misc.as<char>() + 8);
    unsigned long long* d_total64 = reinterpret_cast<unsigned long long*>(ctx->misc.as<char>() + 16);
    launch_fill_u32(reinterpret_cast<uint32_t*>(d_total64), 0u, 2, s);
    launch_sum_u64(ctx->counts.as<uint32_t>(), ni, d_total64, s);
    launch_scan(ctx->counts.as<uint32_t>(), ctx->offsets.as<uint32_t>(), ni, d_total,
                ctx->sort_scratch.as<uint32_t>(), s);
    delete scan_t;
    GSC_LAUNCHED("count scan");
    GSC_HIP(hipMemcpyAsync(ctx->h_total, ctx->misc.as<char>() + 8, 16, hipMemcpyDeviceToHost, s));
    GSC_HIP(hipStreamSynchronize(s));
    uint64_t pairs64 = 0;
    memcpy(&pairs64, reinterpret_cast<const char*>(ctx->h_total) + 8, 8);
    if (pairs64 > batch_pair_limit(ctx->opt) && nv > 1) return kSplit;
    if (pairs64 >= kMaxPairsPerBatch) {
        return fail(GSC_ERR_CAPACITY, "one view produces %llu tile pairs (limit %llu)",
                    (unsigned long long)pairs64, (unsigned long long)kMaxPairsPerBatch);
    }
    const uint64_t pairs = pairs64;
    if (pairs != *ctx->h_total) return fail(GSC_ERR_HIP, "pair count mismatch");
    out->n_pairs = (uint32_t)pairs;
    GSC_HIP(ctx->pkeys.ensure(4 * pairs + 4));
    GSC_HIP(ctx->pvals.ensure(4 * pairs + 4));
    GSC_HIP(ctx->pkeys_alt.ensure(4 * pairs + 4));
    GSC_HIP(ctx->pvals_alt.ensure(4 * pairs + 4));
    {
        StageTimer t(ctx, s, GSC_STAGE_EMIT);
        launch_emit(dviews, nv, ctx->vals.as<uint32_t>(), ctx->offsets.as<uint32_t>(),
                    ctx->counts.as<uint32_t>(), ctx->rec0.as<float4>(),
                    ctx->rec1.as<float4>(), bp, ni, (uint32_t)tiles, ctx->pkeys.as<uint32_t>(),
                    ctx->pvals.as<uint32_t>(), ctx->bin, s);
        GSC_LAUNCHED("emit");
    }
    size_t pscr = radix_scratch_words((uint32_t)pairs);
    GSC_HIP(ctx->sort_scratch.ensure(4 * std::max(pscr, scr) + 256));
    {
        StageTimer t(ctx, s, GSC_STAGE_TILE_SORT);
        bool in_alt = false;
        radix_sort(ctx->pkeys.as<uint32_t>(), ctx->pvals.as<uint32_t>(), ctx->pkeys_alt.as<uint32_t>(),
                   ctx->pvals_alt.as<uint32_t>(), (uint32_t)pairs, bits_for(tiles + 1),
                   ctx->sort_scratch.as<uint32_t>(), s, nullptr, &in_alt);
        GSC_LAUNCHED("tile sort");
        if (in_alt) {  // the sorted pairs are in the alternate buffers: swap roles, no copy
            std::swap(ctx->pkeys, ctx->pkeys_alt);
            std::swap(ctx->pvals, ctx->pvals_alt);
        }
        launch_fill_u32(ctx->ranges.as<uint32_t>(), 0u, (uint64_t)2 * tiles, s);
        launch_tile_ranges(ctx->pkeys.as<uint32_t>(), (uint32_t)pairs, (uint32_t)tiles,
                           ctx->ranges.as<uint2>(), s);
        GSC_LAUNCHED("tile ranges");
        ctx->order_valid = false;
        if (ctx->opt.schedule != GSC_SCHEDULE_GRID) {
            GSC_HIP(ctx->order.ensure(4 * tile_order_words((uint32_t)tiles)));
            launch_tile_order(ctx->ranges.as<uint2>(), (uint32_t)tiles, ctx->order.as<uint32_t>(), s);
            GSC_LAUNCHED("tile order");
            ctx->order_valid = true;
        }
    }
    return GSC_OK;
}

// Run `body(v0, nv, binned)` over consecutive view batches.  A batch holds at
// most batch_item_limit() items (or one view); a batch of several views whose
// tile pairs exceed batch_pair_limit() is halved.
template <typename Body>
gsc_status for_view_batches(gsc_ctx* ctx, const ViewInfo* all, int n_cams,
                            const float* means, const float* opac, int64_t N, const BlendParams& bp,
                            hipStream_t s, Body body, const BinKey* key = nullptr, bool reuse = false) {
    if (reuse) {  // the only batch of the previous call is still in place
        Binned bn;
        bn.n_tiles = ctx->cache_tiles;
        bn.n_pairs = ctx->cache_pairs;
        bn.n_items = ctx->cache_items;
        gsc_status st = body(0, n_cams, bn);
        if (st != GSC_OK) return st;
        ctx->stats.pairs += bn.n_pairs;
        ctx->stats.items += bn.n_items;
        ctx->stats.view_batches += 1;
        return GSC_OK;
    }
    int per = (int)std::max<int64_t>(1, (int64_t)(batch_item_limit(ctx->opt) / (uint64_t)std::max<int64_t>(N, 1)));
    int v = 0, batches = 0;
    ctx->cache_valid = false;
    Binned last;
    while (v < n_cams) {
        int nv = std::min(per, n_cams - v);
        Binned bn;
        gsc_status st = bin_views(ctx, all, v, nv, means, opac, N, bp, s, &bn);
        if (st == kSplit) {
            per = std::max(1, nv / 2);
            continue;
        }
        if (st != GSC_OK) return st;
        if ((st = body(v, nv, bn)) != GSC_OK) return st;
        ctx->stats.pairs += bn.n_pairs;
        ctx->stats.items += bn.n_items;
        ctx->stats.view_batches += 1;
        v += nv;
        ++batches;
        last = bn;
    }
    if (key && batches == 1) {
        ctx->cache_valid = true;
        ctx->cache_key = *key;
        ctx->cache_bin = ctx->bin;
        ctx->cache_tiles = last.n_tiles;
        ctx->cache_pairs = last.n_pairs;
        ctx->cache_items = last.n_items;
    }
    return GSC_OK;
}

template <typename Body>
gsc_status for_view_batches_k(gsc_ctx* ctx, const ViewInfo* all, int n_cams,
                              const float* means, const float* opac, int64_t N, const BlendParams& bp,
                              hipStream_t s, const BinKey* key, bool reuse, Body body) {
    return for_view_batches(ctx, all, n_cams, means, opac, N, bp, s, body, key, reuse);
}

BinKey make_key(const gsc_ctx* ctx, const float* means, const float* scales, const float* quats,
                const float* opac, int64_t N, const gsc_camera* cams, int n_cams, const BlendParams& bp) {
    BinKey k;
    k.means = means;
    k.scales = scales;
    k.quats = quats;
    k.opac = opac;
    k.N = N;
    k.cams.assign(cams, cams + n_cams);
    k.bp = bp;
    k.bin_opt = ctx->opt.bin_size;
    return k;
}

bool can_reuse(const gsc_ctx* ctx, const BinKey& key) {
    return (ctx->opt.flags & GSC_FLAG_REUSE_BINNING) && ctx->cache_valid && ctx->cache_key.same(key);
}

gsc_status ensure_common(gsc_ctx* ctx, const float* means, const float* scales,
                         const float* quats, const float* opac, int64_t N, const gsc_camera* cams,
                         int n_cams, hipStream_t s, bool reuse = false) {
    GSC_HIP(ctx->misc.ensure(kMiscBytes));
    if (!ctx->h_total) GSC_HIP(hipHostMalloc((void**)&ctx->h_total, 64));
    if (reuse) {  // bin size and packed geometry of the cached binning
        ctx->bin = ctx->cache_bin;
        launch_fill_u32(ctx->misc.as<uint32_t>(), 0u, kMiscBytes / 4, s);
        return GSC_OK;
    }
    ctx->bin = ctx->opt.bin_size;
    if (ctx->bin == 0 && ctx->no_alloc) {  // no remembered choice (that would allocate)
        double* d_stats = reinterpret_cast<double*>(ctx->misc.as<char>() + 32);
        launch_geometry_stats(means, scales, N, d_stats, s);
        GSC_LAUNCHED("geometry stats");
        GSC_HIP(hipMemcpyAsync(ctx->h_total, d_stats, 32, hipMemcpyDeviceToHost, s));
        GSC_HIP(hipStreamSynchronize(s));
        double st[4];
        memcpy(st, ctx->h_total, sizeof(st));
        ctx->bin = choose_bin(st, N, cams, n_cams);
    } else if (ctx->bin == 0) {
        BinKey key;
        key.means = means;
        key.scales = scales;
        key.N = N;
        key.cams.assign(cams, cams + n_cams);
        if (ctx->bin_choice != 0 && key.same(ctx->bin_choice_key)) {
            ctx->bin = ctx->bin_choice;
        } else {
            double* d_stats = reinterpret_cast<double*>(ctx->misc.as<char>() + 32);
            launch_geometry_stats(means, scales, N, d_stats, s);
            GSC_LAUNCHED("geometry stats");
            GSC_HIP(hipMemcpyAsync(ctx->h_total, d_stats, 32, hipMemcpyDeviceToHost, s));
            GSC_HIP(hipStreamSynchronize(s));
            double st[4];
            memcpy(st, ctx->h_total, sizeof(st));
            ctx->bin = choose_bin(st, N, cams, n_cams);
            ctx->bin_choice = ctx->bin;
            ctx->bin_choice_key = std::move(key);
        }
    }
    GSC_HIP(ctx->cov.ensure(sizeof(float) * kGeoStride * (size_t)std::max<int64_t>(N, 1)));
    launch_fill_u32(ctx->misc.as<uint32_t>(), 0u, kMiscBytes / 4, s);
    launch_cov3d(means, opac, scales, quats, ctx->cov.as<float>(), N, s);
    GSC_LAUNCHED("cov3d");
    return GSC_OK;
}

// Upload the full camera table to ctx->views_all (used where the views of all
// batches are needed at once: the fold over views).
gsc_status upload_all_views(gsc_ctx* ctx, const ViewInfo* all, int n_cams, hipStream_t s) {
    if (n_cams == 0) return GSC_OK;
    if ((size_t)n_cams > ctx->h_all_cap) {
        if (ctx->h_all) GSC_HIP(hipHostFree(ctx->h_all));
        ctx->h_all = nullptr;
        ctx->h_all_cap = 0;
        GSC_HIP(hipHostMalloc((void**)&ctx->h_all, sizeof(ViewInfo) * (size_t)n_cams));
        ctx->h_all_cap = (size_t)n_cams;
    }
    for (int j = 0; j < n_cams; ++j) ctx->h_all[j] = all[j];
    GSC_HIP(ctx->views_all.ensure(sizeof(ViewInfo) * (size_t)n_cams));
    GSC_HIP(hipMemcpyAsync(ctx->views_all.p, ctx->h_all, sizeof(ViewInfo) * (size_t)n_cams,
                           hipMemcpyHostToDevice, s));
    return GSC_OK;
}

}  // namespace

// A batched multi-scene colorize with every size fixed in advance, so that a
// run allocates nothing, never synchronises and consists of kernel launches
// only (it can be captured into a graph and replayed).
struct gsc_plan {
    gsc_ctx* ctx = nullptr;  // options and profiling
    BlendParams bp;
    std::vector<gsc_scene> scenes;
    const float *means = nullptr, *scales = nullptr, *quats = nullptr, *opac = nullptr;
    int64_t n_total = 0;  // length of the concatenated Gaussian arrays
    int C = 0, sh_deg = 0;
    bool per_view = false;
    struct Batch {
        int v0, nv;
        uint32_t n_items, n_tiles, pair_cap;
        int tile_bits;
    };
    std::vector<Batch> batches;
    std::vector<ViewInfo> views;      // all views, tile_base/item_base local to their batch
    std::vector<int> scene_view0;     // first view of each scene in `views`
    std::vector<int> scene_nviews;    // views of each scene in `views`
    std::vector<int64_t> scene_vs0;   // first per-view slot of each scene
    uint64_t vs_slots = 0;
    uint32_t max_items = 0, max_pairs = 0, max_tiles = 0;
    uint64_t items_total = 0, pairs_total = 0;
    int bin = 16;                     // bin size in pixels
    int acc_chunk = 0;                // accumulate variant (0: default for the targets' type)
    int last_tdtype = GSC_F32;        // target type of the last run
    bool acc_persistent = false;      // persistent work-queue accumulate
    float tune_ms[8] = {};
    int tune_variant[8] = {};
    DevBuf d_views, cov, keys, vals, keys_alt, vals_alt, counts, offsets, rec0, rec1,
        rec2, sort_scratch, pkeys, pvals, pkeys_alt, pvals_alt, ranges, vs, misc, queues, order, obs;
    ~gsc_plan() {
        DevBuf* all[] = {&d_views, &cov, &keys, &vals, &keys_alt, &vals_alt, &counts,
                         &offsets, &rec0, &rec1, &rec2, &sort_scratch, &pkeys, &pvals, &pkeys_alt,
                         &pvals_alt, &ranges, &vs, &misc, &queues, &order, &obs};
        for (DevBuf* b : all) b->release();
    }
};

namespace {
// plan misc layout (device): [0] u64 contributions, [8] u32 live pair count of
// the current batch, [12] u32 dropped-pair events, [16] u32 ill-conditioned
// count, [24] u64 pair total (plan creation), [32..63] geometry statistics
constexpr size_t kPlanMiscBytes = 64;

gsc_status validate_cameras(const gsc_camera* cams, int32_t n_cams) {
    int64_t rows = 0;
    return validate_geometry(nullptr, nullptr, nullptr, nullptr, 0, cams, n_cams, &rows);
}

// Project one batch of the plan and count its tile pairs (synchronises).
gsc_status plan_count_pairs(gsc_plan* P, const gsc_plan::Batch& b, hipStream_t s, uint64_t* pairs) {
    const ViewInfo* dv = P->d_views.as<ViewInfo>() + b.v0;
    launch_project(dv, b.nv, b.n_items, nullptr, P->cov.as<float>(), P->bp,
                   P->counts.as<uint32_t>(), P->rec0.as<float4>(), P->rec1.as<float4>(),
                   P->rec2.as<uint2>(), P->bin, s);
    GSC_LAUNCHED("project");
    unsigned long long* d64 = reinterpret_cast<unsigned long long*>(P->misc.as<char>() + 24);
    launch_fill_u32(reinterpret_cast<uint32_t*>(d64), 0u, 2, s);
    launch_sum_u64(P->counts.as<uint32_t>(), b.n_items, d64, s);
    GSC_LAUNCHED("count");
    uint64_t h = 0;
    GSC_HIP(hipMemcpyAsync(&h, d64, 8, hipMemcpyDeviceToHost, s));
    GSC_HIP(hipStreamSynchronize(s));
    *pairs = h;
    return GSC_OK;
}

// Assign batch-local tile and item numbering to the views of every batch.
void plan_number_views(gsc_plan* P) {
    for (auto& b : P->batches) {
        uint64_t tiles = 0, items = 0;
        bool uniform = true;
        for (int k = 0; k < b.nv; ++k) {
            ViewInfo& v = P->views[b.v0 + k];
            v.tile_base = (uint32_t)tiles;
            v.item_base = (uint32_t)items;
            tiles += (uint64_t)v.tiles_x * v.tiles_y;
            items += v.n_gauss;
            uniform = uniform && v.n_gauss == P->views[b.v0].n_gauss;
        }
        for (int k = 0; k < b.nv; ++k) P->views[b.v0 + k].uniform_n = uniform ? P->views[b.v0].n_gauss : 0u;
        b.n_tiles = (uint32_t)tiles;
        b.n_items = (uint32_t)items;
        b.tile_bits = bits_for(tiles + 1);
    }
}

gsc_status plan_accumulate(gsc_plan* P, const gsc_plan::Batch& b, const void* targets, int tdtype,
                           int chunk, bool persistent, hipStream_t s) {
    const ViewInfo* dv = P->d_views.as<ViewInfo>() + b.v0;
    unsigned long long* d_counter = reinterpret_cast<unsigned long long*>(P->misc.p);
    launch_accumulate_chunked(dv, b.nv, b.n_tiles, P->ranges.as<uint2>(), P->pvals.as<uint32_t>(),
                              P->rec0.as<float4>(), P->rec1.as<float4>(), P->rec2.as<uint2>(),
                              P->bin, targets, tdtype, P->C,
                              P->per_view, P->bp, P->vs.as<float>(), d_counter, nullptr, chunk, s,
                              persistent ? P->queues.as<uint32_t>() : nullptr,
                              P->order.as<uint32_t>() + b.n_tiles);
    GSC_LAUNCHED("accumulate");
    return GSC_OK;
}

// Everything of one batch up to the tile lists, enqueued without host reads.
gsc_status plan_bin_batch(gsc_plan* P, const gsc_plan::Batch& b, hipStream_t s) {
    gsc_ctx* ctx = P->ctx;
    const ViewInfo* dv = P->d_views.as<ViewInfo>() + b.v0;
    uint32_t* d_live = reinterpret_cast<uint32_t*>(P->misc.as<char>() + 8);
    uint32_t* d_drop = reinterpret_cast<uint32_t*>(P->misc.as<char>() + 12);
    {
        StageTimer t(ctx, s, GSC_STAGE_PROJECT);
        launch_depth_keys(dv, b.nv, b.n_items, P->means, P->opac, P->bp, P->keys.as<uint32_t>(),
                          P->vals.as<uint32_t>(), s);
        GSC_LAUNCHED("depth keys");
    }
    {
        StageTimer t(ctx, s, GSC_STAGE_DEPTH_SORT);
        radix_sort(P->keys.as<uint32_t>(), P->vals.as<uint32_t>(), P->keys_alt.as<uint32_t>(),
                   P->vals_alt.as<uint32_t>(), b.n_items, 32, P->sort_scratch.as<uint32_t>(), s);
        GSC_LAUNCHED("depth sort");
    }
    {
        StageTimer t(ctx, s, GSC_STAGE_PROJECT);
        launch_project(dv, b.nv, b.n_items, P->vals.as<uint32_t>(), P->cov.as<float>(),
                       P->bp, P->counts.as<uint32_t>(), P->rec0.as<float4>(), P->rec1.as<float4>(),
                       P->rec2.as<uint2>(), P->bin, s);
        GSC_LAUNCHED("project");
    }
    {
        StageTimer t(ctx, s, GSC_STAGE_SCAN);
        launch_scan(P->counts.as<uint32_t>(), P->offsets.as<uint32_t>(), b.n_items, d_live,
                    P->sort_scratch.as<uint32_t>(), s);
        GSC_LAUNCHED("count scan");
    }
    {
        StageTimer t(ctx, s, GSC_STAGE_EMIT);
        launch_emit(dv, b.nv, P->vals.as<uint32_t>(), P->offsets.as<uint32_t>(),
                    P->counts.as<uint32_t>(), P->rec0.as<float4>(), P->rec1.as<float4>(), P->bp,
                    b.n_items, b.n_tiles, P->pkeys.as<uint32_t>(), P->pvals.as<uint32_t>(), P->bin, s,
                    b.pair_cap, d_drop);
        GSC_LAUNCHED("emit");
    }
    {
        StageTimer t(ctx, s, GSC_STAGE_TILE_SORT);
        bool in_alt = false;
        radix_sort(P->pkeys.as<uint32_t>(), P->pvals.as<uint32_t>(), P->pkeys_alt.as<uint32_t>(),
                   P->pvals_alt.as<uint32_t>(), b.pair_cap, b.tile_bits,
                   P->sort_scratch.as<uint32_t>(), s, d_live, &in_alt);
        if (in_alt) {  // swap roles instead of copying; every run swaps alike
            std::swap(P->pkeys, P->pkeys_alt);
            std::swap(P->pvals, P->pvals_alt);
        }
        launch_fill_u32(P->ranges.as<uint32_t>(), 0u, (uint64_t)2 * b.n_tiles, s);
        launch_tile_ranges(P->pkeys.as<uint32_t>(), b.pair_cap, b.n_tiles, P->ranges.as<uint2>(), s,
                           d_live);
        launch_tile_order(P->ranges.as<uint2>(), b.n_tiles, P->order.as<uint32_t>(), s);
        GSC_LAUNCHED("tile sort");
    }
    return GSC_OK;
}

gsc_status plan_solve(gsc_plan* P, const double* lam, float* coeffs, uint8_t* status, hipStream_t s) {
    gsc_ctx* ctx = P->ctx;
    StageTimer t(ctx, s, GSC_STAGE_SOLVE);
    unsigned int* d_ill = reinterpret_cast<unsigned int*>(P->misc.as<char>() + 16);
    const int nb = (P->sh_deg + 1) * (P->sh_deg + 1);
    if (!P->per_view) {
        launch_fold_solve(nullptr, 0, P->means, P->vs.as<float>(), false, P->n_total, P->C, 0, lam,
                          ctx->opt.kappa_max, coeffs, status, nullptr, nullptr, d_ill, s);
        GSC_LAUNCHED("solve");
        return GSC_OK;
    }
    for (size_t k = 0; k < P->scenes.size(); ++k) {
        const gsc_scene& sc = P->scenes[k];
        if (sc.n_gaussians == 0) continue;
        launch_fold_solve(P->d_views.as<ViewInfo>() + P->scene_view0[k], P->scene_nviews[k],
                          P->means + 3 * sc.gaussian_offset,
                          P->vs.as<float>() + P->scene_vs0[k] * (P->C + 1), true, sc.n_gaussians,
                          P->C, P->sh_deg, lam, ctx->opt.kappa_max,
                          coeffs + sc.gaussian_offset * nb * P->C,
                          status ? status + sc.gaussian_offset : nullptr, nullptr, nullptr, d_ill, s,
                          nullptr, P->obs.as<uint32_t>());
        GSC_LAUNCHED("fold/solve");
    }
    return GSC_OK;
}

gsc_status plan_run(gsc_plan* P, const void* targets, int tdtype, const double* lam, float* coeffs,
                    uint8_t* status, hipStream_t s) {
    P->last_tdtype = tdtype;
    launch_fill_u32(P->misc.as<uint32_t>(), 0u, 6, s);
    launch_fill_u32(P->vs.as<uint32_t>(), 0u, P->vs_slots * (uint64_t)(P->C + 1), s);
    launch_cov3d(P->means, P->opac, P->scales, P->quats, P->cov.as<float>(), P->n_total, s);
    GSC_LAUNCHED("cov3d");
    for (const auto& b : P->batches) {
        gsc_status st = plan_bin_batch(P, b, s);
        if (st != GSC_OK) return st;
        StageTimer t(P->ctx, s, GSC_STAGE_BLEND);
        const int chunk = P->acc_chunk ? P->acc_chunk : P->ctx->opt.accumulate_variant;
        if ((st = plan_accumulate(P, b, targets, tdtype, chunk, P->acc_persistent, s)) != GSC_OK)
            return st;
    }
    return plan_solve(P, lam, coeffs, status, s);
}

}  // namespace

extern "C" {

gsc_status gsc_default_options(gsc_options* out) {
    if (!out) return fail(GSC_ERR_INVALID_ARG, "null options");
    out->alpha_min = 1.0f / 255.0f;
    out->alpha_max = 0.99f;
    out->t_min = 1e-4f;
    out->sigma_cut = 3.0f;
    out->dilation = 0.3f;
    out->znear = 0.01f;
    out->kappa_max = 1e6f;
    out->flags = 0;
    out->bin_size = 0;
    out->accumulate_variant = 0;
    out->schedule = GSC_SCHEDULE_AUTO;
    out->profile_stages = 0u;
    out->batch_items = 0u;
    out->batch_pairs = 0u;
    return GSC_OK;
}

gsc_status gsc_ctx_create(gsc_ctx** ctx, const gsc_options* opt) {
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx pointer");
    *ctx = nullptr;
    gsc_options o;
    gsc_default_options(&o);
    if (opt) o = *opt;
    gsc_status st = validate_options(&o);
    if (st != GSC_OK) return st;
    gsc_ctx* c = new (std::nothrow) gsc_ctx();
    if (!c) return fail(GSC_ERR_HIP, "out of host memory");
    c->opt = o;
    memset(&c->stats, 0, sizeof(c->stats));
    *ctx = c;
    return GSC_OK;
}

void gsc_ctx_destroy(gsc_ctx* ctx) { delete ctx; }

gsc_status gsc_ctx_set_options(gsc_ctx* ctx, const gsc_options* opt) {
    if (!ctx || !opt) return fail(GSC_ERR_INVALID_ARG, "null ctx or options");
    gsc_status st = validate_options(opt);
    if (st != GSC_OK) return st;
    ctx->opt = *opt;
    return GSC_OK;
}

}  // extern "C"

namespace {

// Validation shared by the colorize entry points.
gsc_status validate_colorize(const float* means, const float* scales, const float* quats,
                             const float* opacities, int64_t N, const gsc_camera* cams,
                             int32_t n_cams, const void* targets, int32_t tdtype, int32_t C,
                             int32_t sh_deg, const float* lambda, int32_t n_lambda, float* coeffs,
                             double* lam) {
    int64_t rows = 0;
    gsc_status st = validate_geometry(means, scales, quats, opacities, N, cams, n_cams, &rows);
    if (st != GSC_OK) return st;
    if ((st = validate_channels(C, sh_deg)) != GSC_OK) return st;
    if (tdtype != GSC_F32 && tdtype != GSC_BF16) return fail(GSC_ERR_INVALID_ARG, "tdtype must be GSC_F32 or GSC_BF16");
    if (rows > 0 && !targets) return fail(GSC_ERR_INVALID_ARG, "targets is null");
    if (N > 0 && !coeffs) return fail(GSC_ERR_INVALID_ARG, "coeffs is null");
    return expand_lambda(lambda, n_lambda, sh_deg, lam);
}

// The colorize pipeline on validated arguments (N > 0).  `all` holds n_cams
// view slots, filled here.  key / reuse: binning reuse (key may be null).
// One array to scan for non-finite values (GSC_FLAG_CHECK_FINITE) and for
// its largest magnitude.
struct ScanSeg {
    const char* name;
    const void* p;
    int dtype;
    int64_t n;
    int per;  // values per entity (Gaussian or target row), for the message
};

// Scans the segments on `s`, reads the results back (synchronising `s`) and
// fails with GSC_ERR_INVALID_ARG naming the first segment that holds a
// non-finite value.  absmax (optional): the largest |value| of each segment.
gsc_status scan_inputs(gsc_ctx* ctx, const ScanSeg* seg, int n_seg, hipStream_t s, float* absmax) {
    constexpr int kMaxSeg = 8;
    if (n_seg > kMaxSeg) return fail(GSC_ERR_INVALID_ARG, "too many arrays to scan");
    GSC_HIP(ctx->chk.ensure(16 * kMaxSeg));
    unsigned long long* bad = ctx->chk.as<unsigned long long>();
    uint32_t* mx = reinterpret_cast<uint32_t*>(bad + kMaxSeg);
    launch_fill_u32(reinterpret_cast<uint32_t*>(bad), 0xffffffffu, 2 * kMaxSeg, s);
    launch_fill_u32(mx, 0u, kMaxSeg, s);
    for (int i = 0; i < n_seg; ++i) launch_scan_values(seg[i].p, seg[i].dtype, seg[i].n, bad + i, mx + i, s);
    GSC_LAUNCHED("input scan");
    unsigned long long h[kMaxSeg + kMaxSeg / 2];
    GSC_HIP(hipMemcpyAsync(h, bad, 12 * kMaxSeg, hipMemcpyDeviceToHost, s));
    GSC_HIP(hipStreamSynchronize(s));
    const uint32_t* hm = reinterpret_cast<const uint32_t*>(h + kMaxSeg);
    for (int i = 0; i < n_seg; ++i) {
        if (h[i] != ~0ull)
            return fail(GSC_ERR_INVALID_ARG, "%s holds a non-finite value at element %llu (entry %llu)",
                        seg[i].name, h[i], h[i] / (unsigned long long)seg[i].per);
        if (absmax) {
            float f;
            memcpy(&f, &hm[i], 4);
            absmax[i] = f;
        }
    }
    return GSC_OK;
}

// Fixed-point scales of the deterministic per-view sums: a power of two per
// column kind such that no slot can exceed 2^62 in magnitude.  A slot sums
// one view's pixels, each with weight <= 1: V <= pixels and |S| <= pixels *
// max|y|.
float2 det_scales(const gsc_camera* cams, int n_cams, float ymax) {
    double P = 1.0;
    for (int j = 0; j < n_cams; ++j) P = std::max(P, (double)cams[j].width * cams[j].height);
    auto pow2_for = [](double bound) {
        int e = 62 - (int)ceil(log2(std::max(bound, 1e-30)));
        e = std::min(std::max(e, -126), 126);
        return ldexpf(1.0f, e);
    };
    const float sv = pow2_for(P);
    const float ss = ymax > 0.0f ? pow2_for(P * (double)ymax) : sv;
    return make_float2(sv, ss);
}

gsc_status colorize_core(gsc_ctx* ctx, const float* means, const float* scales,
                         const float* quats, const float* opacities, int64_t N,
                         const gsc_camera* cams, int32_t n_cams, const void* targets,
                         int32_t tdtype, int32_t C, int32_t sh_deg, const double* lam,
                         float* coeffs, uint8_t* status, const gsc_extras* extras, hipStream_t s,
                         const BinKey* key, bool reuse, ViewInfo* all, double* factor = nullptr) {
    gsc_status st;
    float* x_sums = extras ? extras->view_sums : nullptr;
    float* x_vis = extras ? extras->visibility : nullptr;
    uint32_t* x_cnt = extras ? extras->counts : nullptr;
    BlendParams bp = blend_params(ctx->opt);
    const bool det = (ctx->opt.flags & GSC_FLAG_DETERMINISTIC) != 0;
    float2 dsc = make_float2(0.f, 0.f);
    if ((ctx->opt.flags & GSC_FLAG_CHECK_FINITE) || det) {
        int64_t rows = 0;
        for (int j = 0; j < n_cams; ++j)
            rows = std::max<int64_t>(rows, cams[j].pixel_offset + (int64_t)cams[j].width * cams[j].height);
        const ScanSeg all_segs[5] = {{"targets", targets, tdtype, rows * C, C},
                                     {"means", means, GSC_F32, 3 * N, 3},
                                     {"scales", scales, GSC_F32, 3 * N, 3},
                                     {"quats", quats, GSC_F32, 4 * N, 4},
                                     {"opacities", opacities, GSC_F32, N, 1}};
        const int n_seg = (ctx->opt.flags & GSC_FLAG_CHECK_FINITE) ? 5 : 1;
        float mx[5] = {0, 0, 0, 0, 0};
        if ((st = scan_inputs(ctx, all_segs, n_seg, s, mx)) != GSC_OK) return st;
        dsc = det_scales(cams, n_cams, mx[0]);
    }
    if ((st = ensure_common(ctx, means, scales, quats, opacities, N, cams, n_cams, s, reuse)) != GSC_OK) return st;
    for (int j = 0; j < n_cams; ++j) all[j] = make_view(cams[j], j, N, ctx->bin);
    // the deterministic sums keep one slot per view (a slot summed over all
    // views would need a coarser fixed-point step)
    const bool per_view = sh_deg > 0 || x_sums != nullptr || det;
    const uint64_t vs_words = (uint64_t)(per_view ? std::max(n_cams, 1) : 1) * (uint64_t)N * (uint64_t)(C + 1);
    GSC_HIP(ctx->vs.ensure(4 * vs_words));
    float* acc_vs = ctx->vs.as<float>();
    if (det) {
        GSC_HIP(ctx->vsdet.ensure(8 * vs_words));
        launch_fill_u32(ctx->vsdet.as<uint32_t>(), 0u, 2 * vs_words, s);
        acc_vs = ctx->vsdet.as<float>();  // 64-bit words, see launch_accumulate_chunked
    } else {
        launch_fill_u32(ctx->vs.as<uint32_t>(), 0u, vs_words, s);
    }
    if (x_cnt) launch_fill_u32(x_cnt, 0u, (uint64_t)N, s);
    unsigned long long* d_counter = reinterpret_cast<unsigned long long*>(ctx->misc.p);
    st = for_view_batches_k(ctx, all, n_cams, means, opacities, N, bp, s, key, reuse,
                          [&](int v0, int nv, const Binned& bn) -> gsc_status {
        const int chunk = resolve_chunk(ctx->opt.accumulate_variant, C, tdtype);
        StageTimer t(ctx, s, GSC_STAGE_BLEND, (uint32_t)accumulate_launches(C, chunk));
        (void)v0;
        // Tiles in the longest-first order: the vector form as a grid whose
        // blocks map to tiles through the order (the hardware dispatches
        // blocks in index order), the matrix-core form as a persistent grid
        // taking tiles from a work queue (each measured the faster for it).
        uint32_t* queues = nullptr;
        const uint32_t* order = tile_order(ctx, bn.n_tiles);
        if (order != nullptr && (chunk & kChunkMfma)) {
            GSC_HIP(ctx->queues.ensure(4 * (size_t)(kMaxC + 1)));
            queues = ctx->queues.as<uint32_t>();
        }
        launch_accumulate_chunked(ctx->views.as<ViewInfo>(), nv, bn.n_tiles, ctx->ranges.as<uint2>(),
                                  ctx->pvals.as<uint32_t>(), ctx->rec0.as<float4>(), ctx->rec1.as<float4>(),
                                  ctx->rec2.as<uint2>(), ctx->bin, targets, tdtype, C, per_view, bp,
                                  acc_vs, d_counter, x_cnt, chunk, s, queues, order, det ? &dsc : nullptr);
        GSC_LAUNCHED("accumulate");
        return GSC_OK;
    });
    if (st != GSC_OK) return st;
    if (det) {
        launch_det_to_float(ctx->vsdet.as<unsigned long long>(), (int64_t)vs_words, C + 1, 1.0 / dsc.x,
                            1.0 / dsc.y, ctx->vs.as<float>(), s);
        GSC_LAUNCHED("deterministic sums");
    }
    if (x_sums && n_cams > 0)
        GSC_HIP(hipMemcpyAsync(x_sums, ctx->vs.p, 4 * vs_words, hipMemcpyDeviceToDevice, s));
    // fold + solve needs the full camera table (only the camera centres are used)
    if (per_view && (st = upload_all_views(ctx, all, n_cams, s)) != GSC_OK) return st;
    float* dc_scratch = nullptr;
    if (sh_deg == 0 && per_view) {
        GSC_HIP(ctx->gamma.ensure(4 * (size_t)N * (size_t)(C + 1)));
        dc_scratch = ctx->gamma.as<float>();
    }
    unsigned int* d_ill = reinterpret_cast<unsigned int*>(ctx->misc.as<char>() + 12);
    uint32_t* obs = nullptr;
    if (sh_deg > 0) {
        GSC_HIP(ctx->obs.ensure(4 * (size_t)fold_obs_words(N)));
        obs = ctx->obs.as<uint32_t>();
    }
    StageTimer t_solve(ctx, s, GSC_STAGE_SOLVE);
    launch_fold_solve(ctx->views_all.as<ViewInfo>(), per_view ? n_cams : 0, means, ctx->vs.as<float>(),
                      per_view, N, C, sh_deg, lam, ctx->opt.kappa_max, coeffs, status, x_vis,
                      dc_scratch, d_ill, s, factor, obs);
    GSC_LAUNCHED("fold/solve");
    ctx->stats_pending = true;
    ctx->stats_dev = nullptr;
    return GSC_OK;
}

}  // namespace

// The scratch of the allocation-free colorize: one fixed array per GPU.  Host
// code must not use the name as an address; kernels receive the device
// address that hipGetSymbolAddress returns for the current device.
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) char scratch[kNoallocScratchBytes];

namespace {

// ---- allocation-free colorize ---------------------------------------------
//
// Every scratch buffer of gsc_colorize_noalloc is carved from `scratch`, a
// fixed array in device memory that each GPU holds once the library is loaded
// (its address is looked up once per device); the host staging of the view
// tables lives in static arrays.  Calls share both: they are serialised on the
// host by a mutex, and calls on one GPU from different processes race.
constexpr int kNoallocMaxViews = 1024;
constexpr int kNoallocMaxDevices = 64;

std::mutex g_noalloc_mu;
void* g_scratch_ptr[kNoallocMaxDevices];  // device address of `scratch` per device
ViewInfo g_noalloc_table[kNoallocMaxViews];
ViewInfo g_noalloc_batch[kNoallocMaxViews];
ViewInfo g_noalloc_upload[kNoallocMaxViews];
uint32_t g_noalloc_total[16];

// Device address of `scratch` on the current device (under g_noalloc_mu).
gsc_status noalloc_scratch(void** out) {
    int dev = 0;
    GSC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kNoallocMaxDevices) return fail(GSC_ERR_UNSUPPORTED, "device %d out of range", dev);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        GSC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(GSC_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return GSC_OK;
}

}  // namespace

extern "C" {

gsc_status gsc_colorize_ex(gsc_ctx* ctx, const float* means, const float* scales,
                           const float* quats, const float* opacities, int64_t N,
                           const gsc_camera* cams, int32_t n_cams, const void* targets,
                           int32_t tdtype, int32_t C, int32_t sh_deg, const float* lambda,
                           int32_t n_lambda, float* coeffs, uint8_t* status,
                           const gsc_extras* extras, gsc_stream_t stream) {
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx");
    double lam[kMaxNb];
    gsc_status st = validate_colorize(means, scales, quats, opacities, N, cams, n_cams, targets,
                                      tdtype, C, sh_deg, lambda, n_lambda, coeffs, lam);
    if (st != GSC_OK) return st;
    if (ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = refuse_capture(s, "gsc_colorize")) != GSC_OK) return st;
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    if (N == 0) return GSC_OK;
    const BinKey key = make_key(ctx, means, scales, quats, opacities, N, cams, n_cams, blend_params(ctx->opt));
    const bool reuse = can_reuse(ctx, key);
    std::vector<ViewInfo> all(std::max(n_cams, 1));
    return colorize_core(ctx, means, scales, quats, opacities, N, cams, n_cams, targets, tdtype, C,
                         sh_deg, lam, coeffs, status, extras, s, &key, reuse, all.data());
}

gsc_status gsc_colorize_noalloc(gsc_ctx* ctx, const float* means, const float* scales,
                                const float* quats, const float* opacities, int64_t N,
                                const gsc_camera* cams, int32_t n_cams, const void* targets,
                                int32_t tdtype, int32_t C, int32_t sh_deg, const float* lambda,
                                int32_t n_lambda, float* coeffs, uint8_t* status,
                                gsc_stream_t stream) {
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx");
    double lam[kMaxNb];
    gsc_status st = validate_colorize(means, scales, quats, opacities, N, cams, n_cams, targets,
                                      tdtype, C, sh_deg, lambda, n_lambda, coeffs, lam);
    if (st != GSC_OK) return st;
    if (n_cams > kNoallocMaxViews)
        return fail(GSC_ERR_CAPACITY, "gsc_colorize_noalloc takes at most %d cameras (got %d)",
                    kNoallocMaxViews, n_cams);
    // what is known before binning: view tables, geometry records, per-item
    // keys, counts and records, and the per-view sums
    const uint64_t items = (uint64_t)N * (uint64_t)n_cams;
    const uint64_t vs_words = (uint64_t)(sh_deg > 0 ? std::max(n_cams, 1) : 1) * (uint64_t)N * (uint64_t)(C + 1);
    const uint64_t known = 2 * sizeof(ViewInfo) * (uint64_t)n_cams + 4ull * kGeoStride * (uint64_t)N +
                           64ull * items + 4 * vs_words + (sh_deg > 0 ? 4ull * fold_obs_words(N) : 0);
    if (known > kNoallocScratchBytes)
        return fail(GSC_ERR_CAPACITY,
                    "gsc_colorize_noalloc: %llu Gaussians x %d views x %d channels need at least %llu "
                    "bytes of scratch before binning; the static scratch holds %llu",
                    (unsigned long long)N, n_cams, C, (unsigned long long)known,
                    (unsigned long long)kNoallocScratchBytes);
    if (ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = refuse_capture(s, "gsc_colorize_noalloc")) != GSC_OK) return st;
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    ctx->stats_pending = false;
    if (N == 0) return GSC_OK;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    void* base = nullptr;
    if ((st = noalloc_scratch(&base)) != GSC_OK) return st;
    // a working context whose buffers are all carved from the scratch
    Arena arena;
    arena.base = static_cast<char*>(base);
    arena.cap = kNoallocScratchBytes;
    gsc_ctx w;
    for (DevBuf* b : w.bufs()) b->arena = &arena;
    w.no_alloc = true;
    w.h_views = g_noalloc_batch;
    w.h_views_cap = kNoallocMaxViews;
    w.h_all = g_noalloc_upload;
    w.h_all_cap = kNoallocMaxViews;
    w.h_total = g_noalloc_total;
    w.opt = ctx->opt;
    w.opt.flags &= ~(GSC_FLAG_PROFILE | GSC_FLAG_REUSE_BINNING | GSC_FLAG_DETERMINISTIC);
    memset(&w.stats, 0, sizeof(w.stats));
    st = colorize_core(&w, means, scales, quats, opacities, N, cams, n_cams, targets, tdtype, C,
                       sh_deg, lam, coeffs, status, nullptr, s, nullptr, false, g_noalloc_table);
    if (st != GSC_OK) {
        if (arena.need > 0)
            return fail(GSC_ERR_CAPACITY,
                        "gsc_colorize_noalloc: the call needs more than the %llu-byte static scratch "
                        "(a buffer would have ended at byte %llu)",
                        (unsigned long long)kNoallocScratchBytes, (unsigned long long)arena.need);
        return st;
    }
    ctx->stats = w.stats;
    ctx->bin = w.bin;
    ctx->stats_pending = true;
    ctx->stats_dev = w.misc.p;  // inside the scratch: valid until the next call on this GPU
    return GSC_OK;
}

gsc_status gsc_colorize(gsc_ctx* ctx, const float* means, const float* scales, const float* quats,
                        const float* opacities, int64_t N, const gsc_camera* cams, int32_t n_cams,
                        const void* targets, int32_t tdtype, int32_t C, int32_t sh_deg,
                        const float* lambda, int32_t n_lambda, float* coeffs, uint8_t* status,
                        gsc_stream_t stream) {
    return gsc_colorize_ex(ctx, means, scales, quats, opacities, N, cams, n_cams, targets, tdtype,
                           C, sh_deg, lambda, n_lambda, coeffs, status, nullptr, stream);
}

gsc_status gsc_colorize_refine(gsc_ctx* ctx, const float* means, const float* scales,
                               const float* quats, const float* opacities, int64_t N,
                               const gsc_camera* cams, int32_t n_cams, const void* targets,
                               int32_t tdtype, int32_t C, int32_t sh_deg, const float* lambda,
                               int32_t n_lambda, int32_t n_refine, float* coeffs, uint8_t* status,
                               gsc_stream_t stream) {
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx");
    double lam[kMaxNb];
    gsc_status st = validate_colorize(means, scales, quats, opacities, N, cams, n_cams, targets,
                                      tdtype, C, sh_deg, lambda, n_lambda, coeffs, lam);
    if (st != GSC_OK) return st;
    if (n_refine < 0 || n_refine > 10000) return fail(GSC_ERR_INVALID_ARG, "n_refine must be in [0, 10000] (got %d)", n_refine);
    if (ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = refuse_capture(s, "gsc_colorize_refine")) != GSC_OK) return st;
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    if (N == 0) return GSC_OK;
    const BinKey key = make_key(ctx, means, scales, quats, opacities, N, cams, n_cams, blend_params(ctx->opt));
    const bool reuse = can_reuse(ctx, key);
    std::vector<ViewInfo> all(std::max(n_cams, 1));
    // first pass (Algorithm 1, steps 1-6), keeping w_g, the statuses and the factor
    GSC_HIP(ctx->wbuf.ensure(4 * (size_t)N));
    if (!status) {
        GSC_HIP(ctx->stat.ensure((size_t)N));
        status = ctx->stat.as<uint8_t>();
    }
    double* factor = nullptr;
    if (sh_deg > 0) {
        GSC_HIP(ctx->factor.ensure(8 * (size_t)N * (size_t)refine_factor_words(sh_deg)));
        factor = ctx->factor.as<double>();
    }
    gsc_extras ex;
    ex.view_sums = nullptr;
    ex.visibility = ctx->wbuf.as<float>();
    ex.counts = nullptr;
    st = colorize_core(ctx, means, scales, quats, opacities, N, cams, n_cams, targets, tdtype, C,
                       sh_deg, lam, coeffs, status, &ex, s, &key, reuse, all.data(), factor);
    if (st != GSC_OK || n_refine == 0 || n_cams == 0) return st;
    // refinement passes (steps 8-10): render, residual, accumulate, update.
    // The binning of a call with one view batch stays in place; otherwise each
    // pass bins every batch again (once for its render and accumulate).
    const bool single = ctx->cache_valid && ctx->cache_key.same(key);
    const int nb = (sh_deg + 1) * (sh_deg + 1);
    const int kc = nb * C;
    const bool per_view = sh_deg > 0;
    int64_t rows = 0;
    for (int j = 0; j < n_cams; ++j) rows = std::max<int64_t>(rows, cams[j].pixel_offset + (int64_t)cams[j].width * cams[j].height);
    GSC_HIP(ctx->coef_t.ensure(4 * (size_t)N * (size_t)kc));
    GSC_HIP(ctx->img.ensure(4 * (size_t)rows * (size_t)C));
    const uint64_t vs_words = (uint64_t)(per_view ? n_cams : 1) * (uint64_t)N * (uint64_t)(C + 1);
    BlendParams bp = blend_params(ctx->opt);
    // the passes count their contributions apart: the statistics stay the first pass's
    unsigned long long* d_pass_counter = reinterpret_cast<unsigned long long*>(ctx->misc.as<char>() + 24);
    const int chunk = resolve_chunk(ctx->opt.accumulate_variant, C, GSC_F32);
    const gsc_stats first = ctx->stats;
    for (int step = 0; step < n_refine; ++step) {
        launch_transpose(coeffs, N, kc, ctx->coef_t.as<float>(), s);
        launch_fill_u32(ctx->vs.as<uint32_t>(), 0u, vs_words, s);
        GSC_LAUNCHED("refinement setup");
        st = for_view_batches(ctx, all.data(), n_cams, means, opacities, N, bp, s,
                              [&](int v0, int nv, const Binned& bn) -> gsc_status {
            GSC_HIP(ctx->gamma.ensure(4 * (size_t)nv * (size_t)N * (size_t)C));
            int max_px = 0;
            for (int k = 0; k < nv; ++k) max_px = std::max(max_px, all[v0 + k].width * all[v0 + k].height);
            const uint32_t* order = tile_order(ctx, bn.n_tiles);
            StageTimer t(ctx, s, GSC_STAGE_BLEND);
            launch_view_colors(ctx->views.as<ViewInfo>(), nv, (uint32_t)bn.n_items, means,
                               ctx->coef_t.as<float>(), N, C, sh_deg, ctx->gamma.as<float>(), s);
            launch_render(ctx->views.as<ViewInfo>(), nv, bn.n_tiles, ctx->ranges.as<uint2>(),
                          ctx->pvals.as<uint32_t>(), ctx->rec0.as<float4>(), ctx->rec1.as<float4>(),
                          ctx->rec2.as<uint2>(), ctx->bin, ctx->gamma.as<float>(), C, bp,
                          ctx->img.as<float>(), d_pass_counter, s, order);
            launch_residual(ctx->views.as<ViewInfo>(), nv, max_px, targets, tdtype, C, ctx->img.as<float>(), s);
            uint32_t* queues = nullptr;
            if (order != nullptr && (chunk & kChunkMfma)) {
                GSC_HIP(ctx->queues.ensure(4 * (size_t)(kMaxC + 1)));
                queues = ctx->queues.as<uint32_t>();
            }
            launch_accumulate_chunked(ctx->views.as<ViewInfo>(), nv, bn.n_tiles, ctx->ranges.as<uint2>(),
                                      ctx->pvals.as<uint32_t>(), ctx->rec0.as<float4>(),
                                      ctx->rec1.as<float4>(), ctx->rec2.as<uint2>(), ctx->bin,
                                      ctx->img.as<float>(), GSC_F32, C, per_view, bp, ctx->vs.as<float>(),
                                      d_pass_counter, nullptr, chunk, s, queues, order);
            GSC_LAUNCHED("refinement pass");
            (void)v0;
            return GSC_OK;
        }, &key, single);
        if (st != GSC_OK) return st;
        StageTimer t(ctx, s, GSC_STAGE_SOLVE);
        launch_refine_update(ctx->views_all.as<ViewInfo>(), n_cams, means, ctx->vs.as<float>(), N, C,
                             sh_deg, lam, factor, ctx->wbuf.as<float>(), status, coeffs, s);
        GSC_LAUNCHED("refinement update");
    }
    // statistics of the first pass (batches and pairs counted once)
    const gsc_stats last = ctx->stats;
    ctx->stats = first;
    for (int i = 0; i < GSC_N_STAGES; ++i) ctx->stats.stage_ms[i] = last.stage_ms[i];
    ctx->stats_pending = true;
    ctx->stats_dev = nullptr;
    return GSC_OK;
}

gsc_status gsc_render(gsc_ctx* ctx, const float* means, const float* scales, const float* quats,
                      const float* opacities, int64_t N, const gsc_camera* cams, int32_t n_cams,
                      const float* coeffs, int32_t C, int32_t sh_deg, float* images,
                      gsc_stream_t stream) {
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx");
    int64_t rows = 0;
    gsc_status st = validate_geometry(means, scales, quats, opacities, N, cams, n_cams, &rows);
    if (st != GSC_OK) return st;
    if ((st = validate_channels(C, sh_deg)) != GSC_OK) return st;
    if (rows > 0 && !images) return fail(GSC_ERR_INVALID_ARG, "images is null");
    if (N > 0 && !coeffs) return fail(GSC_ERR_INVALID_ARG, "coeffs is null");
    if (ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = refuse_capture(s, "gsc_render")) != GSC_OK) return st;
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    if (n_cams == 0) return GSC_OK;
    BlendParams bp = blend_params(ctx->opt);
    const BinKey key = make_key(ctx, means, scales, quats, opacities, N, cams, n_cams, bp);
    const bool reuse = can_reuse(ctx, key);
    if ((st = ensure_common(ctx, means, scales, quats, opacities, N, cams, n_cams, s, reuse)) != GSC_OK) return st;
    std::vector<ViewInfo> all(n_cams);
    for (int j = 0; j < n_cams; ++j) all[j] = make_view(cams[j], j, N, ctx->bin);
    unsigned long long* d_counter = reinterpret_cast<unsigned long long*>(ctx->misc.p);
    const int kc = (sh_deg + 1) * (sh_deg + 1) * C;
    GSC_HIP(ctx->coef_t.ensure(4 * (size_t)std::max<int64_t>(N, 1) * (size_t)kc));
    launch_transpose(coeffs, N, kc, ctx->coef_t.as<float>(), s);
    GSC_LAUNCHED("transpose");
    st = for_view_batches_k(ctx, all.data(), n_cams, means, opacities, N, bp, s, &key, reuse,
                          [&](int v0, int nv, const Binned& bn) -> gsc_status {
        (void)v0;
        StageTimer t(ctx, s, GSC_STAGE_BLEND, 1 + (uint32_t)((C + 3) / 4));
        GSC_HIP(ctx->gamma.ensure(4 * (size_t)nv * (size_t)std::max<int64_t>(N, 1) * (size_t)C));
        launch_view_colors(ctx->views.as<ViewInfo>(), nv, (uint32_t)bn.n_items, means,
                           ctx->coef_t.as<float>(), N, C, sh_deg, ctx->gamma.as<float>(), s);
        GSC_LAUNCHED("view colors");
        launch_render(ctx->views.as<ViewInfo>(), nv, bn.n_tiles, ctx->ranges.as<uint2>(),
                      ctx->pvals.as<uint32_t>(), ctx->rec0.as<float4>(), ctx->rec1.as<float4>(), ctx->rec2.as<uint2>(), ctx->bin,
                      ctx->gamma.as<float>(), C, bp, images, d_counter, s, tile_order(ctx, bn.n_tiles));
        GSC_LAUNCHED("render");
        return GSC_OK;
    });
    if (st != GSC_OK) return st;
    ctx->stats_pending = true;
    ctx->stats_dev = nullptr;
    return GSC_OK;
}

gsc_status gsc_colorize_backward(gsc_ctx* ctx, const float* means, const float* scales,
                                 const float* quats, const float* opacities, int64_t N,
                                 const gsc_camera* cams, int32_t n_cams, const void* targets,
                                 int32_t tdtype, int32_t C, int32_t sh_deg, const float* lambda,
                                 int32_t n_lambda, const float* coeffs, const float* grad_coeffs,
                                 float* grad_targets, float* grad_opacities, gsc_stream_t stream) {
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx");
    int64_t rows = 0;
    gsc_status st = validate_geometry(means, scales, quats, opacities, N, cams, n_cams, &rows);
    if (st != GSC_OK) return st;
    if ((st = validate_channels(C, sh_deg)) != GSC_OK) return st;
    if (tdtype != GSC_F32 && tdtype != GSC_BF16) return fail(GSC_ERR_INVALID_ARG, "tdtype must be GSC_F32 or GSC_BF16");
    if (grad_opacities && rows > 0 && !targets) return fail(GSC_ERR_INVALID_ARG, "targets is null");
    if (N > 0 && (!coeffs || !grad_coeffs)) return fail(GSC_ERR_INVALID_ARG, "coeffs or grad_coeffs is null");
    double lam[kMaxNb];
    if ((st = expand_lambda(lambda, n_lambda, sh_deg, lam)) != GSC_OK) return st;
    if (ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;

    hipStream_t s = (hipStream_t)stream;
    if ((st = refuse_capture(s, "gsc_colorize_backward")) != GSC_OK) return st;
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    if (grad_targets && rows > 0) launch_fill_u32((uint32_t*)grad_targets, 0u, (uint64_t)rows * C, s);
    if (grad_opacities && N > 0) launch_fill_u32((uint32_t*)grad_opacities, 0u, (uint64_t)N, s);
    if (N == 0 || n_cams == 0 || (!grad_targets && !grad_opacities)) return GSC_OK;
    const int nb = (sh_deg + 1) * (sh_deg + 1);
    BlendParams bp = blend_params(ctx->opt);
    const BinKey key = make_key(ctx, means, scales, quats, opacities, N, cams, n_cams, bp);
    const bool reuse = can_reuse(ctx, key);
    if ((st = ensure_common(ctx, means, scales, quats, opacities, N, cams, n_cams, s, reuse)) != GSC_OK) return st;
    std::vector<ViewInfo> all(n_cams);
    for (int j = 0; j < n_cams; ++j) all[j] = make_view(cams[j], j, N, ctx->bin);
    // 1. visibilities V_gj (the normal matrices depend on the weights only)
    const bool per_view = sh_deg > 0;
    const uint64_t v_words = (uint64_t)(per_view ? n_cams : 1) * (uint64_t)N;
    GSC_HIP(ctx->vs.ensure(4 * v_words));
    launch_fill_u32(ctx->vs.as<uint32_t>(), 0u, v_words, s);
    unsigned long long* d_counter = reinterpret_cast<unsigned long long*>(ctx->misc.p);
    Binned last;
    st = for_view_batches_k(ctx, all.data(), n_cams, means, opacities, N, bp, s, &key, reuse,
                          [&](int v0, int nv, const Binned& bn) -> gsc_status {
        StageTimer t(ctx, s, GSC_STAGE_BLEND);
        (void)v0;
        launch_accumulate_weights(ctx->views.as<ViewInfo>(), nv, bn.n_tiles, ctx->ranges.as<uint2>(),
                                  ctx->pvals.as<uint32_t>(), ctx->rec0.as<float4>(),
                                  ctx->rec1.as<float4>(), ctx->rec2.as<uint2>(), ctx->bin, per_view, bp, ctx->vs.as<float>(),
                                  d_counter, s, tile_order(ctx, bn.n_tiles));
        GSC_LAUNCHED("accumulate weights");
        last = bn;
        return GSC_OK;
    });
    if (st != GSC_OK) return st;
    const gsc_stats pass1 = ctx->stats;
    // 2. Bbar = (A + w Lambda)^{-1} dL/dc and rho
    if (per_view && (st = upload_all_views(ctx, all.data(), n_cams, s)) != GSC_OK) return st;
    const size_t nbc = (size_t)N * nb * C;
    GSC_HIP(ctx->bbar.ensure(4 * (nbc + (size_t)N) + 4 * (size_t)N));
    float* d_bbar = ctx->bbar.as<float>();
    float* d_rho = d_bbar + nbc;
    float* d_wsum = d_rho + N;
    {
        StageTimer t(ctx, s, GSC_STAGE_SOLVE);
        launch_adjoint_solve(ctx->views_all.as<ViewInfo>(), n_cams, means, ctx->vs.as<float>(), per_view,
                             N, C, sh_deg, lam, grad_coeffs, coeffs, d_bbar, d_rho, d_wsum, s);
        GSC_LAUNCHED("adjoint solve");
    }
    // coefficients and Bbar transposed for the adjoint colours
    GSC_HIP(ctx->coef_t.ensure(4 * 2 * nbc));
    float* d_coef_t = ctx->coef_t.as<float>();
    float* d_bbar_t = d_coef_t + nbc;
    launch_transpose(coeffs, N, nb * C, d_coef_t, s);
    launch_transpose(d_bbar, N, nb * C, d_bbar_t, s);
    GSC_LAUNCHED("transpose");
    // 3. per view batch: adjoint colours, then the two-pass blend adjoint
    auto body = [&](int v0, int nv, const Binned& bn) -> gsc_status {
        (void)v0;
        GSC_HIP(ctx->gamma.ensure(4 * (size_t)nv * (size_t)N * (size_t)(C + 1)));
        StageTimer t(ctx, s, GSC_STAGE_BLEND_ADJOINT);
        launch_view_adjoint(ctx->views.as<ViewInfo>(), nv, (uint32_t)bn.n_items, means, d_coef_t,
                            d_bbar_t, N, d_rho, C, sh_deg, false, ctx->gamma.as<float>(), s);
        GSC_LAUNCHED("view adjoint");
        launch_blend_adjoint(ctx->views.as<ViewInfo>(), nv, bn.n_tiles, ctx->ranges.as<uint2>(),
                             ctx->pvals.as<uint32_t>(), ctx->rec0.as<float4>(), ctx->rec1.as<float4>(), ctx->rec2.as<uint2>(), ctx->bin,
                             targets, tdtype, C, ctx->gamma.as<float>(), bp, grad_targets,
                             grad_opacities, s, tile_order(ctx, bn.n_tiles));
        GSC_LAUNCHED("blend adjoint");
        return GSC_OK;
    };
    if (pass1.view_batches == 1) {
        st = body(0, n_cams, last);  // the binning of the only batch is still in place
    } else {
        st = for_view_batches(ctx, all.data(), n_cams, means, opacities, N, bp, s, body, &key, false);
    }
    if (st != GSC_OK) return st;
    ctx->stats.pairs = pass1.pairs;
    ctx->stats.items = pass1.items;
    ctx->stats.view_batches = pass1.view_batches;
    ctx->stats_pending = true;
    ctx->stats_dev = nullptr;
    return GSC_OK;
}

gsc_status gsc_render_backward(gsc_ctx* ctx, const float* means, const float* scales,
                               const float* quats, const float* opacities, int64_t N,
                               const gsc_camera* cams, int32_t n_cams, const float* coeffs,
                               int32_t C, int32_t sh_deg, const float* grad_images,
                               float* grad_coeffs, float* grad_opacities, gsc_stream_t stream) {
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx");
    int64_t rows = 0;
    gsc_status st = validate_geometry(means, scales, quats, opacities, N, cams, n_cams, &rows);
    if (st != GSC_OK) return st;
    if ((st = validate_channels(C, sh_deg)) != GSC_OK) return st;
    if (rows > 0 && !grad_images) return fail(GSC_ERR_INVALID_ARG, "grad_images is null");
    if (N > 0 && !coeffs) return fail(GSC_ERR_INVALID_ARG, "coeffs is null");
    if (ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = refuse_capture(s, "gsc_render_backward")) != GSC_OK) return st;
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    const int nb = (sh_deg + 1) * (sh_deg + 1);
    if (grad_coeffs && N > 0) launch_fill_u32((uint32_t*)grad_coeffs, 0u, (uint64_t)N * nb * C, s);
    if (grad_opacities && N > 0) launch_fill_u32((uint32_t*)grad_opacities, 0u, (uint64_t)N, s);
    if (N == 0 || n_cams == 0 || (!grad_coeffs && !grad_opacities)) return GSC_OK;
    BlendParams bp = blend_params(ctx->opt);
    const BinKey key = make_key(ctx, means, scales, quats, opacities, N, cams, n_cams, bp);
    const bool reuse = can_reuse(ctx, key);
    if ((st = ensure_common(ctx, means, scales, quats, opacities, N, cams, n_cams, s, reuse)) != GSC_OK) return st;
    std::vector<ViewInfo> all(n_cams);
    for (int j = 0; j < n_cams; ++j) all[j] = make_view(cams[j], j, N, ctx->bin);
    const bool per_view = sh_deg > 0;
    const uint64_t vs_words = (uint64_t)(per_view ? n_cams : 1) * (uint64_t)N * (uint64_t)(C + 1);
    if (grad_coeffs) {
        GSC_HIP(ctx->vs.ensure(4 * vs_words));
        launch_fill_u32(ctx->vs.as<uint32_t>(), 0u, vs_words, s);
    }
    unsigned long long* d_counter = reinterpret_cast<unsigned long long*>(ctx->misc.p);
    if (grad_opacities) {
        GSC_HIP(ctx->coef_t.ensure(4 * (size_t)N * (size_t)(nb * C)));
        launch_transpose(coeffs, N, nb * C, ctx->coef_t.as<float>(), s);
        GSC_LAUNCHED("transpose");
    }
    st = for_view_batches_k(ctx, all.data(), n_cams, means, opacities, N, bp, s, &key, reuse,
                          [&](int v0, int nv, const Binned& bn) -> gsc_status {
        if (grad_coeffs) {
            // dL/dc folds sum_p w (dL/dimages_p) per (view, Gaussian): the
            // forward accumulate with dL/dimages in place of the targets
            StageTimer t(ctx, s, GSC_STAGE_BLEND);
            (void)v0;
            launch_accumulate(ctx->views.as<ViewInfo>(), nv, bn.n_tiles, ctx->ranges.as<uint2>(),
                              ctx->pvals.as<uint32_t>(), ctx->rec0.as<float4>(), ctx->rec1.as<float4>(), ctx->rec2.as<uint2>(), ctx->bin,
                              grad_images, GSC_F32, C, per_view, bp, ctx->vs.as<float>(),
                              d_counter, nullptr, s, tile_order(ctx, bn.n_tiles));
            GSC_LAUNCHED("accumulate");
        }
        if (grad_opacities) {
            GSC_HIP(ctx->gamma.ensure(4 * (size_t)nv * (size_t)N * (size_t)(C + 1)));
            StageTimer t(ctx, s, GSC_STAGE_BLEND_ADJOINT);
            launch_view_adjoint(ctx->views.as<ViewInfo>(), nv, (uint32_t)bn.n_items, means,
                                ctx->coef_t.as<float>(), nullptr, N, nullptr, C, sh_deg, true,
                                ctx->gamma.as<float>(), s);
            GSC_LAUNCHED("view colours");
            launch_blend_adjoint(ctx->views.as<ViewInfo>(), nv, bn.n_tiles, ctx->ranges.as<uint2>(),
                                 ctx->pvals.as<uint32_t>(), ctx->rec0.as<float4>(),
                                 ctx->rec1.as<float4>(), ctx->rec2.as<uint2>(), ctx->bin, grad_images, GSC_F32, C,
                                 ctx->gamma.as<float>(), bp, nullptr, grad_opacities, s,
                                 tile_order(ctx, bn.n_tiles));
            GSC_LAUNCHED("blend adjoint");
        }
        return GSC_OK;
    });
    if (st != GSC_OK) return st;
    if (grad_coeffs) {
        if (per_view && (st = upload_all_views(ctx, all.data(), n_cams, s)) != GSC_OK) return st;
        StageTimer t(ctx, s, GSC_STAGE_SOLVE);
        launch_fold_rhs(ctx->views_all.as<ViewInfo>(), n_cams, means, ctx->vs.as<float>(), per_view, N,
                        C, sh_deg, grad_coeffs, s);
        GSC_LAUNCHED("fold");
    }
    ctx->stats_pending = true;
    ctx->stats_dev = nullptr;
    return GSC_OK;
}

gsc_status gsc_plan_create(gsc_ctx* ctx, const gsc_scene* scenes, int32_t n_scenes,
                           const float* means, const float* scales, const float* quats,
                           const float* opacities, const gsc_camera* cams, int32_t n_cams,
                           int32_t C, int32_t sh_deg, gsc_plan** out, gsc_stream_t stream) {
    if (!out) return fail(GSC_ERR_INVALID_ARG, "null plan pointer");
    *out = nullptr;
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx");
    if (n_scenes < 0 || (n_scenes > 0 && !scenes)) return fail(GSC_ERR_INVALID_ARG, "bad scene table");
    gsc_status st = validate_channels(C, sh_deg);
    if (st != GSC_OK) return st;
    if ((st = validate_cameras(cams, n_cams)) != GSC_OK) return st;
    int64_t n_total = 0;
    std::vector<std::pair<int64_t, int64_t>> ranges;
    for (int k = 0; k < n_scenes; ++k) {
        const gsc_scene& sc = scenes[k];
        if (sc.n_gaussians < 0 || sc.n_gaussians > (int64_t)kItemMask)
            return fail(GSC_ERR_INVALID_ARG, "scene %d: n_gaussians must be in [0, 2^26)", k);
        if (sc.gaussian_offset < 0) return fail(GSC_ERR_INVALID_ARG, "scene %d: negative gaussian_offset", k);
        if (sc.camera_offset < 0 || sc.n_cameras < 0 || (int64_t)sc.camera_offset + sc.n_cameras > n_cams)
            return fail(GSC_ERR_INVALID_ARG, "scene %d: cameras out of range", k);
        n_total = std::max<int64_t>(n_total, sc.gaussian_offset + sc.n_gaussians);
        if (sc.n_gaussians > 0) ranges.push_back({sc.gaussian_offset, sc.gaussian_offset + sc.n_gaussians});
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t k = 1; k < ranges.size(); ++k)
        if (ranges[k].first < ranges[k - 1].second)
            return fail(GSC_ERR_INVALID_ARG, "scenes share Gaussians");
    if (n_total > 0 && (!means || !scales || !quats || !opacities))
        return fail(GSC_ERR_INVALID_ARG, "null Gaussian array");
    if (ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;

    gsc_plan* P = new (std::nothrow) gsc_plan();
    if (!P) return fail(GSC_ERR_HIP, "out of host memory");
    std::unique_ptr<gsc_plan> guard(P);
    hipStream_t s = (hipStream_t)stream;
    P->ctx = ctx;
    P->bp = blend_params(ctx->opt);
    P->bin = ctx->opt.bin_size;
    GSC_HIP(P->misc.ensure(kPlanMiscBytes));
    if (P->bin == 0) {
        double* d_stats = reinterpret_cast<double*>(P->misc.as<char>() + 32);
        launch_geometry_stats(means, scales, n_total, d_stats, s);
        GSC_LAUNCHED("geometry stats");
        double st[4] = {0.0, 0.0, 0.0, 0.0};
        GSC_HIP(hipMemcpyAsync(st, d_stats, sizeof(st), hipMemcpyDeviceToHost, s));
        GSC_HIP(hipStreamSynchronize(s));
        P->bin = choose_bin(st, n_total, cams, n_cams);
    }
    P->scenes.assign(scenes, scenes + n_scenes);
    P->means = means; P->scales = scales; P->quats = quats; P->opac = opacities;
    P->n_total = n_total;
    P->C = C;
    P->sh_deg = sh_deg;
    P->per_view = sh_deg > 0;
    // views scene by scene (scenes without Gaussians contribute none)
    int64_t vs0 = 0;
    for (int k = 0; k < n_scenes; ++k) {
        const gsc_scene& sc = scenes[k];
        P->scene_view0.push_back((int)P->views.size());
        P->scene_vs0.push_back(vs0);
        const int nv = sc.n_gaussians > 0 ? sc.n_cameras : 0;
        P->scene_nviews.push_back(nv);
        for (int j = 0; j < nv; ++j) {
            ViewInfo v = make_view(cams[sc.camera_offset + j], 0, 0, P->bin);
            v.g_offset = sc.gaussian_offset;
            v.n_gauss = (uint32_t)sc.n_gaussians;
            v.scene = (uint32_t)k;
            v.vs_base = vs0 + (int64_t)j * sc.n_gaussians;
            P->views.push_back(v);
        }
        vs0 += (int64_t)nv * sc.n_gaussians;
    }
    P->vs_slots = P->per_view ? (uint64_t)vs0 : (uint64_t)std::max<int64_t>(n_total, 1);
    // batches: consecutive views up to the item and tile limits
    {
        uint64_t items = 0, tiles = 0;
        int v0 = 0;
        for (int v = 0; v < (int)P->views.size(); ++v) {
            const uint64_t ni = P->views[v].n_gauss, nt = (uint64_t)P->views[v].tiles_x * P->views[v].tiles_y;
            if (v > v0 && (items + ni > plan_item_limit(ctx->opt) || tiles + nt >= (1ull << 31))) {
                P->batches.push_back({v0, v - v0, 0, 0, 0, 0});
                v0 = v;
                items = tiles = 0;
            }
            items += ni;
            tiles += nt;
        }
        if (v0 < (int)P->views.size()) P->batches.push_back({v0, (int)P->views.size() - v0, 0, 0, 0, 0});
    }
    plan_number_views(P);
    for (const auto& b : P->batches) P->max_items = std::max(P->max_items, b.n_items);
    const size_t mi = (size_t)P->max_items;
    GSC_HIP(P->misc.ensure(kPlanMiscBytes));
    GSC_HIP(P->cov.ensure(sizeof(float) * kGeoStride * (size_t)std::max<int64_t>(n_total, 1)));
    GSC_HIP(P->keys.ensure(4 * mi + 4));
    GSC_HIP(P->vals.ensure(4 * mi + 4));
    GSC_HIP(P->keys_alt.ensure(4 * mi + 4));
    GSC_HIP(P->vals_alt.ensure(4 * mi + 4));
    GSC_HIP(P->counts.ensure(4 * mi + 4));
    GSC_HIP(P->offsets.ensure(4 * mi + 4));
    GSC_HIP(P->rec0.ensure(16 * mi + 16));
    GSC_HIP(P->rec1.ensure(16 * mi + 16));
    GSC_HIP(P->rec2.ensure(8 * mi + 8));
    GSC_HIP(P->d_views.ensure(sizeof(ViewInfo) * std::max<size_t>(P->views.size(), 1)));
    if (!P->views.empty())
        GSC_HIP(hipMemcpyAsync(P->d_views.p, P->views.data(), sizeof(ViewInfo) * P->views.size(),
                               hipMemcpyHostToDevice, s));
    launch_cov3d(means, opacities, scales, quats, P->cov.as<float>(), n_total, s);
    GSC_LAUNCHED("cov3d");
    // exact pair counts per batch (the geometry is fixed); split oversized batches
    for (size_t k = 0; k < P->batches.size();) {
        uint64_t pairs = 0;
        if ((st = plan_count_pairs(P, P->batches[k], s, &pairs)) != GSC_OK) return st;
        if (pairs >= kMaxPairsPerBatch || (pairs > batch_pair_limit(ctx->opt) && P->batches[k].nv > 1)) {
            gsc_plan::Batch b = P->batches[k];
            if (b.nv == 1) return fail(GSC_ERR_CAPACITY, "one view produces %llu tile pairs", (unsigned long long)pairs);
            const int h = b.nv / 2;
            P->batches[k].nv = h;
            P->batches.insert(P->batches.begin() + k + 1, gsc_plan::Batch{b.v0 + h, b.nv - h, 0, 0, 0, 0});
            plan_number_views(P);
            GSC_HIP(hipMemcpyAsync(P->d_views.p, P->views.data(), sizeof(ViewInfo) * P->views.size(),
                                   hipMemcpyHostToDevice, s));
            continue;
        }
        P->batches[k].pair_cap = (uint32_t)pairs;
        ++k;
    }
    GSC_HIP(hipStreamSynchronize(s));
    for (const auto& b : P->batches) {
        P->max_pairs = std::max(P->max_pairs, b.pair_cap);
        P->max_tiles = std::max(P->max_tiles, b.n_tiles);
        P->items_total += b.n_items;
        P->pairs_total += b.pair_cap;
    }
    const size_t mp = (size_t)P->max_pairs;
    GSC_HIP(P->pkeys.ensure(4 * mp + 4));
    GSC_HIP(P->pvals.ensure(4 * mp + 4));
    GSC_HIP(P->pkeys_alt.ensure(4 * mp + 4));
    GSC_HIP(P->pvals_alt.ensure(4 * mp + 4));
    GSC_HIP(P->ranges.ensure(sizeof(uint2) * ((size_t)P->max_tiles + 1)));
    GSC_HIP(P->order.ensure(4 * tile_order_words(P->max_tiles)));
    const size_t scr = std::max({radix_scratch_words(P->max_items), scan_scratch_words(P->max_items),
                                 radix_scratch_words(P->max_pairs)});
    GSC_HIP(P->sort_scratch.ensure(4 * scr + 256));
    GSC_HIP(P->vs.ensure(4 * P->vs_slots * (size_t)(C + 1)));
    GSC_HIP(P->queues.ensure(4 * (size_t)kMaxC));
    if (sh_deg > 0) {  // observed lists of the fold, one scene at a time
        int64_t nmax = 1;
        for (const gsc_scene& sc : P->scenes) nmax = std::max<int64_t>(nmax, sc.n_gaussians);
        GSC_HIP(P->obs.ensure(4 * (size_t)fold_obs_words(nmax)));
    }
    *out = guard.release();
    return GSC_OK;
}

void gsc_plan_destroy(gsc_plan* plan) { delete plan; }

gsc_status gsc_colorize_batched(gsc_plan* plan, const void* targets, int32_t tdtype,
                                const float* lambda, int32_t n_lambda, float* coeffs,
                                uint8_t* status, gsc_stream_t stream) {
    if (!plan) return fail(GSC_ERR_INVALID_ARG, "null plan");
    if (tdtype != GSC_F32 && tdtype != GSC_BF16) return fail(GSC_ERR_INVALID_ARG, "tdtype must be GSC_F32 or GSC_BF16");
    if (!plan->views.empty() && !targets) return fail(GSC_ERR_INVALID_ARG, "targets is null");
    if (plan->n_total > 0 && !coeffs) return fail(GSC_ERR_INVALID_ARG, "coeffs is null");
    double lam[kMaxNb];
    gsc_status st = expand_lambda(lambda, n_lambda, plan->sh_deg, lam);
    if (st != GSC_OK) return st;
    if (plan->ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;
    return plan_run(plan, targets, tdtype, lam, coeffs, status, (hipStream_t)stream);
}

gsc_status gsc_plan_autotune(gsc_plan* plan, const void* targets, int32_t tdtype,
                             const float* lambda, int32_t n_lambda, float* coeffs,
                             uint8_t* status, gsc_stream_t stream) {
    if (!plan) return fail(GSC_ERR_INVALID_ARG, "null plan");
    if (tdtype != GSC_F32 && tdtype != GSC_BF16) return fail(GSC_ERR_INVALID_ARG, "tdtype must be GSC_F32 or GSC_BF16");
    if (!plan->views.empty() && !targets) return fail(GSC_ERR_INVALID_ARG, "targets is null");
    if (plan->n_total > 0 && !coeffs) return fail(GSC_ERR_INVALID_ARG, "coeffs is null");
    double lam[kMaxNb];
    gsc_status st = expand_lambda(lambda, n_lambda, plan->sh_deg, lam);
    if (st != GSC_OK) return st;
    if (plan->ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;
    hipStream_t s = (hipStream_t)stream;
    // candidates: (channels per launch, persistent or not); the default split
    // of C plus wider and narrower chunks
    std::vector<int> chunks;
    std::vector<int> pool;
    if (plan->C <= (tdtype == GSC_BF16 ? 15 : 7)) pool.push_back(kChunkPacked);
    if (tdtype == GSC_BF16)  // matrix-core forms up to the channels needed
        for (int ch : {16, 32, 64})
            if (ch < plan->C + 16) pool.push_back(kChunkMfma | ch);
    for (int c : {accumulate_chunk(plan->C, GSC_F32), 16, 8, 4}) pool.push_back(c);
    for (int c : pool)
        if (std::find(chunks.begin(), chunks.end(), c) == chunks.end() &&
            chunk_channels(c) <= std::max(4, plan->C + ((c & kChunkMfma) ? 15 : 0)))
            chunks.push_back(c);
    std::vector<int> cand;  // chunk | persistent << 8
    for (int c : chunks)
        for (int p = 0; p < 2; ++p) cand.push_back(c | (p << 8));
    if (cand.size() > 8) cand.resize(8);
    std::vector<float> tot(cand.size(), 0.0f);
    hipEvent_t e0, e1;
    GSC_HIP(hipEventCreate(&e0));
    GSC_HIP(hipEventCreate(&e1));
    const int saved_flags = plan->ctx->opt.flags;
    plan->ctx->opt.flags &= ~GSC_FLAG_PROFILE;
    auto cleanup = [&]() {
        plan->ctx->opt.flags = saved_flags;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    };
    launch_fill_u32(plan->misc.as<uint32_t>(), 0u, 6, s);
    launch_cov3d(plan->means, plan->opac, plan->scales, plan->quats, plan->cov.as<float>(), plan->n_total, s);
    for (const auto& b : plan->batches) {
        if ((st = plan_bin_batch(plan, b, s)) != GSC_OK) { cleanup(); return st; }
        for (size_t k = 0; k < cand.size(); ++k) {
            float best = 1e30f;
            for (int rep = 0; rep < 2; ++rep) {
                hipError_t e = hipEventRecord(e0, s);
                if (e == hipSuccess) {
                    if ((st = plan_accumulate(plan, b, targets, tdtype, cand[k] & 255, (cand[k] >> 8) != 0,
                                              s)) != GSC_OK) { cleanup(); return st; }
                    e = hipEventRecord(e1, s);
                }
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.0f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) { cleanup(); return fail(GSC_ERR_HIP, "autotune timing: %s", hipGetErrorString(e)); }
                best = std::min(best, ms);
            }
            tot[k] += best;
        }
    }
    size_t bi = 0;
    for (size_t k = 0; k < cand.size(); ++k) {
        plan->tune_variant[k] = cand[k];
        plan->tune_ms[k] = tot[k];
        if (tot[k] < tot[bi]) bi = k;
    }
    // the plain grid over the persistent form of the same chunk when within
    // 3%: its XCD-aware tile order moves less HBM traffic (a quarter less on
    // the feature workload)
    if (!cand.empty() && (cand[bi] >> 8) != 0)
        for (size_t k = 0; k < cand.size(); ++k)
            if (cand[k] == (cand[bi] & 255) && tot[k] <= 1.03f * tot[bi]) bi = k;
    plan->acc_chunk = cand.empty() ? 0 : (cand[bi] & 255);
    plan->acc_persistent = !cand.empty() && (cand[bi] >> 8) != 0;
    cleanup();
    if ((st = plan_run(plan, targets, tdtype, lam, coeffs, status, s)) != GSC_OK) return st;
    GSC_HIP(hipStreamSynchronize(s));
    return GSC_OK;
}

gsc_status gsc_plan_get_info(gsc_plan* plan, gsc_plan_info* out) {
    if (!plan || !out) return fail(GSC_ERR_INVALID_ARG, "null plan or output");
    memset(out, 0, sizeof(*out));
    uint32_t buf[6] = {0, 0, 0, 0, 0, 0};
    if (plan->misc.p) {
        GSC_HIP(hipDeviceSynchronize());
        GSC_HIP(hipMemcpy(buf, plan->misc.p, sizeof(buf), hipMemcpyDeviceToHost));
    }
    uint64_t contrib = 0;
    memcpy(&contrib, buf, 8);
    out->contributions = contrib;
    out->dropped_pairs = buf[3];
    out->ill_conditioned = buf[4];
    out->batches = (uint32_t)plan->batches.size();
    out->views = (uint32_t)plan->views.size();
    out->items = plan->items_total;
    out->pair_capacity = plan->pairs_total;
    out->bin_size = plan->bin;
    const int chosen = plan->acc_chunk ? plan->acc_chunk : plan->ctx->opt.accumulate_variant;
    out->accumulate_variant = resolve_chunk(chosen, plan->C, plan->last_tdtype) |
                              (plan->acc_persistent ? 256 : 0);
    for (int i = 0; i < 8; ++i) {
        out->tuned_variant[i] = plan->tune_variant[i];
        out->tuned_ms[i] = plan->tune_ms[i];
    }
    return GSC_OK;
}

gsc_status gsc_combine_coeffs(const float* const* sets, const float* weights, int32_t n_sets,
                              const float* filter, int64_t N, int32_t sh_deg, int32_t C, float* out,
                              gsc_stream_t stream) {
    if (N < 0) return fail(GSC_ERR_INVALID_ARG, "N must be >= 0 (got %lld)", (long long)N);
    gsc_status st = validate_channels(C, sh_deg);
    if (st != GSC_OK) return st;
    if (n_sets < 1 || n_sets > 4096) return fail(GSC_ERR_INVALID_ARG, "n_sets must be in [1,4096] (got %d)", n_sets);
    if (!sets || !weights) return fail(GSC_ERR_INVALID_ARG, "sets or weights is null");
    for (int k = 0; k < n_sets; ++k) {
        if (!isfinite(weights[k])) return fail(GSC_ERR_INVALID_ARG, "weights[%d] is not finite", k);
        if (N > 0 && !sets[k]) return fail(GSC_ERR_INVALID_ARG, "sets[%d] is null", k);
        if (n_sets > kCombineSets && sets[k] == out)
            return fail(GSC_ERR_INVALID_ARG, "out may alias a set only when n_sets <= %d", kCombineSets);
    }
    if (filter)
        for (int c = 0; c < C; ++c)
            if (!isfinite(filter[c])) return fail(GSC_ERR_INVALID_ARG, "filter[%d] is not finite", c);
    if (N > 0 && !out) return fail(GSC_ERR_INVALID_ARG, "out is null");
    const int64_t n = N * (int64_t)(sh_deg + 1) * (sh_deg + 1) * C;
    if (n == 0) return GSC_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    bool vec4 = n % 4 == 0 && (reinterpret_cast<uintptr_t>(out) & 15) == 0;
    for (int k = 0; k < n_sets; ++k) vec4 = vec4 && (reinterpret_cast<uintptr_t>(sets[k]) & 15) == 0;
    for (int k0 = 0; k0 < n_sets; k0 += kCombineSets) {
        CombineArgs a{};
        a.n = std::min(kCombineSets, n_sets - k0);
        for (int k = 0; k < a.n; ++k) {
            a.p[k] = sets[k0 + k];
            a.w[k] = weights[k0 + k];
        }
        a.accumulate = k0 > 0;
        a.filter = filter && k0 + a.n == n_sets;
        for (int c = 0; c < C; ++c) a.f[c] = filter ? filter[c] : 1.0f;
        launch_combine(a, n, C, vec4, out, s);
        GSC_LAUNCHED("combine");
    }
    return GSC_OK;
}

gsc_status gsc_mask_filter(gsc_ctx* ctx, const float* coeffs, int64_t N, int32_t sh_deg, int32_t C,
                           int32_t channel, float threshold, const uint8_t* status, uint8_t* keep,
                           int64_t* indices, int64_t* n_kept, gsc_stream_t stream) {
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx");
    if (N < 0) return fail(GSC_ERR_INVALID_ARG, "N must be >= 0 (got %lld)", (long long)N);
    if (N > (int64_t)kItemMask) return fail(GSC_ERR_UNSUPPORTED, "N must be < 2^26 (got %lld)", (long long)N);
    gsc_status st = validate_channels(C, sh_deg);
    if (st != GSC_OK) return st;
    if (channel < 0 || channel >= C) return fail(GSC_ERR_INVALID_ARG, "channel must be in [0,C) (got %d)", channel);
    if (!isfinite(threshold)) return fail(GSC_ERR_INVALID_ARG, "threshold is not finite");
    if (!keep && !indices && !n_kept) return fail(GSC_ERR_INVALID_ARG, "no output requested");
    if (N > 0 && !coeffs) return fail(GSC_ERR_INVALID_ARG, "coeffs is null");
    if (ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int nb = mask_blocks(N);
    GSC_HIP(ctx->post.ensure((size_t)std::max(nb, 1) * sizeof(uint32_t)));
    launch_mask_filter(coeffs, N, (int64_t)(sh_deg + 1) * (sh_deg + 1) * C, channel, threshold, status,
                       keep, indices, n_kept, ctx->post.as<uint32_t>(), s);
    GSC_LAUNCHED("mask filter");
    return GSC_OK;
}

gsc_status gsc_select_views(gsc_ctx* ctx, const float* means, const float* scales, const float* quats,
                            const float* opacities, int64_t N, const gsc_camera* cams, int32_t n_cams,
                            int32_t k, int32_t multiplicity, int32_t* chosen, int64_t* objective,
                            gsc_stream_t stream) {
    if (!ctx) return fail(GSC_ERR_INVALID_ARG, "null ctx");
    int64_t rows = 0;
    gsc_status st = validate_geometry(means, scales, quats, opacities, N, cams, n_cams, &rows);
    if (st != GSC_OK) return st;
    if (k < 0 || k > n_cams) return fail(GSC_ERR_INVALID_ARG, "k must be in [0, n_cams] (got %d)", k);
    if (multiplicity < 1 || multiplicity > 64)
        return fail(GSC_ERR_INVALID_ARG, "multiplicity must be in [1, 64] (got %d)", multiplicity);
    if (k > 0 && !chosen) return fail(GSC_ERR_INVALID_ARG, "chosen is null");
    if (ctx->opt.flags & GSC_FLAG_VALIDATE_ONLY) return GSC_OK;
    hipStream_t s = (hipStream_t)stream;
    if ((st = refuse_capture(s, "gsc_select_views")) != GSC_OK) return st;
    memset(&ctx->stats, 0, sizeof(ctx->stats));
    if (objective) *objective = 0;
    if (k == 0) return GSC_OK;
    const int64_t words = (N + 63) / 64;
    std::vector<uint64_t> bits((size_t)n_cams * (size_t)words, 0);
    if (N > 0) {
        // 1. per-view visibilities V_gj from a weights-only blend of every view
        BlendParams bp = blend_params(ctx->opt);
        if ((st = ensure_common(ctx, means, scales, quats, opacities, N, cams, n_cams, s)) != GSC_OK) return st;
        std::vector<ViewInfo> all(n_cams);
        for (int j = 0; j < n_cams; ++j) all[j] = make_view(cams[j], j, N, ctx->bin);
        const uint64_t v_words = (uint64_t)n_cams * (uint64_t)N;
        GSC_HIP(ctx->vs.ensure(4 * v_words));
        launch_fill_u32(ctx->vs.as<uint32_t>(), 0u, v_words, s);
        unsigned long long* d_counter = reinterpret_cast<unsigned long long*>(ctx->misc.p);
        st = for_view_batches_k(ctx, all.data(), n_cams, means, opacities, N, bp, s, nullptr, false,
                                [&](int v0, int nv, const Binned& bn) -> gsc_status {
            StageTimer t(ctx, s, GSC_STAGE_BLEND);
            (void)v0;
            launch_accumulate_weights(ctx->views.as<ViewInfo>(), nv, bn.n_tiles, ctx->ranges.as<uint2>(),
                                      ctx->pvals.as<uint32_t>(), ctx->rec0.as<float4>(),
                                      ctx->rec1.as<float4>(), ctx->rec2.as<uint2>(), ctx->bin, true, bp,
                                      ctx->vs.as<float>(), d_counter, s, tile_order(ctx, bn.n_tiles));
            GSC_LAUNCHED("accumulate weights");
            return GSC_OK;
        });
        if (st != GSC_OK) return st;
        // 2. one bitset per view of the Gaussians it observed, read back
        GSC_HIP(ctx->post.ensure(8 * bits.size()));
        launch_seen_bits(ctx->vs.as<float>(), n_cams, N, ctx->post.as<unsigned long long>(), s);
        GSC_LAUNCHED("seen bits");
        GSC_HIP(hipMemcpyAsync(bits.data(), ctx->post.p, 8 * bits.size(), hipMemcpyDeviceToHost, s));
        GSC_HIP(hipStreamSynchronize(s));
        ctx->stats_pending = true;
        ctx->stats_dev = nullptr;
    }
    // 3. greedy maximum coverage of sum_g min(views seeing g, multiplicity):
    // layer r holds the Gaussians seen by at least r + 1 chosen views; a new
    // view raises each Gaussian it sees by one, so its gain is the number of
    // them not yet in the top layer.  Ties go to the lower view index.
    const int R = multiplicity;
    std::vector<uint64_t> layer((size_t)R * (size_t)words, 0);
    std::vector<char> used(n_cams, 0);
    int64_t total = 0;
    for (int pick = 0; pick < k; ++pick) {
        int best = -1;
        int64_t best_gain = -1;
        for (int j = 0; j < n_cams; ++j) {
            if (used[j]) continue;
            const uint64_t* b = bits.data() + (size_t)j * words;
            const uint64_t* top = layer.data() + (size_t)(R - 1) * words;
            int64_t gain = 0;
            for (int64_t w = 0; w < words; ++w) gain += __builtin_popcountll(b[w] & ~top[w]);
            if (gain > best_gain) {
                best_gain = gain;
                best = j;
            }
        }
        used[best] = 1;
        chosen[pick] = best;
        total += best_gain;
        // a Gaussian seen by the new view moves up one layer
        const uint64_t* b = bits.data() + (size_t)best * words;
        for (int r = R - 1; r >= 0; --r) {
            uint64_t* l = layer.data() + (size_t)r * words;
            const uint64_t* below = r > 0 ? layer.data() + (size_t)(r - 1) * words : nullptr;
            for (int64_t w = 0; w < words; ++w) l[w] |= b[w] & (below ? below[w] : ~0ull);
        }
    }
    if (objective) *objective = total;
    return GSC_OK;
}

gsc_status gsc_get_stats(gsc_ctx* ctx, gsc_stats* out) {
    if (!ctx || !out) return fail(GSC_ERR_INVALID_ARG, "null ctx or output");
    if (ctx->stats_pending && (ctx->stats_dev || ctx->misc.p)) {
        uint64_t buf[2] = {0, 0};
        GSC_HIP(hipDeviceSynchronize());
        GSC_HIP(hipMemcpy(buf, ctx->stats_dev ? ctx->stats_dev : ctx->misc.p, 16, hipMemcpyDeviceToHost));
        ctx->stats.contributions = buf[0];
        ctx->stats.ill_conditioned = (uint32_t)(buf[1] >> 32);
        ctx->stats_pending = false;
    }
    if (!ctx->marks.empty()) {
        GSC_HIP(hipDeviceSynchronize());
        for (int i = 0; i < GSC_N_STAGES; ++i) {
            ctx->stats.stage_ms[i] = 0.0f;
            ctx->stats.stage_launches[i] = 0;
        }
        for (const auto& m : ctx->marks) {
            float ms = 0.0f;
            GSC_HIP(hipEventElapsedTime(&ms, m.a, m.b));
            ctx->stats.stage_ms[m.stage] += ms;
            ctx->stats.stage_launches[m.stage] += m.launches;
        }
        ctx->marks.clear();
        ctx->ev_used = 0;
    }
    ctx->stats.bin_size = (uint32_t)ctx->bin;
    *out = ctx->stats;
    return GSC_OK;
}

const char* gsc_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
