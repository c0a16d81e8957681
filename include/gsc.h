/*
 * gsc.h -- C ABI of the MI355X (gfx950) Gaussian-splat colorization library.
 *
 * The library maps 2D images (colours, features, masks) back onto a fixed
 * scene of 3D Gaussian splats as described in "Instant Colorization of
 * Gaussian Splats" (arXiv 2604.17155): every view is tile-rasterised front to
 * back to obtain each Gaussian's blending weight w = alpha*T per pixel (the
 * pixel visibility of eq. 4); per Gaussian the weighted normal equations
 *   A_g = sum_{j,p} w phi_gj phi_gj^T,  B_g = sum_{j,p} w phi_gj y_p^T,
 *   w_g = sum_{j,p} w                                         (eqs. 10-13)
 * are accumulated, where phi_gj are the real spherical harmonics of the view
 * direction camera -> Gaussian (eq. 3, eq. 9), and the Tikhonov-regularised
 * systems (A_g + w_g Lambda) c_g = B_g (eq. 14, Algorithm 1 steps 1-6) are
 * solved for the SH coefficients c_g.
 *
 * Conventions
 *   - Every array argument is a DEVICE pointer owned by the caller unless it
 *     is marked "host".  The library never frees or retains caller memory.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     Calls that size their scratch from data (colorize, render and their
 *     adjoints) read one 4-byte count back from the device and therefore
 *     synchronise `stream` once per call; on a stream under graph capture
 *     they return GSC_ERR_NOT_CAPTURABLE without enqueueing anything.
 *   - Return value: GSC_OK or a negative gsc_status.  On failure
 *     gsc_last_error() returns a message for the calling thread.  Invalid
 *     arguments are rejected before any device work is enqueued.
 *   - A gsc_ctx owns reusable device scratch and is not thread-safe; use one
 *     context per host thread.  Calls on one context must not overlap.
 *
 * Geometry and pixel conventions
 *   - Cameras: world -> camera x_cam = R x + t, R row-major, OpenCV axes
 *     (x right, y down, z forward).  Pinhole projection
 *     u = fx*x/z + cx, v = fy*y/z + cy; the centre of pixel (x, y) is at
 *     (x + 0.5, y + 0.5).
 *   - Gaussians: means [N,3]; scales [N,3] are linear standard deviations;
 *     quats [N,4] are (w, x, y, z), normalised inside; opacities [N] in (0,1)
 *     are already activated.  Sigma = R(q) diag(scale^2) R(q)^T.
 *   - Projection: EWA splatting Sigma_2D = J R Sigma R^T J^T + dilation*I.
 *   - Depth order: key = camera-space z of the mean computed in binary32 as
 *     fmaf(R[6],mx, fmaf(R[7],my, fmaf(R[8],mz, t[2]))); ascending, ties by
 *     lower Gaussian index.  key <= znear culls the Gaussian in that view.
 *   - Per pixel, front to back: q = d^T Sigma_2D^{-1} d with d = pixel centre
 *     minus projected mean; candidates need q <= sigma_cut^2;
 *     alpha = min(alpha_max, o*exp(-q/2)); alpha < alpha_min is skipped;
 *     if T*(1-alpha) < t_min the pixel stops (that Gaussian is not used);
 *     otherwise w = alpha*T and T <- T*(1-alpha).  Background is zero.
 *   - SH basis: real orthonormal spherical harmonics, flat index l*l+l+m,
 *     Y_{l,0} = K P_l, Y_{l,m>0} = sqrt2 K P_l^m cos(m phi),
 *     Y_{l,m<0} = sqrt2 K P_l^|m| sin(|m| phi) (no Condon-Shortley phase),
 *     evaluated at the unit direction from the camera centre -R^T t to the
 *     Gaussian mean.  Y_0 = 1/sqrt(4 pi).
 *   - targets / images: [sum_j H_j W_j, C] row-major, channel-last; camera
 *     j's pixel (x, y) is row cams[j].pixel_offset + y*W_j + x.
 *   - coeffs: [N, (L+1)^2, C] float32.
 *   - lambda (host): n_lambda = 1 (one value), L+1 (one per band) or
 *     (L+1)^2 (one per coefficient); all >= 0.
 */
#ifndef GSC_H
#define GSC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsc_ctx gsc_ctx;
typedef void* gsc_stream_t; /* hipStream_t */

typedef enum {
    GSC_OK = 0,
    GSC_ERR_INVALID_ARG = -1,
    GSC_ERR_HIP = -2,
    GSC_ERR_CAPACITY = -3,
    GSC_ERR_UNSUPPORTED = -4,
    GSC_ERR_NOT_CAPTURABLE = -5 /* called on a stream under graph capture by an entry
                                   point that must read a count back (colorize, render
                                   and their adjoints); nothing was enqueued.  Plans
                                   (gsc_colorize_batched) are capturable. */
} gsc_status;

typedef enum { GSC_F32 = 0, GSC_BF16 = 1 } gsc_dtype;

/* Per-Gaussian status bits written by gsc_colorize. */
enum {
    GSC_G_UNOBSERVED = 1, /* w_g = 0: coefficients set to zero */
    GSC_G_ILL_COND = 2,   /* Cholesky-diagonal estimate of kappa exceeded kappa_max */
    GSC_G_FAILED = 4      /* factorisation failed (not positive definite); coefficients zero */
};

/* Option flags. */
enum {
    GSC_FLAG_VALIDATE_ONLY = 1, /* check the arguments and return; enqueue nothing */
    GSC_FLAG_PROFILE = 2,       /* time each pipeline stage with events on the call's stream */
    GSC_FLAG_REUSE_BINNING = 4, /* reuse the tile lists of the previous call on this context
                                   when it had one view batch and this call passes the same
                                   means, scales, quats and opacities pointers, N, cameras
                                   and blend options: the caller guarantees that the
                                   contents of those arrays are unchanged since that call
                                   (e.g. colorize, render and their adjoints in one
                                   optimisation step); otherwise the call bins anew */
    GSC_FLAG_DETERMINISTIC = 8, /* gsc_colorize / gsc_colorize_ex (and the first pass of
                                   gsc_colorize_refine): bit-identical results from run to
                                   run.  The per-view sums are added as 64-bit fixed-point
                                   integers (exact, so independent of the order of the
                                   tiles) at a power-of-two step of at most 2^-62 times the
                                   largest sum a view's pixels can form (pixels, and pixels
                                   * max|y|; the step is about 2^-42 for 1280x720 views and
                                   |y| <= 1), then converted to binary32 before the FP64
                                   fold.  Costs a scan of the targets (one read-back),
                                   [n_cams, N, C+1] 64-bit words of scratch and the vector
                                   blend (the matrix-core form is not used).  Ignored by
                                   gsc_colorize_noalloc and by plans. */
    GSC_FLAG_CHECK_FINITE = 16  /* gsc_colorize / gsc_colorize_ex / gsc_colorize_refine:
                                   before any other work, scan the targets and the
                                   Gaussian arrays (one read-back) and return
                                   GSC_ERR_INVALID_ARG naming the first array that holds
                                   a NaN or an infinity, and where */
};

/* Pipeline stages timed under GSC_FLAG_PROFILE (indices of gsc_stats.stage_ms). */
enum {
    GSC_STAGE_PROJECT = 0,    /* covariance, projection, footprint, depth key */
    GSC_STAGE_DEPTH_SORT = 1, /* stable radix sort of (view, Gaussian) items by depth */
    GSC_STAGE_SCAN = 2,       /* tile counts in depth order and their exclusive scan */
    GSC_STAGE_EMIT = 3,       /* (tile, item) pair emission */
    GSC_STAGE_TILE_SORT = 4,  /* stable radix sort of pairs by tile, tile ranges */
    GSC_STAGE_BLEND = 5,      /* fused blend + accumulate (colorize) or blend + render */
    GSC_STAGE_SOLVE = 6,      /* fold into normal equations + Cholesky solve (or its adjoint) */
    GSC_STAGE_BLEND_ADJOINT = 7, /* backward: adjoint colours + two-pass blend adjoint */
    GSC_N_STAGES = 8
};

typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    int64_t pixel_offset; /* first target row of this camera */
} gsc_camera;

typedef struct {
    float alpha_min; /* 1/255 */
    float alpha_max; /* 0.99 */
    float t_min;     /* 1e-4; 0 disables the early stop */
    float sigma_cut; /* 3 */
    float dilation;  /* 0.3 px^2 */
    float znear;     /* 0.01 */
    float kappa_max; /* 1e6: threshold for the GSC_G_ILL_COND bit */
    int32_t flags;
    int32_t bin_size; /* 0 (automatic), 16 or 32: pixels per side of the screen
                         bins the Gaussians are sorted into; the result does not
                         depend on it (the footprint test is per pixel).  The
                         automatic choice reads geometry statistics back once
                         and is reused by later calls on the same geometry
                         pointers, Gaussian count and cameras. */
    int32_t accumulate_variant; /* 0 (automatic) or a variant code of the blend +
                         accumulate launch: channels per launch (1, 2, 3, 4, 8, 16);
                         128 + 16, 32 or 64 for the matrix-core form on BF16
                         targets; 129 for the packed matrix-core form (all
                         channels and a ones column in one block: C <= 15 for
                         BF16, C <= 7 for FP32 targets).  A code that does not
                         apply to the call falls back to the automatic choice.
                         A tuned plan uses its own. */
    int32_t schedule;   /* order in which the blend + accumulate launch takes
                           its 16x16 tiles: GSC_SCHEDULE_AUTO (0),
                           GSC_SCHEDULE_GRID (1: one wave per tile, in tile
                           index order) or GSC_SCHEDULE_LONGEST_FIRST (2:
                           bins in decreasing octave of list length, tile
                           index order within an octave; the grid's blocks
                           map to tiles in that order, or, for the
                           matrix-core form, a persistent grid takes them from
                           a work queue).  The result does not depend
                           on it beyond the order of floating-point atomic
                           additions. */
    uint32_t profile_stages; /* GSC_FLAG_PROFILE: the stages to time, bit s for
                                stage s (GSC_STAGE_*); 0 times every stage.
                                Each timed stage adds an event pair to the
                                stream, so a caller timing the whole call can
                                keep to the stages it needs. */
    uint32_t batch_items;    /* 0, or at most 2^26: (view, Gaussian) items per view
                                batch.  Views are binned and blended in batches
                                of consecutive views whose items stay within
                                this bound (a view with more items forms a batch
                                of its own); 0 = 2^26 for single calls and 2^24
                                for plans.  Smaller batches need less scratch and
                                take more launches.  The result does not depend
                                on it. */
    uint32_t batch_pairs;    /* 0, or at most 2^31 - 1: (bin, item) pairs per view
                                batch.  A batch of several views whose pairs
                                exceed it is split in halves until they fit or
                                it holds one view; 0 = 2^31 - 1, the limit of a
                                single view.  The result does not depend on it. */
} gsc_options;

enum { GSC_SCHEDULE_AUTO = 0, GSC_SCHEDULE_GRID = 1, GSC_SCHEDULE_LONGEST_FIRST = 2 };

typedef struct {
    uint64_t contributions; /* accepted (Gaussian, view, pixel) triples of the last call */
    uint64_t pairs;         /* (tile, Gaussian) list entries of the last call */
    uint64_t items;         /* (view, Gaussian) projections of the last call */
    uint32_t view_batches;  /* view batches the last call was split into */
    uint32_t ill_conditioned; /* Gaussians flagged GSC_G_ILL_COND by the last colorize */
    uint32_t bin_size;      /* screen bin size used by the last call (16 or 32 pixels) */
    /* GSC_FLAG_PROFILE: device time and kernel launches per stage, summed over
     * every call since the previous gsc_get_stats (up to 8192 stage records). */
    float stage_ms[GSC_N_STAGES];
    uint32_t stage_launches[GSC_N_STAGES];
} gsc_stats;

/* Fill `out` (host) with the default options listed above. */
gsc_status gsc_default_options(gsc_options* out);

/* Create a context.  `opt` (host) may be NULL for the defaults.  No device
 * work happens here; device scratch is allocated on first use. */
gsc_status gsc_ctx_create(gsc_ctx** ctx, const gsc_options* opt);
void gsc_ctx_destroy(gsc_ctx* ctx);

/* Replace the context's options (host pointer). */
gsc_status gsc_ctx_set_options(gsc_ctx* ctx, const gsc_options* opt);

/*
 * Colorize (Algorithm 1, steps 1-6; eqs. 2-14).
 *   means, scales, quats, opacities: device float32 arrays described above.
 *   cams: host array of n_cams cameras (n_cams >= 0).
 *   targets: device [rows, C], float32 (tdtype GSC_F32) or bfloat16
 *            (GSC_BF16), rows >= max_j(pixel_offset_j + H_j W_j).
 *   C: 1..64 channels.  sh_deg: 0..3.
 *   lambda: host, n_lambda values (see above).
 *   coeffs: device output [N, (L+1)^2, C] float32, fully overwritten.
 *   status: device output [N] uint8 (GSC_G_* bits) or NULL.
 * Unobserved Gaussians (w_g = 0) get zero coefficients.
 */
gsc_status gsc_colorize(gsc_ctx* ctx, const float* means, const float* scales, const float* quats,
                        const float* opacities, int64_t N, const gsc_camera* cams, int32_t n_cams,
                        const void* targets, int32_t tdtype, int32_t C, int32_t sh_deg,
                        const float* lambda, int32_t n_lambda, float* coeffs, uint8_t* status,
                        gsc_stream_t stream);

/* Optional extra outputs of gsc_colorize_ex (each device pointer may be NULL). */
typedef struct {
    float* view_sums;    /* [n_cams, N, C+1] float32: per view j and Gaussian g the
                            visibility V_gj = sum_p w (eq. 5) followed by the C
                            weighted target sums S_gj = sum_p w y_p (numerator of eq. 6) */
    float* visibility;   /* [N] float32: total visibility w_g = sum_j V_gj (eq. 14) */
    uint32_t* counts;    /* [N]: accepted (view, pixel) contributions per Gaussian */
} gsc_extras;

/* gsc_colorize plus the optional outputs in `extras` (host struct, may be NULL). */
gsc_status gsc_colorize_ex(gsc_ctx* ctx, const float* means, const float* scales,
                           const float* quats, const float* opacities, int64_t N,
                           const gsc_camera* cams, int32_t n_cams, const void* targets,
                           int32_t tdtype, int32_t C, int32_t sh_deg, const float* lambda,
                           int32_t n_lambda, float* coeffs, uint8_t* status,
                           const gsc_extras* extras, gsc_stream_t stream);

/*
 * Colorize with iterative refinement (Algorithm 1: steps 1-6, then n_refine
 * passes of steps 8-10; Sec. 3 "Iterative Refinement").  After the first
 * pass each refinement pass renders the current coefficients (eqs. 1-3),
 * accumulates the right-hand side B_g of the residual targets (targets minus
 * that render) and updates
 *   c_g <- c_g + (A_g + w_g Lambda)^{-1} (B_g - w_g Lambda c_g)
 * with the Cholesky factor of the first pass, kept on the device: the
 * geometry, hence A_g and w_g, does not change.  The fixed point is the
 * coupled regularised least-squares solution over all Gaussians, in which the
 * colours of overlapping transparent splats mix.
 *   Arguments as for gsc_colorize, plus n_refine in [0, 10000] (0: the same
 *   as gsc_colorize).  coeffs receives the refined coefficients; status, the
 *   first pass's bits (may be NULL).
 * Unobserved Gaussians and failed factorisations keep zero coefficients.
 * Scratch beyond gsc_colorize's: one FP32 image of the targets' size and,
 * for L >= 1, ((L+1)^2 ((L+1)^2 + 1) / 2 + 1) doubles per Gaussian.  A call
 * with one view batch bins once; otherwise every pass bins each batch again.
 * gsc_get_stats reports the first pass's counts; its stage times cover every
 * pass.
 */
gsc_status gsc_colorize_refine(gsc_ctx* ctx, const float* means, const float* scales,
                               const float* quats, const float* opacities, int64_t N,
                               const gsc_camera* cams, int32_t n_cams, const void* targets,
                               int32_t tdtype, int32_t C, int32_t sh_deg, const float* lambda,
                               int32_t n_lambda, int32_t n_refine, float* coeffs, uint8_t* status,
                               gsc_stream_t stream);

/*
 * gsc_colorize for callers that cannot allocate memory (code under graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation and arguments as gsc_colorize, with every scratch buffer taken
 * from a fixed 64 MiB array of device memory that each GPU holds from the
 * time the library is loaded until the process ends, and the host staging
 * of the camera tables held in static arrays.  No hipMalloc, hipFree or other
 * allocation happens in the call; the caller still passes every input and
 * output.  Like gsc_colorize it reads the tile-pair count back once, so it
 * synchronises `stream`.
 *   ctx supplies the options (GSC_FLAG_PROFILE and GSC_FLAG_REUSE_BINNING are
 *   ignored) and receives the statistics; its own scratch is not used.
 * Limits: at most 1024 cameras, and the whole call (geometry records,
 * per-item keys and records, tile pairs and sort scratch, per-view sums of
 * [n_cams, N, C+1] floats for L > 0) must fit in the 64 MiB: a call whose
 * known sizes exceed it is rejected before any device work with
 * GSC_ERR_CAPACITY; one whose tile pairs turn out not to fit returns
 * GSC_ERR_CAPACITY after the pair count (coefficients then unspecified).
 * All calls on one GPU share the array, which keeps the last call's
 * contents (statistics of the last call are read from it): calls are
 * serialised within a process, and calls on one GPU that overlap (other
 * processes, or enqueued work still running on another stream) race.
 */
gsc_status gsc_colorize_noalloc(gsc_ctx* ctx, const float* means, const float* scales,
                                const float* quats, const float* opacities, int64_t N,
                                const gsc_camera* cams, int32_t n_cams, const void* targets,
                                int32_t tdtype, int32_t C, int32_t sh_deg, const float* lambda,
                                int32_t n_lambda, float* coeffs, uint8_t* status,
                                gsc_stream_t stream);

/*
 * Render (eqs. 1-3): images[p] = sum_g w_gp * c_g^T phi_gj over the same
 * front-to-back blend, background zero.
 *   coeffs: device [N, (L+1)^2, C] float32; images: device output
 *   [sum_j H_j W_j, C] float32 (rows of every camera overwritten).
 */
gsc_status gsc_render(gsc_ctx* ctx, const float* means, const float* scales, const float* quats,
                      const float* opacities, int64_t N, const gsc_camera* cams, int32_t n_cams,
                      const float* coeffs, int32_t C, int32_t sh_deg, float* images,
                      gsc_stream_t stream);

/*
 * Adjoint of gsc_colorize with respect to the targets and the opacities
 * (eqs. 2, 10-14 differentiated; the pixel weights are recomputed, not
 * stored).  With Bbar_g = (A_g + w_g Lambda)^{-1} grad_coeffs_g:
 *   grad_targets_p = sum_g w_gp Bbar_g^T phi_gj
 *   dL/dw_gp = beta^T (y_p - c_g^T phi_gj) - sum_{m,c} lambda_m Bbar_g[m][c] c_g[m][c],
 *   beta = Bbar_g^T phi_gj,
 * and dL/dw is taken through the front-to-back blend to the opacities:
 *   dL/dalpha_k = u_k T_k - (1 - alpha_k)^{-1} sum_{i>k} u_i w_i,
 *   dalpha/do = exp(-q/2) unless alpha is clamped at alpha_max.
 * Footprint, alpha_min and early-stop decisions are piecewise constant and
 * contribute nothing.
 *   Inputs as for gsc_colorize, plus
 *   coeffs: device [N, (L+1)^2, C] float32, the output of gsc_colorize for
 *           the same inputs (the point of linearisation);
 *   grad_coeffs: device [N, (L+1)^2, C] float32, dL/dcoeffs.
 *   grad_targets: device output [rows, C] float32 or NULL with
 *           rows = max_j(pixel_offset_j + H_j W_j); all of these rows are
 *           overwritten (rows that no camera covers get zero).
 *   grad_opacities: device output [N] float32 or NULL; overwritten.
 * Unobserved Gaussians (w_g = 0) and Gaussians whose factorisation failed
 * contribute zero.  Opacity gradients are summed with float atomics, so their
 * last bits vary from run to run.
 */
gsc_status gsc_colorize_backward(gsc_ctx* ctx, const float* means, const float* scales,
                                 const float* quats, const float* opacities, int64_t N,
                                 const gsc_camera* cams, int32_t n_cams, const void* targets,
                                 int32_t tdtype, int32_t C, int32_t sh_deg, const float* lambda,
                                 int32_t n_lambda, const float* coeffs, const float* grad_coeffs,
                                 float* grad_targets, float* grad_opacities, gsc_stream_t stream);

/*
 * Adjoint of gsc_render (eqs. 1-3) for an upstream gradient grad_images
 * (device [rows, C] float32):
 *   grad_coeffs_g = sum_{j,p} w_gp phi_gj grad_images_p^T
 *   dL/dw_gp = (c_g^T phi_gj)^T grad_images_p, taken to the opacities as in
 *   gsc_colorize_backward.
 *   grad_coeffs: device output [N, (L+1)^2, C] float32 or NULL; overwritten.
 *   grad_opacities: device output [N] float32 or NULL; overwritten.
 */
gsc_status gsc_render_backward(gsc_ctx* ctx, const float* means, const float* scales,
                               const float* quats, const float* opacities, int64_t N,
                               const gsc_camera* cams, int32_t n_cams, const float* coeffs,
                               int32_t C, int32_t sh_deg, const float* grad_images,
                               float* grad_coeffs, float* grad_opacities, gsc_stream_t stream);

/*
 * Linear combination of coefficient sets (Sec. 4.1, qualitative results:
 * light fields are linear, so solved coefficient sets can be summed and
 * filtered into lightings that no capture contained).  Elementwise
 *   out[g][m][c] = filter[c] * sum_k weights[k] * sets[k][g][m][c],
 * the sum taken as one binary32 fma chain in k order, then the product with
 * the filter.  Because colorize is linear in its targets, combining the
 * coefficients of several target sets equals colorizing the same
 * combination of the targets (up to rounding).
 *   sets: host array of n_sets (1..4096) device pointers, each
 *         [N, (L+1)^2, C] float32; weights: host [n_sets], finite;
 *   filter: host [C] per-channel gains (a colour filter), or NULL for 1;
 *   out: device output [N, (L+1)^2, C] float32.  It may be one of the sets
 *        when n_sets <= 16 (each element is read before it is written);
 *        otherwise it must not alias any set.
 * No scratch, no synchronisation; capturable.
 */
gsc_status gsc_combine_coeffs(const float* const* sets, const float* weights, int32_t n_sets,
                              const float* filter, int64_t N, int32_t sh_deg, int32_t C, float* out,
                              gsc_stream_t stream);

/*
 * Segmentation filter (Sec. 4.3: after masks are colorized at L = 0 onto the
 * splats, Gaussians whose mask value falls below a threshold, 0.6 there, are
 * removed).  The mask value of Gaussian g in `channel` is its colour averaged
 * over view directions, Y_0 * coeffs[g][0][channel] (the colour itself at
 * L = 0).  Gaussian g is kept when that value, computed in binary32, is
 * >= threshold and, when status is given, neither GSC_G_UNOBSERVED nor
 * GSC_G_FAILED is set.
 *   coeffs: device [N, (L+1)^2, C] float32; status: device [N] or NULL;
 *   keep: device output [N] uint8 (1 kept, 0 dropped) or NULL;
 *   indices: device output with room for N int64, receiving the kept
 *            indices in increasing order (entries past the count untouched),
 *            or NULL;
 *   n_kept: device output, one int64 (the number kept), or NULL.
 * At least one output must be given.  Scratch: 4 bytes per 1024 Gaussians in
 * the context, grown on demand.  No synchronisation.
 */
gsc_status gsc_mask_filter(gsc_ctx* ctx, const float* coeffs, int64_t N, int32_t sh_deg, int32_t C,
                           int32_t channel, float threshold, const uint8_t* status, uint8_t* keep,
                           int64_t* indices, int64_t* n_kept, gsc_stream_t stream);

/*
 * View selection (Sec. 5: fewer camera images, chosen by visibility).  Picks
 * k of the n_cams views greedily to maximise the coverage objective
 *   sum_g min(number of chosen views that observe g, multiplicity),
 * where view j observes Gaussian g when g receives weight at some pixel of j
 * (V_gj > 0 under the context's blend options).  Each pick takes the view
 * with the largest gain; ties go to the lower index.  The objective is
 * monotone and submodular, so the greedy choice reaches at least (1 - 1/e) of
 * the best k-view objective.  Colorize the chosen views by passing those
 * cameras (with their pixel_offset unchanged, so the targets stay where they
 * are).
 *   cams: host [n_cams]; k in [0, n_cams]; multiplicity in [1, 64] (1:
 *   cover every Gaussian once; L >= 1 solves profit from several views per
 *   Gaussian).
 *   chosen: host output [k], view indices in the order picked.
 *   objective: host output (may be NULL), the objective of the chosen set.
 * Runs one weights-only blend of every view, reads n_cams * ceil(N / 64)
 * 64-bit words back (synchronises `stream`), then picks on the host.
 */
gsc_status gsc_select_views(gsc_ctx* ctx, const float* means, const float* scales, const float* quats,
                            const float* opacities, int64_t N, const gsc_camera* cams, int32_t n_cams,
                            int32_t k, int32_t multiplicity, int32_t* chosen, int64_t* objective,
                            gsc_stream_t stream);

/*
 * Batched colorize of many scenes (plans).
 *
 * Several scenes of uneven size are colorized in one pass: all their views
 * are binned and blended by the same launches, view batch by view batch.  A
 * plan fixes every size in advance (gsc_plan_create projects the geometry
 * once and counts its tile pairs exactly), so that gsc_colorize_batched
 * allocates nothing, never synchronises and enqueues kernel launches only: it
 * may be captured into a graph (hipStreamBeginCapture) and replayed.
 *
 * The scenes' Gaussians are concatenated: scene k owns the entries
 * [gaussian_offset, gaussian_offset + n_gaussians) of means, scales, quats,
 * opacities and of the coeffs / status outputs; ranges must not overlap.
 * Its cameras are cams[camera_offset .. camera_offset + n_cameras), whose
 * pixel_offset fields index one concatenated target array.  C, sh_deg and
 * lambda are common to all scenes.
 */
typedef struct {
    int64_t gaussian_offset;
    int64_t n_gaussians; /* < 2^26 */
    int32_t camera_offset;
    int32_t n_cameras;
} gsc_scene;

typedef struct gsc_plan gsc_plan;

typedef struct {
    uint64_t contributions;     /* accepted contributions of the last run */
    uint64_t items;             /* (view, Gaussian) items per run */
    uint64_t pair_capacity;     /* tile pairs per run (exact for the planned geometry) */
    uint32_t dropped_pairs;     /* items of the last run whose pairs exceeded the capacity
                                   (non-zero only if the geometry changed after planning) */
    uint32_t ill_conditioned;   /* Gaussians flagged GSC_G_ILL_COND by the last run */
    uint32_t batches;           /* view batches per run */
    uint32_t views;             /* views per run */
    int32_t bin_size;           /* screen bin size of the plan (16 or 32 pixels) */
    int32_t accumulate_variant; /* accumulate launch shape in use: a variant code as
                                   for gsc_options.accumulate_variant, plus 256 for the
                                   persistent work-queue launch */
    int32_t tuned_variant[8];   /* shapes timed by gsc_plan_autotune (0: unused) */
    float tuned_ms[8];          /* their accumulate time per run, ms */
} gsc_plan_info;

/*
 * Create a plan for `n_scenes` scenes (host table).  The geometry arrays
 * (device) and the cameras (host, n_cams entries; copied) are recorded; the
 * device arrays must stay valid, and unchanged, for the plan's lifetime.
 * Projects every view once and synchronises `stream`.  The plan keeps `ctx`
 * (options, profiling): destroy the plan before the context.
 */
gsc_status gsc_plan_create(gsc_ctx* ctx, const gsc_scene* scenes, int32_t n_scenes,
                           const float* means, const float* scales, const float* quats,
                           const float* opacities, const gsc_camera* cams, int32_t n_cams,
                           int32_t C, int32_t sh_deg, gsc_plan** plan, gsc_stream_t stream);
void gsc_plan_destroy(gsc_plan* plan);

/*
 * Colorize every scene of the plan (the per-scene result equals gsc_colorize
 * on that scene alone, up to the order of float atomics).
 *   targets: device [rows, C] (GSC_F32 or GSC_BF16), rows covering every camera;
 *   lambda: host; coeffs: device output [n_total, (L+1)^2, C] with n_total =
 *   max(gaussian_offset + n_gaussians); status: device output [n_total] or NULL.
 *   Only the scenes' Gaussian ranges are written (L >= 1); for L = 0 every
 *   entry below n_total is written (entries outside all scenes as unobserved).
 * No allocation, no synchronisation, kernel launches only.  Runs of one plan
 * must not overlap (they share its scratch).
 */
gsc_status gsc_colorize_batched(gsc_plan* plan, const void* targets, int32_t tdtype,
                                const float* lambda, int32_t n_lambda, float* coeffs,
                                uint8_t* status, gsc_stream_t stream);

/*
 * Autotune the plan's accumulate launch shape on the given inputs: channels
 * per launch (each launch re-blends the tiles for its channel chunk), the
 * arithmetic (vector lanes, or for BF16 targets matrix cores on blocks of 16
 * channels) and the grid form (one block per few tiles, or a persistent grid
 * whose waves take tiles from a queue).  Times each candidate over all view batches, keeps the
 * fastest (the plain grid over the persistent form of the same arithmetic
 * when it is within 3% of it: its tiles map to the XCDs so that neighbours
 * share an L2, which moves less HBM traffic), then runs the plan once more so
 * that coeffs/status hold a clean result.  Synchronises `stream`.  Not
 * capturable.
 */
gsc_status gsc_plan_autotune(gsc_plan* plan, const void* targets, int32_t tdtype,
                             const float* lambda, int32_t n_lambda, float* coeffs,
                             uint8_t* status, gsc_stream_t stream);

/* Sizes of the plan and counters of its last run (host output; synchronises the device). */
gsc_status gsc_plan_get_info(gsc_plan* plan, gsc_plan_info* out);

/* Statistics of the last call on `ctx` (host output).  Synchronises with the
 * device work of that call. */
gsc_status gsc_get_stats(gsc_ctx* ctx, gsc_stats* out);

/* Message of the last failure on the calling thread ("" if none). */
const char* gsc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GSC_H */
