/*
 * gsc_oracle.c -- plain, slow FP64 reference for Gaussian-splat colorization.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * with the HIP library.
 *
 * What it computes (paper: "Instant Colorization of Gaussian Splats"):
 *   - per view j and Gaussian g: the projected 2D Gaussian (EWA splatting as
 *     in the 3DGS renderer the paper builds on, Sec. 3 "Differentiable
 *     renderer"), the camera-space depth used for ordering, and the real
 *     spherical-harmonic basis phi_gj of the view direction (eq. 3, eq. 9);
 *   - per pixel p: front-to-back alpha blending over the depth-ordered
 *     Gaussians covering it (eq. 2); the blending weight w = alpha*T is the
 *     pixel visibility V_{g,p}^j of eq. 4;
 *   - per Gaussian: V_gj = sum_p w (eq. 5), S_gj = sum_p w*y_p (numerator of
 *     eq. 6), the normal matrix A_g = sum_j V_gj phi phi^T, the right-hand
 *     side B_g = sum_j phi S_gj^T and w_g = sum_j V_gj (eqs. 10-13);
 *   - the regularised solve (A_g + w_g Lambda) c_g = B_g (eqs. 14-15,
 *     Algorithm 1, steps 1-6) with a textbook Cholesky factorisation;
 *   - render (eq. 1-3), the adjoint of colorize with respect to the targets
 *     and the opacities, and the adjoint of render.
 *
 * Everything is double precision except the depth ordering key, which is the
 * camera-space z of the mean evaluated in IEEE binary32 as
 *   fmaf(R[6], mx, fmaf(R[7], my, fmaf(R[8], mz, t[2])))
 * so that the order of nearly equal depths is a defined, reproducible choice
 * (ties broken by the lower Gaussian index).
 *
 * Pixel decisions (footprint q <= sigma_cut^2, alpha >= alpha_min, early stop
 * when T*(1-alpha) < T_min) are discontinuous.  Whenever such a decision falls
 * within a relative margin of its threshold the oracle records an "event":
 * the weight that the other outcome could add, remove or rescale.  After the
 * solve it bounds, per Gaussian, the coefficient change those events could
 * cause (first order); callers exclude Gaussians whose bound is not
 * negligible from element-wise comparison, since there several results are
 * correct.
 *
 * Build: gcc -O2 -std=c99 -fopenmp -ffp-contract=off -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    int64_t pixel_offset;
} oc_camera;

/*
 * Blend constants, plus a model of how far an implementation that evaluates
 * the decision quantities in binary32 may stray from their exact values
 * (used only to record near-threshold decisions, see blend_view):
 *   eps_q   relative error of q = d^T Sigma_2D^{-1} d per unit of the sum of
 *           its terms' magnitudes (conic rounded to binary32, two products
 *           and two fused adds);
 *   eps_p   relative error of a pixel offset d formed in binary32 from a
 *           centre held exactly, per unit of (|d| + p_span), p_span being
 *           the largest distance from the point the offsets are formed
 *           against;
 *   eps_cov relative error of the binary32 3D covariance entries per unit of
 *           the largest squared axis scale;
 *   eps_a   relative error of alpha beyond that inherited from q (exp and
 *           the product with the opacity);
 *   eps_t   relative rounding of each transmittance update T (1 - alpha).
 */
typedef struct {
    float alpha_min, alpha_max, t_min, sigma_cut, dilation, znear;
    double eps_q, eps_a, eps_t, eps_p, p_span, eps_cov;
} oc_options;

#define OC_MAX_NB 16

/* Progress for long runs: with GSC_ORACLE_PROGRESS set in the environment,
 * the view loops print a line to stderr as every tenth of their views starts
 * (test infrastructure; the arithmetic is unaffected). */
static int oc_progress_on(void) { return getenv("GSC_ORACLE_PROGRESS") != NULL; }

static void oc_progress(const char* what, int* started, int n_views, int on) {
    if (!on) return;
    int d;
#pragma omp atomic capture
    d = ++(*started);
    const int step = n_views >= 10 ? n_views / 10 : 1;
    if (d % step == 0 || d == n_views) {
        fprintf(stderr, "[oracle] %s: view %d of %d\n", what, d, n_views);
        fflush(stderr);
    }
}

/* ------------------------------------------------------------------ */
/* Real spherical harmonics (eq. 3), from the definition:              */
/*   Y_{l,0}  = K_l^0 P_l^0(cos th)                                    */
/*   Y_{l,m}  = sqrt2 K_l^m P_l^m(cos th) cos(m ph)        m > 0       */
/*   Y_{l,-m} = sqrt2 K_l^m P_l^m(cos th) sin(m ph)        m > 0       */
/* with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and P_l^m the         */
/* associated Legendre function WITHOUT the Condon-Shortley phase.     */
/* Flat index l*l + l + m.                                             */
/* ------------------------------------------------------------------ */
static double factorial(int n) {
    double r = 1.0;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

static double assoc_legendre(int l, int m, double x) {
    /* P_m^m = (2m-1)!! (1-x^2)^(m/2), then the three-term recurrence in l. */
    double pmm = 1.0;
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    for (int i = 1; i <= m; ++i) pmm *= (2.0 * i - 1.0) * s;
    if (l == m) return pmm;
    double pmm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pmm1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = ((2.0 * ll - 1.0) * x * pmm1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pmm1;
        pmm1 = pll;
    }
    return pll;
}

static void sh_basis(int L, const double d[3], double* out) {
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double x = d[0] / r, y = d[1] / r, z = d[2] / r;
    double ph = atan2(y, x);
    for (int l = 0; l <= L; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double P = assoc_legendre(l, am, z);
            double v;
            if (m == 0) v = K * P;
            else if (m > 0) v = sqrt(2.0) * K * P * cos(am * ph);
            else v = sqrt(2.0) * K * P * sin(am * ph);
            out[l * l + l + m] = v;
        }
    }
}

int oc_sh_basis(int L, const double* dirs, int64_t n, double* out) {
    if (L < 0 || L > 3) return -1;
    int nb = (L + 1) * (L + 1);
    for (int64_t i = 0; i < n; ++i) sh_basis(L, dirs + 3 * i, out + nb * i);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Scene geometry                                                      */
/* ------------------------------------------------------------------ */
typedef struct {
    const float* means;
    const float* opac;
    const float* scales;
    double* cov3; /* [N][6]: xx xy xz yy yz zz */
    double* rot;  /* [N][9]: R(q), row-major (for the covariance margin) */
    int64_t N;
} scene_t;

/* Sigma = R(q) diag(s^2) R(q)^T with q = (w,x,y,z) normalised; rot_out
 * (9 doubles, may be NULL) receives R(q). */
static void covariance3d(const float* s, const float* q, double* out, double* rot_out) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double n = sqrt(w * w + x * x + y * y + z * z);
    w /= n; x /= n; y /= n; z /= n;
    double R[3][3] = {
        {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
        {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
        {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
    double s2[3] = {(double)s[0] * s[0], (double)s[1] * s[1], (double)s[2] * s[2]};
    double S[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0.0;
            for (int k = 0; k < 3; ++k) a += R[i][k] * s2[k] * R[j][k];
            S[i][j] = a;
        }
    out[0] = S[0][0]; out[1] = S[0][1]; out[2] = S[0][2];
    out[3] = S[1][1]; out[4] = S[1][2]; out[5] = S[2][2];
    if (rot_out)
        for (int i = 0; i < 9; ++i) rot_out[i] = R[i / 3][i % 3];
}

typedef struct {
    int visible;
    float key;
    double u, v;       /* projected mean, pixel units */
    double ca, cb, cc; /* conic = inverse of the 2D covariance */
    double sxx, sxy, syy;
    double JW[2][3];   /* J W: world directions -> pixels, for the covariance margin */
    const double* rot; /* R(q) of the Gaussian */
    double s2[3];      /* squared axis scales */
    int x0, x1, y0, y1; /* inclusive pixel range that may satisfy q <= sigma_cut^2 */
} proj_t;

static float depth_key(const oc_camera* c, const float* m) {
    return fmaf(c->R[6], m[0], fmaf(c->R[7], m[1], fmaf(c->R[8], m[2], c->t[2])));
}

static void project_one(const scene_t* sc, const oc_camera* cam, const oc_options* o, int64_t g,
                        proj_t* P) {
    const float* m = sc->means + 3 * g;
    P->key = depth_key(cam, m);
    P->visible = P->key > o->znear;
    if (!P->visible) return;
    double W[3][3];
    for (int i = 0; i < 9; ++i) W[i / 3][i % 3] = cam->R[i];
    double t[3];
    for (int i = 0; i < 3; ++i)
        t[i] = W[i][0] * m[0] + W[i][1] * m[1] + W[i][2] * m[2] + (double)cam->t[i];
    double tz = t[2];
    double fx = cam->fx, fy = cam->fy;
    P->u = fx * t[0] / tz + cam->cx;
    P->v = fy * t[1] / tz + cam->cy;
    /* EWA: Sigma_2D = J W Sigma W^T J^T + dilation * I. */
    double J[2][3] = {{fx / tz, 0.0, -fx * t[0] / (tz * tz)}, {0.0, fy / tz, -fy * t[1] / (tz * tz)}};
    const double* c6 = sc->cov3 + 6 * g;
    double S[3][3] = {{c6[0], c6[1], c6[2]}, {c6[1], c6[3], c6[4]}, {c6[2], c6[4], c6[5]}};
    double WS[3][3], Sc[3][3], JS[2][3], S2[2][2];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0.0;
            for (int k = 0; k < 3; ++k) a += W[i][k] * S[k][j];
            WS[i][j] = a;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0.0;
            for (int k = 0; k < 3; ++k) a += WS[i][k] * W[j][k];
            Sc[i][j] = a;
        }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 3; ++j) {
            double a = 0.0;
            for (int k = 0; k < 3; ++k) a += J[i][k] * Sc[k][j];
            JS[i][j] = a;
        }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
            double a = 0.0;
            for (int k = 0; k < 3; ++k) a += JS[i][k] * J[j][k];
            S2[i][j] = a;
        }
    S2[0][0] += o->dilation;
    S2[1][1] += o->dilation;
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k) P->JW[i][k] = J[i][0] * W[0][k] + J[i][1] * W[1][k] + J[i][2] * W[2][k];
    P->rot = sc->rot + 9 * g;
    for (int k = 0; k < 3; ++k) P->s2[k] = (double)sc->scales[3 * g + k] * sc->scales[3 * g + k];
    P->sxx = S2[0][0];
    P->sxy = 0.5 * (S2[0][1] + S2[1][0]);
    P->syy = S2[1][1];
    double det = P->sxx * P->syy - P->sxy * P->sxy;
    P->ca = P->syy / det;
    P->cb = -P->sxy / det;
    P->cc = P->sxx / det;
    /* The ellipse q <= s^2 spans exactly +-s*sqrt(Sxx) in x and +-s*sqrt(Syy)
     * in y; widen by one pixel so the per-pixel test alone decides. */
    double rx = o->sigma_cut * sqrt(P->sxx), ry = o->sigma_cut * sqrt(P->syy);
    double fx0 = ceil(P->u - rx - 0.5) - 1, fx1 = floor(P->u + rx - 0.5) + 1;
    double fy0 = ceil(P->v - ry - 0.5) - 1, fy1 = floor(P->v + ry - 0.5) + 1;
    if (fx0 < 0) fx0 = 0;
    if (fy0 < 0) fy0 = 0;
    if (fx1 > cam->width - 1) fx1 = cam->width - 1;
    if (fy1 > cam->height - 1) fy1 = cam->height - 1;
    if (fx0 > fx1 || fy0 > fy1 || !isfinite(P->u) || !isfinite(P->v)) {
        P->visible = 0;
        return;
    }
    P->x0 = (int)fx0; P->x1 = (int)fx1; P->y0 = (int)fy0; P->y1 = (int)fy1;
}

/* view direction camera centre -> mean, camera centre c = -R^T t */
static void view_dir(const oc_camera* cam, const float* m, double d[3]) {
    double c[3];
    for (int i = 0; i < 3; ++i)
        c[i] = -((double)cam->R[0 + i] * cam->t[0] + (double)cam->R[3 + i] * cam->t[1] +
                 (double)cam->R[6 + i] * cam->t[2]);
    for (int i = 0; i < 3; ++i) d[i] = (double)m[i] - c[i];
}

/* ------------------------------------------------------------------ */
/* Per-view front-to-back blend                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t x;
    int32_t g;
    double w, alpha, G; /* weight, alpha, exp(-q/2) */
    double werr;        /* relative error bound of w evaluated in binary32 (margin model) */
    int clamped;        /* alpha hit alpha_max: d alpha / d o = 0 */
} entry_t;

typedef struct {
    entry_t* e;
    int64_t n, cap;
} elist_t;

static void push(elist_t* L, entry_t en) {
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->e = (entry_t*)realloc(L->e, sizeof(entry_t) * (size_t)L->cap);
    }
    L->e[L->n++] = en;
}

/* A near-threshold decision: the weight `m` of Gaussian g at pixel (x, y)
 * may appear, vanish or be rescaled in an implementation that decides the
 * other way within rounding.  kind 0: g's own acceptance at that pixel may
 * differ (its contribution count may change by one); kind 1: only its weight
 * may be rescaled (an earlier decision at that pixel may differ). */
typedef struct {
    int32_t g, x, y, kind;
    double m;
} event_t;

typedef struct {
    event_t* e;
    int64_t n, cap;
} evlist_t;

static void push_ev(evlist_t* L, int64_t g, int x, int y, double m, int kind) {
    if (!L) return;
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 256;
        L->e = (event_t*)realloc(L->e, sizeof(event_t) * (size_t)L->cap);
    }
    L->e[L->n].g = (int32_t)g;
    L->e[L->n].x = x;
    L->e[L->n].y = y;
    L->e[L->n].kind = kind;
    L->e[L->n].m = m;
    L->n++;
}

static const proj_t* g_sort_P;
static int cmp_key(const void* a, const void* b) {
    int64_t ia = *(const int64_t*)a, ib = *(const int64_t*)b;
    float ka = g_sort_P[ia].key, kb = g_sort_P[ib].key;
    if (ka < kb) return -1;
    if (ka > kb) return 1;
    return (ia > ib) - (ia < ib);
}

/* Insertion-free depth order: merge sort keyed on (key, index). qsort with a
 * global comparator context is not re-entrant, so use a thread-safe local
 * merge sort instead. */
static void sort_by_key(int64_t* idx, int64_t n, const proj_t* P, int64_t* tmp) {
    for (int64_t width = 1; width < n; width *= 2) {
        for (int64_t lo = 0; lo < n; lo += 2 * width) {
            int64_t mid = lo + width < n ? lo + width : n;
            int64_t hi = lo + 2 * width < n ? lo + 2 * width : n;
            int64_t a = lo, b = mid, k = lo;
            while (a < mid && b < hi) {
                int64_t ia = idx[a], ib = idx[b];
                int take_a = (P[ia].key < P[ib].key) || (P[ia].key == P[ib].key && ia < ib);
                tmp[k++] = take_a ? idx[a++] : idx[b++];
            }
            while (a < mid) tmp[k++] = idx[a++];
            while (b < hi) tmp[k++] = idx[b++];
        }
        memcpy(idx, tmp, sizeof(int64_t) * (size_t)n);
    }
    (void)cmp_key;
}

typedef struct {
    int64_t count;   /* accepted contributions */
    int64_t events;  /* near-threshold decisions (kind 0 events) */
} vstats_t;

/* How far a binary32 evaluation may move q and alpha at one pixel (oc_options):
 *   q: eps_q times the sum of the magnitudes of q's terms; the pixel offset
 *      error eps_p (|d| + p_span) per axis through dq/dd = 2 r, r = conic d;
 *      the covariance error |r^T dSigma_2D r| = |v^T dSigma_3D v| with
 *      v = (J W)^T r.  A rotation R + dR and rounded products give
 *      v^T dSigma v <= 2 |dR^T v| |D R^T v| + (rounding) sum_k s_k^2 ((|R|^T |v|)_k)^2,
 *      and |D R^T v| <= s_max sqrt(v^T Sigma v) <= s_max sqrt(q) (since
 *      q = r^T Sigma_2D r >= v^T Sigma v); so the bound is
 *      eps_cov (s_max sqrt(q) |v| + sum_k s_k^2 ((|R|^T |v|)_k)^2);
 *   alpha (relative): eps_a plus half the q bound (exp(-q/2)). */
static void pixel_margins(const proj_t* p, const oc_options* o, double dx, double dy, double q,
                          double* mq, double* ma) {
    double qa = fabs(p->ca * dx * dx) + 2.0 * fabs(p->cb * dx * dy) + fabs(p->cc * dy * dy);
    double rx = p->ca * dx + p->cb * dy, ry = p->cb * dx + p->cc * dy;
    double m = o->eps_q * qa + 2.0 * o->eps_p * (fabs(rx) * (fabs(dx) + o->p_span) +
                                                 fabs(ry) * (fabs(dy) + o->p_span));
    double v[3], vn = 0.0, smax = 0.0, rs = 0.0;
    for (int k = 0; k < 3; ++k) {
        v[k] = p->JW[0][k] * rx + p->JW[1][k] * ry;
        vn += v[k] * v[k];
        smax = fmax(smax, p->s2[k]);
    }
    for (int k = 0; k < 3; ++k) {
        double a = 0.0; /* (|R|^T |v|)_k */
        for (int i = 0; i < 3; ++i) a += fabs(p->rot[3 * i + k]) * fabs(v[i]);
        rs += p->s2[k] * a * a;
    }
    m += o->eps_cov * (sqrt(smax) * sqrt(fmax(q, 0.0)) * sqrt(vn) + rs);
    *mq = m;
    *ma = o->eps_a + 0.5 * m;
}

/*
 * Blend one view.  Appends every accepted contribution (pixel, Gaussian,
 * weight) to `out` in front-to-back order per pixel (rows ascending).
 * pix_mask (H*W bytes, may be NULL) restricts the pixels evaluated.
 * ev (may be NULL) receives the decisions that an implementation evaluating
 * q, alpha and T in binary32 (margins of oc_options) might take the other
 * way, as events carrying the weight that could appear, vanish or be
 * rescaled:
 *   - footprint or alpha-floor decision within its margin: g's own weight
 *     alpha T (kind 0); the weights of every later Gaussian at the pixel may
 *     then be rescaled by (1 - alpha)^(+-1), tracked as the pending mass
 *     pend = sum alpha/(1 - alpha) and recorded as (e^pend - 1) w (kind 1);
 *   - stop decision within the transmittance margin (accumulated rounding
 *     of T plus the pending mass): if the pixel stops here, an
 *     implementation that does not stop accepts this and possibly further
 *     candidates while its T stays above t_min (kind 0 each); if the pixel
 *     goes on, an implementation may stop here, dropping this and every
 *     later weight at the pixel (kind 0 each).
 */
static void blend_view(const scene_t* sc, const oc_camera* cam, const oc_options* o,
                       const uint8_t* pix_mask, proj_t* P, elist_t* out, evlist_t* ev,
                       vstats_t* st) {
    int64_t N = sc->N;
    int W = cam->width, H = cam->height;
    for (int64_t g = 0; g < N; ++g) project_one(sc, cam, o, g, &P[g]);
    int64_t nvis = 0;
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    for (int64_t g = 0; g < N; ++g)
        if (P[g].visible) order[nvis++] = g;
    sort_by_key(order, nvis, P, tmp);
    /* Bucket the depth-ordered Gaussians by the rows they may cover. */
    int64_t* rcount = (int64_t*)calloc((size_t)H + 1, sizeof(int64_t));
    for (int64_t k = 0; k < nvis; ++k) {
        const proj_t* p = &P[order[k]];
        for (int y = p->y0; y <= p->y1; ++y) rcount[y + 1]++;
    }
    for (int y = 0; y < H; ++y) rcount[y + 1] += rcount[y];
    int64_t* rlist = (int64_t*)malloc(sizeof(int64_t) * (size_t)(rcount[H] > 0 ? rcount[H] : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)H);
    for (int y = 0; y < H; ++y) fill[y] = rcount[y];
    for (int64_t k = 0; k < nvis; ++k) {
        const proj_t* p = &P[order[k]];
        for (int y = p->y0; y <= p->y1; ++y) rlist[fill[y]++] = order[k];
    }
    /* per pixel of the current row */
    double* T = (double*)malloc(sizeof(double) * (size_t)W);
    double* terr = (double*)malloc(sizeof(double) * (size_t)W);  /* relative error bound of T */
    double* pend = (double*)malloc(sizeof(double) * (size_t)W);  /* pending rescale mass */
    double* ghostT = (double*)malloc(sizeof(double) * (size_t)W);  /* T of a walk that did not stop */
    double* ghostM = (double*)malloc(sizeof(double) * (size_t)W);
    uint8_t* done = (uint8_t*)malloc((size_t)W);
    uint8_t* fragile = (uint8_t*)malloc((size_t)W);  /* an implementation may have stopped earlier */
    double s2 = (double)o->sigma_cut * (double)o->sigma_cut;
    double amin = o->alpha_min, amax = o->alpha_max, tmin = o->t_min;
    for (int y = 0; y < H; ++y) {
        const uint8_t* mrow = pix_mask ? pix_mask + (int64_t)y * W : NULL;
        int xlo = 0, xhi = W - 1;
        if (mrow) {
            while (xlo < W && !mrow[xlo]) ++xlo;
            while (xhi >= 0 && !mrow[xhi]) --xhi;
            if (xlo > xhi) continue;
        }
        for (int x = 0; x < W; ++x) {
            T[x] = 1.0;
            terr[x] = 0.0;
            pend[x] = 0.0;
            ghostT[x] = 0.0;
            ghostM[x] = 0.0;
            done[x] = mrow ? (mrow[x] ? 0 : 1) : 0;
            fragile[x] = 0;
        }
        double py = y + 0.5;
        for (int64_t k = rcount[y]; k < rcount[y + 1]; ++k) {
            int64_t g = rlist[k];
            const proj_t* p = &P[g];
            int xs = p->x0 > xlo ? p->x0 : xlo, xe = p->x1 < xhi ? p->x1 : xhi;
            double o_g = sc->opac[g];
            for (int x = xs; x <= xe; ++x) {
                if (done[x] && !(ghostT[x] > 0.0)) continue;
                double dx = x + 0.5 - p->u, dy = py - p->v;
                double q = p->ca * dx * dx + 2.0 * p->cb * dx * dy + p->cc * dy * dy;
                double G = exp(-0.5 * q);
                double araw = o_g * G;
                double alpha = araw < amax ? araw : amax;
                double mq = 0.0, ma = 0.0;
                if (ev) pixel_margins(p, o, dx, dy, q, &mq, &ma);
                double mq_cut = mq + o->eps_q * s2; /* plus the rounding of the threshold */
                int may_pass = q <= s2 + mq_cut && araw >= amin * (1.0 - ma);
                if (ghostT[x] > 0.0) {
                    /* the pixel stopped near the threshold; an implementation
                     * that went on may accept g while its T stays above t_min */
                    if (may_pass) {
                        if (ghostT[x] * (1.0 - alpha) >= tmin * (1.0 - ghostM[x])) {
                            push_ev(ev, g, x, y, alpha * ghostT[x], 0);
                            st->events++;
                            ghostT[x] *= 1.0 - alpha;
                        } else {
                            ghostT[x] = 0.0;
                        }
                    }
                    continue; /* done[x] */
                }
                if (ev && fabs(q - s2) <= mq_cut && araw >= amin * (1.0 - ma)) {
                    st->events++;
                    push_ev(ev, g, x, y, alpha * T[x], 0);
                    pend[x] += alpha / (1.0 - alpha);
                }
                if (q > s2) continue;
                if (ev && fabs(araw - amin) <= ma * amin) {
                    st->events++;
                    push_ev(ev, g, x, y, alpha * T[x], 0);
                    pend[x] += alpha / (1.0 - alpha);
                }
                if (alpha < amin) continue;
                /* alpha's own error does not reach T where it is surely clamped */
                double da = araw >= amax * (1.0 + ma) ? 0.0 : ma;
                double terr_new = terr[x] + da * alpha / (1.0 - alpha) + o->eps_t;
                double mrel = terr_new + expm1(pend[x]);
                double test = T[x] * (1.0 - alpha);
                int tnear = ev && fabs(test - tmin) <= mrel * tmin;
                if (test < tmin) {
                    if (tnear) {
                        st->events++;
                        push_ev(ev, g, x, y, alpha * T[x], 0);
                        ghostT[x] = test;
                        ghostM[x] = mrel;
                    }
                    done[x] = 1;
                    continue;
                }
                double w = alpha * T[x];
                if (tnear || fragile[x]) {
                    st->events++;
                    push_ev(ev, g, x, y, w, 0);
                    fragile[x] = 1;
                }
                if (pend[x] > 0.0) push_ev(ev, g, x, y, expm1(pend[x]) * w, 1);
                entry_t en;
                en.x = x;
                en.g = (int32_t)g;
                en.w = w;
                en.alpha = alpha;
                en.G = G;
                en.werr = da + terr[x]; /* alpha's own error and that of T so far */
                en.clamped = araw >= amax;
                push(out, en);
                st->count++;
                T[x] = test;
                terr[x] = terr_new;
            }
        }
        /* row marker: x of entries is within the row; encode the row by
         * pushing a sentinel with g = -1 and x = y. */
        entry_t sentinel;
        memset(&sentinel, 0, sizeof(sentinel));
        sentinel.x = y;
        sentinel.g = -1;
        push(out, sentinel);
    }
    free(T); free(terr); free(pend); free(ghostT); free(ghostM); free(done); free(fragile);
    free(order); free(tmp); free(rcount); free(rlist); free(fill);
}

/* ------------------------------------------------------------------ */
/* Dense helpers                                                       */
/* ------------------------------------------------------------------ */
static void expand_lambda(const float* lam, int n_lambda, int L, double* out) {
    int nb = (L + 1) * (L + 1);
    for (int l = 0; l <= L; ++l)
        for (int m = -l; m <= l; ++m) {
            int i = l * l + l + m;
            if (n_lambda == 1) out[i] = lam[0];
            else if (n_lambda == L + 1) out[i] = lam[l];
            else out[i] = lam[i];
        }
    (void)nb;
}

/* Textbook Cholesky A = L L^T (row-major, lower part written). 0 = ok. */
static int cholesky(int n, const double* A, double* Lm) {
    for (int i = 0; i < n * n; ++i) Lm[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int k = 0; k < j; ++k) s -= Lm[j * n + k] * Lm[j * n + k];
        if (!(s > 0.0)) return -1;
        Lm[j * n + j] = sqrt(s);
        for (int i = j + 1; i < n; ++i) {
            double a = A[i * n + j];
            for (int k = 0; k < j; ++k) a -= Lm[i * n + k] * Lm[j * n + k];
            Lm[i * n + j] = a / Lm[j * n + j];
        }
    }
    return 0;
}

/* Solve L L^T X = B for C right-hand sides; B is [n][C], overwritten. */
static void chol_solve(int n, int C, const double* Lm, double* B) {
    for (int c = 0; c < C; ++c) {
        for (int i = 0; i < n; ++i) {
            double s = B[i * C + c];
            for (int k = 0; k < i; ++k) s -= Lm[i * n + k] * B[k * C + c];
            B[i * C + c] = s / Lm[i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = B[i * C + c];
            for (int k = i + 1; k < n; ++k) s -= Lm[k * n + i] * B[k * C + c];
            B[i * C + c] = s / Lm[i * n + i];
        }
    }
}

/* Cyclic Jacobi eigenvalues of a symmetric matrix; returns max/min. */
static double jacobi_cond(int n, const double* A) {
    double M[OC_MAX_NB * OC_MAX_NB];
    memcpy(M, A, sizeof(double) * (size_t)(n * n));
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                if (i != j) off += M[i * n + j] * M[i * n + j];
                else diag += M[i * n + j] * M[i * n + j];
            }
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = M[p * n + q];
                if (apq == 0.0) continue;
                double theta = (M[q * n + q] - M[p * n + p]) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double mkp = M[k * n + p], mkq = M[k * n + q];
                    M[k * n + p] = c * mkp - s * mkq;
                    M[k * n + q] = s * mkp + c * mkq;
                }
                for (int k = 0; k < n; ++k) {
                    double mpk = M[p * n + k], mqk = M[q * n + k];
                    M[p * n + k] = c * mpk - s * mqk;
                    M[q * n + k] = s * mpk + c * mqk;
                }
            }
    }
    double lo = INFINITY, hi = 0.0;
    for (int i = 0; i < n; ++i) {
        double e = M[i * n + i];
        if (e < lo) lo = e;
        if (e > hi) hi = e;
    }
    return lo > 0.0 ? hi / lo : INFINITY;
}

/* tdtype 0: float32, 1: bfloat16 bits, 2: float64 */
static double target_at(const void* targets, int tdtype, int64_t row, int C, int c) {
    if (tdtype == 2) return ((const double*)targets)[row * C + c];
    if (tdtype == 1) {
        uint16_t b = ((const uint16_t*)targets)[row * C + c];
        uint32_t u = (uint32_t)b << 16;
        float f;
        memcpy(&f, &u, 4);
        return f;
    }
    return ((const float*)targets)[row * C + c];
}

static int check_common(int64_t N, int n_cams, int C, int L) {
    if (N < 0 || n_cams < 0 || C < 1 || C > 64 || L < 0 || L > 3) return -1;
    return 0;
}

static void build_scene(scene_t* sc, const float* means, const float* scales, const float* quats,
                        const float* opac, int64_t N) {
    sc->means = means;
    sc->opac = opac;
    sc->scales = scales;
    sc->N = N;
    sc->cov3 = (double*)malloc(sizeof(double) * 6 * (size_t)(N > 0 ? N : 1));
    sc->rot = (double*)malloc(sizeof(double) * 9 * (size_t)(N > 0 ? N : 1));
    for (int64_t g = 0; g < N; ++g)
        covariance3d(scales + 3 * g, quats + 4 * g, sc->cov3 + 6 * g, sc->rot + 9 * g);
}

/* Pixel mask of one view: union of the pixel ranges of the wanted Gaussians. */
static uint8_t* wanted_mask(const scene_t* sc, const oc_camera* cam, const oc_options* o,
                            const uint8_t* want, proj_t* P) {
    int W = cam->width, H = cam->height;
    uint8_t* m = (uint8_t*)calloc((size_t)W * (size_t)H, 1);
    for (int64_t g = 0; g < sc->N; ++g) {
        if (!want[g]) continue;
        project_one(sc, cam, o, g, &P[g]);
        if (!P[g].visible) continue;
        for (int y = P[g].y0; y <= P[g].y1; ++y) memset(m + (int64_t)y * W + P[g].x0, 1, (size_t)(P[g].x1 - P[g].x0 + 1));
    }
    return m;
}

/* ------------------------------------------------------------------ */
/* Colorize: Algorithm 1 steps 1-6                                     */
/* ------------------------------------------------------------------ */
/*
 * targets: [sum_j H_j W_j, C] float32 (tdtype 0), bfloat16 bits (tdtype 1) or float64
 *          (tdtype 2),
 *          camera j's pixels start at cams[j].pixel_offset, row-major.
 * lam:     n_lambda in {1, L+1, (L+1)^2} (per coefficient / band / all).
 * want:    N bytes or NULL; only Gaussians with want[g] != 0 are solved.
 * Outputs (each may be NULL except coeffs):
 *   coeffs [N][nb][C]; status [N] (bit0 unobserved, bit2 factorisation failed);
 *   A_out [N][nb][nb] regularised normal matrix; B_out [N][nb][C]; w_out [N];
 *   flip_out [N]: bound on ||dc_g||_F from every near-threshold
 *   event touching g, sum_e m_e ||(A_g + w_g Lambda)^{-1} (phi (y_p - c^T phi)^T
 *   - Lambda c)||_F (a weight m added at pixel p changes B by m phi y^T and
 *   A + w Lambda by m (phi phi^T + Lambda));
 *   the factor 1/(1 - s), s = sum_e m_e ||(A_g + w_g Lambda)^{-1}
 *   (phi phi^T + Lambda)||, makes it hold beyond first order (infinite when
 *   s >= 1);
 *   kappa_out [N]; cnt_out [N] accepted contributions per Gaussian;
 *   ndec_out [N] near-threshold decisions on g's own acceptance: an
 *   implementation within the margins accepts g exactly cnt_out[g] times
 *   when ndec_out[g] = 0, and differs by at most ndec_out[g] otherwise;
 *   werr_out [N]: the largest over views of the weight-averaged relative
 *   error bound of g's pixel weights w = alpha T evaluated in binary32 under
 *   the margin model (alpha's own margin unless it is surely clamped, plus
 *   the accumulated bound of T), so that an implementation's per-view sum
 *   V_gj lies within a factor 1 +- werr_out[g] of the exact one, before the
 *   rounding of the summation itself;
 *   stats[0] total accepted contributions of the wanted Gaussians,
 *   stats[1] near-threshold decisions.
 */
int oc_colorize(const float* means, const float* scales, const float* quats, const float* opac,
                int64_t N, const oc_camera* cams, int n_cams, const void* targets, int tdtype,
                int C, int L, const float* lam, int n_lambda, const oc_options* o,
                const uint8_t* want, double* coeffs, uint8_t* status, double* A_out, double* B_out,
                double* w_out, double* flip_out, double* kappa_out, int64_t* cnt_out,
                int64_t* ndec_out, double* werr_out, int64_t* stats, int n_threads) {
    if (check_common(N, n_cams, C, L)) return -1;
    if (!(n_lambda == 1 || n_lambda == L + 1 || n_lambda == (L + 1) * (L + 1))) return -1;
    int nb = (L + 1) * (L + 1);
    double lamx[OC_MAX_NB];
    expand_lambda(lam, n_lambda, L, lamx);
    scene_t sc;
    build_scene(&sc, means, scales, quats, opac, N);
    /* Compact index of the wanted Gaussians. */
    int64_t* kidx = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
    int64_t K = 0;
    for (int64_t g = 0; g < N; ++g) kidx[g] = (!want || want[g]) ? K++ : -1;
    int stride = C + 3; /* V, S[C], count, sum of w times its error bound */
    double* per_view = (double*)calloc((size_t)(K > 0 ? K : 1) * (size_t)(n_cams > 0 ? n_cams : 1) * stride, sizeof(double));
    evlist_t* evs = (evlist_t*)calloc((size_t)(n_cams > 0 ? n_cams : 1), sizeof(evlist_t));
    int64_t tot_events = 0;
    if (n_threads > 0) {
#ifdef _OPENMP
        omp_set_num_threads(n_threads);
#endif
    }
    int prog_started = 0;
    const int prog_on = oc_progress_on();
#pragma omp parallel reduction(+ : tot_events)
    {
        proj_t* P = (proj_t*)malloc(sizeof(proj_t) * (size_t)(N > 0 ? N : 1));
        elist_t lst = {0, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < n_cams; ++j) {
            oc_progress("colorize", &prog_started, n_cams, prog_on);
            const oc_camera* cam = &cams[j];
            uint8_t* mask = want ? wanted_mask(&sc, cam, o, want, P) : NULL;
            lst.n = 0;
            vstats_t st = {0, 0};
            blend_view(&sc, cam, o, mask, P, &lst, &evs[j], &st);
            tot_events += st.events;
            double* pv = per_view + (size_t)j * (size_t)K * stride;
            /* entries of a row come before that row's sentinel */
            int64_t row_start = 0;
            for (int64_t i = 0; i < lst.n; ++i) {
                if (lst.e[i].g >= 0) continue;
                int y = lst.e[i].x;
                for (int64_t r = row_start; r < i; ++r) {
                    const entry_t* en = &lst.e[r];
                    int64_t k = kidx[en->g];
                    if (k < 0) continue;
                    int64_t row = cam->pixel_offset + (int64_t)y * cam->width + en->x;
                    double* a = pv + (size_t)k * stride;
                    a[0] += en->w;
                    for (int c = 0; c < C; ++c) a[1 + c] += en->w * target_at(targets, tdtype, row, C, c);
                    a[C + 1] += 1.0;
                    a[C + 2] += en->w * en->werr;
                }
                row_start = i + 1;
            }
            free(mask);
        }
        free(P); free(lst.e);
    }
    /* Events grouped by Gaussian (view order kept). */
    int64_t* ev_start = (int64_t*)calloc((size_t)(N > 0 ? N : 1) + 1, sizeof(int64_t));
    for (int j = 0; j < n_cams; ++j)
        for (int64_t i = 0; i < evs[j].n; ++i)
            if (kidx[evs[j].e[i].g] >= 0) ev_start[evs[j].e[i].g + 1]++;
    for (int64_t g = 0; g < N; ++g) ev_start[g + 1] += ev_start[g];
    int64_t n_ev = ev_start[N > 0 ? N : 0];
    event_t* ev_all = (event_t*)malloc(sizeof(event_t) * (size_t)(n_ev > 0 ? n_ev : 1));
    int32_t* ev_view = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_ev > 0 ? n_ev : 1));
    {
        int64_t* fillp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N > 0 ? N : 1));
        for (int64_t g = 0; g < N; ++g) fillp[g] = ev_start[g];
        for (int j = 0; j < n_cams; ++j)
            for (int64_t i = 0; i < evs[j].n; ++i) {
                const event_t* e = &evs[j].e[i];
                if (kidx[e->g] < 0) continue;
                ev_all[fillp[e->g]] = *e;
                ev_view[fillp[e->g]] = j;
                fillp[e->g]++;
            }
        free(fillp);
    }
    /* Fold over views in view order (eq. 11-13), then regularise and solve. */
    int64_t tot_count = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : tot_count)
    for (int64_t g = 0; g < N; ++g) {
        int64_t k = kidx[g];
        if (k < 0) continue;
        double A[OC_MAX_NB * OC_MAX_NB], B[OC_MAX_NB * 64], Lm[OC_MAX_NB * OC_MAX_NB];
        double phi[OC_MAX_NB];
        memset(A, 0, sizeof(A));
        memset(B, 0, sizeof(B));
        double w = 0.0, werr = 0.0;
        int64_t cnt = 0;
        for (int j = 0; j < n_cams; ++j) {
            const double* a = per_view + ((size_t)j * (size_t)K + (size_t)k) * stride;
            cnt += (int64_t)a[C + 1];
            if (a[0] == 0.0) continue;
            werr = fmax(werr, a[C + 2] / a[0]);
            double d[3];
            view_dir(&cams[j], means + 3 * g, d);
            sh_basis(L, d, phi);
            w += a[0];
            for (int r = 0; r < nb; ++r) {
                for (int s = 0; s < nb; ++s) A[r * nb + s] += a[0] * phi[r] * phi[s];
                for (int c = 0; c < C; ++c) B[r * C + c] += phi[r] * a[1 + c];
            }
        }
        tot_count += cnt;
        for (int r = 0; r < nb; ++r) A[r * nb + r] += w * lamx[r];
        if (A_out) memcpy(A_out + (size_t)g * nb * nb, A, sizeof(double) * (size_t)(nb * nb));
        if (B_out) memcpy(B_out + (size_t)g * nb * C, B, sizeof(double) * (size_t)(nb * C));
        if (w_out) w_out[g] = w;
        if (werr_out) werr_out[g] = werr;
        if (cnt_out) cnt_out[g] = cnt;
        uint8_t stt = 0;
        double* cg = coeffs + (size_t)g * nb * C;
        double flip = 0.0;
        if (w == 0.0) {
            stt |= 1;
            memset(cg, 0, sizeof(double) * (size_t)(nb * C));
            if (kappa_out) kappa_out[g] = 1.0;
        } else {
            if (cholesky(nb, A, Lm)) {
                stt |= 4;
                memset(cg, 0, sizeof(double) * (size_t)(nb * C));
            } else {
                chol_solve(nb, C, Lm, B);
                memcpy(cg, B, sizeof(double) * (size_t)(nb * C));
            }
            if (kappa_out) kappa_out[g] = jacobi_cond(nb, A);
        }
        int64_t ndec = 0;
        for (int64_t i = ev_start[g]; i < ev_start[g + 1]; ++i) ndec += ev_all[i].kind == 0;
        if (ndec_out) ndec_out[g] = ndec;
        if (flip_out && ev_start[g + 1] > ev_start[g]) {
            /* an event on a Gaussian the oracle sees as unobserved: its weight
             * alone would make it observed; report an unbounded effect */
            if (w == 0.0 || (stt & 4)) {
                flip = INFINITY;
            } else {
                /* Events change the system to (A + E) c' = B + F with
                 * E = sum +-m (phi phi^T + Lambda), F = sum +-m phi y^T, so
                 * c' - c = (A + E)^{-1} sum +-m r,  r = phi (y - c^T phi)^T - Lambda c
                 * (A c = B).  Hence ||c' - c|| <= sum m ||A^{-1} r|| / (1 - s)
                 * with s = sum m ||A^{-1} (phi phi^T + Lambda)|| < 1. */
                double M[OC_MAX_NB * 64], Lam[OC_MAX_NB * OC_MAX_NB], u[OC_MAX_NB];
                memset(Lam, 0, sizeof(Lam));
                for (int r = 0; r < nb; ++r) Lam[r * nb + r] = lamx[r];
                chol_solve(nb, nb, Lm, Lam);
                double nl = 0.0;
                for (int i2 = 0; i2 < nb * nb; ++i2) nl += Lam[i2] * Lam[i2];
                nl = sqrt(nl);
                double first = 0.0, sres = 0.0;
                for (int64_t i = ev_start[g]; i < ev_start[g + 1]; ++i) {
                    const event_t* e = &ev_all[i];
                    const oc_camera* cam = &cams[ev_view[i]];
                    int64_t row = cam->pixel_offset + (int64_t)e->y * cam->width + e->x;
                    double d[3];
                    view_dir(cam, means + 3 * g, d);
                    sh_basis(L, d, phi);
                    for (int c = 0; c < C; ++c) {
                        double gam = 0.0;
                        for (int r = 0; r < nb; ++r) gam += phi[r] * cg[r * C + c];
                        double yv = target_at(targets, tdtype, row, C, c);
                        for (int r = 0; r < nb; ++r) M[r * C + c] = phi[r] * (yv - gam) - lamx[r] * cg[r * C + c];
                    }
                    chol_solve(nb, C, Lm, M);
                    double mn = 0.0;
                    for (int i2 = 0; i2 < nb * C; ++i2) mn += M[i2] * M[i2];
                    first += e->m * sqrt(mn);
                    double pn = 0.0;
                    for (int r = 0; r < nb; ++r) { u[r] = phi[r]; pn += phi[r] * phi[r]; }
                    chol_solve(nb, 1, Lm, u);
                    double un = 0.0;
                    for (int r = 0; r < nb; ++r) un += u[r] * u[r];
                    sres += e->m * (sqrt(un) * sqrt(pn) + nl);
                }
                flip = sres < 1.0 ? first / (1.0 - sres) : INFINITY;
            }
        }
        if (flip_out) flip_out[g] = flip;
        if (status) status[g] = stt;
    }
    if (stats) {
        stats[0] = tot_count;
        stats[1] = tot_events;
    }
    for (int j = 0; j < n_cams; ++j) free(evs[j].e);
    free(evs); free(ev_start); free(ev_all); free(ev_view);
    free(per_view); free(kidx); free(sc.cov3); free(sc.rot);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Render (eq. 1-3): img_p = sum_g w_gp * phi_gj^T c_g                 */
/* ------------------------------------------------------------------ */
/* pix_bound [rows] (may be NULL): per pixel, a bound on how far an
 * implementation within the event margins may render that pixel away from
 * `images` (max over channels): sum over the pixel's events of m ||gamma_g||_inf. */
int oc_render(const float* means, const float* scales, const float* quats, const float* opac,
              int64_t N, const oc_camera* cams, int n_cams, const double* coeffs, int C, int L,
              const oc_options* o, double* images, double* pix_bound, int64_t* stats,
              int n_threads) {
    if (check_common(N, n_cams, C, L)) return -1;
    int nb = (L + 1) * (L + 1);
    scene_t sc;
    build_scene(&sc, means, scales, quats, opac, N);
    int64_t tot = 0;
    if (n_threads > 0) {
#ifdef _OPENMP
        omp_set_num_threads(n_threads);
#endif
    }
    int prog_started = 0;
    const int prog_on = oc_progress_on();
#pragma omp parallel reduction(+ : tot)
    {
        proj_t* P = (proj_t*)malloc(sizeof(proj_t) * (size_t)(N > 0 ? N : 1));
        double* gam = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * C);
        elist_t lst = {0, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < n_cams; ++j) {
            oc_progress("render", &prog_started, n_cams, prog_on);
            const oc_camera* cam = &cams[j];
            double phi[OC_MAX_NB];
            for (int64_t g = 0; g < N; ++g) {
                double d[3];
                view_dir(cam, means + 3 * g, d);
                sh_basis(L, d, phi);
                for (int c = 0; c < C; ++c) {
                    double a = 0.0;
                    for (int m = 0; m < nb; ++m) a += coeffs[((size_t)g * nb + m) * C + c] * phi[m];
                    gam[g * C + c] = a;
                }
            }
            lst.n = 0;
            vstats_t st = {0, 0};
            evlist_t ev = {0, 0, 0};
            blend_view(&sc, cam, o, NULL, P, &lst, pix_bound ? &ev : NULL, &st);
            tot += st.count;
            double* img = images + (size_t)cam->pixel_offset * C;
            memset(img, 0, sizeof(double) * (size_t)cam->width * cam->height * C);
            if (pix_bound) {
                double* pb = pix_bound + (size_t)cam->pixel_offset;
                memset(pb, 0, sizeof(double) * (size_t)cam->width * cam->height);
                for (int64_t i = 0; i < ev.n; ++i) {
                    const event_t* e = &ev.e[i];
                    double gm = 0.0;
                    for (int c = 0; c < C; ++c) gm = fmax(gm, fabs(gam[(size_t)e->g * C + c]));
                    pb[(size_t)e->y * cam->width + e->x] += e->m * gm;
                }
                free(ev.e);
            }
            int64_t row_start = 0;
            for (int64_t i = 0; i < lst.n; ++i) {
                if (lst.e[i].g >= 0) continue;
                int y = lst.e[i].x;
                for (int64_t r = row_start; r < i; ++r) {
                    const entry_t* en = &lst.e[r];
                    double* px = img + ((size_t)y * cam->width + en->x) * C;
                    for (int c = 0; c < C; ++c) px[c] += en->w * gam[(size_t)en->g * C + c];
                }
                row_start = i + 1;
            }
        }
        free(P); free(gam); free(lst.e);
    }
    if (stats) stats[0] = tot;
    free(sc.cov3); free(sc.rot);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Adjoint through one view's blend                                    */
/* ------------------------------------------------------------------ */
/*
 * Given the per-contribution adjoint u = dL/dw for every accepted entry, the
 * weight w_k = alpha_k prod_{i<k}(1-alpha_i) gives, per pixel,
 *   dL/dalpha_k = u_k T_k - (1/(1-alpha_k)) sum_{i>k, accepted} u_i w_i
 * and alpha = min(alpha_max, o exp(-q/2)) gives dalpha/do = exp(-q/2) when
 * not clamped.  Skip and stop decisions are piecewise constant and carry no
 * derivative.  u is supplied per entry; the walk goes back to front.
 */
static void alpha_adjoint_row(const entry_t* e, int64_t n, const double* u, int W, double* acc,
                              double* grad_o) {
    for (int x = 0; x < W; ++x) acc[x] = 0.0;
    for (int64_t r = n - 1; r >= 0; --r) {
        const entry_t* en = &e[r];
        double Tk = en->w / en->alpha;
        double dalpha = u[r] * Tk - acc[en->x] / (1.0 - en->alpha);
        acc[en->x] += u[r] * en->w;
        if (!en->clamped) grad_o[en->g] += dalpha * en->G;
    }
}

/*
 * Adjoint of c = colorize(y, o) at the solution `coeffs`, for an upstream
 * gradient grad_coeffs = dL/dc.  With Bbar_g = (A_g + w_g Lambda)^{-1} dL/dc_g,
 *   dL/dy_p       = sum_g w_gp Bbar_g^T phi_gj
 *   dL/dw_gp      = beta^T (y_p - gamma) - rho_g,
 *     beta = Bbar_g^T phi_gj, gamma = c_g^T phi_gj,
 *     rho_g = sum_{m,k} lambda_m Bbar_g[m,k] c_g[m,k]
 * (from dL = <Bbar, dB - dA_reg c> with dA_reg = sum dw (phi phi^T + Lambda)).
 * grad_targets [rows][C] and grad_opac [N] are overwritten (either may be NULL).
 */
int oc_colorize_backward(const float* means, const float* scales, const float* quats,
                         const float* opac, int64_t N, const oc_camera* cams, int n_cams,
                         const void* targets, int tdtype, int C, int L, const float* lam,
                         int n_lambda, const oc_options* o, const double* coeffs,
                         const double* grad_coeffs, double* grad_targets, double* grad_opac,
                         int n_threads) {
    if (check_common(N, n_cams, C, L)) return -1;
    if (!(n_lambda == 1 || n_lambda == L + 1 || n_lambda == (L + 1) * (L + 1))) return -1;
    int nb = (L + 1) * (L + 1);
    double lamx[OC_MAX_NB];
    expand_lambda(lam, n_lambda, L, lamx);
    /* Regularised normal matrices (targets only enter B, which is unused). */
    double* A = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * nb * nb);
    double* w = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1));
    double* tmpc = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * nb * C);
    int rc = oc_colorize(means, scales, quats, opac, N, cams, n_cams, targets, tdtype, C, L, lam,
                         n_lambda, o, NULL, tmpc, NULL, A, NULL, w, NULL, NULL, NULL, NULL, NULL,
                         NULL, n_threads);
    if (rc) { free(A); free(w); free(tmpc); return rc; }
    double* Bbar = (double*)calloc((size_t)(N > 0 ? N : 1) * nb * C, sizeof(double));
    double* rho = (double*)calloc((size_t)(N > 0 ? N : 1), sizeof(double));
    int prog_started = 0;
    const int prog_on = oc_progress_on();
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < N; ++g) {
        if (w[g] == 0.0) continue;
        double Lm[OC_MAX_NB * OC_MAX_NB];
        if (cholesky(nb, A + (size_t)g * nb * nb, Lm)) continue;
        double* bb = Bbar + (size_t)g * nb * C;
        memcpy(bb, grad_coeffs + (size_t)g * nb * C, sizeof(double) * (size_t)(nb * C));
        chol_solve(nb, C, Lm, bb);
        double r = 0.0;
        for (int m = 0; m < nb; ++m)
            for (int c = 0; c < C; ++c) r += lamx[m] * bb[m * C + c] * coeffs[((size_t)g * nb + m) * C + c];
        rho[g] = r;
    }
    scene_t sc;
    build_scene(&sc, means, scales, quats, opac, N);
    double* go_view = (double*)calloc((size_t)(N > 0 ? N : 1) * (size_t)(n_cams > 0 ? n_cams : 1), sizeof(double));
#pragma omp parallel
    {
        proj_t* P = (proj_t*)malloc(sizeof(proj_t) * (size_t)(N > 0 ? N : 1));
        double* beta = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * C);
        double* gam = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * C);
        elist_t lst = {0, 0, 0};
        double* u = NULL;
        int64_t ucap = 0;
        double* acc = NULL;
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < n_cams; ++j) {
            oc_progress("colorize adjoint", &prog_started, n_cams, prog_on);
            const oc_camera* cam = &cams[j];
            double phi[OC_MAX_NB];
            for (int64_t g = 0; g < N; ++g) {
                double d[3];
                view_dir(cam, means + 3 * g, d);
                sh_basis(L, d, phi);
                for (int c = 0; c < C; ++c) {
                    double b = 0.0, a = 0.0;
                    for (int m = 0; m < nb; ++m) {
                        b += Bbar[((size_t)g * nb + m) * C + c] * phi[m];
                        a += coeffs[((size_t)g * nb + m) * C + c] * phi[m];
                    }
                    beta[g * C + c] = b;
                    gam[g * C + c] = a;
                }
            }
            lst.n = 0;
            vstats_t st = {0, 0};
            blend_view(&sc, cam, o, NULL, P, &lst, NULL, &st);
            if (lst.n > ucap) {
                ucap = lst.n;
                u = (double*)realloc(u, sizeof(double) * (size_t)ucap);
            }
            acc = (double*)realloc(acc, sizeof(double) * (size_t)cam->width);
            double* gt = grad_targets ? grad_targets + (size_t)cam->pixel_offset * C : NULL;
            if (gt) memset(gt, 0, sizeof(double) * (size_t)cam->width * cam->height * C);
            double* go = go_view + (size_t)j * N;
            int64_t row_start = 0;
            for (int64_t i = 0; i < lst.n; ++i) {
                if (lst.e[i].g >= 0) continue;
                int y = lst.e[i].x;
                for (int64_t r = row_start; r < i; ++r) {
                    const entry_t* en = &lst.e[r];
                    int64_t row = cam->pixel_offset + (int64_t)y * cam->width + en->x;
                    double uu = -rho[en->g];
                    for (int c = 0; c < C; ++c) {
                        double yv = target_at(targets, tdtype, row, C, c);
                        double b = beta[(size_t)en->g * C + c];
                        uu += b * (yv - gam[(size_t)en->g * C + c]);
                        if (gt) gt[((size_t)y * cam->width + en->x) * C + c] += en->w * b;
                    }
                    u[r - row_start] = uu;
                }
                alpha_adjoint_row(lst.e + row_start, i - row_start, u, cam->width, acc, go);
                row_start = i + 1;
            }
        }
        free(P); free(beta); free(gam); free(lst.e); free(u); free(acc);
    }
    if (grad_opac) {
        for (int64_t g = 0; g < N; ++g) {
            double s = 0.0;
            for (int j = 0; j < n_cams; ++j) s += go_view[(size_t)j * N + g];
            grad_opac[g] = s;
        }
    }
    free(go_view); free(Bbar); free(rho); free(A); free(w); free(tmpc); free(sc.cov3); free(sc.rot);
    return 0;
}

/*
 * Adjoint of images = render(c, o) for an upstream gradient grad_images:
 *   dL/dc_g  = sum_{j,p} w_gp phi_gj grad_images_p^T
 *   dL/dw_gp = gamma_gj^T grad_images_p, gamma = c_g^T phi_gj
 * followed by the same back-to-front alpha adjoint as above.
 * grad_coeffs [N][nb][C] and grad_opac [N] are overwritten (either may be NULL).
 */
int oc_render_backward(const float* means, const float* scales, const float* quats,
                       const float* opac, int64_t N, const oc_camera* cams, int n_cams,
                       const double* coeffs, int C, int L, const oc_options* o,
                       const double* grad_images, double* grad_coeffs, double* grad_opac,
                       int n_threads) {
    if (check_common(N, n_cams, C, L)) return -1;
    int nb = (L + 1) * (L + 1);
    scene_t sc;
    build_scene(&sc, means, scales, quats, opac, N);
    double* go_view = (double*)calloc((size_t)(N > 0 ? N : 1) * (size_t)(n_cams > 0 ? n_cams : 1), sizeof(double));
    /* per-view dL/dc contributions: V-style [view][g][C] sums of w*Ibar, folded with phi after */
    double* gs_view = (double*)calloc((size_t)(N > 0 ? N : 1) * (size_t)(n_cams > 0 ? n_cams : 1) * C, sizeof(double));
    int prog_started = 0;
    const int prog_on = oc_progress_on();
#pragma omp parallel
    {
        proj_t* P = (proj_t*)malloc(sizeof(proj_t) * (size_t)(N > 0 ? N : 1));
        double* gam = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * C);
        elist_t lst = {0, 0, 0};
        double* u = NULL;
        int64_t ucap = 0;
        double* acc = NULL;
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < n_cams; ++j) {
            oc_progress("render adjoint", &prog_started, n_cams, prog_on);
            const oc_camera* cam = &cams[j];
            double phi[OC_MAX_NB];
            for (int64_t g = 0; g < N; ++g) {
                double d[3];
                view_dir(cam, means + 3 * g, d);
                sh_basis(L, d, phi);
                for (int c = 0; c < C; ++c) {
                    double a = 0.0;
                    for (int m = 0; m < nb; ++m) a += coeffs[((size_t)g * nb + m) * C + c] * phi[m];
                    gam[g * C + c] = a;
                }
            }
            lst.n = 0;
            vstats_t st = {0, 0};
            blend_view(&sc, cam, o, NULL, P, &lst, NULL, &st);
            if (lst.n > ucap) {
                ucap = lst.n;
                u = (double*)realloc(u, sizeof(double) * (size_t)ucap);
            }
            acc = (double*)realloc(acc, sizeof(double) * (size_t)cam->width);
            double* go = go_view + (size_t)j * N;
            double* gs = gs_view + (size_t)j * N * C;
            int64_t row_start = 0;
            for (int64_t i = 0; i < lst.n; ++i) {
                if (lst.e[i].g >= 0) continue;
                int y = lst.e[i].x;
                for (int64_t r = row_start; r < i; ++r) {
                    const entry_t* en = &lst.e[r];
                    const double* gi = grad_images + ((size_t)cam->pixel_offset + (size_t)y * cam->width + en->x) * C;
                    double uu = 0.0;
                    for (int c = 0; c < C; ++c) {
                        uu += gam[(size_t)en->g * C + c] * gi[c];
                        gs[(size_t)en->g * C + c] += en->w * gi[c];
                    }
                    u[r - row_start] = uu;
                }
                alpha_adjoint_row(lst.e + row_start, i - row_start, u, cam->width, acc, go);
                row_start = i + 1;
            }
        }
        free(P); free(gam); free(lst.e); free(u); free(acc);
    }
    if (grad_opac) {
        for (int64_t g = 0; g < N; ++g) {
            double s = 0.0;
            for (int j = 0; j < n_cams; ++j) s += go_view[(size_t)j * N + g];
            grad_opac[g] = s;
        }
    }
    if (grad_coeffs) {
#pragma omp parallel for schedule(static)
        for (int64_t g = 0; g < N; ++g) {
            double phi[OC_MAX_NB];
            double* gc = grad_coeffs + (size_t)g * nb * C;
            memset(gc, 0, sizeof(double) * (size_t)(nb * C));
            for (int j = 0; j < n_cams; ++j) {
                const double* s = gs_view + ((size_t)j * N + g) * C;
                int any = 0;
                for (int c = 0; c < C; ++c) any |= s[c] != 0.0;
                if (!any) continue;
                double d[3];
                view_dir(&cams[j], means + 3 * g, d);
                sh_basis(L, d, phi);
                for (int m = 0; m < nb; ++m)
                    for (int c = 0; c < C; ++c) gc[m * C + c] += phi[m] * s[c];
            }
        }
    }
    free(go_view); free(gs_view); free(sc.cov3); free(sc.rot);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Inspection helpers for the tests                                    */
/* ------------------------------------------------------------------ */
/* Projection of every Gaussian into one camera: per g
 * [visible, key, u, v, ca, cb, cc, sxx, sxy, syy] (10 doubles). */
int oc_project(const float* means, const float* scales, const float* quats, const float* opac,
               int64_t N, const oc_camera* cam, const oc_options* o, double* out) {
    scene_t sc;
    build_scene(&sc, means, scales, quats, opac, N);
    for (int64_t g = 0; g < N; ++g) {
        proj_t P;
        memset(&P, 0, sizeof(P));
        project_one(&sc, cam, o, g, &P);
        double* r = out + 10 * g;
        r[0] = P.visible; r[1] = P.key; r[2] = P.u; r[3] = P.v;
        r[4] = P.ca; r[5] = P.cb; r[6] = P.cc; r[7] = P.sxx; r[8] = P.sxy; r[9] = P.syy;
    }
    free(sc.cov3); free(sc.rot);
    return 0;
}

/* Every accepted contribution of every view: rows of (view, pixel row index
 * into the target array, g, w).  Returns the number written (<= cap), or -1. */
int64_t oc_contributions(const float* means, const float* scales, const float* quats,
                         const float* opac, int64_t N, const oc_camera* cams, int n_cams,
                         const oc_options* o, int64_t* out_idx /* [cap][3] */, double* out_w,
                         int64_t cap) {
    scene_t sc;
    build_scene(&sc, means, scales, quats, opac, N);
    proj_t* P = (proj_t*)malloc(sizeof(proj_t) * (size_t)(N > 0 ? N : 1));
    elist_t lst = {0, 0, 0};
    int64_t n = 0;
    for (int j = 0; j < n_cams; ++j) {
        lst.n = 0;
        vstats_t st = {0, 0};
        blend_view(&sc, &cams[j], o, NULL, P, &lst, NULL, &st);
        int64_t row_start = 0;
        for (int64_t i = 0; i < lst.n; ++i) {
            if (lst.e[i].g >= 0) continue;
            int y = lst.e[i].x;
            for (int64_t r = row_start; r < i; ++r) {
                if (n < cap) {
                    out_idx[3 * n] = j;
                    out_idx[3 * n + 1] = cams[j].pixel_offset + (int64_t)y * cams[j].width + lst.e[r].x;
                    out_idx[3 * n + 2] = lst.e[r].g;
                    out_w[n] = lst.e[r].w;
                }
                ++n;
            }
            row_start = i + 1;
        }
    }
    free(P); free(lst.e); free(sc.cov3); free(sc.rot);
    return n;
}

/* The target rows (camera pixel_offset + y W + x) inside the pixel ranges of
 * the wanted Gaussians, view by view in ascending order: the only target
 * values a colorize restricted to those Gaussians reads.  Returns the number
 * of rows (rows_out receives at most cap of them). */
/* Every accepted contribution at the given pixels only: rows (sorted
 * ascending global target rows) select pixels of every camera; the blend runs
 * over those pixels (a pixel's full front-to-back walk) and writes rows of
 * (view, pixel row, g, w) in view order.  Returns the number of contributions
 * (<= cap written), or -1. */
int64_t oc_contributions_rows(const float* means, const float* scales, const float* quats,
                              const float* opac, int64_t N, const oc_camera* cams, int n_cams,
                              const oc_options* o, const int64_t* rows, int64_t n_rows,
                              int64_t* out_idx /* [cap][3] */, double* out_w, int64_t cap,
                              int n_threads) {
    scene_t sc;
    build_scene(&sc, means, scales, quats, opac, N);
    elist_t* lists = (elist_t*)calloc((size_t)(n_cams > 0 ? n_cams : 1), sizeof(elist_t));
    if (n_threads > 0) {
#ifdef _OPENMP
        omp_set_num_threads(n_threads);
#endif
    }
#pragma omp parallel
    {
        proj_t* P = (proj_t*)malloc(sizeof(proj_t) * (size_t)(N > 0 ? N : 1));
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < n_cams; ++j) {
            const oc_camera* cam = &cams[j];
            const int64_t lo = cam->pixel_offset, hi = lo + (int64_t)cam->width * cam->height;
            /* first requested row of this camera (rows are sorted) */
            int64_t a = 0, b = n_rows;
            while (a < b) {
                int64_t m = (a + b) / 2;
                if (rows[m] < lo) a = m + 1; else b = m;
            }
            if (a >= n_rows || rows[a] >= hi) continue;
            uint8_t* mask = (uint8_t*)calloc((size_t)cam->width * (size_t)cam->height, 1);
            for (int64_t k = a; k < n_rows && rows[k] < hi; ++k) mask[rows[k] - lo] = 1;
            vstats_t st = {0, 0};
            blend_view(&sc, cam, o, mask, P, &lists[j], NULL, &st);
            free(mask);
        }
        free(P);
    }
    int64_t n = 0;
    for (int j = 0; j < n_cams; ++j) {
        const elist_t* L = &lists[j];
        int64_t row_start = 0;
        for (int64_t i = 0; i < L->n; ++i) {
            if (L->e[i].g >= 0) continue;
            int y = L->e[i].x;
            for (int64_t r = row_start; r < i; ++r) {
                if (n < cap) {
                    out_idx[3 * n] = j;
                    out_idx[3 * n + 1] = cams[j].pixel_offset + (int64_t)y * cams[j].width + L->e[r].x;
                    out_idx[3 * n + 2] = L->e[r].g;
                    out_w[n] = L->e[r].w;
                }
                ++n;
            }
            row_start = i + 1;
        }
        free(L->e);
    }
    free(lists); free(sc.cov3); free(sc.rot);
    return n;
}

int64_t oc_wanted_rows(const float* means, const float* scales, const float* quats,
                       const float* opac, int64_t N, const oc_camera* cams, int n_cams,
                       const oc_options* o, const uint8_t* want, int64_t* rows_out, int64_t cap) {
    scene_t sc;
    build_scene(&sc, means, scales, quats, opac, N);
    uint8_t** masks = (uint8_t**)calloc((size_t)(n_cams > 0 ? n_cams : 1), sizeof(uint8_t*));
    int64_t* cnt = (int64_t*)calloc((size_t)(n_cams > 0 ? n_cams : 1) + 1, sizeof(int64_t));
#pragma omp parallel
    {
        proj_t* P = (proj_t*)malloc(sizeof(proj_t) * (size_t)(N > 0 ? N : 1));
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < n_cams; ++j) {
            masks[j] = wanted_mask(&sc, &cams[j], o, want, P);
            int64_t npx = (int64_t)cams[j].width * cams[j].height, c = 0;
            for (int64_t i = 0; i < npx; ++i) c += masks[j][i] != 0;
            cnt[j + 1] = c;
        }
        free(P);
    }
    for (int j = 0; j < n_cams; ++j) cnt[j + 1] += cnt[j];
    int64_t n = cnt[n_cams > 0 ? n_cams : 0];
    for (int j = 0; j < n_cams; ++j) {
        int64_t npx = (int64_t)cams[j].width * cams[j].height, k = cnt[j];
        for (int64_t i = 0; i < npx; ++i) {
            if (!masks[j][i]) continue;
            if (k < cap) rows_out[k] = cams[j].pixel_offset + i;
            ++k;
        }
        free(masks[j]);
    }
    free(masks); free(cnt); free(sc.cov3); free(sc.rot);
    return n;
}

/* Render (eqs. 1-3) of the listed target rows only (ascending, each inside
 * one camera): out[k][c] = sum_g w_g phi_g^T c_g at row rows[k]. */
int oc_render_rows(const float* means, const float* scales, const float* quats, const float* opac,
                   int64_t N, const oc_camera* cams, int n_cams, const double* coeffs, int C, int L,
                   const oc_options* o, const int64_t* rows, int64_t n_rows, double* out,
                   int n_threads) {
    if (check_common(N, n_cams, C, L)) return -1;
    int nb = (L + 1) * (L + 1);
    scene_t sc;
    build_scene(&sc, means, scales, quats, opac, N);
    memset(out, 0, sizeof(double) * (size_t)n_rows * C);
    if (n_threads > 0) {
#ifdef _OPENMP
        omp_set_num_threads(n_threads);
#endif
    }
    int prog_started = 0;
    const int prog_on = oc_progress_on();
#pragma omp parallel
    {
        proj_t* P = (proj_t*)malloc(sizeof(proj_t) * (size_t)(N > 0 ? N : 1));
        double* gam = (double*)malloc(sizeof(double) * (size_t)(N > 0 ? N : 1) * C);
        elist_t lst = {0, 0, 0};
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < n_cams; ++j) {
            oc_progress("render rows", &prog_started, n_cams, prog_on);
            const oc_camera* cam = &cams[j];
            int64_t npx = (int64_t)cam->width * cam->height;
            /* the listed rows of this camera: [k0, k1) */
            int64_t lo = 0, hi = n_rows;
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (rows[mid] < cam->pixel_offset) lo = mid + 1; else hi = mid;
            }
            int64_t k0 = lo;
            hi = n_rows;
            while (lo < hi) {
                int64_t mid = (lo + hi) / 2;
                if (rows[mid] < cam->pixel_offset + npx) lo = mid + 1; else hi = mid;
            }
            int64_t k1 = lo;
            if (k0 == k1) continue;
            int64_t* slot = (int64_t*)malloc(sizeof(int64_t) * (size_t)npx);
            uint8_t* mask = (uint8_t*)calloc((size_t)npx, 1);
            for (int64_t i = 0; i < npx; ++i) slot[i] = -1;
            for (int64_t k = k0; k < k1; ++k) {
                slot[rows[k] - cam->pixel_offset] = k;
                mask[rows[k] - cam->pixel_offset] = 1;
            }
            double phi[OC_MAX_NB];
            for (int64_t g = 0; g < N; ++g) {
                double d[3];
                view_dir(cam, means + 3 * g, d);
                sh_basis(L, d, phi);
                for (int c = 0; c < C; ++c) {
                    double a = 0.0;
                    for (int m = 0; m < nb; ++m) a += coeffs[((size_t)g * nb + m) * C + c] * phi[m];
                    gam[g * C + c] = a;
                }
            }
            lst.n = 0;
            vstats_t st = {0, 0};
            blend_view(&sc, cam, o, mask, P, &lst, NULL, &st);
            int64_t row_start = 0;
            for (int64_t i = 0; i < lst.n; ++i) {
                if (lst.e[i].g >= 0) continue;
                int y = lst.e[i].x;
                for (int64_t r = row_start; r < i; ++r) {
                    const entry_t* en = &lst.e[r];
                    int64_t k = slot[(int64_t)y * cam->width + en->x];
                    if (k < 0) continue;
                    for (int c = 0; c < C; ++c) out[k * C + c] += en->w * gam[(size_t)en->g * C + c];
                }
                row_start = i + 1;
            }
            free(slot); free(mask);
        }
        free(P); free(gam); free(lst.e);
    }
    free(sc.cov3); free(sc.rot);
    return 0;
}

/* Regularised solve of given normal equations (for checking the solver). */
int oc_solve(int nb, int C, const double* A, const double* B, double* X) {
    double Lm[OC_MAX_NB * OC_MAX_NB];
    if (nb < 1 || nb > OC_MAX_NB || cholesky(nb, A, Lm)) return -1;
    memcpy(X, B, sizeof(double) * (size_t)(nb * C));
    chol_solve(nb, C, Lm, X);
    return 0;
}

double oc_cond(int nb, const double* A) { return jacobi_cond(nb, A); }
