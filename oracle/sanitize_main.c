/*
 * Test driver for the oracle under AddressSanitizer / UndefinedBehaviorSanitizer
 * (test infrastructure only; built and run by the CPU test-suite).
 *
 * Compiles the oracle source into this translation unit and calls every entry
 * point on a small hand-built scene: four cameras on the coordinate axes, a
 * few dozen Gaussians drawn by a local linear congruential generator (no
 * method arithmetic here), FP32, BF16 and FP64 targets, SH degrees 0 and 2,
 * with one and with two OpenMP threads.  Exit status 0 when every call
 * returns success and every output is finite; the sanitizers report any
 * out-of-bounds access, use after free, leak or undefined operation.
 */
#include "gsc_oracle.c"

#include <stdio.h>

static uint64_t lcg_state = 0x9e3779b97f4a7c15ull;
static double uniform01(void) {
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}
static float uni(double a, double b) { return (float)(a + (b - a) * uniform01()); }

static int all_finite(const double* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(p[i])) return 0;
    return 1;
}

enum { NG = 48, NCAM = 4, RES = 24, CMAX = 2, NBMAX = 9 };

static void make_cameras(oc_camera* cams) {
    /* rows of R for cameras looking at the origin from -z, +z, -x, +x (x right, y down) */
    static const float Rs[NCAM][9] = {{1, 0, 0, 0, 1, 0, 0, 0, 1},
                                      {-1, 0, 0, 0, 1, 0, 0, 0, -1},
                                      {0, 0, -1, 0, 1, 0, 1, 0, 0},
                                      {0, 0, 1, 0, 1, 0, -1, 0, 0}};
    for (int j = 0; j < NCAM; ++j) {
        memcpy(cams[j].R, Rs[j], sizeof(Rs[j]));
        cams[j].t[0] = 0.0f;
        cams[j].t[1] = 0.0f;
        cams[j].t[2] = 3.0f;
        cams[j].fx = cams[j].fy = 20.0f;
        cams[j].cx = cams[j].cy = RES / 2.0f;
        cams[j].width = RES;
        cams[j].height = RES - 4 * (j & 1); /* ragged heights */
        cams[j].pixel_offset = 0;
    }
    int64_t off = 0;
    for (int j = 0; j < NCAM; ++j) {
        cams[j].pixel_offset = off;
        off += (int64_t)cams[j].width * cams[j].height;
    }
}

static int run(int L, int C, int tdtype, int threads) {
    float means[NG * 3], scales[NG * 3], quats[NG * 4], opac[NG];
    for (int g = 0; g < NG; ++g) {
        for (int k = 0; k < 3; ++k) {
            means[3 * g + k] = uni(-0.6, 0.6);
            scales[3 * g + k] = uni(0.02, 0.12);
        }
        for (int k = 0; k < 4; ++k) quats[4 * g + k] = uni(-1.0, 1.0);
        opac[g] = uni(0.05, 0.95);
    }
    opac[3] = 0.999f; /* clamped at alpha_max */
    scales[0] = 1e-4f; /* a splat smaller than a pixel */
    oc_camera cams[NCAM];
    make_cameras(cams);
    const int64_t rows = cams[NCAM - 1].pixel_offset + (int64_t)cams[NCAM - 1].width * cams[NCAM - 1].height;
    const int nb = (L + 1) * (L + 1);
    oc_options o = {1.0f / 255.0f, 0.99f, 1e-4f, 3.0f, 0.3f, 0.01f,
                    6.0 / 16777216.0, 4.0 / 16777216.0, 1.5 / 16777216.0, 4.5 / 16777216.0, 5.0, 1e-14};
    float lam[NBMAX];
    for (int m = 0; m < nb; ++m) lam[m] = 1e-4f * (float)(m + 1);

    float* y32 = malloc(sizeof(float) * rows * C);
    uint16_t* y16 = malloc(sizeof(uint16_t) * rows * C);
    double* y64 = malloc(sizeof(double) * rows * C);
    for (int64_t i = 0; i < rows * C; ++i) {
        y32[i] = uni(0.0, 1.0);
        uint32_t b;
        memcpy(&b, &y32[i], 4);
        y16[i] = (uint16_t)(b >> 16);
        y64[i] = (double)y32[i];
    }
    const void* targets = tdtype == 0 ? (const void*)y32 : (tdtype == 1 ? (const void*)y16 : (const void*)y64);

    double* coeffs = calloc((size_t)NG * nb * C, sizeof(double));
    uint8_t status[NG];
    double* A = calloc((size_t)NG * nb * nb, sizeof(double));
    double* B = calloc((size_t)NG * nb * C, sizeof(double));
    double w[NG], flip[NG], kappa[NG], werr[NG];
    int64_t cnt[NG], ndec[NG], stats[2];
    uint8_t want[NG];
    for (int g = 0; g < NG; ++g) want[g] = (uint8_t)(g % 3 != 0);
    int bad = 0;
    bad |= oc_colorize(means, scales, quats, opac, NG, cams, NCAM, targets, tdtype, C, L, lam, nb, &o,
                       NULL, coeffs, status, A, B, w, flip, kappa, cnt, ndec, werr, stats, threads) != 0;
    bad |= !all_finite(coeffs, (int64_t)NG * nb * C) || !all_finite(w, NG) || !all_finite(flip, NG) ||
           !all_finite(werr, NG);
    bad |= oc_colorize(means, scales, quats, opac, NG, cams, NCAM, targets, tdtype, C, L, lam, 1, &o,
                       want, coeffs, status, A, B, w, flip, NULL, cnt, ndec, NULL, stats, threads) != 0;

    double* img = calloc((size_t)rows * C, sizeof(double));
    double* pix = calloc((size_t)rows, sizeof(double));
    bad |= oc_render(means, scales, quats, opac, NG, cams, NCAM, coeffs, C, L, &o, img, pix, stats, threads) != 0;
    bad |= !all_finite(img, rows * C) || !all_finite(pix, rows);

    double* gc = calloc((size_t)NG * nb * C, sizeof(double));
    double* gt = calloc((size_t)rows * C, sizeof(double));
    double go[NG];
    for (int64_t i = 0; i < (int64_t)NG * nb * C; ++i) gc[i] = uni(-1.0, 1.0);
    bad |= oc_colorize_backward(means, scales, quats, opac, NG, cams, NCAM, targets, tdtype, C, L, lam, nb,
                                &o, coeffs, gc, gt, go, threads) != 0;
    bad |= !all_finite(gt, rows * C) || !all_finite(go, NG);
    double* gi = calloc((size_t)rows * C, sizeof(double));
    for (int64_t i = 0; i < rows * C; ++i) gi[i] = uni(-1.0, 1.0);
    bad |= oc_render_backward(means, scales, quats, opac, NG, cams, NCAM, coeffs, C, L, &o, gi, gc, go,
                              threads) != 0;
    bad |= !all_finite(gc, (int64_t)NG * nb * C) || !all_finite(go, NG);

    double proj[NG * 16];
    bad |= oc_project(means, scales, quats, opac, NG, &cams[1], &o, proj) != 0;
    const int64_t cap = 200000;
    int64_t* idx = malloc(sizeof(int64_t) * 3 * cap);
    double* cw = malloc(sizeof(double) * cap);
    const int64_t n_con = oc_contributions(means, scales, quats, opac, NG, cams, NCAM, &o, idx, cw, cap);
    bad |= n_con < 0 || n_con > cap;
    int64_t* rws = malloc(sizeof(int64_t) * rows);
    const int64_t n_rows = oc_wanted_rows(means, scales, quats, opac, NG, cams, NCAM, &o, want, rws, rows);
    bad |= n_rows < 0 || n_rows > rows;
    if (!bad && n_rows > 0) {
        double* sub = calloc((size_t)n_rows * C, sizeof(double));
        bad |= oc_render_rows(means, scales, quats, opac, NG, cams, NCAM, coeffs, C, L, &o, rws, n_rows, sub,
                              threads) != 0;
        bad |= !all_finite(sub, n_rows * C);
        free(sub);
    }

    /* the solver and the condition estimate on a well-posed system */
    double M[NBMAX * NBMAX], R[NBMAX * CMAX], X[NBMAX * CMAX];
    for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) M[i * nb + j] = (i == j ? 2.0 : 0.0) + 0.1 / (1 + i + j);
    for (int i = 0; i < nb * C; ++i) R[i] = uni(-1.0, 1.0);
    bad |= oc_solve(nb, C, M, R, X) != 0;
    bad |= !(oc_cond(nb, M) >= 1.0);
    double dirs[3 * 5], basis[5 * 16];
    for (int i = 0; i < 15; ++i) dirs[i] = uni(-1.0, 1.0);
    bad |= oc_sh_basis(3, dirs, 5, basis) != 0;
    bad |= oc_sh_basis(4, dirs, 5, basis) == 0; /* degree out of range is rejected */

    free(y32); free(y16); free(y64); free(coeffs); free(A); free(B); free(img); free(pix);
    free(gc); free(gt); free(gi); free(idx); free(cw); free(rws);
    if (bad) fprintf(stderr, "oracle call failed: L=%d C=%d tdtype=%d threads=%d\n", L, C, tdtype, threads);
    return bad;
}

int main(void) {
#ifdef OC_SANITIZE_SELFTEST
    {   /* a planted read one past the end of a heap block: the sanitizer must report it */
        volatile double* p = malloc(4 * sizeof(double));
        double x = p[4];
        printf("%f\n", x);
        free((void*)p);
    }
#endif
    int bad = 0;
    bad |= run(0, 1, 0, 1);
    bad |= run(2, 2, 1, 2);
    bad |= run(2, 2, 2, 1);
    bad |= run(0, 2, 0, 2);
    if (!bad) printf("oracle entry points ran clean\n");
    return bad;
}
