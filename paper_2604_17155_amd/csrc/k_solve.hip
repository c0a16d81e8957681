// Fold of the per-view sums into the normal equations and the regularised
// solve (eqs. 11-14, Algorithm 1 steps 5-6).
//
// L >= 1: four lanes per Gaussian.  Lane r owns the rows i = 4k + r of
//   A_g = sum_j V_gj phi_gj phi_gj^T  and  B_g = sum_j phi_gj S_gj^T
// and accumulates them over the views in FP64 registers (FP32 accumulation
// of A over tens of views loses ~1e-4 relative at the condition numbers the
// paper's Lambda produces).  The quad then factors A_g + w_g Lambda with a
// cooperative FP64 Cholesky and solves four right-hand-side columns at a
// time, all in registers; the factor stays there for further channel chunks.
// L = 0: A_g = w_g Y0^2 is a scalar and c_g = Y0 S_g / (w_g (Y0^2 + lambda_0)).
#include <algorithm>

#include "gsc_internal.h"
#include "sh.h"

namespace gsc {

struct LamNB {
    double v[kMaxNb];
};

constexpr double kY0 = 0.28209479177387814;

__global__ void k_solve_dc(const float* __restrict__ VS, int64_t N, int C, double lam0,
                           float* __restrict__ coeffs, uint8_t* __restrict__ status,
                           float* __restrict__ wout) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const float* s = VS + g * (int64_t)(C + 1);
    double w = s[0];
    if (wout) wout[g] = (float)w;
    float* out = coeffs + g * C;
    if (w == 0.0) {
        for (int c = 0; c < C; ++c) out[c] = 0.0f;
        if (status) status[g] = GSC_G_UNOBSERVED;
        return;
    }
    double den = w * (kY0 * kY0 + lam0);
    for (int c = 0; c < C; ++c) out[c] = (float)(kY0 * (double)s[1 + c] / den);
    if (status) status[g] = 0;
}

// Sum the per-view slots of every Gaussian over the views (L = 0 with
// per-view sums kept for the caller).
__global__ void k_sum_views(const float* __restrict__ VS, int n_views, int64_t N, int stride,
                            float* __restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N * stride) return;
    float a = 0.0f;
    for (int v = 0; v < n_views; ++v) a += VS[(int64_t)v * N * stride + i];
    out[i] = a;
}

// Broadcast lane `o` of each quad to the whole quad (DPP quad_perm [o,o,o,o]).
template <int O>
__device__ __forceinline__ double quad_bcast(double x) {
    constexpr int ctrl = O | (O << 2) | (O << 4) | (O << 6);
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over the quad (DPP quad_perm [1,0,3,2] then [2,3,0,1]); every lane of
// the quad gets the same value.
__device__ __forceinline__ double quad_sum(double x) {
    constexpr int x1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);
    constexpr int x2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
    x += __hiloint2double(__builtin_amdgcn_update_dpp(0, __double2hiint(x), x1, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, __double2loint(x), x1, 0xF, 0xF, false));
    x += __hiloint2double(__builtin_amdgcn_update_dpp(0, __double2hiint(x), x2, 0xF, 0xF, false),
                          __builtin_amdgcn_update_dpp(0, __double2loint(x), x2, 0xF, 0xF, false));
    return x;
}

__device__ __forceinline__ double quad_max(double x) {
    constexpr int x1 = 1 | (0 << 2) | (3 << 4) | (2 << 6);
    constexpr int x2 = 2 | (3 << 2) | (0 << 4) | (1 << 6);
    x = fmax(x, __hiloint2double(__builtin_amdgcn_update_dpp(0, __double2hiint(x), x1, 0xF, 0xF, false),
                                 __builtin_amdgcn_update_dpp(0, __double2loint(x), x1, 0xF, 0xF, false)));
    x = fmax(x, __hiloint2double(__builtin_amdgcn_update_dpp(0, __double2hiint(x), x2, 0xF, 0xF, false),
                                 __builtin_amdgcn_update_dpp(0, __double2loint(x), x2, 0xF, 0xF, false)));
    return x;
}

// Unit direction from a camera centre (FP64) to a Gaussian mean, in FP64:
// the normal equations are assembled in FP64, and a direction rounded to
// binary32 would perturb A_g by an amount that weak regularisation does not
// damp.  1/|d| from the hardware reciprocal square root refined by three
// Newton steps y <- y (3/2 - n y^2 / 2), each of which squares the relative
// error (full FP64 from any start better than 2^-12), at a fraction of the
// cost of a square root and a division.
__device__ __forceinline__ void view_direction(float mx, float my, float mz, const double* centre,
                                               double* dir) {
    const double dx = (double)mx - centre[0];
    const double dy = (double)my - centre[1];
    const double dz = (double)mz - centre[2];
    const double n2 = dx * dx + dy * dy + dz * dz;
    if (!(n2 > 0.0)) {  // a mean at the camera centre: culled there, any unit vector will do
        dir[0] = 0.0;
        dir[1] = 0.0;
        dir[2] = 1.0;
        return;
    }
    double inv = __builtin_amdgcn_rsq(n2);
#pragma unroll
    for (int k = 0; k < 3; ++k) inv = inv * fma(-0.5 * n2 * inv, inv, 1.5);
    dir[0] = dx * inv;
    dir[1] = dy * inv;
    dir[2] = dz * inv;
}

// Broadcast from quad lane j & 3.
__device__ __forceinline__ double quad_from(double x, int j) {
    switch (j & 3) {
        case 0: return quad_bcast<0>(x);
        case 1: return quad_bcast<1>(x);
        case 2: return quad_bcast<2>(x);
        default: return quad_bcast<3>(x);
    }
}

// Fold + solve for L >= 1.  Four lanes (a quad) per Gaussian; lane r owns
// the rows i = 4k + r of A (lower triangle) and of the right-hand sides,
// four channels at a time, all in FP64 registers.  The views' sums are read
// in groups of four (the next group in flight while one is folded) and
// folded two views at a time.  The Cholesky factor is formed in place
// (column j broadcast within the quad; the owner of row j keeps 1/L_jj on
// the diagonal), forward substitution broadcasts each solved entry to the
// quad, and back substitution sums each column's products over the quad.
// No LDS.
//
// ADJ: adjoint solve for the backward pass.  VS then holds only the per-view
// visibilities (stride 1); the right-hand sides are read from `rhs`
// (dL/dc, [N][NB][C]) instead of being folded, the solution
// Bbar = (A + w Lambda)^{-1} dL/dc is written to `out`, and
// rho_g = sum_{m,c} lambda_m Bbar[m][c] cin[m][c] (cin = the forward
// coefficients) to rho[g].
template <int L, bool ADJ>
__global__ __launch_bounds__(256) void k_fold_solve(const ViewInfo* __restrict__ views, int n_views,
                                                    const float* __restrict__ means,
                                                    const float* __restrict__ VS, int vs_stride,
                                                    int64_t N, int C, LamNB lam, float kappa_max,
                                                    const float* __restrict__ rhs,
                                                    const float* __restrict__ cin,
                                                    float* __restrict__ coeffs,
                                                    float* __restrict__ rho,
                                                    uint8_t* __restrict__ status,
                                                    float* __restrict__ wout,
                                                    unsigned int* __restrict__ ill_count,
                                                    double* __restrict__ factor,
                                                    const uint32_t* __restrict__ list,
                                                    const int64_t* __restrict__ n_list) {
    constexpr int NB = (L + 1) * (L + 1);
    constexpr int RPL = (NB + 3) / 4;  // rows per lane
    const int r = threadIdx.x & 3;
    // with a list, quad q takes the q-th observed Gaussian; a wave past the
    // end of the list has nothing to do (one wave per block: no barrier)
    const int64_t q = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
    const bool valid = list ? q < *n_list : q < N;
    if (list && __builtin_amdgcn_ballot_w64(valid) == 0) return;
    const int64_t g = list ? (valid ? (int64_t)list[q] : 0) : q;
    const int stride = vs_stride;
    float mx = 0.f, my = 0.f, mz = 0.f;
    if (valid) {
        mx = means[3 * g];
        my = means[3 * g + 1];
        mz = means[3 * g + 2];
    }
    double sel[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) sel[e] = r == e ? 1.0 : 0.0;
    // accA[k][j]: row 4k+r, column j <= 4k+r; after the factorisation the
    // owner's diagonal entry holds 1/L_ii
    double accA[RPL][NB];
    bool failed = false;
    double wsum = 0.0;
    double rho_part = 0.0;
    for (int c0 = 0; c0 < C; c0 += 4) {
        const bool firstc = c0 == 0;
        double accB[RPL][4];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
#pragma unroll
            for (int j = 0; j < NB; ++j)
                if (firstc) accA[k][j] = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) accB[k][c] = 0.0;
        }
        double wv = 0.0;
        // The view loop and the view index are the same on every lane, so the
        // view centres come through scalar loads and waiting for them never
        // waits for the vector loads of the next group.  The sums are loaded
        // without branches (an invalid lane reads its block's first slot, a
        // view past the end reads the last view) and masked where used.
        const int nvw = (!ADJ || firstc) ? n_views : 0;
        const float* slot = VS + (valid ? g : (list ? 0 : (int64_t)blockIdx.x * (blockDim.x >> 2))) * (int64_t)stride;
        const int64_t vstep = N * (int64_t)stride;
        constexpr int kGroup = 4;
        float cV[kGroup], cS[kGroup][4], nV[kGroup], nS[kGroup][4];
        auto load_group = [&](int v0, float (&gV)[kGroup], float (&gS)[kGroup][4]) {
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                const int vl = v0 + u < nvw ? v0 + u : nvw - 1;
                const float* p = slot + (int64_t)vl * vstep;
                gV[u] = p[0];
#pragma unroll
                for (int c = 0; c < 4; ++c) gS[u][c] = (!ADJ && c0 + c < C) ? p[1 + c0 + c] : 0.0f;
            }
        };
        if (nvw > 0) load_group(0, cV, cS);
#pragma unroll 1
        for (int v0 = 0; v0 < nvw; v0 += kGroup) {
            load_group(v0 + kGroup, nV, nS);
#pragma unroll
            for (int u = 0; u < kGroup; u += 2) {
                // two views at once: independent SH evaluations, in FP64 (as
                // fast as FP32 here, and no widening of the 16 values)
                double phd[2][NB];
                double Vd[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int v = v0 + u + h;
                    const bool use = valid && v < nvw && cV[u + h] != 0.0f;
                    const int vv = v < nvw ? v : 0;
                    double dir[3];
                    view_direction(mx, my, mz, views[vv].centre, dir);
                    sh_eval<double, L>(dir[0], dir[1], dir[2], phd[h]);
                    Vd[h] = use ? (double)cV[u + h] : 0.0;
                    // unused views add nothing to B (their sums read as 0)
#pragma unroll
                    for (int c = 0; c < 4; ++c) cS[u + h][c] = use ? cS[u + h][c] : 0.0f;
                }
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        double own = sel[0] * phd[h][4 * k];
#pragma unroll
                        for (int e = 1; e < 4; ++e)
                            if (4 * k + e < NB) own = fma(sel[e], phd[h][4 * k + e < NB ? 4 * k + e : 0], own);
                        if (firstc) {
                            const double vo = Vd[h] * own;
#pragma unroll
                            for (int j = 0; j < NB; ++j)
                                if (j < 4 * k + 4) accA[k][j] = fma(vo, phd[h][j], accA[k][j]);
                        }
                        if constexpr (!ADJ) {
#pragma unroll
                            for (int c = 0; c < 4; ++c) accB[k][c] = fma(own, (double)cS[u + h][c], accB[k][c]);
                        }
                    }
                }
                wv += Vd[0];
                wv += Vd[1];
            }
#pragma unroll
            for (int u = 0; u < kGroup; ++u) {
                cV[u] = nV[u];
#pragma unroll
                for (int c = 0; c < 4; ++c) cS[u][c] = nS[u][c];
            }
        }
        if (firstc) {
            wsum = wv;
            // regularise: the lane's own diagonal entries, selected arithmetically
#pragma unroll
            for (int k = 0; k < RPL; ++k)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (4 * k + e < NB)
                        accA[k][4 * k + e < NB ? 4 * k + e : 0] =
                            fma(sel[e] * wsum, lam.v[4 * k + e < NB ? 4 * k + e : 0],
                                accA[k][4 * k + e < NB ? 4 * k + e : 0]);
            // Right-looking Cholesky in registers.  Column j is scaled by its
            // owner rows, then each entry L[m][j] is broadcast from the lane
            // owning row m and every lane updates its own rows i >= m.
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                double djj;
                switch (j & 3) {
                    case 0: djj = quad_bcast<0>(accA[j >> 2][j]); break;
                    case 1: djj = quad_bcast<1>(accA[j >> 2][j]); break;
                    case 2: djj = quad_bcast<2>(accA[j >> 2][j]); break;
                    default: djj = quad_bcast<3>(accA[j >> 2][j]); break;
                }
                const bool bad = !(djj > 0.0);
                failed |= bad;
                const double d = bad ? 1.0 : sqrt(djj);
                const double id = 1.0 / d;
#pragma unroll
                for (int k = 0; k < RPL; ++k)
                    if (4 * k + 3 >= j) {
                        const int i = 4 * k + r;
                        accA[k][j] = i > j ? accA[k][j] * id : (i == j ? id : accA[k][j]);
                    }
#pragma unroll
                for (int m = j + 1; m < NB; ++m) {
                    double lmj;
                    switch (m & 3) {
                        case 0: lmj = quad_bcast<0>(accA[m >> 2][j]); break;
                        case 1: lmj = quad_bcast<1>(accA[m >> 2][j]); break;
                        case 2: lmj = quad_bcast<2>(accA[m >> 2][j]); break;
                        default: lmj = quad_bcast<3>(accA[m >> 2][j]); break;
                    }
#pragma unroll
                    for (int k = 0; k < RPL; ++k)
                        if (4 * k + 3 >= m) {  // rows 4k..4k+3 may reach column m
                            const bool act = 4 * k + r >= m;  // own row i = 4k + r needs i >= m
                            accA[k][m] = act ? fma(-accA[k][j], lmj, accA[k][m]) : accA[k][m];
                        }
                }
            }
            // keep the factor for refinement: row i at i (i + 1) / 2, 1/L_ii
            // on the diagonal, then w_g
            if constexpr (!ADJ) {
                if (factor != nullptr && valid) {
                    constexpr int NT = NB * (NB + 1) / 2;
                    double* F = factor + g * (int64_t)(NT + 1);
#pragma unroll
                    for (int k = 0; k < RPL; ++k) {
                        const int i = 4 * k + r;
#pragma unroll
                        for (int j = 0; j < NB; ++j)
                            if (j < 4 * k + 4 && j <= i && i < NB) F[i * (i + 1) / 2 + j] = accA[k][j];
                    }
                    if (r == 0) F[NT] = wsum;
                }
            }
        }
        if constexpr (ADJ) {
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int i = 4 * k + r;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    accB[k][c] = (valid && i < NB && c0 + c < C) ? (double)rhs[(g * NB + i) * C + c0 + c] : 0.0;
            }
        }
        // forward substitution L y = b: y_j = b_j / L_jj is broadcast from its
        // owner, and every lane updates its own rows m > j
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const int kj = j >> 2;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double t = accB[kj][c] * accA[kj][j];
                double yj;
                switch (j & 3) {
                    case 0: yj = quad_bcast<0>(t); break;
                    case 1: yj = quad_bcast<1>(t); break;
                    case 2: yj = quad_bcast<2>(t); break;
                    default: yj = quad_bcast<3>(t); break;
                }
                accB[kj][c] = r == (j & 3) ? yj : accB[kj][c];
#pragma unroll
                for (int k = 0; k < RPL; ++k)
                    if (4 * k + 3 > j) {
                        const bool act = 4 * k + r > j && 4 * k + r < NB;
                        accB[k][c] = act ? fma(-accA[k][j], yj, accB[k][c]) : accB[k][c];
                    }
            }
        }
        // back substitution L^T x = y: x_i = (y_i - sum_{k>i} L_ki x_k) / L_ii,
        // the sum taken over each lane's solved rows, then over the quad
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
            const int ki = i >> 2;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double p = 0.0;
#pragma unroll
                for (int k = 0; k < RPL; ++k)
                    if (4 * k + 3 > i) {
                        const bool act = 4 * k + r > i && 4 * k + r < NB;
                        p = act ? fma(accA[k][i], accB[k][c], p) : p;
                    }
                p = quad_sum(p);
                accB[ki][c] = r == (i & 3) ? (accB[ki][c] - p) * accA[ki][i] : accB[ki][c];
            }
        }
        const bool zero = wsum == 0.0 || failed;
        if (valid) {
            float* out = coeffs + g * NB * C;
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int i = 4 * k + r;
                if (i >= NB) continue;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    if (c0 + c >= C) continue;
                    out[i * C + c0 + c] = zero ? 0.0f : (float)accB[k][c];
                    if constexpr (ADJ) {
                        double lk = lam.v[4 * k];
#pragma unroll
                        for (int e = 1; e < 4; ++e)
                            if (4 * k + e < NB) lk = r == e ? lam.v[4 * k + e < NB ? 4 * k + e : 0] : lk;
                        if (!zero)
                            rho_part = fma(lk * accB[k][c], (double)cin[(g * NB + i) * C + c0 + c],
                                           rho_part);
                    }
                }
            }
        }
    }
    if constexpr (ADJ) {
        rho_part = quad_sum(rho_part);
        if (valid && r == 0) rho[g] = (float)rho_part;
        return;
    }
    // condition estimate from the extremes of 1/L_ii over the quad
    double imax = 0.0, imin = 1e300;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        double dk = accA[k][4 * k];
#pragma unroll
        for (int e = 1; e < 4; ++e)
            if (4 * k + e < NB) dk = r == e ? accA[k][4 * k + e < NB ? 4 * k + e : 0] : dk;
        if (4 * k + r < NB) {
            imax = fmax(imax, dk);
            imin = fmin(imin, dk);
        }
    }
    imax = quad_max(imax);
    imin = -quad_max(-imin);
    // Extreme eigenvalues of M = L L^T: eight steps of power iteration give
    // lambda_max >= x^T M x / x^T x = |L^T x|^2 / |x|^2 (and lambda_max >=
    // max_i M_ii), eight of inverse iteration give 1/lambda_min >=
    // |L^{-1} x|^2 / |x|^2.  Their product is a lower bound of kappa(M) that
    // is close once the iterates align with the extreme eigenvectors (slowest
    // when the largest eigenvalues cluster); with the pivot ratio above it is
    // the estimate.  Vectors are distributed like the rows of L (row 4k + r
    // on lane r); the starts are golden-ratio sequences, free of the
    // symmetries of the SH basis that a regular start can share.
    auto lval = [&](int k, int j) {  // L[4k + r][j] for j <= 4k + r
        const int i = 4 * k + r;
        return i == j ? 1.0 / accA[k][j] : accA[k][j];
    };
    auto norm2 = [&](const double (&x)[RPL]) {
        double p = 0.0;
#pragma unroll
        for (int k = 0; k < RPL; ++k) p = 4 * k + r < NB ? fma(x[k], x[k], p) : p;
        return quad_sum(p);
    };
    auto lt_mul = [&](const double (&x)[RPL], double (&u)[RPL]) {  // u = L^T x
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            double p = 0.0;
#pragma unroll
            for (int k = 0; k < RPL; ++k)
                if (4 * k + 3 >= j) p = (4 * k + r >= j && 4 * k + r < NB) ? fma(lval(k, j), x[k], p) : p;
            p = quad_sum(p);
            if (r == (j & 3)) u[j >> 2] = p;
        }
    };
    auto l_mul = [&](const double (&u)[RPL], double (&z)[RPL]) {  // z = L u
#pragma unroll
        for (int k = 0; k < RPL; ++k) z[k] = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const double uj = quad_from(u[j >> 2], j);
#pragma unroll
            for (int k = 0; k < RPL; ++k)
                if (4 * k + 3 >= j) z[k] = (4 * k + r >= j && 4 * k + r < NB) ? fma(lval(k, j), uj, z[k]) : z[k];
        }
    };
    auto l_solve = [&](double (&x)[RPL]) {  // x <- L^{-1} x
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            const double yj = quad_from(x[j >> 2] * accA[j >> 2][j], j);
            if (r == (j & 3)) x[j >> 2] = yj;
#pragma unroll
            for (int k = 0; k < RPL; ++k)
                if (4 * k + 3 > j) x[k] = (4 * k + r > j && 4 * k + r < NB) ? fma(-accA[k][j], yj, x[k]) : x[k];
        }
    };
    auto lt_solve = [&](double (&x)[RPL]) {  // x <- L^{-T} x
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
            double p = 0.0;
#pragma unroll
            for (int k = 0; k < RPL; ++k)
                if (4 * k + 3 > i) p = (4 * k + r > i && 4 * k + r < NB) ? fma(accA[k][i], x[k], p) : p;
            p = quad_sum(p);
            if (r == (i & 3)) x[i >> 2] = (x[i >> 2] - p) * accA[i >> 2][i];
        }
    };
    double xp[RPL], xi[RPL], tmp[RPL];
    double mdiag = 0.0;  // max_i M_ii = max_i sum_j L_ij^2
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
        const int i = 4 * k + r;
        const double fp = 0.6180339887498949 * i, fi = 0.7548776662466927 * i;
        xp[k] = i < NB ? 2.0 * (fp - floor(fp)) - 0.9 : 0.0;
        xi[k] = i < NB ? 2.0 * (fi - floor(fi)) - 0.9 : 0.0;
        double rn = 0.0;
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < 4 * k + 4) rn = (j <= i && i < NB) ? fma(lval(k, j), lval(k, j), rn) : rn;
        mdiag = fmax(mdiag, rn);
    }
    mdiag = quad_max(mdiag);
    double lmax_est = 0.0, sig = 0.0;
#pragma unroll 1
    for (int it = 0; it < 8; ++it) {
        const double np = norm2(xp), ni = norm2(xi);
        lt_mul(xp, tmp);
        lmax_est = norm2(tmp) / np;
        l_mul(tmp, xp);
        l_solve(xi);
        sig = norm2(xi) / ni;
        lt_solve(xi);
        const double sp = 1.0 / sqrt(norm2(xp)), si = 1.0 / sqrt(norm2(xi));
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            xp[k] *= sp;
            xi[k] *= si;
        }
    }
    if (valid && r == 0) {
        if (wout) wout[g] = (float)wsum;
        uint8_t st = 0;
        if (wsum == 0.0) {
            st = GSC_G_UNOBSERVED;
        } else if (failed) {
            st = GSC_G_FAILED;
        } else {
            const double kap = fmax((imax / imin) * (imax / imin), fmax(lmax_est, mdiag) * sig);
            if (kap > (double)kappa_max) {
                st = GSC_G_ILL_COND;
                if (ill_count) atomicAdd(ill_count, 1u);
            }
        }
        if (status) status[g] = st;
    }
}

// Observed-list pre-pass (one Gaussian per thread, blocks of 1024): a
// Gaussian is observed when some view gave it weight.  Its views' weights are
// loaded eight at a time (independent loads in flight together).
// Unobserved ones get their outputs here (zero coefficients,
// GSC_G_UNOBSERVED, w = 0); the observed ones are flagged and counted per
// block, then listed in index order.
__global__ __launch_bounds__(1024) void k_obs_count(const float* __restrict__ VS, int n_views, int64_t N,
                                                    int stride, int64_t row, float* __restrict__ coeffs,
                                                    uint8_t* __restrict__ status, float* __restrict__ wout,
                                                    uint8_t* __restrict__ flag,
                                                    uint32_t* __restrict__ block_counts) {
    __shared__ uint32_t wsum[16];
    const int64_t g = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    bool seen = false;
    if (g < N) {
        for (int v0 = 0; v0 < n_views && !seen; v0 += 8) {
            float x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = v0 + u < n_views ? VS[((int64_t)(v0 + u) * N + g) * stride] : 0.0f;
#pragma unroll
            for (int u = 0; u < 8; ++u) seen |= x[u] > 0.0f;
        }
        flag[g] = seen ? 1 : 0;
        if (!seen) {
            for (int64_t i = 0; i < row; ++i) coeffs[g * row + i] = 0.0f;
            if (status) status[g] = GSC_G_UNOBSERVED;
            if (wout) wout[g] = 0.0f;
        }
    }
    const uint64_t bal = __builtin_amdgcn_ballot_w64(seen);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = (uint32_t)__popcll(bal);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < 16; ++w) t += wsum[w];
        block_counts[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_obs_scatter(const uint8_t* __restrict__ flag, int64_t N,
                                                      const uint32_t* __restrict__ block_offsets,
                                                      uint32_t* __restrict__ list) {
    __shared__ uint32_t wcnt[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * 1024 + threadIdx.x;
    const bool o = g < N && flag[g] != 0;
    const uint64_t bal = __builtin_amdgcn_ballot_w64(o);
    if (lane == 0) wcnt[wave] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = block_offsets[blockIdx.x];
    for (int w = 0; w < wave; ++w) before += wcnt[w];
    const uint64_t lt = lane ? (bal & (~0ull >> (64 - lane))) : 0ull;
    if (o) list[before + (uint32_t)__popcll(lt)] = (uint32_t)g;
}

void launch_fold_solve(const ViewInfo* views, int n_views, const float* means, const float* VS,
                       bool per_view, int64_t N, int C, int sh_deg, const double* lam_nb,
                       float kappa_max, float* coeffs, uint8_t* status, float* wout,
                       float* dc_scratch, unsigned int* ill_count, hipStream_t s, double* factor,
                       uint32_t* obs_scratch) {
    if (N <= 0) return;
    if (sh_deg == 0) {
        const float* src = VS;
        if (per_view) {
            int64_t n = N * (int64_t)(C + 1);
            hipLaunchKernelGGL(k_sum_views, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, VS,
                               n_views, N, C + 1, dc_scratch);
            src = dc_scratch;
        }
        hipLaunchKernelGGL(k_solve_dc, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, src, N, C,
                           lam_nb[0], coeffs, status, wout);
        return;
    }
    LamNB lam;
    for (int i = 0; i < kMaxNb; ++i) lam.v[i] = 0.0;
    int nb = (sh_deg + 1) * (sh_deg + 1);
    for (int i = 0; i < nb; ++i) lam.v[i] = lam_nb[i];
    // one wave (16 Gaussians) per block: at one wave per SIMD a block then
    // starts on any free SIMD, not only when four are free on one CU
    dim3 grid((unsigned)((N + 15) / 16)), block(64);
    const float* nf = nullptr;
    float* nw = nullptr;
    const uint32_t* list = nullptr;
    const int64_t* n_list = nullptr;
    if (obs_scratch && per_view && n_views > 0) {
        // layout: list [N], block counts [nblk], int64 total (8-byte aligned), flags [N bytes]
        const int nblk = (int)((N + 1023) / 1024);
        uint32_t* lst = obs_scratch;
        uint32_t* blocks = obs_scratch + N;
        const int64_t t_word = (N + nblk + 1) & ~(int64_t)1;
        int64_t* total = reinterpret_cast<int64_t*>(obs_scratch + t_word);
        uint8_t* flag = reinterpret_cast<uint8_t*>(obs_scratch + t_word + 2);
        hipLaunchKernelGGL(k_obs_count, dim3(nblk), dim3(1024), 0, s, VS, n_views, N, C + 1,
                           (int64_t)nb * C, coeffs, status, wout, flag, blocks);
        launch_block_scan(blocks, nblk, total, s);
        hipLaunchKernelGGL(k_obs_scatter, dim3(nblk), dim3(1024), 0, s, flag, N, blocks, lst);
        list = lst;
        n_list = total;
    }
    switch (sh_deg) {
        case 1: hipLaunchKernelGGL((k_fold_solve<1, false>), grid, block, 0, s, views, n_views, means, VS, C + 1, N, C, lam, kappa_max, nf, nf, coeffs, nw, status, wout, ill_count, factor, list, n_list); break;
        case 2: hipLaunchKernelGGL((k_fold_solve<2, false>), grid, block, 0, s, views, n_views, means, VS, C + 1, N, C, lam, kappa_max, nf, nf, coeffs, nw, status, wout, ill_count, factor, list, n_list); break;
        default: hipLaunchKernelGGL((k_fold_solve<3, false>), grid, block, 0, s, views, n_views, means, VS, C + 1, N, C, lam, kappa_max, nf, nf, coeffs, nw, status, wout, ill_count, factor, list, n_list); break;
    }
}

// ---- refinement (Algorithm 1, steps 8-10) --------------------------------
//
// One thread per Gaussian: fold the residual's per-view sums into
// B = sum_j phi_gj S_gj^T in FP64 (four channels at a time, the SH values of
// each view evaluated as in the fold above), form B - w_g Lambda c_g and solve
// with the factor stored by the first pass (forward substitution L y = rhs,
// back substitution L^T x = y, 1/L_ii kept on the diagonal), then c_g += x.
template <int L>
__global__ __launch_bounds__(256) void k_refine_update(const ViewInfo* __restrict__ views, int n_views,
                                                       const float* __restrict__ means,
                                                       const float* __restrict__ VS, int64_t N, int C,
                                                       LamNB lam, const double* __restrict__ factor,
                                                       const uint8_t* __restrict__ status,
                                                       float* __restrict__ coeffs) {
    constexpr int NB = (L + 1) * (L + 1);
    constexpr int NT = NB * (NB + 1) / 2;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    if (status[g] & (GSC_G_UNOBSERVED | GSC_G_FAILED)) return;
    const double* F = factor + g * (int64_t)(NT + 1);
    const double wg = F[NT];
    const float mx = means[3 * g], my = means[3 * g + 1], mz = means[3 * g + 2];
    const int stride = C + 1;
    const int64_t vstep = N * (int64_t)stride;
    float* out = coeffs + g * NB * C;
    for (int c0 = 0; c0 < C; c0 += 4) {
        double b[NB][4];
#pragma unroll
        for (int m = 0; m < NB; ++m)
#pragma unroll
            for (int c = 0; c < 4; ++c) b[m][c] = 0.0;
        for (int v = 0; v < n_views; ++v) {
            const float* p = VS + (int64_t)v * vstep + g * stride;
            if (p[0] == 0.0f) continue;  // no contribution in this view
            double dir[3];
            view_direction(mx, my, mz, views[v].centre, dir);
            double ph[NB];
            sh_eval<double, L>(dir[0], dir[1], dir[2], ph);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const double sc = c0 + c < C ? (double)p[1 + c0 + c] : 0.0;
#pragma unroll
                for (int m = 0; m < NB; ++m) b[m][c] = fma(ph[m], sc, b[m][c]);
            }
        }
#pragma unroll
        for (int m = 0; m < NB; ++m)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c0 + c < C) b[m][c] = fma(-wg * lam.v[m], (double)out[m * C + c0 + c], b[m][c]);
        // L y = rhs
#pragma unroll
        for (int i = 0; i < NB; ++i) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double t = b[i][c];
#pragma unroll
                for (int j = 0; j < i; ++j) t = fma(-F[i * (i + 1) / 2 + j], b[j][c], t);
                b[i][c] = t * F[i * (i + 1) / 2 + i];
            }
        }
        // L^T x = y
#pragma unroll
        for (int i = NB - 1; i >= 0; --i) {
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double t = b[i][c];
#pragma unroll
                for (int k = i + 1; k < NB; ++k) t = fma(-F[k * (k + 1) / 2 + i], b[k][c], t);
                b[i][c] = t * F[i * (i + 1) / 2 + i];
            }
        }
#pragma unroll
        for (int m = 0; m < NB; ++m)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c0 + c < C) out[m * C + c0 + c] = (float)((double)out[m * C + c0 + c] + b[m][c]);
    }
}

// L = 0: the matrix is w_g (Y0^2 + lambda_0) and B = Y0 S_g (VS summed over views).
__global__ void k_refine_update_dc(const float* __restrict__ VS, int64_t N, int C, double lam0,
                                   const float* __restrict__ w, const uint8_t* __restrict__ status,
                                   float* __restrict__ coeffs) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    if (status[g] & (GSC_G_UNOBSERVED | GSC_G_FAILED)) return;
    const double wg = w[g];
    const float* sg = VS + g * (int64_t)(C + 1);
    const double den = wg * (kY0 * kY0 + lam0);
    for (int c = 0; c < C; ++c) {
        const double cg = coeffs[g * C + c];
        coeffs[g * C + c] = (float)(cg + (kY0 * (double)sg[1 + c] - wg * lam0 * cg) / den);
    }
}

void launch_refine_update(const ViewInfo* views, int n_views, const float* means, const float* VS,
                          int64_t N, int C, int sh_deg, const double* lam_nb, const double* factor,
                          const float* w, const uint8_t* status, float* coeffs, hipStream_t s) {
    if (N <= 0) return;
    const dim3 grid((unsigned)((N + 255) / 256)), block(256);
    if (sh_deg == 0) {
        hipLaunchKernelGGL(k_refine_update_dc, grid, block, 0, s, VS, N, C, lam_nb[0], w, status, coeffs);
        return;
    }
    LamNB lam;
    for (int i = 0; i < kMaxNb; ++i) lam.v[i] = 0.0;
    const int nb = (sh_deg + 1) * (sh_deg + 1);
    for (int i = 0; i < nb; ++i) lam.v[i] = lam_nb[i];
    switch (sh_deg) {
        case 1: hipLaunchKernelGGL((k_refine_update<1>), grid, block, 0, s, views, n_views, means, VS, N, C, lam, factor, status, coeffs); break;
        case 2: hipLaunchKernelGGL((k_refine_update<2>), grid, block, 0, s, views, n_views, means, VS, N, C, lam, factor, status, coeffs); break;
        default: hipLaunchKernelGGL((k_refine_update<3>), grid, block, 0, s, views, n_views, means, VS, N, C, lam, factor, status, coeffs); break;
    }
}

// Residual targets in place over the pixels of a batch's views (grid y: view).
__global__ __launch_bounds__(256) void k_residual(const ViewInfo* __restrict__ views, const void* __restrict__ y,
                                                  int ydtype, int C, float* __restrict__ img) {
    const ViewInfo& V = views[blockIdx.y];
    const int64_t n = (int64_t)V.width * V.height * C;
    const int64_t base = V.pixel_offset * (int64_t)C;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = base + i;
        const float yv = ydtype == GSC_BF16 ? __uint_as_float((uint32_t)((const uint16_t*)y)[e] << 16)
                                            : ((const float*)y)[e];
        img[e] = yv - img[e];
    }
}

void launch_residual(const ViewInfo* views, int n_views, int max_pixels, const void* y, int ydtype,
                     int C, float* img, hipStream_t s) {
    if (n_views <= 0 || max_pixels <= 0) return;
    const int64_t per = (int64_t)max_pixels * C;
    const unsigned bx = (unsigned)std::min<int64_t>((per + 255) / 256, 1024);
    hipLaunchKernelGGL(k_residual, dim3(bx, (unsigned)n_views), dim3(256), 0, s, views, y, ydtype, C, img);
}

// L = 0 adjoint: A_g + w_g Lambda = w_g (Y0^2 + lambda_0).
__global__ void k_adjoint_dc(const float* __restrict__ W, int64_t N, int C, double lam0,
                             const float* __restrict__ gc, const float* __restrict__ cin,
                             float* __restrict__ bbar, float* __restrict__ rho) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    const double w = W[g];
    double r = 0.0;
    for (int c = 0; c < C; ++c) {
        const double b = w == 0.0 ? 0.0 : (double)gc[g * C + c] / (w * (kY0 * kY0 + lam0));
        bbar[g * C + c] = (float)b;
        r += lam0 * b * (double)cin[g * C + c];
    }
    rho[g] = (float)r;
}

void launch_adjoint_solve(const ViewInfo* views, int n_views, const float* means, const float* V,
                          bool per_view, int64_t N, int C, int sh_deg, const double* lam_nb,
                          const float* grad_coeffs, const float* coeffs, float* bbar, float* rho,
                          float* w_scratch, hipStream_t s) {
    if (N <= 0) return;
    if (sh_deg == 0) {
        const float* src = V;
        if (per_view) {
            hipLaunchKernelGGL(k_sum_views, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, V,
                               n_views, N, 1, w_scratch);
            src = w_scratch;
        }
        hipLaunchKernelGGL(k_adjoint_dc, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, src, N,
                           C, lam_nb[0], grad_coeffs, coeffs, bbar, rho);
        return;
    }
    LamNB lam;
    for (int i = 0; i < kMaxNb; ++i) lam.v[i] = 0.0;
    int nb = (sh_deg + 1) * (sh_deg + 1);
    for (int i = 0; i < nb; ++i) lam.v[i] = lam_nb[i];
    // one wave (16 Gaussians) per block: at one wave per SIMD a block then
    // starts on any free SIMD, not only when four are free on one CU
    dim3 grid((unsigned)((N + 15) / 16)), block(64);
    uint8_t* ns = nullptr;
    float* nw = nullptr;
    unsigned int* ni = nullptr;
    switch (sh_deg) {
        case 1: hipLaunchKernelGGL((k_fold_solve<1, true>), grid, block, 0, s, views, n_views, means, V, 1, N, C, lam, 0.0f, grad_coeffs, coeffs, bbar, rho, ns, nw, ni, nullptr, nullptr, nullptr); break;
        case 2: hipLaunchKernelGGL((k_fold_solve<2, true>), grid, block, 0, s, views, n_views, means, V, 1, N, C, lam, 0.0f, grad_coeffs, coeffs, bbar, rho, ns, nw, ni, nullptr, nullptr, nullptr); break;
        default: hipLaunchKernelGGL((k_fold_solve<3, true>), grid, block, 0, s, views, n_views, means, V, 1, N, C, lam, 0.0f, grad_coeffs, coeffs, bbar, rho, ns, nw, ni, nullptr, nullptr, nullptr); break;
    }
}

}  // namespace gsc
