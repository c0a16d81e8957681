// Fold of the per-view sums into the normal equations and the regularised
// solve (eqs. 11-14, Algorithm 1 steps 5-6).
//
// L >= 1: four lanes per Gaussian.  Lane r owns the rows i = 4k + r of
//   A_g = sum_j V_gj phi_gj phi_gj^T  and  B_g = sum_j phi_gj S_gj^T
// and accumulates them over the views in FP64 registers (FP32 accumulation
// of A over tens of views loses ~1e-4 relative at the condition numbers the
// paper's Lambda produces).  The quad then writes A_g + w_g Lambda to LDS,
// factors it with a cooperative FP64 Cholesky and each lane solves one
// right-hand-side column.  The factor stays in LDS for further channel
// chunks of four.
// L = 0: A_g = w_g Y0^2 is a scalar and c_g = Y0 S_g / (w_g (Y0^2 + lambda_0)).
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

template <int L>
__global__ __launch_bounds__(64) void k_fold_solve(const ViewInfo* __restrict__ views, int n_views,
                                                   const float* __restrict__ means,
                                                   const float* __restrict__ VS, int64_t N, int C,
                                                   LamNB lam, float kappa_max,
                                                   float* __restrict__ coeffs,
                                                   uint8_t* __restrict__ status,
                                                   float* __restrict__ wout,
                                                   unsigned int* __restrict__ ill_count) {
    constexpr int NB = (L + 1) * (L + 1);
    constexpr int RPL = (NB + 3) / 4;  // rows per lane
    constexpr int LDA = NB + 1;
    __shared__ double As[16][NB * LDA];
    __shared__ double Bs[16][NB * 4];
    __shared__ double Dg[16][NB];
    const int lane = threadIdx.x, q = lane >> 2, r = lane & 3;
    const int64_t g = (int64_t)blockIdx.x * 16 + q;
    const bool valid = g < N;
    const int stride = C + 1;
    double* A = As[q];
    double* Bq = Bs[q];
    double mx = 0, my = 0, mz = 0;
    if (valid) {
        mx = means[3 * g];
        my = means[3 * g + 1];
        mz = means[3 * g + 2];
    }
    bool failed = false;
    double wsum = 0.0;
    for (int c0 = 0; c0 < C; c0 += 4) {
        const bool firstc = c0 == 0;
        double accA[RPL][NB];
        double accB[RPL][4];
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
#pragma unroll
            for (int j = 0; j < NB && j < 4 * k + 4; ++j) accA[k][j] = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) accB[k][c] = 0.0;
        }
        double wv = 0.0;
        if (valid) {
            for (int v = 0; v < n_views; ++v) {
                const float* slot = VS + ((int64_t)v * N + g) * stride;
                const float Vf = slot[0];
                if (Vf == 0.0f) continue;
                const double Vd = Vf;
                const ViewInfo& Vi = views[v];
                double dx = mx - Vi.centre[0], dy = my - Vi.centre[1], dz = mz - Vi.centre[2];
                double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
                double phi[NB];
                sh_eval<double, L>(dx * inv, dy * inv, dz * inv, phi);
                double S[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) S[c] = (c0 + c < C) ? (double)slot[1 + c0 + c] : 0.0;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    double own = phi[4 * k];
                    if (4 * k + 1 < NB && r == 1) own = phi[4 * k + 1 < NB ? 4 * k + 1 : 0];
                    if (4 * k + 2 < NB && r == 2) own = phi[4 * k + 2 < NB ? 4 * k + 2 : 0];
                    if (4 * k + 3 < NB && r == 3) own = phi[4 * k + 3 < NB ? 4 * k + 3 : 0];
                    if (firstc) {
                        // lower triangle only: row 4k+r needs columns j <= 4k+r
                        const double vo = Vd * own;
#pragma unroll
                        for (int j = 0; j < NB && j < 4 * k + 4; ++j) accA[k][j] += vo * phi[j];
                    }
#pragma unroll
                    for (int c = 0; c < 4; ++c) accB[k][c] += own * S[c];
                }
                wv += Vd;
            }
        }
        if (firstc) wsum = wv;
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int i = 4 * k + r;
            if (i < NB) {
                if (firstc) {
#pragma unroll
                    for (int j = 0; j < NB && j < 4 * k + 4; ++j)
                        if (j <= i) A[i * LDA + j] = accA[k][j];
                    A[i * LDA + i] += wsum * lam.v[i];
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) Bq[i * 4 + c] = accB[k][c];
            }
        }
        __syncthreads();
        if (firstc) {
            // Right-looking Cholesky of the lower triangle, rows split over the quad.
#pragma unroll 1
            for (int j = 0; j < NB; ++j) {
                double d = A[j * LDA + j];
                const bool bad = !(d > 0.0);
                failed |= bad;
                d = bad ? 1.0 : sqrt(d);
                const double id = 1.0 / d;
                for (int i = j + 1; i < NB; ++i)
                    if ((i & 3) == r) A[i * LDA + j] *= id;
                if (r == 0) Dg[q][j] = d;
                __syncthreads();
                for (int i = j + 1; i < NB; ++i) {
                    if ((i & 3) == r) {
                        const double lij = A[i * LDA + j];
                        for (int k = j + 1; k <= i; ++k) A[i * LDA + k] -= lij * A[k * LDA + j];
                    }
                }
                __syncthreads();
            }
        }
        const int c = c0 + r;
        if (valid && c < C) {
            double x[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) x[i] = Bq[i * 4 + r];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                double s = x[i];
#pragma unroll
                for (int k = 0; k < i; ++k) s -= A[i * LDA + k] * x[k];
                x[i] = s / Dg[q][i];
            }
#pragma unroll
            for (int i = NB - 1; i >= 0; --i) {
                double s = x[i];
#pragma unroll
                for (int k = i + 1; k < NB; ++k) s -= A[k * LDA + i] * x[k];
                x[i] = s / Dg[q][i];
            }
            const bool zero = wsum == 0.0 || failed;
            float* out = coeffs + g * NB * C;
#pragma unroll
            for (int i = 0; i < NB; ++i) out[i * C + c] = zero ? 0.0f : (float)x[i];
        }
        __syncthreads();
    }
    if (valid && r == 0) {
        if (wout) wout[g] = (float)wsum;
        uint8_t st = 0;
        if (wsum == 0.0) {
            st = GSC_G_UNOBSERVED;
        } else if (failed) {
            st = GSC_G_FAILED;
        } else {
            double dmax = 0.0, dmin = 1e300;
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                dmax = fmax(dmax, Dg[q][i]);
                dmin = fmin(dmin, Dg[q][i]);
            }
            const double kap = (dmax / dmin) * (dmax / dmin);
            if (kap > (double)kappa_max) {
                st = GSC_G_ILL_COND;
                atomicAdd(ill_count, 1u);
            }
        }
        if (status) status[g] = st;
    }
}

void launch_fold_solve(const ViewInfo* views, int n_views, const float* means, const float* VS,
                       bool per_view, int64_t N, int C, int sh_deg, const double* lam_nb,
                       float kappa_max, float* coeffs, uint8_t* status, float* wout,
                       float* dc_scratch, unsigned int* ill_count, hipStream_t s) {
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
    dim3 grid((unsigned)((N + 15) / 16)), block(64);
    switch (sh_deg) {
        case 1: hipLaunchKernelGGL(k_fold_solve<1>, grid, block, 0, s, views, n_views, means, VS, N, C, lam, kappa_max, coeffs, status, wout, ill_count); break;
        case 2: hipLaunchKernelGGL(k_fold_solve<2>, grid, block, 0, s, views, n_views, means, VS, N, C, lam, kappa_max, coeffs, status, wout, ill_count); break;
        default: hipLaunchKernelGGL(k_fold_solve<3>, grid, block, 0, s, views, n_views, means, VS, N, C, lam, kappa_max, coeffs, status, wout, ill_count); break;
    }
}

}  // namespace gsc
