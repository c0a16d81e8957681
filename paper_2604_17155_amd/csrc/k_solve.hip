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

constexpr int kStageFloats = 2048;  // LDS staging of per-view sums (8 KB)
constexpr int kMaxStageViews = 64;

// Broadcast lane `o` of each quad to the whole quad (DPP quad_perm [o,o,o,o]).
template <int O>
__device__ __forceinline__ double quad_bcast(double x) {
    constexpr int ctrl = O | (O << 2) | (O << 4) | (O << 6);
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double quad_bcast_rt(double x, int o) {
    switch (o) {
        case 0: return quad_bcast<0>(x);
        case 1: return quad_bcast<1>(x);
        case 2: return quad_bcast<2>(x);
        default: return quad_bcast<3>(x);
    }
}

// Fold + solve for L >= 1.  Four lanes per Gaussian; lane r owns the rows
// i = 4k + r of A (lower triangle, FP64) and of B (four channels at a time).
// The Cholesky factor is formed in registers (column j broadcast within the
// quad), then L and B go through LDS so each lane can substitute one channel.
//
// ADJ: adjoint solve for the backward pass.  VS then holds only the per-view
// visibilities (stride 1); the right-hand sides are read from `rhs`
// (dL/dc, [N][NB][C]) instead of being folded, the solution
// Bbar = (A + w Lambda)^{-1} dL/dc is written to `out`, and
// rho_g = sum_{m,c} lambda_m Bbar[m][c] cin[m][c] (cin = the forward
// coefficients) to rho[g].
template <int L, bool ADJ>
__global__ __launch_bounds__(64) void k_fold_solve(const ViewInfo* __restrict__ views, int n_views,
                                                   const float* __restrict__ means,
                                                   const float* __restrict__ VS, int vs_stride,
                                                   int64_t N, int C, LamNB lam, float kappa_max,
                                                   const float* __restrict__ rhs,
                                                   const float* __restrict__ cin,
                                                   float* __restrict__ coeffs,
                                                   float* __restrict__ rho,
                                                   uint8_t* __restrict__ status,
                                                   float* __restrict__ wout,
                                                   unsigned int* __restrict__ ill_count) {
    constexpr int NB = (L + 1) * (L + 1);
    constexpr int RPL = (NB + 3) / 4;  // rows per lane
    constexpr int NL = NB * (NB + 1) / 2;  // packed lower triangle
    __shared__ float stage[kStageFloats];
    __shared__ float cen[kMaxStageViews][3];
    __shared__ double Ls[16][NL];
    __shared__ double Bs[16][NB * 4];
    const int lane = threadIdx.x, q = lane >> 2, r = lane & 3;
    const int64_t g0 = (int64_t)blockIdx.x * 16;
    const int64_t g = g0 + q;
    const bool valid = g < N;
    const int stride = vs_stride;
    const int per_view = 16 * stride;
    const int vch = max(1, min(kMaxStageViews, kStageFloats / per_view));
    const int64_t lim = N * (int64_t)stride;
    float mx = 0.f, my = 0.f, mz = 0.f;
    if (valid) {
        mx = means[3 * g];
        my = means[3 * g + 1];
        mz = means[3 * g + 2];
    }
    double sel[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) sel[e] = r == e ? 1.0 : 0.0;
    double accA[RPL][NB];  // accA[k][j]: row 4k+r, column j <= 4k+r
    double dinv[NB];       // reciprocal diagonal of the factor
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
        for (int v0 = 0; v0 < ((!ADJ || firstc) ? n_views : 0); v0 += vch) {
            const int nv = min(vch, n_views - v0);
            __syncthreads();
            // coalesced staging: for each view the block's 16 slots are
            // contiguous; eight independent loads per lane are in flight
            const int total = nv * per_view;
            for (int base = lane; base < total; base += 64 * 8) {
                float tmp[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const int idx = base + 64 * u;
                    const int vv = idx / per_view, rr = idx - vv * per_view;
                    const int64_t gi = g0 * stride + rr;
                    tmp[u] = (idx < total && gi < lim) ? VS[(int64_t)(v0 + vv) * lim + gi] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (base + 64 * u < total) stage[base + 64 * u] = tmp[u];
            }
            for (int idx = lane; idx < nv; idx += 64) {
                cen[idx][0] = (float)views[v0 + idx].centre[0];
                cen[idx][1] = (float)views[v0 + idx].centre[1];
                cen[idx][2] = (float)views[v0 + idx].centre[2];
            }
            __syncthreads();
            if (!valid) continue;
#pragma unroll 1
            for (int vv = 0; vv < nv; ++vv) {
                const float* slot = stage + vv * per_view + q * stride;
                const float Vf = slot[0];
                if (Vf == 0.0f) continue;
                const float dx = mx - cen[vv][0], dy = my - cen[vv][1], dz = mz - cen[vv][2];
                const float inv = rsqrtf(dx * dx + dy * dy + dz * dz);
                float phf[NB];
                sh_eval<float, L>(dx * inv, dy * inv, dz * inv, phf);
                double phi[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) phi[j] = (double)phf[j];
                const double Vd = Vf;
                double S[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) S[c] = (!ADJ && c0 + c < C) ? (double)slot[1 + c0 + c] : 0.0;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    // phi of this lane's row 4k + r, selected arithmetically
                    double own = sel[0] * phi[4 * k];
#pragma unroll
                    for (int e = 1; e < 4; ++e)
                        if (4 * k + e < NB) own = fma(sel[e], phi[4 * k + e < NB ? 4 * k + e : 0], own);
                    if (firstc) {
                        const double vo = Vd * own;
#pragma unroll
                        for (int j = 0; j < NB; ++j)
                            if (j < 4 * k + 4) accA[k][j] = fma(vo, phi[j], accA[k][j]);
                    }
                    if constexpr (!ADJ) {
#pragma unroll
                        for (int c = 0; c < 4; ++c) accB[k][c] = fma(own, S[c], accB[k][c]);
                    }
                }
                wv += Vd;
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
                const double djj = quad_bcast_rt(accA[j >> 2][j], j & 3);
                const bool bad = !(djj > 0.0);
                failed |= bad;
                const double d = bad ? 1.0 : sqrt(djj);
                const double id = 1.0 / d;
                dinv[j] = id;
#pragma unroll
                for (int k = 0; k < RPL; ++k)
                    if (4 * k + 3 > j) accA[k][j] = (4 * k + r > j) ? accA[k][j] * id : accA[k][j];
#pragma unroll
                for (int m = j + 1; m < NB; ++m) {
                    const double lmj = quad_bcast_rt(accA[m >> 2][j], m & 3);
#pragma unroll
                    for (int k = 0; k < RPL; ++k)
                        if (4 * k + 3 >= m) {  // rows 4k..4k+3 may reach column m
                            const bool act = 4 * k + r >= m;  // own row i = 4k + r needs i >= m
                            accA[k][m] = act ? fma(-accA[k][j], lmj, accA[k][m]) : accA[k][m];
                        }
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
        // factor (packed lower, diagonal stored as 1/L_ii) and right-hand sides to LDS
        if (firstc) {
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int i = 4 * k + r;
#pragma unroll
                for (int j = 0; j < NB; ++j)
                    if (j < 4 * k + 4 && i < NB && j <= i)
                        Ls[q][i * (i + 1) / 2 + j] = (j == i) ? dinv[j] : accA[k][j];
            }
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            const int i = 4 * k + r;
            if (i < NB) {
#pragma unroll
                for (int c = 0; c < 4; ++c) Bs[q][i * 4 + c] = accB[k][c];
            }
        }
        __syncthreads();
        const int c = c0 + r;
        if (valid && c < C) {
            double* x = Bs[q] + r;
            const double* Lq = Ls[q];
#pragma unroll 1
            for (int i = 0; i < NB; ++i) {
                double s = x[i * 4];
                const double* row = Lq + i * (i + 1) / 2;
                for (int k = 0; k < i; ++k) s -= row[k] * x[k * 4];
                x[i * 4] = s * row[i];
            }
#pragma unroll 1
            for (int i = NB - 1; i >= 0; --i) {
                double s = x[i * 4];
                for (int k = i + 1; k < NB; ++k) s -= Lq[k * (k + 1) / 2 + i] * x[k * 4];
                x[i * 4] = s * Lq[i * (i + 1) / 2 + i];
            }
            const bool zero = wsum == 0.0 || failed;
            float* out = coeffs + g * NB * C;
            for (int i = 0; i < NB; ++i) out[i * C + c] = zero ? 0.0f : (float)x[i * 4];
            if constexpr (ADJ) {
                if (!zero)
                    for (int i = 0; i < NB; ++i)
                        rho_part = fma(lam.v[i] * x[i * 4], (double)cin[(g * NB + i) * C + c], rho_part);
            }
        }
        __syncthreads();
    }
    if constexpr (ADJ) {
        rho_part += __shfl_xor(rho_part, 1, 64);
        rho_part += __shfl_xor(rho_part, 2, 64);
        if (valid && r == 0) rho[g] = (float)rho_part;
        return;
    }
    if (valid && r == 0) {
        if (wout) wout[g] = (float)wsum;
        uint8_t st = 0;
        if (wsum == 0.0) {
            st = GSC_G_UNOBSERVED;
        } else if (failed) {
            st = GSC_G_FAILED;
        } else {
            double imax = 0.0, imin = 1e300;  // extremes of 1/L_ii
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                imax = fmax(imax, dinv[i]);
                imin = fmin(imin, dinv[i]);
            }
            const double kap = (imax / imin) * (imax / imin);
            if (kap > (double)kappa_max) {
                st = GSC_G_ILL_COND;
                if (ill_count) atomicAdd(ill_count, 1u);
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
    const float* nf = nullptr;
    float* nw = nullptr;
    switch (sh_deg) {
        case 1: hipLaunchKernelGGL((k_fold_solve<1, false>), grid, block, 0, s, views, n_views, means, VS, C + 1, N, C, lam, kappa_max, nf, nf, coeffs, nw, status, wout, ill_count); break;
        case 2: hipLaunchKernelGGL((k_fold_solve<2, false>), grid, block, 0, s, views, n_views, means, VS, C + 1, N, C, lam, kappa_max, nf, nf, coeffs, nw, status, wout, ill_count); break;
        default: hipLaunchKernelGGL((k_fold_solve<3, false>), grid, block, 0, s, views, n_views, means, VS, C + 1, N, C, lam, kappa_max, nf, nf, coeffs, nw, status, wout, ill_count); break;
    }
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
    dim3 grid((unsigned)((N + 15) / 16)), block(64);
    uint8_t* ns = nullptr;
    float* nw = nullptr;
    unsigned int* ni = nullptr;
    switch (sh_deg) {
        case 1: hipLaunchKernelGGL((k_fold_solve<1, true>), grid, block, 0, s, views, n_views, means, V, 1, N, C, lam, 0.0f, grad_coeffs, coeffs, bbar, rho, ns, nw, ni); break;
        case 2: hipLaunchKernelGGL((k_fold_solve<2, true>), grid, block, 0, s, views, n_views, means, V, 1, N, C, lam, 0.0f, grad_coeffs, coeffs, bbar, rho, ns, nw, ni); break;
        default: hipLaunchKernelGGL((k_fold_solve<3, true>), grid, block, 0, s, views, n_views, means, V, 1, N, C, lam, 0.0f, grad_coeffs, coeffs, bbar, rho, ns, nw, ni); break;
    }
}

}  // namespace gsc
