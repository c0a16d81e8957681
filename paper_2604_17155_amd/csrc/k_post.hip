// Post-processing of solved coefficients (Sec. 4.1 qualitative results and
// Sec. 4.3): linear combinations of coefficient sets with per-channel colour
// filters, and the segmentation filter that keeps the Gaussians whose mask
// value reaches a threshold, compacted in index order.
#include <algorithm>

#include "gsc_internal.h"

namespace gsc {

// out[i] = f[i mod C] * sum_k w_k sets_k[i]  (one FP32 fma chain in k order).
// With `accumulate`, out[i] already holds the sum over earlier sets and
// continues it.  `vec4`: every pointer 16-byte aligned and n divisible by 4.
template <bool VEC4>
__global__ __launch_bounds__(256) void k_combine(CombineArgs a, int64_t n, int C, float* out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (VEC4) {
        for (; 4 * t < n; t += stride) {
            float4 acc = a.accumulate ? reinterpret_cast<const float4*>(out)[t] : make_float4(0.f, 0.f, 0.f, 0.f);
            for (int k = 0; k < a.n; ++k) {
                const float4 x = reinterpret_cast<const float4*>(a.p[k])[t];
                const float w = a.w[k];
                acc.x = fmaf(w, x.x, acc.x);
                acc.y = fmaf(w, x.y, acc.y);
                acc.z = fmaf(w, x.z, acc.z);
                acc.w = fmaf(w, x.w, acc.w);
            }
            if (a.filter) {
                const int c0 = (int)((4 * t) % C);
                acc.x *= a.f[c0];
                acc.y *= a.f[(c0 + 1) % C];
                acc.z *= a.f[(c0 + 2) % C];
                acc.w *= a.f[(c0 + 3) % C];
            }
            reinterpret_cast<float4*>(out)[t] = acc;
        }
    } else {
        for (; t < n; t += stride) {
            float acc = a.accumulate ? out[t] : 0.0f;
            for (int k = 0; k < a.n; ++k) acc = fmaf(a.w[k], a.p[k][t], acc);
            if (a.filter) acc *= a.f[(int)(t % C)];
            out[t] = acc;
        }
    }
}

void launch_combine(const CombineArgs& a, int64_t n, int C, bool vec4, float* out, hipStream_t s) {
    if (n <= 0) return;
    const int64_t units = vec4 ? n / 4 : n;
    // enough blocks to fill every CU several times; each thread strides on
    const int64_t want = (units + 255) / 256;
    const unsigned blocks = (unsigned)std::min<int64_t>(want, 256 * 16);
    if (vec4)
        hipLaunchKernelGGL(k_combine<true>, dim3(blocks), dim3(256), 0, s, a, n, C, out);
    else
        hipLaunchKernelGGL(k_combine<false>, dim3(blocks), dim3(256), 0, s, a, n, C, out);
}

// ---------------------------------------------------------------------------
// Segmentation filter.  The mask value of Gaussian g is its colour averaged
// over all view directions: only the l = 0 harmonic has a non-zero mean on
// the sphere, so the average is Y_0 c_g[0][channel], which is the colour
// itself at L = 0 (the paper's setting for masks).  keep = value >= threshold,
// taken in binary32, and not unobserved or failed when status is given.

namespace {
constexpr int kMaskBlock = 1024;  // Gaussians per block: 256 threads x 4 rounds
constexpr uint8_t kDropBits = 1 | 4;  // GSC_G_UNOBSERVED | GSC_G_FAILED

__device__ inline bool mask_keep(const float* coeffs, int64_t g, int64_t row, int channel, float thr,
                                 const uint8_t* status) {
    const float v = 0.28209479177387814f * coeffs[g * row + channel];
    bool k = v >= thr;
    if (status && (status[g] & kDropBits)) k = false;
    return k;
}
}  // namespace

// Kept Gaussians per block of kMaskBlock; also writes the keep bytes.
__global__ __launch_bounds__(256) void k_mask_count(const float* __restrict__ coeffs, int64_t N,
                                                    int64_t row, int channel, float thr,
                                                    const uint8_t* __restrict__ status,
                                                    uint8_t* __restrict__ keep,
                                                    uint32_t* __restrict__ block_counts) {
    __shared__ uint32_t wsum[4];
    const int64_t g0 = (int64_t)blockIdx.x * kMaskBlock;
    uint32_t mine = 0;
    for (int r = 0; r < 4; ++r) {
        const int64_t g = g0 + r * 256 + threadIdx.x;
        if (g < N) {
            const bool k = mask_keep(coeffs, g, row, channel, thr, status);
            if (keep) keep[g] = k ? 1 : 0;
            mine += k ? 1u : 0u;
        }
    }
    // wave sum, then the block's four waves
    for (int off = 32; off > 0; off >>= 1) mine += __shfl_xor(mine, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = mine;
    __syncthreads();
    if (threadIdx.x == 0) block_counts[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Exclusive scan of the block counts in place (one block of 1024 threads,
// chunk by chunk), and the total.
__global__ __launch_bounds__(1024) void k_mask_scan(uint32_t* __restrict__ counts, int n_blocks,
                                                    int64_t* __restrict__ n_kept) {
    __shared__ uint32_t wtot[16];
    __shared__ uint32_t carry_s;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int base = 0; base < n_blocks; base += 1024) {
        const int i = base + (int)threadIdx.x;
        const uint32_t v = i < n_blocks ? counts[i] : 0u;
        // inclusive scan within the wave
        uint32_t x = v;
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane == 63) wtot[wave] = x;
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wave; ++w) before += wtot[w];
        if (i < n_blocks) counts[i] = carry + before + x - v;
        if (threadIdx.x == 1023) carry_s = carry + before + x;
        __syncthreads();
        carry = carry_s;
        __syncthreads();
    }
    if (threadIdx.x == 0 && n_kept) *n_kept = (int64_t)carry;
}

// Indices of the kept Gaussians in increasing order.
__global__ __launch_bounds__(256) void k_mask_scatter(const float* __restrict__ coeffs, int64_t N,
                                                      int64_t row, int channel, float thr,
                                                      const uint8_t* __restrict__ status,
                                                      const uint32_t* __restrict__ block_offsets,
                                                      int64_t* __restrict__ indices) {
    __shared__ uint32_t wcnt[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t g0 = (int64_t)blockIdx.x * kMaskBlock;
    uint32_t base = block_offsets[blockIdx.x];
    for (int r = 0; r < 4; ++r) {
        const int64_t g = g0 + r * 256 + threadIdx.x;
        const bool k = g < N && mask_keep(coeffs, g, row, channel, thr, status);
        const uint64_t bal = __builtin_amdgcn_ballot_w64(k);
        if (lane == 0) wcnt[wave] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0;
        for (int w = 0; w < wave; ++w) before += wcnt[w];
        const uint64_t lt = lane ? (bal & (~0ull >> (64 - lane))) : 0ull;
        if (k) indices[base + before + (uint32_t)__popcll(lt)] = g;
        base += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
        __syncthreads();
    }
}

int mask_blocks(int64_t N) { return (int)((N + kMaskBlock - 1) / kMaskBlock); }

void launch_block_scan(uint32_t* counts, int n_blocks, int64_t* total, hipStream_t s) {
    hipLaunchKernelGGL(k_mask_scan, dim3(1), dim3(1024), 0, s, counts, n_blocks, total);
}

void launch_mask_filter(const float* coeffs, int64_t N, int64_t row, int channel, float thr,
                        const uint8_t* status, uint8_t* keep, int64_t* indices, int64_t* n_kept,
                        uint32_t* block_scratch, hipStream_t s) {
    const int nb = mask_blocks(N);
    if (nb == 0) {
        if (n_kept) hipLaunchKernelGGL(k_mask_scan, dim3(1), dim3(1024), 0, s, block_scratch, 0, n_kept);
        return;
    }
    hipLaunchKernelGGL(k_mask_count, dim3(nb), dim3(256), 0, s, coeffs, N, row, channel, thr, status,
                       keep, block_scratch);
    if (!indices && !n_kept) return;
    hipLaunchKernelGGL(k_mask_scan, dim3(1), dim3(1024), 0, s, block_scratch, nb, n_kept);
    if (indices)
        hipLaunchKernelGGL(k_mask_scatter, dim3(nb), dim3(256), 0, s, coeffs, N, row, channel, thr,
                           status, block_scratch, indices);
}

// bits[v][w] bit b = (V[v][64 w + b] > 0): which Gaussians view v observed.
__global__ __launch_bounds__(256) void k_seen_bits(const float* __restrict__ V, int n_views, int64_t N,
                                                   int64_t words, unsigned long long* __restrict__ bits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // one thread per bit
    const int64_t total = (int64_t)n_views * words * 64;
    if (i >= total) return;  // whole trailing waves only: words * 64 is a multiple of 64
    const int64_t v = i / (words * 64), g = i % (words * 64);
    const bool seen = g < N && V[v * N + g] > 0.0f;
    const uint64_t bal = __builtin_amdgcn_ballot_w64(seen);
    if ((threadIdx.x & 63) == 0) bits[v * words + g / 64] = bal;
}

void launch_seen_bits(const float* V, int n_views, int64_t N, unsigned long long* bits, hipStream_t s) {
    const int64_t words = (N + 63) / 64;
    const int64_t total = (int64_t)n_views * words * 64;
    if (total == 0) return;
    hipLaunchKernelGGL(k_seen_bits, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, V, n_views, N,
                       words, bits);
}

}  // namespace gsc
