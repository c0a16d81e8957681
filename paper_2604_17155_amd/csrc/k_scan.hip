// Input scans (non-finite values, largest magnitude) and the conversion of
// the deterministic fixed-point per-view sums back to binary32.
#include <algorithm>

#include "gsc_internal.h"

namespace gsc {

template <int DT>
__device__ __forceinline__ float load_value(const void* p, int64_t i) {
    if constexpr (DT == GSC_BF16) {
        const uint16_t b = reinterpret_cast<const uint16_t*>(p)[i];
        return __uint_as_float((uint32_t)b << 16);
    } else {
        return reinterpret_cast<const float*>(p)[i];
    }
}

template <int DT>
__global__ __launch_bounds__(256) void k_scan_values(const void* __restrict__ p, int64_t n,
                                                     unsigned long long* __restrict__ first_bad,
                                                     uint32_t* __restrict__ absmax) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long bad = ~0ull;
    uint32_t mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        // |x| as bits: finite values order as their magnitudes, then +inf,
        // then NaN patterns
        const uint32_t a = __float_as_uint(load_value<DT>(p, i)) & 0x7fffffffu;
        mx = std::max(mx, a);
        if (a >= 0x7f800000u) bad = std::min(bad, (unsigned long long)i);
    }
    for (int off = 32; off > 0; off >>= 1) {
        mx = std::max(mx, (uint32_t)__shfl_xor((int)mx, off, 64));
        const unsigned long long o = __shfl_xor(bad, off, 64);
        bad = std::min(bad, o);
    }
    if ((threadIdx.x & 63) == 0) {
        if (mx) atomicMax(absmax, mx);
        if (bad != ~0ull) atomicMin(first_bad, bad);
    }
}

void launch_scan_values(const void* p, int dtype, int64_t n, unsigned long long* first_bad,
                        uint32_t* absmax, hipStream_t s) {
    if (n <= 0) return;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 256 * 8);
    if (dtype == GSC_BF16)
        hipLaunchKernelGGL(k_scan_values<GSC_BF16>, dim3(blocks), dim3(256), 0, s, p, n, first_bad, absmax);
    else
        hipLaunchKernelGGL(k_scan_values<GSC_F32>, dim3(blocks), dim3(256), 0, s, p, n, first_bad, absmax);
}

__global__ __launch_bounds__(256) void k_det_to_float(const unsigned long long* __restrict__ in, int64_t n,
                                                      int stride, double inv_v, double inv_s,
                                                      float* __restrict__ out) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const double v = (double)(long long)in[i];
        out[i] = (float)(v * (i % stride == 0 ? inv_v : inv_s));
    }
}

void launch_det_to_float(const unsigned long long* in, int64_t n, int stride, double inv_v,
                         double inv_s, float* out, hipStream_t s) {
    if (n <= 0) return;
    const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 256 * 16);
    hipLaunchKernelGGL(k_det_to_float, dim3(blocks), dim3(256), 0, s, in, n, stride, inv_v, inv_s, out);
}

}  // namespace gsc
