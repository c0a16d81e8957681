// Real orthonormal spherical harmonics up to degree 3 as polynomials of the
// unit direction (x, y, z); flat index l*l + l + m.  Normalisation
// K_l^m = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!), sqrt(2) on m != 0, no
// Condon-Shortley phase (eq. 3; the constant term is 1/sqrt(4 pi)).
#pragma once

#include <hip/hip_runtime.h>

namespace gsc {

template <typename T, int L>
__device__ __forceinline__ void sh_eval(T x, T y, T z, T* out) {
    out[0] = T(0.28209479177387814);
    if constexpr (L >= 1) {
        const T c1 = T(0.4886025119029199);
        out[1] = c1 * y;
        out[2] = c1 * z;
        out[3] = c1 * x;
    }
    if constexpr (L >= 2) {
        const T xx = x * x, yy = y * y, zz = z * z;
        out[4] = T(1.0925484305920792) * x * y;
        out[5] = T(1.0925484305920792) * y * z;
        out[6] = T(0.31539156525252005) * (T(3) * zz - T(1));
        out[7] = T(1.0925484305920792) * x * z;
        out[8] = T(0.5462742152960396) * (xx - yy);
        if constexpr (L >= 3) {
            out[9] = T(0.5900435899266435) * y * (T(3) * xx - yy);
            out[10] = T(2.890611442640554) * x * y * z;
            out[11] = T(0.4570457994644658) * y * (T(5) * zz - T(1));
            out[12] = T(0.3731763325901154) * z * (T(5) * zz - T(3));
            out[13] = T(0.4570457994644658) * x * (T(5) * zz - T(1));
            out[14] = T(1.445305721320277) * z * (xx - yy);
            out[15] = T(0.5900435899266435) * x * (xx - T(3) * yy);
        }
    }
}

}  // namespace gsc
