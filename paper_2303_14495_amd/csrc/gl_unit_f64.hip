// Sweep and Laplacian kernels for double fields (double weights only).
#include "gl_launch_impl.hpp"

namespace gl {
hipError_t launch_sweep_f64(int K, const SweepLaunch& L, hipStream_t s) {
    if (L.r.wdt != GL_F64) return hipErrorInvalidValue;
    return L.r.idx64 ? sweep_k<double, double, int64_t>(K, L, s) : sweep_k<double, double, int32_t>(K, L, s);
}
hipError_t launch_laplacian_f64(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s) {
    if (r.wdt != GL_F64) return hipErrorInvalidValue;
    return r.idx64 ? laplacian_k<double, double, int64_t>(K, r, x, y, s)
                   : laplacian_k<double, double, int32_t>(K, r, x, y, s);
}
}  // namespace gl
