// Sweep and Laplacian kernels for float fields (weights float, bf16 or f16).
#include "gl_launch_impl.hpp"

namespace gl {
hipError_t launch_sweep_f32(int K, const SweepLaunch& L, hipStream_t s) { return sweep_lowp<float>(K, L, s); }
hipError_t launch_laplacian_f32(int K, const RowLaunch& r, const void* x, void* y, hipStream_t s) {
    return laplacian_lowp<float>(K, r, x, y, s);
}
}  // namespace gl
