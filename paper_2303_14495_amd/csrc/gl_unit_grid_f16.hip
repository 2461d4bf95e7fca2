// Grid-layout sweep kernels for f16 fields.
#include "gl_launch_impl.hpp"

namespace gl {
hipError_t launch_grid_sweep_f16(int K, const SweepLaunch& L, hipStream_t s) { return grid_sweep_typed<f16>(K, L, s); }
}  // namespace gl
