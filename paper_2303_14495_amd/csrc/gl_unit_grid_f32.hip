// Grid-layout sweep kernels for float fields.
#include "gl_launch_impl.hpp"

namespace gl {
hipError_t launch_grid_sweep_f32(int K, const SweepLaunch& L, hipStream_t s) { return grid_sweep_typed<float>(K, L, s); }
}  // namespace gl
