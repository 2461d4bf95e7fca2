// Grid-layout sweep kernels for double fields.
#include "gl_launch_impl.hpp"

namespace gl {
hipError_t launch_grid_sweep_f64(int K, const SweepLaunch& L, hipStream_t s) { return grid_sweep_typed<double>(K, L, s); }
}  // namespace gl
