// Shading kernels (placeholder until the fused kernels land).
#include <hip/hip_runtime.h>

#include "svlf_internal.hpp"

namespace svlf {

int shade_grid_limit() { return 1024; }

hipError_t launch_shade(const ShadeArgs&, int, hipStream_t, int* grid_used) {
  *grid_used = 0;
  return hipErrorNotSupported;
}

hipError_t launch_mlp_forward(const float*, int, int, int, int, const float*, int64_t, float*,
                              hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace svlf
