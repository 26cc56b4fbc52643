// Collide-and-stream launches of the D3Q27 lattice in float.
#include "step_kernel.h"

namespace mclbm {

hipError_t launch_step_d3q27_f32(StepKind kind, const StepLaunch& L, hipStream_t s) {
  return launch_step_k<27, float>(kind, L, s);
}

}  // namespace mclbm
