// Collide-and-stream launches of the D3Q19 lattice in float.
#include "step_kernel.h"

namespace mclbm {

hipError_t launch_step_d3q19_f32(StepKind kind, const StepLaunch& L, hipStream_t s) {
  return launch_step_k<19, float>(kind, L, s);
}

}  // namespace mclbm
