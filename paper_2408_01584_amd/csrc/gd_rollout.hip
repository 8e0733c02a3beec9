// Differentiable rollout kernels (forward with checkpoints, backward by recomputation).
#include "gd_internal.h"

namespace gdk {

hipError_t launch_rollout_fwd_impl(const SimArgs &, const float2 *, int, int, float *, float *,
                                   hipStream_t) {
    return hipErrorNotSupported;
}

hipError_t launch_rollout_bwd_impl(const SimArgs &, const float2 *, const float *, int, int,
                                   const float *, float2 *, float *, hipStream_t) {
    return hipErrorNotSupported;
}

}  // namespace gdk
