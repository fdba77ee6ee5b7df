// Adjoint of blending and of the projection (placeholder until implemented).
#include "gs_internal.h"

namespace gs {

hipError_t launch_blend_bwd(const BlendParams &, int64_t, const float *, const float *, const float *,
                            const uint32_t *, const uint32_t *, const float *, const uint32_t *, const float *,
                            float *, float *, float *, hipStream_t) {
  return hipErrorNotSupported;
}

hipError_t launch_preprocess_bwd(const PreParams &, int64_t, const float *, const float *, const float *,
                                 const float *, const float *, const uint32_t *, const float *, const float *,
                                 const float *, float *, float *, float *, float *, float *, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace gs
