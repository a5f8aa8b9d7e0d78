// Backward DRK raster: placeholder until the hand-written backward lands.
#include "raster_common.hpp"

namespace drk {
hipError_t launch_render_bwd(int, const float*, const uint32_t*, const uint32_t*, const CamDev&, const OptsDev&,
                             const float*, const float*, const int32_t*, float*, int64_t, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_preprocess_bwd(const SceneDev&, const Views&, const OptsDev&, const uint32_t*, const float*, int64_t,
                                 const drk_scene_grad&, hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace drk
