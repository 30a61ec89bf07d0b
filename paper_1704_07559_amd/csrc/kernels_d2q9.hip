// D2Q9 kernels (placeholder launchers until the D2Q9 path lands).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace lbm {
namespace d2q9 {
hipError_t launch_init(int, const Geo&, const ModelF&, void*, float*, const float*, const float*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_step(int, const Geo&, const ModelF&, const ViscF&, const ForceF&, const StepIO&, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_strain(int, const Geo&, const ModelF&, const ForceF&, const void*, const float*, int, float*,
                         hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t launch_get(int, const Geo&, const void*, float*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_set(int, const Geo&, void*, const float*, hipStream_t) { return hipErrorNotSupported; }
hipError_t launch_reduce(int, const Geo&, const ModelF&, const ForceF&, const void*, const float*, double*, double*,
                         hipStream_t) {
  return hipErrorNotSupported;
}
}  // namespace d2q9
}  // namespace lbm
