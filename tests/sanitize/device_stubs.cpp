// Stand-ins for the device-side entry points of libnlse (the kernel launch
// wrappers in the .hip sources), so the library's host code can be built for
// the host alone under the sanitizers (test infrastructure).  Every launch
// reports hipErrorNotSupported; the host driver never reaches one.
#include <hip/hip_runtime.h>

#include "nlse_batch.h"
#include "nlse_internal.h"
#include "nlse_surrogate.h"

hipError_t nlse_launch_stage_1d(const nlse::StageLaunch&, hipStream_t) { return hipErrorNotSupported; }
hipError_t nlse_launch_stage_2d(const nlse::StageLaunch&, hipStream_t) { return hipErrorNotSupported; }
hipError_t nlse_launch_stage_3d(const nlse::StageLaunch&, hipStream_t) { return hipErrorNotSupported; }
hipError_t nlse_launch_fused3d(const nlse::StageLaunch&, const void*, void*, void*, void*, void*, double,
                               hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t nlse_launch_pair2d(const nlse::StageLaunch&, const void*, void*, void*, void*, void*, double, int,
                              hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t nlse_launch_fused3d_pair0(const nlse::StageLaunch&, const void*, void*, void*, double, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t nlse_launch_reduce(const nlse::ReduceLaunch&, hipStream_t) { return hipErrorNotSupported; }
hipError_t nlse_launch_resident1d(const nlse::StageLaunch&, int64_t, double, hipStream_t) {
  return hipErrorNotSupported;
}
int64_t nlse_resident1d_max_points(int) { return 0; }
hipError_t nlse_launch_fill_zero(void*, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t nlse_launch_copy(void*, const void*, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t nlse_static_reduce_scratch(double**, double**) { return hipErrorNotSupported; }
hipError_t nlse_launch_batch(const nlse::BatchLaunch&, hipStream_t) { return hipErrorNotSupported; }
hipError_t nlse_batch_occupancy(int, int, int, int, int, int*) { return hipErrorNotSupported; }
hipError_t sg_pack_input(const void*, void*, int64_t, hipStream_t) { return hipErrorNotSupported; }
hipError_t sg_conv(int, const SgConv&, hipStream_t) { return hipErrorNotSupported; }
hipError_t sg_net_forward(const SgNet&, hipStream_t) { return hipErrorNotSupported; }
hipError_t sg_loss(const void*, const void*, uint16_t*, double*, int, int64_t, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t sg_wgrad(int, const uint16_t*, const uint16_t*, float*, int, int, int, int, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t sg_wgrad_reduce(const float*, int, int, int, int, int, float*, float*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t sg_prep_weights(const float*, int, int, int, int, uint16_t*, uint16_t*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t sg_adam(float*, const float*, float*, float*, int, float, float, float, float, float, float, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t sg_field_mass(const void*, int, int64_t, double, double*, int, double*, hipStream_t) {
  return hipErrorNotSupported;
}
hipError_t sg_msd_project(const void*, void*, int, int, int, hipStream_t) { return hipErrorNotSupported; }
hipError_t sg_tile_mass_final(const double*, int, int, double, double*, hipStream_t) { return hipErrorNotSupported; }
