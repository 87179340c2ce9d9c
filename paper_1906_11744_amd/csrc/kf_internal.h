// Internal launch interface between the C ABI (kf_api.hip) and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kf_device.h"

namespace kfi {

// Everything a fit launch needs, by value.
struct FitArgs {
  int64_t n;
  int32_t nl;
  int32_t seed_from_hits;
  kfd::Model md;
  float srphi, sz;
  const float* hits;
  const uint32_t* mask;
  const float* seed_state;
  const float* seed_cov;
  const kfd::LayerK* layers;  // [nl], prepared on the device
  float* state;
  float* cov;
  float* chi2;
  int32_t* ndf;
  uint32_t* status;
  float* ckpt;
};

// Writes the per-layer constants (radius, alignment, its cos/sin, material).
hipError_t launch_layer_prep(int nl, const float* radius_host, const float* align, const float* xX0,
                             kfd::LayerK* out, hipStream_t stream);
hipError_t launch_fit(const FitArgs& a, hipStream_t stream);

}  // namespace kfi
