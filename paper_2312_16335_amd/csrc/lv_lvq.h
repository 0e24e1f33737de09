// The LVQ code of one component, shared by the encoders (files compiled
// without floating-point contraction, so the bytes are exact).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lv {

// clamp(floor((r - lo) / delta + 0.5), 0, levels) in IEEE float64; 0 when
// delta = 0.
__device__ __forceinline__ uint32_t lvq_code(double r, double lo, double delta, double levels) {
  if (delta == 0.0) return 0u;
  double c = floor((r - lo) / delta + 0.5);
  c = c < 0.0 ? 0.0 : (c > levels ? levels : c);
  return (uint32_t)c;
}

}  // namespace lv
