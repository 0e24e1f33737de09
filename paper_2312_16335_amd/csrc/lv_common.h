// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "lv_error.h"

namespace lv {

#define LV_CHECK_HIP(expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      LV_FAIL(LV_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));           \
  } while (0)

// Launch status check (catches configuration errors at launch time).
#define LV_CHECK_LAUNCH()                                                           \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess)                                                           \
      LV_FAIL(LV_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e_));       \
  } while (0)

constexpr uint32_t kSentinel = LV_SENTINEL;

// Components per secondary row: D, or D - d for residual coordinates, or d
// for the second level of the primaries.
inline int32_t secondary_dims(const lv_index_desc &d) {
  return d.sec_dtype == LV_F16_RESID ? d.D - d.d : (d.sec_dtype == LV_LVQ8_LEVEL2 ? d.d : d.D);
}

}  // namespace lv

// The index handle: a validated copy of the descriptor plus derived launch
// choices.  Device pointers are borrowed.
struct lv_index {
  lv_index_desc desc;
  int32_t code_bytes;  // d * bits / 8
  int32_t group;       // lanes cooperating on one primary record
  int32_t vbytes;      // bytes each of those lanes loads
  int32_t sec_packets; // 16-byte packets per secondary row
  int32_t qp_width;    // projected query floats: d, or D with LV_F16_RESID (P q, then P_perp q)
};

namespace lv {
// Launchers implemented in lv_search.hip.
int launch_beam(const lv_index *ix, const float *Q, const float *Qp, int64_t m, int32_t k,
                int32_t L, uint32_t *ids, float *scores, uint32_t *counters,
                const lv_search_params *params, hipStream_t stream);
int launch_project(const float *V, int64_t rows, int32_t D, const uint16_t *M, int32_t d,
                   float *out, hipStream_t stream);
}  // namespace lv
