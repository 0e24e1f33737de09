// lv_search for callers that cannot allocate device memory (code under
// graph capture, serving loops, harnesses that forbid allocation): the
// projected queries, which lv_search keeps in a caller workspace, live in a
// fixed device array of this library instead.
//
// The array is a file-scope __device__ variable; host code never passes its
// name to a kernel (in host code the name is a host-side stand-in).  Its
// device address is taken once per device with hipGetSymbolAddress, on the
// entry point's first call on that device with the device current, and that
// address is what the launches receive.  Every call on a device shares the
// device's array: calls that overlap on one device race, and the array holds
// the last call's projected queries afterwards (every call overwrites what
// it reads, so nothing needs clearing).
#include <mutex>

#include "lv_common.h"
#include "lv_search.h"

namespace lv {
namespace {

constexpr size_t kScratchBytes = LV_NOALLOC_SCRATCH_BYTES;  // projected queries
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device).
int scratch_address(void **out) {
  int dev = 0;
  LV_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) LV_FAIL(LV_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    LV_CHECK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) LV_FAIL(LV_EDEVICE, "no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LV_OK;
}

}  // namespace
}  // namespace lv

extern "C" int lv_search_noalloc(const lv_index *index, const float *Q, int64_t m, int32_t k,
                                 int32_t L, uint32_t *ids, float *scores, uint32_t *counters,
                                 const lv_search_params *params, void *stream) {
  lv::clear_error();
  if (!index) LV_FAIL(LV_EINVAL, "NULL index");
  if (m < 0) LV_FAIL(LV_EINVAL, "m must be >= 0");
  if (k < 1 || k > LV_MAX_K) LV_FAIL(LV_EINVAL, "k must be in [1, %d] (got %d)", LV_MAX_K, k);
  if (L < k) LV_FAIL(LV_EINVAL, "window L (%d) must be >= k (%d)", L, k);
  if (L > LV_MAX_L) LV_FAIL(LV_EINVAL, "window L must be <= %d", LV_MAX_L);
  if (m > 0 && (!Q || !ids || !scores)) LV_FAIL(LV_EINVAL, "NULL query or output pointer");
  if (!index->desc.A) LV_FAIL(LV_EINVAL, "index has no query projection A");
  const size_t need = lv_search_workspace_size(index, m);
  if (need > lv::kScratchBytes)
    LV_FAIL(LV_EINVAL, "%lld queries need %zu bytes of projected queries; at most %zu (%lld "
            "queries of %d floats)", (long long)m, need, lv::kScratchBytes,
            (long long)(lv::kScratchBytes / (sizeof(float) * index->qp_width)), index->qp_width);
  lv::VisitedCfg vc;  // search options are checked before anything is launched
  int rc = lv::visited_config(params, &vc);
  if (rc != LV_OK) return rc;
  if (m == 0) return LV_OK;
  void *qp = nullptr;
  rc = lv::scratch_address(&qp);
  if (rc != LV_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *Qp = static_cast<float *>(qp);
  rc = lv::launch_project(Q, m, index->desc.D, index->desc.A, index->qp_width, Qp, s);
  if (rc != LV_OK) return rc;
  return lv::launch_beam(index, Q, Qp, m, k, L, ids, scores, counters, params, s);
}
