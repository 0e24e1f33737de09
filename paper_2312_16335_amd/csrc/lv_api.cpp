// Index handles and the search entry points: host-side validation, then
// the device launches (query projection, then the per-query traversal).
#include <new>

#include "lv_common.h"
#include "lv_search.h"

namespace {

int validate_desc(const lv_index_desc *d, lv_index *ix) {
  if (!d) LV_FAIL(LV_EINVAL, "NULL descriptor");
  if (d->N < 1 || d->N >= 0x7FFFFFFF) LV_FAIL(LV_EINVAL, "N must be in [1, 2^31-2]");
  if (d->d < 8 || d->d % 8 != 0) LV_FAIL(LV_EINVAL, "d must be a positive multiple of 8");
  if (d->D < d->d) LV_FAIL(LV_EINVAL, "D must be >= d");
  if (d->bits != 4 && d->bits != 8) LV_FAIL(LV_EINVAL, "bits must be 4 or 8");
  if (d->sec_dtype != LV_F32 && d->sec_dtype != LV_F16 && d->sec_dtype != LV_LVQ8 &&
      d->sec_dtype != LV_F16_RESID && d->sec_dtype != LV_LVQ8_LEVEL2)
    LV_FAIL(LV_EINVAL, "bad sec_dtype");
  const bool resid = d->sec_dtype == LV_F16_RESID;
  if (resid && d->D <= d->d) LV_FAIL(LV_EINVAL, "LV_F16_RESID needs D > d");
  if (d->sec_dtype == LV_LVQ8 && !d->sec_mu) LV_FAIL(LV_EINVAL, "LV_LVQ8 secondaries need sec_mu");
  if (d->R < 1 || d->R > 1024) LV_FAIL(LV_EINVAL, "R must be in [1, 1024]");
  if ((uint64_t)d->entry >= (uint64_t)d->N) LV_FAIL(LV_EINVAL, "entry out of range");
  if (!d->records || !d->mu || !d->secondaries || !d->adjacency)
    LV_FAIL(LV_EINVAL, "NULL device pointer in descriptor");
  const int32_t cb = d->d * d->bits / 8;
  if (d->record_stride < cb + 8) LV_FAIL(LV_EINVAL, "record_stride smaller than codes + 8");
  int group = 0, vbytes = 0;
  switch (d->record_stride) {
    case 64: group = 16; vbytes = 4; break;
    case 96: group = 8; vbytes = 12; break;
    case 128: group = 16; vbytes = 8; break;
    case 192: group = 16; vbytes = 12; break;
    case 256: group = 16; vbytes = 16; break;
    case 512: group = 64; vbytes = 8; break;
    case 768: group = 64; vbytes = 12; break;
    case 1024: group = 64; vbytes = 16; break;
    default:
      LV_FAIL(LV_EUNSUPPORTED, "record_stride %d unsupported (use lv_record_stride)",
              d->record_stride);
  }
  const int64_t row_bytes = lv_secondary_row_bytes(lv::secondary_dims(*d), d->sec_dtype);
  if (row_bytes == 0)
    LV_FAIL(LV_EUNSUPPORTED, "secondary rows of D = %d and type %d are not supported", d->D,
            d->sec_dtype);
  if (d->A && d->D % 8 != 0) LV_FAIL(LV_EUNSUPPORTED, "query projection needs D % 8 == 0");
  ix->desc = *d;
  ix->code_bytes = cb;
  ix->group = group;
  ix->vbytes = vbytes;
  ix->sec_packets = (int32_t)(row_bytes / 16);
  ix->qp_width = resid ? d->D : d->d;
  return LV_OK;
}

int validate_query(const lv_index *ix, const float *Q, int64_t m, int32_t k, int32_t L,
                   uint32_t *ids, float *scores) {
  if (!ix) LV_FAIL(LV_EINVAL, "NULL index");
  if (m < 0) LV_FAIL(LV_EINVAL, "m must be >= 0");
  if (k < 1 || k > LV_MAX_K) LV_FAIL(LV_EINVAL, "k must be in [1, %d] (got %d)", LV_MAX_K, k);
  if (L < k) LV_FAIL(LV_EINVAL, "window L (%d) must be >= k (%d)", L, k);
  if (L > LV_MAX_L) LV_FAIL(LV_EINVAL, "window L must be <= %d", LV_MAX_L);
  if (m > 0 && (!Q || !ids || !scores)) LV_FAIL(LV_EINVAL, "NULL query or output pointer");
  return LV_OK;
}

}  // namespace

extern "C" int32_t lv_secondary_row_bytes(int32_t D, int32_t sec_dtype) {
  int64_t b = 0;
  if (D < 1) return 0;
  if (sec_dtype == LV_F32) b = 4 * (int64_t)D;
  else if (sec_dtype == LV_F16 || sec_dtype == LV_F16_RESID) b = 2 * (int64_t)D;
  else if (sec_dtype == LV_LVQ8) b = D % 16 == 0 && D <= 1008 ? (int64_t)D + 16 : 0;
  else if (sec_dtype == LV_LVQ8_LEVEL2) b = D <= 1008 ? ((int64_t)D + 15) / 16 * 16 + 16 : 0;
  if (b == 0 || b % 16 != 0 || b > 2048) return 0;
  return (int32_t)b;
}

extern "C" int lv_index_create(const lv_index_desc *desc, lv_index **out) {
  lv::clear_error();
  if (!out) LV_FAIL(LV_EINVAL, "NULL out");
  *out = nullptr;
  lv_index tmp;
  const int rc = validate_desc(desc, &tmp);
  if (rc != LV_OK) return rc;
  lv_index *ix = new (std::nothrow) lv_index(tmp);
  if (!ix) LV_FAIL(LV_ENOMEM, "out of host memory");
  *out = ix;
  return LV_OK;
}

extern "C" int lv_index_destroy(lv_index *index) {
  lv::clear_error();
  delete index;
  return LV_OK;
}

extern "C" size_t lv_search_workspace_size(const lv_index *index, int64_t m) {
  if (!index || m < 0) return 0;
  const size_t b = (size_t)m * (size_t)index->qp_width * sizeof(float);
  return (b + 255) & ~(size_t)255;
}

extern "C" int lv_search(const lv_index *index, const float *Q, int64_t m, int32_t k, int32_t L,
                         uint32_t *ids, float *scores, uint32_t *counters, void *ws,
                         size_t ws_bytes, const lv_search_params *params, void *stream) {
  lv::clear_error();
  int rc = validate_query(index, Q, m, k, L, ids, scores);
  if (rc != LV_OK) return rc;
  if (!index->desc.A) LV_FAIL(LV_EINVAL, "index has no query projection A");
  if (m == 0) return LV_OK;
  const size_t need = lv_search_workspace_size(index, m);
  if (!ws || ws_bytes < need)
    LV_FAIL(LV_EINVAL, "workspace of %zu bytes needed (got %zu)", need, ws_bytes);
  lv::VisitedCfg vc;  // search options are checked before anything is launched
  rc = lv::visited_config(params, &vc);
  if (rc != LV_OK) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float *Qp = static_cast<float *>(ws);
  rc = lv::launch_project(Q, m, index->desc.D, index->desc.A, index->qp_width, Qp, s);
  if (rc != LV_OK) return rc;
  return lv::launch_beam(index, Q, Qp, m, k, L, ids, scores, counters, params, s);
}

extern "C" int lv_search_projected(const lv_index *index, const float *Q, const float *Qp,
                                   int64_t m, int32_t k, int32_t L, uint32_t *ids, float *scores,
                                   uint32_t *counters, const lv_search_params *params,
                                   void *stream) {
  lv::clear_error();
  int rc = validate_query(index, Q, m, k, L, ids, scores);
  if (rc != LV_OK) return rc;
  if (m > 0 && !Qp) LV_FAIL(LV_EINVAL, "NULL projected queries");
  if (m == 0) return LV_OK;
  return lv::launch_beam(index, Q, Qp, m, k, L, ids, scores, counters, params,
                         static_cast<hipStream_t>(stream));
}
