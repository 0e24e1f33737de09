// Batched search: several sub-indexes, uneven requests, one persistent
// launch per step, captured as hipGraphs; plus the autotuner.
//
// A step is two graph launches on the caller's stream: pre[i] (copy of the
// pinned request table i, grouped query projection) and trav[i] (counter
// reset if persistent, then the search kernel).  The split lets a caller
// bracket the search alone with its own timing events.
//
// Steps rotate through kSets sets of device state (request table, work
// counter, projected queries), so up to kSets consecutive steps may run at
// once when the caller issues them on different streams: later steps'
// wavefronts then fill the compute units that the slowest queries of earlier
// steps leave idle.  A set is reused kSets steps later, after the step that
// last used it has finished (its stream is made to wait for that); with a
// number of streams that divides kSets that step ran on the same stream, so
// the wait costs nothing.
#include <algorithm>
#include <new>
#include <vector>

#include "lv_common.h"
#include "lv_search.h"

struct lv_multi {
  std::vector<const lv_index *> subs;
  lv::IndexView *d_views = nullptr;  // device copy of the views
  int bits = 0, group = 0, vbytes = 0, D = 0, d = 0;
  int pw = 0;  // projected query width: d, or D with residual secondaries
};

constexpr int kSets = 4;

struct lv_batch {
  lv_multi *multi = nullptr;
  lv_batch_caps caps{};
  lv::VisitedCfg vc{};
  int launch = LV_LAUNCH_PER_QUERY;
  int grid = 0;
  int max_tiles = 0;
  size_t table_bytes = 0;
  // per step parity
  unsigned char *d_table[kSets] = {};  // StepHeader + Request[max_requests]
  unsigned char *h_table[kSets] = {};  // pinned
  unsigned int *d_counter[kSets] = {};
  float *d_qp[kSets] = {};
  hipGraph_t pre_graph[kSets] = {};
  hipGraphExec_t pre_exec[kSets] = {};
  hipGraph_t trav_graph[kSets] = {};
  hipGraphExec_t trav_exec[kSets] = {};
  hipEvent_t copied[kSets] = {};  // pinned table i consumed
  hipEvent_t done[kSets] = {};    // step on set i finished
  bool used[kSets] = {};
  hipStream_t capture = nullptr;
  int next = 0;
};

namespace {

void free_batch(lv_batch *b) {
  if (!b) return;
  for (int i = 0; i < kSets; ++i) {
    if (b->done[i]) {
      (void)hipEventSynchronize(b->done[i]);
      (void)hipEventDestroy(b->done[i]);
    }
    if (b->copied[i]) {
      (void)hipEventSynchronize(b->copied[i]);
      (void)hipEventDestroy(b->copied[i]);
    }
    if (b->pre_exec[i]) (void)hipGraphExecDestroy(b->pre_exec[i]);
    if (b->pre_graph[i]) (void)hipGraphDestroy(b->pre_graph[i]);
    if (b->trav_exec[i]) (void)hipGraphExecDestroy(b->trav_exec[i]);
    if (b->trav_graph[i]) (void)hipGraphDestroy(b->trav_graph[i]);
    if (b->h_table[i]) (void)hipHostFree(b->h_table[i]);
    if (b->d_table[i]) (void)hipFree(b->d_table[i]);
    if (b->d_counter[i]) (void)hipFree(b->d_counter[i]);
    if (b->d_qp[i]) (void)hipFree(b->d_qp[i]);
  }
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

}  // namespace

extern "C" int lv_multi_create(const lv_index *const *subs, int32_t count, lv_multi **out) {
  lv::clear_error();
  if (!out) LV_FAIL(LV_EINVAL, "NULL out");
  *out = nullptr;
  if (!subs || count < 1) LV_FAIL(LV_EINVAL, "need at least one sub-index");
  for (int i = 0; i < count; ++i)
    if (!subs[i]) LV_FAIL(LV_EINVAL, "sub-index %d is NULL", i);
  const lv_index *s0 = subs[0];
  for (int i = 0; i < count; ++i) {
    const lv_index *s = subs[i];
    if (s->desc.D != s0->desc.D || s->desc.d != s0->desc.d || s->desc.bits != s0->desc.bits ||
        s->desc.record_stride != s0->desc.record_stride ||
        s->desc.sec_dtype != s0->desc.sec_dtype)
      LV_FAIL(LV_EINVAL, "sub-index %d differs in D, d, bits, stride or secondary type", i);
    if (!s->desc.A) LV_FAIL(LV_EINVAL, "sub-index %d has no query projection A", i);
  }
  if (s0->desc.d > 256) LV_FAIL(LV_EUNSUPPORTED, "batched search needs d <= 256");
  lv_multi *m = new (std::nothrow) lv_multi();
  if (!m) LV_FAIL(LV_ENOMEM, "out of host memory");
  m->subs.assign(subs, subs + count);
  m->bits = s0->desc.bits;
  m->group = s0->group;
  m->vbytes = s0->vbytes;
  m->D = s0->desc.D;
  m->d = s0->desc.d;
  m->pw = s0->qp_width;
  std::vector<lv::IndexView> views(count);
  for (int i = 0; i < count; ++i) views[i] = lv::make_view(subs[i]);
  if (hipMalloc(&m->d_views, sizeof(lv::IndexView) * count) != hipSuccess) {
    delete m;
    LV_FAIL(LV_ENOMEM, "device allocation of the sub-index table failed");
  }
  if (hipMemcpy(m->d_views, views.data(), sizeof(lv::IndexView) * count,
                hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(m->d_views);
    delete m;
    LV_FAIL(LV_EDEVICE, "copy of the sub-index table failed");
  }
  *out = m;
  return LV_OK;
}

extern "C" int lv_multi_destroy(lv_multi *multi) {
  lv::clear_error();
  if (multi) {
    if (multi->d_views) (void)hipFree(multi->d_views);
    delete multi;
  }
  return LV_OK;
}

#define LV_BATCH_TRY(expr)                                                              \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) {                                                             \
      lv::set_error("%s failed: %s", #expr, hipGetErrorString(e_));                     \
      free_batch(b);                                                                    \
      return e_ == hipErrorOutOfMemory ? LV_ENOMEM : LV_EDEVICE;                         \
    }                                                                                   \
  } while (0)

extern "C" int lv_batch_create(lv_multi *multi, const lv_batch_caps *caps,
                               const lv_search_params *params, lv_batch **out) {
  lv::clear_error();
  if (!out) LV_FAIL(LV_EINVAL, "NULL out");
  *out = nullptr;
  if (!multi || !caps) LV_FAIL(LV_EINVAL, "NULL multi or caps");
  if (caps->max_requests < 1 || caps->max_queries < 1 || caps->max_queries > 0x7FFFFFFF)
    LV_FAIL(LV_EINVAL, "bad capacities");
  if (caps->max_L < 1 || caps->max_L > LV_MAX_L) LV_FAIL(LV_EINVAL, "max_L must be in [1, %d]", LV_MAX_L);
  lv::VisitedCfg vc{};
  int rc = lv::visited_config(params, &vc);
  if (rc != LV_OK) return rc;
  const int launch = params ? params->launch : LV_LAUNCH_PER_QUERY;
  if (launch != LV_LAUNCH_PER_QUERY && launch != LV_LAUNCH_PERSISTENT)
    LV_FAIL(LV_EINVAL, "launch must be LV_LAUNCH_PER_QUERY or LV_LAUNCH_PERSISTENT");
  int blocks = 0;
  rc = lv::batched_occupancy(multi->bits, multi->group, multi->vbytes, caps->max_L, vc,
                                &blocks);
  if (rc != LV_OK) return rc;
  if (blocks < 1) LV_FAIL(LV_EUNSUPPORTED, "the persistent kernel does not fit on a compute unit");
  int dev = 0, cus = 0;
  LV_CHECK_HIP(hipGetDevice(&dev));
  LV_CHECK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));

  lv_batch *b = new (std::nothrow) lv_batch();
  if (!b) LV_FAIL(LV_ENOMEM, "out of host memory");
  b->multi = multi;
  b->caps = *caps;
  b->vc = vc;
  b->launch = launch;
  b->grid = blocks * cus;
  b->max_tiles = (int)((caps->max_queries + 31) / 32) + caps->max_requests;
  b->table_bytes = sizeof(lv::StepHeader) + sizeof(lv::Request) * (size_t)caps->max_requests;
  for (int i = 0; i < kSets; ++i) {
    LV_BATCH_TRY(hipMalloc(&b->d_table[i], b->table_bytes));
    LV_BATCH_TRY(hipMalloc(&b->d_counter[i], sizeof(unsigned int)));
    LV_BATCH_TRY(hipMalloc(&b->d_qp[i], sizeof(float) * (size_t)caps->max_queries * multi->pw));
    LV_BATCH_TRY(hipHostMalloc(reinterpret_cast<void **>(&b->h_table[i]), b->table_bytes,
                               hipHostMallocDefault));
    std::fill(b->h_table[i], b->h_table[i] + b->table_bytes, (unsigned char)0);
    LV_BATCH_TRY(hipEventCreateWithFlags(&b->copied[i], hipEventDisableTiming));
    LV_BATCH_TRY(hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming));
  }
  LV_BATCH_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
  for (int i = 0; i < kSets; ++i) {
    const lv::StepHeader *hdr = reinterpret_cast<const lv::StepHeader *>(b->d_table[i]);
    LV_BATCH_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed));
    hipError_t e1 = hipMemcpyAsync(b->d_table[i], b->h_table[i], b->table_bytes,
                                   hipMemcpyHostToDevice, b->capture);
    int r1 = e1 == hipSuccess
                 ? lv::launch_project_grouped(hdr, multi->d_views, b->max_tiles, multi->pw,
                                              multi->D, b->capture)
                 : LV_EDEVICE;
    hipError_t e2 = hipStreamEndCapture(b->capture, &b->pre_graph[i]);
    if (e1 != hipSuccess || r1 != LV_OK || e2 != hipSuccess) {
      if (r1 == LV_OK) lv::set_error("graph capture failed");
      free_batch(b);
      return r1 != LV_OK ? r1 : LV_EDEVICE;
    }
    LV_BATCH_TRY(hipGraphInstantiate(&b->pre_exec[i], b->pre_graph[i], nullptr, nullptr, 0));
    LV_BATCH_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed));
    // per query: one workgroup per query slot of the step (slots past the
    // step's queries exit at once); persistent: resident wavefronts and a counter
    const bool pq = launch == LV_LAUNCH_PER_QUERY;
    int r2 = lv::launch_batched(multi->bits, multi->group, multi->vbytes, hdr, multi->d_views,
                                   pq ? nullptr : b->d_counter[i], caps->max_L, vc,
                                   pq ? (int)caps->max_queries : b->grid, b->capture);
    hipError_t e3 = hipStreamEndCapture(b->capture, &b->trav_graph[i]);
    if (r2 != LV_OK || e3 != hipSuccess) {
      if (r2 == LV_OK) lv::set_error("graph capture failed");
      free_batch(b);
      return r2 != LV_OK ? r2 : LV_EDEVICE;
    }
    LV_BATCH_TRY(hipGraphInstantiate(&b->trav_exec[i], b->trav_graph[i], nullptr, nullptr, 0));
  }
  *out = b;
  return LV_OK;
}

extern "C" int lv_batch_destroy(lv_batch *batch) {
  lv::clear_error();
  free_batch(batch);
  return LV_OK;
}

namespace {

int batch_step(lv_batch *b, const lv_request *reqs, int32_t nreq, const float *Q, uint32_t *ids,
               float *scores, uint32_t *counters, hipEvent_t ev_begin, hipEvent_t ev_end,
               hipStream_t s) {
  if (!b) LV_FAIL(LV_EINVAL, "NULL batch");
  if (!reqs || nreq < 1 || nreq > b->caps.max_requests)
    LV_FAIL(LV_EINVAL, "nreq must be in [1, %d]", b->caps.max_requests);
  if (!Q || !ids || !scores) LV_FAIL(LV_EINVAL, "NULL query or output pointer");
  const int nsub = (int)b->multi->subs.size();
  int64_t nq = 0, nout = 0;
  int tiles = 0;
  for (int i = 0; i < nreq; ++i) {
    const lv_request &r = reqs[i];
    if (r.sub < 0 || r.sub >= nsub) LV_FAIL(LV_EINVAL, "request %d: bad sub-index %d", i, r.sub);
    if (r.k < 1 || r.k > LV_MAX_K) LV_FAIL(LV_EINVAL, "request %d: bad k %d", i, r.k);
    if (r.L < r.k || r.L > b->caps.max_L)
      LV_FAIL(LV_EINVAL, "request %d: L %d outside [k, max_L=%d]", i, r.L, b->caps.max_L);
    if (r.count < 1) LV_FAIL(LV_EINVAL, "request %d: count must be >= 1", i);
    nq += r.count;
    if (nq > b->caps.max_queries)
      LV_FAIL(LV_EINVAL, "step has more than max_queries=%lld queries",
              (long long)b->caps.max_queries);
    nout += (int64_t)r.count * r.k;
    tiles += (r.count + 31) / 32;
  }
  const int i = b->next;
  // the pinned table is rewritten once the copy of the step that last used
  // it has been done
  LV_CHECK_HIP(hipEventSynchronize(b->copied[i]));
  lv::StepHeader *hdr = reinterpret_cast<lv::StepHeader *>(b->h_table[i]);
  lv::Request *rq = reinterpret_cast<lv::Request *>(hdr + 1);
  hdr->Q = Q;
  hdr->Qp = b->d_qp[i];
  hdr->ids = ids;
  hdr->scores = scores;
  hdr->counters = counters;
  hdr->nq = nq;
  hdr->qp_stride = b->multi->pw;
  hdr->nreq = nreq;
  hdr->ntiles = tiles;
  int64_t qb = 0, ob = 0;
  int t0 = 0;
  for (int r = 0; r < nreq; ++r) {
    rq[r].sub = reqs[r].sub;
    rq[r].k = reqs[r].k;
    rq[r].L = reqs[r].L;
    rq[r].tile0 = t0;
    rq[r].q_begin = qb;
    rq[r].q_end = qb + reqs[r].count;
    rq[r].out_off = ob;
    qb += reqs[r].count;
    ob += (int64_t)reqs[r].count * reqs[r].k;
    t0 += (reqs[r].count + 31) / 32;
  }
  (void)nout;
  // device set i is free once the step that last used it has finished, on
  // whatever stream that step ran
  if (b->used[i]) LV_CHECK_HIP(hipStreamWaitEvent(s, b->done[i], 0));
  LV_CHECK_HIP(hipGraphLaunch(b->pre_exec[i], s));
  LV_CHECK_HIP(hipEventRecord(b->copied[i], s));
  if (ev_begin) LV_CHECK_HIP(hipEventRecord(ev_begin, s));
  LV_CHECK_HIP(hipGraphLaunch(b->trav_exec[i], s));
  if (ev_end) LV_CHECK_HIP(hipEventRecord(ev_end, s));
  LV_CHECK_HIP(hipEventRecord(b->done[i], s));
  b->used[i] = true;
  b->next = (b->next + 1) % kSets;
  return LV_OK;
}

}  // namespace

extern "C" int lv_batch_step(lv_batch *b, const lv_request *reqs, int32_t nreq, const float *Q,
                             uint32_t *ids, float *scores, uint32_t *counters, void *stream) {
  lv::clear_error();
  return batch_step(b, reqs, nreq, Q, ids, scores, counters, nullptr, nullptr,
                    static_cast<hipStream_t>(stream));
}

extern "C" int lv_batch_step_timed(lv_batch *b, const lv_request *reqs, int32_t nreq,
                                   const float *Q, uint32_t *ids, float *scores,
                                   uint32_t *counters, void *ev_begin, void *ev_end,
                                   void *stream) {
  lv::clear_error();
  if (!ev_begin || !ev_end) LV_FAIL(LV_EINVAL, "NULL timing event");
  return batch_step(b, reqs, nreq, Q, ids, scores, counters, static_cast<hipEvent_t>(ev_begin),
                    static_cast<hipEvent_t>(ev_end), static_cast<hipStream_t>(stream));
}

namespace {

double recall_host(const std::vector<uint32_t> &got, int k, const uint32_t *truth, int truth_k,
                   int64_t m) {
  int64_t hit = 0;
  for (int64_t q = 0; q < m; ++q)
    for (int a = 0; a < k; ++a) {
      const uint32_t id = got[(size_t)q * k + a];
      if (id == LV_SENTINEL) continue;
      for (int t = 0; t < k; ++t)
        if (truth[(size_t)q * truth_k + t] == id) {
          ++hit;
          break;
        }
    }
  return (double)hit / ((double)k * (double)m);
}

}  // namespace

extern "C" int lv_autotune_window(lv_multi *multi, int32_t sub, const float *Q, int64_t m,
                                  const uint32_t *truth, int32_t truth_k, int32_t k,
                                  double target, int32_t L_max, const lv_search_params *params,
                                  int32_t *L_out, double *recall_out, void *stream) {
  lv::clear_error();
  if (!multi || !Q || !truth || !L_out) LV_FAIL(LV_EINVAL, "NULL argument");
  if (sub < 0 || sub >= (int)multi->subs.size()) LV_FAIL(LV_EINVAL, "bad sub-index");
  if (m < 1 || k < 1 || truth_k < k || L_max < k || L_max > LV_MAX_L)
    LV_FAIL(LV_EINVAL, "bad sizes");
  const lv_index *ix = multi->subs[sub];
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t *d_ids = nullptr;
  float *d_sc = nullptr, *d_qp = nullptr;
  auto cleanup = [&]() {
    if (d_ids) (void)hipFree(d_ids);
    if (d_sc) (void)hipFree(d_sc);
    if (d_qp) (void)hipFree(d_qp);
  };
  if (hipMalloc(&d_ids, sizeof(uint32_t) * m * k) != hipSuccess ||
      hipMalloc(&d_sc, sizeof(float) * m * k) != hipSuccess ||
      hipMalloc(&d_qp, sizeof(float) * m * ix->qp_width) != hipSuccess) {
    cleanup();
    LV_FAIL(LV_ENOMEM, "autotune buffers");
  }
  int rc = lv::launch_project(Q, m, ix->desc.D, ix->desc.A, ix->qp_width, d_qp, s);
  std::vector<uint32_t> got((size_t)m * k);
  auto eval = [&](int L, double *rec) -> int {
    int r = lv::launch_beam(ix, Q, d_qp, m, k, L, d_ids, d_sc, nullptr, params, s);
    if (r != LV_OK) return r;
    if (hipMemcpyAsync(got.data(), d_ids, sizeof(uint32_t) * got.size(), hipMemcpyDeviceToHost,
                       s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      lv::set_error("autotune copy failed");
      return LV_EDEVICE;
    }
    *rec = recall_host(got, k, truth, truth_k, m);
    return LV_OK;
  };
  double rec = 0.0;
  int lo = k, hi = k;
  if (rc == LV_OK) rc = eval(hi, &rec);
  while (rc == LV_OK && rec < target && hi < L_max) {
    lo = hi;
    hi = std::min(L_max, hi * 2);
    rc = eval(hi, &rec);
  }
  double rec_hi = rec;
  if (rc == LV_OK && rec_hi >= target && hi > lo) {
    // smallest L in (lo, hi] reaching the target
    int a = lo, c = hi;
    while (c - a > 1 && rc == LV_OK) {
      const int mid = (a + c) / 2;
      double r = 0.0;
      rc = eval(mid, &r);
      if (rc != LV_OK) break;
      if (r >= target) {
        c = mid;
        rec_hi = r;
      } else {
        a = mid;
      }
    }
    hi = c;
  }
  cleanup();
  if (rc != LV_OK) return rc;
  *L_out = hi;
  if (recall_out) *recall_out = rec_hi;
  return LV_OK;
}

extern "C" int lv_autotune_knobs(lv_multi *multi, const lv_batch_caps *caps,
                                 const lv_request *reqs, int32_t nreq, const float *Q,
                                 uint32_t *ids, float *scores, int32_t reps, lv_search_params *best,
                                 double *best_ms, void *stream) {
  lv::clear_error();
  if (!multi || !caps || !reqs || !best || reps < 1) LV_FAIL(LV_EINVAL, "bad arguments");
  if (nreq < 1 || nreq > caps->max_requests) LV_FAIL(LV_EINVAL, "bad request count");
  int64_t nout = 0;
  for (int i = 0; i < nreq; ++i) nout += (int64_t)reqs[i].count * reqs[i].k;
  constexpr int kFlight = 2;  // steps in flight, as a server would run them (divides kSets)
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipStream_t st[kFlight] = {s, nullptr};
  uint32_t *xids[kFlight] = {ids, nullptr};
  float *xsc[kFlight] = {scores, nullptr};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    for (int f = 1; f < kFlight; ++f) {
      if (st[f]) (void)hipStreamDestroy(st[f]);
      if (xids[f]) (void)hipFree(xids[f]);
      if (xsc[f]) (void)hipFree(xsc[f]);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  bool ok = hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
  for (int f = 1; f < kFlight && ok; ++f)
    ok = hipStreamCreateWithFlags(&st[f], hipStreamNonBlocking) == hipSuccess &&
         hipMalloc(&xids[f], sizeof(uint32_t) * (size_t)(nout > 0 ? nout : 1)) == hipSuccess &&
         hipMalloc(&xsc[f], sizeof(float) * (size_t)(nout > 0 ? nout : 1)) == hipSuccess;
  if (!ok) {
    cleanup();
    LV_FAIL(LV_ENOMEM, "autotune streams or buffers");
  }
  double best_t = -1.0;
  const int32_t expand = best->expand;  // the traversal is the caller's choice, not a knob
  lv_search_params keep{0, 0, 0, expand};
  int last_rc = LV_OK;
  // The persistent launch is not searched: with steps in flight its resident
  // wavefronts keep the next step's query projection waiting for compute
  // units, which stalls the pipeline (and it is not faster on its own).
  for (int launch : {LV_LAUNCH_PER_QUERY}) {
    // Sizes between 1024 and 2048 matter: a smaller set forgets more ids
    // (more re-scoring), a larger one leaves room in LDS for fewer wavefronts.
    for (int hs : {1024, 1280, 1536, 2048, 4096, 8192}) {
      lv_search_params p{hs, 0, launch, expand};
      lv_batch *b = nullptr;
      int rc = lv_batch_create(multi, caps, &p, &b);
      if (rc != LV_OK) {
        last_rc = rc;
        continue;  // e.g. does not fit in LDS
      }
      // f-th step of a round on stream f; streams 1.. start after `s` reaches e0
      auto round = [&]() -> int {
        for (int f = 0; f < kFlight; ++f) {
          int r = lv_batch_step(b, reqs, nreq, Q, xids[f], xsc[f], nullptr, st[f]);
          if (r != LV_OK) return r;
        }
        return LV_OK;
      };
      auto fork = [&]() {
        (void)hipEventRecord(e0, s);
        for (int f = 1; f < kFlight; ++f) (void)hipStreamWaitEvent(st[f], e0, 0);
      };
      auto join = [&]() {
        for (int f = 1; f < kFlight; ++f) {
          (void)hipEventRecord(e1, st[f]);
          (void)hipStreamWaitEvent(s, e1, 0);
        }
      };
      fork();
      rc = round();  // warm-up
      join();
      float ms = 0.f;
      if (rc == LV_OK) {
        fork();
        for (int r = 0; r < reps && rc == LV_OK; ++r) rc = round();
        join();
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
      }
      lv_batch_destroy(b);
      if (rc != LV_OK) {
        cleanup();
        return rc;
      }
      const double t = ms / (reps * kFlight);
      if (best_t < 0 || t < best_t) {
        best_t = t;
        keep = p;
      }
    }
  }
  cleanup();
  if (best_t < 0) return last_rc != LV_OK ? last_rc : LV_EDEVICE;
  *best = keep;
  if (best_ms) *best_ms = best_t;
  return LV_OK;
}
