/*
 * leanvec.h -- C ABI of the MI355X (gfx950) LeanVec search library.
 *
 * LeanVec (Tepper et al., "LeanVec: Searching vectors faster by making them
 * fit") answers maximum-inner-product queries (Section 2, notation) with the
 * approximation <q, x> ~ <A q, quant(B x)> (Eq. 1): a greedy graph traversal
 * scores candidates against quantised d-dimensional "primary" vectors, and
 * the surviving candidates are re-ranked against full-dimension "secondary"
 * vectors (Section 2, "Search").  The projections A, B come from LeanVec-ID
 * (Section 2.1) or LeanVec-OOD (Sections 2.2-2.4).
 *
 * Conventions for every call:
 *  - Return value: LV_OK (0) on success, LV_WNOTCONVERGED (1) as a warning,
 *    a negative LV_E* code on error.  lv_last_error() then returns a
 *    thread-local message.  No C++ exception crosses this interface.
 *  - All argument validation happens on the host before any device work, so
 *    a rejected call has enqueued nothing.
 *  - Matrices are row-major; vectors are rows.  Projections are [d][D].
 *  - "device" pointers are HIP device memory owned by the caller; "host"
 *    pointers are ordinary host memory owned by the caller.  The library
 *    keeps no pointer beyond the call except where a handle says it borrows.
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).  Device
 *    calls are asynchronous on that stream; a kernel fault surfaces at the
 *    caller's next synchronising call.
 *  - Integer sizes are int64_t for element counts, int32_t for dimensions.
 */
#ifndef LEANVEC_H
#define LEANVEC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LV_OK 0
#define LV_WNOTCONVERGED 1
#define LV_EINVAL (-1)
#define LV_ENOMEM (-2)
#define LV_EDEVICE (-3)
#define LV_EUNSUPPORTED (-4)

#define LV_SENTINEL 0xFFFFFFFFu /* padding id in adjacency rows and results */
#define LV_MAX_L 1024           /* largest search window */
#define LV_MAX_K 1024

/* Secondary-vector element types. */
#define LV_F32 0
#define LV_F16 1
#define LV_LVQ8 2 /* secondary vectors compressed with LVQ-8 */
#define LV_F16_RESID 3 /* float16 residual coordinates: only D - d per vector (see below) */
#define LV_LVQ8_LEVEL2 4 /* 8-bit second level of the primaries' LVQ: d per vector (see below) */

/* Library version (major * 10000 + minor * 100 + patch). */
int lv_version(void);

/* Message describing the last error on the calling thread ("" if none). */
const char *lv_last_error(void);

/* ------------------------------------------------------------------------
 * Projection learning (host, float64, synchronous).
 * ---------------------------------------------------------------------- */

/*
 * Second moment accumulation, K += sum_i v_i v_i^T (the matrices K_Q = Q Q^T
 * and K_X = X X^T of Problem leanvec_efficient, with vectors as columns of
 * Q and X).  Accumulating lets the caller sample or stream chunks (the
 * paper subsamples m = 1e4 queries and n = 1e5 database vectors).
 *   V:   host float32 [n][D]
 *   K:   host float64 [D][D], accumulated in place (symmetric)
 *   sum: host float64 [D] or NULL; if given, sum += sum_i v_i (for the LVQ
 *        centring vector)
 * Errors: LV_EINVAL for NULL V/K, n < 0 or D < 1.
 */
int lv_second_moment(const float *V, int64_t n, int32_t D, double *K, double *sum);

/*
 * LeanVec-ID (Section 2.1, Problem pca): P = the d leading eigenvectors of
 * K_X, as rows, so that A = B = P.  Rows are ordered by decreasing
 * eigenvalue and signed so that each row's largest-magnitude entry is
 * positive.
 *   KX:    host float64 [D][D], symmetric
 *   P:     host float64 [d][D] out
 *   evals: host float64 [D] out (all eigenvalues, decreasing) or NULL
 * Errors: LV_EINVAL unless 1 <= d <= D.
 */
int lv_fit_id(const double *KX, int32_t D, int32_t d, double *P, double *evals);

/* Options of lv_fit_ood. */
typedef struct {
  double alpha;     /* step-size exponent, gamma_t = (t+1)^-alpha; 0 < alpha < 1 */
  double tol;       /* stop when |f_{t+1} - f_t| / f_t <= tol */
  int32_t max_iter; /* at most this many iterations */
  int32_t init;     /* LV_FW_INIT_* */
} lv_fw_params;

#define LV_FW_INIT_ES 0    /* eigenvectors of K_Q/m + K_X/n (eigenvector search at beta = 1/2) */
#define LV_FW_INIT_ZERO 1  /* A = B = 0 as suggested in Algorithm 1 */
#define LV_FW_INIT_GIVEN 2 /* start from the A and B passed in */

/* Progress of lv_fit_ood. */
typedef struct {
  int32_t iters;     /* iterations performed */
  int32_t converged; /* 1 if the stop rule fired */
  double f_first;    /* f(A_0, B_0) on the normalised moments */
  double f_last;     /* f at the returned A, B */
  double *f_hist;    /* caller array of max_iter + 1 entries, or NULL */
  double *gap_hist;  /* caller array of max_iter entries (FW gap of the A and B steps summed), or NULL */
} lv_fw_report;

/*
 * LeanVec-OOD by Frank-Wolfe block coordinate descent (Algorithm 1) on the
 * relaxed problem (Problem leanvec) over the spectral-norm ball C (Eq.
 * stiefel_convex_hull), with the partial gradients of Eq. leanvec_gradients
 * and the linear step S = U V^T from the SVD of the negative gradient
 * (Section 2.3).  K_Q / m and K_X / n are used (this leaves the iterates
 * unchanged).
 *   KQ, KX: host float64 [D][D]; m, n: the sample counts behind them
 *   p:      options (NULL = alpha 0.9, tol 1e-3, 500 iterations, ES start)
 *   A, B:   host float64 [d][D] out (inputs too with LV_FW_INIT_GIVEN)
 *   r:      report or NULL
 * Returns LV_OK, or LV_WNOTCONVERGED if max_iter was reached first.
 * Errors: LV_EINVAL for bad sizes or options.
 */
int lv_fit_ood(const double *KQ, int64_t m, const double *KX, int64_t n, int32_t D,
               int32_t d, const lv_fw_params *p, double *A, double *B, lv_fw_report *r);

/*
 * LeanVec-OOD by eigenvector search (Section 2.4, Algorithm 2): A = B = P,
 * the d leading eigenvectors of K_beta = (1-beta)/m K_Q + beta/n K_X, with
 * beta in [0, 1] minimising the equalised loss (Problem
 * leanvec_loss_same_proj_equalized) by golden-section/parabolic (Brent)
 * search to within xtol.
 *   P:    host float64 [d][D] out;  beta: host double out (may be NULL)
 * Errors: LV_EINVAL for bad sizes or xtol <= 0.
 */
int lv_fit_es(const double *KQ, int64_t m, const double *KX, int64_t n, int32_t D, int32_t d,
              double xtol, double *P, double *beta);

/*
 * The LeanVec-OOD objective f(A, B) in its trace form (Problem
 * leanvec_efficient) on K_Q / m and K_X / n, in float64.
 */
int lv_ood_loss(const double *KQ, int64_t m, const double *KX, int64_t n, int32_t D, int32_t d,
                const double *A, const double *B, double *f);

/*
 * LVQ centring vector mu = M (sum / n): the projection of the mean of the
 * vectors whose sum lv_second_moment accumulated, rounded to float32.
 *   M: host float64 [d][D]; sum: host float64 [D]; mu: host float32 [d] out
 * Errors: LV_EINVAL for NULL pointers, n < 1 or bad sizes.
 */
int lv_mean_reduced(const double *M, int32_t d, int32_t D, const double *sum, int64_t n,
                    float *mu);

/* Host float64 -> float32 -> bfloat16 (each step round to nearest even),
 * for the device projections. */
int lv_to_bf16(const double *src, int64_t count, uint16_t *dst);

/* ------------------------------------------------------------------------
 * Index construction (device).
 * ---------------------------------------------------------------------- */

/*
 * Reduced vectors out[i] = M v_i (Eq. 1: B x for the database, A q for the
 * queries) on the matrix cores: bfloat16 operands (V is rounded to
 * bfloat16 on load), float32 accumulation.
 *   V:   device float32 [rows][D]
 *   M:   device bfloat16 bits [d][D]
 *   out: device float32 [rows][d]
 * Errors: LV_EINVAL for NULL pointers, rows < 0, D < 1, D % 8 != 0,
 *         d < 1, d > 1024.
 */
int lv_project(const float *V, int64_t rows, int32_t D, const uint16_t *M, int32_t d,
               float *out, void *stream);

/*
 * Record stride the search kernels support for d components at 4 or 8
 * bits: code bytes + 8, rounded up to 64, 96, 128, 192, 256, 512, 768 or
 * 1024 (0 if none fits).  A record is read by a group of lanes, one chunk
 * each: 16 x 4, 8 x 12, 16 x 8, 16 x 12, 16 x 16, 64 x 8, 64 x 12 or 64 x 16
 * bytes.
 */
int32_t lv_record_stride(int32_t d, int32_t bits);

/*
 * LVQ encoding of primary vectors (quant in Eq. 1; LVQ is a per-vector
 * scale-and-bias scalar quantiser).  With r = y - mu computed in float64:
 * l = min r, u = max r, delta = float32((u - l)/(2^bits - 1)),
 * lo = float32(l), code_j = clamp(floor((r_j - lo)/delta + 0.5), 0,
 * 2^bits - 1) (all zero when delta = 0).  Record layout per vector:
 * code bytes (bits = 8: one per component; bits = 4: component 2i in the
 * low nibble of byte i, 2i+1 in the high nibble), float32 delta, float32
 * lo, zero padding to record_stride.  Results are bit-exact (IEEE float64
 * division and floor, no contraction).
 *   Y:       device float32 [n][d];  mu: device float32 [d]
 *   records: device [n][record_stride] bytes out
 * Errors: LV_EINVAL unless bits is 4 or 8, d % 8 == 0, 8 <= d <= 2048 and
 *         record_stride >= d*bits/8 + 8 is a multiple of 4.
 */
int lv_lvq_encode(const float *Y, int64_t n, int32_t d, const float *mu, int32_t bits,
                  void *records, int32_t record_stride, void *stream);

/*
 * Reconstruction of LVQ records (the decode of the quantiser of Eq. 1; for
 * checks and tests, not on the search path):
 * out[v][j] = float32((mu_j + lo_v) + delta_v c_vj), evaluated in float64 in
 * that order (delta c is exact), i.e. the float64 reconstruction rounded to
 * float32.
 *   records: device [n][record_stride] bytes (lv_lvq_encode's layout)
 *   mu: device float32 [d];  out: device float32 [n][d]
 * Errors: LV_EINVAL as for lv_lvq_encode, or NULL pointers with n > 0.
 */
int lv_lvq_decode(const void *records, int64_t n, int32_t d, int32_t bits, int32_t record_stride,
                  const float *mu, float *out, void *stream);

/*
 * Database projection and LVQ encoding in one pass (Eq. 1: quant(B x) for
 * every database vector): the records lv_project(V, rows, D, M, d) followed
 * by lv_lvq_encode(out, rows, d, mu, bits) would write, bit for bit, without
 * the float32 reduced vectors going through memory (each workgroup holds
 * whole rows of B x and encodes them from the accumulators).
 *   V: device float32 [rows][D];  M: device bfloat16 bits [d][D] (B)
 *   mu: device float32 [d];  records: device [rows][record_stride] bytes out
 * Errors: LV_EINVAL for rows < 0, D < 8 or D % 8 != 0, d outside [8, 256] or
 *         d % 8 != 0, bits not 4 or 8, record_stride < d*bits/8 + 8 or not a
 *         multiple of 4, NULL pointers with rows > 0.
 */
int lv_project_encode(const float *V, int64_t rows, int32_t D, const uint16_t *M, int32_t d,
                      const float *mu, int32_t bits, void *records, int32_t record_stride,
                      void *stream);

/*
 * Second level of a two-level LVQ (LV_LVQ8_LEVEL2 rows; the scheme LVQ4x8
 * of the LVQ baseline in Appendix D and Fig. 1, which the paper names
 * without restating): for every vector, the residual of its primary record
 * r2_j = (y_j - mu_j) - (lo + delta c_j) in float64 (in this order; delta c_j
 * is exact), then l2 = min r2, u2 = max r2, delta2 = float32((u2 - l2) / 255),
 * lo2 = float32(l2), c2_j = clamp(floor((r2_j - lo2) / delta2 + 0.5), 0, 255)
 * (all zero when delta2 = 0).  Row layout: see lv_secondary_row_bytes.
 * Results are bit-exact (IEEE float64 division and floor, no contraction).
 *   Y, mu, bits: as given to lv_lvq_encode for the records
 *   records: device [n][record_stride] bytes, the vectors' primary records
 *   rows:    device [n][row_bytes] bytes out; row_bytes must equal
 *            lv_secondary_row_bytes(d, LV_LVQ8_LEVEL2)
 * Errors: LV_EINVAL as for lv_lvq_encode, for d > 1008, a row_bytes other
 *         than that, or NULL pointers with n > 0.
 */
int lv_lvq_encode_level2(const float *Y, int64_t n, int32_t d, const float *mu, int32_t bits,
                         const void *records, int32_t record_stride, void *rows,
                         int32_t row_bytes, void *stream);

/* Secondary vectors (Section 2: quant(x), here float16): float32 -> float16,
 * round to nearest even.  X: device float32 [count]; out: device [count]. */
int lv_to_f16(const float *X, int64_t count, uint16_t *out, void *stream);

/* ------------------------------------------------------------------------
 * Search (device).
 * ---------------------------------------------------------------------- */

/* Everything a search reads.  All pointers are device memory BORROWED by
 * the index handle: they must stay valid and unchanged while it lives. */
typedef struct {
  int64_t N;               /* database size (< 2^31) */
  int32_t D;               /* full dimension */
  int32_t d;               /* reduced dimension */
  int32_t bits;            /* LVQ bits of the primary records: 4 or 8 */
  int32_t record_stride;   /* bytes per primary record (lv_record_stride) */
  const void *records;     /* [N][record_stride] LVQ records */
  const float *mu;         /* [d] LVQ centring vector */
  int32_t sec_dtype;       /* LV_F32, LV_F16, LV_LVQ8, LV_F16_RESID or LV_LVQ8_LEVEL2 */
  const void *secondaries; /* [N][lv_secondary_row_bytes(D, sec_dtype)] bytes
                              (D - d in place of D for LV_F16_RESID, d for
                              LV_LVQ8_LEVEL2) */
  int32_t R;               /* graph out-degree, 1..1024 */
  const uint32_t *adjacency; /* [N][R]; valid ids first, then LV_SENTINEL */
  uint32_t entry;          /* traversal start node */
  const uint16_t *A;       /* [d][D] bfloat16 query projection, or NULL; for
                              LV_F16_RESID [D][D]: the primary projection's d rows
                              followed by D - d rows completing an orthonormal basis */
  const float *sec_mu;     /* [D] centring vector of LV_LVQ8 secondaries, else NULL */
} lv_index_desc;

/*
 * Bytes per secondary row: 4 D (LV_F32), 2 D (LV_F16), or for LV_LVQ8 (the
 * secondary vectors compressed with 8-bit LVQ, Section 3 ablation on the
 * secondary representation) D code bytes, float32 delta, float32 lo and zero
 * padding to D + 16 bytes, written by lv_lvq_encode(X, N, D, sec_mu, 8, rows,
 * D + 16) and scored as <q, sec_mu + lo + delta * c>.  Returns 0 when the
 * search kernels do not support the combination (rows above 2 KiB, or
 * LV_LVQ8 with D not a multiple of 16 or above 1008).
 *
 * LV_F16_RESID (LeanVec-ID, A = B = P with orthonormal rows; the remark after
 * Eq. pca that the error (I - P^T P) x needs only D - d coordinates): with
 * R = [P; P_perp] orthonormal, <q, x> = <P q, P x> + <P_perp q, P_perp x>.
 * A secondary row holds P_perp x in float16 (2 (D - d) bytes: pass D - d here),
 * and the re-rank score is the traversal's primary score <P q, y^> plus
 * <P_perp q, P_perp x>, so the first d coordinates are not stored twice.
 *
 * LV_LVQ8_LEVEL2 (two-level LVQ of the primaries; LVQ4x8 when the records
 * have 4 bits, the scheme of the LVQ baseline in Appendix D and Fig. 1): a
 * row refines the primary record of the same vector with an 8-bit LVQ of its
 * quantisation residual r2 = (y - mu) - (lo + delta c), per-vector min / max
 * and no centring: 16 ceil(d / 16) code bytes (one per reduced component,
 * zero padded), float32 delta2, float32 lo2, 8 zero bytes (pass d here; d <=
 * 1008), written by lv_lvq_encode_level2.  The re-rank score is the
 * traversal's primary score plus <A q, lo2 + delta2 c2>, which is <A q, y^>
 * for the two-level reconstruction y^ = mu + lo + delta c + lo2 + delta2 c2:
 * re-ranking reads d more bytes per candidate and no full-dimension vector
 * (Q is not read).
 */
int32_t lv_secondary_row_bytes(int32_t D, int32_t sec_dtype);

typedef struct lv_index lv_index;

/* Validate desc and make a handle (host memory only; borrows the device
 * pointers).  Errors: LV_EINVAL for inconsistent sizes or NULL data,
 * LV_EUNSUPPORTED for a record stride or dimension the kernels lack. */
int lv_index_create(const lv_index_desc *desc, lv_index **out);
int lv_index_destroy(lv_index *index);

/*
 * Performance knobs.  They never change results.  The per-query visited set
 * lives in LDS and may forget an id (a forgotten node met again is scored
 * again and dropped if it is already in the window), so its size trades LDS
 * (and hence resident wavefronts) against repeated scoring.
 */
typedef struct {
  int32_t hash_slots; /* visited-set slots per query (a multiple of 256 in 256..65536;
                         0 = 1024) */
  int32_t probes;     /* slots tried before an id replaces the one in its home slot
                         (1..16; 0 = 2 below 4096 slots, 8 from 4096 slots) */
  int32_t launch;     /* batched traversal: LV_LAUNCH_PER_QUERY (0, one workgroup
                         per query, scheduled by the hardware) or LV_LAUNCH_PERSISTENT
                         (1, resident wavefronts pull queries from a device counter).
                         lv_search / lv_search_projected: 0 and 1 give one wavefront
                         per query; LV_LAUNCH_TEAM (2) gives each query a workgroup of
                         4 wavefronts that score every batch of candidates together
                         (lower latency for batches too small to fill the GPU; same
                         results as one wavefront with the same `expand`).  The batched
                         traversal refuses LV_LAUNCH_TEAM (LV_EINVAL). */
  int32_t expand;     /* entries expanded per iteration: 0 or 1 = the paper's traversal
                         (one expansion at a time); 2..8 = a throughput variant that
                         expands the `expand` best unexpanded entries together (its results
                         differ; they are exact for that variant) */
} lv_search_params;
#define LV_LAUNCH_PER_QUERY 0
#define LV_LAUNCH_PERSISTENT 1
#define LV_LAUNCH_TEAM 2

/* Bytes of device workspace lv_search needs for m queries. */
size_t lv_search_workspace_size(const lv_index *index, int64_t m);

/*
 * Search m queries (Section 2 "Search"): q' = A q on the matrix cores, then
 * one wavefront per query runs the best-first traversal with window L on
 * the primary records (expand the best unexpanded candidate under the
 * order (score descending, id ascending), score its unvisited
 * out-neighbours, keep the best L), then re-ranks every candidate left in
 * the window with <q, secondary> and returns the best k (ties: smaller id).
 * Scores are float64.  Primary scores use the projected query on a grid of
 * its own, q~_j = rint(q_j 2^s) 2^-s with s = 22 - e for the largest |q_j| =
 * f 2^e, f in [0.5, 1) (within 2^-22 of the largest component), on which the
 * inner product with the codes is an exact integer sum; re-ranking reads the
 * query as given.  Projected queries must be finite.
 *   Q:        device float32 [m][D]
 *   ids:      device uint32 [m][k] out;  scores: device float32 [m][k] out
 *   counters: device uint32 [m][2] out (expansions, primary scorings) or NULL
 *   ws:       device workspace of lv_search_workspace_size bytes
 * If fewer than k nodes were reached, the tail is LV_SENTINEL / -inf.
 * Errors: LV_EINVAL for k < 1, L < k, L > LV_MAX_L, k > LV_MAX_K, m < 0,
 *         missing A, small workspace or NULL pointers.
 */
int lv_search(const lv_index *index, const float *Q, int64_t m, int32_t k, int32_t L,
              uint32_t *ids, float *scores, uint32_t *counters, void *ws, size_t ws_bytes,
              const lv_search_params *params, void *stream);

/*
 * The same search with the projected queries supplied by the caller
 * (Qp: device float32 [m][d]); Q is still needed for the re-ranking.  With
 * LV_F16_RESID secondaries Qp rows hold D values, P q then P_perp q (what
 * lv_search computes with the [D][D] matrix A), and Q is not read.
 */
int lv_search_projected(const lv_index *index, const float *Q, const float *Qp, int64_t m,
                        int32_t k, int32_t L, uint32_t *ids, float *scores, uint32_t *counters,
                        const lv_search_params *params, void *stream);

/*
 * lv_search without a workspace, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that
 * forbid allocation).  It allocates nothing: the projected queries, which
 * lv_search keeps in the caller's workspace, go to a fixed array of
 * LV_NOALLOC_SCRATCH_BYTES (16 MiB) that the library holds on each device it
 * runs on until the process ends, so m * (d, or D with LV_F16_RESID) * 4
 * bytes must fit in it (about 26,000 queries at d = 160); larger m is
 * refused with LV_EINVAL before anything is launched.  All calls on one
 * device share its array: calls that overlap on a device race (serialise
 * them, e.g. on one stream).  Arguments, results and other errors as for
 * lv_search; the results are identical to lv_search's.
 */
#define LV_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
int lv_search_noalloc(const lv_index *index, const float *Q, int64_t m, int32_t k, int32_t L,
                      uint32_t *ids, float *scores, uint32_t *counters,
                      const lv_search_params *params, void *stream);

/* ------------------------------------------------------------------------
 * Batched search over several indexes (device, persistent kernel).
 *
 * The paper answers one query per thread with no batching (Eq. 1 needs no
 * batch processing).  A GPU needs many queries in flight, and a serving
 * stream brings requests of uneven size against different indexes, so a
 * step packs many requests into one persistent launch: its wavefronts take
 * queries from a device counter, each query searched exactly as by
 * lv_search (same results).  Steps are captured as hipGraphs.
 * ---------------------------------------------------------------------- */

typedef struct lv_multi lv_multi;

/* A set of sub-indexes searched together.  All must share D, d, bits,
 * record_stride, secondary type and have a query projection A; d <= 256.
 * The handle copies the index descriptors to the device (it borrows the
 * indexes' device data, which must outlive it).
 * Errors: LV_EINVAL for count < 1, NULL entries or mismatched layouts. */
int lv_multi_create(const lv_index *const *subs, int32_t count, lv_multi **out);
int lv_multi_destroy(lv_multi *multi);

/* One request of a step: `count` consecutive queries searched in sub-index
 * `sub` with (k, L).  Queries of request i follow those of request i-1 in
 * the step's query array; results of request i (count * k ids and scores)
 * follow those of request i-1 in the output arrays. */
typedef struct {
  int32_t sub;
  int32_t k;
  int32_t L;
  int32_t count;
} lv_request;

typedef struct {
  int32_t max_requests; /* requests per step */
  int32_t max_L;        /* largest window of any request */
  int64_t max_queries;  /* queries per step */
} lv_batch_caps;

typedef struct lv_batch lv_batch;

/* Allocate a step's device buffers (request table, projected-query
 * workspace) and pinned request tables, size the persistent grid to the
 * device's resident wavefronts, and capture the step (request-table copy,
 * grouped query projection on the matrix cores, persistent search) as two
 * hipGraphs used alternately.  Knobs in params change no result.
 * Errors: LV_EINVAL for bad caps, LV_ENOMEM, LV_EDEVICE. */
int lv_batch_create(lv_multi *multi, const lv_batch_caps *caps, const lv_search_params *params,
                    lv_batch **out);
int lv_batch_destroy(lv_batch *batch);

/*
 * Run one step on `stream`: validate and pack the requests on the host,
 * then launch the two captured graphs (table copy + grouped projection,
 * then counter reset + persistent traversal).  Asynchronous.  Steps rotate
 * through four sets of pinned table and device state; a set is reused four
 * steps later, once the step that used it has finished (the host waits for
 * its table copy, `stream` waits for its traversal).  Up to four
 * consecutive steps issued on different streams therefore run concurrently;
 * their output buffers must then be distinct.  Rotate over 2 or 4 streams:
 * the step that reuses a set is then on the stream of the step that used it
 * (with 3 streams the reuse waits cross streams and stall the pipeline).
 *   Q:        device float32 [sum count][D]
 *   ids:      device uint32 [sum count * k] out; scores: device float32, same
 *   counters: device uint32 [sum count][2] out (expansions, scorings) or NULL
 * Errors: LV_EINVAL for nreq outside [1, max_requests], a request with a bad
 *         sub-index, k < 1, L < k, L > max_L, count < 1, or more than
 *         max_queries queries in total.
 */
int lv_batch_step(lv_batch *batch, const lv_request *reqs, int32_t nreq, const float *Q,
                  uint32_t *ids, float *scores, uint32_t *counters, void *stream);

/*
 * lv_batch_step, and record two caller-owned hipEvents (created with timing
 * enabled) on `stream`: ev_begin after the table copy and query projection,
 * ev_end after the persistent traversal, so that their elapsed time is the
 * traversal kernel's own duration (counter reset included).
 * Errors: those of lv_batch_step; LV_EINVAL if an event is NULL.
 */
int lv_batch_step_timed(lv_batch *batch, const lv_request *reqs, int32_t nreq, const float *Q,
                        uint32_t *ids, float *scores, uint32_t *counters, void *ev_begin,
                        void *ev_end, void *stream);

/*
 * Autotuner, result-affecting part: the smallest window L in [k, L_max]
 * whose k-recall@k on learning queries (Q: device float32 [m][D]) against
 * their true neighbours (truth: host uint32 [m][truth_k], truth_k >= k)
 * reaches `target` in sub-index `sub` (runtime parameters are calibrated on
 * a learning query set, Section 3).  Doubling, then bisection; recall is
 * taken as non-decreasing in L.  Writes L_out (L_max if never reached) and
 * the recall there.  Synchronises `stream`.
 */
int lv_autotune_window(lv_multi *multi, int32_t sub, const float *Q, int64_t m,
                       const uint32_t *truth, int32_t truth_k, int32_t k, double target,
                       int32_t L_max, const lv_search_params *params, int32_t *L_out,
                       double *recall_out, void *stream);

/*
 * Autotuner, performance part: for each visited-set size in {1024, 1280,
 * 1536, 2048, 4096, 8192} that fits, times `reps` rounds of two steps of the given
 * requests in flight at once (on internal streams, the way consecutive steps
 * overlap in service) with the per-query launch, and returns the fastest in
 * best (these knobs never change results).  The persistent launch is not
 * searched: with steps in flight its resident wavefronts hold the compute
 * units that the next step's query projection needs.  best_ms gets the mean
 * time per step.  ids/scores receive one step's output.  best->expand is read
 * on input and kept (the traversal is the caller's choice, not a knob).
 * Synchronises `stream`.
 */
int lv_autotune_knobs(lv_multi *multi, const lv_batch_caps *caps, const lv_request *reqs,
                      int32_t nreq, const float *Q, uint32_t *ids, float *scores, int32_t reps,
                      lv_search_params *best, double *best_ms, void *stream);

/* ------------------------------------------------------------------------
 * Graph construction on the primary vectors (device).
 * ---------------------------------------------------------------------- */

#define LV_MAX_BUILD_PASSES 8

typedef struct {
  int32_t R;          /* largest out-degree, 1..64 */
  int32_t L;          /* search window while building, 1..LV_MAX_L (more than R
                         gives the pruning a choice) */
  int32_t passes;     /* 1..LV_MAX_BUILD_PASSES */
  int32_t hash_slots; /* visited-set slots of the construction searches (0: 2048);
                         the result does not depend on it */
  double alphas[LV_MAX_BUILD_PASSES]; /* pruning factor of each pass, >= 0 */
  int64_t max_batch;  /* largest number of nodes inserted together, >= 1 */
  int64_t stop_after; /* 0: complete build; n > 0: stop after n batches */
  int64_t *stats;     /* optional host [LV_BUILD_STATS]: work done (see below), or NULL */
} lv_build_params;

/* Work counters of lv_graph_build (indexes into lv_build_params.stats). */
#define LV_BUILD_STATS 7
#define LV_BS_SEARCHES 0    /* construction searches */
#define LV_BS_EXPANSIONS 1  /* adjacency rows read by them */
#define LV_BS_SCORINGS 2    /* records scored by them */
#define LV_BS_FWD_CANDS 3   /* candidates scored by forward pruning */
#define LV_BS_REV_TARGETS 4 /* nodes that received reverse edges */
#define LV_BS_REV_PRUNES 5  /* of those, rows pruned (union longer than R) */
#define LV_BS_REV_CANDS 6   /* candidates scored by reverse pruning */

/*
 * Build a graph of out-degree <= R over the primary vectors (Appendix A:
 * per node, a search of the current graph with the node as query collects
 * L candidates, which are pruned to at most R diverse out-neighbours;
 * Section 2 "Graph construction": only the primary vectors take part;
 * Appendix D: Vamana's pruning with factor alpha).  Distances are squared
 * Euclidean distances between LVQ reconstructions, from exact integer code
 * sums and one fixed sequence of float64 operations.
 *
 * Nodes are inserted in `order` (host [N], a permutation of 0..N-1) in
 * batches: 1, 2, 4, ... up to max_batch nodes in pass 0, max_batch nodes in
 * later passes.  Inside a batch every search sees the graph as it was when
 * the batch began; a node's pool is its final window followed by its current
 * out-neighbours; pruning sorts the pool by (distance, id), skips the node
 * and repeats, and keeps c unless a kept k has alpha^2 d(k,c) <= d(p,c), up
 * to R.  Then every target j of a new edge p -> j gets the new sources
 * (ascending) that are not in its row; a row longer than R is pruned around
 * j.  The result is fully determined by the inputs (no dependence on
 * scheduling).
 *
 * records: device, [N][record_stride] in the lv_lvq_encode layout (d
 *   components of `bits` bits, d * bits / 8 <= 256 bytes).  entry: start
 *   node of every search.  adjacency: device [N][R], written (valid ids
 *   first, then LV_SENTINEL).  Allocates and frees its own device scratch;
 *   runs on `stream` and synchronizes it before returning.
 * Errors: LV_EINVAL for NULL pointers, bad sizes or parameters, an order
 *   that is not a permutation; LV_EUNSUPPORTED for R > 64, wider records,
 *   an unsupported stride, or a node receiving more than 256 new edges in
 *   one batch (lower max_batch); LV_EDEVICE, LV_ENOMEM.
 */
int lv_graph_build(const void *records, int32_t record_stride, int64_t N, int32_t d,
                   int32_t bits, const uint32_t *order, uint32_t entry,
                   const lv_build_params *params, uint32_t *adjacency, void *stream);

/* ------------------------------------------------------------------------
 * Differentiable projection refinement (device, matrix cores).
 * ---------------------------------------------------------------------- */

/*
 * C = alpha * op(A) op(B)^T + beta * C on the matrix cores (operands rounded
 * to bfloat16, float32 accumulation), the product the loss kernels use.
 * a(m, k) is A[m*lda + k] if a_kcont else A[k*lda + m]; likewise b(n, k).
 * C: device float32 [M][ldc].  beta = 0 does not read C.
 * workspace: optional device buffer of workspace_bytes (caller-owned; NULL
 * or 0 for none).  With one, a product with few output tiles and a long K
 * is split over K into partial products there, which a second kernel adds
 * in a fixed order (the result does not depend on scheduling); a smaller
 * workspace than lv_gemm_workspace_size gives fewer parts.  Calls that
 * share a workspace must not overlap, nor may the workspace overlap A, B or
 * C.
 */
int lv_gemm(const float *A, int32_t a_kcont, int64_t lda, const float *B, int32_t b_kcont,
            int64_t ldb, float *C, int64_t ldc, int32_t M, int32_t N, int32_t K, float alpha,
            float beta, void *workspace, size_t workspace_bytes, void *stream);

/*
 * The same product with split-precision operands: every float32 operand x
 * is taken as hi + lo, hi = bf16(x), lo = bf16(x - hi), and the product is
 * accumulated as hi*hi + hi*lo + lo*hi (three matrix-core passes), for a
 * relative error per operand of about 2^-17 instead of 2^-9.  The loss
 * kernels use it for the products whose results cancel (the residual of
 * Problem leanvec_orthonormal and the trace gradients of Eq.
 * leanvec_gradients).  Arguments, workspace and errors as for lv_gemm.
 */
int lv_gemm_split(const float *A, int32_t a_kcont, int64_t lda, const float *B,
                  int32_t b_kcont, int64_t ldb, float *C, int64_t ldc, int32_t M, int32_t N,
                  int32_t K, float alpha, float beta, void *workspace, size_t workspace_bytes,
                  void *stream);

/*
 * The same matrix-core product (the projections' arithmetic: bfloat16
 * operands, float32 accumulation) for operands already held as bfloat16,
 * as a caller converts them once for many products:
 *   C[m][n] = alpha * sum_k A[m][k] B[n][k] + beta * C[m][n]
 * A: device bfloat16 bits [M][lda], B: device bfloat16 bits [N][ldb] (both
 * k-contiguous rows), C: device float32 [M][ldc]; beta = 0 does not read C.
 * Runs on 256 x 256 output tiles (meant for large products; no split over
 * K, no workspace).  Errors: LV_EINVAL for negative sizes, NULL pointers,
 * leading dimensions below K (A, B) or N (C), and rows of A or B that are
 * not 16-byte aligned (pointers aligned, lda and ldb multiples of 8).
 */
int lv_gemm_bf16(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb, float *C,
                 int64_t ldc, int32_t M, int32_t N, int32_t K, float alpha, float beta,
                 void *stream);

/* Workspace bytes with which lv_gemm may split an M x N product the most. */
size_t lv_gemm_workspace_size(int32_t M, int32_t N);

/* Device workspace bytes for lv_projloss_fwd / lv_projloss_bwd. */
size_t lv_projloss_workspace_size(int32_t bq, int32_t bx, int32_t D, int32_t d);

/*
 * Sampled-pair refinement loss of the LeanVec-OOD objective (Problem
 * leanvec_orthonormal): for queries Qb [bq][D] and database vectors Xb
 * [bx][D] (device float32 rows) and projections A, B [d][D],
 *   loss = ||Qb Xb^T - (Qb A^T)(Xb B^T)^T||_F^2 / (bq bx) + lam * f(A, B),
 * f the trace form (Problem leanvec_efficient) on normalised moments KQn =
 * K_Q/m, KXn = K_X/n (device float32 [D][D], symmetric; both NULL to drop
 * the trace part) with trace_const = tr(KQn KXn) supplied by the caller.
 * loss: device float32 [3] out = {total, pair part, trace part f}.
 * Leaves the intermediates lv_projloss_bwd needs in ws (device buffer of
 * lv_projloss_workspace_size bytes, 16-byte aligned, caller-owned).
 * Stream-ordered on `stream`: independent products run on a second stream
 * of the library's own (one per device, default priority), forked from
 * `stream` and joined back to it with events before the call's last
 * kernels, so the results are ready in `stream` order.  Calls from several
 * host threads on one device share that second stream.  Errors: LV_EINVAL
 * for bad sizes, NULL or unaligned pointers, a short workspace, or one of
 * KQn / KXn NULL; LV_EDEVICE for a failed stream, event or launch.
 */
int lv_projloss_fwd(const float *A, const float *B, const float *Qb, const float *Xb, int32_t bq,
                    int32_t bx, int32_t D, int32_t d, const float *KQn, const float *KXn,
                    double trace_const, float lam, float *loss, void *ws, size_t ws_bytes,
                    void *stream);

/*
 * Gradients of that loss times grad_scale (Eq. leanvec_gradients for the
 * trace part; the pair part by differentiating the squared residual):
 * dA, dB device float32 [d][D] out.  ws must hold the intermediates of the
 * preceding lv_projloss_fwd on the same arguments.  Streams and errors as
 * for lv_projloss_fwd (the second stream is used with or without the trace
 * part).
 */
int lv_projloss_bwd(const float *A, const float *B, const float *Qb, const float *Xb, int32_t bq,
                    int32_t bx, int32_t D, int32_t d, const float *KQn, const float *KXn,
                    float lam, float grad_scale, float *dA, float *dB, void *ws, size_t ws_bytes,
                    void *stream);

/* One Adam update (Kingma & Ba) of n parameters: m, v are the moment
 * buffers (device float32), t >= 1 the step number for bias correction. */
int lv_adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr, float beta1,
                 float beta2, float eps, int32_t t, void *stream);

/* Host float64: project M [d][D] onto the spectral-norm ball C (Eq.
 * stiefel_convex_hull) by clipping its singular values at 1, in place. */
int lv_clip_spectral(double *M, int32_t d, int32_t D);

/*
 * The same projection for a device float32 M [d][D] (1 <= d <= 1024), in
 * place on `stream`: the Gram matrix M M^T is formed on the device in
 * float64, its eigendecomposition and the d x d factor are computed on the
 * host in float64 (as lv_clip_spectral does), and the factor is applied on
 * the device in float64 with the result rounded to float32.  ws: device
 * buffer of lv_clip_spectral_device_workspace_size bytes, 8-byte aligned,
 * caller-owned.  Synchronises with `stream` (the Gram matrix is read back).
 * Errors: LV_EINVAL for NULL pointers, bad sizes or a small workspace.
 */
int lv_clip_spectral_device(float *M, int32_t d, int32_t D, void *ws, size_t ws_bytes,
                            void *stream);
size_t lv_clip_spectral_device_workspace_size(int32_t d, int32_t D);

#ifdef __cplusplus
}
#endif

#endif /* LEANVEC_H */
