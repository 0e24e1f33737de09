// Differentiable projection loss on the matrix cores, Adam, and the
// projection of A and B onto the spectral-norm ball after a step.
//
// For a block of b_q queries Qb and b_x database vectors Xb (rows), with
// P = b_q * b_x pairs, the refinement loss built from the LeanVec-OOD
// objective (Problem leanvec_orthonormal, trace form Problem
// leanvec_efficient on the normalised moments K_Q/m, K_X/n) is
//
//   G = Qb A^T, H = Xb B^T, Rm = Qb Xb^T - G H^T
//   loss = ||Rm||_F^2 / P + lam * f(A, B)
//   f = <A K_Q A^T, B K_X B^T>_F + tr(K_Q K_X) - 2 <A K_Q, B K_X>_F
//
// with gradients (pair part by differentiating the squared residual, trace
// part Eq. leanvec_gradients):
//   dA = -(2/P) (Rm H)^T Qb + 2 lam ((B K_X B^T) A - B K_X) K_Q
//   dB = -(2/P) (Rm^T G)^T Xb + 2 lam ((A K_Q A^T) B - A K_Q) K_X
//
// Products run on the bfloat16 matrix-core GEMM (float32 accumulation);
// two independent products of the same operand layouts share one launch
// (gemm_pair), and the trace term's products (forward) and the trace
// gradients and S (backward) run on a second stream of the library's, forked
// from the caller's stream and joined back with events.  A difference of two
// products is one launch over two K segments, with one factor kept negated
// in the workspace: Rm is
// [Qb | G] [Xb | -H]^T (K = D + d), and the trace gradients, written with
// U1 = B K_X and U2 = A K_Q as 2 lam (M2 U2 - U1 K_Q) and
// 2 lam (M1 U1 - U2 K_X), are -2 lam [-M2 | U1] [U2 ; K_Q] (K = d + D) and
// its mirror (M1 and M2 are both kept negated, which leaves <M1, M2>
// unchanged).  Rm and the trace gradients are small differences of large
// products: the products that feed them (G, H, Qb Xb^T, G H^T, B K_X, A K_Q,
// M1, M2, and the trace gradients themselves) take split-precision operands
// (hi + lo bfloat16, three matrix-core passes), which brings the relative
// error of the gradients from about 1e-2 (plain bfloat16) to about 2e-4 at
// the refinement shape.  The pair-part
// products of the backward (Rm H, Rm^T G, and their products with Qb, Xb)
// involve no cancellation and stay in plain bfloat16.  Sums of squares and inner products
// use a fixed-order two-pass float64 reduction, so results are deterministic.
#include <algorithm>
#include <mutex>
#include <vector>

#include "lv_common.h"
#include "lv_fit.h"
#include "lv_gemm.h"

namespace lv {
namespace {

constexpr int kRedBlocks = 512;

// Up to three inner products <a[j], b[j]> of n[j] floats, one per grid row.
struct DotPairs {
  const float *a[3];
  const float *b[3];
  int64_t n[3];
};

__device__ __forceinline__ double dot4(const float4 x, const float4 y) {
  return (double)x.x * (double)y.x + (double)x.y * (double)y.y + (double)x.z * (double)y.z +
         (double)x.w * (double)y.w;
}

// partial[j * gridDim.x + blockIdx.x] = sum over a grid-stride slice of
// a[j][i] * b[j][i] (float64), j = blockIdx.y.  Groups of four floats
// (16-byte aligned arrays), four groups in flight per thread, the last
// n % 4 elements by the first threads of block 0; a fixed order, so the
// sums are deterministic.
__global__ __launch_bounds__(256) void dot_partials(DotPairs p, double *__restrict__ partial) {
  __shared__ double red[256];
  const int j = blockIdx.y;
  const float *__restrict__ a = p.a[j];
  const float *__restrict__ b = p.b[j];
  const int64_t n = p.n[j];
  const float4 *__restrict__ a4 = reinterpret_cast<const float4 *>(a);
  const float4 *__restrict__ b4 = reinterpret_cast<const float4 *>(b);
  const int64_t n4 = n >> 2, stride = (int64_t)gridDim.x * 256;
  double s = 0.0;
  int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n4; i += 4 * stride) {
    float4 x[4], y[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      x[u] = a4[i + u * stride];
      y[u] = b4[i + u * stride];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) s += dot4(x[u], y[u]);
  }
  for (; i < n4; i += stride) s += dot4(a4[i], b4[i]);
  if (blockIdx.x == 0 && (int64_t)threadIdx.x < n - 4 * n4) {
    const int64_t t = 4 * n4 + threadIdx.x;
    s += (double)a[t] * (double)b[t];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)j * gridDim.x + blockIdx.x] = red[0];
}

// out[0] = total, out[1] = pair part, out[2] = trace part.  One workgroup of
// kRedBlocks threads adds the partial sums in a fixed tree order.
__global__ __launch_bounds__(kRedBlocks) void finish_loss(const double *__restrict__ partial,
                                                          int nblocks, double inv_pairs,
                                                          double trace_const, float lam,
                                                          int with_trace, float *__restrict__ out) {
  __shared__ double red[3][kRedBlocks];
  const int t = threadIdx.x;
  const int nparts = with_trace ? 3 : 1;
  for (int j = 0; j < 3; ++j)
    red[j][t] = (j < nparts && t < nblocks) ? partial[j * nblocks + t] : 0.0;
  __syncthreads();
  for (int w = kRedBlocks / 2; w > 0; w >>= 1) {
    if (t < w)
      for (int j = 0; j < 3; ++j) red[j][t] += red[j][t + w];
    __syncthreads();
  }
  if (t != 0) return;
  const double pair = red[0][0] * inv_pairs;
  const double tr = with_trace ? red[1][0] + trace_const - 2.0 * red[2][0] : 0.0;
  out[0] = (float)(pair + (double)lam * tr);
  out[1] = (float)pair;
  out[2] = (float)tr;
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p,
                                                   const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   int64_t n, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// Workspace carve (floats, each region 64-float aligned).
struct Ws {
  float *G, *H, *Rm, *T, *S, *U1, *U2, *M1, *M2;
  float *SP;          // partial products of GEMMs split over K
  float *SP2;         // the same for the products on the side stream
  size_t sp_floats;
  double *partial;
};

size_t align64(size_t n) { return (n + 63) & ~(size_t)63; }

size_t ws_floats(int64_t bq, int64_t bx, int64_t D, int64_t d, Ws *w, float *base) {
  size_t off = 0;
  auto take = [&](float **p, size_t n) {
    if (w) *p = base + off;
    off += align64(n);
  };
  Ws dummy;
  Ws *t = w ? w : &dummy;
  take(&t->G, bq * d);
  take(&t->H, bx * d);
  take(&t->Rm, bq * bx);
  take(&t->T, bq * d);
  take(&t->S, bx * d);
  take(&t->U1, d * D);
  take(&t->U2, d * D);
  take(&t->M1, d * d);
  take(&t->M2, d * d);
  // the split products have at most max(b_q, b_x) x d or d x D outputs
  // (pairs of them: twice that)
  const int64_t mn = std::max(std::max(bq, bx) * d, d * D);
  t->sp_floats = 2 * gemm_split_floats(mn, 1);
  take(&t->SP, t->sp_floats);
  take(&t->SP2, t->sp_floats);
  float *pp = nullptr;
  take(&pp, 2 * 3 * kRedBlocks);  // float64 partials
  if (w) w->partial = reinterpret_cast<double *>(pp);
  return off;
}

int check_args(const float *A, const float *B, const float *Qb, const float *Xb, int32_t bq,
               int32_t bx, int32_t D, int32_t d, void *ws, size_t ws_bytes) {
  if (bq < 1 || bx < 1 || D < 1 || d < 1 || d > D) LV_FAIL(LV_EINVAL, "bad sizes");
  if (!A || !B || !Qb || !Xb || !ws) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (reinterpret_cast<uintptr_t>(ws) & 15u) LV_FAIL(LV_EINVAL, "workspace not 16-byte aligned");
  const size_t need = ws_floats(bq, bx, D, d, nullptr, nullptr) * sizeof(float);
  if (ws_bytes < need) LV_FAIL(LV_EINVAL, "workspace of %zu bytes needed (got %zu)", need, ws_bytes);
  return LV_OK;
}

// A second stream per device for the loss's independent chains of
// products, and the events that fork work onto it from the caller's stream
// and join it back.  Each record and its wait are made under the lock, so
// that calls from several host threads cannot mix up their events; work of
// such calls on one device is serialised on the side stream.
constexpr int kMaxDevices = 64;
struct Side {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
std::mutex g_side_mu;
Side g_side[kMaxDevices];

int side_stream(Side **out) {
  int dev = 0;
  LV_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) LV_FAIL(LV_EDEVICE, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_side_mu);
  Side &sd = g_side[dev];
  if (!sd.s) {
    LV_CHECK_HIP(hipEventCreateWithFlags(&sd.fork, hipEventDisableTiming));
    LV_CHECK_HIP(hipEventCreateWithFlags(&sd.join, hipEventDisableTiming));
    LV_CHECK_HIP(hipStreamCreateWithFlags(&sd.s, hipStreamNonBlocking));
  }
  *out = &sd;
  return LV_OK;
}

// `to` waits for the work queued on `from` so far (event e).
int stream_wait(hipEvent_t e, hipStream_t from, hipStream_t to) {
  std::lock_guard<std::mutex> lock(g_side_mu);
  LV_CHECK_HIP(hipEventRecord(e, from));
  LV_CHECK_HIP(hipStreamWaitEvent(to, e, 0));
  return LV_OK;
}

// One product (arguments of lv::gemm), split over K in the workspace when
// that gives more workgroups.
#define LV_G(...)                                         \
  do {                                                    \
    int rc_ = ::lv::gemm(__VA_ARGS__, w.SP, w.sp_floats); \
    if (rc_ != LV_OK) return rc_;                         \
  } while (0)

// Two independent products of the same layouts in one launch.
#define LV_G2(...)                                             \
  do {                                                         \
    int rc_ = ::lv::gemm_pair(__VA_ARGS__, w.SP, w.sp_floats); \
    if (rc_ != LV_OK) return rc_;                              \
  } while (0)

// The same on the side stream's split workspace.
#define LV_G_SIDE(...)                                     \
  do {                                                     \
    int rc_ = ::lv::gemm(__VA_ARGS__, w.SP2, w.sp_floats); \
    if (rc_ != LV_OK) return rc_;                          \
  } while (0)
#define LV_G2_SIDE(...)                                         \
  do {                                                          \
    int rc_ = ::lv::gemm_pair(__VA_ARGS__, w.SP2, w.sp_floats); \
    if (rc_ != LV_OK) return rc_;                               \
  } while (0)

#define LV_TRY(expr)              \
  do {                            \
    int rc_ = (expr);             \
    if (rc_ != LV_OK) return rc_; \
  } while (0)

}  // namespace
}  // namespace lv

extern "C" size_t lv_projloss_workspace_size(int32_t bq, int32_t bx, int32_t D, int32_t d) {
  if (bq < 1 || bx < 1 || D < 1 || d < 1) return 0;
  return lv::ws_floats(bq, bx, D, d, nullptr, nullptr) * sizeof(float);
}

extern "C" int lv_projloss_fwd(const float *A, const float *B, const float *Qb, const float *Xb,
                               int32_t bq, int32_t bx, int32_t D, int32_t d, const float *KQn,
                               const float *KXn, double trace_const, float lam, float *loss,
                               void *ws, size_t ws_bytes, void *stream) {
  lv::clear_error();
  int rc = lv::check_args(A, B, Qb, Xb, bq, bx, D, d, ws, ws_bytes);
  if (rc != LV_OK) return rc;
  if (!loss) LV_FAIL(LV_EINVAL, "NULL loss");
  if ((KQn == nullptr) != (KXn == nullptr)) LV_FAIL(LV_EINVAL, "give both K_Q and K_X or neither");
  hipStream_t s = static_cast<hipStream_t>(stream);
  lv::Ws w;
  lv::ws_floats(bq, bx, D, d, &w, static_cast<float *>(ws));
  using lv::GemmArgs;
  const int with_trace = KQn != nullptr;
  lv::Side *side = nullptr;
  if (with_trace) {
    // on the side stream: U1 = B K_X, U2 = A K_Q (moments symmetric);
    // w.M2 = -U1 B^T, w.M1 = -U2 A^T
    LV_TRY(lv::side_stream(&side));
    LV_TRY(lv::stream_wait(side->fork, s, side->s));
    LV_G2_SIDE(GemmArgs{B, D, KXn, D, w.U1, D, d, D, D, 1.f, 0.f, 1},
               GemmArgs{A, D, KQn, D, w.U2, D, d, D, D, 1.f, 0.f, 1}, true, true, side->s);
    LV_G2_SIDE(GemmArgs{w.U1, D, B, D, w.M2, d, d, d, D, -1.f, 0.f, 1},
               GemmArgs{w.U2, D, A, D, w.M1, d, d, d, D, -1.f, 0.f, 1}, true, true, side->s);
  }
  // G = Qb A^T, and H = Xb B^T kept negated (w.H = -H)
  LV_G2(GemmArgs{Qb, D, A, D, w.G, d, bq, d, D, 1.f, 0.f, 1},
        GemmArgs{Xb, D, B, D, w.H, d, bx, d, D, -1.f, 0.f, 1}, true, true, s);
  // Rm = Qb Xb^T - G H^T = Qb Xb^T + G (-H)^T: one product over K = D + d
  {
    GemmArgs r{Qb, D, Xb, D, w.Rm, bx, bq, bx, D, 1.f, 0.f, 1};
    r.A2 = w.G;
    r.lda2 = d;
    r.B2 = w.H;
    r.ldb2 = d;
    r.K2 = d;
    LV_G(r, true, true, s);
  }
  if (side) LV_TRY(lv::stream_wait(side->join, side->s, s));
  // ||Rm||^2, then <M1, M2> and <U2, U1> (w.M1 and w.M2 both negated)
  const lv::DotPairs dp{{w.Rm, w.M1, w.U2}, {w.Rm, w.M2, w.U1},
                        {(int64_t)bq * bx, (int64_t)d * d, (int64_t)d * D}};
  hipLaunchKernelGGL(lv::dot_partials, dim3(lv::kRedBlocks, with_trace ? 3u : 1u), dim3(256), 0,
                     s, dp, w.partial);
  hipLaunchKernelGGL(lv::finish_loss, dim3(1), dim3(lv::kRedBlocks), 0, s, w.partial,
                     lv::kRedBlocks,
                     1.0 / ((double)bq * (double)bx), trace_const, lam, with_trace, loss);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

extern "C" int lv_projloss_bwd(const float *A, const float *B, const float *Qb, const float *Xb,
                               int32_t bq, int32_t bx, int32_t D, int32_t d, const float *KQn,
                               const float *KXn, float lam, float grad_scale, float *dA,
                               float *dB, void *ws, size_t ws_bytes, void *stream) {
  lv::clear_error();
  int rc = lv::check_args(A, B, Qb, Xb, bq, bx, D, d, ws, ws_bytes);
  if (rc != LV_OK) return rc;
  if (!dA || !dB) LV_FAIL(LV_EINVAL, "NULL gradient output");
  if ((KQn == nullptr) != (KXn == nullptr)) LV_FAIL(LV_EINVAL, "give both K_Q and K_X or neither");
  hipStream_t s = static_cast<hipStream_t>(stream);
  lv::Ws w;
  lv::ws_floats(bq, bx, D, d, &w, static_cast<float *>(ws));
  using lv::GemmArgs;
  const float c = -2.f * grad_scale / (float)((double)bq * (double)bx);
  lv::Side *side = nullptr;
  LV_TRY(lv::side_stream(&side));
  LV_TRY(lv::stream_wait(side->fork, s, side->s));
  if (KQn) {  // on the side stream, first: the trace part of dA and dB
    const float t = 2.f * lam * grad_scale;
    // dA = t (M2 U2 - U1 K_Q) = -t ((-M2) U2 + U1 K_Q): K = d, then K = D
    // (b(n, k) read as U2[k][n] and K_Q[k][n])
    GemmArgs ga{w.M2, d, w.U2, D, dA, D, d, D, d, -t, 0.f, 1};
    ga.A2 = w.U1;
    ga.lda2 = D;
    ga.B2 = KQn;
    ga.ldb2 = D;
    ga.K2 = D;
    // dB = t (M1 U1 - U2 K_X) = -t ((-M1) U1 + U2 K_X)
    GemmArgs gb{w.M1, d, w.U1, D, dB, D, d, D, d, -t, 0.f, 1};
    gb.A2 = w.U2;
    gb.lda2 = D;
    gb.B2 = KXn;
    gb.ldb2 = D;
    gb.K2 = D;
    LV_G2_SIDE(ga, gb, true, false, side->s);
  }
  // S = Rm^T G (bx x d) on the side stream, T = Rm H = -(Rm (-H)) (bq x d;
  // w.H holds -H) on the caller's
  LV_G_SIDE(GemmArgs{w.Rm, bx, w.G, d, w.S, d, bx, d, bq, 1.f, 0.f}, false, false, side->s);
  LV_G(GemmArgs{w.Rm, bx, w.H, d, w.T, d, bq, d, bx, -1.f, 0.f}, true, false, s);
  LV_TRY(lv::stream_wait(side->join, side->s, s));
  // dA (+)= c T^T Qb, dB (+)= c S^T Xb (added to the trace part if any)
  const float beta = KQn ? 1.f : 0.f;
  LV_G2(GemmArgs{w.T, d, Qb, D, dA, D, d, D, bq, c, beta},
        GemmArgs{w.S, d, Xb, D, dB, D, d, D, bx, c, beta}, false, false, s);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

extern "C" int lv_adam_step(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                            float beta1, float beta2, float eps, int32_t t, void *stream) {
  lv::clear_error();
  if (n < 0 || t < 1) LV_FAIL(LV_EINVAL, "bad n or step");
  if (n > 0 && (!p || !g || !m || !v)) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && lr >= 0.f && eps > 0.f))
    LV_FAIL(LV_EINVAL, "bad Adam hyper-parameters");
  if (n == 0) return LV_OK;
  const float c1 = 1.f - powf(beta1, (float)t);
  const float c2 = 1.f - powf(beta2, (float)t);
  const unsigned blocks = (unsigned)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
  hipLaunchKernelGGL(lv::adam_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     p, g, m, v, n, lr, beta1, beta2, eps, c1, c2);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

namespace lv {
namespace {

// G = M M^T for M [d][D] float32: one thread per entry, float64 sums in
// order of k (the products of float32 values are exact in float64).
__global__ __launch_bounds__(256) void gram_kernel(const float *__restrict__ M, int32_t d,
                                                   int32_t D, double *__restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)d * d) return;
  const int i = (int)(e / d), j = (int)(e % d);
  const float *a = M + (int64_t)i * D;
  const float *b = M + (int64_t)j * D;
  double s = 0.0;
  for (int k = 0; k < D; ++k) s = fma((double)a[k], (double)b[k], s);
  G[e] = s;
}

// out = T M (T [d][d] float64, M [d][D] float32), float64 sums, rounded to
// float32.
__global__ __launch_bounds__(256) void apply_clip_kernel(const double *__restrict__ T,
                                                         const float *__restrict__ M, int32_t d,
                                                         int32_t D, float *__restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)d * D) return;
  const int i = (int)(e / D), c = (int)(e % D);
  double s = 0.0;
  for (int j = 0; j < d; ++j) s = fma(T[(int64_t)i * d + j], (double)M[(int64_t)j * D + c], s);
  out[e] = (float)s;
}

}  // namespace
}  // namespace lv

extern "C" size_t lv_clip_spectral_device_workspace_size(int32_t d, int32_t D) {
  if (d < 1 || D < 1) return 0;
  return (size_t)2 * d * d * sizeof(double) + (size_t)d * D * sizeof(float);
}

extern "C" int lv_clip_spectral_device(float *M, int32_t d, int32_t D, void *ws, size_t ws_bytes,
                                       void *stream) {
  lv::clear_error();
  if (!M) LV_FAIL(LV_EINVAL, "NULL matrix");
  if (d < 1 || D < 1 || d > 1024) LV_FAIL(LV_EINVAL, "bad sizes (1 <= d <= 1024, D >= 1)");
  if (!ws || ws_bytes < lv_clip_spectral_device_workspace_size(d, D))
    LV_FAIL(LV_EINVAL, "workspace too small (need %zu bytes)",
            lv_clip_spectral_device_workspace_size(d, D));
  if (reinterpret_cast<uintptr_t>(ws) & 7u) LV_FAIL(LV_EINVAL, "workspace not 8-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *G = static_cast<double *>(ws);
  double *T = G + (size_t)d * d;
  float *out = reinterpret_cast<float *>(T + (size_t)d * d);
  const size_t dd = (size_t)d * d;
  hipLaunchKernelGGL(lv::gram_kernel, dim3((unsigned)((dd + 255) / 256)), dim3(256), 0, s, M, d,
                     D, G);
  LV_CHECK_LAUNCH();
  std::vector<double> g(dd), t(dd);
  LV_CHECK_HIP(hipMemcpyAsync(g.data(), G, dd * sizeof(double), hipMemcpyDeviceToHost, s));
  LV_CHECK_HIP(hipStreamSynchronize(s));
  if (!lv::clip_factor(d, g.data(), t.data())) return LV_OK;
  LV_CHECK_HIP(hipMemcpyAsync(T, t.data(), dd * sizeof(double), hipMemcpyHostToDevice, s));
  const size_t n = (size_t)d * D;
  hipLaunchKernelGGL(lv::apply_clip_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     T, M, d, D, out);
  LV_CHECK_LAUNCH();
  LV_CHECK_HIP(hipMemcpyAsync(M, out, n * sizeof(float), hipMemcpyDeviceToDevice, s));
  // the host copy of T must outlive the transfer
  LV_CHECK_HIP(hipStreamSynchronize(s));
  return LV_OK;
}
