// LVQ encoding of the primary vectors, the second level of a two-level LVQ
// (LVQ4x8 of the baseline setup, Appendix D), and float16 conversion of the
// secondary vectors (Section 2: primary vectors quant(Bx), secondary vectors
// quant(x)).
//
// One wavefront encodes one vector: lanes own component pairs (2i, 2i+1),
// the min / max of r = y - mu are wave reductions in float64, and every
// code is computed with IEEE float64 division and floor, so the bytes equal
// a float64 reference exactly.  This file is compiled without floating-point
// contraction.
#include "lv_common.h"
#include "lv_lvq.h"

namespace lv {
namespace {

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

template <int BITS>
__global__ __launch_bounds__(256) void encode_kernel(const float *__restrict__ Y, int64_t n,
                                                     int32_t d, const float *__restrict__ mu,
                                                     unsigned char *__restrict__ rec,
                                                     int32_t stride) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (v >= n) return;
  const float *y = Y + v * d;
  double lmin = INFINITY, lmax = -INFINITY;
  for (int j = lane; j < d; j += 64) {
    const double r = (double)y[j] - (double)mu[j];
    lmin = fmin(lmin, r);
    lmax = fmax(lmax, r);
  }
  const double l = wave_min(lmin);
  const double u = wave_max(lmax);
  const double levels = (double)((1 << BITS) - 1);
  const float delta32 = (float)((u - l) / levels);
  const float lo32 = (float)l;
  const double delta = (double)delta32, lo = (double)lo32;
  unsigned char *out = rec + v * (int64_t)stride;
  for (int i = lane; 2 * i < d; i += 64) {
    const double r0 = (double)y[2 * i] - (double)mu[2 * i];
    const double r1 = (double)y[2 * i + 1] - (double)mu[2 * i + 1];
    const uint32_t c0 = lvq_code(r0, lo, delta, levels);
    const uint32_t c1 = lvq_code(r1, lo, delta, levels);
    if (BITS == 8) {
      *reinterpret_cast<uint16_t *>(out + 2 * i) = (uint16_t)(c0 | (c1 << 8));
    } else {
      out[i] = (unsigned char)(c0 | (c1 << 4));
    }
  }
  const int cb = d * BITS / 8;
  if (lane == 0) {
    uint32_t *w = reinterpret_cast<uint32_t *>(out + cb);
    w[0] = __float_as_uint(delta32);
    w[1] = __float_as_uint(lo32);
  }
  for (int b = cb + 8 + 4 * lane; b < stride; b += 256)
    *reinterpret_cast<uint32_t *>(out + b) = 0u;
}

// Second level of a two-level LVQ: one wavefront per vector re-reads the
// vector's primary record, forms the residual r2 = (y - mu) - (lo + delta c)
// in float64 and quantises it to 8 bits (per-vector min / max, no centring).
// Row: 16 ceil(d / 16) code bytes, float32 delta2, float32 lo2, 8 zero bytes.
template <int BITS>
__global__ __launch_bounds__(256) void encode_level2_kernel(
    const float *__restrict__ Y, int64_t n, int32_t d, const float *__restrict__ mu,
    const unsigned char *__restrict__ rec, int32_t stride, unsigned char *__restrict__ rows,
    int32_t row_bytes) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (v >= n) return;
  const float *y = Y + v * d;
  const unsigned char *r1 = rec + v * (int64_t)stride;
  const int cb = d * BITS / 8;
  const double delta = (double)__uint_as_float(*reinterpret_cast<const uint32_t *>(r1 + cb));
  const double lo = (double)__uint_as_float(*reinterpret_cast<const uint32_t *>(r1 + cb + 4));
  auto resid = [&](int j) {
    const uint32_t c = BITS == 8 ? r1[j] : (r1[j >> 1] >> (4 * (j & 1))) & 0xFu;
    const double r = (double)y[j] - (double)mu[j];
    return r - (lo + delta * (double)c);
  };
  double lmin = INFINITY, lmax = -INFINITY;
  for (int j = lane; j < d; j += 64) {
    const double r2 = resid(j);
    lmin = fmin(lmin, r2);
    lmax = fmax(lmax, r2);
  }
  const double l = wave_min(lmin);
  const double u = wave_max(lmax);
  const float delta32 = (float)((u - l) / 255.0);
  const float lo32 = (float)l;
  const double delta2 = (double)delta32, lo2 = (double)lo32;
  unsigned char *out = rows + v * (int64_t)row_bytes;
  const int padded = (d + 15) / 16 * 16;
  for (int j = lane; j < padded; j += 64)
    out[j] = j < d ? (unsigned char)lvq_code(resid(j), lo2, delta2, 255.0) : (unsigned char)0;
  if (lane < 4) {
    const uint32_t w = lane == 0 ? __float_as_uint(delta32) : (lane == 1 ? __float_as_uint(lo32) : 0u);
    *reinterpret_cast<uint32_t *>(out + padded + 4 * lane) = w;
  }
}

// Reconstruction of LVQ records: out[v][j] = float32((mu_j + lo) + delta c_j),
// evaluated in float64 in that order (delta c_j is exact), one wavefront per
// vector.
template <int BITS>
__global__ __launch_bounds__(256) void decode_kernel(const unsigned char *__restrict__ rec,
                                                     int64_t n, int32_t d, int32_t stride,
                                                     const float *__restrict__ mu,
                                                     float *__restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t v = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (v >= n) return;
  const unsigned char *r = rec + v * (int64_t)stride;
  const int cb = d * BITS / 8;
  const double delta = (double)__uint_as_float(*reinterpret_cast<const uint32_t *>(r + cb));
  const double lo = (double)__uint_as_float(*reinterpret_cast<const uint32_t *>(r + cb + 4));
  for (int j = lane; j < d; j += 64) {
    const uint32_t c = BITS == 8 ? r[j] : (r[j >> 1] >> (4 * (j & 1))) & 0xFu;
    out[v * d + j] = (float)(((double)mu[j] + lo) + delta * (double)c);
  }
}

// float32 -> float16 with the hardware conversion (round to nearest even).
__global__ __launch_bounds__(256) void to_f16_kernel(const float *__restrict__ x, int64_t count,
                                                     _Float16 *__restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
    out[i] = (_Float16)x[i];
}

}  // namespace
}  // namespace lv

extern "C" int32_t lv_record_stride(int32_t d, int32_t bits) {
  if (d < 1 || (bits != 4 && bits != 8) || (d * bits) % 32 != 0) return 0;
  const int32_t need = d * bits / 8 + 8;
  static const int32_t strides[] = {64, 96, 128, 192, 256, 512, 768, 1024};
  for (int32_t s : strides)
    if (need <= s) return s;
  return 0;
}

extern "C" int lv_lvq_encode(const float *Y, int64_t n, int32_t d, const float *mu, int32_t bits,
                             void *records, int32_t record_stride, void *stream) {
  lv::clear_error();
  if (bits != 4 && bits != 8) LV_FAIL(LV_EINVAL, "bits must be 4 or 8 (got %d)", bits);
  if (d < 8 || d > 2048 || d % 8 != 0) LV_FAIL(LV_EINVAL, "d must be a multiple of 8 in [8, 2048]");
  if (n < 0) LV_FAIL(LV_EINVAL, "n must be >= 0");
  if (record_stride < d * bits / 8 + 8 || record_stride % 4 != 0)
    LV_FAIL(LV_EINVAL, "record_stride %d too small or not a multiple of 4", record_stride);
  if (n > 0 && (!Y || !mu || !records)) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (n == 0) return LV_OK;
  const int per_block = 4;
  const int64_t blocks = (n + per_block - 1) / per_block;
  if (blocks > 0x7FFFFFFF) LV_FAIL(LV_EINVAL, "n too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (bits == 8)
    hipLaunchKernelGGL(lv::encode_kernel<8>, dim3((unsigned)blocks), dim3(64 * per_block), 0, s, Y,
                       n, d, mu, static_cast<unsigned char *>(records), record_stride);
  else
    hipLaunchKernelGGL(lv::encode_kernel<4>, dim3((unsigned)blocks), dim3(64 * per_block), 0, s, Y,
                       n, d, mu, static_cast<unsigned char *>(records), record_stride);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

extern "C" int lv_lvq_encode_level2(const float *Y, int64_t n, int32_t d, const float *mu,
                                    int32_t bits, const void *records, int32_t record_stride,
                                    void *rows, int32_t row_bytes, void *stream) {
  lv::clear_error();
  if (bits != 4 && bits != 8) LV_FAIL(LV_EINVAL, "bits must be 4 or 8 (got %d)", bits);
  if (d < 8 || d > 1008 || d % 8 != 0) LV_FAIL(LV_EINVAL, "d must be a multiple of 8 in [8, 1008]");
  if (n < 0) LV_FAIL(LV_EINVAL, "n must be >= 0");
  if (record_stride < d * bits / 8 + 8 || record_stride % 4 != 0)
    LV_FAIL(LV_EINVAL, "record_stride %d too small or not a multiple of 4", record_stride);
  const int32_t want = lv_secondary_row_bytes(d, LV_LVQ8_LEVEL2);
  if (row_bytes != want)
    LV_FAIL(LV_EINVAL, "row_bytes %d must be %d for d = %d", row_bytes, want, d);
  if (n > 0 && (!Y || !mu || !records || !rows)) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (n == 0) return LV_OK;
  const int per_block = 4;
  const int64_t blocks = (n + per_block - 1) / per_block;
  if (blocks > 0x7FFFFFFF) LV_FAIL(LV_EINVAL, "n too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned char *rec = static_cast<const unsigned char *>(records);
  unsigned char *out = static_cast<unsigned char *>(rows);
  if (bits == 8)
    hipLaunchKernelGGL(lv::encode_level2_kernel<8>, dim3((unsigned)blocks), dim3(64 * per_block), 0,
                       s, Y, n, d, mu, rec, record_stride, out, row_bytes);
  else
    hipLaunchKernelGGL(lv::encode_level2_kernel<4>, dim3((unsigned)blocks), dim3(64 * per_block), 0,
                       s, Y, n, d, mu, rec, record_stride, out, row_bytes);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

extern "C" int lv_lvq_decode(const void *records, int64_t n, int32_t d, int32_t bits,
                             int32_t record_stride, const float *mu, float *out, void *stream) {
  lv::clear_error();
  if (bits != 4 && bits != 8) LV_FAIL(LV_EINVAL, "bits must be 4 or 8 (got %d)", bits);
  if (d < 8 || d > 2048 || d % 8 != 0) LV_FAIL(LV_EINVAL, "d must be a multiple of 8 in [8, 2048]");
  if (n < 0) LV_FAIL(LV_EINVAL, "n must be >= 0");
  if (record_stride < d * bits / 8 + 8 || record_stride % 4 != 0)
    LV_FAIL(LV_EINVAL, "record_stride %d too small or not a multiple of 4", record_stride);
  if (n > 0 && (!records || !mu || !out)) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (n == 0) return LV_OK;
  const int per_block = 4;
  const int64_t blocks = (n + per_block - 1) / per_block;
  if (blocks > 0x7FFFFFFF) LV_FAIL(LV_EINVAL, "n too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const unsigned char *rec = static_cast<const unsigned char *>(records);
  if (bits == 8)
    hipLaunchKernelGGL(lv::decode_kernel<8>, dim3((unsigned)blocks), dim3(64 * per_block), 0, s,
                       rec, n, d, record_stride, mu, out);
  else
    hipLaunchKernelGGL(lv::decode_kernel<4>, dim3((unsigned)blocks), dim3(64 * per_block), 0, s,
                       rec, n, d, record_stride, mu, out);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

extern "C" int lv_to_f16(const float *X, int64_t count, uint16_t *out, void *stream) {
  lv::clear_error();
  if (count < 0) LV_FAIL(LV_EINVAL, "count must be >= 0");
  if (count == 0) return LV_OK;
  if (!X || !out) LV_FAIL(LV_EINVAL, "NULL pointer");
  int64_t blocks = (count + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(lv::to_f16_kernel, dim3((unsigned)blocks), dim3(256), 0,
                     static_cast<hipStream_t>(stream), X, count, reinterpret_cast<_Float16 *>(out));
  LV_CHECK_LAUNCH();
  return LV_OK;
}
