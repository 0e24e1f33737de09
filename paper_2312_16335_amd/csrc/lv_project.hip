// Reduced vectors out = V M^T on the gfx950 matrix cores (Eq. 1: A q and
// B x).  bfloat16 operands, float32 accumulation.
//
// The projection streams V once and is bound by HBM bandwidth (about 2d/4
// flop per byte for float32 input), so the design goal is one pass over V
// with full cache lines: each wavefront owns 32 rows and all d output
// columns (ceil(d/32) 32x32 accumulator tiles), walks D in steps of 32
// (two 32x32x16 MFMAs per tile per step, so every 128-byte line of a row is
// consumed by one wavefront in one step), rounds V to bfloat16 in
// registers, and reads M (d x D bfloat16, a few hundred KB, L2-resident)
// directly as the B operand.  No LDS is needed.
#include "lv_common.h"
#include "lv_lvq.h"
#include "lv_search.h"

namespace lv {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;

// Two floats to bfloat16 (round to nearest even) in one conversion instruction.
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
  typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
  const bf16x2 h = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, h);
}

// A operand: 8 consecutive k of one row, as bfloat16.
__device__ __forceinline__ bf16x8 load_a(const float *p, bool ok) {
  u32x4 w;
  if (ok) {
    const float4 x0 = *reinterpret_cast<const float4 *>(p);
    const float4 x1 = *reinterpret_cast<const float4 *>(p + 4);
    w[0] = pack2(x0.x, x0.y);
    w[1] = pack2(x0.z, x0.w);
    w[2] = pack2(x1.x, x1.y);
    w[3] = pack2(x1.z, x1.w);
  } else {
    w[0] = w[1] = w[2] = w[3] = 0u;
  }
  return __builtin_bit_cast(bf16x8, w);
}

__device__ __forceinline__ bf16x8 load_b(const uint16_t *p, bool ok) {
  u32x4 w;
  if (ok) {
    const uint4 x = *reinterpret_cast<const uint4 *>(p);
    w[0] = x.x; w[1] = x.y; w[2] = x.z; w[3] = x.w;
  } else {
    w[0] = w[1] = w[2] = w[3] = 0u;
  }
  return __builtin_bit_cast(bf16x8, w);
}

// One wavefront computes out[row][col0 + c] for rows [row0, row0 + 32) that
// are < row_end and the NT * 32 columns from col0 (those < d).
template <int NT>
__device__ __forceinline__ void project_rows(const float *__restrict__ V, int64_t row0,
                                             int64_t row_end, int32_t D,
                                             const uint16_t *__restrict__ M, int32_t d,
                                             int32_t col0, float *__restrict__ out,
                                             int64_t out_stride, int lane) {
  const int r = lane & 31;   // row of the A operand / column of the B operand
  const int kh = lane >> 5;  // which 8-wide k half of a 16-wide step
  const int64_t arow = row0 + r;
  const bool arow_ok = arow < row_end;
  const float *ap = V + (arow_ok ? arow : row0) * (int64_t)D;

  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;

  for (int k0 = 0; k0 < D; k0 += 32) {
    const int ka = k0 + 8 * kh;       // first MFMA of the step
    const int kb = k0 + 16 + 8 * kh;  // second MFMA
    const bf16x8 a0 = load_a(ap + ka, arow_ok && ka < D);
    const bf16x8 a1 = load_a(ap + kb, arow_ok && kb < D);
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = col0 + t * 32 + r;
      const bool cok = col < d;
      const uint16_t *bp = M + (int64_t)(cok ? col : 0) * D;
      const bf16x8 b0 = load_b(bp + ka, cok && ka < D);
      const bf16x8 b1 = load_b(bp + kb, cok && kb < D);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[t], 0, 0, 0);
    }
  }
  // accumulator layout: lane holds column (lane % 32); register i holds row
  // 8 * (i / 4) + 4 * (lane / 32) + (i % 4)
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = col0 + t * 32 + r;
    if (col >= d) continue;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int64_t row = row0 + 8 * (i >> 2) + 4 * kh + (i & 3);
      if (row < row_end) out[row * out_stride + col] = acc[t][i];
    }
  }
}

// Large row counts (the database projection): a workgroup of kRowWaves
// wavefronts owns kRowWaves x 32 rows and NT x 32 columns from col0.  Per
// K step of 32 the slab of M it needs (NT x 32 columns x 32 k, bfloat16) is
// staged once in LDS for all its wavefronts (double-buffered, one barrier
// per step) instead of every wavefront reading it from L2, and each
// wavefront's next step of V is in flight while the current step's
// products run.  Every output gets the same MFMA sequence as project_rows
// (same operand slices, same order), so the result is bit-identical to the
// query kernels'.
constexpr int kRowWaves = 8;
constexpr int kSlabPitch = 40;  // bfloat16 per LDS slab row: 32 k + 8 (bank spread)

template <int CTRL>
__device__ __forceinline__ double dpp64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, 0xF, 0xF, false);
  const uint32_t hi =
      (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double xor16_64(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)b, 16, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(b >> 32), 16, 64);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Minimum and maximum over each half wavefront (32 lanes): quad swaps, row
// rotations by 4 and 8, then the other row of the half.
__device__ __forceinline__ void half_minmax(double &mn, double &mx) {
  mn = fmin(mn, dpp64<0xB1>(mn));  // quad_perm [1, 0, 3, 2]
  mx = fmax(mx, dpp64<0xB1>(mx));
  mn = fmin(mn, dpp64<0x4E>(mn));  // quad_perm [2, 3, 0, 1]
  mx = fmax(mx, dpp64<0x4E>(mx));
  mn = fmin(mn, dpp64<0x124>(mn));  // row_ror 4
  mx = fmax(mx, dpp64<0x124>(mx));
  mn = fmin(mn, dpp64<0x128>(mn));  // row_ror 8
  mx = fmax(mx, dpp64<0x128>(mx));
  mn = fmin(mn, xor16_64(mn));
  mx = fmax(mx, xor16_64(mx));
}

// LVQ records (Eq. 1 quant(Bx); the layout and arithmetic of lv_lvq_encode)
// of the wavefront's 32 projected rows, straight from the accumulators: per
// row the float64 min / max of y - mu over the d columns (a reduction across
// the 32 lanes holding the row), then each lane's codes, stored as bytes
// (32 consecutive bytes of a row per half wavefront), the row's delta and lo,
// and the zero padding up to the stride.
template <int NT, int BITS>
__device__ __forceinline__ void encode_rows(const f32x16 (&acc)[NT], int64_t row0, int64_t rows,
                                            int32_t d, const float *__restrict__ mu,
                                            unsigned char *__restrict__ rec, int32_t stride,
                                            int lane) {
  const int r = lane & 31, kh = lane >> 5;
  constexpr double levels = (double)((1 << BITS) - 1);
  const int cb = d * BITS / 8;
  const int npad = (stride - cb - 8) / 4;  // zero words after delta and lo
  double muv[NT];
  bool cok[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int col = t * 32 + r;
    cok[t] = col < d;
    muv[t] = cok[t] ? (double)mu[col] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    // one row at a time: keeps the float64 temporaries of one row live, not of all 16
    __builtin_amdgcn_sched_barrier(0);
    const int64_t grow = row0 + 8 * (i >> 2) + 4 * kh + (i & 3);
    const bool live = grow < rows;
    double mn = INFINITY, mx = -INFINITY;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (cok[t]) {
        const double v = (double)acc[t][i] - muv[t];
        mn = fmin(mn, v);
        mx = fmax(mx, v);
      }
    }
    half_minmax(mn, mx);
    const float delta32 = (float)((mx - mn) / levels);
    const float lo32 = (float)mn;
    const double delta = (double)delta32, lo = (double)lo32;
    unsigned char *row = rec + (live ? grow : 0) * (int64_t)stride;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = t * 32 + r;
      const uint32_t c = cok[t] ? lvq_code((double)acc[t][i] - muv[t], lo, delta, levels) : 0u;
      if constexpr (BITS == 8) {
        if (live && cok[t]) row[col] = (unsigned char)c;
      } else {  // component 2j in the low nibble of byte j, 2j + 1 in the high nibble
        const uint32_t odd = (uint32_t)__builtin_amdgcn_mov_dpp((int)c, 0xB1, 0xF, 0xF, false);
        if (live && cok[t] && (r & 1) == 0) row[col >> 1] = (unsigned char)(c | (odd << 4));
      }
    }
    if (live) {
      uint32_t *w = reinterpret_cast<uint32_t *>(row + cb);
      if (r == 0) w[0] = __float_as_uint(delta32);
      if (r == 1) w[1] = __float_as_uint(lo32);
      for (int j = r; j < npad; j += 32) w[2 + j] = 0u;
    }
  }
}

//
// ENC = 4 or 8: the workgroup holds all d <= 256 columns (col0 = 0) and
// writes LVQ records of ENC bits (encode_rows) instead of the float32 rows,
// so the reduced vectors never go through memory.
template <int NT, int ENC = 0>
__global__ __launch_bounds__(64 * kRowWaves) void project_kernel(
    const float *__restrict__ V, int64_t rows, int32_t D, const uint16_t *__restrict__ M,
    int32_t d, int32_t col0, float *__restrict__ out, const float *__restrict__ mu = nullptr,
    unsigned char *__restrict__ rec = nullptr, int32_t stride = 0) {
  __shared__ __align__(16) uint16_t slab[2][NT * 32 * kSlabPitch];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * kRowWaves + (tid >> 6)) * 32;
  const int r = lane & 31, kh = lane >> 5;
  const int64_t arow = row0 + r;
  const bool arow_ok = arow < rows;
  const float *ap = V + (arow_ok ? arow : 0) * (int64_t)D;
  constexpr int kPieces = NT * 32 * 4;  // 16-byte pieces of one slab (4 per column)
  constexpr int kPer = (kPieces + 64 * kRowWaves - 1) / (64 * kRowWaves);  // per thread
  // the slab of step k0 (columns past d and k past D are zero): global -> registers,
  // then registers -> LDS buffer b
  uint4 mreg[kPer];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int pc = tid + i * 64 * kRowWaves;
      const int c = pc >> 2, part = pc & 3;
      const int col = col0 + c, k = k0 + 8 * part;
      mreg[i] = make_uint4(0u, 0u, 0u, 0u);
      if (pc < kPieces && col < d && k < D)
        mreg[i] = *reinterpret_cast<const uint4 *>(M + (int64_t)col * D + k);
    }
  };
  auto put = [&](int b) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int pc = tid + i * 64 * kRowWaves;
      if (pc < kPieces)
        *reinterpret_cast<uint4 *>(&slab[b][(pc >> 2) * kSlabPitch + 8 * (pc & 3)]) = mreg[i];
    }
  };
  f32x16 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[t][i] = 0.f;
  const int nsteps = (D + 31) / 32;
  fetch(0);
  put(0);
  bf16x8 a0 = load_a(ap + 8 * kh, arow_ok && 8 * kh < D);
  bf16x8 a1 = load_a(ap + 16 + 8 * kh, arow_ok && 16 + 8 * kh < D);
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    const int k0 = 32 * s;
    const bool more = s + 1 < nsteps;
    bf16x8 n0 = a0, n1 = a1;
    if (more) {  // next step's rows of V and slab of M in flight during this step's products
      const int ka = k0 + 32 + 8 * kh, kb = k0 + 48 + 8 * kh;
      n0 = load_a(ap + ka, arow_ok && ka < D);
      n1 = load_a(ap + kb, arow_ok && kb < D);
      fetch(k0 + 32);
    }
    const uint16_t *sb = slab[s & 1];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const uint16_t *bp = sb + (t * 32 + r) * kSlabPitch;
      const bf16x8 b0 = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(bp + 8 * kh));
      const bf16x8 b1 =
          __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(bp + 16 + 8 * kh));
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[t], 0, 0, 0);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[t], 0, 0, 0);
    }
    if (more) put((s + 1) & 1);  // that buffer was last read two steps ago
    __syncthreads();
    a0 = n0;
    a1 = n1;
  }
  if (row0 >= rows) return;
  if constexpr (ENC != 0) {
    encode_rows<NT, ENC>(acc, row0, rows, d, mu, rec, stride, lane);
  } else {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int col = col0 + t * 32 + r;
      if (col >= d) continue;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t row = row0 + 8 * (i >> 2) + 4 * kh + (i & 3);
        if (row < rows) out[row * d + col] = acc[t][i];
      }
    }
  }
}

// Few rows (query batches): one workgroup per 32-row tile and one wavefront
// per 32-column tile (kColWaves per workgroup, grid y for more), so that a
// batch of a few thousand rows still reaches every CU; the wavefronts of a
// workgroup share the tile's rows through the caches.  Every output column
// gets the same sequence of MFMAs as in project_kernel, so the two kernels
// give bit-identical results.
constexpr int kColWaves = 8;
// Up to this many rows the column-tiled kernel is used (the row-tiled one
// streams a large matrix once; both give the same bits).
constexpr int64_t kFewRows = 65536;

__global__ __launch_bounds__(64 * kColWaves) void project_cols_kernel(
    const float *__restrict__ V, int64_t rows, int32_t D, const uint16_t *__restrict__ M,
    int32_t d, float *__restrict__ out) {
  const int64_t row0 = (int64_t)blockIdx.x * 32;
  const int32_t col0 = ((int32_t)blockIdx.y * kColWaves + (int32_t)(threadIdx.x >> 6)) * 32;
  if (row0 >= rows || col0 >= d) return;
  project_rows<1>(V, row0, rows, D, M, d, col0, out, d, threadIdx.x & 63);
}

// Batched form, laid out as project_cols_kernel: one workgroup per 32-row
// tile of the step's requests (each tile uses the query projection of its
// request's sub-index), one wavefront per 32-column tile.  Tiles beyond the
// step's count exit (the grid is sized for the capacity).
__global__ __launch_bounds__(64 * kColWaves) void project_grouped_kernel(
    const StepHeader *__restrict__ hdr, const IndexView *__restrict__ subs, int32_t D,
    int32_t d) {
  const int32_t col0 = ((int32_t)blockIdx.y * kColWaves + (int32_t)(threadIdx.x >> 6)) * 32;
  const int t = blockIdx.x;
  if (t >= hdr->ntiles || col0 >= d) return;
  const Request *req = reinterpret_cast<const Request *>(hdr + 1);
  int lo = 0, hi = hdr->nreq - 1;  // last request with tile0 <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (req[mid].tile0 <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const Request r = req[lo];
  const int64_t row0 = r.q_begin + (int64_t)(t - r.tile0) * 32;
  project_rows<1>(hdr->Q, row0, r.q_end, D, subs[r.sub].A, d, col0, hdr->Qp, hdr->qp_stride,
                  threadIdx.x & 63);
}

// Wavefronts per workgroup and workgroups along y for d output columns.
void col_layout(int32_t d, unsigned *waves, unsigned *yblocks) {
  const unsigned tiles = (unsigned)((d + 31) / 32);
  *waves = tiles < (unsigned)kColWaves ? tiles : (unsigned)kColWaves;
  *yblocks = (tiles + *waves - 1) / *waves;
}

template <int NT>
void launch_nt(const float *V, int64_t rows, int32_t D, const uint16_t *M, int32_t d, int32_t col0,
               float *out, hipStream_t s) {
  const int64_t blocks = (rows + 32 * kRowWaves - 1) / (32 * kRowWaves);
  hipLaunchKernelGGL(project_kernel<NT>, dim3((unsigned)blocks), dim3(64 * kRowWaves), 0, s, V,
                     rows, D, M, d, col0, out);
}

template <int NT, int ENC>
void launch_enc(const float *V, int64_t rows, int32_t D, const uint16_t *M, int32_t d,
                const float *mu, unsigned char *rec, int32_t stride, hipStream_t s) {
  const int64_t blocks = (rows + 32 * kRowWaves - 1) / (32 * kRowWaves);
  hipLaunchKernelGGL((project_kernel<NT, ENC>), dim3((unsigned)blocks), dim3(64 * kRowWaves), 0, s,
                     V, rows, D, M, d, 0, nullptr, mu, rec, stride);
}

template <int ENC>
void launch_enc_bits(const float *V, int64_t rows, int32_t D, const uint16_t *M, int32_t d,
                     const float *mu, unsigned char *rec, int32_t stride, hipStream_t s) {
  switch ((d + 31) / 32) {
    case 1: launch_enc<1, ENC>(V, rows, D, M, d, mu, rec, stride, s); break;
    case 2: launch_enc<2, ENC>(V, rows, D, M, d, mu, rec, stride, s); break;
    case 3: launch_enc<3, ENC>(V, rows, D, M, d, mu, rec, stride, s); break;
    case 4: launch_enc<4, ENC>(V, rows, D, M, d, mu, rec, stride, s); break;
    case 5: launch_enc<5, ENC>(V, rows, D, M, d, mu, rec, stride, s); break;
    case 6: launch_enc<6, ENC>(V, rows, D, M, d, mu, rec, stride, s); break;
    case 7: launch_enc<7, ENC>(V, rows, D, M, d, mu, rec, stride, s); break;
    default: launch_enc<8, ENC>(V, rows, D, M, d, mu, rec, stride, s); break;
  }
}

}  // namespace

int launch_project_grouped(const StepHeader *hdr, const IndexView *subs, int max_tiles, int d,
                           int D, hipStream_t stream) {
  if (d < 1 || d > 1024) LV_FAIL(LV_EUNSUPPORTED, "batched projection needs d <= 1024");
  unsigned waves = 0, yblocks = 0;
  col_layout(d, &waves, &yblocks);
  hipLaunchKernelGGL(project_grouped_kernel, dim3((unsigned)max_tiles, yblocks), dim3(64 * waves),
                     0, stream, hdr, subs, D, d);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

int launch_project(const float *V, int64_t rows, int32_t D, const uint16_t *M, int32_t d,
                   float *out, hipStream_t stream) {
  if (rows == 0) return LV_OK;
  if ((rows + 255) / 256 > 0x7FFFFFFF) LV_FAIL(LV_EINVAL, "too many rows");
  if (rows <= kFewRows) {  // query batches: a wavefront per 32 x 32 output tile
    unsigned waves = 0, yblocks = 0;
    col_layout(d, &waves, &yblocks);
    hipLaunchKernelGGL(project_cols_kernel, dim3((unsigned)((rows + 31) / 32), yblocks),
                       dim3(64 * waves), 0, stream, V, rows, D, M, d, out);
    LV_CHECK_LAUNCH();
    return LV_OK;
  }
  for (int32_t col0 = 0; col0 < d; col0 += 256) {
    const int nt = ((d - col0) + 31) / 32;
    switch (nt > 8 ? 8 : nt) {
      case 1: launch_nt<1>(V, rows, D, M, d, col0, out, stream); break;
      case 2: launch_nt<2>(V, rows, D, M, d, col0, out, stream); break;
      case 3: launch_nt<3>(V, rows, D, M, d, col0, out, stream); break;
      case 4: launch_nt<4>(V, rows, D, M, d, col0, out, stream); break;
      case 5: launch_nt<5>(V, rows, D, M, d, col0, out, stream); break;
      case 6: launch_nt<6>(V, rows, D, M, d, col0, out, stream); break;
      case 7: launch_nt<7>(V, rows, D, M, d, col0, out, stream); break;
      default: launch_nt<8>(V, rows, D, M, d, col0, out, stream); break;
    }
    LV_CHECK_LAUNCH();
  }
  return LV_OK;
}

}  // namespace lv

extern "C" int lv_project(const float *V, int64_t rows, int32_t D, const uint16_t *M, int32_t d,
                          float *out, void *stream) {
  lv::clear_error();
  if (rows < 0) LV_FAIL(LV_EINVAL, "rows must be >= 0");
  if (D < 8 || D % 8 != 0) LV_FAIL(LV_EINVAL, "D must be a positive multiple of 8 (got %d)", D);
  if (d < 1 || d > 1024) LV_FAIL(LV_EINVAL, "d must be in [1, 1024] (got %d)", d);
  if (rows > 0 && (!V || !M || !out)) LV_FAIL(LV_EINVAL, "NULL pointer");
  return lv::launch_project(V, rows, D, M, d, out, static_cast<hipStream_t>(stream));
}

extern "C" int lv_project_encode(const float *V, int64_t rows, int32_t D, const uint16_t *M,
                                 int32_t d, const float *mu, int32_t bits, void *records,
                                 int32_t record_stride, void *stream) {
  lv::clear_error();
  if (rows < 0) LV_FAIL(LV_EINVAL, "rows must be >= 0");
  if (D < 8 || D % 8 != 0) LV_FAIL(LV_EINVAL, "D must be a positive multiple of 8 (got %d)", D);
  if (d < 8 || d > 256 || d % 8 != 0)
    LV_FAIL(LV_EINVAL, "d must be a multiple of 8 in [8, 256] (got %d)", d);
  if (bits != 4 && bits != 8) LV_FAIL(LV_EINVAL, "bits must be 4 or 8 (got %d)", bits);
  if (record_stride < d * bits / 8 + 8 || record_stride % 4 != 0)
    LV_FAIL(LV_EINVAL, "record_stride %d too small or not a multiple of 4", record_stride);
  if (rows > 0 && (!V || !M || !mu || !records)) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (rows == 0) return LV_OK;
  if ((rows + 255) / 256 > 0x7FFFFFFF) LV_FAIL(LV_EINVAL, "too many rows");
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char *rec = static_cast<unsigned char *>(records);
  if (bits == 8)
    lv::launch_enc_bits<8>(V, rows, D, M, d, mu, rec, record_stride, s);
  else
    lv::launch_enc_bits<4>(V, rows, D, M, d, mu, rec, record_stride, s);
  LV_CHECK_LAUNCH();
  return LV_OK;
}
