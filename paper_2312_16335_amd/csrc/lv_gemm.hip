// General matrix product on the gfx950 matrix cores for the projection-loss
// kernels: C[M][N] = alpha * sum_k a(m, k) b(n, k) + beta * C, float32 in
// memory, operands rounded to bfloat16 when staged, float32 accumulation.
//
// Each operand is either "k-contiguous" (a(m, k) at A[m * lda + k]) or
// "m-contiguous" (a(m, k) at A[k * lda + m]); the staging step writes both
// kinds into LDS as [row][k] tiles so the MFMA operand reads are 16-byte
// vector loads.  Tile 128 x 128 per 256-thread workgroup, each wavefront a
// 64 x 64 quadrant (2 x 2 tiles of 32 x 32x16 MFMAs), two LDS buffers.
//
// Kernels: when both operands allow 16-byte loads (aligned pointers,
// leading dimensions multiples of 4 floats), gemm_vec_kernel walks K in
// steps of 64 and keeps the next tile's float32 operands in registers while
// the current tile is multiplied (one barrier per step), with float4 loads
// for both operand layouts; gemm_tile_kernel (below) takes large products on
// 256 x 256 tiles and the split-precision ones; otherwise gemm_kernel stages
// element by element in steps of 32.  The vector and tile kernels also serve
// two independent products in one launch (gemm_pair), the split-precision
// tile kernel a second K segment (C = A B^T + A2 B2^T), and the large tile
// operands already held as bfloat16 (lv_gemm_bf16).
//
// Split precision (GemmArgs::split): each float32 operand x is written as
// hi + lo with hi = bf16(x) and lo = bf16(x - hi) (x - hi is exact in
// float32), and the product is accumulated as hi*hi + hi*lo + lo*hi in three
// passes over K through the same LDS tiles (the lo*lo term is below 2^-16 of
// the product).  The relative error per operand falls from about 2^-9 to
// about 2^-17, at three times the matrix-core work; products whose result
// cancels (a difference of nearly equal products) need it.
#include <algorithm>
#include <type_traits>

#include "lv_common.h"
#include "lv_gemm.h"

namespace lv {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(4))) unsigned int u32x4;

constexpr int BM = 128, BN = 128, BK = 32;
constexpr int LDK = BK + 8;  // padded row (bf16 elements) against LDS bank conflicts

// The second product of a pair run in one launch: workgroups with
// blockIdx.z >= z1 compute it (z1 = gridDim.z: no second product).
struct Second {
  GemmArgs g;
  int z1;
  int sps;
  float *part;
};

__device__ __forceinline__ uint16_t bf16_bits(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// bfloat16 bits of x (LO = false) or of the remainder x - bf16(x) (LO = true).
template <bool LO>
__device__ __forceinline__ uint16_t bf16_part(float x) {
  if constexpr (LO) {
    const float hi = __uint_as_float((uint32_t)bf16_bits(x) << 16);
    return bf16_bits(x - hi);
  } else {
    return bf16_bits(x);
  }
}

// Stage a BM x BK tile of operand X (rows r0.., k k0..) into S[row][k].
template <bool KCONT, bool LO = false>
__device__ __forceinline__ void stage(const float *__restrict__ X, int64_t ld, int rows,
                                      int kdim, int r0, int k0, uint16_t *S, int tid) {
  if constexpr (KCONT) {
    // thread: row tid / 2, 16 consecutive k at (tid % 2) * 16
    const int r = tid >> 1;
    const int kk = (tid & 1) * 16;
    const int gr = r0 + r;
    uint16_t v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int gk = k0 + kk + i;
      v[i] = (gr < rows && gk < kdim) ? bf16_part<LO>(X[(int64_t)gr * ld + gk]) : (uint16_t)0;
    }
    uint4 *dst = reinterpret_cast<uint4 *>(S + r * LDK + kk);
    uint32_t w[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) w[i] = (uint32_t)v[2 * i] | ((uint32_t)v[2 * i + 1] << 16);
    dst[0] = make_uint4(w[0], w[1], w[2], w[3]);
    dst[1] = make_uint4(w[4], w[5], w[6], w[7]);
  } else {
    // thread: k row tid / 8, 16 consecutive rows at (tid % 8) * 16
    const int kk = tid >> 3;
    const int rr = (tid & 7) * 16;
    const int gk = k0 + kk;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int gr = r0 + rr + i;
      S[(rr + i) * LDK + kk] =
          (gr < rows && gk < kdim) ? bf16_part<LO>(X[(int64_t)gk * ld + gr]) : (uint16_t)0;
    }
  }
}

// One pass over K of the product of the (LA, LB) parts of the operands,
// accumulated into acc.
template <bool AK, bool BKC, bool LA, bool LB>
__device__ __forceinline__ void gemm_pass(const GemmArgs &g, uint16_t (*As)[BM * LDK],
                                          uint16_t (*Bs)[BN * LDK], int m0, int n0, int wm,
                                          int wn, int tid, f32x16 (&acc)[2][2]) {
  const int lane = tid & 63;
  const int nk = (g.K + BK - 1) / BK;
  stage<AK, LA>(g.A, g.lda, g.M, g.K, m0, 0, As[0], tid);
  stage<BKC, LB>(g.B, g.ldb, g.N, g.K, n0, 0, Bs[0], tid);
  __syncthreads();
  const int r = lane & 31, kh = lane >> 5;
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    if (t + 1 < nk) {
      stage<AK, LA>(g.A, g.lda, g.M, g.K, m0, (t + 1) * BK, As[cur ^ 1], tid);
      stage<BKC, LB>(g.B, g.ldb, g.N, g.K, n0, (t + 1) * BK, Bs[cur ^ 1], tid);
    }
#pragma unroll
    for (int ks = 0; ks < BK; ks += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const u32x4 wa =
            *reinterpret_cast<const u32x4 *>(&As[cur][(wm + 32 * i + r) * LDK + ks + 8 * kh]);
        a[i] = __builtin_bit_cast(bf16x8, wa);
        const u32x4 wb =
            *reinterpret_cast<const u32x4 *>(&Bs[cur][(wn + 32 * i + r) * LDK + ks + 8 * kh]);
        b[i] = __builtin_bit_cast(bf16x8, wb);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
}

template <bool AK, bool BKC, bool SPLIT>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs g) {
  __shared__ __align__(16) uint16_t As[2][BM * LDK];
  __shared__ __align__(16) uint16_t Bs[2][BN * LDK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
  gemm_pass<AK, BKC, false, false>(g, As, Bs, m0, n0, wm, wn, tid, acc);
  if constexpr (SPLIT) {
    gemm_pass<AK, BKC, false, true>(g, As, Bs, m0, n0, wm, wn, tid, acc);
    gemm_pass<AK, BKC, true, false>(g, As, Bs, m0, n0, wm, wn, tid, acc);
  }
  const int r = lane & 31, kh = lane >> 5;
  // accumulator: lane holds column (lane % 32), register e holds row
  // 8 * (e / 4) + 4 * (lane / 32) + (e % 4) of its 32 x 32 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + 32 * j + r;
      if (col >= g.N) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = m0 + wm + 32 * i + 8 * (e >> 2) + 4 * kh + (e & 3);
        if (row >= g.M) continue;
        float *c = g.C + (int64_t)row * g.ldc + col;
        const float v = g.alpha * acc[i][j][e];
        *c = g.beta == 0.f ? v : v + g.beta * *c;
      }
    }
}

// ---- vector-load kernel

constexpr int VK = 64;       // K per step
constexpr int VLD = VK + 8;  // LDS row (bf16 elements): 144 bytes, 16-byte aligned rows

// The float32 values one thread stages for one operand in one step.
struct Frag {
  float4 v[8];
};

__device__ __forceinline__ float4 load4(const float *p, bool all, bool e0, bool e1, bool e2,
                                        bool e3) {
  if (all) return *reinterpret_cast<const float4 *>(p);
  return make_float4(e0 ? p[0] : 0.f, e1 ? p[1] : 0.f, e2 ? p[2] : 0.f, e3 ? p[3] : 0.f);
}

// Global -> registers.  k-contiguous: thread row tid / 2, 32 consecutive k at
// (tid % 2) * 32.  m-contiguous (memory rows are k): thread k rows 2 (tid / 8)
// and 2 (tid / 8) + 1, 16 consecutive m at (tid % 8) * 16.
template <bool KCONT>
__device__ __forceinline__ void vload(const float *__restrict__ X, int64_t ld, int rows, int kdim,
                                      int r0, int k0, Frag &f, int tid) {
  if constexpr (KCONT) {
    const int r = tid >> 1, kk = (tid & 1) * 32;
    const int gr = r0 + r;
    const bool rok = gr < rows;
    const float *p = X + (int64_t)(rok ? gr : 0) * ld + k0 + kk;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int gk = k0 + kk + 4 * i;
      f.v[i] = load4(p + 4 * i, rok && gk + 3 < kdim, rok && gk < kdim, rok && gk + 1 < kdim,
                     rok && gk + 2 < kdim, false);
    }
  } else {
    const int k = 2 * (tid >> 3), mm = (tid & 7) * 16;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int gk = k0 + k + h;
      const bool kok = gk < kdim;
      const float *p = X + (int64_t)(kok ? gk : 0) * ld + r0 + mm;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gm = r0 + mm + 4 * i;
        f.v[4 * h + i] = load4(p + 4 * i, kok && gm + 3 < rows, kok && gm < rows,
                               kok && gm + 1 < rows, kok && gm + 2 < rows, false);
      }
    }
  }
}

// Two floats to bfloat16 (round to nearest even) in one conversion
// instruction; LO: the remainders x - bf16(x) instead (exact in float32).
template <bool LO = false>
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
  bf16x2 h = {(__bf16)lo, (__bf16)hi};
  if constexpr (LO) {
    h = bf16x2{(__bf16)(lo - (float)h[0]), (__bf16)(hi - (float)h[1])};
  }
  return __builtin_bit_cast(uint32_t, h);
}

// Registers -> LDS tile S[row][k] (bfloat16; LO: the remainders' bfloat16).
template <bool KCONT, bool LO = false>
__device__ __forceinline__ void vstore(const Frag &f, uint16_t *S, int tid) {
  if constexpr (KCONT) {
    const int r = tid >> 1, kk = (tid & 1) * 32;
    uint4 *dst = reinterpret_cast<uint4 *>(S + r * VLD + kk);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 a = f.v[2 * i], b = f.v[2 * i + 1];
      dst[i] = make_uint4(pack_bf16<LO>(a.x, a.y), pack_bf16<LO>(a.z, a.w),
                          pack_bf16<LO>(b.x, b.y), pack_bf16<LO>(b.z, b.w));
    }
  } else {
    const int k = 2 * (tid >> 3), mm = (tid & 7) * 16;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float4 a = f.v[i], b = f.v[4 + i];  // rows k and k + 1, m = mm + 4i ..
      uint32_t *d = reinterpret_cast<uint32_t *>(S + (mm + 4 * i) * VLD + k);
      d[0] = pack_bf16<LO>(a.x, b.x);
      d[VLD / 2] = pack_bf16<LO>(a.y, b.y);
      d[VLD] = pack_bf16<LO>(a.z, b.z);
      d[3 * VLD / 2] = pack_bf16<LO>(a.w, b.w);
    }
  }
}

// One pass over steps [t0, t0 + nk) of K of the product of the (LA, LB)
// parts of the operands, accumulated into acc.
template <bool AK, bool BKC, bool LA, bool LB>
__device__ __forceinline__ void vec_pass(const GemmArgs &g, uint16_t (*As)[BM * VLD],
                                         uint16_t (*Bs)[BN * VLD], int m0, int n0, int wm,
                                         int wn, int t0, int nk, int tid, f32x16 (&acc)[2][2]) {
  const int lane = tid & 63;
  Frag fa, fb;
  vload<AK>(g.A, g.lda, g.M, g.K, m0, t0 * VK, fa, tid);
  vload<BKC>(g.B, g.ldb, g.N, g.K, n0, t0 * VK, fb, tid);
  vstore<AK, LA>(fa, As[0], tid);
  vstore<BKC, LB>(fb, Bs[0], tid);
  __syncthreads();
  const int r = lane & 31, kh = lane >> 5;
  for (int t = 0; t < nk; ++t) {
    const int cur = t & 1;
    const bool more = t + 1 < nk;
    if (more) {  // next step's operands in flight during this step's products
      vload<AK>(g.A, g.lda, g.M, g.K, m0, (t0 + t + 1) * VK, fa, tid);
      vload<BKC>(g.B, g.ldb, g.N, g.K, n0, (t0 + t + 1) * VK, fb, tid);
    }
#pragma unroll
    for (int ks = 0; ks < VK; ks += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        a[i] = __builtin_bit_cast(
            bf16x8,
            *reinterpret_cast<const u32x4 *>(&As[cur][(wm + 32 * i + r) * VLD + ks + 8 * kh]));
        b[i] = __builtin_bit_cast(
            bf16x8,
            *reinterpret_cast<const u32x4 *>(&Bs[cur][(wn + 32 * i + r) * VLD + ks + 8 * kh]));
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {  // the other buffer was last read before the previous barrier
      vstore<AK, LA>(fa, As[cur ^ 1], tid);
      vstore<BKC, LB>(fb, Bs[cur ^ 1], tid);
    }
    __syncthreads();
  }
}

// Split over K (grid z): part z covers steps [z * sps, (z + 1) * sps) and,
// when `part` is set, writes alpha times its partial product to
// part[z][M][N]; otherwise the whole K range goes to C.  Workgroups with
// blockIdx.z >= sec.z1 compute the second product of a pair (its part
// blockIdx.z - sec.z1); those past the output tiles of their product exit.
template <bool AK, bool BKC, bool SPLIT>
__global__ __launch_bounds__(256) void gemm_vec_kernel(GemmArgs g0, int sps0, float *part0,
                                                       Second sec) {
  __shared__ __align__(16) uint16_t As[2][BM * VLD];
  __shared__ __align__(16) uint16_t Bs[2][BN * VLD];
  const bool two = (int)blockIdx.z >= sec.z1;
  const GemmArgs g = two ? sec.g : g0;
  const int sps = two ? sec.sps : sps0;
  float *const part = two ? sec.part : part0;
  const int z = two ? (int)blockIdx.z - sec.z1 : (int)blockIdx.z;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  if (m0 >= g.M || n0 >= g.N) return;  // (whole workgroup)
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  const int nk_all = (g.K + VK - 1) / VK;
  const int t0 = z * sps;
  const int nk = (t0 + sps < nk_all ? t0 + sps : nk_all) - t0;  // steps of this part
  vec_pass<AK, BKC, false, false>(g, As, Bs, m0, n0, wm, wn, t0, nk, tid, acc);
  if constexpr (SPLIT) {
    vec_pass<AK, BKC, false, true>(g, As, Bs, m0, n0, wm, wn, t0, nk, tid, acc);
    vec_pass<AK, BKC, true, false>(g, As, Bs, m0, n0, wm, wn, t0, nk, tid, acc);
  }
  const int r = lane & 31, kh = lane >> 5;
  float *pz = part ? part + (int64_t)z * g.M * g.N : nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + 32 * j + r;
      if (col >= g.N) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = m0 + wm + 32 * i + 8 * (e >> 2) + 4 * kh + (e & 3);
        if (row >= g.M) continue;
        const float v = g.alpha * acc[i][j][e];
        if (pz) {
          pz[(int64_t)row * g.N + col] = v;
        } else {
          float *c = g.C + (int64_t)row * g.ldc + col;
          *c = g.beta == 0.f ? v : v + g.beta * *c;
        }
      }
    }
}

// ---- tiled kernel: TBM x TBN output tile per workgroup of WM x WN
// wavefronts (each a (TBM / WM) x (TBN / WN) block of 32 x 32 MFMA tiles),
// K steps of TK, two LDS buffers and one barrier per step, and the operands
// of the next two steps in flight in registers (float32, or bfloat16 with
// BF) while the current step's products run.  Whole tiles (FULL: M, N multiples of the tile and K
// of TK) load with plain 16-byte loads and no edge tests.
// SPLIT: both parts of every operand (hi, lo) are staged in the same step
// and each fragment pair takes the three products hi*hi, hi*lo, lo*hi, so
// the operands are read and converted once (not once per part).
constexpr int TK = 32;
// LDS tiles: rows of TK bfloat16 (64 bytes, four 16-byte chunks), chunk c of
// row r stored at chunk c ^ ((r / 4) % 4): the 16-byte reads of a fragment
// (sixteen rows, one chunk) and the row writes (four rows, four chunks each)
// then touch distinct banks of a 256-byte bank line.
constexpr int TLD = TK;

__device__ __forceinline__ int tswz(int r, int c) { return r * TLD + 8 * (c ^ ((r >> 2) & 3)); }

template <int ROWS, int THREADS, bool KCONT>
struct TileFrag {
  // float4 pieces of a ROWS x TK tile per thread
  static constexpr int kPer = ROWS * TK / 4 / THREADS;
  float4 v[kPer];
};

// bfloat16 operands in memory (k-contiguous): 16-byte pieces of 8 k per
// thread, unit u = row u / 4, k 8 (u % 4) (the float32 path's units).
template <int ROWS, int THREADS>
struct TileFrag16 {
  static constexpr int kPer = ROWS * TK / 8 / THREADS;
  u32x4 v[kPer];
};

template <int ROWS, int THREADS, bool FULL>
__device__ __forceinline__ void tload16(const uint16_t *__restrict__ X, int64_t ld, int rows,
                                        int kdim, int r0, int k0, TileFrag16<ROWS, THREADS> &f,
                                        int tid) {
#pragma unroll
  for (int j = 0; j < TileFrag16<ROWS, THREADS>::kPer; ++j) {
    const int u = tid + THREADS * j;
    const int gr = r0 + (u >> 2), gk = k0 + 8 * (u & 3);
    if (FULL || (gr < rows && gk + 7 < kdim)) {
      f.v[j] = *reinterpret_cast<const u32x4 *>(X + (int64_t)gr * ld + gk);
    } else {  // edge: element by element, zeros past the matrix
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t lo = gr < rows && gk + 2 * e < kdim ? X[(int64_t)gr * ld + gk + 2 * e] : 0u;
        const uint32_t hi =
            gr < rows && gk + 2 * e + 1 < kdim ? X[(int64_t)gr * ld + gk + 2 * e + 1] : 0u;
        w[e] = lo | (hi << 16);
      }
      f.v[j] = u32x4{w[0], w[1], w[2], w[3]};
    }
  }
}

template <int ROWS, int THREADS>
__device__ __forceinline__ void tstore16(const TileFrag16<ROWS, THREADS> &f, uint16_t *S,
                                         int tid) {
#pragma unroll
  for (int j = 0; j < TileFrag16<ROWS, THREADS>::kPer; ++j) {
    const int u = tid + THREADS * j;
    *reinterpret_cast<u32x4 *>(S + tswz(u >> 2, u & 3)) = f.v[j];
  }
}

// Global -> registers.  k-contiguous: unit u (row u / 4, k 8 (u % 4) ..), two
// pieces per unit, so four consecutive threads read one row's 128 bytes.
// m-contiguous: unit u (k rows 2 kp and 2 kp + 1, m 4 mq ..), two pieces.
template <int ROWS, int THREADS, bool KCONT, bool FULL>
__device__ __forceinline__ void tload(const float *__restrict__ X, int64_t ld, int rows,
                                      int kdim, int r0, int k0,
                                      TileFrag<ROWS, THREADS, KCONT> &f, int tid) {
  constexpr int P = TileFrag<ROWS, THREADS, KCONT>::kPer;
  if constexpr (FULL) {  // whole tiles: plain 16-byte loads, no edge tests
    if constexpr (KCONT) {
#pragma unroll
      for (int j = 0; j < P / 2; ++j) {
        const int u = tid + THREADS * j;
        const float *p = X + (int64_t)(r0 + (u >> 2)) * ld + k0 + 8 * (u & 3);
        f.v[2 * j] = *reinterpret_cast<const float4 *>(p);
        f.v[2 * j + 1] = *reinterpret_cast<const float4 *>(p + 4);
      }
    } else {
      constexpr int MQ = ROWS / 4;
#pragma unroll
      for (int j = 0; j < P / 2; ++j) {
        const int u = tid + THREADS * j;
        const int kp = u / MQ, mq = u % MQ;
        const float *p = X + (int64_t)(k0 + 2 * kp) * ld + r0 + 4 * mq;
        f.v[2 * j] = *reinterpret_cast<const float4 *>(p);
        f.v[2 * j + 1] = *reinterpret_cast<const float4 *>(p + ld);
      }
    }
    return;
  }
  if constexpr (KCONT) {
#pragma unroll
    for (int j = 0; j < P / 2; ++j) {
      const int u = tid + THREADS * j;
      const int gr = r0 + (u >> 2);
      const bool rok = gr < rows;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int gk = k0 + 8 * (u & 3) + 4 * h;
        const float *p = X + (int64_t)(rok ? gr : 0) * ld + (gk < kdim ? gk : 0);
        f.v[2 * j + h] = load4(p, rok && gk + 3 < kdim, rok && gk < kdim, rok && gk + 1 < kdim,
                               rok && gk + 2 < kdim, false);
      }
    }
  } else {
    constexpr int MQ = ROWS / 4;  // float4 pieces along m
#pragma unroll
    for (int j = 0; j < P / 2; ++j) {
      const int u = tid + THREADS * j;
      const int kp = u / MQ, mq = u % MQ;
      const int gm = r0 + 4 * mq;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int gk = k0 + 2 * kp + h;
        const bool kok = gk < kdim;
        const float *p = X + (int64_t)(kok ? gk : 0) * ld + (gm < rows ? gm : 0);
        f.v[2 * j + h] = load4(p, kok && gm + 3 < rows, kok && gm < rows, kok && gm + 1 < rows,
                               kok && gm + 2 < rows, false);
      }
    }
  }
}

// Registers -> LDS tile S[row][k] (bfloat16 hi part, or the remainders' bf16).
template <int ROWS, int THREADS, bool KCONT, bool LO>
__device__ __forceinline__ void tstore(const TileFrag<ROWS, THREADS, KCONT> &f, uint16_t *S,
                                       int tid) {
  constexpr int P = TileFrag<ROWS, THREADS, KCONT>::kPer;
  if constexpr (KCONT) {
#pragma unroll
    for (int j = 0; j < P / 2; ++j) {
      const int u = tid + THREADS * j;
      const float4 a = f.v[2 * j], b = f.v[2 * j + 1];
      *reinterpret_cast<uint4 *>(S + tswz(u >> 2, u & 3)) =
          make_uint4(pack_bf16<LO>(a.x, a.y), pack_bf16<LO>(a.z, a.w), pack_bf16<LO>(b.x, b.y),
                     pack_bf16<LO>(b.z, b.w));
    }
  } else {
    constexpr int MQ = ROWS / 4;
#pragma unroll
    for (int j = 0; j < P / 2; ++j) {
      const int u = tid + THREADS * j;
      const int kp = u / MQ, mq = u % MQ;
      const float4 a = f.v[2 * j], b = f.v[2 * j + 1];  // k rows 2 kp and 2 kp + 1
      const int c = (2 * kp) >> 3, w = (2 * kp) & 7;   // chunk and place of the pair
      const int m = 4 * mq;
      *reinterpret_cast<uint32_t *>(S + tswz(m, c) + w) = pack_bf16<LO>(a.x, b.x);
      *reinterpret_cast<uint32_t *>(S + tswz(m + 1, c) + w) = pack_bf16<LO>(a.y, b.y);
      *reinterpret_cast<uint32_t *>(S + tswz(m + 2, c) + w) = pack_bf16<LO>(a.z, b.z);
      *reinterpret_cast<uint32_t *>(S + tswz(m + 3, c) + w) = pack_bf16<LO>(a.w, b.w);
    }
  }
}

// (pairs of products and split over K as for gemm_vec_kernel)
// BF: A and B hold bfloat16 bits (k-contiguous, no split precision)
template <int TBM, int TBN, int WM, int WN, bool AK, bool BKC, bool SPLIT, bool FULL,
          bool BF = false>
__global__ __launch_bounds__(64 * WM * WN) void gemm_tile_kernel(GemmArgs g0, int sps0,
                                                                  float *part0, Second sec) {
  static_assert(!BF || (AK && BKC && !SPLIT), "bfloat16 operands: k-contiguous, one part");
  constexpr int THREADS = 64 * WM * WN;
  constexpr int NP = SPLIT ? 2 : 1;   // operand parts staged per step
  constexpr int IM = TBM / WM / 32;   // MFMA tiles per wavefront along m
  constexpr int JN = TBN / WN / 32;   // and along n
  constexpr int SA = TBM * TLD, SB = TBN * TLD;
  __shared__ __align__(16) uint16_t tsm[2 * NP * (SA + SB)];
  uint16_t *As = tsm;                       // [2][NP][SA]
  uint16_t *Bs = tsm + 2 * NP * SA;         // [2][NP][SB]
  const bool two = (int)blockIdx.z >= sec.z1;
  const GemmArgs g = two ? sec.g : g0;
  const int sps = two ? sec.sps : sps0;
  float *const part = two ? sec.part : part0;
  const int z = two ? (int)blockIdx.z - sec.z1 : (int)blockIdx.z;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int m0 = blockIdx.y * TBM, n0 = blockIdx.x * TBN;
  if (m0 >= g.M || n0 >= g.N) return;  // (whole workgroup)
  const int wm = (wave / WN) * (TBM / WM), wn = (wave % WN) * (TBN / WN);
  const int r = lane & 31, kh = lane >> 5;
  f32x16 acc[IM][JN];
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;

  // steps of the first K segment, then of the second (A2, B2; none if K2 = 0;
  // split-precision instances only, the others take one segment)
  const int nk1 = (g.K + TK - 1) / TK;
  const int nk_all = nk1 + (SPLIT ? (g.K2 + TK - 1) / TK : 0);
  const int t0 = z * sps;
  const int nk = (t0 + sps < nk_all ? t0 + sps : nk_all) - t0;
  // two register sets: at step t the operands of step t + 1 (loaded during
  // step t - 1) go to LDS while those of step t + 2 are in flight
  using FragA = std::conditional_t<BF, TileFrag16<TBM, THREADS>, TileFrag<TBM, THREADS, AK>>;
  using FragB = std::conditional_t<BF, TileFrag16<TBN, THREADS>, TileFrag<TBN, THREADS, BKC>>;
  FragA fa[2];
  FragB fb[2];
  auto load = [&](int t, int q) {
    const int T = t0 + t;
    if constexpr (BF) {
      tload16<TBM, THREADS, FULL>(reinterpret_cast<const uint16_t *>(g.A), g.lda, g.M, g.K, m0,
                                  T * TK, fa[q], tid);
      tload16<TBN, THREADS, FULL>(reinterpret_cast<const uint16_t *>(g.B), g.ldb, g.N, g.K, n0,
                                  T * TK, fb[q], tid);
    } else if constexpr (SPLIT) {
      const bool s2 = T >= nk1;  // uniform: the segment of this step
      const int k = (s2 ? T - nk1 : T) * TK, kseg = s2 ? g.K2 : g.K;
      tload<TBM, THREADS, AK, FULL>(s2 ? g.A2 : g.A, s2 ? g.lda2 : g.lda, g.M, kseg, m0, k,
                                    fa[q], tid);
      tload<TBN, THREADS, BKC, FULL>(s2 ? g.B2 : g.B, s2 ? g.ldb2 : g.ldb, g.N, kseg, n0, k,
                                     fb[q], tid);
    } else {
      tload<TBM, THREADS, AK, FULL>(g.A, g.lda, g.M, g.K, m0, T * TK, fa[q], tid);
      tload<TBN, THREADS, BKC, FULL>(g.B, g.ldb, g.N, g.K, n0, T * TK, fb[q], tid);
    }
  };
  auto put = [&](int b, int q) {
    if constexpr (BF) {
      tstore16<TBM, THREADS>(fa[q], As + b * SA, tid);
      tstore16<TBN, THREADS>(fb[q], Bs + b * SB, tid);
    } else {
      tstore<TBM, THREADS, AK, false>(fa[q], As + (b * NP) * SA, tid);
      tstore<TBN, THREADS, BKC, false>(fb[q], Bs + (b * NP) * SB, tid);
      if constexpr (SPLIT) {
        tstore<TBM, THREADS, AK, true>(fa[q], As + (b * NP + 1) * SA, tid);
        tstore<TBN, THREADS, BKC, true>(fb[q], Bs + (b * NP + 1) * SB, tid);
      }
    }
  };
  auto compute = [&](int cur) {
    const uint16_t *ac = As + (cur * NP) * SA;
    const uint16_t *bc = Bs + (cur * NP) * SB;
#pragma unroll
    for (int ks = 0; ks < TK; ks += 16) {
      bf16x8 a[NP][IM], b[NP][JN];
#pragma unroll
      for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int i = 0; i < IM; ++i)
          a[q][i] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(
                                                   ac + q * SA + tswz(wm + 32 * i + r,
                                                                      (ks >> 3) + kh)));
#pragma unroll
        for (int j = 0; j < JN; ++j)
          b[q][j] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4 *>(
                                                   bc + q * SB + tswz(wn + 32 * j + r,
                                                                      (ks >> 3) + kh)));
      }
#pragma unroll
      for (int i = 0; i < IM; ++i)
#pragma unroll
        for (int j = 0; j < JN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[0][j], acc[i][j], 0, 0, 0);
          if constexpr (SPLIT) {
            acc[i][j] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[0][i], b[1][j], acc[i][j], 0, 0, 0);
            acc[i][j] =
                __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[1][i], b[0][j], acc[i][j], 0, 0, 0);
          }
        }
    }
  };
  // step t: compute from LDS buffer t % 2, operands of step t + 1 from
  // register set (t + 1) % 2 into the other buffer, step t + 2 into set t % 2
  // (scheduling barriers keep the loads in program order, so that the wait
  // before storing a set covers only that set's loads, not the newer set's)
  // The loads are unconditional (past the last step they fetch the last step
  // again, unused) so that every path has the same loads in flight and the
  // wait before a store counts only the older set.
  auto step = [&](int t, int q) {  // q = t % 2 (a constant at each call)
    load(t + 2 < nk ? t + 2 : nk - 1, q);
    __builtin_amdgcn_sched_barrier(0);
    compute(q);
    __builtin_amdgcn_sched_barrier(0);
    if (t + 1 < nk) put(q ^ 1, q ^ 1);  // that buffer was last read before the previous barrier
    __syncthreads();
  };
  if (nk > 0) {
    load(0, 0);
    __builtin_amdgcn_sched_barrier(0);
    load(nk > 1 ? 1 : 0, 1);
    __builtin_amdgcn_sched_barrier(0);
    put(0, 0);
  }
  __syncthreads();
  int t = 0;
  for (; t + 1 < nk; t += 2) {
    step(t, 0);
    step(t + 1, 1);
  }
  if (t < nk) step(t, 0);
  float *pz = part ? part + (int64_t)z * g.M * g.N : nullptr;
#pragma unroll
  for (int i = 0; i < IM; ++i)
#pragma unroll
    for (int j = 0; j < JN; ++j) {
      const int col = n0 + wn + 32 * j + r;
      if (col >= g.N) continue;
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int row = m0 + wm + 32 * i + 8 * (e >> 2) + 4 * kh + (e & 3);
        if (row >= g.M) continue;
        const float v = g.alpha * acc[i][j][e];
        if (pz) {
          pz[(int64_t)row * g.N + col] = v;
        } else {
          float *c = g.C + (int64_t)row * g.ldc + col;
          *c = g.beta == 0.f ? v : v + g.beta * *c;
        }
      }
    }
}

// C = sum over z of part[z] (in order z = 0, 1, ...) + beta * C; grid row 1
// does the same for a second product (part1, nz1, g1).
__global__ __launch_bounds__(256) void split_sum_kernel(const float *__restrict__ part0, int nz0,
                                                        GemmArgs g0, const float *part1, int nz1,
                                                        GemmArgs g1) {
  const bool two = blockIdx.y != 0;
  const float *__restrict__ part = two ? part1 : part0;
  const int nz = two ? nz1 : nz0;
  const GemmArgs g = two ? g1 : g0;
  const int64_t mn = (int64_t)g.M * g.N;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < mn;
       i += (int64_t)gridDim.x * 256) {
    float v = part[i];
    for (int z = 1; z < nz; ++z) v += part[z * mn + i];
    float *c = g.C + (i / g.N) * g.ldc + i % g.N;
    *c = g.beta == 0.f ? v : v + g.beta * *c;
  }
}

constexpr int kMaxSplit = 16;

struct VecLaunch {
  const GemmArgs &g;
  dim3 grid;
  int sps;
  float *part;
  hipStream_t s;
  Second sec;
  template <bool AK, bool BKC, bool SPLIT>
  void go() {
    hipLaunchKernelGGL((gemm_vec_kernel<AK, BKC, SPLIT>), grid, dim3(256), 0, s, g, sps, part,
                       sec);
  }
};

template <int TBM, int TBN, int WM, int WN>
struct TileLaunch {
  const GemmArgs &g;
  dim3 grid;
  int sps;
  float *part;
  hipStream_t s;
  bool full;
  Second sec;
  template <bool AK, bool BKC, bool SPLIT>
  void go() {
    // split precision runs on 128 x 128 tiles only (the large tile has no
    // registers left for the second parts)
    if constexpr (!SPLIT || TBM * TBN <= 128 * 128) {
      if (full)
        hipLaunchKernelGGL((gemm_tile_kernel<TBM, TBN, WM, WN, AK, BKC, SPLIT, true>), grid,
                           dim3(64 * WM * WN), 0, s, g, sps, part, sec);
      else
        hipLaunchKernelGGL((gemm_tile_kernel<TBM, TBN, WM, WN, AK, BKC, SPLIT, false>), grid,
                           dim3(64 * WM * WN), 0, s, g, sps, part, sec);
    }
  }
};

struct ElemLaunch {
  const GemmArgs &g;
  dim3 grid;
  hipStream_t s;
  template <bool AK, bool BKC, bool SPLIT>
  void go() {
    hipLaunchKernelGGL((gemm_kernel<AK, BKC, SPLIT>), grid, dim3(256), 0, s, g);
  }
};

// The kernel instance for the operand layouts and precision.
template <class F>
void dispatch_layout(bool ak, bool bk, bool split, F &f) {
  if (split) {
    if (ak && bk) f.template go<true, true, true>();
    else if (ak) f.template go<true, false, true>();
    else if (bk) f.template go<false, true, true>();
    else f.template go<false, false, true>();
  } else {
    if (ak && bk) f.template go<true, true, false>();
    else if (ak) f.template go<true, false, false>();
    else if (bk) f.template go<false, true, false>();
    else f.template go<false, false, false>();
  }
}

bool vec_ok(const float *p, int64_t ld) {
  return (reinterpret_cast<uintptr_t>(p) & 15u) == 0 && ld % 4 == 0;
}

}  // namespace

size_t gemm_split_floats(int64_t M, int64_t N) { return (size_t)kMaxSplit * M * N; }

// Tile of the large-product kernel (no split precision): 256 x 256 per
// workgroup of 8 wavefronts, each 128 x 64; used when it still gives at
// least this many workgroups.
constexpr int kBigTile = 256;
constexpr int kBigTileMinTiles = 128;

namespace {

// How a product runs on the vector-load kernels (no big tile, one K segment
// unless on the tile kernel): the tile grid and the split over K.
struct Plan {
  dim3 grid;  // x: tiles along N, y: along M
  int parts, sps;
  bool full;  // whole tiles and K steps (tile kernel)
};

Plan plan_small(const GemmArgs &g, size_t split_floats, bool have_ws) {
  const bool split = g.split != 0;
  Plan p;
  p.grid = dim3((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM));
  const int tk_steps = (g.K + TK - 1) / TK + (g.K2 + TK - 1) / TK;  // tile kernel steps
  p.full = g.M % BM == 0 && g.N % BN == 0 && g.K % TK == 0 && g.K2 % TK == 0;
  // few output tiles and a long K: split K so that about 128 workgroups run
  const int tiles = (int)(p.grid.x * p.grid.y);
  const int step = split ? TK : VK;  // K per step of the kernel used
  const int nk = split ? tk_steps : (g.K + step - 1) / step;
  const int ktot = g.K + g.K2;
  // (split precision: three products per step, so parts of at least 64 of K,
  // about 256 workgroups in all, and from K = 256 on)
  const int min_k = split ? 256 : 512, part_k = split ? 64 : 256, target = split ? 256 : 128;
  int parts = 1;
  if (have_ws && tiles < 64 && ktot >= min_k) {
    parts = target / tiles;
    if (parts > (ktot + part_k - 1) / part_k) parts = (ktot + part_k - 1) / part_k;
    if (parts > kMaxSplit) parts = kMaxSplit;
    while (parts > 1 && (size_t)parts * g.M * g.N > split_floats) --parts;
  }
  p.sps = nk > 0 ? (nk + parts - 1) / parts : 1;  // steps per part
  p.parts = nk > 0 ? (nk + p.sps - 1) / p.sps : 1;
  return p;
}

bool vec_operands(const GemmArgs &g) {
  return vec_ok(g.A, g.lda) && vec_ok(g.B, g.ldb) &&
         (g.K2 <= 0 || (vec_ok(g.A2, g.lda2) && vec_ok(g.B2, g.ldb2)));
}

// The split sums of up to two products (n of them, part buffers and counts).
void split_sums(int n, const float *p0, int nz0, const GemmArgs &g0, const float *p1, int nz1,
                const GemmArgs &g1, hipStream_t s) {
  const int64_t mn = std::max((int64_t)g0.M * g0.N, n > 1 ? (int64_t)g1.M * g1.N : 0);
  const unsigned blocks = (unsigned)((mn + 255) / 256 < 2048 ? (mn + 255) / 256 : 2048);
  hipLaunchKernelGGL(split_sum_kernel, dim3(blocks, (unsigned)n), dim3(256), 0, s, p0, nz0, g0,
                     p1, nz1, g1);
}

}  // namespace

int gemm(const GemmArgs &g, bool a_kcont, bool b_kcont, hipStream_t s, float *split_ws,
         size_t split_floats) {
  if (g.M <= 0 || g.N <= 0) return LV_OK;
  const bool two = g.K2 > 0;  // a second K segment
  // the two segments as separate products: C = alpha A B^T + beta C, then
  // C += alpha A2 B2^T (the kernels other than the tile kernels)
  auto two_launches = [&]() -> int {
    GemmArgs g1 = g, g2 = g;
    g1.A2 = g1.B2 = nullptr;
    g1.K2 = 0;
    g2.A = g.A2;
    g2.lda = g.lda2;
    g2.B = g.B2;
    g2.ldb = g.ldb2;
    g2.K = g.K2;
    g2.beta = 1.f;
    g2.A2 = g2.B2 = nullptr;
    g2.K2 = 0;
    int rc = gemm(g1, a_kcont, b_kcont, s, split_ws, split_floats);
    return rc != LV_OK ? rc : gemm(g2, a_kcont, b_kcont, s, split_ws, split_floats);
  };
  const dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM));
  if (vec_operands(g)) {
    const bool split = g.split != 0;
    // the second K segment runs in the split-precision tile kernel only
    if (two && !split) return two_launches();
    const int tk_steps = (g.K + TK - 1) / TK + (g.K2 + TK - 1) / TK;  // tile kernel steps
    const bool k_full = g.K % TK == 0 && g.K2 % TK == 0;
    const int big_tiles = ((g.M + kBigTile - 1) / kBigTile) * ((g.N + kBigTile - 1) / kBigTile);
    if (!split && big_tiles >= kBigTileMinTiles) {
      const dim3 gb((unsigned)((g.N + kBigTile - 1) / kBigTile),
                    (unsigned)((g.M + kBigTile - 1) / kBigTile), 1u);
      const bool full = g.M % kBigTile == 0 && g.N % kBigTile == 0 && k_full;
      TileLaunch<kBigTile, kBigTile, 2, 4> f{g, gb, tk_steps > 0 ? tk_steps : 1, nullptr, s,
                                          full, Second{g, 1, 0, nullptr}};
      dispatch_layout(a_kcont, b_kcont, false, f);
      LV_CHECK_LAUNCH();
      return LV_OK;
    }
    const Plan p = plan_small(g, split_floats, split_ws != nullptr);
    float *part = p.parts > 1 ? split_ws : nullptr;
    const dim3 gz(p.grid.x, p.grid.y, (unsigned)p.parts);
    const Second none{g, p.parts, 0, nullptr};
    if (split) {  // both parts staged once per step
      TileLaunch<BM, BN, 2, 2> f{g, gz, p.sps, part, s, p.full, none};
      dispatch_layout(a_kcont, b_kcont, true, f);
    } else {
      VecLaunch f{g, gz, p.sps, part, s, none};
      dispatch_layout(a_kcont, b_kcont, false, f);
    }
    if (part) split_sums(1, part, p.parts, g, nullptr, 0, g, s);
    LV_CHECK_LAUNCH();
    return LV_OK;
  }
  if (two) return two_launches();
  ElemLaunch f{g, grid, s};
  dispatch_layout(a_kcont, b_kcont, g.split != 0, f);
  LV_CHECK_LAUNCH();
  return LV_OK;
}


int gemm_pair(const GemmArgs &g0, const GemmArgs &g1, bool a_kcont, bool b_kcont, hipStream_t s,
              float *split_ws, size_t split_floats) {
  // half of the workspace each (64-float aligned)
  const size_t half = (split_floats / 2) & ~(size_t)63;
  float *ws1 = split_ws ? split_ws + half : nullptr;
  auto separate = [&]() -> int {
    int rc = gemm(g0, a_kcont, b_kcont, s, split_ws, half);
    return rc != LV_OK ? rc : gemm(g1, a_kcont, b_kcont, s, ws1, split_floats - half);
  };
  if (g0.M <= 0 || g0.N <= 0 || g1.M <= 0 || g1.N <= 0) return separate();
  const bool split = g0.split != 0;
  // one launch when both take the small-product path of the same kernel
  const auto big = [](const GemmArgs &g) {
    return ((g.M + kBigTile - 1) / kBigTile) * ((g.N + kBigTile - 1) / kBigTile) >=
           kBigTileMinTiles;
  };
  if ((g1.split != 0) != split || !vec_operands(g0) || !vec_operands(g1) ||
      (!split && (big(g0) || big(g1) || g0.K2 > 0 || g1.K2 > 0)))
    return separate();
  const Plan p0 = plan_small(g0, half, split_ws != nullptr);
  const Plan p1 = plan_small(g1, split_floats - half, split_ws != nullptr);
  float *part0 = p0.parts > 1 ? split_ws : nullptr;
  float *part1 = p1.parts > 1 ? ws1 : nullptr;
  const dim3 gz(std::max(p0.grid.x, p1.grid.x), std::max(p0.grid.y, p1.grid.y),
                (unsigned)(p0.parts + p1.parts));
  const Second sec{g1, p0.parts, p1.sps, part1};
  if (split) {
    TileLaunch<BM, BN, 2, 2> f{g0, gz, p0.sps, part0, s, p0.full && p1.full, sec};
    dispatch_layout(a_kcont, b_kcont, true, f);
  } else {
    VecLaunch f{g0, gz, p0.sps, part0, s, sec};
    dispatch_layout(a_kcont, b_kcont, false, f);
  }
  if (part0 && part1) split_sums(2, part0, p0.parts, g0, part1, p1.parts, g1, s);
  else if (part0) split_sums(1, part0, p0.parts, g0, nullptr, 0, g0, s);
  else if (part1) split_sums(1, part1, p1.parts, g1, nullptr, 0, g1, s);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

}  // namespace lv

namespace {

int gemm_entry(const float *A, int32_t a_kcont, int64_t lda, const float *B, int32_t b_kcont,
               int64_t ldb, float *C, int64_t ldc, int32_t M, int32_t N, int32_t K, float alpha,
               float beta, void *workspace, size_t workspace_bytes, void *stream, int split) {
  lv::clear_error();
  if (M < 0 || N < 0 || K < 0) LV_FAIL(LV_EINVAL, "negative size");
  if ((int64_t)M * N > 0 && (!A || !B || !C)) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (ldc < N || lda < (a_kcont ? K : M) || ldb < (b_kcont ? K : N))
    LV_FAIL(LV_EINVAL, "leading dimension too small");
  lv::GemmArgs g{A, lda, B, ldb, C, ldc, M, N, K, alpha, beta, split};
  if (workspace_bytes > 0 && !workspace) LV_FAIL(LV_EINVAL, "NULL workspace");
  if (workspace && (reinterpret_cast<uintptr_t>(workspace) & 3u))
    LV_FAIL(LV_EINVAL, "workspace not 4-byte aligned");
  return lv::gemm(g, a_kcont != 0, b_kcont != 0, static_cast<hipStream_t>(stream),
                  static_cast<float *>(workspace), workspace ? workspace_bytes / sizeof(float) : 0);
}

}  // namespace

extern "C" int lv_gemm(const float *A, int32_t a_kcont, int64_t lda, const float *B,
                       int32_t b_kcont, int64_t ldb, float *C, int64_t ldc, int32_t M, int32_t N,
                       int32_t K, float alpha, float beta, void *workspace,
                       size_t workspace_bytes, void *stream) {
  return gemm_entry(A, a_kcont, lda, B, b_kcont, ldb, C, ldc, M, N, K, alpha, beta, workspace,
                    workspace_bytes, stream, 0);
}

extern "C" int lv_gemm_split(const float *A, int32_t a_kcont, int64_t lda, const float *B,
                             int32_t b_kcont, int64_t ldb, float *C, int64_t ldc, int32_t M,
                             int32_t N, int32_t K, float alpha, float beta, void *workspace,
                             size_t workspace_bytes, void *stream) {
  return gemm_entry(A, a_kcont, lda, B, b_kcont, ldb, C, ldc, M, N, K, alpha, beta, workspace,
                    workspace_bytes, stream, 1);
}

namespace lv {
namespace {

int gemm_bf16(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return LV_OK;
  const dim3 gb((unsigned)((g.N + kBigTile - 1) / kBigTile),
                (unsigned)((g.M + kBigTile - 1) / kBigTile), 1u);
  const int steps = (g.K + TK - 1) / TK;
  const bool full = g.M % kBigTile == 0 && g.N % kBigTile == 0 && g.K % TK == 0;
  const Second none{g, 1, 0, nullptr};
  if (full)
    hipLaunchKernelGGL((gemm_tile_kernel<kBigTile, kBigTile, 2, 4, true, true, false, true, true>),
                       gb, dim3(512), 0, s, g, steps > 0 ? steps : 1, nullptr, none);
  else
    hipLaunchKernelGGL((gemm_tile_kernel<kBigTile, kBigTile, 2, 4, true, true, false, false, true>),
                       gb, dim3(512), 0, s, g, steps > 0 ? steps : 1, nullptr, none);
  LV_CHECK_LAUNCH();
  return LV_OK;
}

}  // namespace
}  // namespace lv

extern "C" int lv_gemm_bf16(const uint16_t *A, int64_t lda, const uint16_t *B, int64_t ldb,
                            float *C, int64_t ldc, int32_t M, int32_t N, int32_t K, float alpha,
                            float beta, void *stream) {
  lv::clear_error();
  if (M < 0 || N < 0 || K < 0) LV_FAIL(LV_EINVAL, "negative size");
  if ((int64_t)M * N == 0) return LV_OK;
  if (!C || (K > 0 && (!A || !B))) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (ldc < N || lda < K || ldb < K) LV_FAIL(LV_EINVAL, "leading dimension too small");
  if (lda % 8 != 0 || ldb % 8 != 0 || (reinterpret_cast<uintptr_t>(A) & 15u) ||
      (reinterpret_cast<uintptr_t>(B) & 15u))
    LV_FAIL(LV_EINVAL, "A and B need 16-byte aligned rows (pointers aligned, lda and ldb "
                       "multiples of 8)");
  lv::GemmArgs g{reinterpret_cast<const float *>(A), lda, reinterpret_cast<const float *>(B),
                 ldb, C, ldc, M, N, K, alpha, beta, 0};
  return lv::gemm_bf16(g, static_cast<hipStream_t>(stream));
}

extern "C" size_t lv_gemm_workspace_size(int32_t M, int32_t N) {
  if (M <= 0 || N <= 0) return 0;
  return lv::gemm_split_floats(M, N) * sizeof(float);
}
