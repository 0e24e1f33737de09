// Matrix-core matrix product used by the projection-loss kernels.
#pragma once

#include <cstdint>

#include "lv_common.h"

namespace lv {

struct GemmArgs {
  const float *A;
  int64_t lda;
  const float *B;
  int64_t ldb;
  float *C;
  int64_t ldc;
  int32_t M, N, K;
  float alpha, beta;
  int32_t split = 0;  // 1: split-precision operands (hi + lo bfloat16), three passes
  // optional second K segment: C = alpha * (op(A) op(B)^T + op(A2) op(B2)^T)
  // + beta * C, A2 / B2 in the layouts of A / B, K2 columns (0: none)
  const float *A2 = nullptr;
  int64_t lda2 = 0;
  const float *B2 = nullptr;
  int64_t ldb2 = 0;
  int32_t K2 = 0;
};

// C = alpha * op(A) op(B)^T + beta * C; a_kcont / b_kcont select whether
// a(m, k) is A[m * lda + k] (true) or A[k * lda + m] (false), same for b(n, k).
// A second K segment (K2 > 0) runs in the same launch on the split-precision
// tile kernel and as a second product (beta = 1) otherwise.
// With a workspace (split_ws, split_floats floats), a product with few output
// tiles and a long K is split over K: each part writes alpha times its
// partial product to the workspace, and a second kernel adds the parts in a
// fixed order (deterministic) before beta * C.
int gemm(const GemmArgs &g, bool a_kcont, bool b_kcont, hipStream_t s, float *split_ws = nullptr,
         size_t split_floats = 0);
// Two independent products with the same operand layouts and precision, in
// one launch (and one launch of split sums) when both are small products on
// the same kernel, else one after the other; each gets half of the workspace.
// Results are those of two gemm calls with those halves.
int gemm_pair(const GemmArgs &g0, const GemmArgs &g1, bool a_kcont, bool b_kcont, hipStream_t s,
              float *split_ws, size_t split_floats);
// Workspace floats gemm may use for an M x N product split over K.
size_t gemm_split_floats(int64_t M, int64_t N);

}  // namespace lv
