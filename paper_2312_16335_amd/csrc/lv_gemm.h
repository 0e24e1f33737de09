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
};

// C = alpha * op(A) op(B)^T + beta * C; a_kcont / b_kcont select whether
// a(m, k) is A[m * lda + k] (true) or A[k * lda + m] (false), same for b(n, k).
int gemm(const GemmArgs &g, bool a_kcont, bool b_kcont, hipStream_t s);

}  // namespace lv
