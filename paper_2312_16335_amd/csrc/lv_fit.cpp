// Projection learning on the host in float64 (Sections 2.1-2.4).
//
// * second moments K = sum v v^T (Problem leanvec_efficient), accumulated
//   with one thread per output row so results do not depend on the thread
//   count;
// * a symmetric eigensolver: Householder reduction to tridiagonal form with
//   the orthogonal factor accumulated, then implicit symmetric QR steps with
//   Wilkinson shifts (Golub & Van Loan, Matrix Computations, 8.3);
// * LeanVec-ID: the leading eigenvectors of K_X (Section 2.1);
// * LeanVec-OOD: Frank-Wolfe block coordinate descent (Algorithm 1) with
//   the gradients of Eq. leanvec_gradients and the linear step S = U V^T,
//   computed as the polar factor (C C^T)^{-1/2} C of the d x D gradient;
// * eigenvector search (Algorithm 2) with Brent's bounded minimisation.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <vector>

#include "lv_error.h"
#include "lv_fit.h"

namespace lv {
namespace {

using Mat = std::vector<double>;

// C[MxN] = A[MxK] * B[KxN] (all row-major); op flags transpose A or B.
void gemm(int M, int N, int K, const double *A, bool ta, const double *B, bool tb, double *C) {
#pragma omp parallel for schedule(static)
  for (int i = 0; i < M; ++i) {
    double *c = C + (size_t)i * N;
    for (int j = 0; j < N; ++j) c[j] = 0.0;
    for (int k = 0; k < K; ++k) {
      const double a = ta ? A[(size_t)k * M + i] : A[(size_t)i * K + k];
      if (a == 0.0) continue;
      if (!tb) {
        const double *b = B + (size_t)k * N;
        for (int j = 0; j < N; ++j) c[j] += a * b[j];
      } else {
        for (int j = 0; j < N; ++j) c[j] += a * B[(size_t)j * K + k];
      }
    }
  }
}

double trace_prod(int n, const double *A, const double *B) {  // tr(A B), both n x n
  double t = 0.0;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < n; ++k) t += A[(size_t)i * n + k] * B[(size_t)k * n + i];
  return t;
}

// Symmetric eigen-decomposition of S (n x n).  Returns eigenvalues in w and
// eigenvectors as ROWS of V (V[i] belongs to w[i]), unsorted.
void sym_eig(int n, const double *S, double *w, double *V) {
  Mat A(S, S + (size_t)n * n);
  std::vector<double> e(n > 1 ? n - 1 : 1, 0.0);
  Mat Hv((size_t)n * n, 0.0);  // Householder vectors, row k holds v_k
  std::vector<double> beta(n, 0.0);
  std::vector<double> p(n), wv(n);
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of x = A[k+1.., k]
    double *x = &A[(size_t)k * n + k + 1];  // row k == column k (symmetric)
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm += x[i] * x[i];
    nrm = std::sqrt(nrm);
    double *v = &Hv[(size_t)k * n + k + 1];
    if (nrm == 0.0) {
      beta[k] = 0.0;
      continue;
    }
    const double alpha = x[0] > 0 ? -nrm : nrm;
    for (int i = 0; i < m; ++i) v[i] = x[i];
    v[0] -= alpha;
    double vv = 0.0;
    for (int i = 0; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0) {
      beta[k] = 0.0;
      continue;
    }
    const double b = 2.0 / vv;
    beta[k] = b;
    // p = b * A22 v
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
      const double *row = &A[(size_t)(k + 1 + i) * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = b * s;
    }
    double pv = 0.0;
    for (int i = 0; i < m; ++i) pv += p[i] * v[i];
    const double K = 0.5 * b * pv;
    for (int i = 0; i < m; ++i) wv[i] = p[i] - K * v[i];
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
      double *row = &A[(size_t)(k + 1 + i) * n + k + 1];
      for (int j = 0; j < m; ++j) row[j] -= v[i] * wv[j] + wv[i] * v[j];
    }
    x[0] = alpha;
    for (int i = 1; i < m; ++i) x[i] = 0.0;
    for (int i = 0; i < m; ++i) A[(size_t)(k + 1 + i) * n + k] = x[i];
  }
  std::vector<double> d(n);
  for (int i = 0; i < n; ++i) d[i] = A[(size_t)i * n + i];
  for (int i = 0; i + 1 < n; ++i) e[i] = A[(size_t)(i + 1) * n + i];
  // Z^T = H_{n-3} ... H_1 H_0 (rows of Z^T are the columns of Q)
  Mat Zt((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0;
  for (int k = 0; k + 2 < n; ++k) {
    if (beta[k] == 0.0) continue;
    const int m = n - k - 1;
    const double *v = &Hv[(size_t)k * n + k + 1];
    // Zt[k+1.., :] -= beta v (v^T Zt[k+1.., :])
    std::vector<double> t(n, 0.0);
    for (int i = 0; i < m; ++i) {
      const double *row = &Zt[(size_t)(k + 1 + i) * n];
      for (int j = 0; j < n; ++j) t[j] += v[i] * row[j];
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < m; ++i) {
      double *row = &Zt[(size_t)(k + 1 + i) * n];
      const double f = beta[k] * v[i];
      for (int j = 0; j < n; ++j) row[j] -= f * t[j];
    }
  }
  // implicit symmetric QR with Wilkinson shifts on (d, e)
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  long guard = 60L * n + 100;
  while (hi > 0 && guard-- > 0) {
    for (int i = 0; i < hi; ++i)
      if (std::fabs(e[i]) <= eps * (std::fabs(d[i]) + std::fabs(d[i + 1]))) e[i] = 0.0;
    if (e[hi - 1] == 0.0) {
      --hi;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    const double dd = 0.5 * (d[hi - 1] - d[hi]);
    const double ee = e[hi - 1];
    const double den = dd + (dd >= 0 ? 1.0 : -1.0) * std::hypot(dd, ee);
    const double mu = den != 0.0 ? d[hi] - ee * ee / den : d[hi] - std::fabs(ee);
    double x = d[lo] - mu;
    double z = e[lo];
    for (int k = lo; k < hi; ++k) {
      const double r = std::hypot(x, z);
      const double c = r == 0.0 ? 1.0 : x / r;
      const double s = r == 0.0 ? 0.0 : -z / r;
      if (k > lo) e[k - 1] = r;
      const double a = d[k], b = e[k], cc = d[k + 1];
      d[k] = a * c * c - 2.0 * b * c * s + cc * s * s;
      d[k + 1] = a * s * s + 2.0 * b * c * s + cc * c * c;
      e[k] = (a - cc) * c * s + b * (c * c - s * s);
      if (k + 1 < hi) {
        const double f = e[k + 1];
        z = -f * s;
        e[k + 1] = f * c;
      }
      x = e[k];
      double *zk = &Zt[(size_t)k * n];
      double *zk1 = &Zt[(size_t)(k + 1) * n];
      for (int j = 0; j < n; ++j) {
        const double u0 = zk[j], u1 = zk1[j];
        zk[j] = c * u0 - s * u1;
        zk1[j] = s * u0 + c * u1;
      }
    }
  }
  for (int i = 0; i < n; ++i) w[i] = d[i];
  std::memcpy(V, Zt.data(), sizeof(double) * (size_t)n * n);
}

// Leading d eigenvectors (rows, decreasing eigenvalue, largest-|entry| positive).
void top_eigvecs(int n, const double *S, int d, double *P, double *evals) {
  std::vector<double> w(n);
  Mat V((size_t)n * n);
  sym_eig(n, S, w.data(), V.data());
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
  for (int r = 0; r < d; ++r) {
    const double *v = &V[(size_t)order[r] * n];
    int arg = 0;
    for (int j = 1; j < n; ++j)
      if (std::fabs(v[j]) > std::fabs(v[arg])) arg = j;
    const double sg = v[arg] < 0 ? -1.0 : 1.0;
    for (int j = 0; j < n; ++j) P[(size_t)r * n + j] = sg * v[j];
  }
  if (evals)
    for (int i = 0; i < n; ++i) evals[i] = w[order[i]];
}

// Trace-form loss (Problem leanvec_efficient) on already-normalised moments.
struct Moments {
  int D, d;
  const double *KQ, *KX;  // normalised
  Mat KQKX;               // K_Q K_X
  double trQX;            // tr(K_Q K_X)
};

double loss(const Moments &mo, const double *A, const double *B) {
  const int D = mo.D, d = mo.d;
  Mat AKQ((size_t)d * D), BKX((size_t)d * D), M1((size_t)d * d), M2((size_t)d * d);
  gemm(d, D, D, A, false, mo.KQ, false, AKQ.data());
  gemm(d, D, D, B, false, mo.KX, false, BKX.data());
  gemm(d, d, D, AKQ.data(), false, A, true, M1.data());   // A K_Q A^T
  gemm(d, d, D, BKX.data(), false, B, true, M2.data());   // B K_X B^T
  const double t1 = trace_prod(d, M1.data(), M2.data());
  // tr(K_Q A^T B K_X) = tr(B K_X K_Q A^T) = <B K_X K_Q, A>_F
  Mat BKXKQ((size_t)d * D);
  gemm(d, D, D, BKX.data(), false, mo.KQ, false, BKXKQ.data());
  double t3 = 0.0;
  for (size_t i = 0; i < (size_t)d * D; ++i) t3 += BKXKQ[i] * A[i];
  return t1 + mo.trQX - 2.0 * t3;
}

// -dA f = 2 B K_X K_Q - 2 B K_X B^T A K_Q   (Eq. leanvec_gradients, negated)
void neg_grad_A(const Moments &mo, const double *A, const double *B, double *C) {
  const int D = mo.D, d = mo.d;
  Mat BKX((size_t)d * D), M2((size_t)d * d), T((size_t)d * D), U((size_t)d * D);
  gemm(d, D, D, B, false, mo.KX, false, BKX.data());
  gemm(d, d, D, BKX.data(), false, B, true, M2.data());       // B K_X B^T
  gemm(d, D, d, M2.data(), false, A, false, T.data());        // B K_X B^T A
  gemm(d, D, D, T.data(), false, mo.KQ, false, U.data());     // ... K_Q
  gemm(d, D, D, BKX.data(), false, mo.KQ, false, T.data());   // B K_X K_Q
  for (size_t i = 0; i < (size_t)d * D; ++i) C[i] = 2.0 * T[i] - 2.0 * U[i];
}

// -dB f = 2 A K_Q K_X - 2 A K_Q A^T B K_X
void neg_grad_B(const Moments &mo, const double *A, const double *B, double *C) {
  const int D = mo.D, d = mo.d;
  Mat AKQ((size_t)d * D), M1((size_t)d * d), T((size_t)d * D), U((size_t)d * D);
  gemm(d, D, D, A, false, mo.KQ, false, AKQ.data());
  gemm(d, d, D, AKQ.data(), false, A, true, M1.data());       // A K_Q A^T
  gemm(d, D, d, M1.data(), false, B, false, T.data());        // A K_Q A^T B
  gemm(d, D, D, T.data(), false, mo.KX, false, U.data());     // ... K_X
  gemm(d, D, D, AKQ.data(), false, mo.KX, false, T.data());   // A K_Q K_X
  for (size_t i = 0; i < (size_t)d * D; ++i) C[i] = 2.0 * T[i] - 2.0 * U[i];
}

// S = argmax_{||S||_op <= 1} <S, C> = U V^T (thin SVD of C), computed as
// W diag(lambda^-1/2) W^T C from C C^T = W diag(lambda) W^T; directions with
// negligible singular value get 0 (any value in [-1, 1] is optimal there).
void lmo(int d, int D, const double *C, double *S) {
  Mat CC((size_t)d * d), W((size_t)d * d), T((size_t)d * d);
  std::vector<double> lam(d);
  gemm(d, d, D, C, false, C, true, CC.data());
  sym_eig(d, CC.data(), lam.data(), W.data());  // rows of W are eigenvectors
  double lmax = 0.0;
  for (double l : lam) lmax = std::max(lmax, l);
  const double cut = lmax * 1e-24;
  // T = W^T diag(f) W with f = lambda^-1/2
  std::vector<double> f(d);
  for (int i = 0; i < d; ++i) f[i] = lam[i] > cut && lam[i] > 0 ? 1.0 / std::sqrt(lam[i]) : 0.0;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double s = 0.0;
      for (int i = 0; i < d; ++i) s += W[(size_t)i * d + a] * f[i] * W[(size_t)i * d + b];
      T[(size_t)a * d + b] = s;
    }
  gemm(d, D, d, T.data(), false, C, false, S);
}

// Brent's bounded scalar minimisation (golden section with parabolic steps).
template <class F>
double brent_min(F f, double a, double b, double xtol, double *fbest) {
  const double cgold = 0.3819660112501051;
  double x = a + cgold * (b - a), w = x, v = x;
  double fx = f(x), fw = fx, fv = fx;
  double dstep = 0.0, e = 0.0;
  for (int it = 0; it < 500; ++it) {
    const double m = 0.5 * (a + b);
    const double tol1 = 1e-10 * std::fabs(x) + xtol / 3.0;
    const double tol2 = 2.0 * tol1;
    if (std::fabs(x - m) <= tol2 - 0.5 * (b - a)) break;
    bool golden = true;
    if (std::fabs(e) > tol1) {
      double r = (x - w) * (fx - fv);
      double q = (x - v) * (fx - fw);
      double p = (x - v) * q - (x - w) * r;
      q = 2.0 * (q - r);
      if (q > 0) p = -p;
      q = std::fabs(q);
      const double etemp = e;
      e = dstep;
      if (std::fabs(p) < std::fabs(0.5 * q * etemp) && p > q * (a - x) && p < q * (b - x)) {
        dstep = p / q;
        const double u = x + dstep;
        if (u - a < tol2 || b - u < tol2) dstep = x < m ? tol1 : -tol1;
        golden = false;
      }
    }
    if (golden) {
      e = (x >= m ? a : b) - x;
      dstep = cgold * e;
    }
    const double u = std::fabs(dstep) >= tol1 ? x + dstep : x + (dstep > 0 ? tol1 : -tol1);
    const double fu = f(u);
    if (fu <= fx) {
      if (u >= x) a = x; else b = x;
      v = w; fv = fw; w = x; fw = fx; x = u; fx = fu;
    } else {
      if (u < x) a = u; else b = u;
      if (fu <= fw || w == x) {
        v = w; fv = fw; w = u; fw = fu;
      } else if (fu <= fv || v == x || v == w) {
        v = u; fv = fu;
      }
    }
  }
  if (fbest) *fbest = fx;
  return x;
}

}  // namespace

}  // namespace lv

using lv::Mat;

extern "C" int lv_second_moment(const float *V, int64_t n, int32_t D, double *K, double *sum) {
  lv::clear_error();
  if (!V && n > 0) LV_FAIL(LV_EINVAL, "NULL V");
  if (!K) LV_FAIL(LV_EINVAL, "NULL K");
  if (n < 0 || D < 1) LV_FAIL(LV_EINVAL, "bad sizes n=%lld D=%d", (long long)n, D);
  const int64_t CH = 512;
#pragma omp parallel
  {
    std::vector<double> buf((size_t)CH * D);
#pragma omp for schedule(static)
    for (int i = 0; i < D; ++i) {
      double *krow = K + (size_t)i * D;
      for (int64_t c0 = 0; c0 < n; c0 += CH) {
        const int64_t c1 = std::min(n, c0 + CH);
        for (int64_t r = c0; r < c1; ++r) {
          const float *v = V + r * D;
          const double vi = (double)v[i];
          if (vi == 0.0) continue;
          for (int j = 0; j < D; ++j) krow[j] += vi * (double)v[j];
        }
      }
    }
  }
  if (sum)
    for (int64_t r = 0; r < n; ++r)
      for (int j = 0; j < D; ++j) sum[j] += (double)V[r * D + j];
  return LV_OK;
}

extern "C" int lv_fit_id(const double *KX, int32_t D, int32_t d, double *P, double *evals) {
  lv::clear_error();
  if (!KX || !P) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (D < 1 || d < 1 || d > D) LV_FAIL(LV_EINVAL, "need 1 <= d <= D (d=%d, D=%d)", d, D);
  lv::top_eigvecs(D, KX, d, P, evals);
  return LV_OK;
}

extern "C" int lv_ood_loss(const double *KQ, int64_t m, const double *KX, int64_t n, int32_t D,
                           int32_t d, const double *A, const double *B, double *f) {
  lv::clear_error();
  if (!KQ || !KX || !A || !B || !f) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (m < 1 || n < 1 || D < 1 || d < 1 || d > D) LV_FAIL(LV_EINVAL, "bad sizes");
  Mat KQn(KQ, KQ + (size_t)D * D), KXn(KX, KX + (size_t)D * D);
  for (auto &x : KQn) x /= (double)m;
  for (auto &x : KXn) x /= (double)n;
  lv::Moments mo{D, d, KQn.data(), KXn.data(), {}, lv::trace_prod(D, KQn.data(), KXn.data())};
  *f = lv::loss(mo, A, B);
  return LV_OK;
}

extern "C" int lv_fit_ood(const double *KQ, int64_t m, const double *KX, int64_t n, int32_t D,
                          int32_t d, const lv_fw_params *p, double *A, double *B,
                          lv_fw_report *r) {
  lv::clear_error();
  if (!KQ || !KX || !A || !B) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (m < 1 || n < 1 || D < 1 || d < 1 || d > D) LV_FAIL(LV_EINVAL, "bad sizes");
  lv_fw_params prm{0.9, 1e-3, 500, LV_FW_INIT_ES};
  if (p) prm = *p;
  if (!(prm.alpha > 0.0 && prm.alpha < 1.0)) LV_FAIL(LV_EINVAL, "alpha must be in (0, 1)");
  if (!(prm.tol >= 0.0) || prm.max_iter < 1) LV_FAIL(LV_EINVAL, "bad tol or max_iter");
  if (prm.init < LV_FW_INIT_ES || prm.init > LV_FW_INIT_GIVEN) LV_FAIL(LV_EINVAL, "bad init");
  const size_t dD = (size_t)d * D;
  Mat KQn(KQ, KQ + (size_t)D * D), KXn(KX, KX + (size_t)D * D);
  for (auto &x : KQn) x /= (double)m;
  for (auto &x : KXn) x /= (double)n;
  lv::Moments mo{D, d, KQn.data(), KXn.data(), {}, lv::trace_prod(D, KQn.data(), KXn.data())};
  if (prm.init == LV_FW_INIT_ES) {
    Mat Kb((size_t)D * D);
    for (size_t i = 0; i < Kb.size(); ++i) Kb[i] = 0.5 * KQn[i] + 0.5 * KXn[i];
    lv::top_eigvecs(D, Kb.data(), d, A, nullptr);
    std::memcpy(B, A, sizeof(double) * dD);
  } else if (prm.init == LV_FW_INIT_ZERO) {
    std::fill(A, A + dD, 0.0);
    std::fill(B, B + dD, 0.0);
  }
  double f_prev = lv::loss(mo, A, B);
  if (r) {
    r->iters = 0;
    r->converged = 0;
    r->f_first = f_prev;
    if (r->f_hist) r->f_hist[0] = f_prev;
  }
  Mat C(dD), S(dD);
  bool conv = false;
  int it = 0;
  for (int t = 0; t < prm.max_iter; ++t) {
    const double gamma = 1.0 / std::pow((double)(t + 1), prm.alpha);
    double gap = 0.0;
    lv::neg_grad_A(mo, A, B, C.data());
    bool zero = std::all_of(C.begin(), C.end(), [](double x) { return x == 0.0; });
    if (zero)
      lv::top_eigvecs(D, KQn.data(), d, S.data(), nullptr);
    else
      lv::lmo(d, D, C.data(), S.data());
    for (size_t i = 0; i < dD; ++i) gap += (S[i] - A[i]) * C[i];
    for (size_t i = 0; i < dD; ++i) A[i] = (1.0 - gamma) * A[i] + gamma * S[i];
    lv::neg_grad_B(mo, A, B, C.data());
    zero = std::all_of(C.begin(), C.end(), [](double x) { return x == 0.0; });
    if (zero)
      lv::top_eigvecs(D, KQn.data(), d, S.data(), nullptr);
    else
      lv::lmo(d, D, C.data(), S.data());
    for (size_t i = 0; i < dD; ++i) gap += (S[i] - B[i]) * C[i];
    for (size_t i = 0; i < dD; ++i) B[i] = (1.0 - gamma) * B[i] + gamma * S[i];
    const double f = lv::loss(mo, A, B);
    it = t + 1;
    if (r) {
      if (r->f_hist) r->f_hist[it] = f;
      if (r->gap_hist) r->gap_hist[t] = gap;
    }
    if (f_prev != 0.0 && std::fabs(f - f_prev) / std::fabs(f_prev) <= prm.tol) {
      conv = true;
      f_prev = f;
      break;
    }
    f_prev = f;
  }
  if (r) {
    r->iters = it;
    r->converged = conv ? 1 : 0;
    r->f_last = f_prev;
  }
  return conv ? LV_OK : LV_WNOTCONVERGED;
}

extern "C" int lv_fit_es(const double *KQ, int64_t m, const double *KX, int64_t n, int32_t D,
                         int32_t d, double xtol, double *P, double *beta) {
  lv::clear_error();
  if (!KQ || !KX || !P) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (m < 1 || n < 1 || D < 1 || d < 1 || d > D) LV_FAIL(LV_EINVAL, "bad sizes");
  if (!(xtol > 0.0)) LV_FAIL(LV_EINVAL, "xtol must be > 0");
  Mat KQn(KQ, KQ + (size_t)D * D), KXn(KX, KX + (size_t)D * D);
  for (auto &x : KQn) x /= (double)m;
  for (auto &x : KXn) x /= (double)n;
  lv::Moments mo{D, d, KQn.data(), KXn.data(), {}, lv::trace_prod(D, KQn.data(), KXn.data())};
  Mat Kb((size_t)D * D), Pt((size_t)d * D);
  auto proj = [&](double b, double *out) {
    for (size_t i = 0; i < Kb.size(); ++i) Kb[i] = (1.0 - b) * KQn[i] + b * KXn[i];
    lv::top_eigvecs(D, Kb.data(), d, out, nullptr);
  };
  // equalised loss of Problem leanvec_loss_same_proj_equalized = f - tr(K_Q K_X)
  auto obj = [&](double b) {
    proj(b, Pt.data());
    return lv::loss(mo, Pt.data(), Pt.data()) - mo.trQX;
  };
  const double bst = lv::brent_min(obj, 0.0, 1.0, xtol, nullptr);
  proj(bst, P);
  if (beta) *beta = bst;
  return LV_OK;
}

// float64 -> float32 -> bfloat16, each step round-to-nearest-even.
extern "C" int lv_to_bf16(const double *src, int64_t count, uint16_t *dst) {
  lv::clear_error();
  if (count < 0 || (count > 0 && (!src || !dst))) LV_FAIL(LV_EINVAL, "bad arguments");
  for (int64_t i = 0; i < count; ++i) {
    const float f = (float)src[i];
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) {
      dst[i] = (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
      continue;
    }
    u += 0x7FFFu + ((u >> 16) & 1u);
    dst[i] = (uint16_t)(u >> 16);
  }
  return LV_OK;
}

extern "C" int lv_mean_reduced(const double *M, int32_t d, int32_t D, const double *sum,
                               int64_t n, float *mu) {
  lv::clear_error();
  if (!M || !sum || !mu) LV_FAIL(LV_EINVAL, "NULL pointer");
  if (d < 1 || D < 1 || n < 1) LV_FAIL(LV_EINVAL, "bad sizes");
  for (int i = 0; i < d; ++i) {
    double s = 0.0;
    for (int j = 0; j < D; ++j) s += M[(size_t)i * D + j] * (sum[j] / (double)n);
    mu[i] = (float)s;
  }
  return LV_OK;
}

// Clip singular values at 1: M <- W diag(min(1, 1/sigma)) W^T M with
// M M^T = W diag(sigma^2) W^T (rows of W from the symmetric eigensolver).
namespace lv {

// With M M^T = W^T diag(lam) W (rows of W the eigenvectors), the projection
// of M onto the spectral-norm ball is T M, T = W^T diag(min(1, lam^-1/2)) W:
// singular values above 1 become 1, the singular vectors stay.  Returns
// false (T untouched) when no singular value exceeds 1.
bool clip_factor(int32_t d, const double *MMt, double *T) {
  Mat W((size_t)d * d);
  std::vector<double> lam(d);
  sym_eig(d, MMt, lam.data(), W.data());
  std::vector<double> f(d);
  bool any = false;
  for (int i = 0; i < d; ++i) {
    const double s = lam[i] > 0 ? std::sqrt(lam[i]) : 0.0;
    f[i] = s > 1.0 ? 1.0 / s : 1.0;
    any = any || s > 1.0;
  }
  if (!any) return false;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      double s = 0.0;
      for (int i = 0; i < d; ++i) s += W[(size_t)i * d + a] * f[i] * W[(size_t)i * d + b];
      T[(size_t)a * d + b] = s;
    }
  return true;
}

}  // namespace lv

extern "C" int lv_clip_spectral(double *M, int32_t d, int32_t D) {
  lv::clear_error();
  if (!M) LV_FAIL(LV_EINVAL, "NULL matrix");
  if (d < 1 || D < 1) LV_FAIL(LV_EINVAL, "bad sizes");
  Mat MM((size_t)d * d), T((size_t)d * d), out((size_t)d * D);
  lv::gemm(d, d, D, M, false, M, true, MM.data());
  if (!lv::clip_factor(d, MM.data(), T.data())) return LV_OK;
  lv::gemm(d, D, d, T.data(), false, M, false, out.data());
  std::memcpy(M, out.data(), sizeof(double) * out.size());
  return LV_OK;
}
