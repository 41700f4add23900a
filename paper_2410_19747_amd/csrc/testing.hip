// Kernel-level test entry points (include/ttm_testing.h).
#include <math.h>

#include <algorithm>

#include "../../include/ttm_testing.h"
#include "ttm_internal.h"

extern "C" {

int ttm_test_gemm(int M, int N, int K, int batch, const double *A, int64_t a_rs, int64_t a_cs,
                  int64_t a_bs, const double *B, int64_t b_rs, int64_t b_cs, int64_t b_bs,
                  double *C, int64_t c_bs, int c_rdiv, int c_cdiv, int64_t c_rs1, int64_t c_rs0,
                  int64_t c_cs1, int64_t c_cs0, void *stream) {
  if (M < 1 || N < 1 || K < 1 || batch < 1 || !A || !B || !C || c_rdiv < 1 || c_cdiv < 1)
    return TTM_EINVAL;
  ttm::GemmArgs g;
  g.M = M; g.N = N; g.K = K; g.batch = batch;
  g.A = A; g.a_rs = a_rs; g.a_cs = a_cs; g.a_bs = a_bs;
  g.B = B; g.b_rs = b_rs; g.b_cs = b_cs; g.b_bs = b_bs;
  g.C = C; g.c_bs = c_bs; g.c_rdiv = c_rdiv; g.c_cdiv = c_cdiv;
  g.c_rs1 = c_rs1; g.c_rs0 = c_rs0; g.c_cs1 = c_cs1; g.c_cs0 = c_cs0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ttm::launch_gemm(g, s) != hipSuccess) return TTM_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? TTM_OK : TTM_EHIP;
}

int ttm_test_gemm_prec(int prec, int M, int N, int K, const double *A, int64_t a_rs, int64_t a_cs,
                       const double *B, int64_t b_rs, int64_t b_cs, double *C, int64_t c_rs,
                       void *stream) {
  if (M < 1 || N < 1 || K < 1 || !A || !B || !C) return TTM_EINVAL;
  if (prec < TTM_PREC_F64 || prec > TTM_PREC_BF16X3) return TTM_EINVAL;
  ttm::GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.a_rs = a_rs; g.a_cs = a_cs;
  g.B = B; g.b_rs = b_rs; g.b_cs = b_cs;
  g.C = C; g.c_rs1 = c_rs; g.c_cs1 = 1;
  g.prec = prec;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ttm::launch_gemm(g, s) != hipSuccess) return TTM_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? TTM_OK : TTM_EHIP;
}

size_t ttm_test_qr_scratch(int m, int n) { return ttm::qr_scratch_doubles(m, n); }

int ttm_test_qr(const double *M, int m, int n, double *Q, double *R, double *scratch, void *stream) {
  if (m < 1 || n < 1 || !M || !Q || !R || !scratch) return TTM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ttm::launch_qr(M, m, n, n, 1, Q, R, scratch, s) != hipSuccess) return TTM_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? TTM_OK : TTM_EHIP;
}

size_t ttm_test_qr_pivoted_scratch(int m, int n) {
  if (m < 1 || n < 1) return 0;
  return ttm::qr_inplace_scratch_doubles(m, n);
}

int ttm_test_qr_pivoted(double *S, int m, int n, int *perm, double *scratch, void *stream) {
  if (m < 1 || n < 1 || !S || !perm || !scratch) return TTM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ttm::launch_qr_inplace(S, m, n, scratch, perm, nullptr, s) != hipSuccess) return TTM_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? TTM_OK : TTM_EHIP;
}

size_t ttm_test_svd_ws_bytes(int m, int n) {
  if (m < 1 || n < 1) return 0;
  // the larger of the two orientations, plus a transposed copy of M
  const size_t a = ttm::svd_ws_doubles(ttm::svd_plan(m, n));
  const size_t b = ttm::svd_ws_doubles(ttm::svd_plan(n, m));
  return (std::max(a, b) + (size_t)m * n + 64) * sizeof(double);
}

int ttm_test_svd(const double *M, int m, int n, double eps, int cap, int forced, int left_pow,
                 int right_pow, double *left, double *right, double *sigma, int *rank,
                 int *sweeps, void *ws, size_t ws_bytes, void *stream) {
  if (m < 1 || n < 1 || !M || !left || !right || !sigma || !rank || !ws) return TTM_EINVAL;
  if (left_pow + right_pow != 1 || left_pow < 0 || right_pow < 0) return TTM_EINVAL;
  if (ws_bytes < ttm_test_svd_ws_bytes(m, n)) return TTM_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *base = static_cast<double *>(ws);
  double *Yt = base;                                           // M^T copy when needed
  double *sws = base + ((((size_t)m * n) + 31) & ~(size_t)31);
  ttm::SvdResult res;
  if (right_pow == 0) {
    // right factor orthonormal: Y = M (m x n), column-major copy of row-major M
    if (ttm::launch_transpose(Yt, M, m, n, s) != hipSuccess) return TTM_EHIP;
    const ttm::SvdPlan sp = ttm::svd_plan(m, n);
    res = ttm::svd_oside(sp, Yt, eps, cap, forced, 60, right, ttm::SVD_U_T, sigma, sws, s, nullptr, 0);
    if (res.err == TTM_OK) {
      ttm::GemmArgs g;  // left = M V_r
      g.M = m; g.N = res.rank; g.K = n;
      g.A = M; g.a_rs = n; g.a_cs = 1;
      g.B = right; g.b_rs = 1; g.b_cs = n;
      g.C = left; g.c_rs1 = res.rank; g.c_cs1 = 1;
      if (ttm::launch_gemm(g, s) != hipSuccess) return TTM_EHIP;
    }
  } else {
    // left factor orthonormal: Y = M^T, whose column-major storage is M's
    const ttm::SvdPlan sp = ttm::svd_plan(n, m);
    res = ttm::svd_oside(sp, M, eps, cap, forced, 60, left, ttm::SVD_U, sigma, sws, s, nullptr, 0);
    if (res.err == TTM_OK) {
      ttm::GemmArgs g;  // right = U_r^T M
      g.M = res.rank; g.N = n; g.K = m;
      g.A = left; g.a_rs = 1; g.a_cs = res.rank;
      g.B = M; g.b_rs = n; g.b_cs = 1;
      g.C = right; g.c_rs1 = n; g.c_cs1 = 1;
      if (ttm::launch_gemm(g, s) != hipSuccess) return TTM_EHIP;
    }
  }
  if (sweeps) *sweeps = res.sweeps;
  if (res.err != TTM_OK) return res.err;
  *rank = res.rank;
  return hipStreamSynchronize(s) == hipSuccess ? TTM_OK : TTM_EHIP;
}

}  // extern "C"
