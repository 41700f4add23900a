// Kernel-level test entry points (include/ttm_testing.h).
#include <math.h>

#include <algorithm>

#include "../../include/ttm_testing.h"
#include "ttm_internal.h"

namespace {
typedef double dbl4_t __attribute__((ext_vector_type(4)));

// FP64 matrix-core rate probe: every wave runs eight independent chains of
// v_mfma_f64_16x16x4f64 (2048 flops each) on register operands, so the
// issue rate of the matrix cores is the only limit; the accumulators are
// written out so that nothing is optimised away.
__global__ __launch_bounds__(256) void mfma_f64_rate_kernel(int iters, double *__restrict__ out) {
  const double a = 1.0 + 1e-3 * (threadIdx.x & 63), b = 1.0 - 1e-3 * (threadIdx.x & 63);
  constexpr int CH = 8;
  dbl4_t acc[CH];
#pragma unroll
  for (int k = 0; k < CH; ++k) acc[k] = dbl4_t{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < CH; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
  }
  double sum = 0.0;
#pragma unroll
  for (int k = 0; k < CH; ++k) sum += (acc[k][0] + acc[k][1]) + (acc[k][2] + acc[k][3]);
  out[blockIdx.x * 256 + threadIdx.x] = sum;
}
}  // namespace

extern "C" {

int ttm_test_mfma_f64_rate(int blocks, int iters, double *out, double *seconds, double *flops, void *stream) {
  if (blocks < 1 || blocks > 65535 || iters < 1 || !out || !seconds || !flops) return TTM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return TTM_EHIP;
  int rc = TTM_OK;
  float ms = 0.0f;
  if (hipEventRecord(e0, s) != hipSuccess) rc = TTM_EHIP;
  if (rc == TTM_OK) {
    hipLaunchKernelGGL(mfma_f64_rate_kernel, dim3(blocks), dim3(256), 0, s, iters, out);
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      rc = TTM_EHIP;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *seconds = 1e-3 * ms;
  *flops = (double)blocks * 4 /* waves */ * iters * 8 /* chains */ * 2048.0;
  return rc;
}

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

size_t ttm_test_svd_ws_bytes_bw(int m, int n, int block_width) {
  if (m < 1 || n < 1) return 0;
  if (block_width != 0 && block_width != 16 && block_width != 32) return 0;
  // the larger of the two orientations, plus a transposed copy of M
  const size_t a = ttm::svd_ws_doubles(ttm::svd_plan(m, n, block_width));
  const size_t b = ttm::svd_ws_doubles(ttm::svd_plan(n, m, block_width));
  return (std::max(a, b) + (size_t)m * n + 64) * sizeof(double);
}

size_t ttm_test_svd_ws_bytes(int m, int n) { return ttm_test_svd_ws_bytes_bw(m, n, 0); }

int ttm_test_svd_bw(const double *M, int m, int n, double eps, int cap, int forced, int left_pow,
                    int right_pow, double *left, double *right, double *sigma, int *rank, int *sweeps,
                    int block_width, void *ws, size_t ws_bytes, void *stream) {
  if (m < 1 || n < 1 || !M || !left || !right || !sigma || !rank || !ws) return TTM_EINVAL;
  if (left_pow + right_pow != 1 || left_pow < 0 || right_pow < 0) return TTM_EINVAL;
  if (block_width != 0 && block_width != 16 && block_width != 32) return TTM_EINVAL;
  if (std::min(m, n) > ttm::kSvdMaxSide || (right_pow == 0 ? m : n) > ttm::kSvdMaxSide) return TTM_EUNSUPPORTED;
  if (ws_bytes < ttm_test_svd_ws_bytes_bw(m, n, block_width)) return TTM_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *base = static_cast<double *>(ws);
  double *Yt = base;                                           // M^T copy when needed
  double *sws = base + ((((size_t)m * n) + 31) & ~(size_t)31);
  ttm::SvdResult res;
  if (right_pow == 0) {
    // right factor orthonormal: Y = M (m x n), column-major copy of row-major M
    if (ttm::launch_transpose(Yt, M, m, n, s) != hipSuccess) return TTM_EHIP;
    const ttm::SvdPlan sp = ttm::svd_plan(m, n, block_width);
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
    const ttm::SvdPlan sp = ttm::svd_plan(n, m, block_width);
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

int ttm_test_svd(const double *M, int m, int n, double eps, int cap, int forced, int left_pow,
                 int right_pow, double *left, double *right, double *sigma, int *rank,
                 int *sweeps, void *ws, size_t ws_bytes, void *stream) {
  return ttm_test_svd_bw(M, m, n, eps, cap, forced, left_pow, right_pow, left, right, sigma, rank, sweeps, 0,
                         ws, ws_bytes, stream);
}

size_t ttm_test_cholqr2_ws_bytes(int p, int l) {
  if (p < 1 || l < 1 || l > p) return 0;
  return ttm::cholqr2_ws_doubles(p, l) * sizeof(double);
}

int ttm_test_cholqr2(double *Y, int p, int l, int *breakdown, void *ws, size_t ws_bytes, void *stream) {
  if (p < 1 || l < 1 || l > p || !Y || !breakdown || !ws) return TTM_EINVAL;
  if (ws_bytes < ttm::cholqr2_ws_doubles(p, l) * sizeof(double)) return TTM_EWORKSPACE;
  const hipError_t e = ttm::cholqr2(Y, p, l, static_cast<double *>(ws), breakdown, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? TTM_OK : TTM_EHIP;
}

}  // extern "C"
