// Kernel-level test entry points (include/ttm_testing.h).
#include <math.h>

#include <algorithm>

#include "../../include/ttm_testing.h"
#include "ttm_internal.h"

namespace ttm {
namespace {
__global__ void gather_sigma_kernel(const double *sigma, const int *perm, int n, double *out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = sigma[perm[k]];
}

JacobiBufs carve_test(double *base, const JacobiPlan &jp) {
  JacobiBufs b;
  double *p = base;
  auto adv = [&](size_t nd) {
    double *q = p;
    p += (nd + 31) & ~(size_t)31;
    return q;
  };
  b.W = adv((size_t)jp.L * jp.ncp);
  b.Wt = adv((size_t)jp.L * jp.ncp);
  b.V = adv((size_t)jp.ncp * jp.ncp);
  b.Vt = adv((size_t)jp.ncp * jp.ncp);
  b.part = adv((size_t)jp.pairs * jp.sw * 4 * jp.bw * jp.bw);
  b.conv = adv((size_t)jp.rounds * jp.pairs);
  b.qbuf = adv(2 * (size_t)jp.pairs * 32 * 32);
  b.flag = reinterpret_cast<int *>(adv(2 * (size_t)jp.pairs));
  b.sigma = adv((size_t)jp.ncp);
  b.perm = reinterpret_cast<int *>(adv((size_t)jp.ncp));
  b.result = adv(8);
  return b;
}
}  // namespace
}  // namespace ttm

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

size_t ttm_test_qr_scratch(int m, int n) { return ttm::qr_scratch_doubles(m, n); }

int ttm_test_qr(const double *M, int m, int n, double *Q, double *R, double *scratch, void *stream) {
  if (m < 1 || n < 1 || !M || !Q || !R || !scratch) return TTM_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ttm::launch_qr(M, m, n, n, 1, Q, R, scratch, s) != hipSuccess) return TTM_EHIP;
  return hipStreamSynchronize(s) == hipSuccess ? TTM_OK : TTM_EHIP;
}

size_t ttm_test_svd_ws_bytes(int m, int n) {
  ttm::JacobiPlan jp = ttm::jacobi_plan(std::max(m, n), std::min(m, n));
  return ttm::jacobi_ws_doubles(jp) * sizeof(double);
}

int ttm_test_svd(const double *M, int m, int n, double eps, int cap, int forced, int left_pow,
                 int right_pow, double *left, double *right, double *sigma, int *rank,
                 int *sweeps, void *ws, size_t ws_bytes, void *stream) {
  if (m < 1 || n < 1 || !M || !left || !right || !sigma || !rank || !ws) return TTM_EINVAL;
  if (ws_bytes < ttm_test_svd_ws_bytes(m, n)) return TTM_EWORKSPACE;
  const bool tall = m >= n;
  const int L = tall ? m : n, nc = tall ? n : m;
  ttm::JacobiPlan jp = ttm::jacobi_plan(L, nc);
  ttm::JacobiBufs jb = ttm::carve_test(static_cast<double *>(ws), jp);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // W = M (tall: column-major copy of M) or M^T (wide: M's row-major storage).
  if (tall) {
    if (ttm::launch_transpose(jb.W, M, m, n, s) != hipSuccess) return TTM_EHIP;
  } else {
    if (ttm::launch_copy(jb.W, M, (int64_t)m * n, s) != hipSuccess) return TTM_EHIP;
  }
  if (ttm::launch_jacobi_init(jp, jb, s) != hipSuccess) return TTM_EHIP;
  const double tol = sqrt((double)L) * 2.220446049250313e-16;
  double res[8];
  int sw = 0;
  bool ok = false;
  double prev = INFINITY;
  for (; sw < 60;) {
    if (ttm::launch_jacobi_sort_columns(jp, jb, s) != hipSuccess) return TTM_EHIP;
    if (ttm::launch_jacobi_sweep(jp, jb, tol, s) != hipSuccess) return TTM_EHIP;
    ++sw;
    if (hipMemcpyAsync(res, jb.result, sizeof(res), hipMemcpyDeviceToHost, s) != hipSuccess) return TTM_EHIP;
    if (hipStreamSynchronize(s) != hipSuccess) return TTM_EHIP;
    if (res[3] <= tol || (res[3] < 1e3 * tol && res[3] > 0.5 * prev)) { ok = true; break; }
    prev = res[3];
  }
  if (sweeps) *sweeps = sw;
  if (!ok) return TTM_ENOCONV;
  if (ttm::launch_jacobi_finish(jp, jb, eps, cap, forced, s) != hipSuccess) return TTM_EHIP;
  if (hipMemcpyAsync(res, jb.result, sizeof(res), hipMemcpyDeviceToHost, s) != hipSuccess) return TTM_EHIP;
  if (hipStreamSynchronize(s) != hipSuccess) return TTM_EHIP;
  const int r = (int)res[0];
  *rank = r;
  if (ttm::launch_svd_write(jp, jb, r, tall, left_pow, right_pow, left, right, s) != hipSuccess) return TTM_EHIP;
  hipLaunchKernelGGL(ttm::gather_sigma_kernel, dim3((nc + 255) / 256), dim3(256), 0, s, jb.sigma, jb.perm, nc, sigma);
  return hipStreamSynchronize(s) == hipSuccess ? TTM_OK : TTM_EHIP;
}

}  // extern "C"
