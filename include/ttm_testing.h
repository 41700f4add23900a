/*
 * ttm_testing.h - kernel-level entry points of libttm for parity tests.
 *
 * Each call runs one building block of the TTM sweep on device buffers the
 * caller owns and returns after the stream has finished (0 or a negative
 * TTM_E* code from ttm.h).  They exist so that tests can check every kernel
 * against a plain reference on random operands; the product itself only
 * needs ttm.h.
 */
#ifndef TTM_TESTING_H
#define TTM_TESTING_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Batched FP64 product with the split-stride output mapping used by the
 * Contract (Eq. contract) and swap-merge steps:
 *   C[b](i,j) = sum_k A[b](i,k) B[b](k,j), A(i,k) at A + b*a_bs + i*a_rs + k*a_cs,
 *   B(k,j) at B + b*b_bs + k*b_rs + j*b_cs, C(i,j) at
 *   C + b*c_bs + (i/c_rdiv)*c_rs1 + (i%c_rdiv)*c_rs0 + (j/c_cdiv)*c_cs1 + (j%c_cdiv)*c_cs0. */
int ttm_test_gemm(int M, int N, int K, int batch, const double *A, int64_t a_rs, int64_t a_cs,
                  int64_t a_bs, const double *B, int64_t b_rs, int64_t b_cs, int64_t b_bs,
                  double *C, int64_t c_bs, int c_rdiv, int c_cdiv, int64_t c_rs1, int64_t c_rs0,
                  int64_t c_cs1, int64_t c_cs0, void *stream);

/* As ttm_test_gemm, in the arithmetic `prec` (a TTM_PREC_* value of ttm.h):
 * operands rounded to FP32 / BF16 / three BF16 terms, accumulated in FP32
 * within each 16-deep k-tile and in FP64 across k-tiles. */
int ttm_test_gemm_prec(int prec, int M, int N, int K, const double *A, int64_t a_rs, int64_t a_cs,
                       const double *B, int64_t b_rs, int64_t b_cs, double *C, int64_t c_rs,
                       void *stream);

/* Householder QR of the m x n row-major matrix M (device): Q (m x k,
 * row-major, k = min(m,n)) and R (k x n, row-major).  scratch: device,
 * ttm_test_qr_scratch(m, n) doubles. */
size_t ttm_test_qr_scratch(int m, int n);
int ttm_test_qr(const double *M, int m, int n, double *Q, double *R, double *scratch, void *stream);

/* Rate of the FP64 matrix cores (v_mfma_f64_16x16x4f64) on this device:
 * `blocks` workgroups of four waves, each wave running eight independent
 * chains of `iters` MFMAs on register operands.  Writes the elapsed time
 * (HIP events on the stream) and the flops done (blocks * 4 * iters * 8 *
 * 2048) on the host; out (device, blocks * 256 doubles) receives the
 * accumulator sums.  It measures the peak that the roofline quotes. */
int ttm_test_mfma_f64_rate(int blocks, int iters, double *out, double *seconds, double *flops, void *stream);

/* In-place Householder QR with block column pivoting of the m x n
 * column-major matrix S (device, ld m), n <= 8192: before each 16-column
 * panel the 16 remaining columns of largest norm (over the rows not yet
 * reduced) move into it in decreasing order.  On return the upper trapezoid
 * of S is R with S_in P = Q R; perm (device, n ints) is permuted along with
 * the columns (perm[j] = the entry that was at position j of the input
 * array), so starting from the identity it gives P.  The SVD path does not
 * pivot (the presorted column order costs less overall); this hook keeps
 * the option tested.  scratch: device, ttm_test_qr_pivoted_scratch(m, n)
 * doubles. */
size_t ttm_test_qr_pivoted_scratch(int m, int n);
int ttm_test_qr_pivoted(double *S, int m, int n, int *perm, double *scratch, void *stream);

/* Truncated SVD of the m x n row-major matrix M (device) by the swap's SVD
 * path (column ordering, Householder QR, one-sided block Jacobi on R^T) and
 * the rule of Eq. (eps) (cap > 0 caps the rank, forced > 0 replaces the
 * rule).  Writes left = U_r diag(s)^left_pow (m x r) and
 * right = diag(s)^right_pow V_r^T (r x n), both row-major, with exactly one
 * of left_pow, right_pow equal to 1 (the other factor is the orthonormal
 * one), the sorted singular values (min(m,n) doubles, device) and, on the
 * host, the rank and the number of sweeps.  ws: device,
 * ttm_test_svd_ws_bytes(m, n) bytes.  Returns TTM_EINVAL for other powers. */
size_t ttm_test_svd_ws_bytes(int m, int n);
int ttm_test_svd(const double *M, int m, int n, double eps, int cap, int forced, int left_pow,
                 int right_pow, double *left, double *right, double *sigma, int *rank,
                 int *sweeps, void *ws, size_t ws_bytes, void *stream);

/* As ttm_test_svd with the Jacobi block width chosen by the caller:
 * block_width 16 (32-column block pairs), 32 (64-column pairs, 1024-thread
 * solve, circle pairing, the path every matrix of 8192 rows and more than
 * 256 columns takes) or 0 (the automatic choice).  It lets matrices small
 * enough for a LAPACK reference run the 64-column-pair path.  Workspace:
 * ttm_test_svd_ws_bytes_bw(m, n, block_width) bytes (0 for a bad width).
 * TTM_EUNSUPPORTED when the orthonormal side exceeds 8192. */
size_t ttm_test_svd_ws_bytes_bw(int m, int n, int block_width);
int ttm_test_svd_bw(const double *M, int m, int n, double eps, int cap, int forced, int left_pow,
                    int right_pow, double *left, double *right, double *sigma, int *rank, int *sweeps,
                    int block_width, void *ws, size_t ws_bytes, void *stream);

/* CholeskyQR2 of the p x l column-major Y (ld p, l <= p) in place: two
 * passes of Y^T Y = R^T R, Y <- Y R^-1, as the randomized swap SVD
 * (TTM_SVD_RANDOMIZED) orthonormalises its sketches.  *breakdown = 1 when a
 * Cholesky pivot fell to the rounding level of its column (Y numerically
 * rank deficient, or cond(Y) beyond about 1e7); Y is then not orthonormal.
 * ws: device, ttm_test_cholqr2_ws_bytes(p, l) bytes (0 for bad sizes).
 * Synchronises the stream. */
size_t ttm_test_cholqr2_ws_bytes(int p, int l);
int ttm_test_cholqr2(double *Y, int p, int l, int *breakdown, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TTM_TESTING_H */
