// Internal declarations shared by the kernel and runtime translation units
// of libttm.  Host-side launchers enqueue gfx950 kernels on a stream; they do
// no allocation and no synchronisation.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/ttm.h"

namespace ttm {

// ------------------------------------------------------------------ error text
// Description of the last failure of a library call on the calling thread,
// returned by ttm_last_error: which HIP call or step failed and the runtime's
// own name for the error.  Entry points clear it when they start.
void set_last_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_last_error();
// Records a failed HIP call: "<hipErrorName> in <what>: <hipErrorString>".
void note_hip_error(hipError_t e, const char *what);
const char *last_error_text();

// ------------------------------------------------------------------ kernel timing
// Optional per-launch timing with HIP events on the launching stream.  Kernel
// classes follow ttm_stats.kernel_ms.  Events come from a process-wide pool
// (no device memory); elapsed times are collected after the next
// synchronisation of the stream.
enum KernelClass {
  KC_GEMM = 0,
  KC_QR = 1,
  KC_JAC_GRAM = 2,
  KC_JAC_SOLVE = 3,
  KC_JAC_OTHER = 4,
  KC_OTHER = 5,
  KC_JAC_APPLY = 6,
  KC_COUNT = 7
};
struct KernelTimer {
  bool on = false;
  double ms[KC_COUNT] = {};
  int64_t launches[KC_COUNT] = {};
  // indices into the pool of (start, end) pairs recorded but not yet read
  int pending_cls[4096];
  int npending = 0;
  void begin(int cls, hipStream_t s);
  void end(int cls, hipStream_t s);
  // Reads every pending pair; the stream must have been synchronised.
  void collect();
};
// RAII helper: times one launch when the timer is on.
struct Timed {
  KernelTimer *t;
  int cls;
  hipStream_t s;
  Timed(KernelTimer *t_, int c, hipStream_t s_) : t(t_), cls(c), s(s_) {
    if (t && t->on) t->begin(cls, s);
  }
  ~Timed() {
    if (t && t->on) t->end(cls, s);
  }
};

// ------------------------------------------------------------------ GEMM
// C = alpha * A B + beta * C for a batch of independent products.
//   A[i][k] at A + b*a_bs + i*a_rs + k*a_cs     (i < M, k < K)
//   B[k][j] at B + b*b_bs + k*b_rs + j*b_cs     (k < K, j < N)
//   C[i][j] at C + b*c_bs + (i / c_rdiv)*c_rs1 + (i % c_rdiv)*c_rs0
//                         + (j / c_cdiv)*c_cs1 + (j % c_cdiv)*c_cs0
// The split output mapping lets a product write a permuted layout (the
// leg exchange of a swap) directly.  beta == 0 never reads C.  prec selects
// the arithmetic: FP64, or operands rounded to FP32, BF16 or three BF16 terms
// accumulated in FP32 within each 16-deep k-tile and in FP64 across k-tiles
// (inputs and output FP64 in memory either way).
enum GemmPrec { GEMM_F64 = 0, GEMM_F32 = 1, GEMM_BF16 = 2, GEMM_BF16X3 = 3 };
struct GemmArgs {
  int M = 0, N = 0, K = 0, batch = 1;
  const double *A = nullptr;
  int64_t a_rs = 0, a_cs = 0, a_bs = 0;
  const double *B = nullptr;
  int64_t b_rs = 0, b_cs = 0, b_bs = 0;
  double *C = nullptr;
  int64_t c_bs = 0;
  int c_rdiv = 1, c_cdiv = 1;
  int64_t c_rs1 = 0, c_rs0 = 0, c_cs1 = 0, c_cs0 = 0;
  double alpha = 1.0, beta = 0.0;
  int prec = GEMM_F64;
  // Optional split-K scratch: with part set, launch_gemm may split K over
  // slices when the output has too few tiles to fill the device; each slice
  // writes its partial tile to part and a second kernel sums the slices in a
  // fixed order (deterministic, but a different rounding order from the
  // unsplit product).  ksplit and kchunk are set by launch_gemm.
  double *part = nullptr;
  int64_t part_doubles = 0;
  int ksplit = 1, kchunk = 0;
};

// Plain row-major helper: C[M x N] (ldc) = A[M x K] (lda) * B[K x N] (ldb).
GemmArgs gemm_rowmajor(int M, int N, int K, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double *C, int64_t ldc);

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s);

// ------------------------------------------------------------------ element-wise
// dst[i] = src[i], i < n.
hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t s);
// dst[i] = v, i < n.
hipError_t launch_fill(double *dst, double v, int64_t n, hipStream_t s);
// Reversal of a carriage: out[b][w][a] = in[a][w][b], in is [rl][d][rr].
hipError_t launch_reverse_core(double *out, const double *in, int rl, int d, int rr, hipStream_t s);
// flag[0] = 1 if any of x[0..n) is NaN or Inf (flag must be zeroed first).
hipError_t launch_nonfinite_check(const double *x, int64_t n, int *flag, hipStream_t s);
hipError_t launch_zero_int(int *p, int n, hipStream_t s);
// dst[i] = counter-based SplitMix64 uniform in [-1, 1) for counters start + i.
hipError_t launch_splitmix_fill(double *dst, int64_t n, uint64_t seed, int64_t start, hipStream_t s);
// out[0] = sum_i x[i]^2.
hipError_t launch_sumsq(const double *x, int64_t n, double *out, hipStream_t s);

// ------------------------------------------------------------------ QR
// Householder QR of an m x n matrix M (element (i,j) at M + i*rs + j*cs).
// Writes Q (m x k, k = min(m,n)) row-major with leading dimension k into q,
// and R (k x n) row-major into r.  scratch: qr_scratch_doubles(m, n).
// q, r and scratch must not overlap M.
hipError_t launch_qr(const double *M, int m, int n, int64_t rs, int64_t cs, double *q, double *r,
                     double *scratch, hipStream_t s);
size_t qr_scratch_doubles(int m, int n);
// In-place Householder QR of the column-major m x n matrix S (ld m), R only:
// on return the upper trapezoid of S[0:k, :] is R and the reflectors lie
// below it.  With perm (device, n ints) not null the factorisation uses
// block column pivoting: before each 16-column panel the 16 columns of
// largest remaining norm are moved into it (n <= 8192), so that S P = Q R,
// and perm is permuted along (perm[j] = the column held at position j).
// scratch: qr_inplace_scratch_doubles(m, n).  With Tall not null the
// triangular factor T of panel i (16 x 16, row-major) is kept at
// Tall + 256 i, ceil(k / 16) panels, for launch_apply_q.
hipError_t launch_qr_inplace(double *S, int m, int n, double *scratch, int *perm, double *Tall, hipStream_t s);
size_t qr_inplace_scratch_doubles(int m, int n);
// X <- Q X for the m x nc column-major X (ld m), Q = H_0 ... H_{k-1} the
// orthogonal factor of a launch_qr_inplace factorisation of S (m rows, its
// T factors in Tall).  scratch: qr_apply_q_scratch_doubles(m, nc).
size_t qr_apply_q_scratch_doubles(int m, int nc);
hipError_t launch_apply_q(const double *S, int m, int k, const double *Tall, double *X, int nc, double *scratch,
                          hipStream_t s);

// ------------------------------------------------------------------ Jacobi
// One-sided block Jacobi on an L x nc column-major matrix W (ld = L),
// columns padded with zeros to ncp = nblk * bw (nblk even).
struct JacobiPlan {
  int L = 0, nc = 0;     // rows, real columns
  int bw = 0;            // block width
  int nblk = 0;          // number of blocks (even)
  int ncp = 0;           // padded columns = nblk * bw
  int xs = 0;            // 1: XOR pairing (round r pairs blocks i and i ^ (r + 1)), else circle method
  int rows_per_wg = 0;   // row chunk per workgroup for Gram and update
  int sw = 0;            // row chunks of W
  int gsub = 1;          // row chunks summed by one Gram workgroup (circle pairing)
  int gsw = 0;           // partial Grams per pair: ceil(sw / gsub)
  int rounds = 0;        // nblk - 1
  int pairs = 0;         // nblk / 2
};
// force_bw (16 or 32) overrides the block width chosen from the size; 0
// keeps the automatic choice (a testing hook: it lets small matrices take
// the 64-column-pair path that only 8192-row matrices take otherwise).
JacobiPlan jacobi_plan(int L, int nc, int force_bw = 0);
// Workspace doubles of the Jacobi buffers of a plan.
size_t jacobi_ws_doubles(const JacobiPlan &p);

// Device buffers of one Jacobi run (carved from the workspace).
struct JacobiBufs {
  double *W = nullptr;      // L x ncp (column-major)
  double *Wt = nullptr;     // reordering buffer (swapped with W)
  double *part = nullptr;   // pairs * sw * (2bw)^2 partial Grams
  double *conv = nullptr;   // rounds * pairs: scaled off-diagonal maxima
  double *sigma = nullptr;  // ncp
  int *perm = nullptr;      // ncp: perm[k] = column index of the k-th largest value
  double *qbuf = nullptr;   // pairs * (2bw)^2: rotations of the current round
  int *flag = nullptr;      // pairs: rotation is not the identity
  double *result = nullptr; // 8 doubles: [0]=rank,[1]=discarded,[2]=total,[3]=max off,[4]=nonfinite,
                            // [5]=squared Frobenius norm of W, [6]=count of values above the noise level
};

// One sweep of rounds; after it b.result[3] holds the sweep's largest scaled
// off-diagonal |g_pq| / sqrt(g_pp g_qq) over every visited pair.  Needs
// result[5] = ||W||_F^2.  Per round a Gram, a solve and an apply launch;
// with XOR pairing a round's apply and the next round's Grams are one launch.
hipError_t launch_jacobi_sweep(const JacobiPlan &p, const JacobiBufs &b, double tol, hipStream_t s,
                               KernelTimer *timer = nullptr);
// Reorder the columns of W by decreasing norm (swaps W/Wt).
hipError_t launch_jacobi_sort_columns(const JacobiPlan &p, JacobiBufs &b, hipStream_t s);
// Column norms, descending order, and the rank rule of Eq. (eps):
// r = min{k>=1 : tail_k < eps*total or tail_k == 0}, then min(r, cap) when
// cap > 0; forced > 0 replaces the rule.  Writes result[0..2].
// With full_total set (device), the rule counts full_total - (the sum of
// squares of W's values) as extra weight in every tail and in the total.
hipError_t launch_jacobi_finish(const JacobiPlan &p, const JacobiBufs &b, double eps, int cap,
                                int forced, hipStream_t s, const double *full_total = nullptr);
// u[rowperm[j]*u_os + t*u_ts] = j-th entry of the t-th largest column of W
// divided by its norm (j < L, t < r).
hipError_t launch_jacobi_write_u(const JacobiPlan &p, const JacobiBufs &b, const int *rowperm, int r,
                                 double *u, int64_t u_os, int64_t u_ts, hipStream_t s);

// Helpers shared with the SVD driver.
hipError_t launch_column_norms(const double *W, int L, int nc, double *out, hipStream_t s);
hipError_t launch_sort_desc(const double *v, int n, int *perm, hipStream_t s);  // n <= 8192
hipError_t launch_gather_columns(const double *src, const int *perm, int L, int ncols, double *dst,
                                 hipStream_t s);
hipError_t launch_rt_from_qr(const double *S, int m, int n, int k, int ncp, double *W, hipStream_t s);
hipError_t launch_frob_from_norms(const double *x, int n, double *result, hipStream_t s);

// ------------------------------------------------------------------ truncated SVD
// Truncated SVD Y ~= Z U_r^T of an np x no matrix Y (column-major, ld np)
// whose factor U_r (no x r) must have orthonormal columns: U_r holds the
// leading right singular vectors of Y and Z = Y U_r = U_Y,r S_r.  With
// X = Y^T (no x np):
//   1. the columns of X are ordered by decreasing norm and copied;
//   2. Householder QR of the copy, X P = Q1 R1 (reflectors and T factors
//      kept), then QR of R1^T = Q2 R2 (R2 only, k x k, k = min(np, no));
//   3. one-sided Jacobi on W = R2^T until its columns are orthogonal: then
//      X P = Q1 W Q2^T with W = U_W S, so the leading right singular vectors
//      of Y are U_r = Q1 U_W,r;
//   4. the rank rule of Eq. (eps) on the singular values;
//   5. U_W,r written out and multiplied by Q1 (block reflectors); the
//      caller forms Z = Y U_r with one product.
// The two QRs are the preconditioner of Drmac and Veselic (2008): Jacobi on
// R2^T needs markedly fewer sweeps than on R1^T, which needs fewer than on
// Y itself.
struct SvdPlan {
  int np = 0, no = 0, k = 0;
  JacobiPlan jp;
};
SvdPlan svd_plan(int np, int no, int force_bw = 0);
// Largest matrix side the SVD kernels take: the column sort and the rank
// rule hold one value per column in LDS (64 KB) and in 1024 x 8 registers,
// so np (the columns of X = Y^T, which bound the Jacobi size k as well)
// must not exceed it.
constexpr int kSvdMaxSide = 8192;
size_t svd_ws_doubles(const SvdPlan &p);
struct SvdResult {
  int rank = -1;
  double disc = 0.0, total = 0.0;
  int sweeps = 0;
  int err = 0;  // TTM_OK or a TTM_E* code
};
// Runs the SVD of Y (left intact) and writes U_r into u: as U_r^T (r x no,
// row-major: u[t*no + o]) when u_layout == SVD_U_T, as U_r (no x r,
// row-major: u[o*r + t]) when u_layout == SVD_U.  forced > 0 replaces the
// rank rule.  When sigma_out is not null the k
// singular values are written there in decreasing order.  Synchronises the
// stream once per Jacobi sweep (convergence test) and at the end.  trace > 0
// prints one line per SVD to stderr, trace > 1 also one per sweep.
enum { SVD_U_T = 0, SVD_U = 1 };
// With `all` set, the SVD also hands out every resolved singular vector for
// the reverse mode: the kg values above the rounding-noise level (kg >= r;
// the others' vectors are not resolved, see jacobi_rank_kernel) with their
// orthonormal vectors U_kg as the columns of all->u (no x kg, column-major),
// and the k singular values in decreasing order in all->sigma.  u then
// receives the first r of those columns in its layout.
struct SvdAll {
  double *u = nullptr;      // no x k capacity (column-major), written no x kg
  double *sigma = nullptr;  // k doubles, decreasing
  int kg = 0;               // out
};
// full_total (device, optional): the squared Frobenius norm of a larger
// matrix of which Y is a projection; the rank rule then counts the weight
// outside Y, full_total - ||Y||_F^2, as part of every tail (randomized SVD).
SvdResult svd_oside(const SvdPlan &p, const double *Y, double eps, int cap, int forced, int max_sweeps,
                    double *u, int u_layout, double *sigma_out, double *ws, hipStream_t s,
                    KernelTimer *timer, int trace, SvdAll *all = nullptr, const double *full_total = nullptr);

// Randomized truncated SVD of a swap matrix (rsvd.hip): Theta (m x n,
// column-major, ld m) ~ X' P' with P' = V_r^T (r x n, row-major, written to
// pt, orthonormal rows) from a subspace-iteration range finder with
// rsvd_sketch_cols(cap) columns and `power` iterations (products in the
// GemmPrec sketch_prec), then the Jacobi SVD
// of the projection.  Theta is left intact.  fallback = true (no error)
// when a CholeskyQR broke down or the estimated subspace error exceeded the
// acceptance bound `accept`: the caller runs the full SVD instead.  The
// test matrix is the SplitMix64 stream of `seed` from counter stream_pos.
struct RsvdResult {
  int rank = -1;
  double disc = 0.0, total = 0.0, flops = 0.0;
  double estimate = 0.0;  // the subspace-error estimate of the acceptance test
  int sweeps = 0;
  bool fallback = false;
  int err = 0;
};
int rsvd_sketch_cols(int cap);
// CholeskyQR2 of the p x l column-major Y in place (a testing hook):
// *fail_host = 1 when a Cholesky pivot broke down.  Synchronises s.
size_t cholqr2_ws_doubles(int p, int l);
hipError_t cholqr2(double *Y, int p, int l, double *ws, int *fail_host, hipStream_t s);
bool rsvd_eligible(int m, int n, int cap);
size_t rsvd_ws_doubles(int m, int n, int cap);
RsvdResult rsvd_oside(const double *Theta, int m, int n, int cap, int power, double accept, int max_sweeps,
                      double eps, int sketch_prec, uint64_t seed, int64_t stream_pos, double *pt, double *ws,
                      hipStream_t s, KernelTimer *timer, int trace);

// ------------------------------------------------------------------ reverse mode
// The record a TTM product keeps for its reverse mode: one entry per step,
// with device copies (in a caller workspace region) of what the step's
// adjoint reads.  Shapes are host integers.
struct TapeEntry {
  enum Kind { QR = 0, CONTRACT = 1, SWAP = 2, ROUND = 3, REVERSE = 4 };
  int kind = QR;
  int arr = 0;  // QR: the train moved (0 = A, 1 = B, 2 = the product block)
  int p = 0;    // QR: core index; CONTRACT: site; SWAP: position of P; ROUND: site
  int j = 0;    // SWAP: the site whose carriage moves
  // QR: M (m x n, row-major) = Q R with Q (m x k), R (k x n); the old next
  // core nxt (n x ncol) became R nxt; rl, d: the core's left bond and
  // physical dimension (m = rl d).
  // CONTRACT: K [dl, d, dm], X [dm, d, dr].
  // SWAP: P [dl, dp, dm], X [dm, dx, dr]; theta (m = dl dx by n = dp dr,
  // column-major); V (n x kg, column-major) the resolved right singular
  // vectors, sigma (min(m, n), decreasing); Z = theta V_r (m x r, row-major).
  // ROUND: M = Pi_i (m = rl d by n = rr, row-major); V (m x kg, column-major)
  // its resolved left singular vectors; sigma; Zt = S_r V_r^T (r x n); nxt
  // (n x ncol) the old next core.
  int m = 0, n = 0, k = 0, ncol = 0, r = 0, kg = 0;
  int rl = 0, d = 0, dl = 0, dp = 0, dm = 0, dx = 0, dr = 0;
  double *M = nullptr, *Q = nullptr, *R = nullptr, *nxt = nullptr;
  double *K = nullptr, *X = nullptr, *P = nullptr, *theta = nullptr, *V = nullptr, *sigma = nullptr,
         *Z = nullptr, *Zt = nullptr;
};
struct Tape {
  std::vector<TapeEntry> e;
  double *base = nullptr;
  size_t cap = 0, used = 0;  // doubles
  bool overflow = false;
  double *alloc(size_t n) {
    n = (n + 31) & ~(size_t)31;
    if (used + n > cap) {
      overflow = true;
      return nullptr;
    }
    double *p = base + used;
    used += n;
    return p;
  }
};

// The TTM product with every step recorded in `tape` (default gauge only:
// TTM_EUNSUPPORTED otherwise); *swapped reports whether the two trains
// traded places (move_factor = TTM_MOVE_SMALLER).
int run_ttm_taped(const ttm_tt *A, const ttm_tt *B, int chi_out, double tol, const ttm_options *opt,
                  ttm_tt_out *C, void *ws, size_t ws_bytes, hipStream_t st, ttm_stats *stats, Tape *tape,
                  bool *swapped);
// Sizes for the reverse mode (host only).
int vjp_sizes(const ttm_tt *A, const ttm_tt *B, int chi_out, const ttm_options *opt, size_t *fwd_ws,
              int64_t *tape_doubles, int64_t *max_core, int64_t *max_mn, int64_t *out_capacity);

// ------------------------------------------------------------------ conventional
// Dense transposed copy used by the variational driver:
// out[j][i] = in[i][j] for an m x n row-major input.
hipError_t launch_transpose(double *out, const double *in, int m, int n, hipStream_t s);

}  // namespace ttm

