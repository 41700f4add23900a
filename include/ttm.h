/*
 * ttm.h - C ABI of libttm: elementwise (Hadamard) product of two tensor
 * trains on one AMD Instinct MI355X (gfx950), FP64.
 *
 * Method: Michailidis, Fenton, Kiffner, "Tensor Train Multiplication"
 * (arXiv 2410.19747).  The product Omega = psi * phi of two TTs (problem
 * statement of Sec. II) is formed by the TTM algorithm of Sec. II.B:
 *   - the two trains are concatenated with the second one reversed
 *     (Eq. tensor);
 *   - carriages with the same site index are contracted through the local
 *     COPY tensor (Eq. contract);
 *   - the second train's carriages are moved next to their partners by
 *     Swap operations, each a contraction, an exchange of physical legs and
 *     a truncated SVD under the rule of Eq. (eps), in mixed-canonical gauge;
 *   - the gauge centre is moved with QR decompositions after every
 *     contraction.
 * conventional_multiply is the baseline of Sec. II.A: a single-site
 * variational fit of Omega to the MPO form of phi (Eq. PhiMPO) applied to
 * psi, never forming the Kronecker carriages of Eq. (carriageXi).
 *
 * Layout of a tensor train ("TT"): N cores; core i (0-based) is a row-major
 * array [r_i][d_i][r_{i+1}] of doubles (the carriage of Eq. (TT): one
 * r_i x r_{i+1} matrix per physical value), with r_0 = r_N = 1.  Core i
 * starts at element offsets[i] of the device buffer data.
 *
 * Ownership: the caller owns every pointer.  Input cores, the output buffer
 * and the workspace are device memory that the caller allocates; the
 * library allocates no device memory.  Host arrays (phys, bonds, offsets,
 * traces) are read or written only during the call.
 *
 * Blocking: every compute entry point enqueues its kernels on the given
 * stream (a hipStream_t; NULL is the default stream) and returns only when
 * they have finished, because the ranks chosen by each truncation are read
 * back to size the next step.  Output bonds and offsets are valid on return.
 *
 * Errors: 0 on success, a negative TTM_E* code otherwise; no exception
 * crosses this boundary.  Argument errors are detected on the host before
 * any GPU work is enqueued.  Calls on distinct streams with distinct
 * workspaces and outputs may run concurrently; calls sharing a workspace
 * must not overlap.
 */
#ifndef TTM_H
#define TTM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TTM_OK = 0,
  TTM_EINVAL = -1,       /* null pointer, bad size, bad option value          */
  TTM_ESHAPE = -2,       /* A and B differ in N or d, or a bond is not 1 at an end */
  TTM_EWORKSPACE = -3,   /* workspace missing or smaller than ttm_query says  */
  TTM_ECAPACITY = -4,    /* output buffer smaller than ttm_query says         */
  TTM_ENOCONV = -5,      /* an SVD did not converge within its sweep limit    */
  TTM_ENONFINITE = -6,   /* NaN or Inf met in the data                        */
  TTM_EHIP = -7,         /* a HIP runtime call failed                         */
  TTM_EFORCED = -8,      /* forced rank list too short or out of range        */
  TTM_EUNSUPPORTED = -9  /* dtype other than TTM_F64, an option that the     */
                         /* entry point does not take, or an SVD beyond the   */
                         /* kernels' size limit                               */
};

typedef enum { TTM_F64 = 0 } ttm_dtype;

/* Borrowed view of an input TT. */
typedef struct ttm_tt {
  int32_t n_sites;         /* 1 <= N <= 4096                                  */
  const int32_t *phys;     /* host [N]: 1 <= d_i <= 65536                     */
  const int32_t *bonds;    /* host [N+1]: r_0 = r_N = 1, 1 <= r_i <= 2^20     */
  const int64_t *offsets;  /* host [N]: element offset of core i in data      */
  const void *data;        /* device: doubles                                 */
  int32_t dtype;           /* TTM_F64                                         */
} ttm_tt;

/* Output TT: the caller provides the buffers, the library fills them. */
typedef struct ttm_tt_out {
  int32_t *bonds;          /* host [N+1], written                              */
  int64_t *offsets;        /* host [N], written (cores packed in site order)   */
  void *data;              /* device, at least `capacity` doubles              */
  int64_t capacity;        /* in doubles; must be >= ttm_query's out_capacity  */
} ttm_tt_out;

/* Options.  Fill with ttm_default_options, then change fields. */
typedef struct ttm_options {
  int32_t chi_mid;         /* rank cap of every swap; 0 = uncapped; -1 (default) = chi_out */
  int32_t final_round;     /* 1 (default): left-to-right truncated-SVD sweep with cap chi_out */
  int32_t max_sweeps;      /* conventional_multiply: sweep limit (default 10) */
  int32_t svd_max_sweeps;  /* Jacobi sweep limit per SVD (default 40)         */
  uint64_t seed;           /* conventional_multiply: initial-guess seed (default 12345) */
  const int32_t *forced_ranks; /* host [n_forced]: ranks replacing the rule of Eq. (eps),
                                  consumed in order (swaps, then the final sweep); NULL = none */
  int32_t n_forced;
  int32_t trace_cap;       /* capacity of the two trace arrays              */
  int32_t *rank_trace;     /* host [trace_cap]: rank of each truncating SVD, or NULL */
  double *discard_trace;   /* host [trace_cap]: discarded weight sum_{i>r} lambda_i^2, or NULL */
  int32_t profile;         /* 1: time every kernel launch with HIP events on the stream and
                              report per-class totals in ttm_stats (default 0) */
  int32_t contract_precision; /* arithmetic of the contractions (Eq. (contract) and the swap
                              merges): TTM_PREC_F64 (default), TTM_PREC_F32, TTM_PREC_BF16 or
                              TTM_PREC_BF16X3, the last three on the FP32 / BF16 matrix cores,
                              accumulated in FP32 within each 16-deep k-tile and in FP64
                              across k-tiles; QR, SVD and truncation stay FP64 */
  int32_t move_factor;     /* which train is reversed and moved by the swaps: TTM_MOVE_SECOND
                              (default: the second factor, psi of Sec. II.B) or TTM_MOVE_SMALLER
                              (the train with the smaller largest bond; ties: the second).  The
                              product is the same (A * B = B * A); exact intermediate bonds are
                              bounded by chi_fixed chi_moving^2 */
  int32_t gauge;           /* where each swap leaves the gauge centre: TTM_GAUGE_MOVING (default:
                              the singular values go into the carriage that moves on, so the
                              centre is inside the next pair) or TTM_GAUGE_RIGHT (as Sec. II.B
                              states it: into the right carriage of the pair, after which an LQ
                              factorisation of that carriage moves the centre into the moving
                              one before the next swap; one extra QR per swap, the same result
                              in exact arithmetic) */
  int32_t svd_mode;        /* the truncated SVD of each capped swap: TTM_SVD_JACOBI (default: the
                              full SVD, results within 1e-12 of an exact truncation) or
                              TTM_SVD_RANDOMIZED: a subspace-iteration range finder with 2 cap
                              columns (Halko, Martinsson and Tropp 2011, Alg. 4.4) whose products
                              take the contraction precision, CholeskyQR orthonormalisation in
                              FP64, then the FP64 Jacobi SVD of the 2 cap x 2 cap factor of the
                              projected matrix and the rule of Eq. (eps) with the uncaptured
                              weight counted as tail.  Used where 4 cap <= min(m, n) of the swap
                              matrix, with the default gauge and no forced ranks; other SVDs take
                              the full SVD, and so does any swap whose CholeskyQR breaks down or
                              whose estimated subspace error, (s_2cap / s_r)^(2q+1) s_r /
                              ||Theta||_F from the projected values, exceeds rsvd_tol.  With the
                              defaults about 3e-8 of the FP64 product on the turbulence workloads;
                              see rsvd_tol for FP64 parity.  Not with ttm_multiply_vjp
                              (TTM_EUNSUPPORTED) */
  int32_t rsvd_power;      /* TTM_SVD_RANDOMIZED: subspace iterations q, 0 <= q <= 64 (default 10);
                              the subspace error decays like (sigma_{2 cap + 1} / sigma_r)^(2q+1) */
  double rsvd_tol;         /* TTM_SVD_RANDOMIZED: the acceptance bound on the estimated subspace error,
                              0 < rsvd_tol <= 1 (default 2e-8); swaps above it take the full SVD.  With
                              rsvd_power = 20 and rsvd_tol = 1e-14 the products of the turbulence
                              workloads agree with the full SVD's to FP64 parity (1e-12) */
} ttm_options;

/* Values of ttm_options.svd_mode. */
enum { TTM_SVD_JACOBI = 0, TTM_SVD_RANDOMIZED = 1 };

/* Values of ttm_options.move_factor and ttm_options.gauge. */
enum { TTM_MOVE_SECOND = 0, TTM_MOVE_SMALLER = 1 };
enum { TTM_GAUGE_MOVING = 0, TTM_GAUGE_RIGHT = 1 };

/* Values of ttm_options.contract_precision: operands of the contractions in
 * FP64; rounded to FP32; rounded to BF16; or each split into three BF16
 * terms of which the six leading products are accumulated (about FP32
 * accuracy on the BF16 matrix cores). */
enum { TTM_PREC_F64 = 0, TTM_PREC_F32 = 1, TTM_PREC_BF16 = 2, TTM_PREC_BF16X3 = 3 };

/* Kernel classes of ttm_stats.kernel_ms / kernel_launches. */
enum {
  TTM_KC_GEMM = 0,         /* contractions, merges, R and S V^T products          */
  TTM_KC_QR = 1,           /* Householder QR: gauge moves and the SVDs' preconditioner */
  TTM_KC_JAC_GRAM = 2,     /* Jacobi SVD: partial Gram matrices of block pairs     */
  TTM_KC_JAC_SOLVE = 3,    /* Jacobi SVD: diagonalisation of each block-pair Gram  */
  TTM_KC_JAC_OTHER = 4,    /* SVD: ordering, R^T, convergence, norms, sort, write  */
  TTM_KC_OTHER = 5,        /* copies, reversal, transposes, checks                 */
  TTM_KC_JAC_APPLY = 6,    /* Jacobi SVD: rotation of the column blocks            */
  TTM_KC_COUNT = 7
};

/* Statistics of one call. */
typedef struct ttm_stats {
  int32_t max_bond;        /* largest bond present in the chain during the call */
  int32_t n_contract;      /* contractions (Eq. contract): N                   */
  int32_t n_swap;          /* swaps: N(N-1)/2                                  */
  int32_t n_qr;            /* QR gauge moves, including input canonicalisation */
  int32_t n_svd;           /* truncating SVDs (swaps + final sweep)            */
  int32_t n_trace;         /* entries written to the traces                    */
  int32_t sweeps;          /* conventional: sweeps run; TTM: total Jacobi sweeps */
  int32_t jacobi_max_sweeps; /* most Jacobi sweeps any one SVD needed          */
  double discarded_sq_sum; /* sum over SVDs of the discarded weight            */
  double error_bound;      /* sum over SVDs of sqrt(discarded weight): bounds ||C - A*B|| */
  double model_flops;      /* algorithmic flops of the recorded schedule       */
  double svd_model_flops;  /* the part of model_flops spent in SVDs            */
  double jacobi_solve_flops; /* arithmetic of the Jacobi pair solves themselves (Gram
                              partial sums, the in-LDS rotation sweep, the
                              re-orthogonalisation), counted for every pair
                              launched: the solve kernel's own work       */
  size_t peak_ws_bytes;    /* workspace bytes the call used                    */
  double kernel_ms[TTM_KC_COUNT];        /* with opt.profile: summed event time per class */
  int64_t kernel_launches[TTM_KC_COUNT]; /* with opt.profile: timed regions per class: one launch
                                            each, except a whole QR or a column reordering,
                                            which are timed as one region */
  int32_t n_rsvd;          /* svd_mode TTM_SVD_RANDOMIZED: swaps truncated by the randomized SVD */
  int32_t n_rsvd_fallback; /* ... and eligible swaps that fell back to the full SVD (CholeskyQR
                              breakdown or an estimate above the acceptance bound) */
} ttm_stats;

/* Defaults: chi_mid = -1 (same as chi_out), final_round = 1, max_sweeps = 10,
 * svd_max_sweeps = 40, seed = 12345, no forced ranks, no traces, FP64
 * contractions. */
void ttm_default_options(ttm_options *opt);

/* Sizes for ttm_multiply (host only, no GPU work).  Writes the workspace
 * bytes and the output capacity (doubles) needed for these inputs and
 * options.  With final_round set, out_capacity = sum_i c_i d_i c_{i+1} with
 * c_i = min(prod_{k<i} d_k, prod_{k>=i} d_k, chi_out, chi_mid if > 0) (the
 * final sweep cannot raise a bond the swaps capped).  Without it the bonds
 * are those the swaps leave: at most the swap cap, and bounded by the cuts
 * of the intermediate chain, where a site not yet contracted contributes its
 * dimension twice, so a bond can exceed the product's structural bound.
 * Either output pointer may be NULL.
 * TTM_EINVAL also when a QR or SVD step of the schedule would take a matrix
 * longer than 2^30 on a side or holding more than 2^36 entries, or a core
 * would exceed 2^33 entries.  TTM_EUNSUPPORTED when a truncated SVD of the
 * schedule would have more than 8192 rows on the side that is kept
 * orthonormal: a swap merging (D_l, d) x (d, D_r) with D_l d > 8192, or a
 * final-sweep bond above 8192 (the SVD kernels hold one value per column of
 * that side in 64 KB of LDS).  The bound is checked on the symbolic schedule
 * with every rank at its cap, before any GPU work: with chi_mid = 0 or a
 * chi_mid above chi_out it can reject inputs whose actual ranks would fit. */
int ttm_query(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, const ttm_options *opt,
              size_t *ws_bytes, int64_t *out_capacity);

/* C = A * B elementwise by TTM (Sec. II.B).  tol is the eps of Eq. (eps),
 * applied relative to each SVD's total weight; chi_out caps the output bonds.
 * ws: device workspace of ws_bytes >= ttm_query's size.  stream: hipStream_t. */
int ttm_multiply(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol, ttm_tt_out *C,
                 void *ws, size_t ws_bytes, void *stream);

/* As ttm_multiply, with options (NULL = defaults) and statistics (may be NULL). */
int ttm_multiply_ex(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol,
                    ttm_tt_out *C, void *ws, size_t ws_bytes, void *stream,
                    const ttm_options *opt, ttm_stats *stats);

/* Size in bytes of the static device workspace of ttm_multiply_static. */
#define TTM_STATIC_WS_BYTES ((size_t)32 << 20)

/* ttm_multiply_ex without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The workspace is a static device array of
 * TTM_STATIC_WS_BYTES (32 MiB) that the library holds on every device it
 * runs on until the process ends; the call allocates nothing and creates no
 * HIP object.  Inputs, output, options, statistics, blocking and return codes
 * are those of ttm_multiply_ex, and the result is bitwise the one
 * ttm_multiply_ex gives for the same arguments.  Limits:
 *   - a product whose ttm_query workspace exceeds TTM_STATIC_WS_BYTES returns
 *     TTM_EWORKSPACE before any GPU work (ttm_last_error gives both sizes):
 *     32 MiB holds, e.g., 8 sites of d = 8 at bond 64, not at bond 128;
 *   - opt->profile must be 0 (event timing creates HIP events): TTM_EINVAL.
 * The array of a device is shared by every call on that device (the HIP
 * device current in the calling thread) and keeps the last call's contents;
 * each call clears what it reads before writing.  Calls that overlap in time
 * on one device, from several threads or streams, race on the array and give
 * wrong results: serialise them. */
int ttm_multiply_static(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol, ttm_tt_out *C,
                        void *stream, const ttm_options *opt, ttm_stats *stats);

/* n independent products C[i] = A[i] * B[i] by TTM (Sec. II.B) in one call,
 * for workloads of many products at uneven bonds, such as the nine terms
 * u_j d_j u_i of the advection term that motivates the method (Sec. I).
 * Product i takes chi_out[i], tol[i], options opt[i] (opt NULL: defaults for
 * all), workspace ws[i] of ws_bytes[i] >= ttm_query's size and output C[i];
 * stats (NULL or n entries) receives each product's statistics.  Arrays are
 * host arrays of n entries.
 * Scheduling: the library creates min(n, n_streams) streams of its own
 * (1 <= n_streams <= 4), each of which first waits for the work already
 * enqueued on `stream` (the caller's hipStream_t, which produced the
 * inputs), and drives each from a host thread that takes products from a
 * queue ordered by decreasing estimated cost (swap count times the cube of
 * the swap-matrix side) and runs them as ttm_multiply_ex would.  A product
 * is a chain of small dependent launches, so products overlap only on
 * distinct hardware queues; the streams are created with a CU mask of every
 * CU, which gives each a hardware queue of its own rather than one of the
 * runtime's shared default queues.  The streams (and their queues) are
 * created and destroyed within each call, so the call suits batches whose
 * products take milliseconds or more.  Each product's result is the one
 * ttm_multiply_ex gives for the same arguments.
 * Checks: every product is validated (as ttm_query, plus the workspace and
 * output sizes and a finite tol >= 0) before any starts, and workspaces and
 * outputs must not overlap one another (TTM_EINVAL).  The call returns when
 * every product has finished and its streams are destroyed: 0 if all
 * succeeded, else the code of the lowest-index failure; status (NULL or n
 * entries) receives every product's code, and a failed product does not
 * stop the others.  The HIP device current in the calling thread is used. */
int ttm_multiply_batch(int32_t n, const ttm_tt *A, const ttm_tt *B, const int32_t *chi_out,
                       const double *tol, ttm_tt_out *C, void *const *ws, const size_t *ws_bytes,
                       const ttm_options *opt, ttm_stats *stats, int32_t n_streams, void *stream,
                       int32_t *status);

/* Gradient of the loss L = <W, A*B> = sum_x W(x) A(x) B(x) with respect to
 * the cores of A and B: the elementwise product of Sec. II followed by the
 * inner product with a fixed train W (the paper has no gradients).  L is
 * linear in every core, so dL/dA_k contracts all other cores: the left
 * environment of the sites before k, cores k of W and B, and the right
 * environment of the sites after k (three-train environments).  Wherever the
 * truncations of TTM (Sec. II.B) drop nothing, TTM(A, B) is A*B and this is
 * the gradient of <W, TTM(A, B)>; where they do drop weight it is the
 * gradient of the exact product that TTM approximates, not that of the
 * truncated product (ttm_multiply_vjp differentiates that).
 * The environments are recomputed on every call: a right-to-left sweep
 * keeps the right ones in ws, then one left-to-right sweep forms both
 * gradients at each site and the next left environment.
 * W, A, B: same N and physical dimensions, any bonds (r_0 = r_N = 1).
 * contract_precision: TTM_PREC_* for the environment contractions (FP64
 * storage either way).  value: host, receives L.  dA, dB: device buffers
 * laid out like A's and B's data (core k of the gradient at the same offset
 * as core k of the train), or NULL to skip; with both NULL only L is formed
 * and the right sweep is skipped.  ws: ttm_inner_grad_query's bytes, which
 * returns TTM_EINVAL when an environment or intermediate would exceed 2^36
 * doubles or a contraction extent 2^30.
 * Blocking like the other entry points; TTM_ENONFINITE if L is not finite. */
int ttm_inner_grad_query(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, size_t *ws_bytes);
int ttm_inner_grad(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, int32_t contract_precision,
                   double *value, double *dA, double *dB, void *ws, size_t ws_bytes, void *stream);

/* As ttm_inner_grad_query / ttm_inner_grad, with the right environments
 * kept at checkpoints and recomputed between them instead of all stored.
 * env_stride = 1: all N stored (the plain entry points).  env_stride = s >= 2:
 * F_N, F_{N-s}, F_{N-2s}, ... are kept; when the left sweep reaches a site
 * whose F_{k+1} lies between two checkpoints, the environments of that
 * segment are recomputed from the checkpoint above it into s - 1 further
 * buffers.  Memory: ceil(N / s) + s - 1 environments of the largest size
 * instead of N + 1; work: at most twice the right sweep.  env_stride = 0:
 * s = ceil(sqrt(N)) (at least 2).  Values and gradients are bitwise those of
 * the stored form (the same products on the same inputs).  A negative
 * env_stride is TTM_EINVAL. */
int ttm_inner_grad_query_ex(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, int32_t env_stride,
                            size_t *ws_bytes);
int ttm_inner_grad_ex(const ttm_tt *W, const ttm_tt *A, const ttm_tt *B, int32_t contract_precision,
                      double *value, double *dA, double *dB, int32_t env_stride, void *ws, size_t ws_bytes,
                      void *stream);

/* Reverse mode of the TTM product (the paper has no gradients): given the
 * cotangent Cbar of the output cores (for a loss L(C), Cbar = dL/dC, laid out
 * like C), the cotangents dA = dL/dA and dB = dL/dB of the input cores,
 * through every step of Sec. II.B as computed: the canonicalising QR sweeps,
 * the reversal of the second train (Eq. tensor), the contractions
 * (Eq. contract), the QR gauge moves, the swaps' merges and truncated SVDs
 * (Fig. 1C, Eq. (eps)) and the final rounding sweep.  The ranks chosen by the
 * truncations are piecewise constant and held at the forward pass's.
 * The call runs the product again with every step's operands recorded in
 * ws, writes it to C like ttm_multiply_ex, checks that Cbar has its bonds
 * (TTM_ESHAPE otherwise), then undoes the steps in reverse order on the
 * device.  A truncated SVD's adjoint weights each pair of a kept and a dropped
 * singular value by 1/(sigma_i^2 - sigma_j^2) and the unresolved and null
 * directions by 1/sigma_i^2: it is defined where the kept values are
 * separated from the dropped ones, and its error grows as 1/gap.  A QR
 * adjoint solves with R^T: the unfoldings must have full rank (input bonds
 * within the structural bounds).  Default gauge and the full swap SVD only
 * (TTM_EUNSUPPORTED for TTM_GAUGE_RIGHT or TTM_SVD_RANDOMIZED, from both
 * calls); move_factor is honoured.  dA, dB: device buffers laid out
 * like A's and B's data.  ws: ttm_vjp_query's bytes (the product's own
 * workspace, the record of its steps, the cotangents and scratch).  opt->profile
 * must be 0.  Blocking like the other entry points. */
int ttm_vjp_query(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, const ttm_options *opt,
                  size_t *ws_bytes, int64_t *out_capacity);
int ttm_multiply_vjp(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol, const ttm_options *opt,
                     const ttm_tt *Cbar, ttm_tt_out *C, double *dA, double *dB, void *ws, size_t ws_bytes,
                     void *stream, ttm_stats *stats);

/* Sizes for conventional_multiply (host only).  The fit keeps the structural
 * bonds capped at chi_out: out_capacity = sum_i c_i d_i c_{i+1} with
 * c_i = min(prod_{k<i} d_k, prod_{k>=i} d_k, chi_out).  TTM_EINVAL when an
 * environment or a local tensor would exceed 2^36 doubles, or a QR unfolding
 * 2^30 on a side. */
int conventional_query(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, const ttm_options *opt,
                       size_t *ws_bytes, int64_t *out_capacity);

/* C ~ A * B by the single-site variational fit of Sec. II.A with bonds
 * capped at chi_out.  tol: stop when the norm of the centre changes by at
 * most tol (relative) between two full sweeps. */
int conventional_multiply(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol,
                          ttm_tt_out *C, void *ws, size_t ws_bytes, void *stream);

int conventional_multiply_ex(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol,
                             ttm_tt_out *C, void *ws, size_t ws_bytes, void *stream,
                             const ttm_options *opt, ttm_stats *stats);

/* Static message for an error code. */
const char *ttm_strerror(int code);

/* Text describing the last failure of a compute call (ttm_multiply*,
 * conventional_multiply*, ttm_inner_grad, ttm_multiply_batch) made on the
 * calling thread: for TTM_EHIP the step that was being enqueued or
 * synchronised and the HIP runtime's name and message for the error, for
 * TTM_ENOCONV and TTM_ENONFINITE the SVD concerned.  Empty ("") after a call
 * that succeeded or failed only in argument checks.  The string belongs to
 * the library and stays valid until the thread's next compute call. */
const char *ttm_last_error(void);

/* Library version string. */
const char *ttm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TTM_H */
