// Randomized truncated SVD of a swap matrix (TTM_SVD_RANDOMIZED): a range
// finder by subspace iteration (Halko, Martinsson and Tropp, SIAM Review 53
// (2011), Algorithms 4.3 and 4.4), followed by the one-sided Jacobi SVD of
// the projected matrix.
//
// The Swap of Sec. II.B keeps r = min(r_eps, cap) singular triplets of an
// m x n matrix Theta whose sides are d times the bond, so a cap of chi keeps
// about one eighth of the spectrum.  With l = 2 cap columns:
//   1. Y = Theta^T Omega, Omega (m x l) uniform in [-1, 1) from a
//      counter-based SplitMix64 stream; Y <- orth(Y);
//   2. q times: Z = orth(Theta Y), Y = orth(Theta^T Z); then a second
//      orthonormalisation pass on Y;
//   3. B = Theta Y (m x l, FP64) = Q_B R_B by CholeskyQR2, and the SVD of
//      the l x l factor R_B (B's values and right vectors V_B) by the
//      one-sided Jacobi driver (svd_oside);
//   4. the rule of Eq. (eps) on those values with the weight that the l
//      directions do not capture, ||Theta||_F^2 - ||B||_F^2, added to every
//      tail;
//   5. V_r = Y V_B,r: P' = V_r^T (orthonormal rows), and the caller forms
//      X' = Theta V_r.
// The products of steps 1-2 take the operand precision of the contractions
// (FP64, or FP32 / BF16 terms on the matrix cores with FP32 accumulation
// within each 16-deep k-tile and FP64 across tiles): they only steer the
// subspace.  orth() is one CholeskyQR pass (G = Y^T Y = R^T R, Y <- Y R^-1)
// on the intermediate bases and two (CholeskyQR2; Yamamoto et al., ETNA 44
// (2015)) on the final one, all in FP64: a blocked Cholesky (one workgroup
// per 64 x 64 diagonal block, matrix-core products for the panels and
// trailing updates) and a blocked triangular solve.  CholeskyQR needs
// kappa(Y) well below u^(-1/2); a pivot that falls to the rounding level of
// its column's norm (rank-deficient Theta, or kappa(Y) beyond ~1e7) raises
// a flag, and the caller then runs the full SVD on the same matrix instead.
//
// Accuracy: the subspace error decays like (sigma_{l+1} / sigma_r)^(2q+1).
// After the SVD it is estimated from the computed values, rho =
// sigma_l / sigma_r, as rho^(2q+1) sigma_r / ||Theta||_F (the move of the
// kept part relative to the chain's norm); a swap whose estimate exceeds
// the acceptance bound (default 2e-8; a spectrum too flat at the cut) also
// takes the full SVD.  With the defaults (q = 10) the products of the
// turbulence workloads stay within about 3e-8 of the FP64 product (the
// mixed-precision bar is 1e-6); FP32 sketch products add about 5e-7.  With
// q = 20 and a bound of 1e-14 they agree with the full SVD's to FP64
// parity (below 1e-13).
#include <math.h>
#include <stdio.h>

#include <algorithm>

#include "ttm_internal.h"

namespace ttm {

namespace {
constexpr int CNB = 64;   // Cholesky block
constexpr int CNT = 256;  // threads of the diagonal-block kernel
constexpr double kU = 2.220446049250313e-16;

size_t r32(size_t n) { return (n + 31) & ~(size_t)31; }

// Squared Frobenius norm in two fixed-order passes: 256 block partials
// (grid-stride over x), then their sum by one block.
constexpr int SQB = 256;
__global__ __launch_bounds__(256) void sumsq_part_kernel(const double *__restrict__ x, int64_t n,
                                                         double *__restrict__ part) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)SQB * 256) acc = fma(x[e], x[e], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ __launch_bounds__(256) void sumsq_final_kernel(const double *__restrict__ part, double *__restrict__ out) {
  __shared__ double red[4];
  double acc = part[threadIdx.x];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = (red[0] + red[1]) + (red[2] + red[3]);
}

// dst[i] = G[i * ld + i], i < n.
__global__ void diag_kernel(const double *__restrict__ G, int ld, int n, double *__restrict__ dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = G[(int64_t)i * ld + i];
}

// 1 / sqrt(d) for d > 0: the hardware estimate and two Newton steps.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
  y = y * fma(-0.5 * d * y, y, 1.5);
  y = y * fma(-0.5 * d * y, y, 1.5);
  return y;
}

// Cholesky of the w x w diagonal block at G (row-major, ld), upper:
// G_kk = R^T R, one workgroup, padded to CNB with the identity.  Writes
// R^-1 (upper triangular, CNB x CNB row-major, zero below the diagonal) to
// rinv, and R itself to rout (row-major, ld, w x w) when rout is set.  gd
// holds the block's diagonal as it was before any elimination (the squared
// column norms); a pivot at or below 64 u gd_j, or not positive, sets *fail
// and is replaced by gd_j (or 1) so that everything stays finite.
// Thread t owns the 4 x 4 tile (t / 16, t % 16) of the block in registers.
// Factorisation, four rows per step: the sixteen threads of tile row s
// publish rows 4s .. 4s+3 in LDS (double-buffered), one barrier; every
// thread factors the 4 x 4 diagonal block U^T U itself, forms the block's
// rows of R at its tile's four columns and four rows by U^-T, and tiles
// below and right of the block take the rank-four update; tile row s
// becomes its rows of R.  Inverse, by block rows from the bottom: the
// threads of tile row b form X_b = U_bb^-1 (their accumulated right-hand
// side) and publish it; after one barrier every tile row above subtracts
// R_a,b X_b from its accumulator.
__device__ __forceinline__ void inv4_upper(const double (&u)[4][4], double (&x)[4][4]) {
  const double d0 = 1.0 / u[0][0], d1 = 1.0 / u[1][1], d2 = 1.0 / u[2][2], d3 = 1.0 / u[3][3];
  x[0][0] = d0; x[1][1] = d1; x[2][2] = d2; x[3][3] = d3;
  x[1][0] = x[2][0] = x[2][1] = x[3][0] = x[3][1] = x[3][2] = 0.0;
  x[0][1] = -u[0][1] * d1 * d0;
  x[1][2] = -u[1][2] * d2 * d1;
  x[2][3] = -u[2][3] * d3 * d2;
  x[0][2] = -(u[0][1] * x[1][2] + u[0][2] * d2) * d0;
  x[1][3] = -(u[1][2] * x[2][3] + u[1][3] * d3) * d1;
  x[0][3] = -(u[0][1] * x[1][3] + u[0][2] * x[2][3] + u[0][3] * d3) * d0;
}

__global__ __launch_bounds__(CNT) void chol_diag_kernel(const double *__restrict__ G, int ld, int w,
                                                        const double *__restrict__ gd, double *__restrict__ rinv,
                                                        double *__restrict__ rout, int *__restrict__ fail) {
  static_assert(CNB == 64 && CNT == 256, "one 4 x 4 tile per thread");
  constexpr int LD = CNB + 2;  // 16-byte aligned rows
  __shared__ __align__(16) double R[CNB][LD];
  __shared__ __align__(16) double Xs[CNB][LD];
  __shared__ __align__(16) double rb[2][4][CNB];
  __shared__ double piv[CNB];
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int t = threadIdx.x, ti = t >> 4, tk = t & 15, i0 = 4 * ti, k0 = 4 * tk;
  double a[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int i = i0 + r, k = k0 + c;
      a[r][c] = (i < w && k < w) ? G[(int64_t)i * ld + k] : (i == k ? 1.0 : 0.0);
    }
  if (t < CNB) piv[t] = (t < w) ? gd[t] : 1.0;
  bool bad = false;
  auto pivot = [&](double d, double ref, double &r, double &ri) {
    const bool ok = d > 64.0 * kU * ref;  // false for NaN as well
    bad |= !ok;
    d = ok ? d : (ref > 0.0 ? ref : 1.0);
    ri = rsqrt_nr(d);
    r = d * ri;
  };
  for (int st = 0; st < CNB / 4; ++st) {
    const int j0 = 4 * st;
    double (*buf)[CNB] = rb[st & 1];
    if (ti == st) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        *(d2 *)&buf[r][k0] = d2{a[r][0], a[r][1]};
        *(d2 *)&buf[r][k0 + 2] = d2{a[r][2], a[r][3]};
      }
    }
    __syncthreads();
    // U^T U = the 4 x 4 diagonal block (upper entries of the published rows)
    double u[4][4], iv[4];
    pivot(buf[0][j0], piv[j0], u[0][0], iv[0]);
    u[0][1] = buf[0][j0 + 1] * iv[0];
    u[0][2] = buf[0][j0 + 2] * iv[0];
    u[0][3] = buf[0][j0 + 3] * iv[0];
    pivot(buf[1][j0 + 1] - u[0][1] * u[0][1], piv[j0 + 1], u[1][1], iv[1]);
    u[1][2] = (buf[1][j0 + 2] - u[0][1] * u[0][2]) * iv[1];
    u[1][3] = (buf[1][j0 + 3] - u[0][1] * u[0][3]) * iv[1];
    pivot(buf[2][j0 + 2] - u[0][2] * u[0][2] - u[1][2] * u[1][2], piv[j0 + 2], u[2][2], iv[2]);
    u[2][3] = (buf[2][j0 + 3] - u[0][2] * u[0][3] - u[1][2] * u[1][3]) * iv[2];
    pivot(buf[3][j0 + 3] - u[0][3] * u[0][3] - u[1][3] * u[1][3] - u[2][3] * u[2][3], piv[j0 + 3], u[3][3], iv[3]);
    u[1][0] = u[2][0] = u[2][1] = u[3][0] = u[3][1] = u[3][2] = 0.0;
    // rows j0 .. j0+3 of R at a column k: x = U^-T g_k (forward substitution)
    auto solve = [&](int k, double &x0, double &x1, double &x2, double &x3) {
      const double g0 = buf[0][k], g1 = buf[1][k], g2 = buf[2][k], g3 = buf[3][k];
      x0 = g0 * iv[0];
      x1 = (g1 - u[0][1] * x0) * iv[1];
      x2 = (g2 - u[0][2] * x0 - u[1][2] * x1) * iv[2];
      x3 = (g3 - u[0][3] * x0 - u[1][3] * x1 - u[2][3] * x2) * iv[3];
    };
    double xk[4][4], xi[4][4];  // [block row][own column / own row]
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      solve(k0 + c, xk[0][c], xk[1][c], xk[2][c], xk[3][c]);
      solve(i0 + c, xi[0][c], xi[1][c], xi[2][c], xi[3][c]);
    }
    const bool upd = (ti > st) && (tk > st);
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double nv = fma(-xi[3][r], xk[3][c], fma(-xi[2][r], xk[2][c],
                              fma(-xi[1][r], xk[1][c], fma(-xi[0][r], xk[0][c], a[r][c]))));
        const double rrow = (tk > st) ? xk[r][c] : (tk == st ? u[r][c] : 0.0);
        a[r][c] = (ti == st) ? rrow : (upd ? nv : a[r][c]);
      }
  }
  if (bad && t == 0) atomicOr(fail, 1);
  // R (zero below the diagonal tiles) into LDS, and out when asked for
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double z = (ti > tk) ? 0.0 : 1.0;
    *(d2 *)&R[i0 + r][k0] = d2{a[r][0] * z, a[r][1] * z};
    *(d2 *)&R[i0 + r][k0 + 2] = d2{a[r][2] * z, a[r][3] * z};
    if (rout && i0 + r < w) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (k0 + c < w) rout[(int64_t)(i0 + r) * ld + k0 + c] = a[r][c] * z;
    }
  }
  __syncthreads();
  // R^-1 by block rows from the bottom; acc is this tile's right-hand side.
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = (ti == tk && r == c) ? 1.0 : 0.0;
  for (int bb = CNB / 4 - 1; bb >= 0; --bb) {
    if (ti == bb) {
      double ub[4][4], ui[4][4], xo[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) ub[r][c] = R[4 * bb + r][4 * bb + c];
      inv4_upper(ub, ui);
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          double v = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) v = fma(ui[r][q], acc[q][c], v);
          xo[r][c] = (tk >= bb) ? v : 0.0;
        }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        *(d2 *)&Xs[i0 + r][k0] = d2{xo[r][0], xo[r][1]};
        *(d2 *)&Xs[i0 + r][k0 + 2] = d2{xo[r][2], xo[r][3]};
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = xo[r][c];
      }
    }
    __syncthreads();
    if (ti < bb) {
      double rt[4][4], xt[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const d2 r01 = *(const d2 *)&R[i0 + r][4 * bb], r23 = *(const d2 *)&R[i0 + r][4 * bb + 2];
        rt[r][0] = r01.x; rt[r][1] = r01.y; rt[r][2] = r23.x; rt[r][3] = r23.y;
        const d2 x01 = *(const d2 *)&Xs[4 * bb + r][k0], x23 = *(const d2 *)&Xs[4 * bb + r][k0 + 2];
        xt[r][0] = x01.x; xt[r][1] = x01.y; xt[r][2] = x23.x; xt[r][3] = x23.y;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
          acc[r][c] = fma(-rt[r][3], xt[3][c], fma(-rt[r][2], xt[2][c],
                          fma(-rt[r][1], xt[1][c], fma(-rt[r][0], xt[0][c], acc[r][c]))));
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) rinv[(i0 + r) * CNB + k0 + c] = (tk >= ti) ? acc[r][c] : 0.0;
}

hipError_t launch_chol_diag(const double *G, int ld, int w, const double *gd, double *rinv, double *rout,
                            int *fail, hipStream_t s) {
  hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(CNT), 0, s, G, ld, w, gd, rinv, rout, fail);
  return hipGetLastError();
}

constexpr int64_t kGramPart = (int64_t)2 << 20;  // split-K scratch of the Gram product (doubles)

// Buffers of one CholeskyQR (carved from the workspace).
struct CqrBufs {
  double *G = nullptr;     // l x l
  double *Rf = nullptr;    // l x l: the off-diagonal blocks of R
  double *rinv = nullptr;  // nb x CNB x CNB
  double *gd = nullptr;    // l
  double *part = nullptr;  // kGramPart
};
size_t cqr_doubles(int l) {
  const size_t nb = (l + CNB - 1) / CNB;
  return 2 * r32((size_t)l * l) + r32(nb * CNB * CNB) + r32((size_t)l) + r32((size_t)kGramPart);
}
CqrBufs cqr_carve(int l, double *base) {
  CqrBufs b;
  double *q = base;
  auto adv = [&](size_t n) {
    double *x = q;
    q += r32(n);
    return x;
  };
  const size_t nb = (l + CNB - 1) / CNB;
  b.G = adv((size_t)l * l);
  b.Rf = adv((size_t)l * l);
  b.rinv = adv(nb * CNB * CNB);
  b.gd = adv((size_t)l);
  b.part = adv((size_t)kGramPart);
  return b;
}

// One CholeskyQR pass: Q = Y R^-1 with Y^T Y = R^T R, Y and Q column-major
// p x l (ld p).  Y is overwritten (the block solve updates it in place).
// With want_r, b.Rf holds all of R afterwards (row-major, zero below the
// diagonal); otherwise only its blocks right of the diagonal blocks.
hipError_t cholqr(double *Y, int p, int l, double *Q, const CqrBufs &b, int *fail, hipStream_t s,
                  KernelTimer *timer, bool want_r = false) {
  Timed tm(timer, KC_QR, s);
  hipError_t e;
  if (want_r && (e = launch_fill(b.Rf, 0.0, (int64_t)l * l, s)) != hipSuccess) return e;
  {
    // G = Y^T Y (row-major, ld l), K split when the output is small
    GemmArgs g;
    g.M = l; g.N = l; g.K = p;
    g.A = Y; g.a_rs = p; g.a_cs = 1;
    g.B = Y; g.b_rs = 1; g.b_cs = p;
    g.C = b.G; g.c_rs1 = l; g.c_cs1 = 1;
    g.part = b.part; g.part_doubles = kGramPart;
    if ((e = launch_gemm(g, s)) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(diag_kernel, dim3((l + 255) / 256), dim3(256), 0, s, b.G, l, l, b.gd);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int nb = (l + CNB - 1) / CNB;
  // Blocked Cholesky, right-looking: R_kk from the block, then
  // R_k,rest = R_kk^-T G_k,rest and G_rest,rest -= R_k,rest^T R_k,rest.
  for (int kb = 0; kb < nb; ++kb) {
    const int b0 = kb * CNB, w = std::min(CNB, l - b0), rest = l - b0 - w;
    double *rk = b.rinv + (int64_t)kb * CNB * CNB;
    double *rout = want_r ? b.Rf + (int64_t)b0 * l + b0 : nullptr;
    if ((e = launch_chol_diag(b.G + (int64_t)b0 * l + b0, l, w, b.gd + b0, rk, rout, fail, s)) != hipSuccess)
      return e;
    if (rest == 0) break;
    GemmArgs g;
    g.M = w; g.N = rest; g.K = w;
    g.A = rk; g.a_rs = 1; g.a_cs = CNB;  // (R_kk^-1)^T
    g.B = b.G + (int64_t)b0 * l + b0 + w; g.b_rs = l; g.b_cs = 1;
    g.C = b.Rf + (int64_t)b0 * l + b0 + w; g.c_rs1 = l; g.c_cs1 = 1;
    if ((e = launch_gemm(g, s)) != hipSuccess) return e;
    GemmArgs u;
    u.M = rest; u.N = rest; u.K = w;
    u.A = b.Rf + (int64_t)b0 * l + b0 + w; u.a_rs = 1; u.a_cs = l;
    u.B = b.Rf + (int64_t)b0 * l + b0 + w; u.b_rs = l; u.b_cs = 1;
    u.C = b.G + (int64_t)(b0 + w) * l + b0 + w; u.c_rs1 = l; u.c_cs1 = 1;
    u.alpha = -1.0; u.beta = 1.0;
    if ((e = launch_gemm(u, s)) != hipSuccess) return e;
  }
  // Q = Y R^-1 by block columns: Q_k = Y_k R_kk^-1, then Y_rest -= Q_k R_k,rest.
  for (int kb = 0; kb < nb; ++kb) {
    const int b0 = kb * CNB, w = std::min(CNB, l - b0), rest = l - b0 - w;
    GemmArgs g;
    g.M = p; g.N = w; g.K = w;
    g.A = Y + (int64_t)b0 * p; g.a_rs = 1; g.a_cs = p;
    g.B = b.rinv + (int64_t)kb * CNB * CNB; g.b_rs = CNB; g.b_cs = 1;
    g.C = Q + (int64_t)b0 * p; g.c_rs1 = 1; g.c_cs1 = p;
    if ((e = launch_gemm(g, s)) != hipSuccess) return e;
    if (rest == 0) break;
    GemmArgs u;
    u.M = p; u.N = rest; u.K = w;
    u.A = Q + (int64_t)b0 * p; u.a_rs = 1; u.a_cs = p;
    u.B = b.Rf + (int64_t)b0 * l + b0 + w; u.b_rs = l; u.b_cs = 1;
    u.C = Y + (int64_t)(b0 + w) * p; u.c_rs1 = 1; u.c_cs1 = p;
    u.alpha = -1.0; u.beta = 1.0;
    if ((e = launch_gemm(u, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Buffers of one randomized SVD.
struct RsvdBufs {
  double *Om = nullptr;    // the test matrix (m x l), then a basis
  double *Y = nullptr;     // a basis
  double *T = nullptr;     // a basis (each max(m, n) x l)
  double *B = nullptr;     // m x l
  double *vbt = nullptr;   // l x l: V_B,r^T
  double *sig = nullptr;   // l: the singular values of B, decreasing
  double *full = nullptr;  // [0] = ||Theta||_F^2; [8, 8 + SQB): its block partials
  int *fail = nullptr;     // 1: a CholeskyQR of the range finder broke down
  int *fail2 = nullptr;    // 1: the CholeskyQR2 of B broke down
  double *R1 = nullptr;    // l x l: R of the first pass on B (row-major)
  double *RB = nullptr;    // l x l: R_B = R2 R1 (column-major)
  CqrBufs cq;
  double *svd = nullptr;   // the Jacobi SVD of B
};
}  // namespace

int rsvd_sketch_cols(int cap) { return 2 * cap; }

size_t cholqr2_ws_doubles(int p, int l) { return r32((size_t)p * l) + r32(8) + cqr_doubles(l); }

hipError_t cholqr2(double *Y, int p, int l, double *ws, int *fail_host, hipStream_t s) {
  double *T = ws;
  int *fail = reinterpret_cast<int *>(ws + r32((size_t)p * l));
  const CqrBufs cq = cqr_carve(l, ws + r32((size_t)p * l) + r32(8));
  hipError_t e;
  if ((e = launch_zero_int(fail, 1, s)) != hipSuccess) return e;
  if ((e = cholqr(Y, p, l, T, cq, fail, s, nullptr)) != hipSuccess) return e;
  if ((e = cholqr(T, p, l, Y, cq, fail, s, nullptr)) != hipSuccess) return e;
  if ((e = hipMemcpyAsync(fail_host, fail, sizeof(int), hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  return hipStreamSynchronize(s);
}

bool rsvd_eligible(int m, int n, int cap) {
  // The range finder pays when the kept rank is a small part of the
  // spectrum: the sketch must fit twice into the smaller side.
  return cap > 0 && 2 * rsvd_sketch_cols(cap) <= std::min(m, n) && std::min(m, n) <= kSvdMaxSide;
}

size_t rsvd_ws_doubles(int m, int n, int cap) {
  const int l = rsvd_sketch_cols(cap);
  const size_t mx = std::max(m, n);
  size_t t = 0;
  t += 3 * r32(mx * l) + r32((size_t)m * l) + r32((size_t)l * l);
  t += r32((size_t)l) + r32(8 + SQB) + r32(8) + r32(8) + 2 * r32((size_t)l * l);
  t += cqr_doubles(l);
  t += svd_ws_doubles(svd_plan(m, l));
  return t;
}

namespace {
RsvdBufs rsvd_carve(int m, int n, int cap, double *base) {
  const int l = rsvd_sketch_cols(cap);
  const size_t mx = std::max(m, n);
  RsvdBufs b;
  double *q = base;
  auto adv = [&](size_t nd) {
    double *x = q;
    q += r32(nd);
    return x;
  };
  b.Om = adv(mx * l);
  b.Y = adv(mx * l);
  b.T = adv(mx * l);
  b.B = adv((size_t)m * l);
  b.vbt = adv((size_t)l * l);
  b.sig = adv((size_t)l);
  b.full = adv(8 + SQB);
  b.fail = reinterpret_cast<int *>(adv(8));
  b.fail2 = reinterpret_cast<int *>(adv(8));
  b.R1 = adv((size_t)l * l);
  b.RB = adv((size_t)l * l);
  b.cq = cqr_carve(l, q);
  q += cqr_doubles(l);
  b.svd = q;
  return b;
}
}  // namespace

RsvdResult rsvd_oside(const double *Theta, int m, int n, int cap, int power, double accept, int max_sweeps,
                      double eps, int sketch_prec, uint64_t seed, int64_t stream_pos, double *pt, double *ws,
                      hipStream_t s, KernelTimer *timer, int trace) {
  RsvdResult out;
  const int l = rsvd_sketch_cols(cap);
  RsvdBufs b = rsvd_carve(m, n, cap, ws);
  auto ok = [&](hipError_t e) {
    if (e != hipSuccess) {
      out.err = TTM_EHIP;
      char what[112];
      snprintf(what, sizeof(what), "the randomized truncated SVD of a %d x %d matrix", m, n);
      note_hip_error(e, what);
      if (trace) fprintf(stderr, "[ttm] HIP error %s in %s\n", hipGetErrorName(e), what);
      return false;
    }
    return true;
  };
  // The bases in flight: the current Y (n x l) and Z (m x l) and a spare of
  // the same capacity; one CholeskyQR pass writes into the spare, and the
  // roles swap.  Intermediate bases need only be well conditioned (one pass
  // leaves cond ~ 1 + u cond(Y)^2); the final Y, which becomes P', gets the
  // second pass.
  double *ycur = b.Y, *zcur = b.Om, *spare = b.T;
  auto orth1 = [&](double *&X, int p) {
    if (!ok(cholqr(X, p, l, spare, b.cq, b.fail, s, timer))) return false;
    std::swap(X, spare);
    return true;
  };
  auto prod = [&](bool transposed, const double *Xin, double *Xout) {
    // Xout = Theta Xin (m x l) or Theta^T Xin (n x l), operands in the sketch precision
    GemmArgs g;
    g.prec = sketch_prec;
    if (transposed) {
      g.M = n; g.N = l; g.K = m;
      g.A = Theta; g.a_rs = m; g.a_cs = 1;
      g.B = Xin; g.b_rs = 1; g.b_cs = m;
      g.C = Xout; g.c_rs1 = 1; g.c_cs1 = n;
    } else {
      g.M = m; g.N = l; g.K = n;
      g.A = Theta; g.a_rs = 1; g.a_cs = m;
      g.B = Xin; g.b_rs = 1; g.b_cs = n;
      g.C = Xout; g.c_rs1 = 1; g.c_cs1 = m;
    }
    Timed tm(timer, KC_GEMM, s);
    return ok(launch_gemm(g, s));
  };
  if (!ok(launch_zero_int(b.fail, 1, s))) return out;
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    if (!ok(launch_splitmix_fill(b.Om, (int64_t)m * l, seed, stream_pos, s))) return out;
    hipLaunchKernelGGL(sumsq_part_kernel, dim3(SQB), dim3(256), 0, s, Theta, (int64_t)m * n, b.full + 8);
    hipLaunchKernelGGL(sumsq_final_kernel, dim3(1), dim3(256), 0, s, b.full + 8, b.full);
    if (!ok(hipGetLastError())) return out;
  }
  if (!prod(true, b.Om, ycur) || !orth1(ycur, n)) return out;
  for (int it = 0; it < power; ++it) {
    if (!prod(false, ycur, zcur) || !orth1(zcur, m)) return out;
    if (!prod(true, zcur, ycur) || !orth1(ycur, n)) return out;
  }
  if (!orth1(ycur, n)) return out;  // the second pass on the final basis
  {
    // B = Theta Y in FP64 (m x l, column-major)
    GemmArgs g;
    g.M = m; g.N = l; g.K = n;
    g.A = Theta; g.a_rs = 1; g.a_cs = m;
    g.B = ycur; g.b_rs = 1; g.b_cs = n;
    g.C = b.B; g.c_rs1 = 1; g.c_cs1 = m;
    Timed tm(timer, KC_GEMM, s);
    if (!ok(launch_gemm(g, s))) return out;
  }
  // B = Q_B R_B by CholeskyQR2 with R_B = R2 R1 kept (Q_B is not needed):
  // B's right singular vectors and values are R_B's, and the Jacobi SVD then
  // runs on the l x l R_B instead of the m x l B.
  if (!ok(launch_zero_int(b.fail2, 1, s))) return out;
  if (!ok(cholqr(b.B, m, l, spare, b.cq, b.fail2, s, timer, true))) return out;
  if (!ok(launch_copy(b.R1, b.cq.Rf, (int64_t)l * l, s))) return out;
  if (!ok(cholqr(spare, m, l, zcur, b.cq, b.fail2, s, timer, true))) return out;
  {
    GemmArgs g;
    g.M = l; g.N = l; g.K = l;
    g.A = b.cq.Rf; g.a_rs = l; g.a_cs = 1;
    g.B = b.R1; g.b_rs = l; g.b_cs = 1;
    g.C = b.RB; g.c_rs1 = 1; g.c_cs1 = l;
    Timed tm(timer, KC_GEMM, s);
    if (!ok(launch_gemm(g, s))) return out;
  }
  // A breakdown of the range finder's CholeskyQR makes its result
  // meaningless: read both flags before the SVD.
  int fail[2] = {0, 0};
  if (!ok(hipMemcpyAsync(&fail[0], b.fail, sizeof(int), hipMemcpyDeviceToHost, s))) return out;
  if (!ok(hipMemcpyAsync(&fail[1], b.fail2, sizeof(int), hipMemcpyDeviceToHost, s))) return out;
  if (!ok(hipStreamSynchronize(s))) return out;
  if (timer && timer->on) timer->collect();
  if (fail[0]) {
    out.fallback = true;
    if (trace) fprintf(stderr, "[ttm] rsvd %dx%d cap %d: CholeskyQR breakdown, full SVD instead\n", m, n, cap);
    return out;
  }
  // The SVD of R_B (or of B itself when its CholeskyQR2 broke down, B
  // formed again): the right singular vectors (over the l side) come out
  // orthonormal; the rank rule adds the weight outside span(Y).
  const double *Ysvd = b.RB;
  SvdPlan sp = svd_plan(l, l);
  if (fail[1]) {
    GemmArgs g;
    g.M = m; g.N = l; g.K = n;
    g.A = Theta; g.a_rs = 1; g.a_cs = m;
    g.B = ycur; g.b_rs = 1; g.b_cs = n;
    g.C = b.B; g.c_rs1 = 1; g.c_cs1 = m;
    Timed tm(timer, KC_GEMM, s);
    if (!ok(launch_gemm(g, s))) return out;
    Ysvd = b.B;
    sp = svd_plan(m, l);
  }
  SvdResult so = svd_oside(sp, Ysvd, eps, cap, 0, max_sweeps, b.vbt, SVD_U_T, b.sig, b.svd, s, timer, trace, nullptr,
                           b.full);
  out.sweeps = so.sweeps;
  if (so.err != TTM_OK) {
    out.err = so.err;
    return out;
  }
  const int r = so.rank;
  // Acceptance: the subspace error of direction r after q iterations is
  // about rho^(2q+1) with rho = sigma_{l+1} / sigma_r, bounded here by the
  // computed sigma_l / sigma_r; relative to the chain's norm the kept part
  // moves by about rho^(2q+1) sigma_r / ||Theta||_F.  Swaps whose estimate
  // exceeds `accept` (a spectrum too flat at the cut for q iterations) take
  // the full SVD.
  {
    double sv[2] = {0.0, 0.0};
    if (!ok(hipMemcpyAsync(&sv[0], b.sig + (r - 1), sizeof(double), hipMemcpyDeviceToHost, s))) return out;
    if (!ok(hipMemcpyAsync(&sv[1], b.sig + (l - 1), sizeof(double), hipMemcpyDeviceToHost, s))) return out;
    if (!ok(hipStreamSynchronize(s))) return out;
    if (timer && timer->on) timer->collect();
    const double rho = sv[0] > 0.0 ? sv[1] / sv[0] : 1.0;
    const double est = pow(rho, 2.0 * power + 1.0) * (so.total > 0.0 ? sv[0] / sqrt(so.total) : 1.0);
    out.estimate = est;
    if (!(est <= accept)) {
      out.fallback = true;
      if (trace) fprintf(stderr, "[ttm] rsvd %dx%d cap %d: estimate %.2e above %.0e, full SVD instead\n", m, n, cap,
                         est, accept);
      return out;
    }
  }
  {
    // P' = V_B,r^T Y^T (r x n, row-major)
    GemmArgs g;
    g.M = r; g.N = n; g.K = l;
    g.A = b.vbt; g.a_rs = l; g.a_cs = 1;
    g.B = ycur; g.b_rs = n; g.b_cs = 1;
    g.C = pt; g.c_rs1 = n; g.c_cs1 = 1;
    Timed tm(timer, KC_GEMM, s);
    if (!ok(launch_gemm(g, s))) return out;
  }
  out.rank = r;
  out.disc = so.disc;
  out.total = so.total;
  const double ld = l, md = m, nd = n;
  // products of the range finder and the projection, two CholeskyQRs per
  // orthonormalisation, the SVD of B (the bidiagonalisation model)
  out.flops = (2.0 * power + 2.0) * 2.0 * md * nd * ld +
              (2.0 * power + 1.0) * 2.0 * (2.0 * 0.5 * (md + nd) * ld * ld + ld * ld * ld / 3.0) +
              4.0 * md * ld * ld - (4.0 / 3.0) * ld * ld * ld + 4.0 * (md + ld) * ld * r + 2.0 * r * ld * nd;
  if (trace)
    fprintf(stderr, "[ttm] rsvd %dx%d l=%d q=%d sweeps=%d rank=%d disc=%.3e total=%.3e\n", m, n, l, power,
            out.sweeps, r, out.disc, out.total);
  return out;
}

}  // namespace ttm
