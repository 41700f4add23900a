// One-sided block Jacobi SVD (Hestenes) for the swap and rounding SVDs.
//
// The Swap of Sec. II.B needs the full singular spectrum of each unfolded
// pair (the rule of Eq. (eps) sums the discarded weight from the smallest
// value up) and the leading singular vectors.  One-sided Jacobi
// orthogonalises the columns of W = Theta (or Theta^T) by plane rotations
// accumulated in V; at convergence W = U S and the column norms are the
// singular values, with high relative accuracy.
//
// Blocked form: the columns are split into blocks of width bw; a sweep is a
// round-robin tournament over blocks, every round pairing all blocks at once.
// For a pair (I, J) the 2bw x 2bw Gram matrix G = [W_I W_J]^T [W_I W_J] is
// formed from row chunks (kernel 1, partial sums in the workspace), then
// every workgroup of the pair reduces the partials in a fixed order,
// diagonalises G by cyclic two-sided Jacobi in LDS (identically, so the
// result is deterministic) and applies the accumulated rotation Q to its row
// chunk of W or V (kernel 2).  A rotation is applied only where
// |g_pq| > tol sqrt(g_pp g_qq); a sweep in which no pair exceeds tol means
// the columns are orthogonal to working accuracy.
//
// Accuracy target: that of a backward-stable FP64 SVD (errors of order
// u ||Theta||).  With column norms a_p, a_q (hi = max, lo = min),
// F = ||W||_F and the noise level nz = 8 sqrt(L) u F:
//   * both columns below nz: the pair is rounding noise; it is neither
//     rotated nor counted (relative orthogonality of noise is unattainable);
//   * one column below nz: absolute test |g_pq| <= u F hi (the large
//     column's component in the noise column is below rounding level);
//   * otherwise the relative test |g_pq| <= tol hi lo.
// In one formula: off_pq = |g_pq| / (hi * (lo > nz ? lo : F / sqrt(L))).
// A noise column may never be frozen while it still carries a component of
// a large one: summed over hundreds of columns that leaks ~1e-12 of the
// norm into the discarded part.

#include "ttm_internal.h"

namespace ttm {

namespace {
constexpr int JNT = 256;
constexpr int BW = 16;        // block width
constexpr int MAXB2 = 2 * BW; // columns of a block pair
constexpr int ROWS_PER_WG = 128;

__device__ __forceinline__ void rr_pair(int n, int round, int k, int &a, int &b) {
  // Circle method over n (even) players: player n-1 fixed, the others rotate.
  if (k == 0) {
    a = round;
    b = n - 1;
  } else {
    a = (round + k) % (n - 1);
    b = (round - k + (n - 1)) % (n - 1);
  }
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
}  // namespace

JacobiPlan jacobi_plan(int L, int nc) {
  JacobiPlan p;
  p.L = L;
  p.nc = nc;
  // Fixed block width: the kernels are specialised for 2 * BW = 32 columns;
  // narrower problems are padded with zero columns, which never rotate.
  const int bw = BW;
  int nblk = (nc + bw - 1) / bw;
  if (nblk < 2) nblk = 2;
  if (nblk & 1) ++nblk;
  p.bw = bw;
  p.nblk = nblk;
  p.ncp = nblk * bw;
  p.rows_per_wg = ROWS_PER_WG;
  p.sw = (L + ROWS_PER_WG - 1) / ROWS_PER_WG;
  p.sv = (p.ncp + ROWS_PER_WG - 1) / ROWS_PER_WG;
  p.rounds = nblk - 1;
  p.pairs = nblk / 2;
  return p;
}

size_t jacobi_ws_doubles(const JacobiPlan &p) {
  const size_t b2 = 2 * (size_t)p.bw;
  size_t n = 0;
  n += (size_t)p.L * p.ncp;               // W
  n += (size_t)p.ncp * p.ncp;             // V
  n += (size_t)p.pairs * p.sw * b2 * b2;  // partial Grams
  n += (size_t)p.rounds * p.pairs;        // conv
  n += (size_t)p.ncp;                     // sigma
  n += (size_t)p.ncp;                     // perm (ints, padded as doubles)
  n += 8;                                 // result
  return n + 8 * 32;                      // each of the 7 regions is rounded up to 32 doubles
}

__global__ __launch_bounds__(1024) void jacobi_frob_kernel(const double *__restrict__ W, int64_t n,
                                                           double *__restrict__ result);

// ------------------------------------------------------------------ init
__global__ void jacobi_init_kernel(double *W, double *V, int L, int nc, int ncp) {
  const int64_t nw = (int64_t)L * (ncp - nc);
  const int64_t nv = (int64_t)ncp * ncp;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nw + nv;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nw) {
      W[(int64_t)L * nc + e] = 0.0;
    } else {
      const int64_t v = e - nw;
      const int64_t i = v % ncp, j = v / ncp;
      V[v] = (i == j) ? 1.0 : 0.0;
    }
  }
}

hipError_t launch_jacobi_init(const JacobiPlan &p, const JacobiBufs &b, hipStream_t s) {
  const int64_t n = (int64_t)p.L * (p.ncp - p.nc) + (int64_t)p.ncp * p.ncp;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(jacobi_init_kernel, dim3((int)g), dim3(256), 0, s, b.W, b.V, p.L, p.nc, p.ncp);
  hipLaunchKernelGGL(jacobi_frob_kernel, dim3(1), dim3(1024), 0, s, b.W, (int64_t)p.L * p.nc, b.result);
  return hipGetLastError();
}

// ------------------------------------------------------------------ MFMA helpers
typedef double dbl4 __attribute__((ext_vector_type(4)));

// One wave computes a 16 x 16 tile D = sum_k A(i,k) B(k,j) over k < K (K a
// multiple of 4) with v_mfma_f64_16x16x4f64.  Lane l supplies A(l%16, k+l/16)
// and B(k+l/16, l%16); accumulator register t of lane l holds
// D(4t + l/16, l%16).  a(i,k) / b(k,j) are LDS accessors.
template <typename FA, typename FB>
__device__ __forceinline__ dbl4 mfma_tile(FA a, FB b, int K, int lane) {
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  const int r = lane & 15, kq = lane >> 4;
  for (int k = 0; k < K; k += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a(r, k + kq), b(k + kq, r), acc, 0, 0, 0);
  return acc;
}

// ------------------------------------------------------------------ Gram partials
// grid (pairs, sw).  Partial G = P^T P over rows [s*R, s*R+R) of the pair's
// 2*bw columns (zero-padded to 32), one 16 x 16 tile per wave on MFMA.
__global__ __launch_bounds__(JNT) void jacobi_gram_kernel(const double *__restrict__ W, int L, int bw,
                                                          int nblk, int round,
                                                          double *__restrict__ part, int sw) {
  __shared__ double P[ROWS_PER_WG][MAXB2 + 1];
  const int pair = blockIdx.x, s = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int bi, bj;
  rr_pair(nblk, round, pair, bi, bj);
  const int b2 = 2 * bw;
  const int r0 = s * ROWS_PER_WG;
  const int nr = min(ROWS_PER_WG, L - r0);
  for (int e = tid; e < ROWS_PER_WG * MAXB2; e += JNT) {
    const int c = e / ROWS_PER_WG, i = e % ROWS_PER_WG;
    double v = 0.0;
    if (c < b2 && i < nr) {
      const int col = (c < bw) ? bi * bw + c : bj * bw + (c - bw);
      v = W[(int64_t)col * L + r0 + i];
    }
    P[i][c] = v;
  }
  __syncthreads();
  const int ti = wave >> 1, tj = wave & 1;
  dbl4 acc = mfma_tile([&](int i, int k) { return P[k][ti * 16 + i]; },
                       [&](int k, int j) { return P[k][tj * 16 + j]; }, ROWS_PER_WG, lane);
  double *out = part + ((int64_t)pair * sw + s) * b2 * b2;
  for (int t = 0; t < 4; ++t) {
    const int i = ti * 16 + 4 * t + (lane >> 4), j = tj * 16 + (lane & 15);
    if (i < b2 && j < b2) out[i * b2 + j] = acc[t];
  }
}

// ------------------------------------------------------------------ rotate
// grid (pairs, sw + sv).  Every workgroup of a pair reduces the partial Grams
// in the same fixed order, runs one cyclic sweep of two-sided Jacobi on the
// 2bw x 2bw Gram in LDS (bit-identical in all of them), re-orthogonalises the
// accumulated rotation, and applies it to its row chunk of W (chunk < sw) or
// of V.  A step of the inner sweep rotates bw disjoint index pairs at once;
// G <- J^T G J then splits into independent 2 x 2 blocks, one per thread.
__global__ __launch_bounds__(JNT) void jacobi_rotate_kernel(double *__restrict__ W, double *__restrict__ V,
                                                            int L, int ncp, int bw, int nblk, int round,
                                                            const double *__restrict__ part, int sw,
                                                            double *__restrict__ conv, double tol,
                                                            const double *__restrict__ result,
                                                            double noise2) {
  __shared__ double G[MAXB2][MAXB2 + 1];
  __shared__ double Q[MAXB2][MAXB2 + 1];
  __shared__ double S[MAXB2][MAXB2 + 1];
  __shared__ double P[ROWS_PER_WG][MAXB2 + 1];
  __shared__ double rc[BW], rs[BW];
  __shared__ unsigned char tp[MAXB2 - 1][BW], tq[MAXB2 - 1][BW];
  __shared__ int any_rot;
  __shared__ double redmax[JNT / 64];
  static_assert(JNT == BW * BW, "one 2x2 block per thread");

  const int pair = blockIdx.x, chunk = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int bi, bj;
  rr_pair(nblk, round, pair, bi, bj);
  const int b2 = 2 * bw;
  const double thr = noise2 * result[5];
  const double floor_n = sqrt(result[5] / (double)L);  // F / sqrt(L)

  // Reduce partial Grams in a fixed order; pad to 32 x 32 with the identity.
  for (int e = tid; e < MAXB2 * MAXB2; e += JNT) {
    const int i = e / MAXB2, j = e % MAXB2;
    double acc = 0.0;
    if (i < b2 && j < b2) {
      const double *src = part + (int64_t)pair * sw * b2 * b2 + i * b2 + j;
      for (int s = 0; s < sw; ++s) acc += src[(int64_t)s * b2 * b2];
    }
    G[i][j] = acc;
    Q[i][j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) any_rot = 0;
  __syncthreads();

  // Convergence measure of this visit (scaled off-diagonal, see the header).
  if (chunk == 0) {
    double m = 0.0;
    for (int e = tid; e < b2 * b2; e += JNT) {
      const int p = e / b2, q = e % b2;
      if (p < q) {
        const double gp = G[p][p], gq = G[q][q];
        if (gp > thr || gq > thr) {
          const double a = sqrt(gp), b = sqrt(gq);
          const double lo = fmin(a, b);
          m = fmax(m, fabs(G[p][q]) / (fmax(a, b) * (lo * lo > thr ? lo : floor_n)));
        }
      }
    }
    m = wave_max(m);
    if (lane == 0) redmax[wave] = m;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < JNT / 64; ++w) t = fmax(t, redmax[w]);
      conv[(int64_t)round * (nblk / 2) + pair] = t;
    }
  }

  // One cyclic sweep of two-sided Jacobi over the 32 indices: 31 steps of
  // 16 disjoint rotations (round-robin pairs from a table built here).
  for (int e = tid; e < (MAXB2 - 1) * BW; e += JNT) {
    const int st = e / BW, k = e % BW;
    int p, q;
    rr_pair(MAXB2, st, k, p, q);
    tp[st][k] = (unsigned char)min(p, q);
    tq[st][k] = (unsigned char)max(p, q);
  }
  const double tol2 = tol * tol, floor2 = floor_n * floor_n;
  __syncthreads();
  for (int step = 0; step < MAXB2 - 1; ++step) {
    if (tid < BW) {
      const int p = tp[step][tid], q = tq[step][tid];
      const double gpp = G[p][p], gqq = G[q][q], gpq = G[p][q];
      const double hi2 = fmax(gpp, gqq), lo2 = fmin(gpp, gqq);
      double c = 1.0, sn = 0.0;
      // |g_pq| > tol * hi * (lo^2 > thr ? lo : F/sqrt(L)), squared
      if (hi2 > thr && gpq * gpq > tol2 * hi2 * (lo2 > thr ? lo2 : floor2)) {
        // tan of the rotation angle from zeta = (g_qq - g_pp) / (2 g_pq); the
        // hardware reciprocal / rsqrt approximations are enough for t, and
        // one Newton step on c makes c^2 + s^2 = 1 to rounding.
        const double zeta = (gqq - gpp) * __builtin_amdgcn_rcp(2.0 * gpq);
        const double az = fabs(zeta);
        double t;
        if (az > 1e100) {
          t = 0.5 * __builtin_amdgcn_rcp(zeta);
        } else {
          const double w = 1.0 + zeta * zeta;
          const double root = w * __builtin_amdgcn_rsq(w);
          t = copysign(__builtin_amdgcn_rcp(az + root), zeta);
        }
        const double x = 1.0 + t * t;
        double y = __builtin_amdgcn_rsq(x);
        y = y * (1.5 - 0.5 * x * y * y);
        y = y * (1.5 - 0.5 * x * y * y);
        c = y;
        sn = y * t;
        any_rot = 1;
      }
      rc[tid] = c;
      rs[tid] = sn;
    }
    __syncthreads();
    {
      // G <- J^T G J on 2 x 2 blocks: thread (u, v) owns rows {p_u, q_u} x
      // cols {p_v, q_v}; 16 x 16 blocks = 256 threads.
      const int u = tid >> 4, v = tid & 15;
      const double su = rs[u], sv = rs[v];
      if (su != 0.0 || sv != 0.0) {
        const double cu = rc[u], cv = rc[v];
        const int pu = tp[step][u], qu = tq[step][u], pv = tp[step][v], qv = tq[step][v];
        const double g00 = G[pu][pv], g01 = G[pu][qv], g10 = G[qu][pv], g11 = G[qu][qv];
        const double h00 = cu * g00 - su * g10, h01 = cu * g01 - su * g11;
        const double h10 = su * g00 + cu * g10, h11 = su * g01 + cu * g11;
        G[pu][pv] = cv * h00 - sv * h01;
        G[pu][qv] = sv * h00 + cv * h01;
        G[qu][pv] = cv * h10 - sv * h11;
        G[qu][qv] = sv * h10 + cv * h11;
      }
      // Q <- Q J: row k = tid / 8, pairs 2 (tid % 8) and 2 (tid % 8) + 1
      const int k = tid >> 3;
      for (int h = 0; h < 2; ++h) {
        const int w = 2 * (tid & 7) + h;
        const double sw_ = rs[w];
        if (sw_ != 0.0) {
          const double cw = rc[w];
          const int pw = tp[step][w], qw = tq[step][w];
          const double q0 = Q[k][pw], q1 = Q[k][qw];
          Q[k][pw] = cw * q0 - sw_ * q1;
          Q[k][qw] = sw_ * q0 + cw * q1;
        }
      }
    }
    __syncthreads();
  }
  if (!any_rot) return;  // Q = I: nothing to apply

  // One Newton-Schulz step, Q <- Q (3I - Q^T Q) / 2, restores orthogonality
  // to rounding level; without it the O(u) drift of every visit accumulates
  // over the thousands of visits a column receives.  32 x 32 products on
  // MFMA, one 16 x 16 tile per wave.
  const int ti = wave >> 1, tj = wave & 1;
  {
    dbl4 acc = mfma_tile([&](int i, int k) { return Q[k][ti * 16 + i]; },
                         [&](int k, int j) { return Q[k][tj * 16 + j]; }, MAXB2, lane);
    for (int t = 0; t < 4; ++t) S[ti * 16 + 4 * t + (lane >> 4)][tj * 16 + (lane & 15)] = acc[t];
  }
  __syncthreads();
  {
    dbl4 acc = mfma_tile([&](int i, int k) { return Q[ti * 16 + i][k]; },
                         [&](int k, int j) { return S[k][tj * 16 + j]; }, MAXB2, lane);
    __syncthreads();  // every wave has read Q before it is overwritten
    for (int t = 0; t < 4; ++t) {
      const int i = ti * 16 + 4 * t + (lane >> 4), j = tj * 16 + (lane & 15);
      G[i][j] = 1.5 * Q[i][j] - 0.5 * acc[t];
    }
  }
  __syncthreads();  // the re-orthogonalised rotation is now in G

  // Apply to one row chunk of W (chunk < sw) or of V: P (rows x 32) <- P G.
  double *X;
  int ld, r0, nr;
  if (chunk < sw) {
    X = W; ld = L; r0 = chunk * ROWS_PER_WG; nr = min(ROWS_PER_WG, L - r0);
  } else {
    X = V; ld = ncp; r0 = (chunk - sw) * ROWS_PER_WG; nr = min(ROWS_PER_WG, ncp - r0);
  }
  if (nr <= 0) return;
  for (int e = tid; e < ROWS_PER_WG * MAXB2; e += JNT) {
    const int c = e / ROWS_PER_WG, i = e % ROWS_PER_WG;
    double v = 0.0;
    if (c < b2 && i < nr) {
      const int col = (c < bw) ? bi * bw + c : bj * bw + (c - bw);
      v = X[(int64_t)col * ld + r0 + i];
    }
    P[i][c] = v;
  }
  __syncthreads();
  // 8 x 2 output tiles of 16 x 16; wave w owns row tiles 2w, 2w+1.
  dbl4 acc[2][2];
  for (int x = 0; x < 2; ++x) {
    const int rt = 2 * wave + x;
    for (int y = 0; y < 2; ++y)
      acc[x][y] = mfma_tile([&](int i, int k) { return P[rt * 16 + i][k]; },
                            [&](int k, int j) { return G[k][y * 16 + j]; }, MAXB2, lane);
  }
  for (int x = 0; x < 2; ++x) {
    const int rt = 2 * wave + x;
    for (int y = 0; y < 2; ++y) {
      for (int t = 0; t < 4; ++t) {
        const int i = rt * 16 + 4 * t + (lane >> 4), c = y * 16 + (lane & 15);
        if (i < nr && c < b2) {
          const int col = (c < bw) ? bi * bw + c : bj * bw + (c - bw);
          X[(int64_t)col * ld + r0 + i] = acc[x][y][t];
        }
      }
    }
  }
}

__global__ void jacobi_convmax_kernel(const double *__restrict__ conv, int n, double *result) {
  __shared__ double red[JNT / 64];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += JNT) m = fmax(m, conv[i]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < JNT / 64; ++w) t = fmax(t, red[w]);
    result[3] = t;
  }
}

// result[5] = ||W||_F^2 (invariant under the rotations; sets the noise floor).
__global__ __launch_bounds__(1024) void jacobi_frob_kernel(const double *__restrict__ W, int64_t n,
                                                           double *__restrict__ result) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) acc = fma(W[i], W[i], acc);
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    result[5] = t;
  }
}

hipError_t launch_jacobi_sweep(const JacobiPlan &p, const JacobiBufs &b, double tol, hipStream_t s,
                               KernelTimer *timer) {
  if (2 * p.bw > MAXB2) return hipErrorInvalidValue;
  const double ns = 8.0 * sqrt((double)p.L) * 2.220446049250313e-16;
  const double noise2 = ns * ns;
  for (int round = 0; round < p.rounds; ++round) {
    {
      Timed tm(timer, KC_JAC_GRAM, s);
      hipLaunchKernelGGL(jacobi_gram_kernel, dim3(p.pairs, p.sw), dim3(JNT), 0, s, b.W, p.L, p.bw,
                         p.nblk, round, b.part, p.sw);
    }
    {
      Timed tm(timer, KC_JAC_ROTATE, s);
      hipLaunchKernelGGL(jacobi_rotate_kernel, dim3(p.pairs, p.sw + p.sv), dim3(JNT), 0, s, b.W, b.V,
                         p.L, p.ncp, p.bw, p.nblk, round, b.part, p.sw, b.conv, tol, b.result, noise2);
    }
  }
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    hipLaunchKernelGGL(jacobi_convmax_kernel, dim3(1), dim3(JNT), 0, s, b.conv, p.rounds * p.pairs,
                       b.result);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ finish
// sigma[c] = ||W[:, c]|| for c < nc; one wave per column.
__global__ __launch_bounds__(JNT) void jacobi_sigma_kernel(const double *__restrict__ W, int L, int nc,
                                                           double *__restrict__ sigma) {
  const int c = blockIdx.x * (JNT / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nc) return;
  const double *col = W + (int64_t)c * L;
  double acc = 0.0;
  for (int i = lane; i < L; i += 64) acc = fma(col[i], col[i], acc);
  acc = wave_sum(acc);
  if (lane == 0) sigma[c] = sqrt(acc);
}

// perm[k] = the column holding the k-th largest value (ties by index).
__global__ __launch_bounds__(JNT) void jacobi_sort_kernel(const double *__restrict__ sigma, int nc,
                                                          int *__restrict__ perm) {
  extern __shared__ double sv[];
  for (int i = threadIdx.x; i < nc; i += JNT) sv[i] = sigma[i];
  __syncthreads();
  const int c = blockIdx.x * JNT + threadIdx.x;
  if (c >= nc) return;
  const double me = sv[c];
  int pos = 0;
  for (int j = 0; j < nc; ++j) {
    const double o = sv[j];
    pos += (o > me) || (o == me && j < c);
  }
  perm[pos] = c;
}

// Rule of Eq. (eps) on the sorted values: tails summed from the smallest up.
// One workgroup: thread t owns the contiguous index range of chunk t.
__global__ __launch_bounds__(1024) void jacobi_rank_kernel(const double *__restrict__ sigma,
                                                           const int *__restrict__ perm, int n,
                                                           double eps, int cap, int forced,
                                                           double *__restrict__ result) {
  __shared__ double csum[1024];
  __shared__ int best;
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  double local = 0.0;
  for (int k = hi - 1; k >= lo; --k) {
    const double s = sigma[perm[k]];
    local += s * s;
  }
  csum[t] = local;
  if (t == 0) best = n;
  __syncthreads();
  // suffix: weight of every chunk after this one, summed from the end
  double after = 0.0;
  for (int u = nt - 1; u > t; --u) after += csum[u];
  double total = 0.0;
  for (int u = nt - 1; u >= 0; --u) total += csum[u];
  // tails[k] = sum_{i >= k} s_i^2 ; the kept count k needs tails[k]
  double tail = after;
  int mine = n;
  for (int k = hi - 1; k >= lo; --k) {
    // tail currently = tails[k+1]
    const int kept = k + 1;
    if (kept >= 1 && (tail <= 0.0 || tail < eps * total)) mine = kept;
    const double s = sigma[perm[k]];
    tail += s * s;
  }
  if (mine < n) atomicMin(&best, mine);
  __syncthreads();
  if (t == 0) {
    int r = best;
    if (r < 1) r = 1;
    if (cap > 0 && r > cap) r = cap;
    if (forced > 0) r = forced;
    if (r > n) r = n;
    // discarded weight tails[r], summed from the smallest up
    double disc = 0.0;
    for (int k = n - 1; k >= r; --k) {
      const double s = sigma[perm[k]];
      disc += s * s;
    }
    result[0] = (double)r;
    result[1] = disc;
    result[2] = total;
    result[4] = isfinite(total) ? 0.0 : 1.0;
  }
}

hipError_t launch_jacobi_finish(const JacobiPlan &p, const JacobiBufs &b, double eps, int cap,
                                int forced, hipStream_t s) {
  const int nc = p.nc;
  hipLaunchKernelGGL(jacobi_sigma_kernel, dim3((nc + 3) / 4), dim3(JNT), 0, s, b.W, p.L, nc, b.sigma);
  const size_t shm = (size_t)nc * sizeof(double);
  if (shm > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(jacobi_sort_kernel, dim3((nc + JNT - 1) / JNT), dim3(JNT), shm, s, b.sigma, nc,
                     b.perm);
  hipLaunchKernelGGL(jacobi_rank_kernel, dim3(1), dim3(1024), 0, s, b.sigma, b.perm, nc, eps, cap,
                     forced, b.result);
  return hipGetLastError();
}

// ------------------------------------------------------------------ write-out
__global__ void svd_write_kernel(const double *__restrict__ W, const double *__restrict__ V,
                                 const double *__restrict__ sigma, const int *__restrict__ perm, int L,
                                 int nc, int ncp, int r, int w_holds_u, int left_pow, int right_pow,
                                 double *__restrict__ left, double *__restrict__ right) {
  // left: rows_l x r; right: r x cols_r
  const int rows_l = w_holds_u ? L : nc;
  const int cols_r = w_holds_u ? nc : L;
  const int64_t nl = (int64_t)rows_l * r, nrgt = (int64_t)r * cols_r;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nl + nrgt;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nl) {
      const int i = (int)(e / r), k = (int)(e % r);
      const int c = perm[k];
      const double sg = sigma[c];
      double v;
      if (w_holds_u) {
        v = W[(int64_t)c * L + i];                 // u_k * sigma_k
        if (!left_pow) v = (sg > 0.0) ? v / sg : 0.0;
      } else {
        v = V[(int64_t)c * ncp + i];               // u_k
        if (left_pow) v *= sg;
      }
      left[e] = v;
    } else {
      const int64_t f = e - nl;
      const int k = (int)(f / cols_r), j = (int)(f % cols_r);
      const int c = perm[k];
      const double sg = sigma[c];
      double v;
      if (w_holds_u) {
        v = V[(int64_t)c * ncp + j];               // v_k
        if (right_pow) v *= sg;
      } else {
        v = W[(int64_t)c * L + j];                 // v_k * sigma_k
        if (!right_pow) v = (sg > 0.0) ? v / sg : 0.0;
      }
      right[f] = v;
    }
  }
}

hipError_t launch_svd_write(const JacobiPlan &p, const JacobiBufs &b, int r, bool w_holds_u,
                            int left_pow, int right_pow, double *left, double *right, hipStream_t s) {
  const int rows_l = w_holds_u ? p.L : p.nc;
  const int cols_r = w_holds_u ? p.nc : p.L;
  const int64_t n = (int64_t)rows_l * r + (int64_t)r * cols_r;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(svd_write_kernel, dim3((int)g), dim3(256), 0, s, b.W, b.V, b.sigma, b.perm, p.L,
                     p.nc, p.ncp, r, w_holds_u ? 1 : 0, left_pow, right_pow, left, right);
  return hipGetLastError();
}

}  // namespace ttm
