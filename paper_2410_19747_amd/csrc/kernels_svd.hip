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
constexpr int MAXB2 = 32;     // largest 2*bw
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
  int bw = 16;
  if (const char *e = getenv("TTM_JACOBI_BW")) {
    int v = atoi(e);
    if (v >= 1 && v <= MAXB2 / 2) bw = v;
  }
  if (nc <= 2 * bw) bw = (nc + 1) / 2;
  if (bw < 1) bw = 1;
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

// ------------------------------------------------------------------ Gram partials
// grid (pairs, sw).  Partial G over rows [s*R, s*R+R) of the pair's columns.
__global__ __launch_bounds__(JNT) void jacobi_gram_kernel(const double *__restrict__ W, int L, int bw,
                                                          int nblk, int round,
                                                          double *__restrict__ part, int sw) {
  __shared__ double P[ROWS_PER_WG][MAXB2 + 1];
  const int pair = blockIdx.x, s = blockIdx.y;
  int bi, bj;
  rr_pair(nblk, round, pair, bi, bj);
  const int b2 = 2 * bw;
  const int r0 = s * ROWS_PER_WG;
  const int nr = min(ROWS_PER_WG, L - r0);
  for (int e = threadIdx.x; e < ROWS_PER_WG * b2; e += JNT) {
    const int c = e / ROWS_PER_WG, i = e % ROWS_PER_WG;
    const int col = (c < bw) ? bi * bw + c : bj * bw + (c - bw);
    P[i][c] = (i < nr) ? W[(int64_t)col * L + r0 + i] : 0.0;
  }
  __syncthreads();
  double *out = part + ((int64_t)pair * sw + s) * b2 * b2;
  for (int e = threadIdx.x; e < b2 * b2; e += JNT) {
    const int p = e / b2, q = e % b2;
    double acc = 0.0;
    for (int i = 0; i < nr; ++i) acc = fma(P[i][p], P[i][q], acc);
    out[e] = acc;
  }
}

// ------------------------------------------------------------------ rotate
// grid (pairs, sw + sv).  Reduce partial Grams, diagonalise in LDS, apply.
__global__ __launch_bounds__(JNT) void jacobi_rotate_kernel(double *__restrict__ W, double *__restrict__ V,
                                                            int L, int ncp, int bw, int nblk, int round,
                                                            const double *__restrict__ part, int sw,
                                                            double *__restrict__ conv, double tol,
                                                            const double *__restrict__ result,
                                                            double noise2) {
  __shared__ double G[MAXB2][MAXB2 + 1];
  __shared__ double Q[MAXB2][MAXB2 + 1];
  __shared__ double P[ROWS_PER_WG][MAXB2 + 1];
  __shared__ double rc[MAXB2 / 2], rs[MAXB2 / 2];
  __shared__ int rp[MAXB2 / 2], rq[MAXB2 / 2];
  __shared__ int any_rot, sweep_rot;
  __shared__ double redmax[JNT / 64];

  const int pair = blockIdx.x, chunk = blockIdx.y;
  const int tid = threadIdx.x;
  int bi, bj;
  rr_pair(nblk, round, pair, bi, bj);
  const int b2 = 2 * bw;
  const int npair_in = bw;  // b2 / 2 rotations per inner step
  const double thr = noise2 * result[5];
  const double floor_n = sqrt(result[5] / (double)L);  // F / sqrt(L)

  // Reduce partial Grams in a fixed order.
  for (int e = tid; e < b2 * b2; e += JNT) {
    const double *src = part + (int64_t)pair * sw * b2 * b2 + e;
    double acc = 0.0;
    for (int s = 0; s < sw; ++s) acc += src[(int64_t)s * b2 * b2];
    G[e / b2][e % b2] = acc;
    Q[e / b2][e % b2] = (e / b2 == e % b2) ? 1.0 : 0.0;
  }
  if (tid == 0) any_rot = 0;
  __syncthreads();

  // Convergence measure of this visit: largest scaled off-diagonal.
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
    if ((tid & 63) == 0) redmax[tid >> 6] = m;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < JNT / 64; ++w) t = fmax(t, redmax[w]);
      conv[(int64_t)round * (nblk / 2) + pair] = t;
    }
  }

  // One cyclic sweep of two-sided Jacobi on G (round-robin over the b2
  // indices); the outer sweeps repeat the visit, so one inner sweep suffices.
  for (int isw = 0; isw < 1; ++isw) {
    if (tid == 0) sweep_rot = 0;
    __syncthreads();
    for (int step = 0; step < b2 - 1; ++step) {
      if (tid < npair_in) {
        int p, q;
        rr_pair(b2, step, tid, p, q);
        if (p > q) { int t = p; p = q; q = t; }
        const double gpp = G[p][p], gqq = G[q][q], gpq = G[p][q];
        double c = 1.0, sn = 0.0;
        const double a = sqrt(gpp), b = sqrt(gqq);
        const double lo = fmin(a, b);
        if ((gpp > thr || gqq > thr) && fabs(gpq) > tol * (fmax(a, b) * (lo * lo > thr ? lo : floor_n))) {
          const double zeta = (gqq - gpp) / (2.0 * gpq);
          const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + t * t);
          sn = c * t;
          sweep_rot = 1;
        }
        rc[tid] = c; rs[tid] = sn; rp[tid] = p; rq[tid] = q;
      }
      __syncthreads();
      // rows: G <- J^T G
      for (int e = tid; e < npair_in * b2; e += JNT) {
        const int t = e / b2, k = e % b2;
        const double c = rc[t], sn = rs[t];
        if (sn != 0.0) {
          const int p = rp[t], q = rq[t];
          const double gp = G[p][k], gq = G[q][k];
          G[p][k] = c * gp - sn * gq;
          G[q][k] = sn * gp + c * gq;
        }
      }
      __syncthreads();
      // columns: G <- G J ; Q <- Q J
      for (int e = tid; e < npair_in * b2; e += JNT) {
        const int t = e / b2, k = e % b2;
        const double c = rc[t], sn = rs[t];
        if (sn != 0.0) {
          const int p = rp[t], q = rq[t];
          const double gp = G[k][p], gq = G[k][q];
          G[k][p] = c * gp - sn * gq;
          G[k][q] = sn * gp + c * gq;
          const double qp = Q[k][p], qq = Q[k][q];
          Q[k][p] = c * qp - sn * qq;
          Q[k][q] = sn * qp + c * qq;
        }
      }
      __syncthreads();
    }
    const int did = sweep_rot;
    if (did && tid == 0) any_rot = 1;
    __syncthreads();
    if (!did) break;
  }
  if (!any_rot) return;  // Q = I: nothing to apply

  // One Newton-Schulz step, Q <- Q (3I - Q^T Q) / 2, restores orthogonality
  // to rounding level.  Without it the O(u) drift of every visit accumulates
  // over the thousands of visits a column receives.
  for (int e = tid; e < b2 * b2; e += JNT) {  // G <- Q^T Q
    const int i = e / b2, j = e % b2;
    double acc = 0.0;
    for (int k = 0; k < b2; ++k) acc = fma(Q[k][i], Q[k][j], acc);
    G[i][j] = acc;
  }
  __syncthreads();
  double qn[(MAXB2 * MAXB2 + JNT - 1) / JNT];
  for (int e = tid, t = 0; e < b2 * b2; e += JNT, ++t) {
    const int i = e / b2, j = e % b2;
    double acc = 0.0;
    for (int k = 0; k < b2; ++k) acc = fma(Q[i][k], G[k][j], acc);
    qn[t] = 1.5 * Q[i][j] - 0.5 * acc;
  }
  __syncthreads();
  for (int e = tid, t = 0; e < b2 * b2; e += JNT, ++t) Q[e / b2][e % b2] = qn[t];
  __syncthreads();

  // Apply Q to one row chunk of W (chunk < sw) or of V.
  double *X;
  int ld, r0, nr;
  if (chunk < sw) {
    X = W; ld = L; r0 = chunk * ROWS_PER_WG; nr = min(ROWS_PER_WG, L - r0);
  } else {
    X = V; ld = ncp; r0 = (chunk - sw) * ROWS_PER_WG; nr = min(ROWS_PER_WG, ncp - r0);
  }
  if (nr <= 0) return;
  for (int e = tid; e < ROWS_PER_WG * b2; e += JNT) {
    const int c = e / ROWS_PER_WG, i = e % ROWS_PER_WG;
    const int col = (c < bw) ? bi * bw + c : bj * bw + (c - bw);
    if (i < nr) P[i][c] = X[(int64_t)col * ld + r0 + i];
  }
  __syncthreads();
  for (int e = tid; e < ROWS_PER_WG * b2; e += JNT) {
    const int c = e / ROWS_PER_WG, i = e % ROWS_PER_WG;
    if (i < nr) {
      double acc = 0.0;
      for (int k = 0; k < b2; ++k) acc = fma(P[i][k], Q[k][c], acc);
      const int col = (c < bw) ? bi * bw + c : bj * bw + (c - bw);
      X[(int64_t)col * ld + r0 + i] = acc;
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
