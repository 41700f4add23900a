// Reverse mode of the TTM product (ttm_multiply_vjp): the product is run
// again with every step's operands recorded, then the steps are undone in
// reverse order, each by its adjoint, all on the device:
//   * contraction Pi[a,e,b] = sum_c K[a,e,c] X[c,e,b] (Eq. contract): two
//     products per physical value;
//   * QR of an unfolding M = Q R with R multiplied into the next core (the
//     canonicalisation sweeps and the gauge moves): for a tall M,
//     M_bar = [Q_bar + Q sym_l(R R_bar^T - Q_bar^T Q)] R^{-T}, sym_l keeping
//     the lower triangle and mirroring it, R^{-T} by a triangular solve; a
//     wide M = [X | Y] through its leading square block;
//   * truncated SVD of a swap's merged pair Theta (Fig. 1C, Eq. (eps)) with
//     outputs Z = Theta V_r and V_r^T: the first-order change of the kept
//     right singular vectors, kept-dropped pairs weighted by
//     1 / (sigma_i^2 - sigma_j^2) and the unresolved and null directions by
//     1 / sigma_i^2 (rotations among kept vectors change only a bond's gauge,
//     so they contribute nothing);
//     Theta_bar = (Z_bar + Theta Y) V_r^T + Z Y^T with
//     Y = V_d [F o (V_d^T V_r_bar)] + (I - V V^T) V_r_bar S_r^{-2};
//   * the leg-exchange merge: two products after a permutation;
//   * the final rounding sweep: the same SVD adjoint on Pi_i^T.
// The ranks are those of the recorded forward pass (piecewise constant).
#include <math.h>

#include <algorithm>
#include <vector>

#include "ttm_internal.h"

namespace ttm {
namespace {

constexpr int NT = 256;

int grid_for(int64_t n) {
  int64_t g = (n + NT - 1) / NT;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

// T[a][e][w][b] = Theta[(a dx + w) + (e Dr + b) m]: the merged pair's
// cotangent back in the order of the two carriages' legs.
__global__ void legs_back_kernel(const double *__restrict__ th, int Dl, int dp, int dx, int Dr,
                                 double *__restrict__ T) {
  const int64_t m = (int64_t)Dl * dx;
  const int64_t total = m * dp * Dr;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    int64_t t = q;
    const int b = (int)(t % Dr); t /= Dr;
    const int w = (int)(t % dx); t /= dx;
    const int e = (int)(t % dp); t /= dp;
    const int a = (int)t;
    T[q] = th[((int64_t)a * dx + w) + ((int64_t)e * Dr + b) * m];
  }
}

// Mm[q + t kd] /= (s_t^2 - s_{r+q}^2), q < kd, t < r; a zero gap (a tie at
// the cut, where no derivative exists) contributes nothing.
__global__ void gap_scale_kernel(double *__restrict__ Mm, const double *__restrict__ sig, int r, int kd) {
  const int64_t total = (int64_t)kd * r;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int q = (int)(x % kd), t = (int)(x / kd);
    const double li = sig[t] * sig[t], lj = sig[r + q] * sig[r + q];
    const double g = li - lj;
    Mm[x] = (g != 0.0) ? Mm[x] / g : 0.0;
  }
}

// Y[j + t n] += N[j + t n] / s_t^2 (j < n, t < r); zero for s_t = 0.
__global__ void null_add_kernel(double *__restrict__ Y, const double *__restrict__ N, const double *__restrict__ sig,
                                int n, int r) {
  const int64_t total = (int64_t)n * r;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(x / n);
    const double l = sig[t] * sig[t];
    if (l > 0.0) Y[x] += N[x] / l;
  }
}

// X (n x n, row-major, ld) <- lower triangle mirrored to the upper one.
__global__ void mirror_lower_kernel(double *__restrict__ X, int n, int64_t ld) {
  const int64_t total = (int64_t)n * n;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(x / n), j = (int)(x % n);
    if (j > i) X[i * ld + j] = X[(int64_t)j * ld + i];
  }
}

// Y = Z R^{-T} for the m x n row-major Z (ld n) and the upper triangular
// n x n R (row-major, ld ldr): row i of Y solves y R^T = z by back
// substitution, y_j = (z_j - sum_{l > j} y_l R[j][l]) / R[j][j].  One thread
// per row; Y and Z are distinct.
__global__ void trsm_rt_kernel(double *__restrict__ Y, const double *__restrict__ Z, const double *__restrict__ R,
                               int m, int n, int64_t ldr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double *y = Y + (int64_t)i * n;
  const double *z = Z + (int64_t)i * n;
  for (int j = n - 1; j >= 0; --j) {
    const double *rj = R + (int64_t)j * ldr;
    double acc = z[j];
    for (int l = j + 1; l < n; ++l) acc = fma(-y[l], rj[l], acc);
    y[j] = acc / rj[j];
  }
}

// dst (rows x cols, ld ldd) = src (rows x cols, ld lds), both row-major.
__global__ void copy2d_kernel(double *__restrict__ dst, int64_t ldd, const double *__restrict__ src, int64_t lds,
                              int rows, int cols) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = x / cols, j = x % cols;
    dst[i * ldd + j] = src[i * lds + j];
  }
}

GemmArgs gemm(int M, int N, int K, const double *A, int64_t a_rs, int64_t a_cs, const double *B, int64_t b_rs,
              int64_t b_cs, double *C, int64_t c_rs, int64_t c_cs, double alpha = 1.0, double beta = 0.0) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.a_rs = a_rs; g.a_cs = a_cs;
  g.B = B; g.b_rs = b_rs; g.b_cs = b_cs;
  g.C = C; g.c_rs1 = c_rs; g.c_cs1 = c_cs;
  g.alpha = alpha; g.beta = beta;
  return g;
}

struct Back {
  hipStream_t st;
  int err = TTM_OK;
  double *S[8] = {};  // scratch, each `scap` doubles
  size_t scap = 0;
  bool ok(hipError_t e, const char *what) {
    if (e != hipSuccess) {
      if (err == TTM_OK) {
        err = TTM_EHIP;
        note_hip_error(e, what);
      }
      return false;
    }
    return true;
  }
  bool mm(const GemmArgs &g) { return ok(launch_gemm(g, st), "a product of the reverse mode"); }
  bool copy(double *d, const double *s, int64_t n) { return ok(launch_copy(d, s, n, st), "a copy of the reverse mode"); }

  // Cotangent of the m x n column-major mat (written to `matbar`, column-major)
  // for the outputs Z (m x r; element (i, t) at Z[i zs_r + t zs_c]) = mat V_r and
  // V_r^T, given Z_bar (m x r, row-major) and V_r_bar already formed in Vrb
  // (n x r, column-major) as the cotangent of V_r^T transposed.  V: n x kg
  // column-major resolved right singular vectors; sig: k values, decreasing.
  bool svd_adjoint(const double *mat, int m, int n, const double *V, const double *sig, int r, int kg,
                   const double *Z, int64_t zs_r, int64_t zs_c, const double *Zb, double *Vrb, double *matbar) {
    double *Mm = S[2], *Y = S[3], *Nb = S[4], *G1 = S[5], *T1 = S[6];
    // V_r_bar += mat^T Z_bar  (the dependence of Z on V_r)
    if (!mm(gemm(n, r, m, mat, m, 1, Zb, r, 1, Vrb, 1, n, 1.0, 1.0))) return false;
    // Y = V_d [F o (V_d^T V_r_bar)] over the resolved dropped vectors
    const int kd = kg - r;
    if (kd > 0) {
      if (!mm(gemm(kd, r, n, V + (int64_t)r * n, n, 1, Vrb, 1, n, Mm, 1, kd))) return false;
      hipLaunchKernelGGL(gap_scale_kernel, dim3(grid_for((int64_t)kd * r)), dim3(NT), 0, st, Mm, sig, r, kd);
      if (!ok(hipGetLastError(), "the gap weights of an SVD adjoint")) return false;
      if (!mm(gemm(n, r, kd, V + (int64_t)r * n, 1, n, Mm, 1, kd, Y, 1, n))) return false;
    } else if (!ok(launch_fill(Y, 0.0, (int64_t)n * r, st), "a fill of the reverse mode")) {
      return false;
    }
    // the unresolved and null directions: (I - V V^T) V_r_bar / s^2
    if (kg < n) {
      if (!mm(gemm(kg, r, n, V, n, 1, Vrb, 1, n, G1, 1, kg))) return false;
      if (!copy(Nb, Vrb, (int64_t)n * r)) return false;
      if (!mm(gemm(n, r, kg, V, 1, n, G1, 1, kg, Nb, 1, n, -1.0, 1.0))) return false;
      hipLaunchKernelGGL(null_add_kernel, dim3(grid_for((int64_t)n * r)), dim3(NT), 0, st, Y, Nb, sig, n, r);
      if (!ok(hipGetLastError(), "the null-space weights of an SVD adjoint")) return false;
    }
    // T1 = Z_bar + mat Y (m x r, row-major)
    if (!copy(T1, Zb, (int64_t)m * r)) return false;
    if (!mm(gemm(m, r, n, mat, 1, m, Y, 1, n, T1, r, 1, 1.0, 1.0))) return false;
    // matbar = T1 V_r^T + Z Y^T (column-major m x n)
    if (!mm(gemm(m, n, r, T1, r, 1, V, n, 1, matbar, 1, m))) return false;
    if (!mm(gemm(m, n, r, Z, zs_r, zs_c, Y, n, 1, matbar, 1, m, 1.0, 1.0))) return false;
    return true;
  }

  // Cotangent of a QR-moved core: M (m x n row-major) = Q R, the next core
  // became R nxt (nxt: n x ncol).  In: Qb (m x k, the cotangent of the new
  // core), nb (k x ncol, of the new next core).  Out: Mb (m x n) and nxtb
  // (n x ncol); Mb may alias Qb, nxtb must not alias nb.
  bool qr_adjoint(const TapeEntry &e, const double *Qb, const double *nb, double *Mb, double *nxtb) {
    const int m = e.m, n = e.n, k = e.k, nc = e.ncol;
    double *Rb = S[0], *X = S[1], *W = S[2];
    // R_bar = nb nxt^T (k x n), nxt_bar = R^T nb (n x ncol)
    if (!mm(gemm(k, n, nc, nb, nc, 1, e.nxt, 1, nc, Rb, n, 1))) return false;
    if (!mm(gemm(n, nc, k, e.R, 1, n, nb, nc, 1, nxtb, nc, 1))) return false;
    // square leading block: Q (m x k), U = R[:, :k] (ld n), Qbar' = Qb (+ Y Rb[:, k:]^T when wide)
    if (!copy(W, Qb, (int64_t)m * k)) return false;
    if (k < n) {
      // wide: M = [X | Y] with X = Q U, Y = Q V; Y_bar = Q R_bar[:, k:]
      if (!mm(gemm(m, k, n - k, e.M + k, n, 1, Rb + k, 1, n, W, k, 1, 1.0, 1.0))) return false;
    }
    // X = U Rb_k^T - W^T Q (k x k), Rb_k = R_bar[:, :k]
    if (!mm(gemm(k, k, k, e.R, n, 1, Rb, 1, n, X, k, 1))) return false;
    if (!mm(gemm(k, k, m, W, 1, k, e.Q, k, 1, X, k, 1, -1.0, 1.0))) return false;
    hipLaunchKernelGGL(mirror_lower_kernel, dim3(grid_for((int64_t)k * k)), dim3(NT), 0, st, X, k, (int64_t)k);
    if (!ok(hipGetLastError(), "a mirror of the QR adjoint")) return false;
    // W <- W + Q X (m x k), then M_bar[:, :k] = W U^{-T}
    if (!mm(gemm(m, k, k, e.Q, k, 1, X, k, 1, W, k, 1, 1.0, 1.0))) return false;
    double *Wt = S[3];
    hipLaunchKernelGGL(trsm_rt_kernel, dim3((m + 63) / 64), dim3(64), 0, st, Wt, W, e.R, m, k, (int64_t)n);
    if (!ok(hipGetLastError(), "the triangular solve of the QR adjoint")) return false;
    if (k == n) return copy(Mb, Wt, (int64_t)m * n);
    // wide: M_bar = [Wt | Q R_bar[:, k:]]  (row-major m x n)
    if (!mm(gemm(m, n - k, k, e.Q, k, 1, Rb + k, n, 1, Mb + k, n, 1))) return false;
    hipLaunchKernelGGL(copy2d_kernel, dim3(grid_for((int64_t)m * k)), dim3(NT), 0, st, Mb, (int64_t)n, Wt,
                       (int64_t)k, m, k);
    return ok(hipGetLastError(), "a block copy of the QR adjoint");
  }
};

struct Slot {
  double *p = nullptr;
  int rl = 0, d = 0, rr = 0;
};

size_t al(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

struct VjpLayout {
  size_t fwd = 0, tape = 0, slots = 0, scratch = 0, total = 0;
  int64_t core = 0, sc = 0;
  int nslots = 0;
};

int vjp_layout(const ttm_tt *A, const ttm_tt *B, int chi_out, const ttm_options *opt, VjpLayout &L,
               int64_t *out_capacity) {
  size_t fwd = 0;
  int64_t tape = 0, max_core = 0, max_mn = 0, cap = 0;
  const int e = vjp_sizes(A, B, chi_out, opt, &fwd, &tape, &max_core, &max_mn, &cap);
  if (e) return e;
  // the cotangents of A's, B's (twice: reversed and not) and the product's
  // cores, the moving carriage's two, and one spare
  L.nslots = 4 * A->n_sites + 3;
  L.core = std::max<int64_t>(max_core, 1);
  L.sc = std::max<int64_t>(std::max(max_mn, max_core), 1);
  L.fwd = al(fwd);
  L.tape = al((size_t)tape * 8);
  L.slots = (size_t)L.nslots * al((size_t)L.core * 8);
  L.scratch = 8 * al((size_t)L.sc * 8);
  L.total = L.fwd + L.tape + L.slots + L.scratch;
  if (out_capacity) *out_capacity = cap;
  return TTM_OK;
}

int run_vjp(const ttm_tt *A, const ttm_tt *B, int chi_out, double tol, const ttm_options *opt, const ttm_tt *Cbar,
            ttm_tt_out *C, double *dA, double *dB, void *ws, size_t ws_bytes, hipStream_t st, ttm_stats *stats,
            bool &enqueued) {
  VjpLayout L;
  int64_t cap = 0;
  int e = vjp_layout(A, B, chi_out, opt, L, &cap);
  if (e) return e;
  if (!ws || ws_bytes < L.total) return TTM_EWORKSPACE;
  if (!C || !C->bonds || !C->offsets || !C->data) return TTM_EINVAL;
  if (C->capacity < cap) return TTM_ECAPACITY;
  if (!Cbar || !Cbar->data || !Cbar->bonds || !Cbar->offsets || !Cbar->phys || !dA || !dB) return TTM_EINVAL;
  const int n = A->n_sites;
  if (Cbar->n_sites != n || Cbar->dtype != TTM_F64) return TTM_ESHAPE;
  char *base = static_cast<char *>(ws);
  Tape tape;
  tape.base = reinterpret_cast<double *>(base + L.fwd);
  tape.cap = L.tape / 8;
  bool swapped = false;
  enqueued = true;
  e = run_ttm_taped(A, B, chi_out, tol, opt, C, ws, L.fwd, st, stats, &tape, &swapped);
  if (e) return e;
  for (int i = 0; i < n; ++i)
    if (Cbar->phys[i] != A->phys[i] || Cbar->bonds[i] != C->bonds[i]) return TTM_ESHAPE;
  if (Cbar->bonds[n] != C->bonds[n]) return TTM_ESHAPE;
  const ttm_tt *Af = swapped ? B : A;  // the trains in the roles the product gave them
  const ttm_tt *Bf = swapped ? A : B;

  Back bk;
  bk.st = st;
  char *sbase = base + L.fwd + L.tape;
  std::vector<double *> pool;
  for (int i = 0; i < L.nslots; ++i) pool.push_back(reinterpret_cast<double *>(sbase + (size_t)i * al((size_t)L.core * 8)));
  char *xbase = sbase + L.slots;
  for (int i = 0; i < 8; ++i) bk.S[i] = reinterpret_cast<double *>(xbase + (size_t)i * al((size_t)L.sc * 8));
  bk.scap = (size_t)L.sc;
  size_t next = 0;
  auto slot = [&](int rl, int d, int rr) {
    Slot s;
    s.p = pool[next++];
    s.rl = rl; s.d = d; s.rr = rr;
    return s;
  };
  std::vector<Slot> Ab(n), Bb(n), Btb(n), Pib(n);
  for (int i = 0; i < n; ++i) {
    Pib[i] = slot(Cbar->bonds[i], Cbar->phys[i], Cbar->bonds[i + 1]);
    if (!bk.copy(Pib[i].p, static_cast<const double *>(Cbar->data) + Cbar->offsets[i],
                 (int64_t)Pib[i].rl * Pib[i].d * Pib[i].rr))
      return bk.err;
  }
  Slot Xb = slot(0, 0, 0), tmp = slot(0, 0, 0), tmp2 = slot(0, 0, 0);
  for (int i = 0; i < n; ++i) {
    Ab[i] = slot(0, 0, 0);
    Btb[i] = slot(0, 0, 0);
    Bb[i] = slot(0, 0, 0);
  }
  const std::vector<TapeEntry> &E = tape.e;
  for (size_t q = E.size(); q-- > 0 && bk.err == TTM_OK;) {
    const TapeEntry &t = E[q];
    if (t.kind == TapeEntry::ROUND) {
      const int i = t.p, m = t.m, nn = t.n, r = t.r, nc = t.ncol;
      Slot &nb = Pib[i + 1];
      double *Zb = bk.S[7], *Vrb = bk.S[1];
      // Z_bar (nn x r, row-major) = nxt nb^T; the old next core's cotangent = Zt^T nb
      if (!bk.mm(gemm(nn, r, nc, t.nxt, nc, 1, nb.p, 1, nc, Zb, r, 1))) break;
      if (!bk.mm(gemm(nn, nc, r, t.Zt, 1, nn, nb.p, nc, 1, tmp.p, nc, 1))) break;
      std::swap(nb.p, tmp.p);
      nb.rl = nn;
      // V_r_bar: the cotangent of U_r (m x r, row-major) as an m x r column-major block
      if (!bk.ok(launch_transpose(Vrb, Pib[i].p, m, r, st), "a transpose of the reverse mode")) break;
      // Y = Pi_i^T (nn x m, column-major: Pi_i's row-major storage); its right
      // singular vectors are Pi_i's left ones; Z = Y U_r = Zt^T
      if (!bk.svd_adjoint(t.M, nn, m, t.V, t.sigma, r, t.kg, t.Zt, 1, nn, Zb, Vrb, tmp.p)) break;
      std::swap(Pib[i].p, tmp.p);
      Pib[i].rl = t.rl; Pib[i].d = t.d; Pib[i].rr = nn;
    } else if (t.kind == TapeEntry::SWAP) {
      const int m = t.m, nn = t.n, r = t.r;
      double *thb = bk.S[0], *Vrb = bk.S[1], *T = bk.S[7];
      // the cotangent of P' = V_r^T (r x nn, row-major) is V_r_bar as nn x r column-major
      if (!bk.copy(Vrb, Pib[t.p].p, (int64_t)r * nn)) break;
      if (!bk.svd_adjoint(t.theta, m, nn, t.V, t.sigma, r, t.kg, t.Z, r, 1, Xb.p, Vrb, thb)) break;
      hipLaunchKernelGGL(legs_back_kernel, dim3(grid_for((int64_t)m * nn)), dim3(NT), 0, st, thb, t.dl, t.dp, t.dx,
                         t.dr, T);
      if (!bk.ok(hipGetLastError(), "the leg exchange of the reverse mode")) break;
      const int64_t wd = (int64_t)t.dx * t.dr;
      // P_bar = T X^T ([dl dp] x dm), X_bar = P^T T (dm x [dx dr])
      if (!bk.mm(gemm(t.dl * t.dp, t.dm, (int)wd, T, wd, 1, t.X, 1, wd, tmp.p, t.dm, 1))) break;
      if (!bk.mm(gemm(t.dm, (int)wd, t.dl * t.dp, t.P, 1, t.dm, T, wd, 1, tmp2.p, wd, 1))) break;
      std::swap(Pib[t.p].p, tmp.p);
      Pib[t.p].rl = t.dl; Pib[t.p].d = t.dp; Pib[t.p].rr = t.dm;
      std::swap(Xb.p, tmp2.p);
      Xb.rl = t.dm; Xb.d = t.dx; Xb.rr = t.dr;
      if (t.p == n - 1) {  // the chain's first swap took B~_j
        std::swap(Btb[t.j].p, Xb.p);
        Btb[t.j].rl = Xb.rl; Btb[t.j].d = Xb.d; Btb[t.j].rr = Xb.rr;
      }
    } else if (t.kind == TapeEntry::CONTRACT) {
      const int j = t.p, dl = t.dl, d = t.d, dm = t.dm, dr = t.dr;
      const Slot &pb = Pib[j];
      // K_bar[a,e,c] = sum_b Pi_bar[a,e,b] X[c,e,b];  X_bar[c,e,b] = sum_a K[a,e,c] Pi_bar[a,e,b]
      GemmArgs gk = gemm(dl, dm, dr, pb.p, (int64_t)d * dr, 1, t.X, 1, (int64_t)d * dr, Ab[j].p, (int64_t)d * dm, 1);
      gk.batch = d; gk.a_bs = dr; gk.b_bs = dr; gk.c_bs = dm;
      double *xdst = (j == n - 1) ? Btb[n - 1].p : Xb.p;
      GemmArgs gx = gemm(dm, dr, dl, t.K, 1, (int64_t)d * dm, pb.p, (int64_t)d * dr, 1, xdst, (int64_t)d * dr, 1);
      gx.batch = d; gx.a_bs = dm; gx.b_bs = dr; gx.c_bs = dr;
      if (!bk.mm(gk) || !bk.mm(gx)) break;
      Ab[j].rl = dl; Ab[j].d = d; Ab[j].rr = dm;
      if (j == n - 1) {
        Btb[n - 1].rl = dm; Btb[n - 1].d = d; Btb[n - 1].rr = dr;
      } else {
        Xb.rl = dm; Xb.d = d; Xb.rr = dr;
      }
    } else if (t.kind == TapeEntry::REVERSE) {
      for (int i = 0; i < n; ++i) {
        // B~_i[b, w, a] = B_i[a, w, b]: the cotangent is reversed back
        if (!bk.ok(launch_reverse_core(Bb[i].p, Btb[i].p, Btb[i].rl, Btb[i].d, Btb[i].rr, st),
                   "a reversal of the reverse mode"))
          break;
        Bb[i].rl = Btb[i].rr; Bb[i].d = Btb[i].d; Bb[i].rr = Btb[i].rl;
      }
    } else {  // QR
      std::vector<Slot> &cb = (t.arr == 0) ? Ab : (t.arr == 1) ? Bb : Pib;
      if (!bk.qr_adjoint(t, cb[t.p].p, cb[t.p + 1].p, cb[t.p].p, tmp.p)) break;
      std::swap(cb[t.p + 1].p, tmp.p);
      cb[t.p + 1].rl = t.n;
      cb[t.p].rl = t.rl; cb[t.p].d = t.d; cb[t.p].rr = t.n;
    }
  }
  if (bk.err) return bk.err;
  // the input trains' cotangents, in the caller's layouts
  for (int i = 0; i < n; ++i) {
    const int64_t sa = (int64_t)Af->bonds[i] * Af->phys[i] * Af->bonds[i + 1];
    const int64_t sb = (int64_t)Bf->bonds[i] * Bf->phys[i] * Bf->bonds[i + 1];
    double *da = swapped ? dB : dA, *db = swapped ? dA : dB;
    if (!bk.copy(da + Af->offsets[i], Ab[i].p, sa) || !bk.copy(db + Bf->offsets[i], Bb[i].p, sb)) return bk.err;
  }
  const hipError_t h = hipStreamSynchronize(st);
  if (h != hipSuccess) {
    note_hip_error(h, "the synchronisation at the end of ttm_multiply_vjp");
    return TTM_EHIP;
  }
  return TTM_OK;
}

}  // namespace
}  // namespace ttm

extern "C" int ttm_vjp_query(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, const ttm_options *opt,
                             size_t *ws_bytes, int64_t *out_capacity) {
  ttm::VjpLayout L;
  const int e = ttm::vjp_layout(A, B, chi_out, opt, L, out_capacity);
  if (e) return e;
  if (ws_bytes) *ws_bytes = L.total;
  return TTM_OK;
}

extern "C" int ttm_multiply_vjp(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol,
                                const ttm_options *opt, const ttm_tt *Cbar, ttm_tt_out *C, double *dA, double *dB,
                                void *ws, size_t ws_bytes, void *stream, ttm_stats *stats) {
  ttm::clear_last_error();
  if (!(tol >= 0.0) || !isfinite(tol)) return TTM_EINVAL;
  if (opt && opt->profile != 0) return TTM_EINVAL;
  bool enqueued = false;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int e = ttm::run_vjp(A, B, chi_out, tol, opt, Cbar, C, dA, dB, ws, ws_bytes, st, stats, enqueued);
  if (e != TTM_OK && enqueued) (void)hipStreamSynchronize(st);
  return e;
}
