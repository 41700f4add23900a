// One-sided block Jacobi SVD (Hestenes) for the swap and rounding SVDs.
//
// The Swap of Sec. II.B needs the full singular spectrum of each unfolded
// pair (the rule of Eq. (eps) sums the discarded weight from the smallest
// value up) and the leading singular vectors on the side that must come out
// orthonormal.  One-sided Jacobi orthogonalises the columns of an L x nc
// matrix W by plane rotations; at convergence W = U S, so the normalised
// columns are orthonormal singular vectors over W's row index and the column
// norms are the singular values, with high relative accuracy.  The rotations
// themselves are not accumulated: the driver (svd.hip) arranges W so that
// its rows index the orthonormal side and recovers the other factor with one
// product.
//
// Blocked form: the columns are split into blocks of width bw; a sweep is a
// round-robin tournament over blocks, every round pairing all blocks at once.
// For a pair (I, J) the 2bw x 2bw Gram matrix G = [W_I W_J]^T [W_I W_J] is
// formed from row chunks (partial sums in the workspace); one workgroup per
// pair reduces the partials in a fixed order and diagonalises G by one
// cyclic sweep of two-sided Jacobi in LDS, and the accumulated 2bw x 2bw
// rotation is applied to the pair's columns of W by a third kernel.  A
// rotation is applied only where |g_pq| > tol sqrt(g_pp g_qq); a sweep in
// which no pair exceeds tol means the columns are orthogonal to working
// accuracy.
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
constexpr int JNT = 256;           // threads of the Gram / apply / helper kernels
constexpr int ROWS_PER_WG = 128;   // row chunk of a Gram / apply workgroup (circle pairing)
constexpr int ROWS_XOR = 64;       // row chunk with XOR pairing

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

// XOR pairing over n = 2^k blocks: round r pairs block i with i ^ (r + 1).
// Pair `pair` of the round is the `pair`-th block i < i ^ m (m = r + 1),
// i.e. `pair` with a zero bit inserted at the highest set bit h of m.
__device__ __forceinline__ int insert_zero_bit(int x, int b) { return ((x >> b) << (b + 1)) | (x & ((1 << b) - 1)); }
__device__ __forceinline__ int remove_bit(int x, int b) { return ((x >> (b + 1)) << b) | (x & ((1 << b) - 1)); }
__device__ __forceinline__ int high_bit(int m) { return 31 - __clz(m); }
__device__ __forceinline__ void xor_pair(int round, int pair, int &a, int &b) {
  const int m = round + 1;
  a = insert_zero_bit(pair, high_bit(m));
  b = a ^ m;
}
// Blocks of pair `pair` in round `round` under the plan's pairing.
__device__ __forceinline__ void pair_blocks(int xs, int n, int round, int pair, int &a, int &b) {
  if (xs)
    xor_pair(round, pair, a, b);
  else
    rr_pair(n, round, pair, a, b);
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

JacobiPlan jacobi_plan(int L, int nc, int force_bw) {
  JacobiPlan p;
  p.L = L;
  p.nc = nc;
  // Block width 16 (32-column pairs, 256-thread solve), or 32 (64-column
  // pairs, 1024-thread solve) from 8192 rows and 256 columns up.  Every
  // round streams W through the Gram and apply kernels, so wider pairs, with
  // half the rounds per sweep, halve that traffic; but each of their twice
  // as many inner steps moves four times the LDS bytes, which costs more
  // than the rounds saved until W is large enough for the rounds to be HBM
  // bound.  Columns are padded with zeros to a whole even number of blocks;
  // zero columns never rotate.
  int bw = (L >= 8192 && nc > 256) ? 32 : 16;
  if (force_bw == 16 || force_bw == 32) bw = force_bw;  // testing hook
  int nblk = (nc + bw - 1) / bw;
  if (nblk < 2) nblk = 2;
  if (nblk & 1) ++nblk;
  p.bw = bw;
  p.nblk = nblk;
  p.ncp = nblk * bw;
  // XOR pairing for 32-column pairs when the block count is a power of two
  // (4 or more): consecutive rounds then exchange blocks within groups of
  // four, and one pass per round applies the rotations and forms the next
  // Grams (jacobi_xor_round_kernel).
  p.xs = (bw == 16 && nblk >= 4 && (nblk & (nblk - 1)) == 0) ? 1 : 0;
  p.rows_per_wg = p.xs ? ROWS_XOR : ROWS_PER_WG;
  p.sw = (L + p.rows_per_wg - 1) / p.rows_per_wg;
  p.rounds = nblk - 1;
  p.pairs = nblk / 2;
  // A Gram workgroup sums gsub consecutive row chunks
  // in its matrix-core accumulators, so that the solve reduces gsw partials
  // instead of sw: each partial is a full 2bw x 2bw Gram, and at 8192 rows
  // the partials of one round would otherwise be 268 MB written and read
  // back.  gsub is chosen to keep about 1024 Gram workgroups.  The XOR
  // rotate-and-Gram pass groups its row chunks the same way (one rotation
  // load and one partial per gsub chunks) for about 512 workgroups, and the
  // first round's Gram matches it (measured per product: 2458 -> 2268 ms at
  // chi = 256, 9994 -> 8599 ms at chi = 512; 1024 or 256 workgroups were
  // slower).
  p.gsub = std::max(1, std::min(p.sw, p.xs ? (p.nblk / 4) * p.sw / 512 : p.pairs * p.sw / 1024));
  p.gsw = (p.sw + p.gsub - 1) / p.gsub;
  return p;
}

size_t jacobi_ws_doubles(const JacobiPlan &p) {
  const size_t b2 = 2 * (size_t)p.bw;
  size_t n = 0;
  n += 2 * (size_t)p.L * p.ncp;               // W and its reordering buffer
  n += (size_t)p.pairs * p.gsw * b2 * b2;     // partial Grams
  n += (size_t)p.rounds * p.pairs;            // conv
  n += (size_t)p.pairs * b2 * b2;             // rotations of the current round
  n += (size_t)p.pairs;                       // rotation flags (ints)
  n += (size_t)p.ncp;                         // sigma
  n += (size_t)p.ncp;                         // perm (ints, padded as doubles)
  n += 8;                                     // result
  return n + 9 * 32;                          // each region is rounded up to 32 doubles
}

// ------------------------------------------------------------------ MFMA helpers
typedef double dbl4 __attribute__((ext_vector_type(4)));

// One wave computes a 16 x 16 tile D = sum_k A(i,k) B(k,j) over k < K (K a
// multiple of 4) with v_mfma_f64_16x16x4f64.  Lane l supplies A(l%16, k+l/16)
// and B(k+l/16, l%16); accumulator register t of lane l holds
// D(4t + l/16, l%16).  a(i,k) / b(k,j) are LDS accessors.
template <typename FA, typename FB>
__device__ __forceinline__ dbl4 mfma_tile_acc(FA a, FB b, int K, int lane, dbl4 acc) {
  const int r = lane & 15, kq = lane >> 4;
  for (int k = 0; k < K; k += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a(r, k + kq), b(k + kq, r), acc, 0, 0, 0);
  return acc;
}
template <typename FA, typename FB>
__device__ __forceinline__ dbl4 mfma_tile(FA a, FB b, int K, int lane) {
  const dbl4 zero = {0.0, 0.0, 0.0, 0.0};
  return mfma_tile_acc(a, b, K, lane, zero);
}

// ------------------------------------------------------------------ pair pieces
// A block pair is 2 BW columns: block bi, then block bj.
template <int BW>
struct Pair {
  static constexpr int B2 = 2 * BW;    // columns of the pair
  static constexpr int SNT = BW * BW;  // solve threads that own a 2 x 2 block of the Gram
  // 32-column pairs add SNT threads that accumulate the rotation in
  // registers (see solve_pair); 64-column pairs keep it in LDS.
  static constexpr bool QREG = (BW == 16);
  static constexpr int THREADS = QREG ? 2 * SNT : SNT;
  template <int RC>
  using Tile = double[RC][B2 + 1];  // one row chunk of the pair, zero beyond L
  typedef double Square[B2][B2 + 1];
};

template <int BW>
__device__ __forceinline__ int pair_col(int bi, int bj, int c) {
  return (c < BW) ? bi * BW + c : bj * BW + (c - BW);
}

// One row chunk of a pair in two halves: the thread's loads into
// registers, then their LDS stores, so that the loads of the next chunk can
// be in flight while the current one is consumed.
// Thread t loads row r0 + t % RC of the pair's columns t / RC + q JNT / RC,
// as 32-bit element offsets (BW L < 2^32) from one 64-bit base per block,
// which keeps the addresses of the in-flight loads out of the registers.
template <int BW, int RC>
__device__ __forceinline__ void fetch_pair_chunk(const double *__restrict__ W, int L, int bi, int bj, int chunk,
                                                 double (&v)[RC * Pair<BW>::B2 / JNT]) {
  constexpr int B2 = Pair<BW>::B2, PER = RC * B2 / JNT, CS = JNT / RC;
  static_assert(JNT % RC == 0 && BW % CS == 0, "whole columns per load round, rounds within a block");
  const int r0 = chunk * RC, nr = min(RC, L - r0), i = threadIdx.x % RC, c0 = threadIdx.x / RC;
  const double *wi = W + (int64_t)bi * BW * L, *wj = W + (int64_t)bj * BW * L;
  const unsigned o = (unsigned)(c0 * L + r0 + i);
  if (nr == RC) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int c = q * CS;  // column of the pair at load round q, relative to c0
      v[q] = (c < BW) ? wi[o + (unsigned)(c * L)] : wj[o + (unsigned)((c - BW) * L)];
    }
  } else {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int c = q * CS;
      v[q] = (i < nr) ? ((c < BW) ? wi[o + (unsigned)(c * L)] : wj[o + (unsigned)((c - BW) * L)]) : 0.0;
    }
  }
}
template <int BW, int RC>
__device__ __forceinline__ void stash_pair_chunk(const double (&v)[RC * Pair<BW>::B2 / JNT],
                                                 typename Pair<BW>::template Tile<RC> &P) {
  constexpr int B2 = Pair<BW>::B2, PER = RC * B2 / JNT;
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * JNT;
    P[e % RC][e / RC] = v[q];
  }
}

// Every load of the thread is issued before the first LDS store.
template <int BW, int RC>
__device__ __forceinline__ void load_pair_chunk(const double *__restrict__ W, int L, int bi, int bj, int chunk,
                                                typename Pair<BW>::template Tile<RC> &P) {
  constexpr int B2 = Pair<BW>::B2, PER = RC * B2 / JNT;
  const int r0 = chunk * RC, nr = min(RC, L - r0);
  double v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * JNT, c = e / RC, i = e % RC;
    v[q] = (i < nr) ? W[(int64_t)pair_col<BW>(bi, bj, c) * L + r0 + i] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = threadIdx.x + q * JNT;
    P[e % RC][e / RC] = v[q];
  }
}

// Rotation (c, s) annihilating g_pq of a symmetric 2 x 2 block, or (1, 0)
// when the pair is already orthogonal to tolerance (see the header).  With
// d = g_qq - g_pp and r = sqrt(d^2 + 4 g_pq^2), the smaller root of the
// rotation's quadratic is t = 2 g_pq sign(d) / (|d| + r) (Rutishauser's
// t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)) with zeta = d / (2 g_pq),
// multiplied through by |2 g_pq|), and c = 1 / sqrt(1 + t^2), s = c t.  t is
// invariant under a common scaling of d and g_pq, so both are first brought
// to [1/2, 1) by a power of two (no overflow or underflow in d^2).  The angle
// only has to be close (later sweeps revisit the pair), so r and t use the
// hardware FP64 reciprocal square root and reciprocal directly; c gets one
// Newton step so that c^2 + s^2 = 1 to rounding for the t used.  No branch:
// the identity is selected afterwards.  Every thread that computes a
// rotation from the same inputs gets bitwise the same result.
__device__ __forceinline__ void rot_params(double gpp, double gqq, double gpq, double thr, double tol2,
                                           double floor2, double &c, double &sn) {
  const double hi2 = fmax(gpp, gqq), lo2 = fmin(gpp, gqq);
  const bool on = hi2 > thr && gpq * gpq > tol2 * hi2 * (lo2 > thr ? lo2 : floor2);
  const double d0 = gqq - gpp, g0 = 2.0 * gpq;
  const int e = __builtin_amdgcn_frexp_exp(fmax(fabs(d0), fabs(g0)));
  const double d = __builtin_amdgcn_ldexp(d0, -e), g2 = __builtin_amdgcn_ldexp(g0, -e);
  const double r2 = fma(d, d, g2 * g2);
  const double r = r2 * __builtin_amdgcn_rsq(r2);
  const double t = (d >= 0.0 ? g2 : -g2) * __builtin_amdgcn_rcp(fabs(d) + r);
  const double x = fma(t, t, 1.0);
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  c = on ? y : 1.0;
  sn = on ? y * t : 0.0;
}

// Slot permutation of the circle-method tournament over n (even) indices.
// If step st pairs slots (2k, 2k + 1), k < n/2, holding the indices
// (st, n-1) for k = 0 and ((st + k) mod (n-1), (st - k) mod (n-1)) for
// k >= 1, then the index in slot a at step st sits in slot slot_next(a) at
// step st + 1: 0 -> 3, 1 -> 1, 2 -> 0, 2k -> 2k - 2, 2k + 1 -> 2k + 3,
// n - 1 -> n - 2.  It is one cycle over the n - 1 slots other than 1, so
// n - 1 steps bring every index back to its starting slot.  Moving the data
// by this fixed permutation after each step, with the indices starting in
// slot order, lets every step pair the same slots (2k, 2k + 1): all LDS
// addresses of a thread are loop invariant.
__device__ __forceinline__ int slot_next(int a, int n) {
  if (a == 0) return 3;
  if (a == 1) return 1;
  if (a == 2) return 0;
  if (a == n - 1) return n - 2;
  return (a & 1) ? a + 2 : a - 2;
}

// Shared memory of the block-pair solve: G and the accumulated rotation Q
// double-buffered (a step reads one copy and writes the other at permuted
// positions), rows padded to keep 16-byte alignment for paired loads.
template <int BW>
struct SolveSmem {
  static constexpr int LD = 2 * BW + 2;
  double Gb[2][2 * BW][LD];
  double Qb[2][2 * BW][LD];
  double redmax[BW * BW / 64];
  double cs[BW][2];  // rotations of the current step
};

// Solve of one block pair by its workgroup (BW * BW threads): reduce the sw
// partial Grams (part, B2 x B2 each, consecutive) in a fixed order, measure
// convergence (scaled off-diagonal maximum, returned in *mout in every
// thread), and when some index pair exceeds tol run one cyclic sweep of
// two-sided Jacobi on the B2 x B2 Gram in LDS, re-orthogonalise the
// accumulated rotation and hand it to store(i, j, q_ij).  Returns 0 (nothing
// stored) when no rotation is needed.  A step rotates BW disjoint index pairs
// at once; G <- J^T G J splits into independent 2 x 2 blocks, one per
// thread, read from one copy of G and written to the other.  Every workgroup
// that solves the same partials computes bitwise the same result.
template <int BW, typename Store>
__device__ int solve_pair(const double *__restrict__ part, int sw, double tol, double thr, double floor2,
                          SolveSmem<BW> &sm, double *mout, Store store) {
  constexpr int B2 = Pair<BW>::B2, SNT = Pair<BW>::SNT, NT = B2 / 16;
  static_assert(NT * NT == SNT / 64, "one 16 x 16 tile of the Newton-Schulz products per wave");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double tol2 = tol * tol;
  const int64_t pstride = (int64_t)B2 * B2;
  // Thread tid sums entries tid + SNT j, j < EPT, over the sw partials in
  // order s = 0, 1, ...; the loads of KB partials are issued before any add.
  constexpr int EPT = B2 * B2 / SNT, KB = (BW == 16) ? 16 : 8;
  const bool gt = tid < SNT;  // a Gram thread
  double acc[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) acc[j] = 0.0;
  const double *src = part + (gt ? tid : 0);
  for (int s0 = 0; gt && s0 < sw; s0 += KB) {
    double v[KB][EPT];
#pragma unroll
    for (int u = 0; u < KB; ++u)
#pragma unroll
      for (int j = 0; j < EPT; ++j) v[u][j] = (s0 + u < sw) ? src[(s0 + u) * pstride + j * SNT] : 0.0;
#pragma unroll
    for (int u = 0; u < KB; ++u)
#pragma unroll
      for (int j = 0; j < EPT; ++j) acc[j] += v[u][j];
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = tid + j * SNT, i = e / B2, k = e % B2;
    if (gt) {
      sm.Gb[0][i][k] = acc[j];
      sm.Qb[0][i][k] = (i == k) ? 1.0 : 0.0;
    }
  }
  __syncthreads();
  // Convergence measure of this visit (scaled off-diagonal, see the header),
  // squared: g_pq^2 / (hi^2 (lo^2 > thr ? lo^2 : floor2)), one root at the end.
  double m2 = 0.0;
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    const int e = (gt ? tid : 0) + j * SNT, p = e / B2, q = e % B2;
    const double gp = sm.Gb[0][p][p], gq = sm.Gb[0][q][q];
    const double hi2 = fmax(gp, gq), lo2 = fmin(gp, gq);
    if (gt && p < q && hi2 > thr) m2 = fmax(m2, acc[j] * acc[j] / (hi2 * (lo2 > thr ? lo2 : floor2)));
  }
  m2 = wave_max(m2);
  if (gt && lane == 0) sm.redmax[wave] = m2;
  __syncthreads();
  m2 = 0.0;
  for (int w = 0; w < SNT / 64; ++w) m2 = fmax(m2, sm.redmax[w]);
  const double m = sqrt(m2);
  *mout = m;
  if (!(m > tol)) return 0;  // no index pair above tolerance: nothing would rotate

  // One cyclic sweep of two-sided Jacobi over the B2 indices (B2 - 1 steps),
  // slots (2k, 2k + 1) paired at every step (see slot_next).  Gram thread
  // (u, v) owns the 2 x 2 block of G at slot pairs (u, v).  Per step: every
  // Gram thread loads its block while threads 0 .. BW-1 compute the step's
  // rotations into LDS; after one barrier each applies J_u^T (.) J_v to its
  // block and writes it to the other buffer at the slots of the next step.
  // The accumulated rotation Q (rows: the pair's columns, columns: slots):
  //  * 32-column pairs: thread SNT + 8 i + t holds Q(i, 4t .. 4t+3) in
  //    registers, applies the step's rotations of slot pairs 2t, 2t + 1 after
  //    the same barrier and moves its values to the next step's slots with
  //    two row shifts (slot_next moves one slot a lane down, one a lane up);
  //    it adds no LDS traffic to the Gram threads' critical path;
  //  * 64-column pairs: Gram thread (u, v) also owns rows 2u, 2u + 1 of Q at
  //    slot pair v, double-buffered in LDS like G.
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int u = tid / BW, v = tid % BW;
  const int nu0 = slot_next(2 * u, B2), nu1 = slot_next(2 * u + 1, B2);
  const int nv0 = slot_next(2 * v, B2), nv1 = slot_next(2 * v + 1, B2);
  const int qi = (tid - SNT) >> 3, qt = (tid - SNT) & 7;  // register-Q row and slot quad
  double q0 = 0.0, q1 = 0.0, q2 = 0.0, q3 = 0.0;
  if (Pair<BW>::QREG && !gt) {
    q0 = (qi == 4 * qt) ? 1.0 : 0.0;
    q1 = (qi == 4 * qt + 1) ? 1.0 : 0.0;
    q2 = (qi == 4 * qt + 2) ? 1.0 : 0.0;
    q3 = (qi == 4 * qt + 3) ? 1.0 : 0.0;
  }
  int cur = 0;
  for (int step = 0; step < B2 - 1; ++step) {
    double (*Gc)[SolveSmem<BW>::LD] = sm.Gb[cur];
    double (*Gn)[SolveSmem<BW>::LD] = sm.Gb[cur ^ 1];
    double (*Qc)[SolveSmem<BW>::LD] = sm.Qb[cur];
    double (*Qn)[SolveSmem<BW>::LD] = sm.Qb[cur ^ 1];
    d2 ga = {0.0, 0.0}, gb = {0.0, 0.0}, qa = {0.0, 0.0}, qb = {0.0, 0.0};
    if (gt) {
      ga = *(const d2 *)&Gc[2 * u][2 * v];
      gb = *(const d2 *)&Gc[2 * u + 1][2 * v];
      if (!Pair<BW>::QREG) {
        qa = *(const d2 *)&Qc[2 * u][2 * v];
        qb = *(const d2 *)&Qc[2 * u + 1][2 * v];
      }
    }
    if (tid < BW) {
      const d2 dg = *(const d2 *)&Gc[2 * tid][2 * tid];
      double c, sn;
      rot_params(dg.x, Gc[2 * tid + 1][2 * tid + 1], dg.y, thr, tol2, floor2, c, sn);
      const d2 cs = {c, sn};
      *(d2 *)&sm.cs[tid][0] = cs;
    }
    __syncthreads();
    if (gt) {
      const d2 ru = *(const d2 *)&sm.cs[u][0], rv = *(const d2 *)&sm.cs[v][0];
      const double cu = ru.x, su = ru.y, cv = rv.x, sv = rv.y;
      // rows (J_u^T), then columns (J_v)
      const double h00 = cu * ga.x - su * gb.x, h01 = cu * ga.y - su * gb.y;
      const double h10 = su * ga.x + cu * gb.x, h11 = su * ga.y + cu * gb.y;
      Gn[nu0][nv0] = cv * h00 - sv * h01;
      Gn[nu0][nv1] = sv * h00 + cv * h01;
      Gn[nu1][nv0] = cv * h10 - sv * h11;
      Gn[nu1][nv1] = sv * h10 + cv * h11;
      if (!Pair<BW>::QREG) {
        Qn[2 * u][nv0] = cv * qa.x - sv * qa.y;
        Qn[2 * u][nv1] = sv * qa.x + cv * qa.y;
        Qn[2 * u + 1][nv0] = cv * qb.x - sv * qb.y;
        Qn[2 * u + 1][nv1] = sv * qb.x + cv * qb.y;
      }
    } else if (Pair<BW>::QREG) {
      const d2 r0 = *(const d2 *)&sm.cs[2 * qt][0], r1 = *(const d2 *)&sm.cs[2 * qt + 1][0];
      const double n0 = r0.x * q0 - r0.y * q1, n1 = r0.y * q0 + r0.x * q1;
      const double n2 = r1.x * q2 - r1.y * q3, n3 = r1.y * q2 + r1.x * q3;
      // Slot 4t + 3 of the lane below moves to slot 4t + 1 here, slot 4t of
      // the lane above to slot 4t + 2 (row shifts by one lane); at the ends
      // of a row of Q (t = 0, t = 7) the moves stay within the lane.
      const double from_below = __builtin_amdgcn_mov_dpp(n3, 0x111, 0xf, 0xf, false);  // row_shr:1
      const double from_above = __builtin_amdgcn_mov_dpp(n0, 0x101, 0xf, 0xf, false);  // row_shl:1
      q0 = n2;
      q1 = (qt == 0) ? n1 : from_below;
      q2 = (qt == 7) ? n3 : from_above;
      q3 = (qt == 0) ? n0 : n1;
    }
    cur ^= 1;
    __syncthreads();
  }
  // B2 - 1 steps have returned every index to its own slot: Q is in index
  // order.  G is no longer needed; its other buffer holds Q^T Q below.
  double (*Qf)[SolveSmem<BW>::LD] = Pair<BW>::QREG ? sm.Qb[0] : sm.Qb[cur];
  double (*Sq)[SolveSmem<BW>::LD] = sm.Gb[0];
  if (Pair<BW>::QREG) {
    if (!gt) {
      const d2 a = {q0, q1}, b = {q2, q3};
      *(d2 *)&Qf[qi][4 * qt] = a;
      *(d2 *)&Qf[qi][4 * qt + 2] = b;
    }
    __syncthreads();
  }

  // One Newton-Schulz step, Q <- Q (3I - Q^T Q) / 2, restores orthogonality
  // to rounding level; without it the O(u) drift of every visit accumulates
  // over the thousands of visits a column receives.  B2 x B2 products on
  // MFMA, one 16 x 16 tile per wave.
  const int ti = wave / NT, tj = wave % NT;
  if (gt) {
    dbl4 a4 = mfma_tile([&](int i, int k) { return Qf[k][ti * 16 + i]; },
                        [&](int k, int j) { return Qf[k][tj * 16 + j]; }, B2, lane);
    for (int t = 0; t < 4; ++t) Sq[ti * 16 + 4 * t + (lane >> 4)][tj * 16 + (lane & 15)] = a4[t];
  }
  __syncthreads();
  if (gt) {
    dbl4 a4 = mfma_tile([&](int i, int k) { return Qf[ti * 16 + i][k]; },
                        [&](int k, int j) { return Sq[k][tj * 16 + j]; }, B2, lane);
    for (int t = 0; t < 4; ++t) {
      const int i = ti * 16 + 4 * t + (lane >> 4), j = tj * 16 + (lane & 15);
      store(i, j, 1.5 * Qf[i][j] - 0.5 * a4[t]);
    }
  }
  return 1;
}

// ------------------------------------------------------------------ kernels of a round
// grid (pairs, gsw).  Partial Gram of every block pair over gsub
// consecutive row chunks, accumulated on the matrix cores (each wave owns
// the same 16 x 16 output tiles throughout) and stored once.  For 64-column
// pairs only the ten tiles on and above the diagonal are formed (62.5% of
// the products; the lower tiles are stored as their transposes): each wave
// takes a quarter of the chunk's rows and forms all ten tiles over them,
// with the four 16-column operand blocks of a k-step loaded once for ten
// products, and the four waves' tiles are summed through LDS at the end.
template <int BW, int RC>
__global__ __launch_bounds__(JNT) void jacobi_gram_kernel(const double *__restrict__ W, int L, int nblk, int xs,
                                                          int round, double *__restrict__ part, int gsw,
                                                          int gsub) {
  __shared__ typename Pair<BW>::template Tile<RC> P;
  constexpr int B2 = Pair<BW>::B2, NT = B2 / 16, TPW = NT * NT / (JNT / 64);
  static_assert(TPW * (JNT / 64) == NT * NT, "whole tiles per wave");
  const int pair = blockIdx.x, s = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int bi, bj;
  pair_blocks(xs, nblk, round, pair, bi, bj);
  if constexpr (BW == 32) {
    static_assert(JNT == 256 && RC % 16 == 0, "four waves, whole MFMA k-steps per wave");
    static_assert(sizeof(P) >= 3 * 10 * 256 * sizeof(double), "the tile exchange fits in the chunk tile");
    constexpr int RW = RC / 4;  // rows of a chunk per wave
    // upper tiles (ti, tj), ti <= tj, in the order (0,0) (0,1) (0,2) (0,3) (1,1) (1,2) (1,3) (2,2) (2,3) (3,3)
    constexpr int TI[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3}, TJ[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};
    dbl4 acc[10];
#pragma unroll
    for (int t = 0; t < 10; ++t) acc[t] = (dbl4){0.0, 0.0, 0.0, 0.0};
    const int r = lane & 15, kq = lane >> 4;
    // The chunks of this workgroup; the next one is fetched into registers
    // while the matrix cores work on the current one.
    const int c0 = s * gsub, nsub = max(0, min(gsub, (L + RC - 1) / RC - c0));
    double v[RC * B2 / JNT];
    if (nsub > 0) fetch_pair_chunk<BW, RC>(W, L, bi, bj, c0, v);
    for (int sub = 0; sub < nsub; ++sub) {
      if (sub > 0) __syncthreads();  // the previous chunk's tile has been read
      stash_pair_chunk<BW, RC>(v, P);
      __syncthreads();
      if (sub + 1 < nsub) fetch_pair_chunk<BW, RC>(W, L, bi, bj, c0 + sub + 1, v);
#pragma unroll
      for (int k = 0; k < RW; k += 4) {
        const int row = wave * RW + k + kq;
        double x[4];  // operand of 16-column block c at this k-step: P(row, 16 c + r)
#pragma unroll
        for (int c = 0; c < 4; ++c) x[c] = P[row][16 * c + r];
#pragma unroll
        for (int t = 0; t < 10; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[TI[t]], x[TJ[t]], acc[t], 0, 0, 0);
      }
    }
    __syncthreads();  // every wave is done with the chunk tile
    double *xch = &P[0][0];
    if (wave > 0)
#pragma unroll
      for (int t = 0; t < 10; ++t)
        for (int q = 0; q < 4; ++q) xch[((wave - 1) * 10 + t) * 256 + q * 64 + lane] = acc[t][q];
    __syncthreads();
    if (wave == 0) {
      double *out = part + ((int64_t)pair * gsw + s) * B2 * B2;
#pragma unroll
      for (int t = 0; t < 10; ++t) {
        for (int q = 0; q < 4; ++q) {
          double v = acc[t][q];
          for (int w = 0; w < 3; ++w) v += xch[(w * 10 + t) * 256 + q * 64 + lane];
          const int i = TI[t] * 16 + 4 * q + kq, j = TJ[t] * 16 + r;
          out[i * B2 + j] = v;
          if (TI[t] != TJ[t]) out[j * B2 + i] = v;
        }
      }
    }
    return;
  }
  dbl4 acc[TPW];
#pragma unroll
  for (int i = 0; i < TPW; ++i) acc[i] = (dbl4){0.0, 0.0, 0.0, 0.0};
  for (int sub = 0; sub < gsub; ++sub) {
    const int chunk = s * gsub + sub;
    if (chunk * RC >= L) break;  // uniform over the workgroup
    if (sub > 0) __syncthreads();  // the previous chunk's tile has been read
    load_pair_chunk<BW, RC>(W, L, bi, bj, chunk, P);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      const int t = wave + i * (JNT / 64), ti = t / NT, tj = t % NT;
      acc[i] = mfma_tile_acc([&](int r, int k) { return P[k][ti * 16 + r]; },
                             [&](int k, int j) { return P[k][tj * 16 + j]; }, RC, lane, acc[i]);
    }
  }
  double *out = part + ((int64_t)pair * gsw + s) * B2 * B2;
#pragma unroll
  for (int i = 0; i < TPW; ++i) {
    const int t = wave + i * (JNT / 64), ti = t / NT, tj = t % NT;
    for (int q = 0; q < 4; ++q) out[(ti * 16 + 4 * q + (lane >> 4)) * B2 + tj * 16 + (lane & 15)] = acc[i][q];
  }
}

// grid (pairs).  One workgroup per block pair: the solve, the rotation into
// qbuf[pair] (B2 x B2 row-major) and flag[pair] = 1 when it is not the identity.
template <int BW>
__global__ __launch_bounds__(Pair<BW>::THREADS) void jacobi_solve_kernel(int L, int nblk, int round,
                                                              const double *__restrict__ part, int sw,
                                                              double *__restrict__ conv, double tol,
                                                              const double *__restrict__ result, double noise2,
                                                              double *__restrict__ qbuf, int *__restrict__ flag) {
  __shared__ SolveSmem<BW> sm;
  constexpr int B2 = Pair<BW>::B2;
  const int pair = blockIdx.x;
  const double thr = noise2 * result[5];
  const double floor2 = result[5] / (double)L;  // (F / sqrt(L))^2
  double *qo = qbuf + (int64_t)pair * B2 * B2;
  double m;
  const int rot = solve_pair<BW>(part + (int64_t)pair * sw * B2 * B2, sw, tol, thr, floor2, sm, &m,
                                 [&](int i, int j, double q) { qo[i * B2 + j] = q; });
  if (threadIdx.x == 0) {
    conv[(int64_t)round * (nblk / 2) + pair] = m;
    flag[pair] = rot;
  }
}

// grid (pairs, sw).  Apply the stored rotation Q of each pair to one row
// chunk of W: W_rows <- W_rows Q.  Only Q is staged in LDS.  Each wave takes
// 16-row tiles and forms the transposed product Q^T W_rows^T on the matrix
// cores: the operand W_rows^T is then read straight from W with sixteen
// consecutive rows of one column per sixteen lanes, and the accumulator
// layout (lane l, register t: output column 4t + l/16 of the 16-column tile,
// row l%16) stores sixteen consecutive rows of a column per sixteen lanes.
// A wave reads all of its rows before it writes them.  A pair that did not
// rotate stores nothing.
template <int BW, int RC>
__global__ __launch_bounds__(JNT) void jacobi_apply_kernel(double *__restrict__ W, int L, int nblk, int xs,
                                                           int round, const double *__restrict__ qbuf,
                                                           const int *__restrict__ flag) {
  constexpr int B2 = Pair<BW>::B2, QPER = B2 * B2 / JNT, KS = B2 / 4, NC = B2 / 16;
  __shared__ double Qs[B2][B2 + 1];
  const int pair = blockIdx.x, chunk = blockIdx.y;
  if (flag[pair] == 0) return;  // uniform over the workgroup
  int bi, bj;
  pair_blocks(xs, nblk, round, pair, bi, bj);
  const double *qsrc = qbuf + (int64_t)pair * B2 * B2;
  double qv[QPER];
#pragma unroll
  for (int q = 0; q < QPER; ++q) qv[q] = qsrc[threadIdx.x + q * JNT];
#pragma unroll
  for (int q = 0; q < QPER; ++q) {
    const int e = threadIdx.x + q * JNT;
    Qs[e / B2][e % B2] = qv[q];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, r = lane & 15, kq = lane >> 4;
  for (int rt = wave; rt < RC / 16; rt += JNT / 64) {
    const int row = chunk * RC + rt * 16 + r;
    const bool in = row < L;
    double bv[KS];  // operand: W(row, 4k + kq)
#pragma unroll
    for (int k = 0; k < KS; ++k) bv[k] = in ? W[(int64_t)pair_col<BW>(bi, bj, 4 * k + kq) * L + row] : 0.0;
#pragma unroll
    for (int ct = 0; ct < NC; ++ct) {
      dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int k = 0; k < KS; ++k)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Qs[4 * k + kq][ct * 16 + r], bv[k], acc, 0, 0, 0);
      if (in) {
#pragma unroll
        for (int t = 0; t < 4; ++t) W[(int64_t)pair_col<BW>(bi, bj, ct * 16 + 4 * t + kq) * L + row] = acc[t];
      }
    }
  }
}

// grid (nblk / 4, sw), XOR pairing, 32-column pairs, in place.  Round
// `round` (mask m = round + 1) and the next (m' = round + 2) pair the four
// blocks {i, i^m, i^m', i^m^m'} among themselves: (i, i^m) and
// (i^m', i^m^m') now, (i, i^m') and (i^m, i^m^m') next.  One workgroup per
// such group and ROWS_XOR-row chunk applies both rotations of the round to
// its rows of the four blocks, writes them back and forms the two partial
// Grams of the next round over those rows: W is read and written once per
// round.  No LDS staging: the columns are loaded in the MFMA operand layout
// (lane l: row l % 16 of the wave's 16-row tile, column 4 k + l / 16 of the
// pair) and the accumulator layout of the rotation product (lane l,
// register t: row 4 t + l / 16, column l % 16) is the operand layout of the
// Gram product over those rows.  A pair that did not rotate goes through
// the identity (exact in FP64).
template <bool MULTI>
__global__ __launch_bounds__(JNT) void jacobi_xor_round_kernel(double *__restrict__ W, int L, int round,
                                                               const double *__restrict__ qbuf,
                                                               const int *__restrict__ flag,
                                                               double *__restrict__ part, int gsw, int xsub) {
  constexpr int BW = 16, B2 = 32, KS = B2 / 4;
  // LDS: the round's two rotations; one region for the two later phases:
  // each wave's 16 rows of the four new blocks, transposed for the stores,
  // then each wave's Gram tiles.  With one row chunk per workgroup (!MULTI)
  // the rotations are dead before the first store and share that region
  // (52 KB, three workgroups per CU); with several (MULTI) they are kept.
  typedef double QsT[2][B2][B2 + 1];
  typedef double TwT[JNT / 64][4 * 16][17];
  typedef double RedT[JNT / 64][2][3][16][17];
  __shared__ double qlds[MULTI ? sizeof(QsT) / sizeof(double) : 1];
  __shared__ double lds[sizeof(RedT) / sizeof(double)];
  static_assert(sizeof(RedT) >= sizeof(TwT) && sizeof(RedT) >= sizeof(QsT), "LDS phases");
  QsT &qs = *reinterpret_cast<QsT *>(MULTI ? qlds : lds);
  TwT &tw = *reinterpret_cast<TwT *>(lds);
  RedT &red = *reinterpret_cast<RedT *>(lds);
  const int s = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, r16 = lane & 15, q4 = lane >> 4;
  const int m = round + 1, mn = round + 2;
  // Group representative: zero bits at two positions that the span of m and
  // m' covers one-to-one (the highest bit of m, and of m' reduced by m).
  const int h1 = high_bit(m), mr = ((mn >> h1) & 1) ? (mn ^ m) : mn, h2 = high_bit(mr);
  const int blo = min(h1, h2), bhi = max(h1, h2);
  const int i0 = insert_zero_bit(insert_zero_bit(blockIdx.x, blo), bhi);
  const int blk[4] = {i0, i0 ^ m, i0 ^ mn, i0 ^ m ^ mn};
  // Row chunks s*xsub .. s*xsub + n - 1 of ROWS_XOR rows.  This lane's
  // operand values of a chunk: W(row, column 4 ks + q4 of pair pp) for the
  // row of the wave's 16-row tile.  The first chunk's loads are issued
  // before the rotations', and each later chunk's while the previous one is
  // still being rotated and stored.
  const int c0 = s * xsub, n = MULTI ? min(xsub, (L + ROWS_XOR - 1) / ROWS_XOR - c0) : 1;
  double wv[2][KS];
  auto fetch = [&](int chunk) {
    const int row = chunk * ROWS_XOR + 16 * w + r16;
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
      const int lo = min(blk[2 * pp], blk[2 * pp + 1]), hi = max(blk[2 * pp], blk[2 * pp + 1]);
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const int k = 4 * ks + q4;
        const int col = (k < BW) ? lo * BW + k : hi * BW + (k - BW);
        wv[pp][ks] = (row < L) ? W[(int64_t)col * L + row] : 0.0;
      }
    }
  };
  if (n > 0) fetch(c0);
  // The round's two rotations into LDS once (identity for a pair that did
  // not rotate).
  {
    // Both flags and both rotations are loaded unconditionally (qbuf holds a
    // matrix for every pair) and the identity is selected afterwards, so that
    // the loads are in flight together.
    double qg[2][B2 * B2 / JNT];
    int rot[2];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) rot[pp] = flag[remove_bit(min(blk[2 * pp], blk[2 * pp + 1]), h1)];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
      const double *Q = qbuf + (int64_t)remove_bit(min(blk[2 * pp], blk[2 * pp + 1]), h1) * B2 * B2;
#pragma unroll
      for (int e = 0; e < B2 * B2 / JNT; ++e) qg[pp][e] = Q[threadIdx.x + JNT * e];
    }
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
      for (int e = 0; e < B2 * B2 / JNT; ++e) {
        const int idx = threadIdx.x + JNT * e;
        qg[pp][e] = rot[pp] ? qg[pp][e] : ((idx / B2 == idx % B2) ? 1.0 : 0.0);
      }
#pragma unroll
    for (int pp = 0; pp < 2; ++pp)
#pragma unroll
      for (int e = 0; e < B2 * B2 / JNT; ++e) {
        const int idx = threadIdx.x + JNT * e;
        qs[pp][idx / B2][idx % B2] = qg[pp][e];
      }
  }
  __syncthreads();
  // The next round's Gram tiles accumulate over the chunks in the
  // matrix-core registers.
  dbl4 gt[2][3];
#pragma unroll
  for (int pp = 0; pp < 2; ++pp)
#pragma unroll
    for (int tl = 0; tl < 3; ++tl) gt[pp][tl] = (dbl4){0.0, 0.0, 0.0, 0.0};
  for (int sub = 0; sub < n; ++sub) {
    const int chunk = c0 + sub;
    const int row = chunk * ROWS_XOR + 16 * w + r16;  // this lane's row of the operand tile
    // The round's two pairs: (blk[0], blk[1]) and (blk[2], blk[3]), each as
    // (lower block, higher block) = columns 0..15, 16..31 of its rotation.
    dbl4 nb[4];
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
      const int x = blk[2 * pp], y = blk[2 * pp + 1];
      const int lo = min(x, y);
      double qv[2][KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) qv[ct][ks] = qs[pp][4 * ks + q4][ct * BW + r16];
      dbl4 d0 = {0.0, 0.0, 0.0, 0.0}, d1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        d0 = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[pp][ks], qv[0][ks], d0, 0, 0, 0);
        d1 = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[pp][ks], qv[1][ks], d1, 0, 0, 0);
      }
      // d0 is block lo, d1 block hi
      nb[2 * pp] = (x == lo) ? d0 : d1;
      nb[2 * pp + 1] = (x == lo) ? d1 : d0;
    }
    if (MULTI && sub + 1 < n) fetch(chunk + 1);
    // The next round's pairs: (blk[0], blk[2]) and (blk[1], blk[3]).
#pragma unroll
    for (int pp = 0; pp < 2; ++pp) {
      const int xa = blk[pp], xb = blk[pp + 2];
      const dbl4 A = (xa < xb) ? nb[pp] : nb[pp + 2], B = (xa < xb) ? nb[pp + 2] : nb[pp];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        gt[pp][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[t], A[t], gt[pp][0], 0, 0, 0);
        gt[pp][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(A[t], B[t], gt[pp][1], 0, 0, 0);
        gt[pp][2] = __builtin_amdgcn_mfma_f64_16x16x4f64(B[t], B[t], gt[pp][2], 0, 0, 0);
      }
    }
    // New columns back in place through LDS, so that a store covers 16
    // consecutive rows of a column (rows beyond L were zero, not stored).
    // Before the first store every wave must be done with the rotations
    // when they share the region; later, with the previous chunk's rows.
    if (sub > 0 || !MULTI) __syncthreads();
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) tw[w][b * BW + r16][4 * t + q4] = nb[b][t];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int c = 4 * e + q4;  // column c of the four blocks
      if (row < L) W[(int64_t)(blk[c >> 4] * BW + (c & 15)) * L + row] = tw[w][c][r16];
    }
  }
  __syncthreads();  // the transposed rows have been read out
#pragma unroll
  for (int pp = 0; pp < 2; ++pp)
#pragma unroll
    for (int tl = 0; tl < 3; ++tl)
#pragma unroll
      for (int t = 0; t < 4; ++t) red[w][pp][tl][4 * t + q4][r16] = gt[pp][tl][t];
  __syncthreads();
  // Sum over the waves (fixed order); tile (1,0) is the transpose of (0,1).
  const int ii = threadIdx.x >> 4, jj = threadIdx.x & 15;
  const int h1n = high_bit(mn);
#pragma unroll
  for (int pp = 0; pp < 2; ++pp) {
    const int lo = min(blk[pp], blk[pp + 2]);
    double *out = part + ((int64_t)remove_bit(lo, h1n) * gsw + s) * B2 * B2;
    double v[3];
#pragma unroll
    for (int tl = 0; tl < 3; ++tl)
      v[tl] = (red[0][pp][tl][ii][jj] + red[1][pp][tl][ii][jj]) + (red[2][pp][tl][ii][jj] + red[3][pp][tl][ii][jj]);
    out[ii * B2 + jj] = v[0];
    out[ii * B2 + BW + jj] = v[1];
    out[(BW + jj) * B2 + ii] = v[1];
    out[(BW + ii) * B2 + BW + jj] = v[2];
  }
}

// result[3] = max of conv[0..n).
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

namespace {
template <int BW, int RC>
void launch_round(const JacobiPlan &p, const JacobiBufs &b, int round, double tol, double noise2, hipStream_t s,
                  KernelTimer *timer, bool gram, bool apply) {
  if (gram) {
    Timed tm(timer, KC_JAC_GRAM, s);
    hipLaunchKernelGGL((jacobi_gram_kernel<BW, RC>), dim3(p.pairs, p.gsw), dim3(JNT), 0, s, b.W, p.L, p.nblk,
                       p.xs, round, b.part, p.gsw, p.gsub);
  }
  {
    Timed tm(timer, KC_JAC_SOLVE, s);
    hipLaunchKernelGGL(jacobi_solve_kernel<BW>, dim3(p.pairs), dim3(Pair<BW>::THREADS), 0, s, p.L, p.nblk, round,
                       b.part, p.gsw, b.conv, tol, b.result, noise2, b.qbuf, b.flag);
  }
  if (apply) {
    Timed tm(timer, KC_JAC_APPLY, s);
    hipLaunchKernelGGL((jacobi_apply_kernel<BW, RC>), dim3(p.pairs, p.sw), dim3(JNT), 0, s, b.W, p.L, p.nblk, p.xs,
                       round, b.qbuf, b.flag);
  } else {
    // this round's rotations and the next round's Grams in one pass
    Timed tm(timer, KC_JAC_APPLY, s);
    if (p.gsub > 1)
      hipLaunchKernelGGL(jacobi_xor_round_kernel<true>, dim3(p.nblk / 4, p.gsw), dim3(JNT), 0, s, b.W, p.L, round,
                         b.qbuf, b.flag, b.part, p.gsw, p.gsub);
    else
      hipLaunchKernelGGL(jacobi_xor_round_kernel<false>, dim3(p.nblk / 4, p.gsw), dim3(JNT), 0, s, b.W, p.L,
                         round, b.qbuf, b.flag, b.part, p.gsw, 1);
  }
}
}  // namespace

hipError_t launch_jacobi_sweep(const JacobiPlan &p, const JacobiBufs &b, double tol, hipStream_t s,
                               KernelTimer *timer) {
  const double ns = 8.0 * sqrt((double)p.L) * 2.220446049250313e-16;
  const double noise2 = ns * ns;
  if (p.bw != 16 && p.bw != 32) return hipErrorInvalidValue;
  for (int round = 0; round < p.rounds; ++round) {
    if (p.bw == 32) {
      launch_round<32, ROWS_PER_WG>(p, b, round, tol, noise2, s, timer, true, true);
    } else if (p.xs) {
      // the Gram of round 0 alone; later Grams come with the previous
      // round's rotations; the last round's apply alone
      launch_round<16, ROWS_XOR>(p, b, round, tol, noise2, s, timer, round == 0, round + 1 == p.rounds);
    } else {
      launch_round<16, ROWS_PER_WG>(p, b, round, tol, noise2, s, timer, true, true);
    }
  }
  {
    Timed tm(timer, KC_JAC_OTHER, s);
    hipLaunchKernelGGL(jacobi_convmax_kernel, dim3(1), dim3(JNT), 0, s, b.conv, p.rounds * p.pairs, b.result);
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
// The position of value c is the count of values ahead of it (larger, or
// equal at a lower index); eight lanes share that count for one value, lane
// q taking j = q, q + 8, ... (neighbouring LDS words, so no bank conflicts),
// and three lane exchanges add their counts.
constexpr int SORT_SPLIT = 8;
__global__ __launch_bounds__(JNT) void jacobi_sort_kernel(const double *__restrict__ sigma, int nc,
                                                          int *__restrict__ perm) {
  extern __shared__ double sv[];
  for (int i = threadIdx.x; i < nc; i += JNT) sv[i] = sigma[i];
  __syncthreads();
  const int c = blockIdx.x * (JNT / SORT_SPLIT) + threadIdx.x / SORT_SPLIT;
  const int q = threadIdx.x % SORT_SPLIT;
  const int cc = c < nc ? c : nc - 1;
  const double me = sv[cc];
  int pos = 0;
#pragma unroll 4
  for (int j = q; j < nc; j += SORT_SPLIT) {
    const double o = sv[j];
    pos += (int)((o > me) | ((o == me) & (j < cc)));
  }
  pos += __shfl_xor(pos, 1, 64);
  pos += __shfl_xor(pos, 2, 64);
  pos += __shfl_xor(pos, 4, 64);
  if (c < nc && q == 0) perm[pos] = c;
}

// Rule of Eq. (eps) on the sorted values.  One workgroup of 1024 threads:
// thread t owns the contiguous index range of chunk t (at most RANK_PER
// values, kept in registers); tails are suffix sums, within a chunk from its
// smallest value up, the chunk totals combined by a suffix scan.
// Values at or below the rounding-noise level nz = noise * ||W||_F are
// numerically zero: the sweeps neither rotate nor converge pairs of such
// columns, so their normalised columns are not orthonormal singular vectors
// and are never kept (r <= the count of values above nz), whatever eps; with
// eps at or above the square of that level the rule drops them anyway.
constexpr int RANK_PER = 8;  // n <= 8192
__global__ __launch_bounds__(1024) void jacobi_rank_kernel(const double *__restrict__ sigma,
                                                           const int *__restrict__ perm, int n,
                                                           double eps, double noise, int cap, int forced,
                                                           const double *__restrict__ full_total,
                                                           double *__restrict__ result) {
  __shared__ double csum[2][1024];
  __shared__ int best, nsig;
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  double suf[RANK_PER];  // suf[j] = sum over lo + j <= i < hi of s_i^2
  double local = 0.0;
#pragma unroll
  for (int j = RANK_PER - 1; j >= 0; --j) {
    if (lo + j < hi) {
      const double s = sigma[perm[lo + j]];
      local += s * s;
    }
    suf[j] = local;
  }
  csum[0][t] = local;
  if (t == 0) {
    best = n;
    nsig = 0;
  }
  __syncthreads();
  // Inclusive suffix scan of the chunk totals (fixed order: Hillis-Steele).
  int src = 0;
  for (int d = 1; d < nt; d <<= 1) {
    const double v = csum[src][t] + ((t + d < nt) ? csum[src][t + d] : 0.0);
    csum[src ^ 1][t] = v;
    src ^= 1;
    __syncthreads();
  }
  // With full_total, the weight outside the resolved values joins every
  // tail (and the total).
  const double wsum = csum[src][0];
  const double extra = full_total ? fmax(full_total[0] - wsum, 0.0) : 0.0;
  const double after = ((t + 1 < nt) ? csum[src][t + 1] : 0.0) + extra;  // sum over i >= hi
  const double total = wsum + extra;
  // The smallest kept count r < n whose tail (sum over i >= r) is zero or
  // below eps * total; the tail of kept = k + 1 is suf[k + 1 - lo] + after
  // inside the chunk and `after` at its end.
  int mine = n;
#pragma unroll
  for (int j = RANK_PER - 1; j >= 0; --j) {
    const int kept = lo + j + 1;
    if (lo + j < hi && kept < n) {
      const double tail = (j + 1 < RANK_PER && kept < hi) ? suf[j + 1] + after : after;
      if (tail <= 0.0 || tail < eps * total) mine = kept;
    }
  }
  if (mine < n) atomicMin(&best, mine);
  // values above the noise level (sorted, so they are the leading ones)
  const double nz2 = noise * noise * wsum;
  int above = 0;
#pragma unroll
  for (int j = 0; j < RANK_PER; ++j)
    if (lo + j < hi) {
      const double sv = sigma[perm[lo + j]];
      above += (sv * sv > nz2) ? 1 : 0;
    }
  if (above) atomicAdd(&nsig, above);
  __syncthreads();
  int r = min(best, nsig);
  if (r < 1) r = 1;
  if (cap > 0 && r > cap) r = cap;
  if (forced > 0) r = forced;
  if (r > n) r = n;
  // Discarded weight: the tail at r, written by the chunk that holds r.
#pragma unroll
  for (int j = 0; j < RANK_PER; ++j)
    if (lo + j < hi && lo + j == r) result[1] = suf[j] + after;
  if (t == 0) {
    if (r == n) result[1] = extra;
    result[0] = (double)r;
    result[2] = total;
    result[4] = isfinite(total) ? 0.0 : 1.0;
    result[6] = (double)nsig;  // values above the noise level (resolved vectors)
  }
}

hipError_t launch_jacobi_finish(const JacobiPlan &p, const JacobiBufs &b, double eps, int cap,
                                int forced, hipStream_t s, const double *full_total) {
  const int nc = p.nc;
  hipLaunchKernelGGL(jacobi_sigma_kernel, dim3((nc + 3) / 4), dim3(JNT), 0, s, b.W, p.L, nc, b.sigma);
  const size_t shm = (size_t)nc * sizeof(double);
  if (shm > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(jacobi_sort_kernel, dim3((nc + JNT / SORT_SPLIT - 1) / (JNT / SORT_SPLIT)), dim3(JNT), shm, s,
                     b.sigma, nc,
                     b.perm);
  if (nc > 1024 * RANK_PER) return hipErrorInvalidValue;
  const double noise = 8.0 * sqrt((double)p.L) * 2.220446049250313e-16;  // as in the sweeps
  hipLaunchKernelGGL(jacobi_rank_kernel, dim3(1), dim3(1024), 0, s, b.sigma, b.perm, nc, eps, noise, cap,
                     forced, full_total, b.result);
  return hipGetLastError();
}

// ------------------------------------------------------------------ column order
// dst[:, k] = src[:, perm[k]] for k < ncols; columns of L doubles.
__global__ void gather_columns_kernel(const double *__restrict__ src, const int *__restrict__ perm, int L,
                                      int ncols, double *__restrict__ dst) {
  const int64_t n = (int64_t)L * ncols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(e / L), i = (int)(e % L);
    dst[e] = src[(int64_t)perm[k] * L + i];
  }
}

hipError_t launch_gather_columns(const double *src, const int *perm, int L, int ncols, double *dst,
                                 hipStream_t s) {
  const int64_t tot = (int64_t)L * ncols;
  int64_t g = (tot + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(gather_columns_kernel, dim3((int)g), dim3(256), 0, s, src, perm, L, ncols, dst);
  return hipGetLastError();
}

hipError_t launch_column_norms(const double *W, int L, int nc, double *out, hipStream_t s) {
  hipLaunchKernelGGL(jacobi_sigma_kernel, dim3((nc + 3) / 4), dim3(JNT), 0, s, W, L, nc, out);
  return hipGetLastError();
}

hipError_t launch_sort_desc(const double *v, int n, int *perm, hipStream_t s) {
  const size_t shm = (size_t)n * sizeof(double);
  if (shm > 64 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(jacobi_sort_kernel, dim3((n + JNT / SORT_SPLIT - 1) / (JNT / SORT_SPLIT)), dim3(JNT), shm, s,
                     v, n, perm);
  return hipGetLastError();
}

hipError_t launch_jacobi_sort_columns(const JacobiPlan &p, JacobiBufs &b, hipStream_t s) {
  // De Rijk-style ordering: before each sweep the columns are sorted by
  // decreasing norm, so large columns meet each other first.  Zero padding
  // columns sort last.
  const int n = p.ncp;
  hipError_t e = launch_column_norms(b.W, p.L, n, b.sigma, s);
  if (e == hipSuccess) e = launch_sort_desc(b.sigma, n, b.perm, s);
  if (e == hipSuccess) e = launch_gather_columns(b.W, b.perm, p.L, n, b.Wt, s);
  double *t = b.W; b.W = b.Wt; b.Wt = t;
  return e;
}

// ------------------------------------------------------------------ write-out
// u[rowperm[j] * u_os + t * u_ts] = W[:, perm[t]](j) / sigma[perm[t]] for
// j < L, t < r: the leading r columns of W normalised, their rows put back
// in the caller's order (rowperm[j] = original index of row j; a null
// rowperm keeps the order).  Zero singular values give zero vectors.
__global__ void jacobi_write_u_kernel(const double *__restrict__ W, const double *__restrict__ sigma,
                                      const int *__restrict__ perm, const int *__restrict__ rowperm, int L,
                                      int r, double *__restrict__ u, int64_t u_os, int64_t u_ts) {
  const int64_t n = (int64_t)L * r;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int t = (int)(e / L), j = (int)(e % L);
    const int c = perm[t];
    const double sg = sigma[c];
    const double v = W[(int64_t)c * L + j];
    const int row = rowperm ? rowperm[j] : j;
    u[(int64_t)row * u_os + (int64_t)t * u_ts] = (sg > 0.0) ? v / sg : 0.0;
  }
}

hipError_t launch_jacobi_write_u(const JacobiPlan &p, const JacobiBufs &b, const int *rowperm, int r,
                                 double *u, int64_t u_os, int64_t u_ts, hipStream_t s) {
  const int64_t n = (int64_t)p.L * r;
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(jacobi_write_u_kernel, dim3((int)g), dim3(256), 0, s, b.W, b.sigma, b.perm, rowperm, p.L,
                     r, u, u_os, u_ts);
  return hipGetLastError();
}

// W (L x ncp, column-major) = R^T for R = the upper trapezoid of S[0:k, :]
// (S column-major, ld m, L = n columns): W[c*L + j] = S[j*m + c] for
// c < k, j >= c; zero below the diagonal of R and in padding columns.
// 32 x 32 tiles through LDS.
__global__ void rt_from_qr_kernel(const double *__restrict__ S, int m, int n, int k, int ncp,
                                  double *__restrict__ W) {
  __shared__ double tile[32][33];
  const int c0 = blockIdx.y * 32, j0 = blockIdx.x * 32;  // tile of R: rows c0.., cols j0..
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int q = ty; q < 32; q += 8) {
    const int j = j0 + q, c = c0 + tx;  // read S[j*m + c]: consecutive c along a column of S
    double v = 0.0;
    if (j < n && c < k && j >= c) v = S[(int64_t)j * m + c];
    tile[q][tx] = v;
  }
  __syncthreads();
  for (int q = ty; q < 32; q += 8) {
    const int c = c0 + q, j = j0 + tx;  // write W[c*L + j]: consecutive j
    if (c < ncp && j < n) W[(int64_t)c * n + j] = tile[tx][q];
  }
}

hipError_t launch_rt_from_qr(const double *S, int m, int n, int k, int ncp, double *W, hipStream_t s) {
  dim3 grid((n + 31) / 32, (ncp + 31) / 32);
  if (grid.y > 65535u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(rt_from_qr_kernel, grid, dim3(256), 0, s, S, m, n, k, ncp, W);
  return hipGetLastError();
}

// result[5] = sum_i x[i]^2 (the squared Frobenius norm from column norms).
hipError_t launch_frob_from_norms(const double *x, int n, double *result, hipStream_t s) {
  hipLaunchKernelGGL(jacobi_frob_kernel, dim3(1), dim3(1024), 0, s, x, (int64_t)n, result);
  return hipGetLastError();
}

}  // namespace ttm
