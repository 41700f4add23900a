// Blocked Householder QR (the geqrf / orgqr structure of LAPACK).
//
// Panels of QB = 16 columns are factored by one 1024-thread workgroup; the
// panel's reflectors H_0 ... H_15 are combined into the compact-WY block
// reflector I - V T V^T (T upper triangular, built column by column while the
// panel is factored), and the block reflector is applied to the trailing
// columns (and, when Q is wanted, to the identity) by one fused kernel whose
// two 16-wide products run on FP64 MFMA.
//
// Panel layout: thread (wave w, lane l) owns column l & 15 of the panel at
// the rows 64 s + 4 w + (l >> 4), s = 0 .. SL-1, in registers.  Every
// reduction over rows is then a per-lane sum, two shuffles across the four
// row groups of a wave and one LDS exchange across the 16 waves, and it
// yields the sums of all 16 columns at once: one pass gives v^T x for every
// trailing column of the panel and V^T v for T.  The column being reflected
// reaches every lane at its own rows by a DPP row broadcast (the 16 lanes
// of a row group hold the 16 columns at the same rows); T is assembled
// after the last column.
#include <hip/hip_cooperative_groups.h>

#include "ttm_internal.h"

namespace ttm {
namespace {
constexpr int QB = 16;              // panel width
constexpr int PNT = 1024;           // threads of a panel workgroup
constexpr int UNT = 256;            // threads of an update workgroup
constexpr int MAX_REG_SLOTS = 16;   // register panels cover up to 64 * 16 rows

typedef double dbl4 __attribute__((ext_vector_type(4)));

int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (int)g;
}

}  // namespace

// S[i + j*m] = M[i*rs + j*cs]
__global__ void strided_to_colmajor_kernel(double *__restrict__ S, const double *__restrict__ M, int m, int n,
                                           int64_t rs, int64_t cs) {
  const int64_t tot = (int64_t)m * n;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < tot;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % m), j = (int)(e / m);
    S[e] = M[(int64_t)i * rs + (int64_t)j * cs];
  }
}

// Block column pivoting for panel j0 (all PNT threads): the jb columns of
// largest norm among positions [j0, n) (norms over rows j0.. in cnorm) move
// to positions j0 .. j0+jb-1 in decreasing order (ties: lower position
// first), and the columns they displace take the vacated positions.  Whole
// columns move, since rows above j0 hold R.  perm[j] (the original index of
// the column at position j) follows the moves.  scratch: 2 * QB * m doubles.
constexpr int PIVOT_MAX_CAND = 8;  // candidates per thread: n - j0 <= PNT * 8
__device__ void panel_pivot(double *__restrict__ S, int m, int n, int j0, int jb,
                            const double *__restrict__ cnorm, int *__restrict__ perm,
                            double *__restrict__ scratch) {
  __shared__ double fv[PNT / 64][QB];  // each wave's top jb: values
  __shared__ int fi[PNT / 64][QB];     // and positions
  __shared__ int sel[QB], dpos[QB], vpos[QB], oldp[2 * QB];
  __shared__ int nmove;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // Order: larger norm first, then lower position; taken candidates get -1.
  auto better = [](double v1, int i1, double v2, int i2) { return v1 > v2 || (v1 == v2 && i1 < i2); };
  auto wave_best = [&](double &bv, int &bi) {
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (better(ov, oi, bv, bi)) {
        bv = ov;
        bi = oi;
      }
    }
  };
  double cv[PIVOT_MAX_CAND];
  int ci[PIVOT_MAX_CAND];
#pragma unroll
  for (int q = 0; q < PIVOT_MAX_CAND; ++q) {
    ci[q] = j0 + tid + PNT * q;
    cv[q] = (ci[q] < n) ? cnorm[ci[q]] : -1.0;
  }
  // Every wave: its own jb best candidates, by jb rounds of a wave arg-max.
  for (int t = 0; t < jb; ++t) {
    double bv = -2.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int q = 0; q < PIVOT_MAX_CAND; ++q)
      if (better(cv[q], ci[q], bv, bi)) {
        bv = cv[q];
        bi = ci[q];
      }
    wave_best(bv, bi);
#pragma unroll
    for (int q = 0; q < PIVOT_MAX_CAND; ++q)
      if (ci[q] == bi) cv[q] = -1.0;
    if (lane == 0) {
      fv[w][t] = bv;
      fi[w][t] = bi;
    }
  }
  __syncthreads();
  // Wave 0: the jb best of the 16 waves' finalists (each global top-jb
  // column is among its wave's top jb).
  if (w == 0) {
    constexpr int PER = (PNT / 64) * QB / 64;  // finalists per lane
    double gv[PER];
    int gi[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int f = lane + 64 * q, ww = f / QB, t = f % QB;
      gv[q] = (t < jb) ? fv[ww][t] : -2.0;
      gi[q] = (t < jb) ? fi[ww][t] : 0x7fffffff;
    }
    for (int t = 0; t < jb; ++t) {
      double bv = -2.0;
      int bi = 0x7fffffff;
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (better(gv[q], gi[q], bv, bi)) {
          bv = gv[q];
          bi = gi[q];
        }
      wave_best(bv, bi);
#pragma unroll
      for (int q = 0; q < PER; ++q)
        if (gi[q] == bi) gv[q] = -3.0;
      if (lane == 0) sel[t] = bi;
    }
  }
  __syncthreads();
  if (tid == 0) {
    int nd = 0, nv = 0;
    bool identity = true;
    for (int t = 0; t < jb; ++t) {
      const int pos = j0 + t;
      bool chosen = false;
      for (int u = 0; u < jb; ++u) chosen |= (sel[u] == pos);
      if (!chosen) dpos[nd++] = pos;
      if (sel[t] >= j0 + jb) vpos[nv++] = sel[t];
      identity &= (sel[t] == pos);
    }
    nmove = identity ? -1 : nd;
    for (int t = 0; t < jb; ++t) oldp[t] = perm[sel[t]];
    for (int d = 0; d < nd; ++d) oldp[QB + d] = perm[dpos[d]];
  }
  __syncthreads();
  const int nd = nmove;
  if (nd < 0) return;  // already in place
  const int64_t tot = (int64_t)(jb + nd) * m;
  for (int64_t e = tid; e < tot; e += PNT) {
    const int c = (int)(e / m), i = (int)(e % m);
    const int src = (c < jb) ? sel[c] : dpos[c - jb];
    scratch[e] = S[(int64_t)src * m + i];
  }
  __syncthreads();
  for (int64_t e = tid; e < tot; e += PNT) {
    const int c = (int)(e / m), i = (int)(e % m);
    const int dst = (c < jb) ? j0 + c : vpos[c - jb];
    S[(int64_t)dst * m + i] = scratch[e];
  }
  if (tid == 0) {
    for (int t = 0; t < jb; ++t) perm[j0 + t] = oldp[t];
    for (int d = 0; d < nd; ++d) perm[vpos[d]] = oldp[QB + d];
  }
  __syncthreads();
}

// Lane K of each row of 16 lanes to the whole row (64-bit DPP row broadcast).
template <int K>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + K, 0xf, 0xf, false);
}

// Sum of v over the four row groups of a wave (lanes c, c + 16, c + 32,
// c + 48) by the gfx950 lane swaps, which exchange rows of 16 lanes
// (permlane16) or halves of the wave (permlane32) between two registers.
// Every lane adds the same two operands in the same order, so the four
// lanes of a column get bitwise the same sum.
__device__ __forceinline__ double rowgroup_sum(double v) {
  unsigned lo = __double2loint(v), hi = __double2hiint(v);
  auto a = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  auto b = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  v = __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
  lo = __double2loint(v);
  hi = __double2hiint(v);
  a = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  b = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(b[0], a[0]) + __hiloint2double(b[1], a[1]);
}

// 1 / x from the hardware reciprocal and two Newton steps (x finite, nonzero).
__device__ __forceinline__ double recip(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = fma(fma(-x, y, 1.0), y, y);
  y = fma(fma(-x, y, 1.0), y, y);
  return y;
}

// Shared state of a register panel.
struct PanelSmem {
  double red[2][PNT / 64][QB];  // per-wave sums d_c (double-buffered by column parity)
  double xrow[2][QB];           // row CC of every column (same buffering)
  double zs[QB][QB + 1];        // zs[i][b] = v_b^T v_i, b < i
  double taus[QB];
  double Tl[QB][QB + 1];        // T, row r kept by lane r of row group 0 of wave 0
};

// Column I of the compact-WY factor T by lane c (row c of T):
// T(I, I) = tau_I, T(r, I) = -tau_I sum over r <= b < I of T(r, b) zs(I, b).
// Each lane reads and writes only its own row, so no barrier is needed
// between columns; zs(I, :) and tau_I must be visible.
__device__ __forceinline__ void t_column(PanelSmem &sm, int I, int c) {
  double a0 = 0.0, a1 = 0.0;
  for (int b = c; b < I; b += 2) {
    a0 = fma(sm.Tl[c][b], sm.zs[I][b], a0);
    if (b + 1 < I) a1 = fma(sm.Tl[c][b + 1], sm.zs[I][b + 1], a1);
  }
  sm.Tl[c][I] = (c < I) ? -sm.taus[I] * (a0 + a1) : (c == I ? sm.taus[I] : 0.0);
}

// Column CC of a register panel (see qr_panel_reg_kernel), one barrier.
// The row group of 16 lanes that holds a set of rows holds all 16 columns
// there, so lane (g, c) gets column CC at its own rows by a row broadcast
// from lane (g, CC).  One pass forms d_c = sum over rows below CC of
// x_CC x_c for every column c (d_CC is the squared norm below the pivot);
// with v = (1 at row CC, x_CC scale below), v^T x_c = x_c(CC) + scale d_c.
// A reflected column is left unscaled in registers: its lane keeps scale
// and beta, the scale is folded into the update coefficient of the columns
// to its right and into v_c^T v_CC, and the write-out applies it once.  Row
// sums: per lane over slots, the lane swaps over the four row groups, one
// LDS value per (wave, column); a lane reads four of the sixteen waves'
// values and the lane swaps finish the sum, so every lane of a column gets
// bitwise the same total.
template <int SL, int CC>
__device__ __forceinline__ void panel_column(double (&x)[SL], PanelSmem &sm, int w, int g, int c, int i0,
                                             double &myscale, double &mybeta) {
  constexpr int B = CC & 1;
  // Rows at or above the pivot (< 16) occur only in slot 0.
  double b[SL];
#pragma unroll
  for (int s = 0; s < SL; ++s) b[s] = row_bcast<CC>(x[s]);
  double dp[4] = {(i0 > CC) ? b[0] * x[0] : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 1; s < SL; ++s) dp[s & 3] = fma(b[s], x[s], dp[s & 3]);
  // T column CC - 2 (its zs and tau became visible at the last barrier).
  if (CC >= 2 && w == 0 && g == 0) t_column(sm, CC - 2, c);
  double d = rowgroup_sum((dp[0] + dp[1]) + (dp[2] + dp[3]));
  if (g == 0) sm.red[B][w][c] = d;
  if (i0 == CC) sm.xrow[B][c] = x[0];
  __syncthreads();
  const double dc = rowgroup_sum((sm.red[B][g][c] + sm.red[B][4 + g][c]) + (sm.red[B][8 + g][c] + sm.red[B][12 + g][c]));
  const double xnorm2 = row_bcast<CC>(dc);
  const double alpha = sm.xrow[B][CC], xc = sm.xrow[B][c];
  double tau = 0.0, scale = 0.0, beta = alpha;
  if (xnorm2 > 0.0) {
    beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
    tau = (beta - alpha) * recip(beta);
    scale = recip(alpha - beta);
  }
  // v^T x_c for the column as stored (for c < CC: v_CC^T v_c / scale_c).
  const double tot = fma(scale, dc, xc);
  // Columns right of CC: x <- x - tau (v^T x) v, v = (1 at CC, b scale below).
  const double f = (c > CC) ? tau * tot : 0.0, fs = f * scale;
  x[0] = (i0 > CC) ? fma(-fs, b[0], x[0]) : (i0 == CC ? x[0] - f : x[0]);
#pragma unroll
  for (int s = 1; s < SL; ++s) x[s] = fma(-fs, b[s], x[s]);
  if (c == CC) {
    myscale = scale;
    mybeta = beta;
  }
  // Sums v_b^T v_CC of the earlier reflectors, kept for T.
  if (w == 0 && g == 0) {
    if (c < CC) sm.zs[CC][c] = myscale * tot;
    if (c == CC) sm.taus[CC] = tau;
  }
}

template <int SL, int CC = 0>
__device__ __forceinline__ void panel_columns(double (&x)[SL], PanelSmem &sm, int jb, int w, int g, int c, int i0,
                                              double &myscale, double &mybeta) {
  if constexpr (CC < QB) {
    if (CC < jb) {
      panel_column<SL, CC>(x, sm, w, g, c, i0, myscale, mybeta);
      panel_columns<SL, CC + 1>(x, sm, jb, w, g, c, i0, myscale, mybeta);
    }
  }
}

// Factor columns j0 .. j0+jb-1 of S (column-major, ld m) in place, rows
// j0 .. m-1 (mv = m - j0 <= 64 * SL), after block column pivoting when
// cnorm is not null.  Each reflector is H = I - tau v v^T
// with v(pivot) = 1 (LAPACK dlarfg convention); R goes on and above the
// diagonal, v below it (the V that the updates read in place).  Also
// writes T (16 x 16, row-major, zero outside the leading jb x jb upper
// triangle) with H_0 H_1 ... H_{jb-1} = I - V T V^T.
template <int SL>
__global__ __launch_bounds__(PNT) void qr_panel_reg_kernel(double *__restrict__ S, int m, int n, int j0, int jb,
                                                           double *__restrict__ T,
                                                           const double *__restrict__ cnorm, int *__restrict__ perm,
                                                           double *__restrict__ pscratch) {
  if (cnorm) panel_pivot(S, m, n, j0, jb, cnorm, perm, pscratch);
  __shared__ PanelSmem sm;
  // The panel passes through LDS on the way in and out, so that global
  // loads and stores run along the columns.
  constexpr int RT = 64 * SL;
  __shared__ double tile[QB][RT + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int mv = m - j0;
  const int i0 = 4 * w + g;  // row of slot 0; slot s holds row i0 + 64 s
  double x[SL];
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int e = tid + PNT * q, cc = e / RT, i = e % RT;
    x[q] = (i < mv && cc < jb) ? S[(int64_t)(j0 + cc) * m + j0 + i] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int e = tid + PNT * q;
    tile[e / RT][e % RT] = x[q];
  }
  if (w == 0 && g == 0)
    for (int b = 0; b < QB; ++b) sm.Tl[c][b] = 0.0;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SL; ++s) x[s] = tile[c][i0 + 64 * s];
  double myscale = 0.0, mybeta = 0.0;  // of this lane's column once reflected
  panel_columns<SL>(x, sm, jb, w, g, c, i0, myscale, mybeta);
  // Column c: R above row c, beta at row c, v = x scale below.
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const int i = i0 + 64 * s;
    tile[c][i] = (i > c) ? x[s] * myscale : (i == c ? mybeta : x[s]);
  }
  __syncthreads();
  // The last two columns of T, then T out.
  if (w == 0 && g == 0) {
    if (jb >= 2) t_column(sm, jb - 2, c);
    t_column(sm, jb - 1, c);
    for (int b = 0; b < QB; ++b) T[c * QB + b] = (c < jb && b < jb) ? sm.Tl[c][b] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int e = tid + PNT * q, cc = e / RT, i = e % RT;
    if (i < mv) {
      const double val = tile[cc][i];
      if (cc < jb) S[(int64_t)(j0 + cc) * m + j0 + i] = val;
    }
  }
}

// Panels of 1024 < mv <= 2048 rows: rows 0 .. 1023 of the panel in
// registers as in qr_panel_reg_kernel<16>, rows 1024 .. 2047 in LDS
// (ext[c][r] = row 1024 + r of column c, 128 KB), both handled by the lane
// that owns the register rows r = i0 + 64 s.  Column CC's values at the LDS
// rows are read by all 16 lanes of a row group from one address
// (broadcast); only columns right of CC change, and the lane that writes
// ext[c][r] is in the wave that reads it at the next column, after its own
// write in program order.
constexpr int EXT_ROWS = 64 * MAX_REG_SLOTS;  // rows held in LDS
template <int CC>
__device__ __forceinline__ void panel_column_ext(double (&x)[MAX_REG_SLOTS], double (*ext)[EXT_ROWS + 1],
                                                 PanelSmem &sm, int w, int g, int c, int i0, double &myscale,
                                                 double &mybeta) {
  constexpr int SL = MAX_REG_SLOTS;
  constexpr int B = CC & 1;
  // LDS rows first, in short groups so that few loads are live at once.
  double dl[2] = {0.0, 0.0};
#pragma unroll 2
  for (int s = 0; s < SL; ++s) {
    const int r = i0 + 64 * s;
    dl[s & 1] = fma(ext[CC][r], ext[c][r], dl[s & 1]);
  }
  double b[SL];
#pragma unroll
  for (int s = 0; s < SL; ++s) b[s] = row_bcast<CC>(x[s]);
  double dp[4] = {(i0 > CC) ? b[0] * x[0] : 0.0, dl[0], dl[1], 0.0};
#pragma unroll
  for (int s = 1; s < SL; ++s) dp[s & 3] = fma(b[s], x[s], dp[s & 3]);
  if (CC >= 2 && w == 0 && g == 0) t_column(sm, CC - 2, c);
  double d = rowgroup_sum((dp[0] + dp[1]) + (dp[2] + dp[3]));
  if (g == 0) sm.red[B][w][c] = d;
  if (i0 == CC) sm.xrow[B][c] = x[0];
  __syncthreads();
  const double dc = rowgroup_sum((sm.red[B][g][c] + sm.red[B][4 + g][c]) + (sm.red[B][8 + g][c] + sm.red[B][12 + g][c]));
  const double xnorm2 = row_bcast<CC>(dc);
  const double alpha = sm.xrow[B][CC], xc = sm.xrow[B][c];
  double tau = 0.0, scale = 0.0, beta = alpha;
  if (xnorm2 > 0.0) {
    beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
    tau = (beta - alpha) * recip(beta);
    scale = recip(alpha - beta);
  }
  const double tot = fma(scale, dc, xc);
  const double f = (c > CC) ? tau * tot : 0.0, fs = f * scale;
  x[0] = (i0 > CC) ? fma(-fs, b[0], x[0]) : (i0 == CC ? x[0] - f : x[0]);
#pragma unroll
  for (int s = 1; s < SL; ++s) x[s] = fma(-fs, b[s], x[s]);
  if (c > CC) {
#pragma unroll 2
    for (int s = 0; s < SL; ++s) {
      const int r = i0 + 64 * s;
      ext[c][r] = fma(-fs, ext[CC][r], ext[c][r]);
    }
  }
  if (c == CC) {
    myscale = scale;
    mybeta = beta;
  }
  if (w == 0 && g == 0) {
    if (c < CC) sm.zs[CC][c] = myscale * tot;
    if (c == CC) sm.taus[CC] = tau;
  }
}

template <int CC = 0>
__device__ __forceinline__ void panel_columns_ext(double (&x)[MAX_REG_SLOTS], double (*ext)[EXT_ROWS + 1],
                                                  PanelSmem &sm, int jb, int w, int g, int c, int i0,
                                                  double &myscale, double &mybeta) {
  if constexpr (CC < QB) {
    if (CC < jb) {
      panel_column_ext<CC>(x, ext, sm, w, g, c, i0, myscale, mybeta);
      panel_columns_ext<CC + 1>(x, ext, sm, jb, w, g, c, i0, myscale, mybeta);
    }
  }
}

// As qr_panel_reg_kernel<16> for 1024 < mv <= 2048 rows (see
// panel_column_ext).  Loads and stores run along the columns through the
// LDS block: rows 0 .. 1023 pass through it into and out of registers
// first, then it holds rows 1024 .. 2047 for the factorisation.
__global__ __launch_bounds__(PNT) void qr_panel_ext_kernel(double *__restrict__ S, int m, int n, int j0, int jb,
                                                           double *__restrict__ T,
                                                           const double *__restrict__ cnorm,
                                                           int *__restrict__ perm, double *__restrict__ pscratch) {
  if (cnorm) panel_pivot(S, m, n, j0, jb, cnorm, perm, pscratch);
  __shared__ PanelSmem sm;
  __shared__ double ext[QB][EXT_ROWS + 1];
  constexpr int SL = MAX_REG_SLOTS;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int mv = m - j0;
  const int i0 = 4 * w + g;
  auto load_rows = [&](int base) {
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      const int e = tid + PNT * q, cc = e / EXT_ROWS, r = e % EXT_ROWS;
      ext[cc][r] = (base + r < mv && cc < jb) ? S[(int64_t)(j0 + cc) * m + j0 + base + r] : 0.0;
    }
  };
  auto store_rows = [&](int base) {
#pragma unroll
    for (int q = 0; q < SL; ++q) {
      const int e = tid + PNT * q, cc = e / EXT_ROWS, r = e % EXT_ROWS;
      if (base + r < mv && cc < jb) S[(int64_t)(j0 + cc) * m + j0 + base + r] = ext[cc][r];
    }
  };
  double x[SL];
  load_rows(0);
  if (w == 0 && g == 0)
    for (int b = 0; b < QB; ++b) sm.Tl[c][b] = 0.0;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SL; ++s) x[s] = ext[c][i0 + 64 * s];
  __syncthreads();
  load_rows(EXT_ROWS);
  __syncthreads();
  double myscale = 0.0, mybeta = 0.0;
  panel_columns_ext(x, ext, sm, jb, w, g, c, i0, myscale, mybeta);
  // LDS rows: v = x scale (every row there is below the diagonal).
#pragma unroll
  for (int s = 0; s < SL; ++s) ext[c][i0 + 64 * s] *= myscale;
  __syncthreads();
  if (w == 0 && g == 0) {
    if (jb >= 2) t_column(sm, jb - 2, c);
    t_column(sm, jb - 1, c);
    for (int b = 0; b < QB; ++b) T[c * QB + b] = (c < jb && b < jb) ? sm.Tl[c][b] : 0.0;
  }
  store_rows(EXT_ROWS);
  __syncthreads();
  // Register rows: R above row c, beta at row c, v = x scale below.
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const int i = i0 + 64 * s;
    ext[c][i] = (i > c) ? x[s] * myscale : (i == c ? mybeta : x[s]);
  }
  __syncthreads();
  store_rows(0);
}

// Panels taller than 2048 rows on G = ceil(mv / 1024) workgroups launched
// together (cooperative launch: all resident at once), each holding 1024
// rows in registers as qr_panel_reg_kernel<16> does.  Per column every
// workgroup reduces d_c over its rows, publishes its 16 sums (and workgroup
// 0 row CC) in gbuf, and after a grid-wide barrier every workgroup adds the
// G sums in the same order, so all of them take bitwise the same reflector
// and update their own rows.  One grid barrier per column; workgroup 0
// writes T.  gbuf: coop_panel_doubles(m) doubles.
constexpr int COOP_ROWS = 64 * MAX_REG_SLOTS;
__host__ __device__ constexpr int coop_groups(int mv) { return (mv + COOP_ROWS - 1) / COOP_ROWS; }

template <int CC>
__device__ __forceinline__ void coop_column(double (&x)[MAX_REG_SLOTS], PanelSmem &sm, double *__restrict__ gbuf,
                                            int G, int wg, int w, int g, int c, int ig0, double &myscale,
                                            double &mybeta) {
  constexpr int SL = MAX_REG_SLOTS, B = CC & 1;
  double *xr = gbuf + (int64_t)QB * QB * G;  // row CC of every column, per column CC
  double b[SL];
#pragma unroll
  for (int s = 0; s < SL; ++s) b[s] = row_bcast<CC>(x[s]);
  double dp[4] = {(ig0 > CC) ? b[0] * x[0] : 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 1; s < SL; ++s) dp[s & 3] = fma(b[s], x[s], dp[s & 3]);
  if (CC >= 2 && w == 0 && g == 0) t_column(sm, CC - 2, c);
  double d = rowgroup_sum((dp[0] + dp[1]) + (dp[2] + dp[3]));
  if (g == 0) sm.red[B][w][c] = d;
  __syncthreads();
  const double dloc = rowgroup_sum((sm.red[B][g][c] + sm.red[B][4 + g][c]) + (sm.red[B][8 + g][c] + sm.red[B][12 + g][c]));
  if (w == 0 && g == 0) gbuf[((int64_t)CC * G + wg) * QB + c] = dloc;
  if (ig0 == CC) xr[CC * QB + c] = x[0];  // only in workgroup 0
  cooperative_groups::this_grid().sync();
  double dc = 0.0;
  for (int q = 0; q < G; ++q) dc += gbuf[((int64_t)CC * G + q) * QB + c];
  const double xnorm2 = row_bcast<CC>(dc);
  const double alpha = xr[CC * QB + CC], xc = xr[CC * QB + c];
  double tau = 0.0, scale = 0.0, beta = alpha;
  if (xnorm2 > 0.0) {
    beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
    tau = (beta - alpha) * recip(beta);
    scale = recip(alpha - beta);
  }
  const double tot = fma(scale, dc, xc);
  const double f = (c > CC) ? tau * tot : 0.0, fs = f * scale;
  x[0] = (ig0 > CC) ? fma(-fs, b[0], x[0]) : (ig0 == CC ? x[0] - f : x[0]);
#pragma unroll
  for (int s = 1; s < SL; ++s) x[s] = fma(-fs, b[s], x[s]);
  if (c == CC) {
    myscale = scale;
    mybeta = beta;
  }
  if (w == 0 && g == 0) {
    if (c < CC) sm.zs[CC][c] = myscale * tot;
    if (c == CC) sm.taus[CC] = tau;
  }
}

template <int CC = 0>
__device__ __forceinline__ void coop_columns(double (&x)[MAX_REG_SLOTS], PanelSmem &sm, double *gbuf, int G,
                                             int wg, int jb, int w, int g, int c, int ig0, double &myscale,
                                             double &mybeta) {
  if constexpr (CC < QB) {
    if (CC < jb) {  // uniform over the grid
      coop_column<CC>(x, sm, gbuf, G, wg, w, g, c, ig0, myscale, mybeta);
      coop_columns<CC + 1>(x, sm, gbuf, G, wg, jb, w, g, c, ig0, myscale, mybeta);
    }
  }
}

__global__ __launch_bounds__(PNT) void qr_panel_coop_kernel(double *__restrict__ S, int m, int j0, int jb,
                                                            double *__restrict__ T, double *__restrict__ gbuf) {
  __shared__ PanelSmem sm;
  __shared__ double tile[QB][COOP_ROWS + 1];
  constexpr int SL = MAX_REG_SLOTS;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int wg = blockIdx.x, G = gridDim.x;
  const int mv = m - j0, r0 = wg * COOP_ROWS;  // this workgroup's first panel row
  const int i0 = 4 * w + g, ig0 = r0 + i0;
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int e = tid + PNT * q, cc = e / COOP_ROWS, i = e % COOP_ROWS;
    tile[cc][i] = (r0 + i < mv && cc < jb) ? S[(int64_t)(j0 + cc) * m + j0 + r0 + i] : 0.0;
  }
  if (w == 0 && g == 0)
    for (int b = 0; b < QB; ++b) sm.Tl[c][b] = 0.0;
  __syncthreads();
  double x[SL];
#pragma unroll
  for (int s = 0; s < SL; ++s) x[s] = tile[c][i0 + 64 * s];
  double myscale = 0.0, mybeta = 0.0;
  coop_columns(x, sm, gbuf, G, wg, jb, w, g, c, ig0, myscale, mybeta);
#pragma unroll
  for (int s = 0; s < SL; ++s) {
    const int i = i0 + 64 * s, ig = r0 + i;
    tile[c][i] = (ig > c) ? x[s] * myscale : (ig == c ? mybeta : x[s]);
  }
  __syncthreads();
  if (wg == 0 && w == 0 && g == 0) {
    if (jb >= 2) t_column(sm, jb - 2, c);
    t_column(sm, jb - 1, c);
    for (int b = 0; b < QB; ++b) T[c * QB + b] = (c < jb && b < jb) ? sm.Tl[c][b] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < SL; ++q) {
    const int e = tid + PNT * q, cc = e / COOP_ROWS, i = e % COOP_ROWS;
    if (r0 + i < mv && cc < jb) S[(int64_t)(j0 + cc) * m + j0 + r0 + i] = tile[cc][i];
  }
}

// Sum over the 64 lanes of a wave of each of 16 values: after the call lane
// l holds (bitwise the same in the four lanes of its quad) the wave total of
// value col(l) = 8 [l & 32] + 4 [l & 16] + 2 [l & 8] + [l & 4]: at each
// halving step a lane keeps the half of its values its partner sends away.
__device__ __forceinline__ double wave_sum16(const double (&d)[QB], int lane) {
  double e[8], f[4], g[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const bool hi = lane & 32;
    e[k] = (hi ? d[k + 8] : d[k]) + __shfl_xor(hi ? d[k] : d[k + 8], 32, 64);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const bool hi = lane & 16;
    f[k] = (hi ? e[k + 4] : e[k]) + __shfl_xor(hi ? e[k] : e[k + 4], 16, 64);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const bool hi = lane & 8;
    g[k] = (hi ? f[k + 2] : f[k]) + __shfl_xor(hi ? f[k] : f[k + 2], 8, 64);
  }
  const bool hi = lane & 4;
  double h = (hi ? g[1] : g[0]) + __shfl_xor(hi ? g[0] : g[1], 4, 64);
  h += __shfl_xor(h, 2, 64);
  h += __shfl_xor(h, 1, 64);
  return h;
}

// The same factorisation for panels taller than the register panels, with
// the panel in memory (L2).  Per column, all threads stream their rows
// (thread t: rows t + PNT q) of all 16 columns at once, two rows at a time:
// one pass forms d_c = x_CC^T x_c below the pivot for every column (d_CC is
// the squared norm) and publishes row CC; with v = (1 at CC, x_CC scale
// below), v^T x_c = x_c(CC) + scale d_c, so a second pass updates the
// columns right of CC and writes v (scaled) and beta into column CC.  For
// columns left of CC, v^T x_c is the sum v_CC^T v_c that T needs; row r of T
// is built by lane r of wave 0 at the end.
__global__ __launch_bounds__(PNT) void qr_panel_mem_kernel(double *__restrict__ S, int m, int n, int j0, int jb,
                                                           double *__restrict__ T,
                                                           const double *__restrict__ cnorm, int *__restrict__ perm,
                                                           double *__restrict__ pscratch) {
  if (cnorm) panel_pivot(S, m, n, j0, jb, cnorm, perm, pscratch);
  __shared__ double red[PNT / 64][QB];
  __shared__ double dsum[QB], xrow[QB];
  __shared__ double zs[QB][QB + 1];  // zs[i][b] = v_b^T v_i, b < i
  __shared__ double taus[QB];
  __shared__ double Tl[QB][QB + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mv = m - j0;
  double *P = S + (int64_t)j0 * m + j0;  // P(i, c) = P[c * m + i], i < mv, c < 16
  const int col_l = ((lane & 32) ? 8 : 0) + ((lane & 16) ? 4 : 0) + ((lane & 8) ? 2 : 0) + ((lane & 4) ? 1 : 0);
  for (int cc = 0; cc < jb; ++cc) {
    const double *pc = P + (int64_t)cc * m;
    // Pass 1: d_c for every column over rows below cc; row cc published.
    double d[QB];
#pragma unroll
    for (int c = 0; c < QB; ++c) d[c] = 0.0;
    for (int i0 = tid; i0 < mv; i0 += 2 * PNT) {
      double v[2][QB], b[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int i = i0 + r * PNT;
        const bool ok = i < mv;
        b[r] = (ok && i > cc) ? pc[i] : 0.0;
#pragma unroll
        for (int c = 0; c < QB; ++c) v[r][c] = (ok && c < jb) ? P[(int64_t)c * m + i] : 0.0;
      }
      if (i0 == cc)
#pragma unroll
        for (int c = 0; c < QB; ++c) xrow[c] = v[0][c];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < QB; ++c) d[c] = fma(b[r], v[r][c], d[c]);
    }
    const double wsum = wave_sum16(d, lane);
    if ((lane & 3) == 0) red[wave][col_l] = wsum;
    __syncthreads();
    if (tid < QB) {
      double t = 0.0;
      for (int w = 0; w < PNT / 64; ++w) t += red[w][tid];
      dsum[tid] = t;
    }
    __syncthreads();
    const double xnorm2 = dsum[cc], alpha = xrow[cc];
    double tau = 0.0, scale = 0.0, beta = alpha;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    double f[QB];  // tau v^T x_c for the columns right of cc
#pragma unroll
    for (int c = 0; c < QB; ++c) f[c] = (c > cc && c < jb) ? tau * fma(scale, dsum[c], xrow[c]) : 0.0;
    if (tid < QB && tid < cc) zs[cc][tid] = fma(scale, dsum[tid], xrow[tid]);
    if (tid == 0) taus[cc] = tau;
    // Pass 2: columns right of cc updated, column cc becomes (beta, v).
    for (int i0 = tid; i0 < mv; i0 += 2 * PNT) {
      double v[2][QB], b[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int i = i0 + r * PNT;
        const bool ok = i < mv && i >= cc;
        b[r] = ok ? pc[i] : 0.0;
#pragma unroll
        for (int c = 0; c < QB; ++c) v[r][c] = (ok && c > cc && c < jb) ? P[(int64_t)c * m + i] : 0.0;
      }
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int i = i0 + r * PNT;
        if (i < mv && i >= cc) {
          const double vi = (i == cc) ? 1.0 : b[r] * scale;
#pragma unroll
          for (int c = 0; c < QB; ++c)
            if (c > cc && c < jb) P[(int64_t)c * m + i] = fma(-f[c], vi, v[r][c]);
          P[(int64_t)cc * m + i] = (i == cc) ? beta : vi;
        }
      }
    }
    __syncthreads();
  }
  // T(i, i) = tau_i, T(r, i) = -tau_i sum over r <= b < i of T(r, b) zs(i, b):
  // lane r of wave 0 builds row r.
  if (wave == 0 && lane < QB) {
    const int r = lane;
    for (int b = 0; b < QB; ++b) Tl[r][b] = 0.0;
    for (int i = 0; i < jb; ++i) {
      double acc = 0.0;
      for (int b = r; b < i; ++b) acc = fma(Tl[r][b], zs[i][b], acc);
      Tl[r][i] = (r < i) ? -taus[i] * acc : (r == i ? taus[i] : 0.0);
    }
    for (int b = 0; b < QB; ++b) T[r * QB + b] = (r < jb && b < jb) ? Tl[r][b] : 0.0;
  }
}

// Entry (i, c) of the panel's V (unit lower trapezoidal, zero beyond jb
// columns) read from the factored panel Vs (= S + j0 m + j0, ld m).
__device__ __forceinline__ double vload(const double *Vs, int m, int jb, int c, int i) {
  return (c < jb && i >= c) ? (i == c ? 1.0 : Vs[(int64_t)c * m + i]) : 0.0;
}

// A <- (I - V op(T) V^T) A for the rows j0 .. m-1 of columns c0 .. c0+nc-1
// of the column-major S (ld m), with op(T) = T^T when `trans` (applying
// Q^T: the trailing update of the factorisation) and T otherwise (forming
// Q).  V: the panel's reflectors read in place from the factored panel Vs
// (vload), T: 16 x 16 row-major, zero-padded.
// One workgroup per 16 columns:
//   W1 = V^T A (MFMA, the four waves split the rows), W2 = op(T) W1,
//   A^T -= W2^T V^T (MFMA; the lanes of a row group write 16 consecutive
//   rows of one column).
// When cnorm is not null, cnorm[column] receives the norm of the updated
// column over rows j0 + next .. m-1 (the next panel's candidates).
__global__ __launch_bounds__(UNT) void qr_update_kernel(double *S, int m, int j0, int c0, int nc,
                                                        const double *Vs, int jb,
                                                        const double *__restrict__ T, int trans,
                                                        double *__restrict__ cnorm, int next) {
  __shared__ double Wp[4][QB][QB + 1];
  __shared__ double nred[4][QB];
  __shared__ double W2[QB][QB + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int mv = m - j0;
  const int cb = c0 + QB * blockIdx.x;
  const int ncol = min(QB, c0 + nc - cb);
  double *A = S + (int64_t)cb * m + j0;  // A(i, j) = A[j * m + i]
  // Each wave reduces a contiguous quarter of the rows, four MFMA steps per
  // batch of loads.
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
  const int chunk = ((mv + 15) / 16) * 4;
  const int kb = w * chunk, ke = min(mv, kb + chunk);
  for (int k0 = kb; k0 < ke; k0 += 16) {
    double va[4], ab[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int kk = k0 + 4 * u + q4;
      const bool ok = kk < ke;
      va[u] = ok ? vload(Vs, m, jb, r16, kk) : 0.0;
      ab[u] = (ok && r16 < ncol) ? A[(int64_t)r16 * m + kk] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], ab[u], acc, 0, 0, 0);
  }
  for (int t = 0; t < 4; ++t) Wp[w][4 * t + q4][r16] = acc[t];
  __syncthreads();
  const int ti = tid >> 4, tj = tid & 15;
  Wp[0][ti][tj] = (Wp[0][ti][tj] + Wp[1][ti][tj]) + (Wp[2][ti][tj] + Wp[3][ti][tj]);
  __syncthreads();
  {
    double s = 0.0;
    for (int b = 0; b < QB; ++b) s = fma(trans ? T[b * QB + ti] : T[ti * QB + b], Wp[0][b][tj], s);
    W2[ti][tj] = s;
  }
  __syncthreads();
  const double wa0 = W2[q4][r16], wa1 = W2[4 + q4][r16], wa2 = W2[8 + q4][r16], wa3 = W2[12 + q4][r16];
  // Two 16-row tiles per iteration, every load issued before the products.
  double nsq[4] = {0.0, 0.0, 0.0, 0.0};  // squared norms below row `next` of this lane's columns
  for (int i0 = 16 * w; i0 < mv; i0 += 128) {
    double vv[2][4], aa[2][4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = i0 + 64 * h + r16;
      const bool ok = r < mv;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int col = 4 * u + q4;
        vv[h][u] = ok ? vload(Vs, m, jb, col, r) : 0.0;
        aa[h][u] = (ok && col < ncol) ? A[(int64_t)col * m + r] : 0.0;
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = i0 + 64 * h + r16;
      dbl4 d = {0.0, 0.0, 0.0, 0.0};
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(wa0, vv[h][0], d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(wa1, vv[h][1], d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(wa2, vv[h][2], d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(wa3, vv[h][3], d, 0, 0, 0);
      if (r < mv) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int col = 4 * t + q4;
          const double nv = aa[h][t] - d[t];
          if (col < ncol) A[(int64_t)col * m + r] = nv;
          if (r >= next) nsq[t] = fma(nv, nv, nsq[t]);
        }
      }
    }
  }
  if (cnorm) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
      for (int o = 1; o < 16; o <<= 1) nsq[t] += __shfl_xor(nsq[t], o, 64);
    if (r16 == 0)
      for (int t = 0; t < 4; ++t) nred[w][4 * t + q4] = nsq[t];
    __syncthreads();
    if (tid < ncol) cnorm[cb + tid] = sqrt((nred[0][tid] + nred[1][tid]) + (nred[2][tid] + nred[3][tid]));
  }
}

// The same update with the rows split over workgroups, for when no column
// norms are wanted: a tall block reflector applied by one workgroup per 16
// columns is a long serial walk over the rows.  Rows j0 .. m-1 are cut into
// chunks of URC; grid (column blocks, chunks) for both kernels.
//   qr_update_part_kernel:  part[cb][ch] = V_ch^T A_ch (16 x 16, row-major);
//   qr_update_apply_kernel: W1 = sum over ch of part[cb][ch] (fixed order,
//     so every chunk of a column block gets bitwise the same W1),
//     W2 = op(T) W1, A_ch -= V_ch W2.
constexpr int URC = 128;

static inline int update_chunks(int mv) { return (mv + URC - 1) / URC; }

__global__ __launch_bounds__(UNT) void qr_update_part_kernel(const double *S, int m, int j0, int c0, int nc,
                                                             const double *Vs, int jb, double *__restrict__ part) {
  __shared__ double Wp[4][QB][QB + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int mv = m - j0;
  const int cb = c0 + QB * blockIdx.x, ch = blockIdx.y;
  const int ncol = min(QB, c0 + nc - cb);
  const double *A = S + (int64_t)cb * m + j0;
  // Each wave reduces URC / 4 rows of the chunk, all loads issued first.
  constexpr int KS = URC / 16;  // MFMA k-steps of 4 rows per wave
  const int kb = ch * URC + w * (URC / 4);
  double va[KS], ab[KS];
#pragma unroll
  for (int u = 0; u < KS; ++u) {
    const int kk = kb + 4 * u + q4;
    const bool ok = kk < mv;
    va[u] = ok ? vload(Vs, m, jb, r16, kk) : 0.0;
    ab[u] = (ok && r16 < ncol) ? A[(int64_t)r16 * m + kk] : 0.0;
  }
  dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < KS; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u], ab[u], acc, 0, 0, 0);
  for (int t = 0; t < 4; ++t) Wp[w][4 * t + q4][r16] = acc[t];
  __syncthreads();
  const int ti = tid >> 4, tj = tid & 15;
  part[((int64_t)blockIdx.x * gridDim.y + ch) * QB * QB + ti * QB + tj] =
      (Wp[0][ti][tj] + Wp[1][ti][tj]) + (Wp[2][ti][tj] + Wp[3][ti][tj]);
}

__global__ __launch_bounds__(UNT) void qr_update_apply_kernel(double *S, int m, int j0, int c0, int nc,
                                                              const double *Vs, int jb,
                                                              const double *__restrict__ T, int trans,
                                                              const double *__restrict__ part) {
  __shared__ double W1[QB][QB + 1];
  __shared__ double W2[QB][QB + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int mv = m - j0;
  const int cb = c0 + QB * blockIdx.x, ch = blockIdx.y, nch = gridDim.y;
  const int ncol = min(QB, c0 + nc - cb);
  double *A = S + (int64_t)cb * m + j0;
  // This chunk's rows of V and A (two 16-row tiles per wave), loaded first.
  double vv[2][4], aa[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = ch * URC + 16 * w + 64 * h + r16;
    const bool ok = r < mv;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int col = 4 * u + q4;
      vv[h][u] = ok ? vload(Vs, m, jb, col, r) : 0.0;
      aa[h][u] = (ok && col < ncol) ? A[(int64_t)col * m + r] : 0.0;
    }
  }
  const int ti = tid >> 4, tj = tid & 15;
  {
    const double *pp = part + (int64_t)blockIdx.x * nch * QB * QB + ti * QB + tj;
    double sum = 0.0;
    int c = 0;
    for (; c + 4 <= nch; c += 4) {
      const double p0 = pp[(c + 0) * QB * QB], p1 = pp[(c + 1) * QB * QB];
      const double p2 = pp[(c + 2) * QB * QB], p3 = pp[(c + 3) * QB * QB];
      sum += p0;
      sum += p1;
      sum += p2;
      sum += p3;
    }
    for (; c < nch; ++c) sum += pp[c * QB * QB];
    W1[ti][tj] = sum;
  }
  __syncthreads();
  {
    double t2 = 0.0;
    for (int b = 0; b < QB; ++b) t2 = fma(trans ? T[b * QB + ti] : T[ti * QB + b], W1[b][tj], t2);
    W2[ti][tj] = t2;
  }
  __syncthreads();
  const double wa0 = W2[q4][r16], wa1 = W2[4 + q4][r16], wa2 = W2[8 + q4][r16], wa3 = W2[12 + q4][r16];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = ch * URC + 16 * w + 64 * h + r16;
    dbl4 d = {0.0, 0.0, 0.0, 0.0};
    d = __builtin_amdgcn_mfma_f64_16x16x4f64(wa0, vv[h][0], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f64_16x16x4f64(wa1, vv[h][1], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f64_16x16x4f64(wa2, vv[h][2], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f64_16x16x4f64(wa3, vv[h][3], d, 0, 0, 0);
    if (r < mv) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = 4 * t + q4;
        if (col < ncol) A[(int64_t)col * m + r] = aa[h][t] - d[t];
      }
    }
  }
}

// For tall trailing updates (many row chunks) the chunk partials are summed
// once per column block instead of once per (column block, chunk):
//   qr_update_reduce_kernel<K>: grid (column blocks); W1 = sum over chunks of
//     part[cb][ch] (K x 16, fixed order), W2 = op(T) W1 -> w2[cb];
//   qr_update_apply_w2_kernel<K>: grid (column blocks, chunks); A_ch -= V_ch W2.
// K = 16 (one panel, op(T) = T^T when trans) or AGG (aggregated panels, T^T).
constexpr int UPD_REDUCE_MIN_CHUNKS = 17;

template <int K>
__global__ __launch_bounds__(UNT) void qr_update_reduce_kernel(const double *__restrict__ part, int nch,
                                                               const double *__restrict__ T, int trans,
                                                               double *__restrict__ w2) {
  __shared__ double W1[K][QB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < K * QB; e += UNT) {
    const double *pp = part + (int64_t)blockIdx.x * nch * K * QB + e;
    double sum = 0.0;
    for (int c = 0; c < nch; ++c) sum += pp[(int64_t)c * K * QB];
    W1[e / QB][e % QB] = sum;
  }
  __syncthreads();
  for (int e = tid; e < K * QB; e += UNT) {
    const int i = e / QB, j = e % QB;
    double t2 = 0.0;
    if (trans)
      for (int b = 0; b <= i; ++b) t2 = fma(T[b * K + i], W1[b][j], t2);  // T upper triangular
    else
      for (int b = i; b < K; ++b) t2 = fma(T[i * K + b], W1[b][j], t2);
    w2[(int64_t)blockIdx.x * K * QB + e] = t2;
  }
}

template <int K>
__global__ __launch_bounds__(UNT) void qr_update_apply_w2_kernel(double *S, int m, int j0, int c0, int nc,
                                                                 const double *Vs, int nbw,
                                                                 const double *__restrict__ w2) {
  __shared__ double W2[K][QB + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int mv = m - j0;
  const int cb = c0 + QB * blockIdx.x, ch = blockIdx.y;
  const int ncol = min(QB, c0 + nc - cb);
  double *A = S + (int64_t)cb * m + j0;
  for (int e = tid; e < K * QB; e += UNT) W2[e / QB][e % QB] = w2[(int64_t)blockIdx.x * K * QB + e];
  __syncthreads();
  // two 16-row tiles per wave: A^T -= W2^T V^T on the matrix cores
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = ch * URC + 16 * w + 64 * h + r16;
    const bool ok = r < mv;
    dbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < K / 4; ++u) {
      const int col = 4 * u + q4;
      const double vv = ok ? vload(Vs, m, nbw, col, r) : 0.0;
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(W2[col][r16], vv, d, 0, 0, 0);
    }
    if (ok) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = 4 * t + q4;
        if (col < ncol) A[(int64_t)col * m + r] -= d[t];
      }
    }
  }
}

// ------------------------------------------------------------------ aggregated reflectors
// Up to four consecutive panels (NB <= 64 columns) whose reflectors are
// applied to the trailing columns as one block reflector
// H_0 H_1 H_2 H_3 = I - V T V^T, V the NB columns in place (the panels' V
// read by vload over NB columns), T (NB x NB, upper triangular) built from
// the panels' T_p and the cross Grams V_p^T V_q:
//   T = [[T_{0:q}, -T_{0:q} (V_{0:q}^T V_q) T_q], [0, T_q]], q = 1 .. nsub-1.
// The trailing columns are then read twice and written once per 64 columns
// instead of per 16.
constexpr int AGG = 4 * QB;      // columns of an aggregated block reflector
// Aggregation pays only where the trailing matrix is large: per product
// 41.5 against 42.2 s at chi = 1024 (8192 rows), but 8.70 against 8.55 s at
// chi = 512 (4096 rows) with a 2048-row threshold.
constexpr int AGG_MIN_ROWS = 4096;

// grid (chunks).  gpart[ch][t] (t < 6: the cross blocks (p, q), p < q, in
// the order (0,1) (0,2) (0,3) (1,2) (1,3) (2,3); 16 x 16 row-major) =
// V_p^T V_q over the chunk's rows; wave w takes tiles w and w + 4.
__global__ __launch_bounds__(UNT) void qr_vgram_part_kernel(const double *Vs, int m, int mv, int nbw,
                                                            double *__restrict__ gpart) {
  constexpr int PQ[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int ch = blockIdx.x;
  for (int t = w; t < 6; t += UNT / 64) {
    const int bp = PQ[t][0], bq = PQ[t][1];
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    for (int u = 0; u < URC / 4; ++u) {
      const int kk = ch * URC + 4 * u + q4;
      const bool ok = kk < mv;
      const double a = ok ? vload(Vs, m, nbw, QB * bp + r16, kk) : 0.0;
      const double b = ok ? vload(Vs, m, nbw, QB * bq + r16, kk) : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    double *out = gpart + ((int64_t)ch * 6 + t) * QB * QB;
    for (int i = 0; i < 4; ++i) out[(4 * i + q4) * QB + r16] = acc[i];
  }
}

// One workgroup: the cross Grams summed over the chunks (fixed order), then
// T (AGG x AGG, row-major, zero outside nbw x nbw) from Tp (nsub panels'
// 16 x 16 T factors, consecutive).
__global__ __launch_bounds__(UNT) void qr_tagg_kernel(const double *__restrict__ gpart, int nch, int nsub,
                                                      int nbw, const double *__restrict__ Tp,
                                                      double *__restrict__ Tout) {
  __shared__ double G[6][QB][QB + 1];
  __shared__ double T[AGG][AGG + 1];
  __shared__ double Y[AGG][QB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < 6 * QB * QB; e += UNT) {
    const int t = e / (QB * QB), r = e % (QB * QB);
    double sum = 0.0;
    for (int c = 0; c < nch; ++c) sum += gpart[((int64_t)c * 6 + t) * QB * QB + r];
    G[t][r / QB][r % QB] = sum;
  }
  for (int e = tid; e < AGG * AGG; e += UNT) {
    const int i = e / AGG, j = e % AGG, pb = i / QB, qb = j / QB;
    T[i][j] = (pb == qb && pb < nsub) ? Tp[(int64_t)pb * QB * QB + (i % QB) * QB + (j % QB)] : 0.0;
  }
  __syncthreads();
  auto gidx = [](int bp, int bq) { return bp == 0 ? bq - 1 : (bp == 1 ? bq + 1 : 5); };
  for (int q = 1; q < nsub; ++q) {
    const int rows = QB * q;
    // Y = T[0:rows, 0:rows] X, X = the stacked G blocks (p, q), p < q
    for (int e = tid; e < rows * QB; e += UNT) {
      const int i = e / QB, j = e % QB;
      double acc = 0.0;
      for (int l = i; l < rows; ++l) acc = fma(T[i][l], G[gidx(l / QB, q)][l % QB][j], acc);
      Y[i][j] = acc;
    }
    __syncthreads();
    // T[0:rows, q block] = -Y T_q
    for (int e = tid; e < rows * QB; e += UNT) {
      const int i = e / QB, j = e % QB;
      double acc = 0.0;
      for (int l = 0; l <= j; ++l) acc = fma(Y[i][l], T[QB * q + l][QB * q + j], acc);
      T[i][QB * q + j] = -acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < AGG * AGG; e += UNT) {
    const int i = e / AGG, j = e % AGG;
    Tout[e] = (i < nbw && j < nbw) ? T[i][j] : 0.0;
  }
}

// As qr_update_part_kernel with V of AGG columns: part[cb][ch] = V_ch^T A_ch
// (AGG x 16, row-major).  Wave w reduces URC / 4 rows for all four 16-row
// tiles of V^T.
__global__ __launch_bounds__(UNT) void qr_update64_part_kernel(const double *S, int m, int j0, int c0, int nc,
                                                               const double *Vs, int nbw,
                                                               double *__restrict__ part) {
  __shared__ double Wp[4][AGG][QB + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int r16 = lane & 15, q4 = lane >> 4;
  const int mv = m - j0;
  const int cb = c0 + QB * blockIdx.x, ch = blockIdx.y;
  const int ncol = min(QB, c0 + nc - cb);
  const double *A = S + (int64_t)cb * m + j0;
  constexpr int KS = URC / 16;
  const int kb = ch * URC + w * (URC / 4);
  double ab[KS];
#pragma unroll
  for (int u = 0; u < KS; ++u) {
    const int kk = kb + 4 * u + q4;
    ab[u] = (kk < mv && r16 < ncol) ? A[(int64_t)r16 * m + kk] : 0.0;
  }
#pragma unroll
  for (int ti = 0; ti < AGG / QB; ++ti) {
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int u = 0; u < KS; ++u) {
      const int kk = kb + 4 * u + q4;
      const double va = (kk < mv) ? vload(Vs, m, nbw, QB * ti + r16, kk) : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va, ab[u], acc, 0, 0, 0);
    }
    for (int t = 0; t < 4; ++t) Wp[w][QB * ti + 4 * t + q4][r16] = acc[t];
  }
  __syncthreads();
  for (int e = tid; e < AGG * QB; e += UNT) {
    const int i = e / QB, j = e % QB;
    part[((int64_t)blockIdx.x * gridDim.y + ch) * AGG * QB + e] = (Wp[0][i][j] + Wp[1][i][j]) + (Wp[2][i][j] + Wp[3][i][j]);
  }
}

// R (k x n, row-major) = upper triangle of S[0:k, :]; Qs = first k columns of I.
__global__ void qr_r_and_identity_kernel(const double *__restrict__ S, int m, int n, int k,
                                         double *__restrict__ r, double *__restrict__ Qs) {
  const int64_t nr = (int64_t)k * n, nq = (int64_t)m * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nr + nq;
       e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nr) {
      const int i = (int)(e / n), c = (int)(e % n);
      r[e] = (c >= i) ? S[(int64_t)c * m + i] : 0.0;
    } else {
      const int64_t f = e - nr;
      const int i = (int)(f % m), c = (int)(f / m);
      Qs[f] = (i == c) ? 1.0 : 0.0;
    }
  }
}

namespace {
struct Pivot {
  const double *cnorm = nullptr;  // null: no pivoting
  int *perm = nullptr;
  double *scratch = nullptr;
};

hipError_t launch_panel(double *S, int m, int n, int j0, int jb, double *T, const Pivot &pv, double *coop,
                        hipStream_t s) {
  const int sl = (m - j0 + 63) / 64;
  const dim3 g(1), b(PNT);
#define TTM_PANEL_ARGS S, m, n, j0, jb, T, pv.cnorm, pv.perm, pv.scratch
  if (sl <= 1) hipLaunchKernelGGL(qr_panel_reg_kernel<1>, g, b, 0, s, TTM_PANEL_ARGS);
  else if (sl <= 2) hipLaunchKernelGGL(qr_panel_reg_kernel<2>, g, b, 0, s, TTM_PANEL_ARGS);
  else if (sl <= 4) hipLaunchKernelGGL(qr_panel_reg_kernel<4>, g, b, 0, s, TTM_PANEL_ARGS);
  else if (sl <= 8) hipLaunchKernelGGL(qr_panel_reg_kernel<8>, g, b, 0, s, TTM_PANEL_ARGS);
  else if (sl <= MAX_REG_SLOTS) hipLaunchKernelGGL(qr_panel_reg_kernel<16>, g, b, 0, s, TTM_PANEL_ARGS);
  else if (sl <= 2 * MAX_REG_SLOTS) hipLaunchKernelGGL(qr_panel_ext_kernel, g, b, 0, s, TTM_PANEL_ARGS);
  else {
    if (coop && !pv.cnorm) {
      void *args[] = {&S, &m, &j0, &jb, &T, &coop};
      const hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void *>(qr_panel_coop_kernel),
                                                      dim3(coop_groups(m - j0)), b, args, 0, s);
      if (e == hipSuccess) return hipSuccess;
      (void)hipGetLastError();  // not launched: the one-workgroup panel below
    }
    hipLaunchKernelGGL(qr_panel_mem_kernel, g, b, 0, s, TTM_PANEL_ARGS);
  }
#undef TTM_PANEL_ARGS
  return hipGetLastError();
}

// A <- (I - V op(T) V^T) A with V the reflectors of the panel at j0 (jb
// columns) of the factored Sf (ld m); A may be Sf itself (trailing update).
hipError_t launch_update(double *A, int m, int j0, int c0, int nc, const double *Sf, int jb, const double *T,
                         int trans, double *cnorm, int next, double *part, hipStream_t s) {
  if (nc <= 0) return hipSuccess;
  const double *Vs = Sf + (int64_t)j0 * m + j0;
  const int ncb = (nc + QB - 1) / QB;
  if (cnorm == nullptr && part != nullptr) {
    const int nch = update_chunks(m - j0);
    const dim3 grid(ncb, nch);
    hipLaunchKernelGGL(qr_update_part_kernel, grid, dim3(UNT), 0, s, A, m, j0, c0, nc, Vs, jb, part);
    if (nch >= UPD_REDUCE_MIN_CHUNKS) {
      // W2 per column block after the partials (they occupy ncb * nch tiles)
      double *w2 = part + (size_t)ncb * nch * QB * QB;
      hipLaunchKernelGGL(qr_update_reduce_kernel<QB>, dim3(ncb), dim3(UNT), 0, s, part, nch, T, trans, w2);
      hipLaunchKernelGGL(qr_update_apply_w2_kernel<QB>, grid, dim3(UNT), 0, s, A, m, j0, c0, nc, Vs, jb, w2);
    } else {
      hipLaunchKernelGGL(qr_update_apply_kernel, grid, dim3(UNT), 0, s, A, m, j0, c0, nc, Vs, jb, T, trans, part);
    }
  } else {
    hipLaunchKernelGGL(qr_update_kernel, dim3(ncb), dim3(UNT), 0, s, A, m, j0, c0, nc, Vs, jb, T, trans, cnorm,
                       next);
  }
  return hipGetLastError();
}
}  // namespace

// Partial products of the split update over nc columns of an m-row block.
static size_t update_part_doubles(int m, int nc) {
  // the partials, and W2 per column block when they are reduced separately
  return (size_t)((nc + QB - 1) / QB) * (update_chunks(m) + 1) * QB * QB;
}

// Exchange buffer of the cooperative panel: per column the G workgroup sums
// of 16 columns, and row CC.
static size_t coop_panel_doubles(int m) { return (size_t)QB * QB * (coop_groups(m) + 1); }

// Scratch of the aggregated updates: the 64 x 16 partials per column block
// and chunk, the cross-Gram partials, the panels' T and the aggregated T.
static size_t agg_doubles(int m, int n) {
  if (m <= AGG_MIN_ROWS) return 0;
  return (size_t)((n + QB - 1) / QB) * update_chunks(m) * AGG * QB + (size_t)update_chunks(m) * 6 * QB * QB +
         4 * QB * QB + AGG * AGG + (size_t)((n + QB - 1) / QB) * AGG * QB;
}

size_t qr_inplace_scratch_doubles(int m, int n) {
  return QB * QB + (size_t)n + 2 * (size_t)QB * m + update_part_doubles(m, n) + coop_panel_doubles(m) +
         agg_doubles(m, n) + 10 * 32;
}

hipError_t launch_qr_inplace(double *S, int m, int n, double *scratch, int *perm, double *Tall, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipErrorInvalidValue;
  if (perm && n > PNT * PIVOT_MAX_CAND) return hipErrorInvalidValue;
  const int k = m < n ? m : n;
  double *p = scratch;
  auto adv = [&](size_t nd) { double *x = p; p += (nd + 31) & ~(size_t)31; return x; };
  double *T1 = adv(QB * QB);
  double *part = adv(update_part_doubles(m, n));
  double *coop = adv(coop_panel_doubles(m));
  double *apart = nullptr, *gpart = nullptr, *Tp = nullptr, *Tagg = nullptr, *w2buf = nullptr;
  if (m > AGG_MIN_ROWS) {
    apart = adv((size_t)((n + QB - 1) / QB) * update_chunks(m) * AGG * QB);
    gpart = adv((size_t)update_chunks(m) * 6 * QB * QB);
    Tp = adv(4 * QB * QB);
    Tagg = adv(AGG * AGG);
    w2buf = adv((size_t)((n + QB - 1) / QB) * AGG * QB);
  }
  Pivot pv;
  if (perm) {
    double *cnorm = adv((size_t)n);
    pv.cnorm = cnorm;
    pv.perm = perm;
    pv.scratch = adv(2 * (size_t)QB * m);
    hipError_t e = launch_column_norms(S, m, n, cnorm, s);
    if (e != hipSuccess) return e;
  }
  for (int j0 = 0; j0 < k;) {
    const int nsub = std::min(4, (k - j0 + QB - 1) / QB);
    if (!perm && apart && m - j0 > AGG_MIN_ROWS && nsub >= 2 && n - j0 > AGG) {
      // Up to four panels; each updates only the rest of the group, then the
      // group's aggregated reflector updates the trailing columns.
      const int nbw = std::min(AGG, k - j0);
      for (int p = 0; p < nsub; ++p) {
        const int jp = j0 + QB * p, jb = std::min(QB, k - jp);
        double *T = Tp + (size_t)p * QB * QB;
        hipError_t e = launch_panel(S, m, n, jp, jb, T, pv, coop, s);
        if (e != hipSuccess) return e;
        if (Tall) {
          e = launch_copy(Tall + (size_t)(jp / QB) * QB * QB, T, QB * QB, s);
          if (e != hipSuccess) return e;
        }
        e = launch_update(S, m, jp, jp + jb, j0 + nbw - (jp + jb), S, jb, T, 1, nullptr, 0, part, s);
        if (e != hipSuccess) return e;
      }
      const int mv = m - j0, nch = update_chunks(mv);
      const double *Vs = S + (int64_t)j0 * m + j0;
      hipLaunchKernelGGL(qr_vgram_part_kernel, dim3(nch), dim3(UNT), 0, s, Vs, m, mv, nbw, gpart);
      hipLaunchKernelGGL(qr_tagg_kernel, dim3(1), dim3(UNT), 0, s, gpart, nch, nsub, nbw, Tp, Tagg);
      const int c0 = j0 + nbw, nc = n - c0;
      const dim3 grid((nc + QB - 1) / QB, nch);
      hipLaunchKernelGGL(qr_update64_part_kernel, grid, dim3(UNT), 0, s, S, m, j0, c0, nc, Vs, nbw, apart);
      hipLaunchKernelGGL(qr_update_reduce_kernel<AGG>, dim3(grid.x), dim3(UNT), 0, s, apart, nch, Tagg, 1, w2buf);
      hipLaunchKernelGGL(qr_update_apply_w2_kernel<AGG>, grid, dim3(UNT), 0, s, S, m, j0, c0, nc, Vs, nbw, w2buf);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      j0 += nbw;
      continue;
    }
    const int jb = (k - j0) < QB ? (k - j0) : QB;
    double *T = Tall ? Tall + (size_t)(j0 / QB) * QB * QB : T1;
    hipError_t e = launch_panel(S, m, n, j0, jb, T, pv, coop, s);
    if (e != hipSuccess) return e;
    e = launch_update(S, m, j0, j0 + jb, n - (j0 + jb), S, jb, T, 1, const_cast<double *>(pv.cnorm), jb, part, s);
    if (e != hipSuccess) return e;
    j0 += jb;
  }
  return hipSuccess;
}

size_t qr_apply_q_scratch_doubles(int m, int nc) { return update_part_doubles(m, nc) + 32; }

hipError_t launch_apply_q(const double *S, int m, int k, const double *Tall, double *X, int nc, double *scratch,
                          hipStream_t s) {
  if (m <= 0 || k <= 0 || nc <= 0) return hipSuccess;
  double *part = scratch;
  // Q X = H_0 ... H_{k-1} X: block reflectors from the last panel to the first.
  for (int pi = (k - 1) / QB; pi >= 0; --pi) {
    const int j0 = pi * QB, jb = (k - j0) < QB ? (k - j0) : QB;
    hipError_t e = launch_update(X, m, j0, 0, nc, S, jb, Tall + (size_t)pi * QB * QB, 0, nullptr, 0, part, s);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

size_t qr_scratch_doubles(int m, int n) {
  const int k = m < n ? m : n;
  const int np = (k + QB - 1) / QB;
  size_t t = 0;
  t += (size_t)m * n;          // S
  t += (size_t)np * QB * QB;   // T per panel
  t += (size_t)m * k;          // Qs
  t += update_part_doubles(m, n);  // split-update partials
  t += coop_panel_doubles(m);      // cooperative panel exchange
  return t + 5 * 32;
}

hipError_t launch_qr(const double *M, int m, int n, int64_t rs, int64_t cs, double *q, double *r,
                     double *scratch, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipErrorInvalidValue;
  const int k = m < n ? m : n;
  const int np = (k + QB - 1) / QB;
  double *p = scratch;
  auto adv = [&](size_t nd) { double *x = p; p += (nd + 31) & ~(size_t)31; return x; };
  double *S = adv((size_t)m * n);
  double *Tall = adv((size_t)np * QB * QB);
  double *Qs = adv((size_t)m * k);
  double *part = adv(update_part_doubles(m, n));
  double *coop = adv(coop_panel_doubles(m));
  const int64_t tot = (int64_t)m * n;
  hipLaunchKernelGGL(strided_to_colmajor_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, s, S, M, m, n, rs, cs);
  for (int pi = 0; pi < np; ++pi) {
    const int j0 = pi * QB, jb = (k - j0) < QB ? (k - j0) : QB;
    double *T = Tall + (size_t)pi * QB * QB;
    hipError_t e = launch_panel(S, m, n, j0, jb, T, Pivot(), coop, s);
    if (e != hipSuccess) return e;
    e = launch_update(S, m, j0, j0 + jb, n - (j0 + jb), S, jb, T, 1, nullptr, 0, part, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(qr_r_and_identity_kernel, dim3(grid_for((int64_t)k * n + (int64_t)m * k, 256)), dim3(256),
                     0, s, S, m, n, k, r, Qs);
  // Q = H_0 ... H_{np-1} applied to [I_k; 0], panels in reverse order.
  for (int pi = np - 1; pi >= 0; --pi) {
    const int j0 = pi * QB, jb = (k - j0) < QB ? (k - j0) : QB;
    hipError_t e = launch_update(Qs, m, j0, j0, k - j0, S, jb, Tall + (size_t)pi * QB * QB, 0, nullptr, 0, part, s);
    if (e != hipSuccess) return e;
  }
  // q (m x k, row-major) from Qs (column-major)
  return launch_transpose(q, Qs, k, m, s);
}

}  // namespace ttm
