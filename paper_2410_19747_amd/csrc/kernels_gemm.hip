// Batched strided GEMM on the gfx950 matrix cores with a split-stride
// epilogue.  FP64 (v_mfma_f64_16x16x4_f64) throughout, or, for the
// contractions of a mixed-precision product, operands rounded to FP32
// (v_mfma_f32_16x16x4_f32), to BF16 (v_mfma_f32_16x16x16_bf16) or split into
// three BF16 terms (six BF16 products, about FP32 accuracy), all accumulated
// in FP32 within each 16-deep k-tile and in FP64 across k-tiles; inputs and
// outputs stay FP64 in memory.
//
// Used for every contraction of the TTM sweep: the COPY-tensor contraction
// of Eq. (contract) is a batch of d products sharing the physical index; the
// merge of a swap pair is one product whose epilogue stores the leg-exchanged
// unfolding; the R (or S V^T) factor of a gauge move is multiplied into the
// next carriage; the variational baseline's environment contractions.
#include <algorithm>

#include "ttm_internal.h"

namespace ttm {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int BM = 64;
constexpr int BN = 64;
constexpr int BK = 16;
constexpr int NT = 256;  // 4 waves of 64 lanes, 2 x 2 over the 64 x 64 tile
constexpr int64_t kSplitTarget = 512;  // workgroups a split product aims for (two per CU)

constexpr int EA = BM * BK / NT;  // A-tile elements per thread
constexpr int EB = BK * BN / NT;  // B-tile elements per thread

// Tile coordinates of element e of a thread's share: the fast index follows
// the operand's unit stride so that neighbouring lanes read neighbouring
// addresses.
__device__ __forceinline__ void a_coords(int e, bool kfast, int &i, int &k) {
  if (kfast) { k = e % BK; i = e / BK; } else { i = e % BM; k = e / BM; }
}
__device__ __forceinline__ void b_coords(int e, bool jfast, int &j, int &k) {
  if (jfast) { j = e % BN; k = e / BN; } else { k = e % BK; j = e / BK; }
}

__device__ __forceinline__ int64_t out_index(const GemmArgs &g, int i, int j) {
  int64_t oi = (g.c_rdiv == 1) ? (int64_t)i * g.c_rs1
                               : (int64_t)(i / g.c_rdiv) * g.c_rs1 + (int64_t)(i % g.c_rdiv) * g.c_rs0;
  int64_t oj = (g.c_cdiv == 1) ? (int64_t)j * g.c_cs1
                               : (int64_t)(j / g.c_cdiv) * g.c_cs1 + (int64_t)(j % g.c_cdiv) * g.c_cs0;
  return oi + oj;
}
}  // namespace

// Each workgroup computes one 64 x 64 tile of one batch entry.  Wave w owns
// the 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 MFMA blocks of 16 x 16.
// MFMA operand layout (16x16x4, f64): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register t of lane l holds D[4*t + l/16][l % 16]
// (rows interleaved across the four 16-lane groups; measured on gfx950).
__global__ __launch_bounds__(NT) void gemm_f64_kernel(GemmArgs g) {
  __shared__ double As[BK][BM + 1];
  __shared__ double Bs[BK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int tile_m = blockIdx.y * BM;
  const int tile_n = blockIdx.x * BN;
  const int64_t bz = blockIdx.z / g.ksplit;
  const int kbeg = (g.ksplit > 1) ? (int)(blockIdx.z % g.ksplit) * g.kchunk : 0;
  const int kend = (g.ksplit > 1) ? min(g.K, kbeg + g.kchunk) : g.K;
  const double *A = g.A + bz * g.a_bs;
  const double *B = g.B + bz * g.b_bs;
  const bool a_kfast = (g.a_cs == 1);
  const bool b_jfast = (g.b_cs == 1);

  dbl4 acc[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) acc[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};

  // The next k-tile's operands are loaded into registers while the current
  // one is multiplied, then stored to LDS after the barrier.
  double ra[EA], rb[EB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      int i, k;
      a_coords(tid + q * NT, a_kfast, i, k);
      const int gi = tile_m + i, gk = k0 + k;
      ra[q] = (gi < g.M && gk < kend) ? A[(int64_t)gi * g.a_rs + (int64_t)gk * g.a_cs] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      int j, k;
      b_coords(tid + q * NT, b_jfast, j, k);
      const int gj = tile_n + j, gk = k0 + k;
      rb[q] = (gj < g.N && gk < kend) ? B[(int64_t)gk * g.b_rs + (int64_t)gj * g.b_cs] : 0.0;
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      int i, k;
      a_coords(tid + q * NT, a_kfast, i, k);
      As[k][i] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      int j, k;
      b_coords(tid + q * NT, b_jfast, j, k);
      Bs[k][j] = rb[q];
    }
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      double a0 = As[kr][wr * 32 + (lane & 15)];
      double a1 = As[kr][wr * 32 + 16 + (lane & 15)];
      double b0 = Bs[kr][wc * 32 + (lane & 15)];
      double b1 = Bs[kr][wc * 32 + 16 + (lane & 15)];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
    }
    __syncthreads();
  }

  double *C = g.C + bz * g.c_bs;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
#pragma unroll
    for (int y = 0; y < 2; ++y) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = tile_m + wr * 32 + x * 16 + 4 * t + (lane >> 4);
        const int j = tile_n + wc * 32 + y * 16 + (lane & 15);
        if (i < g.M && j < g.N) {
          if (g.ksplit > 1) {
            g.part[((int64_t)blockIdx.z * g.M + i) * g.N + j] = acc[x][y][t];
            continue;
          }
          const int64_t o = out_index(g, i, j);
          double v = g.alpha * acc[x][y][t];
          if (g.beta != 0.0) v += g.beta * C[o];
          C[o] = v;
        }
      }
    }
  }
}

// Sum of the K slices of a split product, slice 0 first, then the epilogue
// of the unsplit kernel (alpha, beta, split-stride output).
__global__ __launch_bounds__(256) void gemm_splitk_reduce_kernel(GemmArgs g) {
  const int64_t mn = (int64_t)g.M * g.N;
  const int64_t total = mn * g.batch;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = e / mn, r = e % mn;
    const double *p = g.part + b * g.ksplit * mn + r;
    double sum = 0.0;
    for (int s = 0; s < g.ksplit; ++s) sum += p[s * mn];
    const int i = (int)(r / g.N), j = (int)(r % g.N);
    double *C = g.C + b * g.c_bs;
    const int64_t o = out_index(g, i, j);
    double v = g.alpha * sum;
    if (g.beta != 0.0) v += g.beta * C[o];
    C[o] = v;
  }
}

// ------------------------------------------------------------------ reduced-precision operands
typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short shr4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf16_bits(float x) {
  __bf16 h = (__bf16)x;  // round to nearest even
  return __builtin_bit_cast(short, h);
}
__device__ __forceinline__ float bf16_value(short b) { return (float)__builtin_bit_cast(__bf16, b); }

// The same tiling with operands rounded to FP32 or BF16 in LDS.  The matrix
// cores accumulate each 16-deep k-tile in FP32, starting from zero; the
// tile's partial sums are then added to FP64 accumulators, so that FP32
// rounding acts on 16-term partials only, not on running sums over all of K
// (with K up to the bond dimension, FP32 running sums lose about sqrt(K)
// units of 2^-24, which over the N(N-1)/2 swaps of a product at bond 1024
// added up to 3e-6).  PREC: 1 = FP32 (16x16x4 f32 MFMA, 4 k per step), 2 = BF16
// (16x16x16 bf16 MFMA, 16 k per step), 3 = BF16 x 3: x = hi + mid + lo with
// each term BF16, and A B ~ hi hi + hi mid + mid hi + hi lo + mid mid + lo hi
// (the six terms above 2^-24 relative).  Operand layouts: f32 as for f64
// (lane l: A[l%16][l/16], B[l/16][l%16]); bf16 lane l: A[l%16][4(l/16)+j],
// B[4(l/16)+j][l%16], j < 4.  Accumulator register t of lane l holds
// D[4(l/16) + t][l%16] for both (checked on gfx950 by the GEMM tests).
template <int PREC>
__global__ __launch_bounds__(NT) void gemm_lowp_kernel(GemmArgs g) {
  constexpr int NS = (PREC == 3) ? 3 : 1;  // BF16 terms per operand
  __shared__ float As[NS][BK][BM + 1];
  __shared__ float Bs[NS][BK][BN + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1;
  const int tile_m = blockIdx.y * BM;
  const int tile_n = blockIdx.x * BN;
  const int64_t bz = blockIdx.z / g.ksplit;
  const int kbeg = (g.ksplit > 1) ? (int)(blockIdx.z % g.ksplit) * g.kchunk : 0;
  const int kend = (g.ksplit > 1) ? min(g.K, kbeg + g.kchunk) : g.K;
  const double *A = g.A + bz * g.a_bs;
  const double *B = g.B + bz * g.b_bs;
  const bool a_kfast = (g.a_cs == 1);
  const bool b_jfast = (g.b_cs == 1);
  // Rounded terms of one operand value: FP32, one BF16, or three BF16.
  auto put = [&](float (*dst)[BK][BM + 1], int k, int i, double x) {
    if (PREC == 1) {
      dst[0][k][i] = (float)x;
    } else {
      const float f = (float)x;
      const float hi = bf16_value(bf16_bits(f));
      dst[0][k][i] = hi;
      if (PREC == 3) {
        const float r = (float)(x - (double)hi);
        const float mid = bf16_value(bf16_bits(r));
        dst[1][k][i] = mid;
        dst[2][k][i] = bf16_value(bf16_bits((float)(x - (double)hi - (double)mid)));
      }
    }
  };

  flt4 acc[2][2];
  dbl4 acc64[2][2];
  for (int x = 0; x < 2; ++x)
    for (int y = 0; y < 2; ++y) acc64[x][y] = dbl4{0.0, 0.0, 0.0, 0.0};

  double ra[EA], rb[EB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      int i, k;
      a_coords(tid + q * NT, a_kfast, i, k);
      const int gi = tile_m + i, gk = k0 + k;
      ra[q] = (gi < g.M && gk < kend) ? A[(int64_t)gi * g.a_rs + (int64_t)gk * g.a_cs] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      int j, k;
      b_coords(tid + q * NT, b_jfast, j, k);
      const int gj = tile_n + j, gk = k0 + k;
      rb[q] = (gj < g.N && gk < kend) ? B[(int64_t)gk * g.b_rs + (int64_t)gj * g.b_cs] : 0.0;
    }
  };
  if (kbeg < kend) fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) acc[x][y] = flt4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int q = 0; q < EA; ++q) {
      int i, k;
      a_coords(tid + q * NT, a_kfast, i, k);
      put(As, k, i, ra[q]);
    }
#pragma unroll
    for (int q = 0; q < EB; ++q) {
      int j, k;
      b_coords(tid + q * NT, b_jfast, j, k);
      put(Bs, k, j, rb[q]);
    }
    __syncthreads();
    if (k0 + BK < kend) fetch(k0 + BK);
    if (PREC == 1) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int kr = kk + (lane >> 4);
        const float a0 = As[0][kr][wr * 32 + (lane & 15)], a1 = As[0][kr][wr * 32 + 16 + (lane & 15)];
        const float b0 = Bs[0][kr][wc * 32 + (lane & 15)], b1 = Bs[0][kr][wc * 32 + 16 + (lane & 15)];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
      }
    } else {
      // one 16-deep step: lane l takes k = 4 (l/16) + j, j < 4
      shr4 a[NS][2], b[NS][2];
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int kr = 4 * (lane >> 4) + j;
          a[s][0][j] = bf16_bits(As[s][kr][wr * 32 + (lane & 15)]);
          a[s][1][j] = bf16_bits(As[s][kr][wr * 32 + 16 + (lane & 15)]);
          b[s][0][j] = bf16_bits(Bs[s][kr][wc * 32 + (lane & 15)]);
          b[s][1][j] = bf16_bits(Bs[s][kr][wc * 32 + 16 + (lane & 15)]);
        }
      // term pairs (sa, sb) with sa + sb <= 2: hi hi, hi mid, mid hi, hi lo, mid mid, lo hi
#pragma unroll
      for (int sa = 0; sa < NS; ++sa)
#pragma unroll
        for (int sb = 0; sb < NS; ++sb) {
          if (sa + sb > 2) continue;
#pragma unroll
          for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
              acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[sa][x], b[sb][y], acc[x][y], 0, 0, 0);
        }
    }
    // this k-tile's FP32 partial sums into the FP64 accumulators
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc64[x][y][t] += (double)acc[x][y][t];
    __syncthreads();
  }

  double *C = g.C + bz * g.c_bs;
#pragma unroll
  for (int x = 0; x < 2; ++x) {
#pragma unroll
    for (int y = 0; y < 2; ++y) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int i = tile_m + wr * 32 + x * 16 + 4 * (lane >> 4) + t;
        const int j = tile_n + wc * 32 + y * 16 + (lane & 15);
        if (i < g.M && j < g.N) {
          if (g.ksplit > 1) {
            g.part[((int64_t)blockIdx.z * g.M + i) * g.N + j] = acc64[x][y][t];
            continue;
          }
          const int64_t o = out_index(g, i, j);
          double v = g.alpha * acc64[x][y][t];
          if (g.beta != 0.0) v += g.beta * C[o];
          C[o] = v;
        }
      }
    }
  }
}

GemmArgs gemm_rowmajor(int M, int N, int K, const double *A, int64_t lda, const double *B,
                       int64_t ldb, double *C, int64_t ldc) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K; g.batch = 1;
  g.A = A; g.a_rs = lda; g.a_cs = 1;
  g.B = B; g.b_rs = ldb; g.b_cs = 1;
  g.C = C; g.c_rs1 = ldc; g.c_cs1 = 1;
  return g;
}

hipError_t launch_gemm(const GemmArgs &g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0) {
    // Empty inner dimension: C = beta * C.  Never happens on the TTM path
    // (every bond is >= 1); rejected rather than special-cased.
    return hipErrorInvalidValue;
  }
  GemmArgs h = g;
  h.ksplit = 1;
  h.kchunk = 0;
  const int64_t tiles = (int64_t)((g.N + BN - 1) / BN) * ((g.M + BM - 1) / BM) * g.batch;
  const int64_t outs = (int64_t)g.M * g.N * g.batch;
  // Split K only when the output tiles leave the device under-filled, and
  // with at least 4 k-steps per slice.
  if (g.part && tiles < kSplitTarget && g.K >= 8 * BK) {
    int64_t ks = std::min<int64_t>((kSplitTarget + tiles - 1) / tiles, g.K / (4 * BK));
    ks = std::min<int64_t>(ks, g.part_doubles / outs);
    ks = std::min<int64_t>(ks, 65535 / g.batch);
    if (ks > 1) {
      const int kchunk = (int)(((g.K + ks - 1) / ks + BK - 1) / BK * BK);
      h.kchunk = kchunk;
      h.ksplit = (g.K + kchunk - 1) / kchunk;
    }
  }
  dim3 grid((g.N + BN - 1) / BN, (g.M + BM - 1) / BM, g.batch * h.ksplit);
  if (grid.y > 65535u || grid.z > 65535u) return hipErrorInvalidValue;
  if (h.ksplit > 1) {
    switch (g.prec) {
      case GEMM_F64: hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(NT), 0, s, h); break;
      case GEMM_F32: hipLaunchKernelGGL(gemm_lowp_kernel<1>, grid, dim3(NT), 0, s, h); break;
      case GEMM_BF16: hipLaunchKernelGGL(gemm_lowp_kernel<2>, grid, dim3(NT), 0, s, h); break;
      case GEMM_BF16X3: hipLaunchKernelGGL(gemm_lowp_kernel<3>, grid, dim3(NT), 0, s, h); break;
      default: return hipErrorInvalidValue;
    }
    const int64_t blocks = std::min<int64_t>((outs + 255) / 256, 4096);
    hipLaunchKernelGGL(gemm_splitk_reduce_kernel, dim3((unsigned)blocks), dim3(256), 0, s, h);
    return hipGetLastError();
  }
  switch (g.prec) {
    case GEMM_F64: hipLaunchKernelGGL(gemm_f64_kernel, grid, dim3(NT), 0, s, g); break;
    case GEMM_F32: hipLaunchKernelGGL(gemm_lowp_kernel<1>, grid, dim3(NT), 0, s, g); break;
    case GEMM_BF16: hipLaunchKernelGGL(gemm_lowp_kernel<2>, grid, dim3(NT), 0, s, g); break;
    case GEMM_BF16X3: hipLaunchKernelGGL(gemm_lowp_kernel<3>, grid, dim3(NT), 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ttm
