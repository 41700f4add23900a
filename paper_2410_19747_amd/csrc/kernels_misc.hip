// Small data-movement kernels and the Householder QR used for gauge moves.
#include "ttm_internal.h"

namespace ttm {

// ---------------------------------------------------------------- kernel timer
namespace {
struct EventPool {
  hipEvent_t ev[2 * 4096];
  int n = 0;  // events created
};
EventPool &pool() {
  static thread_local EventPool p;
  return p;
}
}  // namespace

void KernelTimer::begin(int cls, hipStream_t s) {
  EventPool &p = pool();
  if (npending >= 4096) return;  // callers collect well before this
  pending_cls[npending] = 1 << 30;  // not open until the start event is recorded
  const int i = 2 * npending;
  while (p.n < i + 2) {
    if (hipEventCreate(&p.ev[p.n]) != hipSuccess) return;
    ++p.n;
  }
  if (hipEventRecord(p.ev[i], s) != hipSuccess) return;
  pending_cls[npending] = -1 - cls;  // open
}

void KernelTimer::end(int cls, hipStream_t s) {
  EventPool &p = pool();
  if (npending >= 4096 || pending_cls[npending] != -1 - cls) return;
  if (hipEventRecord(p.ev[2 * npending + 1], s) != hipSuccess) return;
  pending_cls[npending] = cls;
  ++npending;
}

void KernelTimer::collect() {
  EventPool &p = pool();
  for (int k = 0; k < npending; ++k) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, p.ev[2 * k], p.ev[2 * k + 1]) == hipSuccess) {
      ms[pending_cls[k]] += t;
      launches[pending_cls[k]] += 1;
    }
  }
  npending = 0;
}

__global__ void copy_kernel(double *__restrict__ dst, const double *__restrict__ src, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

__global__ void fill_kernel(double *__restrict__ dst, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = v;
}

__global__ void zero_int_kernel(int *p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// out[b][w][a] = in[a][w][b]: reversing the order of a train transposes
// every carriage (the second factor enters Eq. (tensor) reversed).
__global__ void reverse_core_kernel(double *__restrict__ out, const double *__restrict__ in, int rl,
                                    int d, int rr) {
  const int64_t n = (int64_t)rl * d * rr;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int a = (int)(e % rl);
    const int64_t t = e / rl;
    const int w = (int)(t % d);
    const int b = (int)(t / d);
    out[e] = in[((int64_t)a * d + w) * rr + b];
  }
}

__global__ void transpose_kernel(double *__restrict__ out, const double *__restrict__ in, int m, int n) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int i = by + k, j = bx + tx;
    if (i < m && j < n) tile[k][tx] = in[(int64_t)i * n + j];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int j = bx + k, i = by + tx;
    if (i < m && j < n) out[(int64_t)j * m + i] = tile[tx][k];
  }
}

__global__ void nonfinite_kernel(const double *__restrict__ x, int64_t n, int *flag) {
  int bad = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) flag[0] = 1;  // benign race: every writer stores the same value
}

// SplitMix64 (Steele, Lea, Flood 2014) in counter form: output k of stream
// `seed` is mix(seed + (k+1) * gamma), mapped to [-1, 1).
__global__ void splitmix_fill_kernel(double *__restrict__ dst, int64_t n, uint64_t seed, int64_t start) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t z = seed + (uint64_t)(start + i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    dst[i] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
}

// out[0] = sum of squares of x[0..n), one workgroup, fixed order.
__global__ __launch_bounds__(1024) void sumsq_kernel(const double *__restrict__ x, int64_t n,
                                                     double *__restrict__ out) {
  __shared__ double red[16];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 1024) acc = fma(x[i], x[i], acc);
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    out[0] = t;
  }
}

static int grid_for(int64_t n, int threads) {
  int64_t g = (n + threads - 1) / threads;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_copy(double *dst, const double *src, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}

hipError_t launch_fill(double *dst, double v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, v, n);
  return hipGetLastError();
}

hipError_t launch_splitmix_fill(double *dst, int64_t n, uint64_t seed, int64_t start, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(splitmix_fill_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, n, seed, start);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double *x, int64_t n, double *out, hipStream_t s) {
  hipLaunchKernelGGL(sumsq_kernel, dim3(1), dim3(1024), 0, s, x, n, out);
  return hipGetLastError();
}

hipError_t launch_zero_int(int *p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(zero_int_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_reverse_core(double *out, const double *in, int rl, int d, int rr, hipStream_t s) {
  const int64_t n = (int64_t)rl * d * rr;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(reverse_core_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, out, in, rl, d, rr);
  return hipGetLastError();
}

hipError_t launch_transpose(double *out, const double *in, int m, int n, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 grid((n + 31) / 32, (m + 31) / 32);
  if (grid.y > 65535u) return hipErrorInvalidValue;
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, s, out, in, m, n);
  return hipGetLastError();
}

hipError_t launch_nonfinite_check(const double *x, int64_t n, int *flag, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(nonfinite_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, n, flag);
  return hipGetLastError();
}

// ---------------------------------------------------------------- QR
// Blocked Householder QR (LAPACK geqrf / orgqr structure): panels of QB
// columns are factored by one workgroup, the block reflector
// H = I - V T V^T (compact WY form) is built from V^T V, and the trailing
// columns and the explicit Q are updated with FP64 MFMA products.
namespace {
constexpr int QR_NT = 1024;
constexpr int QB = 16;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ double block_sum(double v, double *red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) t += red[w];  // fixed order: every thread gets the same sum
  return t;
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

// Factor columns j0 .. j0+jb-1 of S (column-major, ld m) in place (rows >= j0),
// then write the explicit panel V (rows j0..m-1, unit diagonal, zeros above;
// column-major with ld m - j0) and T (jb x jb, row-major, upper triangular).
__global__ __launch_bounds__(QR_NT) void qr_panel_kernel(double *__restrict__ S, int m, int j0, int jb,
                                                         double *__restrict__ tau, double *__restrict__ Vb,
                                                         double *__restrict__ T) {
  __shared__ double red[QR_NT / 64];
  __shared__ double Y[QB][QB + 1];
  __shared__ double Tl[QB][QB + 1];
  __shared__ double tl[QB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int j = j0; j < j0 + jb; ++j) {
    double *col = S + (int64_t)j * m;
    double part = 0.0;
    for (int i = j + 1 + tid; i < m; i += QR_NT) part += col[i] * col[i];
    const double xnorm2 = block_sum(part, red);
    const double alpha = col[j];
    double t = 0.0, scale = 0.0, beta = alpha;
    if (xnorm2 > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
      t = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();
    if (xnorm2 > 0.0)
      for (int i = j + 1 + tid; i < m; i += QR_NT) col[i] *= scale;
    if (tid == 0) {
      col[j] = beta;
      tau[j] = t;
      tl[j - j0] = t;
    }
    __syncthreads();
    if (t != 0.0) {
      for (int c = j + 1 + wave; c < j0 + jb; c += QR_NT / 64) {
        double *x = S + (int64_t)c * m;
        double w = 0.0;
        for (int i = j + 1 + lane; i < m; i += 64) w += col[i] * x[i];
        w = wave_sum(w) + x[j];
        const double tw = t * w;
        if (lane == 0) x[j] -= tw;
        for (int i = j + 1 + lane; i < m; i += 64) x[i] -= tw * col[i];
      }
    }
    __syncthreads();
  }
  // explicit V
  const int mv = m - j0;
  for (int64_t e = tid; e < (int64_t)mv * jb; e += QR_NT) {
    const int i = (int)(e % mv), c = (int)(e / mv);
    const int gi = j0 + i, gc = j0 + c;
    Vb[e] = (gi < gc) ? 0.0 : (gi == gc ? 1.0 : S[(int64_t)gc * m + gi]);
  }
  __syncthreads();
  // Y = V^T V: 4 threads per entry, rows split four ways
  {
    const int ent = tid >> 2, quarter = tid & 3;
    const int a = ent / QB, b = ent % QB;
    double acc = 0.0;
    if (a < jb && b < jb) {
      const double *va = Vb + (int64_t)a * mv, *vb = Vb + (int64_t)b * mv;
      for (int i = quarter; i < mv; i += 4) acc += va[i] * vb[i];
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    if (quarter == 0 && a < jb && b < jb) Y[a][b] = acc;
  }
  __syncthreads();
  // T: T[i][i] = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] Y[0:i, i]
  if (tid == 0) {
    for (int i = 0; i < jb; ++i) {
      for (int r = 0; r < jb; ++r) Tl[r][i] = 0.0;
      const double ti = tl[i];
      Tl[i][i] = ti;
      for (int r = 0; r < i; ++r) {
        double acc = 0.0;
        for (int c = r; c < i; ++c) acc += Tl[r][c] * Y[c][i];
        Tl[r][i] = -ti * acc;
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < jb * jb; e += QR_NT) T[e] = Tl[e / jb][e % jb];
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

// Explicit V of panel j0 (rows j0..m-1) rebuilt from the factored S.
__global__ void qr_extract_v_kernel(const double *__restrict__ S, int m, int j0, int jb,
                                    double *__restrict__ Vb) {
  const int mv = m - j0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)mv * jb;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % mv), c = (int)(e / mv);
    const int gi = j0 + i, gc = j0 + c;
    Vb[e] = (gi < gc) ? 0.0 : (gi == gc ? 1.0 : S[(int64_t)gc * m + gi]);
  }
}

size_t qr_scratch_doubles(int m, int n) {
  const int k = m < n ? m : n;
  const int np = (k + QB - 1) / QB;
  size_t t = 0;
  t += (size_t)m * n;          // S
  t += (size_t)k + 32;         // tau
  t += (size_t)m * QB;         // Vb
  t += (size_t)np * QB * QB;   // T per panel
  t += 2 * (size_t)QB * n;     // Wt1, Wt2
  t += (size_t)m * k;          // Qs
  return t + 8 * 32;
}

hipError_t launch_qr(const double *M, int m, int n, int64_t rs, int64_t cs, double *q, double *r,
                     double *scratch, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipErrorInvalidValue;
  const int k = m < n ? m : n;
  const int np = (k + QB - 1) / QB;
  double *p = scratch;
  auto adv = [&](size_t nd) { double *x = p; p += (nd + 31) & ~(size_t)31; return x; };
  double *S = adv((size_t)m * n);
  double *tau = adv((size_t)k + 32);
  double *Vb = adv((size_t)m * QB);
  double *Tall = adv((size_t)np * QB * QB);
  double *Wt1 = adv((size_t)QB * n);
  double *Wt2 = adv((size_t)QB * n);
  double *Qs = adv((size_t)m * k);
  const int64_t tot = (int64_t)m * n;
  hipLaunchKernelGGL(strided_to_colmajor_kernel, dim3(grid_for(tot, 256)), dim3(256), 0, s, S, M, m, n, rs, cs);
  for (int pi = 0; pi < np; ++pi) {
    const int j0 = pi * QB, jb = (k - j0) < QB ? (k - j0) : QB;
    double *T = Tall + (size_t)pi * QB * QB;
    hipLaunchKernelGGL(qr_panel_kernel, dim3(1), dim3(QR_NT), 0, s, S, m, j0, jb, tau, Vb, T);
    const int nt = n - (j0 + jb);
    if (nt > 0) {
      const int mv = m - j0;
      GemmArgs g;  // Wt1 = V^T A_trail
      g.M = jb; g.N = nt; g.K = mv;
      g.A = Vb; g.a_rs = mv; g.a_cs = 1;
      g.B = S + (int64_t)(j0 + jb) * m + j0; g.b_rs = 1; g.b_cs = m;
      g.C = Wt1; g.c_rs1 = nt; g.c_cs1 = 1;
      hipError_t e = launch_gemm(g, s);
      if (e != hipSuccess) return e;
      GemmArgs h;  // Wt2 = T^T Wt1
      h.M = jb; h.N = nt; h.K = jb;
      h.A = T; h.a_rs = 1; h.a_cs = jb;
      h.B = Wt1; h.b_rs = nt; h.b_cs = 1;
      h.C = Wt2; h.c_rs1 = nt; h.c_cs1 = 1;
      e = launch_gemm(h, s);
      if (e != hipSuccess) return e;
      GemmArgs u;  // A_trail -= V Wt2
      u.M = mv; u.N = nt; u.K = jb;
      u.A = Vb; u.a_rs = 1; u.a_cs = mv;
      u.B = Wt2; u.b_rs = nt; u.b_cs = 1;
      u.C = S + (int64_t)(j0 + jb) * m + j0; u.c_rs1 = 1; u.c_cs1 = m;
      u.alpha = -1.0; u.beta = 1.0;
      e = launch_gemm(u, s);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(qr_r_and_identity_kernel, dim3(grid_for((int64_t)k * n + (int64_t)m * k, 256)), dim3(256),
                     0, s, S, m, n, k, r, Qs);
  // Q = H_0 ... H_{np-1} applied to [I_k; 0], panels in reverse order.
  for (int pi = np - 1; pi >= 0; --pi) {
    const int j0 = pi * QB, jb = (k - j0) < QB ? (k - j0) : QB;
    const int mv = m - j0, nq = k - j0;
    double *T = Tall + (size_t)pi * QB * QB;
    hipLaunchKernelGGL(qr_extract_v_kernel, dim3(grid_for((int64_t)mv * jb, 256)), dim3(256), 0, s, S, m, j0,
                       jb, Vb);
    GemmArgs g;  // Wt1 = V^T Qsub
    g.M = jb; g.N = nq; g.K = mv;
    g.A = Vb; g.a_rs = mv; g.a_cs = 1;
    g.B = Qs + (int64_t)j0 * m + j0; g.b_rs = 1; g.b_cs = m;
    g.C = Wt1; g.c_rs1 = nq; g.c_cs1 = 1;
    hipError_t e = launch_gemm(g, s);
    if (e != hipSuccess) return e;
    GemmArgs h;  // Wt2 = T Wt1
    h.M = jb; h.N = nq; h.K = jb;
    h.A = T; h.a_rs = jb; h.a_cs = 1;
    h.B = Wt1; h.b_rs = nq; h.b_cs = 1;
    h.C = Wt2; h.c_rs1 = nq; h.c_cs1 = 1;
    e = launch_gemm(h, s);
    if (e != hipSuccess) return e;
    GemmArgs u;  // Qsub -= V Wt2
    u.M = mv; u.N = nq; u.K = jb;
    u.A = Vb; u.a_rs = 1; u.a_cs = mv;
    u.B = Wt2; u.b_rs = nq; u.b_cs = 1;
    u.C = Qs + (int64_t)j0 * m + j0; u.c_rs1 = 1; u.c_cs1 = m;
    u.alpha = -1.0; u.beta = 1.0;
    e = launch_gemm(u, s);
    if (e != hipSuccess) return e;
  }
  // q (m x k, row-major) from Qs (column-major)
  return launch_transpose(q, Qs, k, m, s);
}

}  // namespace ttm
