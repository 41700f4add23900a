// Small data-movement kernels and the per-kernel event timer.
#include "ttm_internal.h"

namespace ttm {

// ---------------------------------------------------------------- kernel timer
namespace {
// One pool per host thread, reused across calls made on that thread.  A
// batched call runs its products on worker threads that end with the call:
// their pools destroy their events as the thread exits (every event is
// complete by then, since each call collects its times before returning).
struct EventPool {
  hipEvent_t ev[2 * 4096];
  int n = 0;  // events created
  EventPool() = default;
  EventPool(const EventPool &) = delete;
  EventPool &operator=(const EventPool &) = delete;
  ~EventPool() {
    for (int i = 0; i < n; ++i) (void)hipEventDestroy(ev[i]);
  }
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

}  // namespace ttm
