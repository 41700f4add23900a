// Many independent TTM products in one call: a host-side work queue that keeps
// one product in flight per stream of its own, so that the chains of small
// launches of several products' SVDs run side by side on the GPU.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include <hip/hip_runtime.h>

#include "ttm.h"
#include "ttm_internal.h"

namespace {

// Products in flight at most.  The measured optimum was 2 (a skewed batch)
// to 4 (nine even products); more streams slowed the critical product
// through contention for the command processor and the CUs, and every
// stream holds a hardware queue of its own.
constexpr int kMaxStreams = 4;

// Relative cost of one product for the start order: the swap SVDs dominate,
// N(N-1)/2 of them on matrices of side (swap cap) x (largest d).
double product_cost(const ttm_tt &A, const ttm_tt &B, int chi_out, const ttm_options *o) {
  int ra = 1, rb = 1, d = 1;
  for (int i = 0; i <= A.n_sites; ++i) ra = std::max(ra, A.bonds[i]);
  for (int i = 0; i <= B.n_sites; ++i) rb = std::max(rb, B.bonds[i]);
  for (int i = 0; i < A.n_sites; ++i) d = std::max(d, A.phys[i]);
  double cap = (double)ra * rb;
  const int cm = o ? o->chi_mid : -1;
  if (cm == -1) cap = std::min(cap, (double)chi_out);
  else if (cm > 0) cap = std::min(cap, (double)cm);
  const double m = cap * d;
  return (double)A.n_sites * A.n_sites * m * m * m;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
  return na && nb && x < y + nb && y < x + na;
}

}  // namespace

extern "C" int ttm_multiply_batch(int32_t n, const ttm_tt *A, const ttm_tt *B, const int32_t *chi_out,
                                  const double *tol, ttm_tt_out *C, void *const *ws, const size_t *ws_bytes,
                                  const ttm_options *opt, ttm_stats *stats, int32_t n_streams, void *stream,
                                  int32_t *status) {
  ttm::clear_last_error();
  if (n < 0 || n_streams < 1 || n_streams > kMaxStreams) return TTM_EINVAL;
  if (n == 0) return TTM_OK;
  if (!A || !B || !chi_out || !tol || !C || !ws || !ws_bytes) return TTM_EINVAL;
  // Every product is checked on the host before any of them starts.
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) {
    if (!(tol[i] >= 0.0) || !isfinite(tol[i])) return TTM_EINVAL;
    size_t need = 0;
    int64_t cap = 0;
    const ttm_options *oi = opt ? &opt[i] : nullptr;
    const int e = ttm_query(&A[i], &B[i], chi_out[i], oi, &need, &cap);
    if (e != TTM_OK) return e;
    if (!ws[i] || ws_bytes[i] < need) return TTM_EWORKSPACE;
    if (!C[i].data || C[i].capacity < cap) return TTM_ECAPACITY;
    cost[i] = product_cost(A[i], B[i], chi_out[i], oi);
  }
  // Products write their workspaces and outputs: no two may share memory.
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j) {
      const size_t ci = (size_t)C[i].capacity * sizeof(double), cj = (size_t)C[j].capacity * sizeof(double);
      if (overlap(ws[i], ws_bytes[i], ws[j], ws_bytes[j]) || overlap(C[i].data, ci, C[j].data, cj) ||
          overlap(ws[i], ws_bytes[i], C[j].data, cj) || overlap(C[i].data, ci, ws[j], ws_bytes[j]))
        return TTM_EINVAL;
    }
  int dev = 0;
  hipError_t he;
  if ((he = hipGetDevice(&dev)) != hipSuccess) {
    ttm::note_hip_error(he, "hipGetDevice of ttm_multiply_batch");
    return TTM_EHIP;
  }
  const int nw = std::min<int>(n, n_streams);
  // One stream per worker, each first waiting for the work already on the
  // caller's stream, which produced the inputs.  The streams carry a CU mask
  // (every CU of the device): the runtime gives a masked stream a hardware
  // queue of its own instead of sharing one of its few default queues, and
  // products overlap only on distinct queues.
  int n_cu = 0;
  if ((he = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess || n_cu < 1) {
    ttm::note_hip_error(he, "the CU count query of ttm_multiply_batch");
    return TTM_EHIP;
  }
  std::vector<uint32_t> mask((n_cu + 31) / 32, 0u);
  for (int c = 0; c < n_cu; ++c) mask[c / 32] |= 1u << (c % 32);
  hipStream_t caller = static_cast<hipStream_t>(stream);
  hipEvent_t ready = nullptr;
  std::vector<hipStream_t> own(nw, nullptr);
  auto release = [&]() {
    for (hipStream_t s : own)
      if (s) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
      }
    if (ready) (void)hipEventDestroy(ready);
  };
  if ((he = hipEventCreateWithFlags(&ready, hipEventDisableTiming)) != hipSuccess ||
      (he = hipEventRecord(ready, caller)) != hipSuccess) {
    ttm::note_hip_error(he, "the start event of ttm_multiply_batch");
    release();
    return TTM_EHIP;
  }
  for (int w = 0; w < nw; ++w) {
    if ((he = hipExtStreamCreateWithCUMask(&own[w], (uint32_t)mask.size(), mask.data())) != hipSuccess ||
        (he = hipStreamWaitEvent(own[w], ready, 0)) != hipSuccess) {
      ttm::note_hip_error(he, "the stream set-up of ttm_multiply_batch");
      release();
      return TTM_EHIP;
    }
  }
  // Longest first: the largest product is the critical path of the batch.
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<int32_t> st(n, TTM_OK);
  std::vector<std::string> why(n);
  std::atomic<int> next{0};
  // Worker w runs on own[w] and takes the next product whenever its last one
  // has finished (list scheduling, largest first).
  auto work = [&](int w) {
    const hipError_t se = hipSetDevice(dev);
    for (;;) {
      const int q = next.fetch_add(1);
      if (q >= n) break;
      const int i = order[q];
      if (se != hipSuccess) {
        st[i] = TTM_EHIP;
        why[i] = std::string("hipSetDevice of a batch worker: ") + hipGetErrorName(se);
        continue;
      }
      st[i] = ttm_multiply_ex(&A[i], &B[i], chi_out[i], tol[i], &C[i], ws[i], ws_bytes[i], own[w],
                              opt ? &opt[i] : nullptr, stats ? &stats[i] : nullptr);
      if (st[i] != TTM_OK) why[i] = ttm_last_error();
    }
  };
  if (nw == 1) {
    work(0);
  } else {
    std::vector<std::thread> pool;
    pool.reserve(nw);
    for (int w = 0; w < nw; ++w) pool.emplace_back(work, w);
    for (auto &t : pool) t.join();
  }
  release();
  int rc = TTM_OK;
  for (int i = 0; i < n; ++i) {
    if (status) status[i] = st[i];
    if (rc == TTM_OK && st[i] != TTM_OK) {
      rc = st[i];
      // the workers' messages are thread-local: hand the first one over
      if (!why[i].empty()) ttm::set_last_error("product %d: %s", i, why[i].c_str());
    }
  }
  return rc;
}
