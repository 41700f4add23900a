// ttm_multiply_static: the TTM product with its workspace in a static device
// array instead of a caller buffer, for callers that cannot allocate device
// memory.  The array is a file-scope __device__ variable: the loader places
// one copy on every device the code object is loaded on, and that memory
// stays with the process.  Host code never uses the array's name as an
// address (on the host it is only a stand-in for the symbol); the device
// address of each device's copy is looked up once with hipGetSymbolAddress,
// with that device current, and kept per device.
#include <math.h>

#include <mutex>

#include "ttm_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[TTM_STATIC_WS_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` on each device, null until looked up

// The device address of this device's copy of the array, looked up on the
// first call on the device.  hipGetSymbolAddress neither allocates nor
// launches anything.
int scratch_on_device(int dev, void **ptr) {
  if (dev < 0 || dev >= kMaxDevices) {
    ttm::set_last_error("device %d is beyond the %d devices ttm_multiply_static tracks", dev, kMaxDevices);
    return TTM_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      ttm::note_hip_error(e, "hipGetSymbolAddress of the static workspace");
      return TTM_EHIP;
    }
    g_scratch[dev] = p;
  }
  *ptr = g_scratch[dev];
  return TTM_OK;
}

}  // namespace

extern "C" int ttm_multiply_static(const ttm_tt *A, const ttm_tt *B, int32_t chi_out, double tol,
                                   ttm_tt_out *C, void *stream, const ttm_options *opt, ttm_stats *stats) {
  ttm::clear_last_error();
  // Event timing creates HIP events, which this entry point must not do.
  if (opt && opt->profile != 0) return TTM_EINVAL;
  if (!(tol >= 0.0) || !isfinite(tol)) return TTM_EINVAL;
  size_t need = 0;
  int64_t cap = 0;
  int e = ttm_query(A, B, chi_out, opt, &need, &cap);
  if (e != TTM_OK) return e;
  if (!C || !C->bonds || !C->offsets || !C->data) return TTM_EINVAL;
  if (C->capacity < cap) return TTM_ECAPACITY;
  if (need > (size_t)TTM_STATIC_WS_BYTES) {
    ttm::set_last_error("the product needs a %zu-byte workspace; the static one holds %zu bytes", need,
                        (size_t)TTM_STATIC_WS_BYTES);
    return TTM_EWORKSPACE;
  }
  int dev = 0;
  const hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) {
    ttm::note_hip_error(he, "hipGetDevice of ttm_multiply_static");
    return TTM_EHIP;
  }
  void *ws = nullptr;
  e = scratch_on_device(dev, &ws);
  if (e != TTM_OK) return e;
  // The product clears the one region it reads before writing (its flag
  // words, by a kernel); every other byte of the workspace is written before
  // it is read, so the previous call's contents do not matter.
  return ttm_multiply_ex(A, B, chi_out, tol, C, ws, (size_t)TTM_STATIC_WS_BYTES, stream, opt, stats);
}
