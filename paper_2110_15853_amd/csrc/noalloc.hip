// The Chebyshev filter without a workspace argument, for callers that cannot
// allocate device memory (code under graph capture, tight serving loops).
//
// The filter's one rows x n_vec work block lives in a fixed device array of this
// file, `scratch`, which every GPU the library runs on holds until the process
// ends.  In host code the array's name stands for a host-side shadow, not a
// device address, so the device address is looked up once per device (with that
// device current) by hipGetSymbolAddress and only that pointer is handed to the
// kernels.  Calls on one GPU share its array: calls that overlap in time on one
// GPU (different streams, or the same stream from threads that interleave) race
// on it.  The filter writes every element of the work block before reading it,
// so nothing needs clearing between calls.
#include <mutex>

#include "ttdft_internal.h"

static __device__ __align__(256) unsigned char scratch[TTDFT_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device (looked up on first use)
hipError_t scratch_on_current_device(void **ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" ttdft_status ttdft_cheb_filter_noalloc(const ttdft_bsr *H, const void *X, int64_t ldx,
                                                  void *Y, int64_t ldy, int64_t n_vec, int32_t m,
                                                  double a, double b, double a0,
                                                  ttdft_dtype x_dtype, void *stream) {
  using namespace ttdft;
  ttdft_status st = filter_check(H, X, ldx, Y, ldy, n_vec, m, a, b, a0, x_dtype);
  if (st != TTDFT_OK) return st;
  const size_t need = ttdft_cheb_filter_workspace(H, n_vec, x_dtype);
  if (m >= 2 && need > (size_t)TTDFT_NOALLOC_SCRATCH_BYTES) {
    char msg[200];
    snprintf(msg, sizeof msg,
             "work block of %zu bytes exceeds the fixed scratch of %llu bytes "
             "(use ttdft_cheb_filter with a workspace)",
             need, (unsigned long long)TTDFT_NOALLOC_SCRATCH_BYTES);
    return api_fail(TTDFT_ERR_WORKSPACE, msg);
  }
  void *work = nullptr;
  if (m >= 2) {
    hipError_t e = scratch_on_current_device(&work);
    if (e != hipSuccess) {
      char msg[200];
      snprintf(msg, sizeof msg, "scratch address lookup: %s", hipGetErrorString(e));
      return api_fail(TTDFT_ERR_HIP, msg);
    }
  }
  return filter_enqueue(*H, X, ldx, Y, ldy, n_vec, m, a, b, a0, x_dtype, work, (hipStream_t)stream);
}
