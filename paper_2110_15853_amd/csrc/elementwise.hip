// Streaming kernels: precision casts (FP64 <-> FP32 <-> BF16, round to nearest
// even) and row gathers between natural and lattice-blocked order.  Both are
// HBM-bound: one read and one write per element, grid-stride over rows with
// the columns of a row mapped to consecutive lanes for coalesced access.
#include "ttdft_internal.h"

namespace ttdft {
namespace {

template <typename S> __device__ inline double load_as_f64(const S *p) { return (double)*p; }
template <> __device__ inline double load_as_f64<__bf16>(const __bf16 *p) { return (double)(float)*p; }

template <typename D> __device__ inline void store_from_f64(D *p, double v) { *p = (D)v; }
// FP64 -> BF16 rounds through FP32 (nearest even at both steps).
template <> __device__ inline void store_from_f64<__bf16>(__bf16 *p, double v) { *p = (__bf16)(float)v; }

template <typename S, typename D>
__global__ __launch_bounds__(256) void cast_kernel(const S *__restrict__ src, int64_t lds,
                                                   D *__restrict__ dst, int64_t ldd,
                                                   int64_t rows, int64_t cols) {
  const int64_t chunks = (cols + 255) / 256;
  for (int64_t w = blockIdx.x; w < rows * chunks; w += gridDim.x) {
    const int64_t r = w / chunks, c = (w % chunks) * 256 + threadIdx.x;
    if (c < cols) store_from_f64<D>(dst + r * ldd + c, load_as_f64<S>(src + r * lds + c));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void gather_kernel(const T *__restrict__ src, int64_t lds,
                                                     T *__restrict__ dst, int64_t ldd,
                                                     int64_t rows, int64_t cols,
                                                     const int64_t *__restrict__ perm) {
  const int64_t chunks = (cols + 255) / 256;
  for (int64_t w = blockIdx.x; w < rows * chunks; w += gridDim.x) {
    const int64_t r = w / chunks, c = (w % chunks) * 256 + threadIdx.x;
    if (c >= cols) continue;
    const int64_t p = perm[r];
    dst[r * ldd + c] = p >= 0 ? src[p * lds + c] : T(0);
  }
}

inline unsigned grid_for(int64_t work) {
  const int64_t cap = 256 * 64;  // enough resident work-groups to fill the chip
  return (unsigned)(work < cap ? (work > 0 ? work : 1) : cap);
}

template <typename S>
hipError_t cast_from(const S *src, int64_t lds, void *dst, ttdft_dtype dt, int64_t ldd,
                     int64_t rows, int64_t cols, hipStream_t s) {
  const unsigned g = grid_for(rows * ((cols + 255) / 256));
  if (dt == TTDFT_F64)
    hipLaunchKernelGGL((cast_kernel<S, double>), dim3(g), dim3(256), 0, s, src, lds, (double *)dst, ldd, rows, cols);
  else if (dt == TTDFT_F32)
    hipLaunchKernelGGL((cast_kernel<S, float>), dim3(g), dim3(256), 0, s, src, lds, (float *)dst, ldd, rows, cols);
  else
    hipLaunchKernelGGL((cast_kernel<S, __bf16>), dim3(g), dim3(256), 0, s, src, lds, (__bf16 *)dst, ldd, rows, cols);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cast(const void *src, ttdft_dtype st, int64_t lds, void *dst, ttdft_dtype dt,
                       int64_t ldd, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows == 0 || cols == 0) return hipSuccess;
  if (st == TTDFT_F64) return cast_from((const double *)src, lds, dst, dt, ldd, rows, cols, s);
  if (st == TTDFT_F32) return cast_from((const float *)src, lds, dst, dt, ldd, rows, cols, s);
  return cast_from((const __bf16 *)src, lds, dst, dt, ldd, rows, cols, s);
}

hipError_t launch_gather_rows(const void *src, int64_t lds, void *dst, int64_t ldd,
                              int64_t rows_dst, int64_t cols, const int64_t *perm, size_t elt,
                              hipStream_t s) {
  if (rows_dst == 0 || cols == 0) return hipSuccess;
  const unsigned g = grid_for(rows_dst * ((cols + 255) / 256));
  if (elt == 8)
    hipLaunchKernelGGL(gather_kernel<double>, dim3(g), dim3(256), 0, s, (const double *)src, lds,
                       (double *)dst, ldd, rows_dst, cols, perm);
  else if (elt == 4)
    hipLaunchKernelGGL(gather_kernel<float>, dim3(g), dim3(256), 0, s, (const float *)src, lds,
                       (float *)dst, ldd, rows_dst, cols, perm);
  else
    hipLaunchKernelGGL(gather_kernel<uint16_t>, dim3(g), dim3(256), 0, s, (const uint16_t *)src,
                       lds, (uint16_t *)dst, ldd, rows_dst, cols, perm);
  return hipGetLastError();
}

}  // namespace ttdft
