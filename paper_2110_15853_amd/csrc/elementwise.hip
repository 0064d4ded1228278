// Streaming kernels: precision casts (FP64 <-> FP32 <-> BF16, round to nearest
// even) and row gathers between natural and lattice-blocked order.  Both are
// HBM-bound: one read and one write per element, grid-stride over rows with
// the columns of a row mapped to consecutive lanes for coalesced access.
#include "ttdft_internal.h"

namespace ttdft {
namespace {

template <typename S> __device__ inline double load_as_f64(const S *p) { return (double)*p; }
template <> __device__ inline double load_as_f64<__bf16>(const __bf16 *p) { return (double)(float)*p; }

// FP64 -> BF16 rounds through FP32 (nearest even at both steps).  The empty asm
// makes the FP32 value exist: without it the compiler may fold the two
// conversions into one rounding from FP64, which differs when the FP32 value is
// a bf16 tie.
__device__ inline __bf16 bf16_via_f32(double v) {
  float f = (float)v;
  asm volatile("" : "+v"(f));
  return (__bf16)f;
}

template <typename D> __device__ inline void store_from_f64(D *p, double v) { *p = (D)v; }
template <> __device__ inline void store_from_f64<__bf16>(__bf16 *p, double v) { *p = bf16_via_f32(v); }

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

namespace {
// Tile values from the 16x4 fragment order of FP64 / FP32 tiles to another tile
// type.  F32 keeps the 16x4 order (a plain rounding).  BF16 and BF16_SPLIT use
// the 16x32 order of the bf16 op: destination value d of a tile holds entry
// (i, j) with fragment d/512 = 4*(j/32) + i/16, lane (d/8)%64 = i%16 + 16*((j%32)/8)
// and j%8 = d%8; it is read from the source position of (i, j).  BF16_SPLIT
// holds hi = bf16(fp32(h)) in the first 4096 values of a tile and
// lo = bf16(fp32(h) - hi) in the next 4096 (the subtraction is exact in FP32).
template <typename S>
__global__ __launch_bounds__(256) void convert_tiles_kernel(const S *__restrict__ src, int64_t total,
                                                            void *__restrict__ dst, int dt) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t t = e / kTileElems;
    const int d = (int)(e % kTileElems);
    if (dt == TTDFT_F32) {
      ((float *)dst)[e] = (float)src[e];
      continue;
    }
    const int f = d >> 9, L = (d >> 3) & 63;
    const int i = 16 * (f & 3) + (L & 15), j = 32 * (f >> 2) + 8 * (L >> 4) + (d & 7);
    float h32 = (float)src[t * kTileElems + tile_pos_16x4(i, j)];
    asm volatile("" : "+v"(h32));   // two roundings from FP64, as bf16_via_f32
    const __bf16 hi = (__bf16)h32;
    if (dt == TTDFT_BF16) {
      ((__bf16 *)dst)[e] = hi;
    } else {
      ((__bf16 *)dst)[2 * t * kTileElems + d] = hi;
      ((__bf16 *)dst)[2 * t * kTileElems + kTileElems + d] = (__bf16)(h32 - (float)hi);
    }
  }
}
}  // namespace

hipError_t launch_convert_tiles(const void *src, ttdft_dtype st, int64_t n_tiles, void *dst,
                                ttdft_dtype dt, hipStream_t s) {
  const int64_t total = n_tiles * kTileElems;
  if (total == 0) return hipSuccess;
  const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 16384);
  if (st == TTDFT_F64)
    hipLaunchKernelGGL(convert_tiles_kernel<double>, dim3(g), dim3(256), 0, s, (const double *)src,
                       total, dst, (int)dt);
  else
    hipLaunchKernelGGL(convert_tiles_kernel<float>, dim3(g), dim3(256), 0, s, (const float *)src,
                       total, dst, (int)dt);
  return hipGetLastError();
}

hipError_t launch_split_bf16(const double *src, int64_t n_tiles, void *dst, hipStream_t s) {
  return launch_convert_tiles(src, TTDFT_F64, n_tiles, dst, TTDFT_BF16_SPLIT, s);
}

namespace {
template <typename T> __device__ inline bool is_finite_elt(T v) { return isfinite(v); }
template <> __device__ inline bool is_finite_elt<__bf16>(__bf16 v) { return isfinite((float)v); }

// *count += number of non-finite entries of a rows x cols block (grid-stride;
// one atomic add of a wave's count per wave and pass; the total is exact)
template <typename T>
__global__ __launch_bounds__(256) void count_nonfinite_kernel(const T *__restrict__ A, int64_t ld,
                                                              int64_t rows, int64_t cols,
                                                              unsigned long long *count) {
  const int64_t chunks = (cols + 255) / 256;
  unsigned long long bad = 0;
  for (int64_t w = blockIdx.x; w < rows * chunks; w += gridDim.x) {
    const int64_t r = w / chunks, c = (w % chunks) * 256 + threadIdx.x;
    if (c < cols && !is_finite_elt<T>(A[r * ld + c])) ++bad;
  }
  for (int o = 32; o > 0; o >>= 1) bad += __shfl_down(bad, o, 64);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(count, bad);
}
}  // namespace

hipError_t launch_count_nonfinite(const void *A, ttdft_dtype dt, int64_t ld, int64_t rows,
                                  int64_t cols, unsigned long long *count, hipStream_t s) {
  if (rows == 0 || cols == 0) return hipSuccess;
  const unsigned g = grid_for(rows * ((cols + 255) / 256));
  if (dt == TTDFT_F64)
    hipLaunchKernelGGL(count_nonfinite_kernel<double>, dim3(g), dim3(256), 0, s, (const double *)A, ld,
                       rows, cols, count);
  else if (dt == TTDFT_F32)
    hipLaunchKernelGGL(count_nonfinite_kernel<float>, dim3(g), dim3(256), 0, s, (const float *)A, ld,
                       rows, cols, count);
  else
    hipLaunchKernelGGL(count_nonfinite_kernel<__bf16>, dim3(g), dim3(256), 0, s, (const __bf16 *)A, ld,
                       rows, cols, count);
  return hipGetLastError();
}

}  // namespace ttdft
