// FP64 matrix-core GEMMs for the dense steps of Algorithm 1 (Sec. 3.4) that
// follow the filter:
//   TN  C = A^T B   (n x n from two tall rows x n blocks): Gram matrix of the
//                   Cholesky-QR (step 2) and the projection X_F^T (H X_F) (step 3);
//   NN  C = A B     (tall rows x n times a small n x n): Y R^{-1} (step 2) and
//                   the rotation Psi = X_F Q (step 5).
// Both share one 128x128 output tile per work-group (4 waves, each a 64x64
// quadrant of 4x4 MFMA f64 16x16x4 blocks) and stage 32-deep K panels of both
// operands in LDS, k-major, so every MFMA operand read is 16 consecutive doubles.
// The TN product splits K across work-groups; partial tiles are summed in a
// fixed order by a second kernel, so results are deterministic.
#include "ttdft_internal.h"

namespace ttdft {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 32, THREADS = 256;
constexpr int LDS_LD = BM + 1;   // +1 double: stride of 258 dwords spreads the banks

__device__ inline v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// acc[mi][ni] covers rows 64*wm + 16*mi .. , cols 64*wn + 16*ni .. of the tile
__device__ inline void mma_panel(const double (*sA)[LDS_LD], const double (*sB)[LDS_LD],
                                 v4d (&acc)[4][4], int wm, int wn, int lane) {
#pragma unroll
  for (int kq = 0; kq < BK; kq += 4) {
    double a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = sA[kq + (lane >> 4)][64 * wm + 16 * i + (lane & 15)];
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = sB[kq + (lane >> 4)][64 * wn + 16 * j + (lane & 15)];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
  }
}

// output item t of lane l in a 16x16 f64 block sits at row (l>>4) + 4t, col l&15
__device__ inline int out_row(int lane, int t) { return (lane >> 4) + 4 * t; }

// ---------------------------------------------------------------- C = A^T B, split K
// grid.x = tile index (lower-triangular pairs when sym), grid.y = split
__global__ __launch_bounds__(THREADS) void gemm_tn_kernel(
    const double *__restrict__ A, int64_t lda, const double *__restrict__ B, int64_t ldb,
    int64_t K, int64_t n, double *__restrict__ partial, int64_t k_per_split, int tiles_n,
    int sym) {
  __shared__ double sA[BK][LDS_LD];
  __shared__ double sB[BK][LDS_LD];
  int ti, tj;
  if (sym) {  // linear index over lower-triangular tile pairs (ti >= tj)
    int t = blockIdx.x;
    ti = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    while (ti * (ti + 1) / 2 > t) --ti;
    tj = t - ti * (ti + 1) / 2;
  } else {
    ti = blockIdx.x / tiles_n;
    tj = blockIdx.x % tiles_n;
  }
  const int64_t i0 = (int64_t)ti * BM, j0 = (int64_t)tj * BN;
  const int64_t kb = (int64_t)blockIdx.y * k_per_split;
  const int64_t ke = min(K, kb + k_per_split);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0, 0, 0, 0};

  for (int64_t k0 = kb; k0 < ke; k0 += BK) {
#pragma unroll
    for (int q = 0; q < BK * BM / THREADS; ++q) {
      const int idx = tid + THREADS * q;
      const int kk = idx / BM, c = idx % BM;
      const int64_t k = k0 + kk;
      const bool kin = k < ke;
      sA[kk][c] = (kin && i0 + c < n) ? A[k * lda + i0 + c] : 0.0;
      sB[kk][c] = (kin && j0 + c < n) ? B[k * ldb + j0 + c] : 0.0;
    }
    __syncthreads();
    mma_panel(sA, sB, acc, wm, wn, lane);
    __syncthreads();
  }

  double *P = partial + (int64_t)blockIdx.y * n * n;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = j0 + 64 * wn + 16 * j + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t row = i0 + 64 * wm + 16 * i + out_row(lane, t);
        if (row < n && col < n) P[row * n + col] = acc[i][j][t];
      }
    }
}

// C[i][j] = sum_s partial[s][i][j] in order s = 0, 1, ...; sym mirrors the
// lower-triangular tiles; symmetrize writes (P + P^T)/2.
__global__ __launch_bounds__(256) void reduce_splits_kernel(const double *__restrict__ partial,
                                                            int splits, int64_t n, double *C,
                                                            int64_t ldc, int sym, int symmetrize) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n, j = e % n;
    int64_t src = e;
    if (sym && (i / BM) < (j / BN)) src = j * n + i;
    double v = 0.0;
    for (int s = 0; s < splits; ++s) v += partial[(int64_t)s * total + src];
    if (symmetrize) {
      double u = 0.0;
      const int64_t srcT = j * n + i;
      for (int s = 0; s < splits; ++s) u += partial[(int64_t)s * total + srcT];
      v = 0.5 * (v + u);
    }
    C[i * ldc + j] = v;
  }
}

// ---------------------------------------------------------------- C = alpha * A B
// A: rows x K (lda), B: K x N (ldb), C: rows x N (ldc).  upper: B[k][j] = 0 for k > j.
__global__ __launch_bounds__(THREADS) void gemm_nn_kernel(
    const double *__restrict__ A, int64_t lda, const double *__restrict__ B, int64_t ldb,
    int64_t rows, int64_t K, int64_t N, double alpha, double *__restrict__ C, int64_t ldc,
    int upper, int tiles_n) {
  __shared__ double sA[BK][LDS_LD];   // transposed A panel: [k][row]
  __shared__ double sB[BK][LDS_LD];
  const int64_t tn = blockIdx.x % tiles_n, tm = blockIdx.x / tiles_n;
  const int64_t i0 = tm * BM, j0 = tn * BN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
  const int64_t kend = upper ? min(K, j0 + BN) : K;

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0, 0, 0, 0};

  for (int64_t k0 = 0; k0 < kend; k0 += BK) {
#pragma unroll
    for (int q = 0; q < BK * BM / THREADS; ++q) {
      const int idx = tid + THREADS * q;
      // A: consecutive threads walk k inside a row (coalesced 256-byte row segments)
      const int r = idx / BK, kk = idx % BK;
      const int64_t k = k0 + kk;
      sA[kk][r] = (i0 + r < rows && k < kend) ? A[(i0 + r) * lda + k] : 0.0;
      const int kb = idx / BN, c = idx % BN;
      const int64_t kB = k0 + kb;
      sB[kb][c] = (kB < kend && j0 + c < N) ? B[kB * ldb + j0 + c] : 0.0;
    }
    __syncthreads();
    mma_panel(sA, sB, acc, wm, wn, lane);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = j0 + 64 * wn + 16 * j + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t row = i0 + 64 * wm + 16 * i + out_row(lane, t);
        if (row < rows && col < N) C[row * ldc + col] = alpha * acc[i][j][t];
      }
    }
}

}  // namespace

int gemm_tn_splits(int64_t rows, int64_t n) {
  const int64_t tiles = ((n + BM - 1) / BM) * ((n + BM - 1) / BM);
  int64_t s = (2048 + tiles - 1) / tiles;              // aim for >= 2048 work-groups
  const int64_t max_by_k = (rows + 16 * BK - 1) / (16 * BK);  // at least 16 panels each
  s = std::max<int64_t>(1, std::min<int64_t>(s, std::min<int64_t>(max_by_k, 64)));
  return (int)s;
}

hipError_t launch_gemm_tn(const double *A, int64_t lda, const double *B, int64_t ldb,
                          int64_t rows, int64_t n, double *C, int64_t ldc, bool sym,
                          double *partial, int splits, hipStream_t s) {
  return launch_gemm_tn_ex(A, lda, B, ldb, rows, n, C, ldc, sym, false, partial, splits, s);
}

hipError_t launch_gemm_tn_ex(const double *A, int64_t lda, const double *B, int64_t ldb,
                             int64_t rows, int64_t n, double *C, int64_t ldc, bool sym,
                             bool symmetrize, double *partial, int splits, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int tiles_n = (int)((n + BM - 1) / BM);
  const int64_t n_tiles = sym ? (int64_t)tiles_n * (tiles_n + 1) / 2 : (int64_t)tiles_n * tiles_n;
  int64_t kps = (rows + splits - 1) / splits;
  kps = (kps + BK - 1) / BK * BK;
  hipLaunchKernelGGL(gemm_tn_kernel, dim3((unsigned)n_tiles, (unsigned)splits), dim3(THREADS), 0,
                     s, A, lda, B, ldb, rows, n, partial, kps, tiles_n, sym ? 1 : 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = n * n;
  const unsigned g = (unsigned)std::min<int64_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL(reduce_splits_kernel, dim3(g), dim3(256), 0, s, partial, splits, n, C, ldc,
                     sym ? 1 : 0, symmetrize ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_gemm_nn(const double *A, int64_t lda, const double *B, int64_t ldb,
                          int64_t rows, int64_t n, double *C, int64_t ldc, bool upper,
                          hipStream_t s) {
  return launch_gemm_nn_ex(A, lda, B, ldb, rows, n, n, 1.0, C, ldc, upper, s);
}

hipError_t launch_gemm_nn_ex(const double *A, int64_t lda, const double *B, int64_t ldb,
                             int64_t rows, int64_t K, int64_t N, double alpha, double *C,
                             int64_t ldc, bool upper, hipStream_t s) {
  if (rows <= 0 || N <= 0) return hipSuccess;
  const int tiles_n = (int)((N + BN - 1) / BN);
  const int64_t tiles_m = (rows + BM - 1) / BM;
  const int64_t g = tiles_m * tiles_n;
  if (g > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(gemm_nn_kernel, dim3((unsigned)g), dim3(THREADS), 0, s, A, lda, B, ldb,
                     rows, K, N, alpha, C, ldc, upper ? 1 : 0, tiles_n);
  return hipGetLastError();
}

}  // namespace ttdft
