// FP64 matrix-core GEMMs for the dense steps of Algorithm 1 (Sec. 3.4) that
// follow the filter:
//   TN  C = A^T B   (n x n from two tall rows x n blocks): Gram matrix of the
//                   Cholesky-QR (step 2) and the projection X_F^T (H X_F) (step 3);
//   NN  C = A B     (tall rows x n times a small n x n): Y R^{-1} (step 2) and
//                   the rotation Psi = X_F Q (step 5).
// Both share one 128x128 output tile per work-group (4 waves, each a 64x64
// quadrant of 4x4 MFMA f64 16x16x4 blocks); 16-deep K panels of both operands
// are double-buffered in LDS, k-major (every operand read is 16 consecutive
// doubles), with the next panel prefetched into registers during the current
// panel's contraction (one barrier per panel).
// The TN product splits K across work-groups; partial tiles are summed in a
// fixed order by a second kernel, so results are deterministic.
#include "ttdft_internal.h"

namespace ttdft {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 16, THREADS = 256;
constexpr int LDS_LD = BM + 4;   // row stride 132 doubles: rows 8 banks apart

__device__ inline v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// output item t of lane l in a 16x16 f64 block sits at row (l>>4) + 4t, col l&15
__device__ inline int out_row(int lane, int t) { return (lane >> 4) + 4 * t; }

// One 128x128 tile, K in panels of 16, double-buffered in LDS with the next
// panel prefetched into registers; both operands held k-major in LDS.
// TN: A is K x M (element (k, i) at A[k*lda + i]); NN: A is M x K (A[i*lda + k]).
// B is always K x N (B[k*ldb + j]).  Wave (wm, wn) owns the 64x64 quadrant.
template <bool TN> struct Tile {
  double (*sA)[BK][LDS_LD];
  double (*sB)[BK][LDS_LD];
  double ra[8], rb[8];
  v4d acc[4][4];

  __device__ void load(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t i0,
                       int64_t j0, int64_t k0, int64_t kend, int64_t M, int64_t N) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = tid + THREADS * q;
      if (TN) {
        const int kk = idx / BM, c = idx % BM;
        const int64_t k = k0 + kk;
        ra[q] = (k < kend && i0 + c < M) ? A[k * lda + i0 + c] : 0.0;
      } else {
        const int r = idx / BK, kk = idx % BK;      // 16 consecutive k of one row
        const int64_t k = k0 + kk;
        ra[q] = (k < kend && i0 + r < M) ? A[(i0 + r) * lda + k] : 0.0;
      }
      const int kb = idx / BN, c = idx % BN;
      const int64_t k = k0 + kb;
      rb[q] = (k < kend && j0 + c < N) ? B[k * ldb + j0 + c] : 0.0;
    }
  }
  __device__ void store(int buf) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = tid + THREADS * q;
      if (TN) sA[buf][idx / BM][idx % BM] = ra[q];
      else sA[buf][idx % BK][idx / BK] = ra[q];
      sB[buf][idx / BN][idx % BN] = rb[q];
    }
  }
  __device__ void compute(int buf, int wm, int wn, int lane) {
#pragma unroll
    for (int kq = 0; kq < BK; kq += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[buf][kq + (lane >> 4)][64 * wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[buf][kq + (lane >> 4)][64 * wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
    }
  }
  // acc = sum over k in [kb, ke) of opA(A)[i][k] B[k][j]
  __device__ void run(const double *A, int64_t lda, const double *B, int64_t ldb, int64_t i0,
                      int64_t j0, int64_t kb, int64_t ke, int64_t M, int64_t N) {
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0, 0, 0, 0};
    if (kb >= ke) return;
    load(A, lda, B, ldb, i0, j0, kb, ke, M, N);
    store(0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = kb; k0 < ke; k0 += BK) {
      const bool more = k0 + BK < ke;
      if (more) load(A, lda, B, ldb, i0, j0, k0 + BK, ke, M, N);
      compute(buf, wm, wn, lane);
      if (more) store(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }
};

// hardware ids are dealt round-robin to the 8 XCDs; give each XCD C consecutive
// logical ids so work-groups sharing an operand panel share that XCD's L2
__device__ inline int64_t xcd_group(int64_t g, int64_t G, int64_t C) {
  const int64_t span = 8 * C, full = (G / span) * span;
  if (g >= full) return g;
  return (g / span) * span + (g % 8) * C + (g / 8) % C;
}

// ---------------------------------------------------------------- C = A^T B, split K
// grid.x = tile index (lower-triangular pairs when sym), grid.y = split
__global__ __launch_bounds__(THREADS, 2) void gemm_tn_kernel(
    const double *__restrict__ A, int64_t lda, const double *__restrict__ B, int64_t ldb,
    int64_t K, int64_t n, double *__restrict__ partial, int64_t k_per_split, int tiles_n,
    int sym) {
  __shared__ double sA[2][BK][LDS_LD];
  __shared__ double sB[2][BK][LDS_LD];
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
  Tile<true> T;
  T.sA = sA;
  T.sB = sB;
  T.run(A, lda, B, ldb, i0, j0, kb, ke, n, n);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  double *P = partial + (int64_t)blockIdx.y * n * n;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = j0 + 64 * wn + 16 * j + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t row = i0 + 64 * wm + 16 * i + out_row(lane, t);
        if (row < n && col < n) P[row * n + col] = T.acc[i][j][t];
      }
    }
}

// ---------------------------------------------------------------- C = A^T B, split K, LDS-DMA
// The same tiles and waves as gemm_tn_kernel, with the panels moved straight into
// LDS (global_load_lds_dwordx4, no register staging) through a ring of DMA_STAGES
// panels of DMA_PK k-rows, issued DMA_STAGES - 1 panels ahead (after the first
// quarter of the current panel's products, so that the issue overlaps them), one
// work-group per CU.  For whole panels only: n a multiple of 128, K a multiple
// of DMA_PK, operands 16-byte aligned (checked on the host; other shapes take
// gemm_tn_kernel).
constexpr int DMA_PK = 16, DMA_STAGES = 4;
typedef __attribute__((address_space(3))) void lds_void_t;

template <int N> __device__ inline void gemm_wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

__global__ __launch_bounds__(THREADS, 1) void gemm_tn_dma_kernel(
    const double *__restrict__ A, int64_t lda, const double *__restrict__ B, int64_t ldb,
    int64_t K, int64_t n, double *__restrict__ partial, int64_t k_per_split, int tiles_n,
    int sym) {
  constexpr int RW = DMA_PK / 4;          // k-rows of each operand a wave moves per panel
  constexpr int XF = 2 * RW;              // transfers per wave per panel
  __shared__ __attribute__((aligned(16))) double sA[DMA_STAGES][DMA_PK][LDS_LD];
  __shared__ __attribute__((aligned(16))) double sB[DMA_STAGES][DMA_PK][LDS_LD];
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
  const int np = kb < ke ? (int)((ke - kb) / DMA_PK) : 0;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wm = w >> 1, wn = w & 1;

  // wave w moves k-rows w, w + 4, ... of both operands of a panel: one 1 KB row
  // (128 doubles) per transfer, 16 bytes per lane; the lane's addresses are its
  // row-w address plus a wave-uniform offset
  const double *a_lane = A + (kb + w) * lda + i0 + 2 * lane;
  const double *b_lane = B + (kb + w) * ldb + j0 + 2 * lane;
  auto issue = [&](int p) {
    const int st = p % DMA_STAGES;
    const int64_t ka = (int64_t)p * DMA_PK * lda, kbb = (int64_t)p * DMA_PK * ldb;
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const int r = w + 4 * q;
      const uint32_t la = (uint32_t)(uintptr_t)(lds_void_t *)(&sA[st][r][0]);
      const uint32_t lb = (uint32_t)(uintptr_t)(lds_void_t *)(&sB[st][r][0]);
      asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                   :
                   : "s"(__builtin_amdgcn_readfirstlane(la)), "v"(a_lane + ka + 4 * q * lda)
                   : "memory", "m0");
      asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                   :
                   : "s"(__builtin_amdgcn_readfirstlane(lb)), "v"(b_lane + kbb + 4 * q * ldb)
                   : "memory", "m0");
    }
  };

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0, 0, 0, 0};
  for (int p = 0; p < min(DMA_STAGES - 1, np); ++p) issue(p);
  for (int p = 0; p < np; ++p) {
    // this wave's transfers of panel p are done once at most those of the panels
    // issued after it (p + 1 .. p + DMA_STAGES - 2) are outstanding
    const int after = min(DMA_STAGES - 2, np - 1 - p);
    if (after >= 2) gemm_wait_vmcnt<2 * XF>();
    else if (after == 1) gemm_wait_vmcnt<XF>();
    else gemm_wait_vmcnt<0>();
    __syncthreads();   // every wave's part of panel p is in LDS; panel p - 1's stage is free
    const int st = p % DMA_STAGES;
#pragma unroll
    for (int kq = 0; kq < DMA_PK; kq += 4) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[st][kq + (lane >> 4)][64 * wm + 16 * i + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[st][kq + (lane >> 4)][64 * wn + 16 * j + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma(a[i], b[j], acc[i][j]);
      if (kq == 0 && p + DMA_STAGES - 1 < np) issue(p + DMA_STAGES - 1);
    }
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
        P[row * n + col] = acc[i][j][t];
      }
    }
}

// C[i][j] = sum_s partial[s][i][j] in order s = 0, 1, ...; sym mirrors the
// lower-triangular tiles; symmetrize writes (P + P^T)/2 (with sym: inside the
// diagonal tiles, the only ones holding both P_ij and P_ji).
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
    if (symmetrize && (!sym || i / BM == j / BN)) {
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
// The column tiles of one row panel of A run on one XCD (they share that panel).
__global__ __launch_bounds__(THREADS, 2) void gemm_nn_kernel(
    const double *__restrict__ A, int64_t lda, const double *__restrict__ B, int64_t ldb,
    int64_t rows, int64_t K, int64_t N, double alpha, double *__restrict__ C, int64_t ldc,
    int upper, int tiles_n, int64_t n_wg, int accumulate, int64_t stride_a, int64_t stride_b,
    int64_t stride_c) {
  __shared__ double sA[2][BK][LDS_LD];
  __shared__ double sB[2][BK][LDS_LD];
  A += (int64_t)blockIdx.y * stride_a;     // batch (grid.y) of equally shaped products
  B += (int64_t)blockIdx.y * stride_b;
  C += (int64_t)blockIdx.y * stride_c;
  const int64_t L = xcd_group(blockIdx.x, n_wg, tiles_n);
  const int64_t tn = L % tiles_n, tm = L / tiles_n;
  const int64_t i0 = tm * BM, j0 = tn * BN;
  const int64_t kend = upper ? min(K, j0 + BN) : K;
  Tile<false> T;
  T.sA = sA;
  T.sB = sB;
  T.run(A, lda, B, ldb, i0, j0, 0, kend, rows, N);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = j0 + 64 * wn + 16 * j + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t row = i0 + 64 * wm + 16 * i + out_row(lane, t);
        if (row < rows && col < N) {
          const double v = alpha * T.acc[i][j][t];
          C[row * ldc + col] = accumulate ? C[row * ldc + col] + v : v;
        }
      }
    }
}

// general C[M x N] = A^T B, A: K x M, B: K x N, K split over grid.y (partials)
__global__ __launch_bounds__(THREADS, 2) void gemm_tn_general_kernel(
    const double *__restrict__ A, int64_t lda, const double *__restrict__ B, int64_t ldb,
    int64_t K, int64_t M, int64_t N, double *__restrict__ partial, int64_t k_per_split,
    int tiles_n) {
  __shared__ double sA[2][BK][LDS_LD];
  __shared__ double sB[2][BK][LDS_LD];
  const int64_t tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int64_t i0 = tm * BM, j0 = tn * BN;
  const int64_t kb = (int64_t)blockIdx.y * k_per_split, ke = min(K, kb + k_per_split);
  Tile<true> T;
  T.sA = sA;
  T.sB = sB;
  T.run(A, lda, B, ldb, i0, j0, kb, ke, M, N);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
  double *P = partial + (int64_t)blockIdx.y * M * N;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = j0 + 64 * wn + 16 * j + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t row = i0 + 64 * wm + 16 * i + out_row(lane, t);
        if (row < M && col < N) P[row * N + col] = T.acc[i][j][t];
      }
    }
}

__global__ __launch_bounds__(256) void reduce_general_kernel(const double *__restrict__ partial,
                                                             int splits, int64_t M, int64_t N,
                                                             double *C, int64_t ldc) {
  const int64_t total = M * N;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    double v = 0.0;
    for (int s = 0; s < splits; ++s) v += partial[(int64_t)s * total + e];
    C[(e / N) * ldc + e % N] = v;
  }
}

// C[M x N] += alpha * A^T B with A: K x M (lda), B: K x N (ldb), small K (no split)
__global__ __launch_bounds__(THREADS, 2) void gemm_tn_acc_kernel(
    const double *__restrict__ A, int64_t lda, const double *__restrict__ B, int64_t ldb,
    int64_t K, int64_t M, int64_t N, double alpha, double *__restrict__ C, int64_t ldc,
    int tiles_n) {
  __shared__ double sA[2][BK][LDS_LD];
  __shared__ double sB[2][BK][LDS_LD];
  const int64_t tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
  const int64_t i0 = tm * BM, j0 = tn * BN;
  Tile<true> T;
  T.sA = sA;
  T.sB = sB;
  T.run(A, lda, B, ldb, i0, j0, 0, K, M, N);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, wm = w >> 1, wn = w & 1;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t col = j0 + 64 * wn + 16 * j + (lane & 15);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t row = i0 + 64 * wm + 16 * i + out_row(lane, t);
        if (row < M && col < N) C[row * ldc + col] += alpha * T.acc[i][j][t];
      }
    }
}

}  // namespace

hipError_t launch_gemm_tn_acc(const double *A, int64_t lda, const double *B, int64_t ldb,
                              int64_t K, int64_t M, int64_t N, double alpha, double *C,
                              int64_t ldc, hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  const int tiles_n = (int)((N + BN - 1) / BN);
  const int64_t g = ((M + BM - 1) / BM) * tiles_n;
  hipLaunchKernelGGL(gemm_tn_acc_kernel, dim3((unsigned)g), dim3(THREADS), 0, s, A, lda, B, ldb, K,
                     M, N, alpha, C, ldc, tiles_n);
  return hipGetLastError();
}

// Split-K count of the TN product.  Every work-group of one launch does the same
// work, so a last round of resident work-groups that is only partly filled
// leaves the rest of the chip idle: take the smallest split count that gives at
// least 3.5 rounds with the last one at least 95% full (two resident
// work-groups on each of the 256 CUs), else about four rounds.
int gemm_tn_splits(int64_t rows, int64_t n, bool sym) {
  const int64_t tn = (n + BM - 1) / BM;
  const int64_t tiles = sym ? tn * (tn + 1) / 2 : tn * tn;
  const int64_t max_s =
      std::max<int64_t>(1, std::min<int64_t>(64, (rows + 16 * BK - 1) / (16 * BK)));  // >= 16 panels each
  constexpr int64_t kResident = 2 * 256;
  for (int64_t s = 1; s <= max_s; ++s) {
    const int64_t wg = tiles * s, rounds = (wg + kResident - 1) / kResident;
    if (2 * wg >= 7 * kResident && 100 * wg >= 95 * rounds * kResident) return (int)s;
  }
  return (int)std::min<int64_t>(max_s, (4 * kResident + tiles - 1) / tiles);
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
  const bool whole = n % BM == 0 && rows % DMA_PK == 0 && kps % DMA_PK == 0 && lda % 2 == 0 &&
                     ldb % 2 == 0 &&
                     ((uintptr_t)A & 15) == 0 && ((uintptr_t)B & 15) == 0;
  if (whole)
    hipLaunchKernelGGL(gemm_tn_dma_kernel, dim3((unsigned)n_tiles, (unsigned)splits), dim3(THREADS),
                       0, s, A, lda, B, ldb, rows, n, partial, kps, tiles_n, sym ? 1 : 0);
  else
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
                     rows, K, N, alpha, C, ldc, upper ? 1 : 0, tiles_n, g, 0, 0, 0, 0);
  return hipGetLastError();
}

hipError_t launch_gemm_nn_batched(const double *A, int64_t lda, int64_t stride_a, const double *B,
                                  int64_t ldb, int64_t stride_b, int64_t rows, int64_t K, int64_t N,
                                  double alpha, double *C, int64_t ldc, int64_t stride_c, int batch,
                                  hipStream_t s) {
  if (rows <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  const int tiles_n = (int)((N + BN - 1) / BN);
  const int64_t g = ((rows + BM - 1) / BM) * tiles_n;
  if (g > 0x7fffffff || batch > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(gemm_nn_kernel, dim3((unsigned)g, (unsigned)batch), dim3(THREADS), 0, s, A, lda,
                     B, ldb, rows, K, N, alpha, C, ldc, 0, tiles_n, g, 0, stride_a, stride_b, stride_c);
  return hipGetLastError();
}

hipError_t launch_gemm_nn_acc(const double *A, int64_t lda, const double *B, int64_t ldb,
                              int64_t rows, int64_t K, int64_t N, double alpha, double *C,
                              int64_t ldc, hipStream_t s) {
  if (rows <= 0 || N <= 0 || K <= 0) return hipSuccess;
  const int tiles_n = (int)((N + BN - 1) / BN);
  const int64_t g = ((rows + BM - 1) / BM) * tiles_n;
  if (g > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(gemm_nn_kernel, dim3((unsigned)g), dim3(THREADS), 0, s, A, lda, B, ldb,
                     rows, K, N, alpha, C, ldc, 0, tiles_n, g, 1, 0, 0, 0);
  return hipGetLastError();
}

hipError_t launch_gemm_tn_general(const double *A, int64_t lda, const double *B, int64_t ldb,
                                  int64_t K, int64_t M, int64_t N, double *C, int64_t ldc,
                                  double *partial, int splits, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int tiles_n = (int)((N + BN - 1) / BN);
  const int64_t tiles = ((M + BM - 1) / BM) * tiles_n;
  int64_t kps = (K + splits - 1) / splits;
  kps = (kps + BK - 1) / BK * BK;
  hipLaunchKernelGGL(gemm_tn_general_kernel, dim3((unsigned)tiles, (unsigned)splits), dim3(THREADS),
                     0, s, A, lda, B, ldb, K, M, N, partial, kps, tiles_n);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned g = (unsigned)std::min<int64_t>((M * N + 255) / 256, 4096);
  hipLaunchKernelGGL(reduce_general_kernel, dim3(g), dim3(256), 0, s, partial, splits, M, N, C, ldc);
  return hipGetLastError();
}

}  // namespace ttdft
