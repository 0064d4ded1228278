// Scaled Cholesky factorisation of a Gram matrix and the upper-triangular
// factor M = D^{-1} R^{-1} used by Cholesky-QR (step 2 of Algorithm 1 carried
// out as Cholesky-QR):
//     D = diag(G)^{1/2},  D^{-1} G D^{-1} = R^T R,  Y D^{-1} R^{-1} = Y M  has
//     orthonormal columns.
// The n x n problem is padded to np = 64*ceil(n/64) with an identity block so
// every tile is a full 64x64 block.  Right-looking blocked factorisation with
// 64-wide panels (one work-group factors the diagonal block in LDS and inverts
// it; the panel below and the trailing lower triangle are updated tile by tile),
// then L^{-1} by block forward substitution.  Breakdown (a non-positive or
// non-finite pivot) sets *info and every later kernel returns immediately.
#include "ttdft_internal.h"

namespace ttdft {
namespace {

constexpr int T = 64;

// acc (rows 4*ty+r, cols 4*tx+c) += opA(A) opB(B) for 64x64 tiles
__device__ inline void tile_mac(const double *A, int64_t lda, bool ta, const double *B,
                                int64_t ldb, bool tb, double (&acc)[4][4], double (*sA)[T + 1],
                                double (*sB)[T + 1]) {
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + 256 * q, r = idx >> 6, c = idx & 63;
    const double va = A[r * lda + c], vb = B[r * ldb + c];   // coalesced global reads
    if (ta) sA[c][r] = va; else sA[r][c] = va;                // sA[m][k]
    if (tb) sB[c][r] = vb; else sB[r][c] = vb;                // sB[k][n]
  }
  __syncthreads();
  for (int k = 0; k < T; ++k) {
    double a[4], b[4];
    for (int r = 0; r < 4; ++r) a[r] = sA[4 * ty + r][k];
    for (int c = 0; c < 4; ++c) b[c] = sB[k][4 * tx + c];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
  }
  __syncthreads();
}

__global__ void gram_scale_diag_kernel(const double *G, int64_t n, int64_t np, double *d,
                                       int *info) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < np; i += (int64_t)gridDim.x * 256) {
    if (i < n) {
      const double g = G[i * np + i];
      if (!(g > 0.0) || !isfinite(g)) {
        atomicCAS(info, 0, (int)(i + 1));
        d[i] = 1.0;
      } else {
        d[i] = sqrt(g);
      }
    } else {
      d[i] = 1.0;
    }
  }
}

// Gs = D^-1 G D^-1 (+ shift on the diagonal) on the n x n part, identity on the
// padding; X (the future L^{-1}) cleared.
__global__ void gram_scale_kernel(double *G, int64_t n, int64_t np, const double *d, double *X,
                                  double shift) {
  const int64_t total = np * np;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / np, j = e % np;
    double v;
    if (i < n && j < n) v = G[e] / (d[i] * d[j]) + (i == j ? shift : 0.0);
    else v = (i == j) ? 1.0 : 0.0;
    G[e] = v;
    X[e] = 0.0;
  }
}

// factor the diagonal block p in LDS; write L_pp (lower) into G and L_pp^{-1} into X
__global__ __launch_bounds__(256) void potrf_diag_kernel(double *G, int64_t np, int p, double *X,
                                                         int *info) {
  if (*info) return;
  __shared__ double a[T][T + 1];
  __shared__ double inv[T][T + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  double *Gp = G + (int64_t)p * T * np + (int64_t)p * T;
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + 256 * q, r = idx >> 6, c = idx & 63;
    a[r][c] = Gp[r * np + c];
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < T; ++j) {
    if (tid == 0) {
      const double piv = a[j][j];
      if (!(piv > 0.0) || !isfinite(piv)) {
        bad = p * T + j + 1;
        a[j][j] = 1.0;
      } else {
        a[j][j] = sqrt(piv);
      }
    }
    __syncthreads();
    const double ljj = a[j][j];
    if (tid > j && tid < T) a[tid][j] /= ljj;
    __syncthreads();
    // trailing update of the lower triangle: a[i][k] -= a[i][j] a[k][j], j < k <= i
    for (int idx = tid; idx < T * T; idx += 256) {
      const int i = idx >> 6, k = idx & 63;
      if (k > j && i >= k) a[i][k] -= a[i][j] * a[k][j];
    }
    __syncthreads();
  }
  if (bad) {
    if (tid == 0) atomicCAS(info, 0, bad);
    return;
  }
  // inverse of the lower factor, one column per thread (forward substitution)
  if (tid < T) {
    const int c = tid;
    for (int i = 0; i < T; ++i) inv[i][c] = 0.0;
    inv[c][c] = 1.0 / a[c][c];
    for (int i = c + 1; i < T; ++i) {
      double s = 0.0;
      for (int k = c; k < i; ++k) s += a[i][k] * inv[k][c];
      inv[i][c] = -s / a[i][i];
    }
  }
  __syncthreads();
  double *Xp = X + (int64_t)p * T * np + (int64_t)p * T;
  for (int q = 0; q < 16; ++q) {
    const int idx = tid + 256 * q, r = idx >> 6, c = idx & 63;
    Gp[r * np + c] = (c <= r) ? a[r][c] : 0.0;
    Xp[r * np + c] = inv[r][c];
  }
}

// L_ip = A_ip L_pp^{-T} for every block row i > p (one work-group each)
__global__ __launch_bounds__(256) void trsm_panel_kernel(double *G, int64_t np, int p,
                                                         const double *X, const int *info) {
  if (*info) return;
  __shared__ double sA[T][T + 1], sB[T][T + 1];
  const int i = p + 1 + blockIdx.x;
  double acc[4][4] = {};
  double *Aip = G + (int64_t)i * T * np + (int64_t)p * T;
  const double *Lpp_inv = X + (int64_t)p * T * np + (int64_t)p * T;
  tile_mac(Aip, np, false, Lpp_inv, np, true, acc, sA, sB);
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) Aip[(4 * ty + r) * np + 4 * tx + c] = acc[r][c];
}

// A_ij -= L_ip L_jp^T for p < j <= i (lower trailing tiles)
__global__ __launch_bounds__(256) void syrk_update_kernel(double *G, int64_t np, int p, int nb,
                                                          const int *info) {
  if (*info) return;
  __shared__ double sA[T][T + 1], sB[T][T + 1];
  // linear index over pairs (i, j) with p < j <= i < nb
  int t = blockIdx.x, i = p + 1, j;
  while (t >= i - p) { t -= i - p; ++i; }
  j = p + 1 + t;
  if (i >= nb) return;
  double acc[4][4] = {};
  const double *Lip = G + (int64_t)i * T * np + (int64_t)p * T;
  const double *Ljp = G + (int64_t)j * T * np + (int64_t)p * T;
  tile_mac(Lip, np, false, Ljp, np, true, acc, sA, sB);
  double *Aij = G + (int64_t)i * T * np + (int64_t)j * T;
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) Aij[(4 * ty + r) * np + 4 * tx + c] -= acc[r][c];
}

// block row i of X = L^{-1}: X_ij = -L_ii^{-1} sum_{k=j}^{i-1} L_ik X_kj, all j < i
__global__ __launch_bounds__(256) void trinv_row_kernel(const double *G, int64_t np, int i,
                                                        double *X, const int *info) {
  if (*info) return;
  __shared__ double sA[T][T + 1], sB[T][T + 1];
  const int j = blockIdx.x;
  double s[4][4] = {};
  for (int k = j; k < i; ++k)
    tile_mac(G + (int64_t)i * T * np + (int64_t)k * T, np, false,
             X + (int64_t)k * T * np + (int64_t)j * T, np, false, s, sA, sB);
  // write S into LDS, then X_ij = -Linv_ii * S
  const int ty = threadIdx.x >> 4, tx = threadIdx.x & 15;
  __shared__ double sS[T][T + 1];
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) sS[4 * ty + r][4 * tx + c] = s[r][c];
  __syncthreads();
  double out[4][4] = {};
  const double *Lii_inv = X + (int64_t)i * T * np + (int64_t)i * T;
  for (int q = 0; q < 16; ++q) {
    const int idx = threadIdx.x + 256 * q, r = idx >> 6, c = idx & 63;
    sA[r][c] = Lii_inv[r * np + c];
  }
  __syncthreads();
  for (int k = 0; k < T; ++k)
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 4; ++c) out[r][c] = fma(sA[4 * ty + r][k], sS[k][4 * tx + c], out[r][c]);
  double *Xij = X + (int64_t)i * T * np + (int64_t)j * T;
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) Xij[(4 * ty + r) * np + 4 * tx + c] = -out[r][c];
}

// M[i][j] = X[j][i] / d_i for i <= j, 0 below the diagonal (M = D^{-1} L^{-T})
__global__ void form_m_kernel(const double *X, const double *d, int64_t np, double *M,
                              const int *info) {
  if (*info) return;
  const int64_t total = np * np;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / np, j = e % np;
    M[e] = (i <= j) ? X[j * np + i] / d[i] : 0.0;
  }
}

inline unsigned grid_for(int64_t work) {
  const int64_t g = (work + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

}  // namespace

size_t chol_rinv_scratch_doubles(int64_t n) {
  const int64_t np = (n + T - 1) / T * T;
  return (size_t)np * np + (size_t)np;   // X = L^{-1} and d
}

// G: np x np (np = padded n, ld np) holding Y^T Y in its n x n part; Rinv: np x np.
hipError_t launch_chol_rinv(double *G, int64_t n, double *Rinv, double *scratch, int *info,
                            hipStream_t s, double shift) {
  const int64_t np = (n + T - 1) / T * T;
  const int nb = (int)(np / T);
  double *X = scratch, *d = scratch + np * np;
  hipLaunchKernelGGL(gram_scale_diag_kernel, dim3(grid_for(np)), dim3(256), 0, s, G, n, np, d, info);
  hipLaunchKernelGGL(gram_scale_kernel, dim3(grid_for(np * np)), dim3(256), 0, s, G, n, np, d, X, shift);
  for (int p = 0; p < nb; ++p) {
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, s, G, np, p, X, info);
    if (p + 1 < nb) {
      hipLaunchKernelGGL(trsm_panel_kernel, dim3(nb - p - 1), dim3(256), 0, s, G, np, p, X, info);
      const int pairs = (nb - p - 1) * (nb - p) / 2;
      hipLaunchKernelGGL(syrk_update_kernel, dim3(pairs), dim3(256), 0, s, G, np, p, nb, info);
    }
  }
  for (int i = 1; i < nb; ++i)
    hipLaunchKernelGGL(trinv_row_kernel, dim3(i), dim3(256), 0, s, G, np, i, X, info);
  hipLaunchKernelGGL(form_m_kernel, dim3(grid_for(np * np)), dim3(256), 0, s, X, d, np, Rinv, info);
  return hipGetLastError();
}

}  // namespace ttdft
