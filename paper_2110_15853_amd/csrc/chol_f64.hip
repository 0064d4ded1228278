// Scaled Cholesky factorisation of a Gram matrix and the upper-triangular
// factor M = D^{-1} R^{-1} used by Cholesky-QR (step 2 of Algorithm 1 carried
// out as Cholesky-QR):
//     D = diag(G)^{1/2},  D^{-1} G D^{-1} = R^T R,  Y D^{-1} R^{-1} = Y M  has
//     orthonormal columns.
// The n x n problem is padded to np = 64*ceil(n/64) with an identity block so
// every tile is a full 64x64 block.  Right-looking blocked factorisation with
// 64-wide panels (one wave factors the diagonal block and inverts it; the panel
// below and the trailing lower triangle are updated tile by tile), then L^{-1}
// by recursive doubling: with the inverses X11, X22 of two adjacent diagonal
// ranges known, the coupling block of the inverse of [[L11, 0], [L21, L22]] is
// X21 = -X22 (L21 X11), formed for all pairs of a level by two batched
// matrix-core products (ranges of 1, 2, 4, ... blocks).  Breakdown (a
// non-positive or non-finite pivot) sets *info and the factorisation kernels
// return immediately.
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
        if (!isfinite(g)) atomicOr(info + 1, 1);   // a NaN or Inf in the block
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

// Factor the diagonal block p with four waves; write L_pp (lower) into G and
// L_pp^{-1} into X.  The block sits in LDS row-major, lane i of every wave on
// row i.  Step j (a rolled loop): lanes i > j of wave 0 form l_ij = a_ij /
// sqrt(a_jj) in place; after a barrier every wave applies a_ik -= l_ij l_kj to
// the columns k > j it owns (wave w: columns 16w .. 16w+15), l_kj read with the
// same address by every lane, and a second barrier closes the step.  Then wave 0
// has lane c hold column c of the identity in registers and eliminate with the
// factor's columns: x_j = b_j / l_jj, b_k -= l_kj x_j (k > j), leaving column c
// of L^{-1} (unrolled; a scheduling barrier between steps bounds the register
// use).
__global__ __launch_bounds__(256) void potrf_diag_kernel(double *G, int64_t np, int p, double *X,
                                                         int *info) {
  if (*info) return;
  __shared__ double La[T][T + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double *Gp = G + (int64_t)p * T * np + (int64_t)p * T;
  for (int r = wv; r < T; r += 4) La[r][lane] = Gp[r * np + lane];   // coalesced rows
  __syncthreads();
  int bad = 0;
  for (int j = 0; j < T; ++j) {
    double piv = La[j][j];                  // the same value in every lane
    if (!(piv > 0.0) || !isfinite(piv)) {
      if (!bad) bad = p * T + j + 1;
      piv = 1.0;
    }
    const double ljj = sqrt(piv);
    if (wv == 0) {
      if (lane > j) La[lane][j] = La[lane][j] / ljj;
      if (lane == j) La[j][j] = ljj;
    }
    __syncthreads();
    // trailing update of this wave's 16 columns in chunks of 8: all reads of a
    // chunk, then the products (kept only for columns k > j; entries above the
    // diagonal are updated too but never read), then the writes
    const double l = lane > j ? La[lane][j] : 0.0;
    for (int kc = max(16 * wv, (j + 1) & ~7); kc < 16 * wv + 16; kc += 8) {
      double lk[8], ak[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        lk[u] = La[kc + u][j];
        ak[u] = La[lane][kc + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double v = fma(-l, lk[u], ak[u]);
        ak[u] = kc + u > j ? v : ak[u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) La[lane][kc + u] = ak[u];
    }
    __syncthreads();
  }
  if (bad) {
    if (threadIdx.x == 0) atomicCAS(info, 0, bad);
    return;
  }
  if (wv == 0) {
    double b[T];
#pragma unroll
    for (int k = 0; k < T; ++k) b[k] = k == lane ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < T; ++j) {
      const double x = b[j] / La[j][j];
      b[j] = x;
#pragma unroll
      for (int k = j + 1; k < T; ++k) b[k] = fma(-La[k][j], x, b[k]);
      __builtin_amdgcn_sched_barrier(0);
    }
    double *Xp = X + (int64_t)p * T * np + (int64_t)p * T;
#pragma unroll
    for (int i = 0; i < T; ++i) Xp[(int64_t)i * np + lane] = b[i];   // lane = column: coalesced
  }
  for (int r = wv; r < T; r += 4) Gp[r * np + lane] = lane <= r ? La[r][lane] : 0.0;
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

// largest product block W = L21 X11 of the doubling levels (doubles)
static size_t doubling_w_doubles(int nb) {
  size_t w = 0;
  for (int s = 1; s < nb; s *= 2) {
    const int full = nb / (2 * s), mid = 2 * s * full + s;
    w = std::max(w, (size_t)full * (size_t)(s * T) * (size_t)(s * T));
    if (mid < nb) w = std::max(w, (size_t)((nb - mid) * T) * (size_t)(s * T));
  }
  return w;
}

size_t chol_rinv_scratch_doubles(int64_t n) {
  const int64_t np = (n + T - 1) / T * T;
  return (size_t)np * np + (size_t)np + doubling_w_doubles((int)(np / T));   // X, d, W
}

// G: np x np (np = padded n, ld np) holding Y^T Y in its n x n part; Rinv: np x np.
hipError_t launch_chol_rinv(double *G, int64_t n, double *Rinv, double *scratch, int *info,
                            hipStream_t s, double shift) {
  const int64_t np = (n + T - 1) / T * T;
  const int nb = (int)(np / T);
  double *X = scratch, *d = scratch + np * np, *W = d + np;
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
  // L^{-1} by doubling: after level s every aligned range of 2s blocks is inverted
  hipError_t e;
  for (int sb = 1; sb < nb; sb *= 2) {
    const int64_t S = (int64_t)sb * T, step = 2 * S * np + 2 * S;   // pair stride (elements)
    const int full = nb / (2 * sb);
    if (full > 0) {
      // W_b = L21_b X11_b, then X21_b = -X22_b W_b
      if ((e = launch_gemm_nn_batched(G + S * np, np, step, X, np, step, S, S, S, 1.0, W, S, S * S,
                                      full, s)) != hipSuccess) return e;
      if ((e = launch_gemm_nn_batched(X + S * np + S, np, step, W, S, S * S, S, S, S, -1.0,
                                      X + S * np, np, step, full, s)) != hipSuccess) return e;
    }
    const int64_t lo = 2 * (int64_t)sb * full, mid = lo + sb;     // a shorter last pair
    if (mid < nb) {
      const int64_t S2 = (nb - mid) * T, L0 = lo * T, M0 = mid * T;
      if ((e = launch_gemm_nn_batched(G + M0 * np + L0, np, 0, X + L0 * np + L0, np, 0, S2, S, S,
                                      1.0, W, S, 0, 1, s)) != hipSuccess) return e;
      if ((e = launch_gemm_nn_batched(X + M0 * np + M0, np, 0, W, S, 0, S2, S2, S, -1.0,
                                      X + M0 * np + L0, np, 0, 1, s)) != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(form_m_kernel, dim3(grid_for(np * np)), dim3(256), 0, s, X, d, np, Rinv, info);
  return hipGetLastError();
}

}  // namespace ttdft
