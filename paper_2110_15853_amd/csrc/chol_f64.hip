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
#include <utility>

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

// the value `v` of lane `src` in every lane (src wave-uniform)
__device__ inline double lane_value(double v, int src) {
  const long long b = __builtin_bit_cast(long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), src);
  return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

constexpr int PW = 16;   // panel width of the diagonal-block factorisation

// column step J of a panel (columns c0 .. c0+PW-1) factored by one wave: lane i
// holds row i of the panel in a[]; the pivot and the multipliers L[c0+k][c0+J]
// reach every lane by readlane (rows above the panel update entries above the
// diagonal, which are never read)
template <int J>
__device__ __forceinline__ void panel_column(double (&a)[PW], int lane, int c0, int p, int &bad) {
  double piv = lane_value(a[J], c0 + J);
  if (!(piv > 0.0) || !isfinite(piv)) {
    if (!bad) bad = p * T + c0 + J + 1;
    piv = 1.0;
  }
  const double ljj = sqrt(piv);
  a[J] = lane > c0 + J ? a[J] / ljj : (lane == c0 + J ? ljj : a[J]);
#pragma unroll
  for (int k = J + 1; k < PW; ++k) a[k] = fma(-a[J], lane_value(a[J], c0 + k), a[k]);
}
template <int... J>
__device__ __forceinline__ void panel_columns(std::integer_sequence<int, J...>, double (&a)[PW],
                                              int lane, int c0, int p, int &bad) {
  (panel_column<J>(a, lane, c0, p, bad), ...);
}

// Factor the diagonal block p with four waves; write L_pp (lower, zeros above)
// into G and L_pp^{-1} into X.  The block sits in LDS row-major.
//  - factorisation in panels of PW columns: wave 0 factors a panel with row i in
//    lane i's registers (no barrier inside the panel), then all four waves apply
//    the panel's rank-PW update to the lower triangle of the trailing block (two
//    barriers per panel);
//  - inverse by blocks: the four 16x16 diagonal blocks are inverted by forward
//    substitution, one per wave, then the coupling blocks of the inverse of
//    [[L11, 0], [L21, L22]] follow as X21 = -X22 (L21 X11), first for the two
//    32x32 halves, then for the whole block.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double *G, int64_t np, int p, double *X,
                                                         int *info) {
  if (*info) return;
  __shared__ double La[T][T + 1], sX[T][T + 1], sW[T][T + 1];
  __shared__ int s_bad;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double *Gp = G + (int64_t)p * T * np + (int64_t)p * T;
  for (int r = wv; r < T; r += 4) {
    La[r][lane] = Gp[r * np + lane];   // coalesced rows
    sX[r][lane] = 0.0;
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int c0 = 0; c0 < T; c0 += PW) {
    if (wv == 0) {
      double a[PW];
#pragma unroll
      for (int k = 0; k < PW; ++k) a[k] = La[lane][c0 + k];
      int bad = 0;
      panel_columns(std::make_integer_sequence<int, PW>{}, a, lane, c0, p, bad);
#pragma unroll
      for (int k = 0; k < PW; ++k) La[lane][c0 + k] = a[k];
      if (lane == 0 && bad && !s_bad) s_bad = bad;
    }
    __syncthreads();
    // rank-PW update of the lower triangle of the trailing block: row i in lane
    // i, columns t0 + wv, t0 + wv + 4, ... <= i
    const int t0 = c0 + PW, i = lane;
    if (i >= t0) {
      double li[PW];
#pragma unroll
      for (int j = 0; j < PW; ++j) li[j] = La[i][c0 + j];
      for (int k = t0 + wv; k <= i; k += 4) {
        double s = La[i][k];
#pragma unroll
        for (int j = 0; j < PW; ++j) s = fma(-li[j], La[k][c0 + j], s);
        La[i][k] = s;
      }
    }
    __syncthreads();
  }
  const int bad = s_bad;
  if (bad) {
    if (tid == 0) atomicCAS(info, 0, bad);
    return;
  }
  // inverse of the four 16x16 diagonal blocks, block wv in wave wv, lane = column
  if (lane < 16) {
    const int o = 16 * wv;
    double b[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) b[k] = k == lane ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const double x = b[j] / La[o + j][o + j];
      b[j] = x;
#pragma unroll
      for (int k = j + 1; k < 16; ++k) b[k] = fma(-La[o + k][o + j], x, b[k]);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) sX[o + k][o + lane] = b[k];
  }
  __syncthreads();
  // coupling blocks: halves of S = 16 (blocks (0,1) and (2,3)), then S = 32
  for (int S = 16; S < T; S *= 2) {
    const int pairs = T / (2 * S), per = S * S;            // entries of one coupling block
    // W = L21 X11 (X11 lower: terms m >= c)
    for (int e = tid; e < pairs * per; e += 256) {
      const int q = e / per, r = (e % per) / S, c = e % S, o = 2 * S * q;
      double w = 0.0;
      for (int m = c; m < S; ++m) w = fma(La[o + S + r][o + m], sX[o + m][o + c], w);
      sW[o + S + r][o + c] = w;
    }
    __syncthreads();
    // X21 = -X22 W (X22 lower: terms m <= r)
    for (int e = tid; e < pairs * per; e += 256) {
      const int q = e / per, r = (e % per) / S, c = e % S, o = 2 * S * q;
      double x = 0.0;
      for (int m = 0; m <= r; ++m) x = fma(sX[o + S + r][o + S + m], sW[o + S + m][o + c], x);
      sX[o + S + r][o + c] = -x;
    }
    __syncthreads();
  }
  double *Xp = X + (int64_t)p * T * np + (int64_t)p * T;
  for (int r = wv; r < T; r += 4) {
    Xp[(int64_t)r * np + lane] = sX[r][lane];               // lane = column: coalesced
    Gp[r * np + lane] = lane <= r ? La[r][lane] : 0.0;
  }
}

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
