// Ritz residual norms res_j = || H psi_j - lambda_j psi_j ||_2 of the output of
// the Rayleigh-Ritz step, the quantity whose size decides when the subspace
// iteration of Algorithm 1 (Sec. 3.4) has converged.  H Psi comes from the fused
// step kernel (alpha = 1, c = 0, beta = 0); the column sums of squares are
// formed per chunk of rows (one thread per column, coalesced rows) and the
// chunk partials summed in a fixed order, so the result is deterministic.
#include <cmath>

#include "ttdft_internal.h"

namespace ttdft {
namespace {

constexpr int RES_THREADS = 256;
constexpr int64_t RES_ROWS = 2048;   // rows per chunk

__global__ __launch_bounds__(RES_THREADS) void residual_partial_kernel(
    const double *__restrict__ W, int64_t ldw, const double *__restrict__ Psi, int64_t ldp,
    const double *__restrict__ lambda, int64_t rows, int64_t n, double *__restrict__ partial) {
  const int64_t j = (int64_t)blockIdx.x * RES_THREADS + threadIdx.x;
  if (j >= n) return;
  const int64_t r0 = (int64_t)blockIdx.y * RES_ROWS, r1 = min(rows, r0 + RES_ROWS);
  const double lam = lambda[j];
  double acc = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double d = W[r * ldw + j] - lam * Psi[r * ldp + j];
    acc = fma(d, d, acc);
  }
  partial[(int64_t)blockIdx.y * n + j] = acc;
}

__global__ __launch_bounds__(RES_THREADS) void residual_final_kernel(const double *__restrict__ partial,
                                                                     int64_t chunks, int64_t n,
                                                                     double *__restrict__ res) {
  const int64_t j = (int64_t)blockIdx.x * RES_THREADS + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int64_t c = 0; c < chunks; ++c) s += partial[c * n + j];
  res[j] = sqrt(s);
}

}  // namespace

size_t residual_work_bytes(int64_t rows, int64_t n) {
  const int64_t chunks = (rows + RES_ROWS - 1) / RES_ROWS;
  return (size_t)(rows * n + chunks * n) * sizeof(double);
}

// work: H Psi (rows x n, ld n), then chunks x n partial sums
hipError_t run_ritz_residuals(const ttdft_bsr &H, const double *Psi, int64_t ldp,
                              const double *lambda, int64_t n, double *res, void *work,
                              hipStream_t s) {
  const int64_t rows = H.n_block_rows * 64, chunks = (rows + RES_ROWS - 1) / RES_ROWS;
  double *W = (double *)work, *partial = W + rows * n;
  hipError_t e = launch_cheb_step(H, Psi, ldp, nullptr, 0, W, n, n, 1.0, 0.0, 0.0, TTDFT_F64, s);
  if (e != hipSuccess) return e;
  const unsigned gx = (unsigned)((n + RES_THREADS - 1) / RES_THREADS);
  if (chunks > 65535) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(residual_partial_kernel, dim3(gx, (unsigned)chunks), dim3(RES_THREADS), 0, s,
                     W, n, Psi, ldp, lambda, rows, n, partial);
  hipLaunchKernelGGL(residual_final_kernel, dim3(gx), dim3(RES_THREADS), 0, s, partial, chunks, n,
                     res);
  return hipGetLastError();
}

}  // namespace ttdft
