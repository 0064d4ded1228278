// Internal declarations shared by the host entry points and the HIP kernel
// launchers of libttdft.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include "ttdft.h"

namespace ttdft {

inline size_t dtype_size(ttdft_dtype t) {
  return t == TTDFT_F64 ? 8 : t == TTDFT_F32 ? 4 : 2;
}
// bytes of one tile value (BF16_SPLIT: a pair of bf16)
inline size_t tile_value_bytes(ttdft_dtype t) { return t == TTDFT_BF16_SPLIT ? 4 : dtype_size(t); }

constexpr int kTile = 64;                    // rows per lattice block (4x4x4)
constexpr int64_t kTileElems = 64 * 64;

// Positions of entry (i, j) inside a stored 64x64 tile.
// FP64 / FP32 tiles: the 16x4 fragment order of the 16x16x4 matrix-core ops;
// fragment (j/4, i/16) is 64 consecutive values, lane l taking value l
// (row i%16 = l%16, column j%4 = l/16).
__host__ __device__ inline int tile_pos_16x4(int i, int j) {
  return 64 * (4 * (j >> 2) + (i >> 4)) + 16 * (j & 3) + (i & 15);
}
// BF16 tiles (and each half of a BF16_SPLIT tile): the 16x32 fragment order of
// the 16x16x32 bf16 op; fragment (j/32, i/16) is 512 consecutive values and
// lane l holds row i%16 = l%16, columns 8(l/16) .. 8(l/16)+7 of it as 16 bytes.
__host__ __device__ inline int tile_pos_16x32(int i, int j) {
  return 512 * (4 * (j >> 5) + (i >> 4)) + 8 * ((i & 15) + 16 * ((j & 31) >> 3)) + (j & 7);
}
__host__ __device__ inline int tile_pos(ttdft_dtype t, int i, int j) {
  return (t == TTDFT_BF16 || t == TTDFT_BF16_SPLIT) ? tile_pos_16x32(i, j) : tile_pos_16x4(i, j);
}

// The step kernel addresses a 64-row panel of a dense block with 32-bit byte
// offsets: 64 * ld * elt must fit in an int32.
inline bool step_ld_ok(int64_t ld, size_t elt) { return ld >= 0 && 64 * ld * (int64_t)elt <= 0x7fffffffLL; }

// ---- coefficient schedule of the scaled recurrence (Algorithm 1, Sec. 3.4):
// step k (k = 0 .. m-1) forms Y_{k+1} = alpha[k] (H - cI) Y_k - beta[k] Y_{k-1},
// beta[0] = 0.  alpha and beta hold m entries.
void cheb_coefficients(int m, double a, double b, double a0, double *c, double *alpha,
                       double *beta);

// ---- the filter's argument checks (no writes) and its m launches; work holds one
// rows x n_vec block (leading dimension n_vec) when m >= 2
ttdft_status filter_check(const ttdft_bsr *H, const void *X, int64_t ldx, const void *Y,
                          int64_t ldy, int64_t n_vec, int32_t m, double a, double b, double a0,
                          ttdft_dtype x_dtype);
ttdft_status filter_enqueue(const ttdft_bsr &H, const void *X, int64_t ldx, void *Y, int64_t ldy,
                            int64_t n_vec, int32_t m, double a, double b, double a0,
                            ttdft_dtype x_dtype, void *work, hipStream_t s);
// as filter_enqueue, the steps k < m - m_late with H_early and the last m_late with H_late
ttdft_status filter_enqueue_schedule(const ttdft_bsr &H_early, const ttdft_bsr &H_late, int32_t m_late,
                                     const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t n_vec,
                                     int32_t m, double a, double b, double a0, ttdft_dtype x_dtype,
                                     void *work, hipStream_t s);
// set the thread-local error string and return s
ttdft_status api_fail(ttdft_status s, const char *msg);
ttdft_status api_ok();

// ---- fused BSR SpMM + Chebyshev recurrence epilogue (one degree step)
hipError_t launch_cheb_step(const ttdft_bsr &H, const void *Yk, int64_t ldk, const void *Yp,
                            int64_t ldp, void *Yo, int64_t ldo, int64_t n_vec, double alpha,
                            double c, double beta, ttdft_dtype xt, hipStream_t s);

// ---- element-wise / layout kernels
hipError_t launch_cast(const void *src, ttdft_dtype st, int64_t lds, void *dst, ttdft_dtype dt,
                       int64_t ldd, int64_t rows, int64_t cols, hipStream_t s);
hipError_t launch_split_bf16(const double *src, int64_t n_tiles, void *dst, hipStream_t s);
// tile values from F64 / F32 (16x4 order) to F32 (16x4), BF16 or BF16_SPLIT (16x32 order)
hipError_t launch_convert_tiles(const void *src, ttdft_dtype st, int64_t n_tiles, void *dst,
                                ttdft_dtype dt, hipStream_t s);
// *count += number of NaN / Inf entries of a rows x cols block (count: device, cleared by the caller)
hipError_t launch_count_nonfinite(const void *A, ttdft_dtype dt, int64_t ld, int64_t rows,
                                  int64_t cols, unsigned long long *count, hipStream_t s);
hipError_t launch_gather_rows(const void *src, int64_t lds, void *dst, int64_t ldd,
                              int64_t rows_dst, int64_t cols, const int64_t *perm, size_t elt,
                              hipStream_t s);

// ---- FP64 dense kernels (MFMA)
// C[n x n] (ldc) = A^T B for A, B : rows x n (lda, ldb), summed over rows; when sym is set
// only the lower-triangular tiles are computed and mirrored.  partial: device scratch of
// splits * n * n doubles (split-K partial sums, reduced in a fixed order).
hipError_t launch_gemm_tn(const double *A, int64_t lda, const double *B, int64_t ldb,
                          int64_t rows, int64_t n, double *C, int64_t ldc, bool sym,
                          double *partial, int splits, hipStream_t s);
// as launch_gemm_tn; symmetrize writes (C + C^T)/2
hipError_t launch_gemm_tn_ex(const double *A, int64_t lda, const double *B, int64_t ldb,
                             int64_t rows, int64_t n, double *C, int64_t ldc, bool sym,
                             bool symmetrize, double *partial, int splits, hipStream_t s);
int gemm_tn_splits(int64_t rows, int64_t n, bool sym);
// C[rows x n] (ldc) = A[rows x n] (lda) * B[n x n] (ldb); when upper is set B is upper
// triangular and its zero blocks are skipped.
hipError_t launch_gemm_nn(const double *A, int64_t lda, const double *B, int64_t ldb,
                          int64_t rows, int64_t n, double *C, int64_t ldc, bool upper,
                          hipStream_t s);
// C[rows x N] = alpha * A[rows x K] B[K x N]
hipError_t launch_gemm_nn_ex(const double *A, int64_t lda, const double *B, int64_t ldb,
                             int64_t rows, int64_t K, int64_t N, double alpha, double *C,
                             int64_t ldc, bool upper, hipStream_t s);
hipError_t launch_clear_ints(int *p, int count, hipStream_t s);
// batch of C_b = alpha * A_b B_b (rows x K times K x N), A_b = A + b*stride_a etc.
hipError_t launch_gemm_nn_batched(const double *A, int64_t lda, int64_t stride_a, const double *B,
                                  int64_t ldb, int64_t stride_b, int64_t rows, int64_t K, int64_t N,
                                  double alpha, double *C, int64_t ldc, int64_t stride_c, int batch,
                                  hipStream_t s);
// C[rows x N] += alpha * A[rows x K] B[K x N]
hipError_t launch_gemm_nn_acc(const double *A, int64_t lda, const double *B, int64_t ldb,
                              int64_t rows, int64_t K, int64_t N, double alpha, double *C,
                              int64_t ldc, hipStream_t s);
// C[M x N] = A^T B, A: K x M, B: K x N, K split in `splits` (partial: splits*M*N doubles)
hipError_t launch_gemm_tn_general(const double *A, int64_t lda, const double *B, int64_t ldb,
                                  int64_t K, int64_t M, int64_t N, double *C, int64_t ldc,
                                  double *partial, int splits, hipStream_t s);
// C[M x N] += alpha * A^T B, A: K x M, B: K x N (small K, no split)
hipError_t launch_gemm_tn_acc(const double *A, int64_t lda, const double *B, int64_t ldb,
                              int64_t K, int64_t M, int64_t N, double alpha, double *C,
                              int64_t ldc, hipStream_t s);

// ---- small dense FP64 factorisations (device)
// In-place scaled Cholesky-QR core: given G (np x np, ld np) with Y^T Y in its
// n x n part, forms D = diag(G)^{1/2}, Gs = D^-1 G D^-1 + shift*I, Gs = R^T R, and
// writes Rinv = D^-1 R^-1 (upper).  info (device int) is set non-zero on breakdown.
hipError_t launch_chol_rinv(double *G, int64_t n, double *Rinv, double *scratch, int *info,
                            hipStream_t s, double shift = 0.0);
size_t chol_rinv_scratch_doubles(int64_t n);

hipError_t launch_symmetrize(double *A, int64_t n, int64_t lda, hipStream_t s);

// symmetric eigensolver; work sized by syev_work_bytes
size_t syev_work_bytes(int64_t n);
hipError_t run_syev(int64_t n, const double *A, int64_t lda, double *lambda, double *Z,
                    int64_t ldz, void *work, hipStream_t s, int *host_info);

// ---- adjoint helper: dH[t] (+)= coef * Abar[rowblock(t)] * B[colblock(t)]^T on the pattern
hipError_t launch_sddmm(const ttdft_bsr &H, const void *Abar, int64_t lda, const void *Bk,
                        int64_t ldb, int64_t n_vec, double coef, void *dH, const uint64_t *mask,
                        bool accumulate, ttdft_dtype xt, hipStream_t s,
                        const double *colw = nullptr, bool sym = false);

// ---- occupancies and density (FP64)
// mu with 2 sum_i f(lambda_i; mu) = n_electrons, f = Fermi-Dirac at kT; host_out = {mu, status}
hipError_t run_fermi_level(const double *lambda, int64_t n, double n_electrons, double kT, double *f,
                           double *scratch, hipStream_t s, double *mu, int *nonfinite);
hipError_t launch_electron_density(const double *Psi, int64_t ldp, const double *f, int64_t rows,
                                   int64_t n, double *rho, hipStream_t s);

// ---- Lanczos estimate of the top of the spectrum
// host_out: theta_max, theta_max + |beta_{k+1} s_k|, theta_max + beta_{k+1}
// Ritz residual norms || H psi_j - lambda_j psi_j || (FP64 H)
size_t residual_work_bytes(int64_t rows, int64_t n);
hipError_t run_ritz_residuals(const ttdft_bsr &H, const double *Psi, int64_t ldp,
                              const double *lambda, int64_t n, double *res, void *work,
                              hipStream_t s);
size_t lanczos_work_bytes(int64_t rows, int k);
// host_out: theta_max, estimate, safeguarded bound, theta_min; *breakdown set when the
// Lanczos process found an invariant subspace (bounds then widened to Gershgorin's)
hipError_t run_lanczos_bound(const ttdft_bsr &H, const int64_t *perm, int k, uint64_t seed,
                             void *work, hipStream_t s, double host_out[4], int *breakdown);

}  // namespace ttdft
