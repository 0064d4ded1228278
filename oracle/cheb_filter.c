/* FP64 CPU oracle of the degree-m Chebyshev filter of Algorithm 1, step 1
 * (Sec. 3.4), in plain C with OpenMP:
 *
 *     Y = T_m((H - cI)/e) X / T_m(tau),  e = (b - a)/2, c = (b + a)/2, tau = (a0 - c)/e,
 *
 * with H in CSR (natural row order, FP64) and X, Y row-major n_rows x n_vec.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests pin it against the closed form and the
 * benchmark times it as the CPU baseline on the host's cores; the GPU library
 * never links or calls it, and it shares no code with it.
 *
 * The definition is computed as written: the matrix Chebyshev polynomial of
 * Hs = (H - cI)/e by its defining recurrence T_0 = I, T_1 = Hs,
 * T_{k+1} = 2 Hs T_k - T_{k-1}, applied to X, then divided by the scalar
 * T_m(tau) (the same recurrence on tau).  The columns are independent, so the
 * threads take blocks of `blk` columns, each block run through the recurrence on
 * its own in three n_rows x blk buffers.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

/* Hs V for a block of w columns: out[i][j] = (sum_k H[i][k] V[k][j] - c V[i][j]) / e */
static void apply_hs(int64_t n_rows, const int64_t *rowptr, const int32_t *col, const double *val,
                     double c, double e, const double *V, double *out, int w) {
  for (int64_t i = 0; i < n_rows; ++i) {
    double acc[64];
    for (int j = 0; j < w; ++j) acc[j] = 0.0;
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
      const double h = val[p];
      const double *v = V + (int64_t)col[p] * w;
      for (int j = 0; j < w; ++j) acc[j] += h * v[j];
    }
    for (int j = 0; j < w; ++j) out[i * w + j] = (acc[j] - c * V[i * w + j]) / e;
  }
}

/* 0 on success, -1 for invalid arguments, -2 when a work buffer cannot be allocated */
int oracle_cheb_filter_csr(int64_t n_rows, const int64_t *rowptr, const int32_t *col,
                           const double *val, const double *X, int64_t ldx, double *Y,
                           int64_t ldy, int64_t n_vec, int m, double a, double b, double a0,
                           int blk, int threads) {
  if (n_rows < 1 || n_vec < 1 || m < 1 || blk < 1 || blk > 64 || ldx < n_vec || ldy < n_vec ||
      !(a0 < a && a < b))
    return -1;
  const double e = (b - a) / 2.0, c = (b + a) / 2.0, tau = (a0 - c) / e;
  double t_prev = 1.0, t = tau;                       /* T_0(tau), T_1(tau) */
  for (int k = 1; k < m; ++k) {
    const double t_next = 2.0 * tau * t - t_prev;
    t_prev = t;
    t = t_next;
  }
  const double tm = t;                                /* T_m(tau) */
  const int64_t n_blocks = (n_vec + blk - 1) / blk;
  int status = 0;
  if (threads > 0) omp_set_num_threads(threads);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t bi = 0; bi < n_blocks; ++bi) {
    const int64_t j0 = bi * blk;
    const int w = (int)(n_vec - j0 < blk ? n_vec - j0 : blk);
    double *zp = (double *)malloc(sizeof(double) * n_rows * w);
    double *z = (double *)malloc(sizeof(double) * n_rows * w);
    double *zn = (double *)malloc(sizeof(double) * n_rows * w);
    if (!zp || !z || !zn) {
#pragma omp atomic write
      status = -2;
    } else {
      for (int64_t i = 0; i < n_rows; ++i)
        for (int j = 0; j < w; ++j) zp[i * w + j] = X[i * ldx + j0 + j];     /* T_0 X */
      apply_hs(n_rows, rowptr, col, val, c, e, zp, z, w);                   /* T_1 X */
      for (int k = 1; k < m; ++k) {                                        /* T_{k+1} X */
        apply_hs(n_rows, rowptr, col, val, c, e, z, zn, w);
        for (int64_t q = 0; q < n_rows * w; ++q) zn[q] = 2.0 * zn[q] - zp[q];
        double *tmp = zp;
        zp = z;
        z = zn;
        zn = tmp;
      }
      for (int64_t i = 0; i < n_rows; ++i)
        for (int j = 0; j < w; ++j) Y[i * ldy + j0 + j] = z[i * w + j] / tm;
    }
    free(zp);
    free(z);
    free(zn);
  }
  return status;
}
