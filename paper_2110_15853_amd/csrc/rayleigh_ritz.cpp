// Host side of steps 2-5 of Algorithm 1 (Sec. 3.4), all in FP64 on the GPU:
// Cholesky-QR twice with column scaling, the projection X_F^T (H X_F) with the
// fused BSR kernel and a matrix-core GEMM, the dense eigensolve and the
// rotation Psi = X_F Q.  The fused entry point keeps X_F = Q1 M2 implicit (the
// projection and the rotation go through the second pass's factor M2).
// Validation runs before any device work.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "ttdft_internal.h"

using namespace ttdft;

namespace ttdft {
// defined in api.cpp
ttdft_status api_fail(ttdft_status s, const char *msg);
ttdft_status api_ok();
}

namespace {

thread_local char g_msg[256];

ttdft_status failf(ttdft_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof g_msg, fmt, ap);
  va_end(ap);
  return api_fail(s, g_msg);
}

ttdft_status hip_fail(hipError_t e, const char *what) {
  return failf(TTDFT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool valid_dtype(int t) { return t == TTDFT_F64 || t == TTDFT_F32 || t == TTDFT_BF16; }

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  if (!a || !b || !na || !nb) return false;
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}
size_t block_bytes(int64_t rows, int64_t ld, int64_t cols, size_t elt) {
  return rows <= 0 || cols <= 0 ? 0 : (size_t)((rows - 1) * ld + cols) * elt;
}

// workspace of the Cholesky-QR core: W (rows x n, ld n), G and M (np x np),
// factorisation scratch, split-K partials, info flags
struct QrLayout {
  int64_t np;
  int splits;
  size_t w, g, m, chol, partial, info, total;
};
QrLayout qr_layout(int64_t rows, int64_t n) {
  QrLayout L;
  L.np = (n + 63) / 64 * 64;
  L.splits = gemm_tn_splits(rows, n, true);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.w = take((size_t)rows * n * 8);
  L.g = take((size_t)L.np * L.np * 8);
  L.m = take((size_t)L.np * L.np * 8);
  L.chol = take(chol_rinv_scratch_doubles(n) * 8);
  L.partial = take((size_t)L.splits * n * n * 8);
  L.info = take(16);
  L.total = off;
  return L;
}

// one Cholesky-QR pass: dst = src D^{-1} R^{-1}, with D^{-1} G D^{-1} + shift I = R^T R
// the factor of one pass alone: M = D^{-1} R^{-1} (np x np, ld np) in work + L.m
hipError_t cholqr_factor(const double *src, int64_t lds, int64_t rows, int64_t n, double shift,
                         char *work, const QrLayout &L, hipStream_t s) {
  double *G = (double *)(work + L.g), *M = (double *)(work + L.m);
  double *chol = (double *)(work + L.chol), *partial = (double *)(work + L.partial);
  int *info = (int *)(work + L.info);
  hipError_t e;
  if ((e = launch_gemm_tn(src, lds, src, lds, rows, n, G, L.np, true, partial, L.splits, s))) return e;
  return launch_chol_rinv(G, n, M, chol, info, s, shift);
}

hipError_t cholqr_pass(const double *src, int64_t lds, double *dst, int64_t ldd, int64_t rows,
                       int64_t n, double shift, char *work, const QrLayout &L, hipStream_t s) {
  hipError_t e = cholqr_factor(src, lds, rows, n, shift, work, L, s);
  if (e != hipSuccess) return e;
  return launch_gemm_nn_ex(src, lds, (const double *)(work + L.m), L.np, rows, n, n, 1.0, dst, ldd,
                           true, s);
}

// FP64 copy of Y into Q when Y is not FP64 (the orthonormalisation is FP64)
const double *fp64_source(const void *Y, int64_t ldy, ttdft_dtype ydt, int64_t rows, int64_t n,
                          double *Q, int64_t ldq, int64_t *lds, hipStream_t s, hipError_t *e) {
  *e = hipSuccess;
  if (ydt == TTDFT_F64) {
    *lds = ldy;
    return (const double *)Y;
  }
  *e = launch_cast(Y, ydt, ldy, Q, TTDFT_F64, ldq, rows, n, s);
  *lds = ldq;
  return Q;
}

// Y (any dtype) -> Q (FP64) = Cholesky-QR applied twice.  Enqueues only.
hipError_t cholqr2_enqueue(const void *Y, int64_t ldy, ttdft_dtype ydt, int64_t rows, int64_t n,
                           double *Q, int64_t ldq, char *work, const QrLayout &L, hipStream_t s) {
  double *W = (double *)(work + L.w);
  hipError_t e;
  if ((e = launch_clear_ints((int *)(work + L.info), 4, s)) != hipSuccess) return e;
  int64_t lds;
  const double *src = fp64_source(Y, ldy, ydt, rows, n, Q, ldq, &lds, s, &e);
  if (e != hipSuccess) return e;
  if ((e = cholqr_pass(src, lds, W, n, rows, n, 0.0, work, L, s)) != hipSuccess) return e;
  return cholqr_pass(W, n, Q, ldq, rows, n, 0.0, work, L, s);
}

// Cholesky-QR twice without the last product: Q1 = Y M1 is formed in Q, and the
// second pass only factors Q1^T Q1 (its M2 is left in work + L.m), so that
// X_F = Q1 M2 can be applied implicitly.  Enqueues only.
hipError_t cholqr2_implicit_enqueue(const void *Y, int64_t ldy, ttdft_dtype ydt, int64_t rows,
                                    int64_t n, double *Q, int64_t ldq, char *work,
                                    const QrLayout &L, hipStream_t s) {
  hipError_t e;
  if ((e = launch_clear_ints((int *)(work + L.info), 4, s)) != hipSuccess) return e;
  int64_t lds;   // a non-FP64 Y is cast into W, so that the product never runs in place
  const double *src = fp64_source(Y, ldy, ydt, rows, n, (double *)(work + L.w), n, &lds, s, &e);
  if (e != hipSuccess) return e;
  if ((e = cholqr_pass(src, lds, Q, ldq, rows, n, 0.0, work, L, s)) != hipSuccess) return e;
  return cholqr_factor(Q, ldq, rows, n, 0.0, work, L, s);
}

// Shifted Cholesky-QR3 (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa): a
// first pass with the diagonal shift s = 11 (rows n + n (n+1)) u ||Gs||, with
// ||Gs|| <= n for the unit-diagonal scaled Gram matrix, makes the block well
// enough conditioned for Cholesky-QR2.  Used after a breakdown of the plain
// passes; needs Y intact (Q must not alias Y).
hipError_t shifted_cholqr3_enqueue(const void *Y, int64_t ldy, ttdft_dtype ydt, int64_t rows,
                                   int64_t n, double *Q, int64_t ldq, char *work, const QrLayout &L,
                                   hipStream_t s) {
  double *W = (double *)(work + L.w);
  hipError_t e;
  if ((e = launch_clear_ints((int *)(work + L.info), 4, s)) != hipSuccess) return e;
  int64_t lds;
  const double *src = fp64_source(Y, ldy, ydt, rows, n, Q, ldq, &lds, s, &e);
  if (e != hipSuccess) return e;
  const double u = 1.1102230246251565e-16;
  const double shift = 11.0 * ((double)rows * n + (double)n * (n + 1)) * u * (double)n;
  if ((e = cholqr_pass(src, lds, W, n, rows, n, shift, work, L, s)) != hipSuccess) return e;
  if ((e = cholqr_pass(W, n, Q, ldq, rows, n, 0.0, work, L, s)) != hipSuccess) return e;
  if ((e = cholqr_pass(Q, ldq, W, n, rows, n, 0.0, work, L, s)) != hipSuccess) return e;
  return launch_cast(W, TTDFT_F64, n, Q, TTDFT_F64, ldq, rows, n, s);
}

ttdft_status check_h64(const ttdft_bsr *H) {
  if (!H) return failf(TTDFT_ERR_NULL, "H is NULL");
  if (H->dtype != TTDFT_F64) return failf(TTDFT_ERR_DTYPE, "the projection needs an FP64 H");
  if (H->n_block_rows < 1 || H->n_tiles < 0) return failf(TTDFT_ERR_SHAPE, "bad H shape");
  if (!H->tile_rowptr || (H->n_tiles > 0 && (!H->tile_col || !H->vals)))
    return failf(TTDFT_ERR_NULL, "H arrays are NULL");
  return TTDFT_OK;
}

struct ProjLayout {
  int splits;
  size_t hq, partial, total;
};
ProjLayout proj_layout(int64_t rows, int64_t n) {
  ProjLayout L;
  L.splits = gemm_tn_splits(rows, n, true);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.hq = take((size_t)rows * n * 8);
  L.partial = take((size_t)L.splits * n * n * 8);
  L.total = off;
  return L;
}

hipError_t project_enqueue(const ttdft_bsr &H, const double *Q, int64_t ldq, int64_t n, double *A,
                           int64_t lda, char *work, const ProjLayout &L, hipStream_t s) {
  const int64_t rows = H.n_block_rows * 64;
  double *HQ = (double *)(work + L.hq), *partial = (double *)(work + L.partial);
  hipError_t e = launch_cheb_step(H, Q, ldq, nullptr, 0, HQ, n, n, 1.0, 0.0, 0.0, TTDFT_F64, s);
  if (e != hipSuccess) return e;
  // Q^T (H Q) is symmetric (H is): only its lower-triangular tiles are formed and
  // mirrored; inside the diagonal tiles the two halves are averaged
  return launch_gemm_tn_ex(Q, ldq, HQ, n, rows, n, A, lda, true, true, partial, L.splits, s);
}

struct RrLayout {
  QrLayout qr;
  ProjLayout pj;
  size_t xf, qr_off, pj_off, hf, zq, m2, syev, total;
};
RrLayout rr_layout(int64_t rows, int64_t n) {
  RrLayout L;
  L.qr = qr_layout(rows, n);
  L.pj = proj_layout(rows, n);
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  L.xf = take((size_t)rows * n * 8);
  // the Cholesky-QR scratch and the projection scratch are used one after the other
  const size_t shared = std::max(L.qr.total, L.pj.total);
  L.qr_off = take(shared);
  L.pj_off = L.qr_off;
  L.hf = take((size_t)n * n * 8);
  L.zq = take((size_t)n * n * 8);
  L.m2 = take((size_t)n * n * 8);
  L.syev = take(syev_work_bytes(n));
  L.total = off;
  return L;
}

// 0 when the enqueued passes succeeded, else the breakdown column (1-based);
// *nonfinite is set when a Gram diagonal entry was NaN or Inf (a non-finite block)
int qr_breakdown(char *work, const QrLayout &L, hipStream_t s, hipError_t *e, bool *nonfinite) {
  *nonfinite = false;
  *e = hipStreamSynchronize(s);
  if (*e != hipSuccess) return 0;
  int info[2] = {0, 0};
  *e = hipMemcpy(info, work + L.info, sizeof info, hipMemcpyDeviceToHost);
  *nonfinite = info[1] != 0;
  return info[0];
}

// Cholesky-QR2, and shifted Cholesky-QR3 when the plain passes break down
ttdft_status orthonormalise(const void *Y, int64_t ldy, ttdft_dtype ydt, int64_t rows, int64_t n,
                            double *Q, int64_t ldq, char *work, const QrLayout &L, hipStream_t s,
                            bool y_intact_after) {
  hipError_t e = cholqr2_enqueue(Y, ldy, ydt, rows, n, Q, ldq, work, L, s);
  if (e != hipSuccess) return hip_fail(e, "cholqr2 launch");
  bool nonfinite;
  int col = qr_breakdown(work, L, s, &e, &nonfinite);
  if (e != hipSuccess) return hip_fail(e, "cholqr2");
  if (nonfinite) return failf(TTDFT_ERR_NONFINITE, "the block holds a NaN or Inf");
  if (col == 0) return TTDFT_OK;
  if (!y_intact_after)
    return failf(TTDFT_ERR_NOT_POSDEF, "Cholesky breakdown at column %d (Q aliases Y: no retry)", col);
  e = shifted_cholqr3_enqueue(Y, ldy, ydt, rows, n, Q, ldq, work, L, s);
  if (e != hipSuccess) return hip_fail(e, "shifted cholqr3 launch");
  col = qr_breakdown(work, L, s, &e, &nonfinite);
  if (e != hipSuccess) return hip_fail(e, "shifted cholqr3");
  if (col) return failf(TTDFT_ERR_NOT_POSDEF, "Cholesky breakdown at column %d: block rank-deficient in FP64", col);
  return TTDFT_OK;
}

}  // namespace

extern "C" {

size_t ttdft_cholqr2_workspace(int64_t n_rows, int64_t n_vec, ttdft_dtype y_dtype) {
  if (n_rows < 1 || n_vec < 1 || !valid_dtype(y_dtype)) return 0;
  return qr_layout(n_rows, n_vec).total;
}

ttdft_status ttdft_cholqr2(const void *Y, int64_t ldy, ttdft_dtype y_dtype, int64_t n_rows,
                           int64_t n_vec, double *Q, int64_t ldq, void *work, size_t work_bytes,
                           void *stream) {
  if (!valid_dtype(y_dtype)) return failf(TTDFT_ERR_DTYPE, "unknown dtype");
  if (!Y || !Q) return failf(TTDFT_ERR_NULL, "Y or Q is NULL");
  if (n_vec < 1 || n_rows < n_vec || ldy < n_vec || ldq < n_vec)
    return failf(TTDFT_ERR_SHAPE, "need n_rows >= n_vec >= 1 and ld >= n_vec");
  const QrLayout L = qr_layout(n_rows, n_vec);
  if (!work || work_bytes < L.total) return failf(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", L.total);
  const size_t yb = block_bytes(n_rows, ldy, n_vec, y_dtype == TTDFT_F64 ? 8 : y_dtype == TTDFT_F32 ? 4 : 2);
  const size_t qb = block_bytes(n_rows, ldq, n_vec, 8);
  if (overlap(Y, yb, Q, qb) && !(y_dtype == TTDFT_F64 && (const void *)Y == (const void *)Q && ldy == ldq))
    return failf(TTDFT_ERR_ALIAS, "Q overlaps Y");
  if (overlap(work, L.total, Q, qb) || overlap(work, L.total, Y, yb))
    return failf(TTDFT_ERR_ALIAS, "workspace overlaps Y or Q");
  hipStream_t s = (hipStream_t)stream;
  const bool intact = (const void *)Y != (const void *)Q;
  ttdft_status st = orthonormalise(Y, ldy, y_dtype, n_rows, n_vec, Q, ldq, (char *)work, L, s, intact);
  return st == TTDFT_OK ? api_ok() : st;
}

size_t ttdft_project_workspace(const ttdft_bsr *H, int64_t n_vec) {
  if (!H || H->n_block_rows < 1 || n_vec < 1) return 0;
  return proj_layout(H->n_block_rows * 64, n_vec).total;
}

ttdft_status ttdft_project(const ttdft_bsr *H, const double *Q, int64_t ldq, int64_t n_vec,
                           double *A, int64_t lda, void *work, size_t work_bytes, void *stream) {
  ttdft_status st = check_h64(H);
  if (st != TTDFT_OK) return st;
  if (!Q || !A) return failf(TTDFT_ERR_NULL, "Q or A is NULL");
  if (n_vec < 1 || ldq < n_vec || lda < n_vec) return failf(TTDFT_ERR_SHAPE, "bad shape");
  if (!step_ld_ok(ldq, 8) || !step_ld_ok(n_vec, 8))
    return failf(TTDFT_ERR_SHAPE, "leading dimension too large for 32-bit panel offsets");
  const int64_t rows = H->n_block_rows * 64;
  const ProjLayout L = proj_layout(rows, n_vec);
  if (!work || work_bytes < L.total) return failf(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", L.total);
  const size_t qb = block_bytes(rows, ldq, n_vec, 8), ab = block_bytes(n_vec, lda, n_vec, 8);
  if (overlap(Q, qb, A, ab) || overlap(work, L.total, A, ab) || overlap(work, L.total, Q, qb))
    return failf(TTDFT_ERR_ALIAS, "buffers overlap");
  hipError_t e = project_enqueue(*H, Q, ldq, n_vec, A, lda, (char *)work, L, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "project launch");
  return api_ok();
}

size_t ttdft_syev_workspace(int64_t n) { return n < 1 ? 0 : syev_work_bytes(n); }

ttdft_status ttdft_syev(int64_t n, const double *A, int64_t lda, double *lambda, double *Z,
                        int64_t ldz, void *work, size_t work_bytes, void *stream) {
  if (!A || !lambda || !Z) return failf(TTDFT_ERR_NULL, "A, lambda or Z is NULL");
  if (n < 1 || lda < n || ldz < n) return failf(TTDFT_ERR_SHAPE, "bad shape");
  const size_t need = syev_work_bytes(n);
  if (!work || work_bytes < need) return failf(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
  const size_t ab = block_bytes(n, lda, n, 8), zb = block_bytes(n, ldz, n, 8);
  if (overlap(A, ab, Z, zb) || overlap(lambda, (size_t)n * 8, Z, zb) || overlap(lambda, (size_t)n * 8, A, ab) ||
      overlap(work, need, Z, zb) || overlap(work, need, A, ab) || overlap(work, need, lambda, (size_t)n * 8))
    return failf(TTDFT_ERR_ALIAS, "buffers overlap");
  int info[2] = {0, 0};
  hipError_t e = run_syev(n, A, lda, lambda, Z, ldz, work, (hipStream_t)stream, info);
  if (e != hipSuccess) return hip_fail(e, "syev");
  if (info[1]) return failf(TTDFT_ERR_NONFINITE, "non-finite value in the tridiagonal reduction");
  if (info[0]) return failf(TTDFT_ERR_NO_CONVERGENCE, "eigenvector block lost rank (column %d)", info[0]);
  return api_ok();
}

ttdft_status ttdft_rotate(const double *XF, int64_t ldx, int64_t n_rows, int64_t n_vec,
                          const double *Q, int64_t ldq, double *Psi, int64_t ldpsi, void *stream) {
  if (!XF || !Q || !Psi) return failf(TTDFT_ERR_NULL, "XF, Q or Psi is NULL");
  if (n_rows < 1 || n_vec < 1 || ldx < n_vec || ldq < n_vec || ldpsi < n_vec)
    return failf(TTDFT_ERR_SHAPE, "bad shape");
  const size_t xb = block_bytes(n_rows, ldx, n_vec, 8), qb = block_bytes(n_vec, ldq, n_vec, 8),
               pb = block_bytes(n_rows, ldpsi, n_vec, 8);
  if (overlap(Psi, pb, XF, xb) || overlap(Psi, pb, Q, qb)) return failf(TTDFT_ERR_ALIAS, "Psi overlaps an input");
  hipError_t e = launch_gemm_nn_ex(XF, ldx, Q, ldq, n_rows, n_vec, n_vec, 1.0, Psi, ldpsi, false,
                                   (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rotate launch");
  return api_ok();
}

size_t ttdft_rayleigh_ritz_workspace(const ttdft_bsr *H, int64_t n_vec, ttdft_dtype y_dtype) {
  if (!H || H->n_block_rows < 1 || n_vec < 1 || !valid_dtype(y_dtype)) return 0;
  return rr_layout(H->n_block_rows * 64, n_vec).total;
}

ttdft_status ttdft_rayleigh_ritz(const ttdft_bsr *H, const void *Y, int64_t ldy, ttdft_dtype y_dtype,
                                 int64_t n_vec, double *lambda, double *Psi, int64_t ldpsi,
                                 void *work, size_t work_bytes, void *stream) {
  ttdft_status st = check_h64(H);
  if (st != TTDFT_OK) return st;
  if (!valid_dtype(y_dtype)) return failf(TTDFT_ERR_DTYPE, "unknown dtype");
  if (!Y || !lambda || !Psi) return failf(TTDFT_ERR_NULL, "Y, lambda or Psi is NULL");
  const int64_t rows = H->n_block_rows * 64;
  if (n_vec < 1 || n_vec > rows || ldy < n_vec || ldpsi < n_vec) return failf(TTDFT_ERR_SHAPE, "bad shape");
  if (!step_ld_ok(n_vec, 8)) return failf(TTDFT_ERR_SHAPE, "n_vec too large for 32-bit panel offsets");
  const RrLayout L = rr_layout(rows, n_vec);
  if (!work || work_bytes < L.total) return failf(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", L.total);
  const size_t elt = y_dtype == TTDFT_F64 ? 8 : y_dtype == TTDFT_F32 ? 4 : 2;
  const size_t yb = block_bytes(rows, ldy, n_vec, elt), pb = block_bytes(rows, ldpsi, n_vec, 8);
  if (overlap(Psi, pb, Y, yb) || overlap(work, L.total, Psi, pb) || overlap(work, L.total, Y, yb) ||
      overlap(lambda, (size_t)n_vec * 8, Psi, pb) || overlap(lambda, (size_t)n_vec * 8, work, L.total))
    return failf(TTDFT_ERR_ALIAS, "buffers overlap");
  char *w = (char *)work;
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = n_vec;
  double *XF = (double *)(w + L.xf), *Hf = (double *)(w + L.hf), *Zq = (double *)(w + L.zq);
  double *M2 = (double *)(w + L.m2);
  // Cholesky-QR twice with X_F = Q1 M2 left implicit: XF holds Q1, the projected
  // matrix is M2^T (Q1^T H Q1) M2 and the Ritz vectors are Q1 (M2 Z), which saves
  // the rows x n x n product that would form X_F.  After a breakdown of the plain
  // passes the shifted Cholesky-QR3 forms X_F explicitly (M2 = identity).
  bool implicit = true;
  hipError_t e = cholqr2_implicit_enqueue(Y, ldy, y_dtype, rows, n, XF, n, w + L.qr_off, L.qr, s);
  if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: cholqr2 launch");
  bool nonfinite;
  int col = qr_breakdown(w + L.qr_off, L.qr, s, &e, &nonfinite);
  if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: cholqr2");
  if (nonfinite) return failf(TTDFT_ERR_NONFINITE, "the filtered block holds a NaN or Inf");
  if (col) {
    implicit = false;
    e = shifted_cholqr3_enqueue(Y, ldy, y_dtype, rows, n, XF, n, w + L.qr_off, L.qr, s);
    if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: shifted cholqr3 launch");
    col = qr_breakdown(w + L.qr_off, L.qr, s, &e, &nonfinite);
    if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: shifted cholqr3");
    if (col) return failf(TTDFT_ERR_NOT_POSDEF, "Cholesky breakdown at column %d: block rank-deficient in FP64", col);
  } else {
    // M2 leaves the Cholesky-QR scratch, which the projection reuses
    e = launch_cast(w + L.qr_off + L.qr.m, TTDFT_F64, L.qr.np, M2, TTDFT_F64, n, n, n, s);
    if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: copy");
  }
  e = project_enqueue(*H, XF, n, n, Hf, n, w + L.pj_off, L.pj, s);
  if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: projection");
  if (implicit) {
    // Hf <- M2^T (Hf M2), exactly symmetric (lower tiles mirrored, diagonal tiles
    // averaged); Zq is free until the eigensolve and holds Hf M2
    const int splits = gemm_tn_splits(n, n, true);
    if (splits > L.pj.splits) return failf(TTDFT_ERR_WORKSPACE, "internal: split-K scratch too small");
    double *partial = (double *)(w + L.pj_off + L.pj.partial);
    e = launch_gemm_nn_ex(Hf, n, M2, n, n, n, n, 1.0, Zq, n, true, s);
    if (e == hipSuccess) e = launch_gemm_tn_ex(M2, n, Zq, n, n, n, Hf, n, true, true, partial, splits, s);
    if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: projection transform");
  }
  int info[2] = {0, 0};
  e = run_syev(n, Hf, n, lambda, Zq, n, w + L.syev, s, info);
  if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: eigensolve");
  if (info[1]) return failf(TTDFT_ERR_NONFINITE, "non-finite value in the projected matrix");
  if (info[0]) return failf(TTDFT_ERR_NO_CONVERGENCE, "eigenvector block lost rank");
  const double *Zr = Zq;
  if (implicit) {   // Hf (copied by the eigensolve) is free: M2 Z
    e = launch_gemm_nn_ex(M2, n, Zq, n, n, n, n, 1.0, Hf, n, false, s);
    if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: rotation factor");
    Zr = Hf;
  }
  e = launch_gemm_nn_ex(XF, n, Zr, n, rows, n, n, 1.0, Psi, ldpsi, false, s);
  if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz: rotation");
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "rayleigh_ritz");
  return api_ok();
}

}  // extern "C"

extern "C" {

size_t ttdft_lanczos_workspace(const ttdft_bsr *H, int32_t k) {
  if (!H || H->n_block_rows < 1 || k < 1) return 0;
  return lanczos_work_bytes(H->n_block_rows * 64, k);
}

ttdft_status ttdft_lanczos_bounds(const ttdft_bsr *H, const int64_t *perm, int32_t k,
                                  uint64_t seed, double *bounds, void *work, size_t work_bytes,
                                  void *stream) {
  ttdft_status st = check_h64(H);
  if (st != TTDFT_OK) return st;
  if (!perm || !bounds) return failf(TTDFT_ERR_NULL, "perm or bounds is NULL");
  if (k < 1 || k > 1000) return failf(TTDFT_ERR_SHAPE, "k = %d outside 1 .. 1000", k);
  const size_t need = lanczos_work_bytes(H->n_block_rows * 64, k);
  if (!work || work_bytes < need) return failf(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
  double out[4];
  int breakdown = 0;
  hipError_t e = run_lanczos_bound(*H, perm, k, seed, work, (hipStream_t)stream, out, &breakdown);
  if (e != hipSuccess) return hip_fail(e, "lanczos");
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(out[i])) return failf(TTDFT_ERR_NONFINITE, "non-finite Lanczos estimate");
  for (int i = 0; i < 4; ++i) bounds[i] = out[i];
  return api_ok();
}

size_t ttdft_ritz_residuals_workspace(const ttdft_bsr *H, int64_t n_vec) {
  if (!H || H->n_block_rows < 1 || n_vec < 1) return 0;
  return residual_work_bytes(H->n_block_rows * 64, n_vec);
}

ttdft_status ttdft_ritz_residuals(const ttdft_bsr *H, const double *Psi, int64_t ldp,
                                  const double *lambda, int64_t n_vec, double *res, void *work,
                                  size_t work_bytes, void *stream) {
  ttdft_status st = check_h64(H);
  if (st != TTDFT_OK) return st;
  if (!Psi || !lambda || !res) return failf(TTDFT_ERR_NULL, "Psi, lambda or res is NULL");
  if (n_vec < 1 || ldp < n_vec) return failf(TTDFT_ERR_SHAPE, "bad shape");
  if (!step_ld_ok(ldp, 8)) return failf(TTDFT_ERR_SHAPE, "leading dimension too large for 32-bit panel offsets");
  const int64_t rows = H->n_block_rows * 64;
  const size_t need = residual_work_bytes(rows, n_vec);
  if (!work || work_bytes < need) return failf(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
  const size_t pb = block_bytes(rows, ldp, n_vec, 8), vb = (size_t)n_vec * 8;
  if (overlap(work, need, Psi, pb) || overlap(work, need, lambda, vb) || overlap(work, need, res, vb) ||
      overlap(res, vb, Psi, pb) || overlap(res, vb, lambda, vb))
    return failf(TTDFT_ERR_ALIAS, "buffers overlap");
  hipError_t e = run_ritz_residuals(*H, Psi, ldp, lambda, n_vec, res, work, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "residual launch");
  return api_ok();
}

size_t ttdft_fermi_level_workspace(void) { return 2 * sizeof(double); }

ttdft_status ttdft_fermi_level(const double *lambda, int64_t n, double n_electrons, double kT,
                               double *f, double *mu, void *work, size_t work_bytes, void *stream) {
  if (!lambda || !f || !mu) return failf(TTDFT_ERR_NULL, "lambda, f or mu is NULL");
  if (n < 1) return failf(TTDFT_ERR_SHAPE, "n = %lld", (long long)n);
  if (!(kT > 0.0) || !std::isfinite(kT)) return failf(TTDFT_ERR_BOUNDS, "kT must be positive and finite");
  if (!(n_electrons > 0.0) || !(n_electrons < 2.0 * (double)n))
    return failf(TTDFT_ERR_BOUNDS, "need 0 < n_electrons < 2n (n = %lld)", (long long)n);
  if (!work || work_bytes < 2 * sizeof(double)) return failf(TTDFT_ERR_WORKSPACE, "workspace of 16 bytes needed");
  const size_t vb = (size_t)n * 8;
  if (overlap(lambda, vb, f, vb) || overlap(work, 16, f, vb) || overlap(work, 16, lambda, vb))
    return failf(TTDFT_ERR_ALIAS, "buffers overlap");
  int bad = 0;
  hipError_t e = run_fermi_level(lambda, n, n_electrons, kT, f, (double *)work, (hipStream_t)stream, mu, &bad);
  if (e != hipSuccess) return hip_fail(e, "fermi level");
  if (bad) return failf(TTDFT_ERR_NONFINITE, "non-finite eigenvalue");
  return api_ok();
}

ttdft_status ttdft_density_matrix(const ttdft_bsr *H, const double *Psi, int64_t ldp, const double *f,
                                  int64_t n_vec, double *P_vals, const uint64_t *mask, void *stream) {
  ttdft_status st = check_h64(H);
  if (st != TTDFT_OK) return st;
  if (!Psi || !f || !P_vals) return failf(TTDFT_ERR_NULL, "Psi, f or P_vals is NULL");
  if (n_vec < 1 || ldp < n_vec) return failf(TTDFT_ERR_SHAPE, "bad shape");
  if (!step_ld_ok(ldp, 8)) return failf(TTDFT_ERR_SHAPE, "leading dimension too large for 32-bit panel offsets");
  const int64_t rows = H->n_block_rows * 64;
  const size_t pb = block_bytes(rows, ldp, n_vec, 8), vb = (size_t)n_vec * 8;
  const size_t hb = (size_t)H->n_tiles * kTileElems * 8;
  if (overlap(P_vals, hb, Psi, pb) || overlap(P_vals, hb, f, vb) || overlap(P_vals, hb, H->vals, hb))
    return failf(TTDFT_ERR_ALIAS, "buffers overlap");
  // P = 2 Psi diag(f) Psi^T is symmetric: each pair of mirror tiles is formed once
  hipError_t e = launch_sddmm(*H, Psi, ldp, Psi, ldp, n_vec, 2.0, P_vals, mask, false, TTDFT_F64,
                              (hipStream_t)stream, f, true);
  if (e != hipSuccess) return hip_fail(e, "density matrix launch");
  return api_ok();
}

ttdft_status ttdft_electron_density(const double *Psi, int64_t ldp, const double *f, int64_t rows,
                                    int64_t n_vec, double *rho, void *stream) {
  if (!Psi || !f || !rho) return failf(TTDFT_ERR_NULL, "Psi, f or rho is NULL");
  if (rows < 1 || n_vec < 1 || ldp < n_vec) return failf(TTDFT_ERR_SHAPE, "bad shape");
  const size_t pb = block_bytes(rows, ldp, n_vec, 8);
  if (overlap(rho, (size_t)rows * 8, Psi, pb) || overlap(rho, (size_t)rows * 8, f, (size_t)n_vec * 8))
    return failf(TTDFT_ERR_ALIAS, "buffers overlap");
  hipError_t e = launch_electron_density(Psi, ldp, f, rows, n_vec, rho, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "electron density launch");
  return api_ok();
}

}  // extern "C"
