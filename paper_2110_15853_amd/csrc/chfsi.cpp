// The subspace iteration of Algorithm 1 (Sec. 3.4) behind the C ABI: one pass
// (filter, FP64 Rayleigh-Ritz, Ritz residuals, the bounds of the next pass) and
// the loop that repeats it until the residuals are small.  Everything here is
// host control flow over the other entry points; the arithmetic runs in their
// kernels.
//
// Bounds.  A pass filters with the unwanted interval [a, b] and the scaling
// point a0.  The next pass keeps b and moves a0 and a to the smallest and the
// largest Ritz value of this pass: the block's Ritz values then lie in
// [a0, a], the wanted part of the spectrum the filter must keep.  The first
// pass takes b from the safeguarded Lanczos bound, a0 from the smallest
// Lanczos Ritz value and the cut a halfway between them, unless the caller
// gives the bounds.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <limits>
#include <vector>

#include "ttdft_internal.h"

using namespace ttdft;

namespace ttdft {
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

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

bool x_dtype_ok(ttdft_dtype t) { return t == TTDFT_F64 || t == TTDFT_F32; }

// workspace of one pass: the filtered block Y, then one region shared in turn by
// the filter's work block, the Rayleigh-Ritz workspace and the residual workspace
struct PassLayout {
  size_t y, shared, total;
};
PassLayout pass_layout(const ttdft_bsr *Hf, const ttdft_bsr *H64, int64_t n, ttdft_dtype xt) {
  PassLayout L;
  const int64_t rows = H64->n_block_rows * 64;
  L.y = align256((size_t)rows * n * dtype_size(xt));
  const size_t shared = std::max({ttdft_cheb_filter_workspace(Hf, n, xt),
                                  ttdft_rayleigh_ritz_workspace(H64, n, xt),
                                  ttdft_ritz_residuals_workspace(H64, n)});
  L.shared = align256(shared);
  L.total = L.y + L.shared;
  return L;
}

ttdft_status check_pair(const ttdft_bsr *Hf, const ttdft_bsr *H64, ttdft_dtype xt, int64_t n) {
  if (!Hf || !H64) return failf(TTDFT_ERR_NULL, "Hf or H64 is NULL");
  if (H64->dtype != TTDFT_F64) return failf(TTDFT_ERR_DTYPE, "the Rayleigh-Ritz step needs an FP64 H64");
  if (!x_dtype_ok(xt)) return failf(TTDFT_ERR_DTYPE, "iterates must be F64 or F32");
  if (Hf->n_block_rows != H64->n_block_rows || Hf->n_tiles != H64->n_tiles)
    return failf(TTDFT_ERR_SHAPE, "Hf and H64 must be the same blocked matrix");
  if (n < 1 || n > H64->n_block_rows * 64) return failf(TTDFT_ERR_SHAPE, "bad n_vec");
  return TTDFT_OK;
}

// (min, max) of the n values at lambda (device), on the host
hipError_t lambda_range(const double *lambda, int64_t n, hipStream_t s, double *lo, double *hi) {
  std::vector<double> h(n);
  hipError_t e = hipStreamSynchronize(s);
  if (e != hipSuccess) return e;
  if ((e = hipMemcpy(h.data(), lambda, n * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  *lo = std::numeric_limits<double>::infinity();
  *hi = -*lo;
  for (double v : h) {
    if (!std::isfinite(v)) {
      *lo = *hi = v;
      return hipSuccess;
    }
    *lo = std::min(*lo, v);
    *hi = std::max(*hi, v);
  }
  return hipSuccess;
}

ttdft_status next_bounds_host(double lo, double hi, double b, double out[3]) {
  if (!(std::isfinite(lo) && std::isfinite(hi)))
    return failf(TTDFT_ERR_NONFINITE, "non-finite Ritz value");
  if (!(lo < hi && hi < b))
    return failf(TTDFT_ERR_BOUNDS, "Ritz values [%g, %g] do not leave a0 < a < b = %g", lo, hi, b);
  out[0] = lo;
  out[1] = hi;
  out[2] = b;
  return TTDFT_OK;
}

struct Timer {
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool ok = false;
  explicit Timer(bool on) {
    if (!on) return;
    ok = true;
    for (auto &e : ev)
      if (hipEventCreate(&e) != hipSuccess) ok = false;
  }
  ~Timer() {
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  void mark(int i, hipStream_t s) {
    if (ok) (void)hipEventRecord(ev[i], s);
  }
  double ms(int i, int j) {
    float t = 0.0f;
    if (!ok || hipEventElapsedTime(&t, ev[i], ev[j]) != hipSuccess) return NAN;
    return t;
  }
};

// one pass on validated arguments; rec (may be NULL) receives the pass's record
ttdft_status run_pass(const ttdft_bsr *Hf, const ttdft_bsr *H64, const void *X, int64_t ldx,
                      ttdft_dtype xt, int64_t n, int32_t m, const double bounds[3], int64_t n_conv,
                      double *lambda, double *Psi, int64_t ldpsi, double *res,
                      ttdft_chfsi_record *rec, double next[3], char *work, const PassLayout &L,
                      hipStream_t s) {
  void *Y = work;
  char *sh = work + L.y;
  Timer tm(rec != nullptr);
  if (rec) {
    rec->m = m;
    rec->rank_deficient = 0;
    rec->a0 = bounds[0];
    rec->a = bounds[1];
    rec->b = bounds[2];
    rec->max_residual = NAN;
    rec->filter_ms = rec->rr_ms = rec->residual_ms = NAN;
  }
  tm.mark(0, s);
  ttdft_status st = ttdft_cheb_filter(Hf, X, ldx, Y, n, n, m, bounds[1], bounds[2], bounds[0], xt,
                                      sh, L.shared, s);
  if (st != TTDFT_OK) return st;
  tm.mark(1, s);
  st = ttdft_rayleigh_ritz(H64, Y, n, xt, n, lambda, Psi, ldpsi, sh, L.shared, s);
  if (st == TTDFT_ERR_NOT_POSDEF && rec) rec->rank_deficient = 1;
  if (st != TTDFT_OK) return st;
  tm.mark(2, s);
  st = ttdft_ritz_residuals(H64, Psi, ldpsi, lambda, n, res, sh, L.shared, s);
  if (st != TTDFT_OK) return st;
  tm.mark(3, s);
  std::vector<double> hres(n_conv);
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(hres.data(), res, n_conv * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return failf(TTDFT_ERR_HIP, "chfsi pass: %s", hipGetErrorString(e));
  double worst = 0.0;
  for (double v : hres) worst = std::isfinite(v) ? std::max(worst, v) : v;
  if (rec) {
    rec->max_residual = worst;
    rec->filter_ms = tm.ms(0, 1);
    rec->rr_ms = tm.ms(1, 2);
    rec->residual_ms = tm.ms(2, 3);
  }
  if (!std::isfinite(worst)) return failf(TTDFT_ERR_NONFINITE, "non-finite Ritz residual");
  double lo, hi;
  if ((e = lambda_range(lambda, n, s, &lo, &hi)) != hipSuccess)
    return failf(TTDFT_ERR_HIP, "chfsi pass: %s", hipGetErrorString(e));
  return next_bounds_host(lo, hi, bounds[2], next);
}

size_t solve_extra_bytes(const ttdft_bsr *H64, int64_t n, ttdft_dtype xt) {
  // the next pass's start block in the iterates' precision (F32 only; F64 starts from Psi)
  return xt == TTDFT_F64 ? 0 : align256((size_t)H64->n_block_rows * 64 * n * dtype_size(xt));
}

}  // namespace

extern "C" {

ttdft_status ttdft_next_bounds(const double *lambda, int64_t n, double b, double *bounds, void *stream) {
  if (!lambda || !bounds) return failf(TTDFT_ERR_NULL, "lambda or bounds is NULL");
  if (n < 2) return failf(TTDFT_ERR_SHAPE, "need at least two Ritz values");
  if (!std::isfinite(b)) return failf(TTDFT_ERR_BOUNDS, "b must be finite");
  double lo, hi, out[3];
  hipError_t e = lambda_range(lambda, n, (hipStream_t)stream, &lo, &hi);
  if (e != hipSuccess) return failf(TTDFT_ERR_HIP, "next bounds: %s", hipGetErrorString(e));
  ttdft_status st = next_bounds_host(lo, hi, b, out);
  if (st != TTDFT_OK) return st;
  for (int i = 0; i < 3; ++i) bounds[i] = out[i];
  return api_ok();
}

size_t ttdft_chfsi_pass_workspace(const ttdft_bsr *Hf, const ttdft_bsr *H64, int64_t n_vec,
                                  ttdft_dtype x_dtype) {
  if (!Hf || !H64 || H64->n_block_rows < 1 || n_vec < 1 || !x_dtype_ok(x_dtype)) return 0;
  return pass_layout(Hf, H64, n_vec, x_dtype).total;
}

ttdft_status ttdft_chfsi_pass(const ttdft_bsr *Hf, const ttdft_bsr *H64, const void *X, int64_t ldx,
                              ttdft_dtype x_dtype, int64_t n_vec, int32_t m, const double *bounds,
                              int64_t n_conv, double *lambda, double *Psi, int64_t ldpsi,
                              double *res, ttdft_chfsi_record *record, double *next_bounds,
                              void *work, size_t work_bytes, void *stream) {
  ttdft_status st = check_pair(Hf, H64, x_dtype, n_vec);
  if (st != TTDFT_OK) return st;
  if (!X || !bounds || !lambda || !Psi || !res || !next_bounds)
    return failf(TTDFT_ERR_NULL, "a required pointer is NULL");
  if (m < 1) return failf(TTDFT_ERR_DEGREE, "degree m = %d < 1", m);
  if (n_conv < 1 || n_conv > n_vec) return failf(TTDFT_ERR_SHAPE, "n_conv outside 1 .. n_vec");
  if (ldx < n_vec || ldpsi < n_vec) return failf(TTDFT_ERR_SHAPE, "leading dimension smaller than n_vec");
  if (!(std::isfinite(bounds[0]) && std::isfinite(bounds[1]) && std::isfinite(bounds[2])) ||
      !(bounds[0] < bounds[1] && bounds[1] < bounds[2]))
    return failf(TTDFT_ERR_BOUNDS, "bounds must be finite with a0 < a < b");
  const PassLayout L = pass_layout(Hf, H64, n_vec, x_dtype);
  if (!work || work_bytes < L.total) return failf(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", L.total);
  if (record) record->pass = 1;
  double next[3];
  st = run_pass(Hf, H64, X, ldx, x_dtype, n_vec, m, bounds, n_conv, lambda, Psi, ldpsi, res, record,
                next, (char *)work, L, (hipStream_t)stream);
  if (st != TTDFT_OK) return st;
  for (int i = 0; i < 3; ++i) next_bounds[i] = next[i];
  return api_ok();
}

size_t ttdft_chfsi_solve_workspace(const ttdft_bsr *Hf, const ttdft_bsr *H64, int64_t n_vec,
                                   ttdft_dtype x_dtype, int32_t lanczos_k) {
  if (!Hf || !H64 || H64->n_block_rows < 1 || n_vec < 1 || !x_dtype_ok(x_dtype)) return 0;
  const PassLayout L = pass_layout(Hf, H64, n_vec, x_dtype);
  const size_t lz = lanczos_k > 0 ? ttdft_lanczos_workspace(H64, lanczos_k) : 0;
  return std::max(L.total, align256(lz)) + solve_extra_bytes(H64, n_vec, x_dtype);
}

ttdft_status ttdft_chfsi_solve(const ttdft_bsr *Hf, const ttdft_bsr *H64, const int64_t *perm,
                               const void *X, int64_t ldx, ttdft_dtype x_dtype, int64_t n_vec,
                               int32_t m, int32_t m_first, double tol, int64_t n_conv,
                               int32_t max_passes, const double *bounds, int32_t lanczos_k,
                               uint64_t seed, double *lambda, double *Psi, int64_t ldpsi,
                               double *res, ttdft_chfsi_record *history, int32_t history_cap,
                               int32_t *n_records, void *work, size_t work_bytes, void *stream) {
  ttdft_status st = check_pair(Hf, H64, x_dtype, n_vec);
  if (st != TTDFT_OK) return st;
  if (!X || !lambda || !Psi || !res || !n_records) return failf(TTDFT_ERR_NULL, "a required pointer is NULL");
  if (!bounds && !perm) return failf(TTDFT_ERR_NULL, "perm is needed for the Lanczos bounds");
  if (history_cap > 0 && !history) return failf(TTDFT_ERR_NULL, "history is NULL");
  if (m < 1 || m_first < 0) return failf(TTDFT_ERR_DEGREE, "degree m = %d, m_first = %d", m, m_first);
  if (n_conv < 1 || n_conv > n_vec) return failf(TTDFT_ERR_SHAPE, "n_conv outside 1 .. n_vec");
  if (ldx < n_vec || ldpsi < n_vec) return failf(TTDFT_ERR_SHAPE, "leading dimension smaller than n_vec");
  if (max_passes < 1) return failf(TTDFT_ERR_SHAPE, "max_passes < 1");
  if (!(tol >= 0.0) || !std::isfinite(tol)) return failf(TTDFT_ERR_BOUNDS, "tol must be finite and >= 0");
  if (!bounds && (lanczos_k < 1 || lanczos_k > 1000)) return failf(TTDFT_ERR_SHAPE, "lanczos_k outside 1 .. 1000");
  if (bounds && (!(std::isfinite(bounds[0]) && std::isfinite(bounds[1]) && std::isfinite(bounds[2])) ||
                 !(bounds[0] < bounds[1] && bounds[1] < bounds[2])))
    return failf(TTDFT_ERR_BOUNDS, "bounds must be finite with a0 < a < b");
  const size_t need = ttdft_chfsi_solve_workspace(Hf, H64, n_vec, x_dtype, bounds ? 0 : lanczos_k);
  if (!work || work_bytes < need) return failf(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
  const int64_t rows = H64->n_block_rows * 64;
  const size_t elt = dtype_size(x_dtype);
  const uintptr_t w0 = (uintptr_t)work, w1 = w0 + need;
  const uintptr_t p0 = (uintptr_t)Psi, p1 = p0 + ((rows - 1) * ldpsi + n_vec) * 8;
  const uintptr_t x0 = (uintptr_t)X, x1 = x0 + ((rows - 1) * ldx + n_vec) * elt;
  if ((p0 < w1 && w0 < p1) || (x0 < w1 && w0 < x1) || (x0 < p1 && p0 < x1))
    return failf(TTDFT_ERR_ALIAS, "X, Psi and the workspace must not overlap");

  hipStream_t s = (hipStream_t)stream;
  const PassLayout L = pass_layout(Hf, H64, n_vec, x_dtype);
  const size_t pass_region = need - solve_extra_bytes(H64, n_vec, x_dtype);
  void *Xc = (char *)work + pass_region;      // F32 start block of the later passes
  double cur[3];
  if (bounds) {
    for (int i = 0; i < 3; ++i) cur[i] = bounds[i];
  } else {
    double lz[4];
    st = ttdft_lanczos_bounds(H64, perm, lanczos_k, seed, lz, work, pass_region, stream);
    if (st != TTDFT_OK) return st;
    cur[2] = lz[2];                    // safeguarded upper bound
    cur[0] = lz[3];                    // smallest Lanczos Ritz value
    cur[1] = 0.5 * (lz[3] + lz[2]);
    if (!(cur[0] < cur[1] && cur[1] < cur[2]))
      return failf(TTDFT_ERR_BOUNDS, "Lanczos bounds do not leave a0 < a < b");
  }
  *n_records = 0;
  const void *Xcur = X;
  int64_t ldcur = ldx;
  for (int32_t pass = 1; pass <= max_passes; ++pass) {
    int32_t deg = (pass == 1 && m_first > 0) ? m_first : m;
    double next[3];
    for (;;) {
      ttdft_chfsi_record rec{};
      rec.pass = pass;
      st = run_pass(Hf, H64, Xcur, ldcur, x_dtype, n_vec, deg, cur, n_conv, lambda, Psi, ldpsi, res,
                    &rec, next, (char *)work, L, s);
      if (*n_records < history_cap) history[*n_records] = rec;
      ++*n_records;
      // a filtered block that lost rank in FP64 (the filter spread its components
      // over more than the FP64 range): the same pass at half the degree
      if (st == TTDFT_ERR_NOT_POSDEF && deg > 1) {
        deg = std::max(1, deg / 2);
        continue;
      }
      if (st != TTDFT_OK) return st;
      if (rec.max_residual <= tol) return api_ok();
      break;
    }
    for (int i = 0; i < 3; ++i) cur[i] = next[i];
    if (x_dtype == TTDFT_F64) {
      Xcur = Psi;
      ldcur = ldpsi;
    } else {
      hipError_t e = launch_cast(Psi, TTDFT_F64, ldpsi, Xc, x_dtype, n_vec, rows, n_vec, s);
      if (e != hipSuccess) return failf(TTDFT_ERR_HIP, "chfsi solve: %s", hipGetErrorString(e));
      Xcur = Xc;
      ldcur = n_vec;
    }
  }
  return failf(TTDFT_ERR_NO_CONVERGENCE, "residuals above tol after %d passes", max_passes);
}

}  // extern "C"
