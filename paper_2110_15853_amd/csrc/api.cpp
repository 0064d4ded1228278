// Host side of libttdft: argument validation, the coefficient schedule of the
// Chebyshev filter, the lattice-blocked BSR builder and dispatch to the HIP
// kernels.  Every entry point validates all arguments before touching the
// device, so error paths can be exercised without a GPU.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ttdft_internal.h"

using namespace ttdft;

namespace {

thread_local char g_err[512] = "";

ttdft_status fail(ttdft_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

ttdft_status ok() {
  g_err[0] = '\0';
  return TTDFT_OK;
}

ttdft_status hip_status(hipError_t e, const char *what) {
  if (e == hipSuccess) return ok();
  return fail(TTDFT_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool valid_dtype(int t) { return t == TTDFT_F64 || t == TTDFT_F32 || t == TTDFT_BF16; }
// types of tile values (dense blocks cannot be BF16_SPLIT)
bool valid_tile_dtype(int t) { return valid_dtype(t) || t == TTDFT_BF16_SPLIT; }

// byte range [lo, hi) touched by a rows x cols block with leading dim ld
struct Span {
  uintptr_t lo = 0, hi = 0;
};
Span span_of(const void *p, int64_t rows, int64_t ld, int64_t cols, size_t elt) {
  Span s;
  if (!p || rows <= 0 || cols <= 0) return s;
  s.lo = (uintptr_t)p;
  s.hi = s.lo + (uintptr_t)(((rows - 1) * ld + cols) * (int64_t)elt);
  return s;
}
Span span_bytes(const void *p, size_t bytes) {
  Span s;
  if (!p || bytes == 0) return s;
  s.lo = (uintptr_t)p;
  s.hi = s.lo + bytes;
  return s;
}
bool overlap(const Span &a, const Span &b) {
  return a.hi > a.lo && b.hi > b.lo && a.lo < b.hi && b.lo < a.hi;
}

ttdft_status check_bsr(const ttdft_bsr *H) {
  if (!H) return fail(TTDFT_ERR_NULL, "H is NULL");
  if (!valid_tile_dtype(H->dtype)) return fail(TTDFT_ERR_DTYPE, "H dtype %d unknown", (int)H->dtype);
  if (H->n_block_rows < 1 || H->n_tiles < 0)
    return fail(TTDFT_ERR_SHAPE, "H has %lld block rows and %lld tiles",
                (long long)H->n_block_rows, (long long)H->n_tiles);
  if (H->n_block_rows > (int64_t)1 << 30 || H->n_tiles > 0x7fffffff)
    return fail(TTDFT_ERR_SHAPE, "H too large for 32-bit tile indices");
  if (!H->tile_rowptr) return fail(TTDFT_ERR_NULL, "H.tile_rowptr is NULL");
  if (H->n_tiles > 0 && (!H->tile_col || !H->vals))
    return fail(TTDFT_ERR_NULL, "H.tile_col or H.vals is NULL");
  return TTDFT_OK;
}

// dtype pairs (H, X) the fused step supports
bool supported_pair(ttdft_dtype h, ttdft_dtype x) {
  return (h == TTDFT_F64 && x == TTDFT_F64) || (h == TTDFT_F32 && x == TTDFT_F32) ||
         (h == TTDFT_BF16 && (x == TTDFT_F32 || x == TTDFT_BF16)) ||
         (h == TTDFT_BF16_SPLIT && x == TTDFT_F32);
}

float bf16_to_f32(uint16_t b) {
  const uint32_t u = (uint32_t)b << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// ---- lattice blocking: natural index (i*r + j)*r + k -> (block, local)
// Inside a 4x4x4 block the 64 sites are ordered so that every 16 consecutive
// rows form a 2x2x4 box (i and j pairs, all four k) and every 4 consecutive
// columns a line along k.  A matrix-core fragment (16 rows x 4 columns) then
// couples a compact box to a line, and for a cube stencil more fragments of a
// neighbouring block's tile are empty than with plain k-fastest order: 1200
// instead of 1296 non-empty fragments per block row at h = 4, 768 instead of
// 840 at h = 3.
// The blocks themselves are numbered by 2x2x2 patches: every complete patch
// takes 8 consecutive numbers (its blocks in (i, j, k) order), patches in
// lexicographic order; the blocks of incomplete patches (the far faces when the
// block count per axis is odd) follow.  Eight consecutive block rows are then
// one patch, whose stencils reach a 4x4x4 set of blocks (h <= 4) instead of
// 8 x 27, so a work-group owning a patch loads each neighbouring panel once for
// up to 8 of its rows; four consecutive block rows are a 2x2 square in (j, k).
struct Lattice {
  int64_t r, nb;
  std::vector<int64_t> number;   // block (bi*nb + bj)*nb + bk -> block number
  explicit Lattice(int64_t r_) : r(r_), nb((r_ + 3) / 4), number(nb * nb * nb, -1) {
    const int64_t np = (nb + 1) / 2;
    int64_t next = 0;
    auto place = [&](bool complete) {
      for (int64_t pi = 0; pi < np; ++pi)
        for (int64_t pj = 0; pj < np; ++pj)
          for (int64_t pk = 0; pk < np; ++pk) {
            const bool full = 2 * pi + 1 < nb && 2 * pj + 1 < nb && 2 * pk + 1 < nb;
            if (full != complete) continue;
            for (int64_t d = 0; d < 8; ++d) {
              const int64_t bi = 2 * pi + (d >> 2), bj = 2 * pj + ((d >> 1) & 1), bk = 2 * pk + (d & 1);
              if (bi < nb && bj < nb && bk < nb) number[(bi * nb + bj) * nb + bk] = next++;
            }
          }
    };
    place(true);
    place(false);
  }
  int64_t n_block_rows() const { return nb * nb * nb; }
  void split(int64_t I, int64_t &blk, int64_t &loc) const {
    const int64_t i = I / (r * r), j = (I / r) % r, k = I % r;
    blk = number[((i / 4) * nb + j / 4) * nb + k / 4];
    const int64_t box = ((i % 4) >> 1) * 2 + ((j % 4) >> 1);   // 2x2x4 box of the block
    const int64_t line = (i & 1) * 2 + (j & 1);                 // k-line inside the box
    loc = (box * 4 + line) * 4 + k % 4;
  }
};

ttdft_status check_csr(int32_t r, const int64_t *rowptr, const int32_t *col) {
  if (!rowptr || !col) return fail(TTDFT_ERR_NULL, "rowptr or col is NULL");
  if (r < 1 || r > 2048) return fail(TTDFT_ERR_SHAPE, "lattice extent r=%d out of range", r);
  const int64_t N = (int64_t)r * r * r;
  if (rowptr[0] != 0) return fail(TTDFT_ERR_PATTERN, "rowptr[0] != 0");
  for (int64_t I = 0; I < N; ++I) {
    if (rowptr[I + 1] < rowptr[I]) return fail(TTDFT_ERR_PATTERN, "rowptr decreases at row %lld", (long long)I);
    for (int64_t p = rowptr[I]; p < rowptr[I + 1]; ++p) {
      if (col[p] < 0 || col[p] >= N)
        return fail(TTDFT_ERR_PATTERN, "column %d out of range in row %lld", col[p], (long long)I);
      if (p > rowptr[I] && col[p] <= col[p - 1])
        return fail(TTDFT_ERR_PATTERN, "columns not strictly ascending in row %lld", (long long)I);
    }
  }
  return TTDFT_OK;
}

// sorted distinct block columns of every block row
void block_pattern(const Lattice &L, const int64_t *rowptr, const int32_t *col,
                   std::vector<int32_t> &tptr, std::vector<int32_t> &tcol) {
  const int64_t NB = L.n_block_rows(), N = L.r * L.r * L.r;
  std::vector<std::vector<int32_t>> rows_of(NB);
  for (int64_t I = 0; I < N; ++I) {
    int64_t b, l;
    L.split(I, b, l);
    rows_of[b].push_back((int32_t)I);
  }
  std::vector<int64_t> stamp(NB, -1);
  tptr.assign(NB + 1, 0);
  tcol.clear();
  std::vector<int32_t> cur;
  for (int64_t B = 0; B < NB; ++B) {
    cur.clear();
    for (int32_t I : rows_of[B])
      for (int64_t p = rowptr[I]; p < rowptr[I + 1]; ++p) {
        int64_t bc, lc;
        L.split(col[p], bc, lc);
        if (stamp[bc] != B) {
          stamp[bc] = B;
          cur.push_back((int32_t)bc);
        }
      }
    std::sort(cur.begin(), cur.end());
    tcol.insert(tcol.end(), cur.begin(), cur.end());
    tptr[B + 1] = (int32_t)tcol.size();
  }
}

}  // namespace

namespace ttdft {
ttdft_status api_fail(ttdft_status s, const char *msg) { return fail(s, "%s", msg); }
ttdft_status api_ok() { return ok(); }

// Algorithm 1: e = (b - a)/2, c = (b + a)/2, sigma_1 = e/(a0 - c), gamma = 2/sigma_1;
// the first step uses alpha = sigma_1/e and no previous block; step i >= 2 uses
// sigma_i = 1/(gamma - sigma_{i-1}), alpha = 2 sigma_i/e, beta = sigma_{i-1} sigma_i.
void cheb_coefficients(int m, double a, double b, double a0, double *c, double *alpha,
                       double *beta) {
  const double e = 0.5 * (b - a);
  *c = 0.5 * (b + a);
  double sigma = e / (a0 - *c);
  const double gamma = 2.0 / sigma;
  alpha[0] = sigma / e;
  beta[0] = 0.0;
  for (int k = 1; k < m; ++k) {
    const double sigma2 = 1.0 / (gamma - sigma);
    alpha[k] = 2.0 * sigma2 / e;
    beta[k] = sigma * sigma2;
    sigma = sigma2;
  }
}
}  // namespace ttdft

extern "C" {

const char *ttdft_version(void) { return "ttdft-gfx950 0.1"; }

const char *ttdft_last_error(void) { return g_err; }

const char *ttdft_status_string(ttdft_status s) {
  switch (s) {
    case TTDFT_OK: return "ok";
    case TTDFT_ERR_NULL: return "null pointer";
    case TTDFT_ERR_SHAPE: return "bad shape";
    case TTDFT_ERR_DTYPE: return "unsupported dtype";
    case TTDFT_ERR_BOUNDS: return "bad filter bounds";
    case TTDFT_ERR_DEGREE: return "bad polynomial degree";
    case TTDFT_ERR_ALIAS: return "overlapping buffers";
    case TTDFT_ERR_WORKSPACE: return "workspace too small";
    case TTDFT_ERR_NOT_POSDEF: return "Cholesky breakdown";
    case TTDFT_ERR_NO_CONVERGENCE: return "eigensolver did not converge";
    case TTDFT_ERR_NONFINITE: return "non-finite value";
    case TTDFT_ERR_HIP: return "HIP error";
    case TTDFT_ERR_PATTERN: return "malformed sparsity pattern";
  }
  return "unknown status";
}

ttdft_status ttdft_bsr_plan(int32_t r, const int64_t *rowptr, const int32_t *col,
                            int64_t *n_block_rows, int64_t *n_tiles) {
  if (!n_block_rows || !n_tiles) return fail(TTDFT_ERR_NULL, "output pointer is NULL");
  ttdft_status st = check_csr(r, rowptr, col);
  if (st != TTDFT_OK) return st;
  Lattice L(r);
  std::vector<int32_t> tptr, tcol;
  block_pattern(L, rowptr, col, tptr, tcol);
  *n_block_rows = L.n_block_rows();
  *n_tiles = (int64_t)tcol.size();
  return ok();
}

ttdft_status ttdft_bsr_build_size(int32_t r, int32_t blk, const int64_t *rowptr, const int32_t *col,
                                  int64_t *n_tiles_out) {
  if (!n_tiles_out) return fail(TTDFT_ERR_NULL, "n_tiles_out is NULL");
  if (blk != 4) return fail(TTDFT_ERR_SHAPE, "tile extent blk = %d: only 4 (64-row tiles) is built", blk);
  int64_t nbr = 0;
  return ttdft_bsr_plan(r, rowptr, col, &nbr, n_tiles_out);
}

ttdft_status ttdft_bsr_build(int32_t r, const int64_t *rowptr, const int32_t *col,
                             const double *val, ttdft_dtype dtype, int32_t *tile_rowptr,
                             int32_t *tile_col, void *vals, int64_t *perm, int64_t *entry_slot,
                             uint64_t *mask, uint64_t *frag_mask) {
  if (!val || !tile_rowptr || !tile_col || !vals || !perm)
    return fail(TTDFT_ERR_NULL, "an output or val pointer is NULL");
  if (!valid_tile_dtype(dtype)) return fail(TTDFT_ERR_DTYPE, "dtype %d unknown", (int)dtype);
  ttdft_status st = check_csr(r, rowptr, col);
  if (st != TTDFT_OK) return st;
  Lattice L(r);
  const int64_t NB = L.n_block_rows(), N = (int64_t)r * r * r;
  std::vector<int32_t> tptr, tcol;
  block_pattern(L, rowptr, col, tptr, tcol);
  const int64_t nt = (int64_t)tcol.size();
  std::copy(tptr.begin(), tptr.end(), tile_rowptr);
  std::copy(tcol.begin(), tcol.end(), tile_col);
  std::memset(vals, 0, (size_t)nt * kTileElems * tile_value_bytes(dtype));
  if (mask) std::memset(mask, 0, (size_t)nt * 64 * sizeof(uint64_t));
  if (frag_mask) std::memset(frag_mask, 0, (size_t)nt * sizeof(uint64_t));
  for (int64_t p = 0; p < NB * 64; ++p) perm[p] = -1;
  for (int64_t I = 0; I < N; ++I) {
    int64_t b, l;
    L.split(I, b, l);
    perm[b * 64 + l] = I;
    for (int64_t p = rowptr[I]; p < rowptr[I + 1]; ++p) {
      int64_t bc, lc;
      L.split(col[p], bc, lc);
      const int32_t *first = tile_col + tptr[b], *last = tile_col + tptr[b + 1];
      const int64_t t = tptr[b] + (std::lower_bound(first, last, (int32_t)bc) - first);
      // fragment order of the tile type (16x4 for F64 / F32, 16x32 for BF16)
      const int64_t pos = tile_pos(dtype, (int)l, (int)lc);
      const int64_t slot = (dtype == TTDFT_BF16_SPLIT ? 2 : 1) * t * kTileElems + pos;
      if (dtype == TTDFT_F64) {
        ((double *)vals)[slot] = val[p];
      } else if (dtype == TTDFT_F32) {
        ((float *)vals)[slot] = (float)val[p];
      } else if (dtype == TTDFT_BF16) {
        ((uint16_t *)vals)[slot] = f32_to_bf16_rne((float)val[p]);
      } else {
        // hi + lo: the residual of fp32(h) - hi is exact in FP32
        const float h32 = (float)val[p];
        const uint16_t hi = f32_to_bf16_rne(h32);
        ((uint16_t *)vals)[slot] = hi;
        ((uint16_t *)vals)[slot + kTileElems] = f32_to_bf16_rne(h32 - bf16_to_f32(hi));
      }
      if (entry_slot) entry_slot[p] = slot;
      if (mask) mask[t * 64 + l] |= (uint64_t)1 << lc;
      if (frag_mask) frag_mask[t] |= (uint64_t)1 << (4 * (lc >> 2) + (l >> 4));
    }
  }
  return ok();
}

ttdft_status ttdft_cheb_step(const ttdft_bsr *H, const void *Yk, int64_t ldk, const void *Yprev,
                             int64_t ldp, void *Yout, int64_t ldo, int64_t n_vec, double alpha,
                             double c, double beta, ttdft_dtype x_dtype, void *stream) {
  ttdft_status st = check_bsr(H);
  if (st != TTDFT_OK) return st;
  if (!valid_dtype(x_dtype) || !supported_pair(H->dtype, x_dtype))
    return fail(TTDFT_ERR_DTYPE, "unsupported (H, X) dtype pair (%d, %d)", (int)H->dtype, (int)x_dtype);
  if (!Yk || !Yout) return fail(TTDFT_ERR_NULL, "Yk or Yout is NULL");
  if (beta != 0.0 && !Yprev) return fail(TTDFT_ERR_NULL, "Yprev is NULL with beta != 0");
  if (n_vec < 1) return fail(TTDFT_ERR_SHAPE, "n_vec = %lld < 1", (long long)n_vec);
  if (ldk < n_vec || ldo < n_vec || (Yprev && ldp < n_vec))
    return fail(TTDFT_ERR_SHAPE, "leading dimension smaller than n_vec");
  if (!step_ld_ok(ldk, dtype_size(x_dtype)))
    return fail(TTDFT_ERR_SHAPE, "ldk = %lld too large for 32-bit panel offsets", (long long)ldk);
  if (!std::isfinite(alpha) || !std::isfinite(c) || !std::isfinite(beta))
    return fail(TTDFT_ERR_NONFINITE, "alpha, c and beta must be finite");
  const int64_t rows = H->n_block_rows * 64;
  const size_t elt = dtype_size(x_dtype);
  const Span sk = span_of(Yk, rows, ldk, n_vec, elt), so = span_of(Yout, rows, ldo, n_vec, elt);
  if (overlap(sk, so)) return fail(TTDFT_ERR_ALIAS, "Yout overlaps Yk");
  if (Yprev && beta != 0.0) {
    const Span sp = span_of(Yprev, rows, ldp, n_vec, elt);
    if (overlap(sp, so) && !(Yprev == Yout && ldp == ldo))
      return fail(TTDFT_ERR_ALIAS, "Yout partially overlaps Yprev");
  }
  return hip_status(launch_cheb_step(*H, Yk, ldk, beta != 0.0 ? Yprev : nullptr, ldp, Yout, ldo,
                                     n_vec, alpha, c, beta, x_dtype, (hipStream_t)stream),
                    "cheb_step launch");
}

size_t ttdft_cheb_filter_workspace(const ttdft_bsr *H, int64_t n_vec, ttdft_dtype x_dtype) {
  if (!H || H->n_block_rows < 1 || n_vec < 1 || !valid_dtype(x_dtype)) return 0;
  return (size_t)H->n_block_rows * 64 * (size_t)n_vec * dtype_size(x_dtype);
}

}  // extern "C"

namespace ttdft {
// Validation of the filter's arguments shared by ttdft_cheb_filter and the
// variant without a workspace argument; writes nothing.
ttdft_status filter_check(const ttdft_bsr *H, const void *X, int64_t ldx, const void *Y,
                          int64_t ldy, int64_t n_vec, int32_t m, double a, double b, double a0,
                          ttdft_dtype x_dtype) {
  ttdft_status st = check_bsr(H);
  if (st != TTDFT_OK) return st;
  if (!valid_dtype(x_dtype) || !supported_pair(H->dtype, x_dtype))
    return fail(TTDFT_ERR_DTYPE, "unsupported (H, X) dtype pair (%d, %d)", (int)H->dtype, (int)x_dtype);
  if (!X || !Y) return fail(TTDFT_ERR_NULL, "X or Y is NULL");
  if (n_vec < 1) return fail(TTDFT_ERR_SHAPE, "n_vec = %lld < 1", (long long)n_vec);
  if (ldx < n_vec || ldy < n_vec) return fail(TTDFT_ERR_SHAPE, "leading dimension smaller than n_vec");
  if (!step_ld_ok(ldx, dtype_size(x_dtype)) || !step_ld_ok(ldy, dtype_size(x_dtype)))
    return fail(TTDFT_ERR_SHAPE, "leading dimension too large for 32-bit panel offsets");
  if (!(std::isfinite(a) && std::isfinite(b) && std::isfinite(a0)) || !(a0 < a && a < b))
    return fail(TTDFT_ERR_BOUNDS, "bounds must be finite with a0 < a < b (got a0=%g a=%g b=%g)", a0, a, b);
  if (m < 1) return fail(TTDFT_ERR_DEGREE, "degree m = %d < 1", m);
  const int64_t rows = H->n_block_rows * 64;
  const size_t elt = dtype_size(x_dtype);
  if (overlap(span_of(X, rows, ldx, n_vec, elt), span_of(Y, rows, ldy, n_vec, elt)))
    return fail(TTDFT_ERR_ALIAS, "Y overlaps X");
  return TTDFT_OK;
}

// The m launches of the filter (arguments already validated).  work holds one
// rows x n_vec block (leading dimension n_vec) when m >= 2.
ttdft_status filter_enqueue(const ttdft_bsr &H, const void *X, int64_t ldx, void *Y, int64_t ldy,
                            int64_t n_vec, int32_t m, double a, double b, double a0,
                            ttdft_dtype x_dtype, void *work, hipStream_t s) {
  return filter_enqueue_schedule(H, H, 0, X, ldx, Y, ldy, n_vec, m, a, b, a0, x_dtype, work, s);
}

// steps k < m - m_late take their product with H_early, the others with H_late
ttdft_status filter_enqueue_schedule(const ttdft_bsr &H_early, const ttdft_bsr &H_late, int32_t m_late,
                                     const void *X, int64_t ldx, void *Y, int64_t ldy, int64_t n_vec,
                                     int32_t m, double a, double b, double a0, ttdft_dtype x_dtype,
                                     void *work, hipStream_t s) {
  // coefficient schedule of Algorithm 1 (Sec. 3.4), FP64 on the host
  std::vector<double> alpha(m), beta(m);
  double c;
  cheb_coefficients(m, a, b, a0, &c, alpha.data(), beta.data());
  // Y_k for k >= 1 lives in Y when k has the parity of m, else in work, so the
  // last iterate lands in Y and Y_{k+1} overwrites Y_{k-1} in place.
  auto buf = [&](int k) -> void * { return (k % 2 == m % 2) ? Y : work; };
  auto ld_of = [&](int k) -> int64_t { return (k % 2 == m % 2) ? ldy : n_vec; };
  for (int k = 0; k < m; ++k) {
    const void *cur = k == 0 ? X : buf(k);
    const int64_t ldc = k == 0 ? ldx : ld_of(k);
    const void *prev = k == 0 ? nullptr : (k == 1 ? X : buf(k - 1));
    const int64_t ldp = k == 0 ? 0 : (k == 1 ? ldx : ld_of(k - 1));
    const ttdft_bsr &H = k < m - m_late ? H_early : H_late;
    hipError_t err = launch_cheb_step(H, cur, ldc, prev, ldp, buf(k + 1), ld_of(k + 1), n_vec,
                                      alpha[k], c, beta[k], x_dtype, s);
    if (err != hipSuccess) return hip_status(err, "cheb_filter step");
  }
  return ok();
}

}  // namespace ttdft

extern "C" {

ttdft_status ttdft_cheb_filter(const ttdft_bsr *H, const void *X, int64_t ldx, void *Y,
                               int64_t ldy, int64_t n_vec, int32_t m, double a, double b,
                               double a0, ttdft_dtype x_dtype, void *work, size_t work_bytes,
                               void *stream) {
  ttdft_status st = filter_check(H, X, ldx, Y, ldy, n_vec, m, a, b, a0, x_dtype);
  if (st != TTDFT_OK) return st;
  const int64_t rows = H->n_block_rows * 64;
  const size_t elt = dtype_size(x_dtype);
  const size_t need = ttdft_cheb_filter_workspace(H, n_vec, x_dtype);
  if (m >= 2 && (!work || work_bytes < need))
    return fail(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
  const Span sw = m >= 2 ? span_bytes(work, need) : Span{};
  if (overlap(sw, span_of(Y, rows, ldy, n_vec, elt)) || overlap(sw, span_of(X, rows, ldx, n_vec, elt)))
    return fail(TTDFT_ERR_ALIAS, "workspace overlaps X or Y");
  return filter_enqueue(*H, X, ldx, Y, ldy, n_vec, m, a, b, a0, x_dtype, work, (hipStream_t)stream);
}

ttdft_status ttdft_cheb_filter_schedule(const ttdft_bsr *H_early, const ttdft_bsr *H_late,
                                        int32_t m_late, const void *X, int64_t ldx, void *Y,
                                        int64_t ldy, int64_t n_vec, int32_t m, double a, double b,
                                        double a0, ttdft_dtype x_dtype, void *work,
                                        size_t work_bytes, void *stream) {
  ttdft_status st = filter_check(H_early, X, ldx, Y, ldy, n_vec, m, a, b, a0, x_dtype);
  if (st != TTDFT_OK) return st;
  st = filter_check(H_late, X, ldx, Y, ldy, n_vec, m, a, b, a0, x_dtype);
  if (st != TTDFT_OK) return st;
  if (H_early->n_block_rows != H_late->n_block_rows || H_early->n_tiles != H_late->n_tiles)
    return fail(TTDFT_ERR_SHAPE, "H_early and H_late must be the same blocked matrix "
                                 "(%lld/%lld block rows, %lld/%lld tiles)",
                (long long)H_early->n_block_rows, (long long)H_late->n_block_rows,
                (long long)H_early->n_tiles, (long long)H_late->n_tiles);
  if (m_late < 0 || m_late > m)
    return fail(TTDFT_ERR_DEGREE, "m_late = %d outside 0 .. m = %d", m_late, m);
  const int64_t rows = H_early->n_block_rows * 64;
  const size_t elt = dtype_size(x_dtype);
  const size_t need = ttdft_cheb_filter_workspace(H_early, n_vec, x_dtype);
  if (m >= 2 && (!work || work_bytes < need))
    return fail(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
  const Span sw = m >= 2 ? span_bytes(work, need) : Span{};
  if (overlap(sw, span_of(Y, rows, ldy, n_vec, elt)) || overlap(sw, span_of(X, rows, ldx, n_vec, elt)))
    return fail(TTDFT_ERR_ALIAS, "workspace overlaps X or Y");
  return filter_enqueue_schedule(*H_early, *H_late, m_late, X, ldx, Y, ldy, n_vec, m, a, b, a0,
                                 x_dtype, work, (hipStream_t)stream);
}

size_t ttdft_check_finite_workspace(void) { return 16; }

ttdft_status ttdft_check_finite(const void *A, ttdft_dtype dtype, int64_t rows, int64_t cols,
                                int64_t ld, int64_t *n_nonfinite, void *work, size_t work_bytes,
                                void *stream) {
  if (!valid_dtype(dtype)) return fail(TTDFT_ERR_DTYPE, "unknown dtype");
  if (!n_nonfinite) return fail(TTDFT_ERR_NULL, "n_nonfinite is NULL");
  if (rows < 0 || cols < 0 || ld < cols) return fail(TTDFT_ERR_SHAPE, "bad block shape");
  if (rows > 0 && cols > 0 && !A) return fail(TTDFT_ERR_NULL, "A is NULL");
  if (!work || work_bytes < 16) return fail(TTDFT_ERR_WORKSPACE, "workspace of 16 bytes needed");
  if (rows == 0 || cols == 0) {
    *n_nonfinite = 0;
    return ok();
  }
  if (overlap(span_of(A, rows, ld, cols, dtype_size(dtype)), span_bytes(work, 16)))
    return fail(TTDFT_ERR_ALIAS, "workspace overlaps the block");
  hipStream_t s = (hipStream_t)stream;
  unsigned long long *cnt = (unsigned long long *)work;
  hipError_t e = launch_clear_ints((int *)work, 2, s);
  if (e == hipSuccess) e = launch_count_nonfinite(A, dtype, ld, rows, cols, cnt, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  unsigned long long h = 0;
  if (e == hipSuccess) e = hipMemcpy(&h, cnt, sizeof h, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_status(e, "check_finite");
  *n_nonfinite = (int64_t)h;
  if (h) return fail(TTDFT_ERR_NONFINITE, "%llu non-finite entries", h);
  return ok();
}

ttdft_status ttdft_cast(const void *src, ttdft_dtype src_dtype, int64_t lds, void *dst,
                        ttdft_dtype dst_dtype, int64_t ldd, int64_t rows, int64_t cols,
                        void *stream) {
  if (!valid_dtype(src_dtype) || !valid_dtype(dst_dtype))
    return fail(TTDFT_ERR_DTYPE, "unknown dtype");
  if (rows < 0 || cols < 0 || lds < cols || ldd < cols)
    return fail(TTDFT_ERR_SHAPE, "bad cast shape");
  if (rows == 0 || cols == 0) return ok();
  if (!src || !dst) return fail(TTDFT_ERR_NULL, "src or dst is NULL");
  if (overlap(span_of(src, rows, lds, cols, dtype_size(src_dtype)),
              span_of(dst, rows, ldd, cols, dtype_size(dst_dtype))))
    return fail(TTDFT_ERR_ALIAS, "cast buffers overlap");
  return hip_status(launch_cast(src, src_dtype, lds, dst, dst_dtype, ldd, rows, cols,
                                (hipStream_t)stream), "cast launch");
}

ttdft_status ttdft_split_bf16(const double *src, int64_t n_tiles, void *dst, void *stream) {
  if (!src || !dst) return fail(TTDFT_ERR_NULL, "src or dst is NULL");
  if (n_tiles < 0) return fail(TTDFT_ERR_SHAPE, "n_tiles = %lld", (long long)n_tiles);
  if (overlap(span_bytes(src, (size_t)n_tiles * kTileElems * 8), span_bytes(dst, (size_t)n_tiles * kTileElems * 4)))
    return fail(TTDFT_ERR_ALIAS, "src and dst overlap");
  return hip_status(launch_split_bf16(src, n_tiles, dst, (hipStream_t)stream), "split launch");
}

ttdft_status ttdft_convert_tiles(const void *src, ttdft_dtype src_dtype, int64_t n_tiles, void *dst,
                                 ttdft_dtype dst_dtype, void *stream) {
  if (!src || !dst) return fail(TTDFT_ERR_NULL, "src or dst is NULL");
  if (n_tiles < 0) return fail(TTDFT_ERR_SHAPE, "n_tiles = %lld", (long long)n_tiles);
  if (!(src_dtype == TTDFT_F64 || src_dtype == TTDFT_F32) ||
      !(dst_dtype == TTDFT_F32 || dst_dtype == TTDFT_BF16 || dst_dtype == TTDFT_BF16_SPLIT) ||
      src_dtype == dst_dtype)
    return fail(TTDFT_ERR_DTYPE, "tile conversion %d -> %d not supported", (int)src_dtype, (int)dst_dtype);
  const size_t nb_src = (size_t)n_tiles * kTileElems * dtype_size(src_dtype);
  const size_t nb_dst = (size_t)n_tiles * kTileElems * tile_value_bytes(dst_dtype);
  if (overlap(span_bytes(src, nb_src), span_bytes(dst, nb_dst)))
    return fail(TTDFT_ERR_ALIAS, "src and dst overlap");
  return hip_status(launch_convert_tiles(src, src_dtype, n_tiles, dst, dst_dtype, (hipStream_t)stream),
                    "convert_tiles launch");
}

ttdft_status ttdft_gather_rows(const void *src, int64_t lds, int64_t rows_src, void *dst,
                               int64_t ldd, int64_t rows_dst, int64_t cols, const int64_t *perm,
                               ttdft_dtype dtype, void *stream) {
  if (!valid_dtype(dtype)) return fail(TTDFT_ERR_DTYPE, "unknown dtype");
  if (rows_src < 0 || rows_dst < 0 || cols < 0 || lds < cols || ldd < cols)
    return fail(TTDFT_ERR_SHAPE, "bad gather shape");
  if (rows_dst == 0 || cols == 0) return ok();
  if (!src || !dst || !perm) return fail(TTDFT_ERR_NULL, "src, dst or perm is NULL");
  const size_t elt = dtype_size(dtype);
  if (overlap(span_of(src, rows_src, lds, cols, elt), span_of(dst, rows_dst, ldd, cols, elt)))
    return fail(TTDFT_ERR_ALIAS, "gather buffers overlap");
  return hip_status(launch_gather_rows(src, lds, dst, ldd, rows_dst, cols, perm, elt,
                                       (hipStream_t)stream), "gather launch");
}

}  // extern "C"
