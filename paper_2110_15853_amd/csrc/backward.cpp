// Adjoint of the Chebyshev filter (step 1 of Algorithm 1, Sec. 3.4).
//
// Forward: Y_0 = X, Y_{k+1} = alpha_k (H - cI) Y_k - beta_k Y_{k-1} (beta_0 = 0),
// output Y_m.  For a loss with dL/dY_m = dY the reverse sweep is
//     Ybar_m = dY,
//     Ybar_k = alpha_k (H - cI) Ybar_{k+1} - beta_{k+1} Ybar_{k+2}   (H symmetric,
//              beta_m = 0, Ybar_{m+1} = 0),
//     dX = Ybar_0,   dH = sum_k alpha_k Ybar_{k+1} Y_k^T  on the pattern of H.
// The reverse recurrence reuses the fused forward step kernel; dH is
// accumulated by the tile SDDMM in a fixed order.  The forward iterates Y_k are
// either all stored (ckpt_every = 0) or stored as pairs (Y_{js}, Y_{js+1}) and
// recomputed per segment of s steps by the same deterministic kernel, so both
// modes give bitwise identical gradients.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "ttdft_internal.h"

using namespace ttdft;

namespace ttdft {
ttdft_status api_fail(ttdft_status s, const char *msg);
ttdft_status api_ok();
}  // namespace ttdft

namespace {

thread_local char g_msg[256];

ttdft_status failf(ttdft_status s, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof g_msg, fmt, ap);
  va_end(ap);
  return api_fail(s, g_msg);
}

bool valid_dtype(int t) { return t == TTDFT_F64 || t == TTDFT_F32 || t == TTDFT_BF16; }
bool supported_pair(ttdft_dtype h, ttdft_dtype x) {
  return (h == TTDFT_F64 && x == TTDFT_F64) || (h == TTDFT_F32 && x == TTDFT_F32) ||
         (h == TTDFT_BF16 && (x == TTDFT_F32 || x == TTDFT_BF16));
}
size_t block_bytes(int64_t rows, int64_t ld, int64_t cols, size_t elt) {
  return rows <= 0 || cols <= 0 ? 0 : (size_t)((rows - 1) * ld + cols) * elt;
}
bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  if (!a || !b || !na || !nb) return false;
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return x < y + nb && y < x + na;
}

// storage plan of the forward iterates Y_1 .. Y_{m-1}
struct Plan {
  int m, s;                 // s = 0: store all
  std::vector<int> slot;    // slot index of Y_k (k >= 1)
  int n_slots;
  Plan(int m_, int s_) : m(m_), s(s_), slot(m_ + 1, -1), n_slots(0) {
    if (s <= 2) {  // every iterate is a checkpoint
      for (int k = 1; k < m; ++k) slot[k] = n_slots++;
      return;
    }
    for (int k = 1; k < m; ++k)
      if (k % s <= 1) slot[k] = n_slots++;
    const int seg0 = n_slots;
    for (int k = 1; k < m; ++k)
      if (k % s >= 2) slot[k] = seg0 + (k % s) - 2;
    n_slots = seg0 + (m > 2 ? std::min(s - 2, m - 2) : 0);
  }
  bool stored(int k) const { return s <= 2 || k % s <= 1; }
};

}  // namespace

extern "C" {

size_t ttdft_cheb_filter_backward_workspace(const ttdft_bsr *H, int64_t n_vec, int32_t m,
                                            int32_t ckpt_every, ttdft_dtype x_dtype) {
  if (!H || H->n_block_rows < 1 || n_vec < 1 || m < 1 || ckpt_every < 0 || !valid_dtype(x_dtype))
    return 0;
  const size_t blk = (size_t)H->n_block_rows * 64 * n_vec * dtype_size(x_dtype);
  const Plan P(m, ckpt_every);
  return blk * (size_t)(1 + P.n_slots);
}

ttdft_status ttdft_cheb_filter_backward(const ttdft_bsr *H, const void *X, int64_t ldx,
                                        const void *dY, int64_t lddy, int64_t n_vec, int32_t m,
                                        double a, double b, double a0, ttdft_dtype x_dtype,
                                        int32_t ckpt_every, void *dX, int64_t lddx,
                                        void *dH_vals, const uint64_t *mask, void *work,
                                        size_t work_bytes, void *stream) {
  if (!H) return failf(TTDFT_ERR_NULL, "H is NULL");
  if (!valid_dtype(H->dtype) || !valid_dtype(x_dtype) || !supported_pair(H->dtype, x_dtype))
    return failf(TTDFT_ERR_DTYPE, "unsupported (H, X) dtype pair");
  if (H->n_block_rows < 1 || H->n_tiles < 0) return failf(TTDFT_ERR_SHAPE, "bad H shape");
  if (!H->tile_rowptr || (H->n_tiles > 0 && (!H->tile_col || !H->vals)))
    return failf(TTDFT_ERR_NULL, "H arrays are NULL");
  if (!X || !dY || !dX || !dH_vals) return failf(TTDFT_ERR_NULL, "X, dY, dX or dH_vals is NULL");
  if (n_vec < 1 || ldx < n_vec || lddy < n_vec || lddx < n_vec)
    return failf(TTDFT_ERR_SHAPE, "leading dimension smaller than n_vec");
  if (!step_ld_ok(ldx, dtype_size(x_dtype)) || !step_ld_ok(lddy, dtype_size(x_dtype)) ||
      !step_ld_ok(lddx, dtype_size(x_dtype)))
    return failf(TTDFT_ERR_SHAPE, "leading dimension too large for 32-bit panel offsets");
  if (!(std::isfinite(a) && std::isfinite(b) && std::isfinite(a0)) || !(a0 < a && a < b))
    return failf(TTDFT_ERR_BOUNDS, "bounds must be finite with a0 < a < b");
  if (m < 1) return failf(TTDFT_ERR_DEGREE, "degree m = %d < 1", m);
  if (ckpt_every < 0) return failf(TTDFT_ERR_SHAPE, "ckpt_every must be >= 0");
  const int64_t rows = H->n_block_rows * 64;
  const size_t elt = dtype_size(x_dtype);
  const size_t need = ttdft_cheb_filter_backward_workspace(H, n_vec, m, ckpt_every, x_dtype);
  if (!work || work_bytes < need) return failf(TTDFT_ERR_WORKSPACE, "workspace of %zu bytes needed", need);
  const size_t xb = block_bytes(rows, ldx, n_vec, elt), yb = block_bytes(rows, lddy, n_vec, elt),
               db = block_bytes(rows, lddx, n_vec, elt);
  const size_t hb = (size_t)H->n_tiles * kTileElems * (x_dtype == TTDFT_F64 ? 8 : 4);
  if (overlap(dX, db, X, xb) || overlap(dX, db, dY, yb) || overlap(dX, db, work, need))
    return failf(TTDFT_ERR_ALIAS, "dX overlaps an input or the workspace");
  if (overlap(dH_vals, hb, X, xb) || overlap(dH_vals, hb, dY, yb) || overlap(dH_vals, hb, dX, db) ||
      overlap(dH_vals, hb, work, need) || overlap(dH_vals, hb, H->vals, hb))
    return failf(TTDFT_ERR_ALIAS, "dH overlaps another buffer");
  if (overlap(work, need, X, xb) || overlap(work, need, dY, yb))
    return failf(TTDFT_ERR_ALIAS, "workspace overlaps X or dY");

  std::vector<double> alpha(m), beta(m + 1, 0.0);
  double c;
  cheb_coefficients(m, a, b, a0, &c, alpha.data(), beta.data());
  beta[m] = 0.0;
  hipStream_t s = (hipStream_t)stream;
  const size_t blk = (size_t)rows * n_vec * elt;
  char *w = (char *)work;
  void *rev = w;                                   // reverse-sweep ping-pong partner of dX
  const Plan plan(m, ckpt_every);
  auto Yp = [&](int k) -> const void * { return k == 0 ? X : (const void *)(w + blk * (1 + plan.slot[k])); };
  auto Yw = [&](int k) -> void * { return w + blk * (1 + plan.slot[k]); };
  auto Yld = [&](int k) -> int64_t { return k == 0 ? ldx : n_vec; };
  auto fwd = [&](int k) -> hipError_t {            // Y_{k+1} from Y_k, Y_{k-1}
    return launch_cheb_step(*H, Yp(k), Yld(k), k == 0 ? nullptr : Yp(k - 1), k == 0 ? 0 : Yld(k - 1),
                            Yw(k + 1), n_vec, n_vec, alpha[k], c, beta[k], x_dtype, s);
  };
  hipError_t e;
  // forward pass: Y_1 .. Y_{m-1}
  for (int k = 0; k + 1 < m; ++k)
    if ((e = fwd(k)) != hipSuccess) return failf(TTDFT_ERR_HIP, "backward: forward step: %s", hipGetErrorString(e));
  // reverse sweep
  auto bar = [&](int j) -> void * { return j % 2 == 0 ? dX : rev; };
  auto bar_ld = [&](int j) -> int64_t { return j % 2 == 0 ? lddx : n_vec; };
  auto barc = [&](int j) -> const void * { return j == m ? dY : bar(j); };
  auto barc_ld = [&](int j) -> int64_t { return j == m ? lddy : bar_ld(j); };
  for (int k = m - 1; k >= 0; --k) {
    if (!plan.stored(k) && k > 0) {
      const int S = plan.s, js = (k / S) * S;
      if (k == std::min(m - 1, js + S - 1)) {       // entering a segment: recompute its interior
        for (int q = js + 1; q < k; ++q)
          if ((e = fwd(q)) != hipSuccess) return failf(TTDFT_ERR_HIP, "backward: recompute: %s", hipGetErrorString(e));
      }
    }
    e = launch_sddmm(*H, barc(k + 1), barc_ld(k + 1), Yp(k), Yld(k), n_vec, alpha[k], dH_vals, mask,
                     k != m - 1, x_dtype, s);
    if (e != hipSuccess) return failf(TTDFT_ERR_HIP, "backward: sddmm: %s", hipGetErrorString(e));
    const bool has_prev = k + 2 <= m;
    e = launch_cheb_step(*H, barc(k + 1), barc_ld(k + 1), has_prev ? barc(k + 2) : nullptr,
                         has_prev ? barc_ld(k + 2) : 0, bar(k), bar_ld(k), n_vec, alpha[k], c,
                         beta[k + 1], x_dtype, s);
    if (e != hipSuccess) return failf(TTDFT_ERR_HIP, "backward: reverse step: %s", hipGetErrorString(e));
  }
  return api_ok();
}

}  // extern "C"
