// Upper bound of the spectrum of H for the Chebyshev filter's interval [a, b]
// (Sec. 3.4 needs an upper bound of the unwanted spectrum) by k steps of the
// Lanczos process on a random start vector:
//     w = H v_j - beta_j v_{j-1},  alpha_j = w . v_j,  w -= alpha_j v_j,
//     beta_{j+1} = |w|,  v_{j+1} = w / beta_{j+1},
// then theta_max, the largest eigenvalue of the k x k tridiagonal T_k (bisection
// on Sturm counts), the Ritz-residual estimate theta_max + |beta_{k+1} s_k| and
// the safeguarded bound theta_max + beta_{k+1}.  The product H v uses
// the fused step kernel with alpha = 1, c = 0, beta = 0 on one vector; the
// reductions run in a single work-group in a fixed order (deterministic).
//
// Breakdown: when some beta_{j+1} vanishes (to rounding, relative to the size of
// T_k) the Krylov space is an invariant subspace of H after j steps.  T_j then
// holds exact eigenvalues of H, but not necessarily its extreme ones, and the
// steps after it would only append spurious zero rows.  The bounds are then
// taken from T_j and widened to the Gershgorin interval of H (every eigenvalue
// lies in some row's disc [H_ii - r_i, H_ii + r_i], r_i = sum_{j != i} |H_ij|).
// With k at least the number of real rows the Krylov space is invariant for
// certain, but in floating point beta need not fall below the threshold (the
// Lanczos vectors lose orthogonality and the process runs on with copies of
// converged Ritz values), so that case takes the Gershgorin widening as well.
#include <algorithm>
#include <cmath>
#include <vector>

#include "ttdft_internal.h"

namespace ttdft {
namespace {

__device__ inline double unit_random(uint64_t i, uint64_t seed) {
  uint64_t h = (i + 0x9E3779B97F4A7C15ull * (seed + 1)) * 0xBF58476D1CE4E5B9ull;
  h ^= h >> 31;
  h *= 0x94D049BB133111EBull;
  h ^= h >> 29;
  return (double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

// v[i] = random for real rows, 0 for padding rows (perm[i] < 0)
__global__ void lz_start_kernel(double *v, int64_t rows, const int64_t *perm, uint64_t seed) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256)
    v[i] = perm[i] >= 0 ? unit_random((uint64_t)perm[i], seed) : 0.0;
}

__device__ inline double wg_sum(double s, double *red) {
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < 16; ++w) t += red[w];
  __syncthreads();
  return t;
}

// out = a . b  (one work-group of 1024 threads, fixed summation order)
__global__ __launch_bounds__(1024) void lz_dot_kernel(const double *a, const double *b,
                                                      int64_t rows, double *out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 1024) s += a[i] * b[i];
  const double t = wg_sum(s, red);
  if (threadIdx.x == 0) *out = t;
}

// w -= alpha_j v_j + beta_j v_{j-1}  (vprev may be NULL for j = 0)
__global__ void lz_update_kernel(double *w, const double *v, const double *vprev,
                                 const double *alpha_j, const double *beta_j, int64_t rows) {
  const double al = *alpha_j, be = vprev ? *beta_j : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < rows; i += (int64_t)gridDim.x * 256)
    w[i] -= al * v[i] + (vprev ? be * vprev[i] : 0.0);
}

// beta = |w|; v_next = w / beta (v_next = 0 when w = 0: a breakdown, which the
// host detects from beta and handles by truncating T_k)
__global__ __launch_bounds__(1024) void lz_normalize_kernel(const double *w, double *v_next,
                                                            int64_t rows, double *beta) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 1024) s += w[i] * w[i];
  const double nrm = sqrt(wg_sum(s, red));
  if (threadIdx.x == 0) *beta = nrm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 1024) v_next[i] = w[i] * inv;
}

// number of eigenvalues of the tridiagonal (alpha, beta[1..k-1]) below x
__device__ inline int tri_count(const double *alpha, const double *beta, int k, double x) {
  int cnt = 0;
  double q = alpha[0] - x;
  for (int i = 0; i < k; ++i) {
    if (i > 0) q = (alpha[i] - x) - beta[i] * beta[i] / q;
    if (fabs(q) < 1e-300) q = -1e-300;
    cnt += q < 0.0;
  }
  return cnt;
}

// largest eigenvalue theta of T_k by bisection; the last component s_k of its
// normalised eigenvector by the three-term recurrence of the tridiagonal
// (rescaled against overflow); out = {theta, theta + |beta_{k+1} s_k|,
// theta + beta_{k+1}, theta_min} with theta_min the smallest eigenvalue of T_k
__global__ void lz_bound_kernel(const double *alpha, const double *beta, int k, double *out) {
  if (threadIdx.x != 0) return;
  double lo = alpha[0], hi = alpha[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(beta[i]) : 0.0) + (i + 1 < k ? fabs(beta[i + 1]) : 0.0);
    lo = fmin(lo, alpha[i] - r);
    hi = fmax(hi, alpha[i] + r);
  }
  for (int it = 0; it < 200 && hi - lo > 1e-15 * fmax(fabs(lo), fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (tri_count(alpha, beta, k, mid) >= k) hi = mid;   // all eigenvalues below mid
    else lo = mid;
  }
  const double theta = hi;   // upper end of its bracket
  // smallest eigenvalue: the lowest x with at least one eigenvalue below it
  double lo1 = alpha[0], hi1 = alpha[0];
  for (int i = 0; i < k; ++i) {
    const double r = (i > 0 ? fabs(beta[i]) : 0.0) + (i + 1 < k ? fabs(beta[i + 1]) : 0.0);
    lo1 = fmin(lo1, alpha[i] - r);
    hi1 = fmax(hi1, alpha[i] + r);
  }
  for (int it = 0; it < 200 && hi1 - lo1 > 1e-15 * fmax(fabs(lo1), fabs(hi1)); ++it) {
    const double mid = 0.5 * (lo1 + hi1);
    if (mid == lo1 || mid == hi1) break;
    if (tri_count(alpha, beta, k, mid) >= 1) hi1 = mid;
    else lo1 = mid;
  }
  double sp = 0.0, sc = 1.0, n2 = 1.0;
  for (int i = 0; i + 1 < k; ++i) {
    if (beta[i + 1] == 0.0) { sc = 0.0; break; }    // T_k splits: residual 0
    const double sn = ((theta - alpha[i]) * sc - (i > 0 ? beta[i] * sp : 0.0)) / beta[i + 1];
    sp = sc;
    sc = sn;
    n2 += sn * sn;
    if (n2 > 1e200) { sp *= 1e-100; sc *= 1e-100; n2 *= 1e-200; }
  }
  const double last = fabs(sc) / sqrt(n2);
  out[0] = theta;
  out[1] = theta + fabs(beta[k]) * last;
  out[2] = theta + fabs(beta[k]);
  out[3] = lo1;   // lower end of its bracket
}

// Gershgorin discs of the real rows of block row B (one work-group of 64
// threads, thread i = local row i): lo[B] = min_i (H_ii - r_i), hi[B] =
// max_i (H_ii + r_i) over rows with perm >= 0 (padding rows are skipped; a
// block row of padding only writes +inf / -inf).  Tile values are in fragment
// order: entry (i, j) of tile t at 64*(4*(j/4) + i/16) + 16*(j%4) + i%16.
__global__ __launch_bounds__(64) void gershgorin_kernel(const int32_t *rowptr, const int32_t *tcol,
                                                        const double *vals, const int64_t *perm,
                                                        double *lo, double *hi) {
  const int64_t B = blockIdx.x;
  const int i = threadIdx.x;
  double diag = 0.0, rad = 0.0;
  for (int t = rowptr[B]; t < rowptr[B + 1]; ++t) {
    const double *tile = vals + (int64_t)t * 4096;
    const bool dtile = tcol[t] == B;
    for (int j = 0; j < 64; ++j) {
      const double v = tile[64 * (4 * (j >> 2) + (i >> 4)) + 16 * (j & 3) + (i & 15)];
      if (dtile && j == i) diag = v;
      else rad += fabs(v);
    }
  }
  const bool real = perm[B * 64 + i] >= 0;
  double l = real ? diag - rad : INFINITY, h = real ? diag + rad : -INFINITY;
  for (int o = 32; o > 0; o >>= 1) {
    l = fmin(l, __shfl_down(l, o, 64));
    h = fmax(h, __shfl_down(h, o, 64));
  }
  if (i == 0) {
    lo[B] = l;
    hi[B] = h;
  }
}

// out = number of real rows (perm >= 0), as a double (one work-group, exact
// below 2^53)
__global__ __launch_bounds__(1024) void count_real_kernel(const int64_t *perm, int64_t rows, double *out) {
  __shared__ double red[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < rows; i += 1024) s += perm[i] >= 0 ? 1.0 : 0.0;
  const double t = wg_sum(s, red);
  if (threadIdx.x == 0) *out = t;
}

// out[0] = min(lo), out[1] = max(hi) over nb entries (one work-group)
__global__ __launch_bounds__(1024) void minmax_kernel(const double *lo, const double *hi, int64_t nb,
                                                      double *out) {
  __shared__ double sl[16], sh[16];
  double l = INFINITY, h = -INFINITY;
  for (int64_t b = threadIdx.x; b < nb; b += 1024) {
    l = fmin(l, lo[b]);
    h = fmax(h, hi[b]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    l = fmin(l, __shfl_down(l, o, 64));
    h = fmax(h, __shfl_down(h, o, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    sl[threadIdx.x >> 6] = l;
    sh[threadIdx.x >> 6] = h;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) {
      l = fmin(l, sl[w]);
      h = fmax(h, sh[w]);
    }
    l = fmin(l, sl[0]);
    h = fmax(h, sh[0]);
    out[0] = l;
    out[1] = h;
  }
}

}  // namespace

size_t lanczos_work_bytes(int64_t rows, int k) {
  return (size_t)(3 * rows + 2 * (k + 2) + 4 + 2 * (rows / 64) + 3) * sizeof(double);
}

// work: 3 vectors + alpha[k+1] + beta[k+2] + out[4] + Gershgorin lo/hi per block
// row + 2 + the count of real rows
hipError_t run_lanczos_bound(const ttdft_bsr &H, const int64_t *perm, int k, uint64_t seed,
                             void *work, hipStream_t s, double host_out[4], int *breakdown) {
  const int64_t rows = H.n_block_rows * 64;
  double *v0 = (double *)work, *v1 = v0 + rows, *w = v1 + rows;
  double *alpha = w + rows, *beta = alpha + (k + 1), *out = beta + (k + 2);
  double *glo = out + 4, *ghi = glo + H.n_block_rows, *gout = ghi + H.n_block_rows;
  double *n_real = gout + 2;
  *breakdown = 0;
  hipLaunchKernelGGL(count_real_kernel, dim3(1), dim3(1024), 0, s, perm, rows, n_real);
  const unsigned g = (unsigned)std::min<int64_t>((rows + 255) / 256, 4096);
  hipLaunchKernelGGL(lz_start_kernel, dim3(g), dim3(256), 0, s, w, rows, perm, seed);
  hipLaunchKernelGGL(lz_normalize_kernel, dim3(1), dim3(1024), 0, s, w, v0, rows, beta);
  double *vprev = nullptr, *vcur = v0, *vnext = v1;
  for (int j = 0; j < k; ++j) {
    hipError_t e = launch_cheb_step(H, vcur, 1, nullptr, 0, w, 1, 1, 1.0, 0.0, 0.0, TTDFT_F64, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lz_dot_kernel, dim3(1), dim3(1024), 0, s, w, vcur, rows, alpha + j);
    hipLaunchKernelGGL(lz_update_kernel, dim3(g), dim3(256), 0, s, w, vcur, vprev, alpha + j,
                       beta + j, rows);
    // beta[j+1] = |w|, v_{j+1} = w / beta[j+1]; the next step's vprev is vcur
    double *target = vprev ? vprev : vnext;
    hipLaunchKernelGGL(lz_normalize_kernel, dim3(1), dim3(1024), 0, s, w, target, rows, beta + j + 1);
    vprev = vcur;
    vcur = target;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // breakdown test on the host: the first beta_{j+1}, j < k, that vanishes
  // relative to the size of T_k ends the usable tridiagonal at order j + 1
  std::vector<double> ha(k), hb(k + 1);
  double hn_real = 0.0;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  if ((e = hipMemcpy(&hn_real, n_real, sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  if ((e = hipMemcpy(ha.data(), alpha, k * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  if ((e = hipMemcpy(hb.data(), beta, (k + 1) * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  double scale = 0.0;
  for (int j = 0; j < k; ++j) scale = std::max(scale, std::fabs(ha[j]) + std::fabs(hb[j + 1]));
  int k_eff = k;
  for (int j = 0; j + 1 < k; ++j)
    if (!(std::fabs(hb[j + 1]) > 1e-12 * scale)) {
      k_eff = j + 1;
      break;
    }
  hipLaunchKernelGGL(lz_bound_kernel, dim3(1), dim3(64), 0, s, alpha, beta, k_eff, out);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  if ((e = hipMemcpy(host_out, out, 4 * sizeof(double), hipMemcpyDeviceToHost)) != hipSuccess) return e;
  if (k_eff < k || !(std::fabs(hb[k]) > 1e-12 * scale) || (double)k >= hn_real) {
    *breakdown = 1;
    hipLaunchKernelGGL(gershgorin_kernel, dim3((unsigned)H.n_block_rows), dim3(64), 0, s,
                       H.tile_rowptr, H.tile_col, (const double *)H.vals, perm, glo, ghi);
    hipLaunchKernelGGL(minmax_kernel, dim3(1), dim3(1024), 0, s, glo, ghi, H.n_block_rows, gout);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    double g[2];
    if ((e = hipMemcpy(g, gout, sizeof g, hipMemcpyDeviceToHost)) != hipSuccess) return e;
    host_out[1] = std::max(host_out[1], g[1]);
    host_out[2] = std::max(host_out[2], g[1]);
    host_out[3] = std::min(host_out[3], g[0]);
  }
  return hipSuccess;
}

}  // namespace ttdft
