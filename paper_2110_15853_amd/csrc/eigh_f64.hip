// Dense symmetric eigensolver in FP64 for the projected matrix H_F of step 4 of
// Algorithm 1 (Sec. 3.4):  H_F Z = Z diag(lambda), lambda ascending.
//
//  1. Householder tridiagonalisation H_F = Q T Q^T, one reflector per column
//     (reflector, symmetric product, correction vector, rank-2 update), the
//     rank-2 update of each step fused with the next step's reflector and
//     product (one launch per step);
//  2. eigenvalues of T by multisection on Sturm counts, one wave per eigenvalue
//     (64 points per step);
//  3. eigenvectors of T by inverse iteration (tridiagonal LU with partial
//     pivoting), one eigenvector per thread, from pseudo-random starts;
//  4. Cholesky-QR twice on the eigenvector block (matrix-core GEMMs), which
//     restores orthogonality lost between close eigenvalues; mixing inside such
//     a group changes residuals only in proportion to the gap;
//  5. back-transformation Z = Q Z_T by the reflectors in reverse order.
// Every stage is parallel across the matrix or across eigenpairs except the
// sequence of n-2 reflectors.
#include "ttdft_internal.h"

namespace ttdft {
namespace {

constexpr double EPS = 2.220446049250313e-16;
constexpr double SAFMIN = 2.2250738585072014e-308;

template <int NT> __device__ inline double block_sum(double v, double *red) {
  // wave reduction then across waves through LDS
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    red[NT / 64] = s;
  }
  __syncthreads();
  s = red[NT / 64];
  __syncthreads();
  return s;
}

__global__ void copy_matrix_kernel(const double *A, int64_t lda, double *B, int64_t ldb, int64_t n) {
  const int64_t total = n * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / n, j = e % n;
    B[i * ldb + j] = A[i * lda + j];
  }
}

// Householder reflector of row k, x = A[k][k+1:n]: beta = -sign(x0) |x|,
// tau = (beta - x0)/beta, v = x/(x0 - beta) with v0 = 1 (tau = 0 when x1: = 0).
// Every work-group of the product kernel computes it from the unmodified row;
// work-group 0 stores v (row k of V), tau, d[k] and e[k].
__device__ inline void reflector(const double *x, int64_t m, double *red, double &tau_k,
                                 double &scale, double &beta) {
  double s = 0.0;
  for (int64_t i = 1 + threadIdx.x; i < m; i += 256) s += x[i] * x[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double xn2 = red[0] + red[1] + red[2] + red[3];
  const double alpha = x[0];
  if (xn2 == 0.0) {
    tau_k = 0.0;
    beta = alpha;
    scale = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    tau_k = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
}

// p = tau * A22 v (one wave per row of the trailing block); pv[b] = the sum of
// p_r v_r over the rows of work-group b
__global__ __launch_bounds__(256) void house_symv_kernel(const double *A, int64_t n, int64_t k,
                                                         double *V, double *tau, double *d,
                                                         double *e, double *p, double *pv,
                                                         int *nonfinite) {
  __shared__ double red[4];
  const int64_t m = n - k - 1;
  const double *x = A + k * n + k + 1;
  double t, scale, beta;
  reflector(x, m, red, t, scale, beta);
  if (blockIdx.x == 0) {
    double *v = V + k * n + k + 1;
    for (int64_t i = threadIdx.x; i < m; i += 256) v[i] = i == 0 ? 1.0 : x[i] * scale;
    if (threadIdx.x == 0) {
      if (!isfinite(beta) || !isfinite(t)) atomicExch(nonfinite, 1);
      tau[k] = t;
      d[k] = A[k * n + k];
      e[k] = beta;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r = (int64_t)blockIdx.x * 4 + wv;
  __shared__ double part[4];
  double pvr = 0.0;
  if (r < m) {
    const double *row = A + (k + 1 + r) * n + k + 1;
    double s = 0.0;
    for (int64_t j = lane; j < m; j += 64) s += row[j] * (j == 0 ? 1.0 : x[j] * scale);
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    const double pi = t * s;
    pvr = pi * (r == 0 ? 1.0 : x[r] * scale);
    if (lane == 0) p[r] = pi;
  }
  if (lane == 0) part[wv] = pvr;
  __syncthreads();
  // pv holds one partial sum of p.v per work-group, summed in a fixed order later
  if (threadIdx.x == 0) pv[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// A22 -= v w^T + w v^T with w = p - (tau/2)(p.v) v; each work-group sums the
// per-work-group partials of p.v (fixed order) and updates a band of 4 rows
__global__ __launch_bounds__(256) void rank2_fused_kernel(double *A, int64_t n, int64_t k,
                                                          const double *V, const double *tau,
                                                          const double *p, const double *pv) {
  __shared__ double red[4];
  const int64_t m = n - k - 1, nparts = (m + 3) / 4;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += 256) s += pv[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double K = 0.5 * tau[k] * (red[0] + red[1] + red[2] + red[3]);
  const double *v = V + k * n + k + 1;
  const int64_t r0 = (int64_t)blockIdx.x * 4, r1 = min(m, r0 + 4);
  for (int64_t i = r0; i < r1; ++i) {
    const double vi = v[i], wi = p[i] - K * vi;
    double *row = A + (k + 1 + i) * n + k + 1;
    for (int64_t j = threadIdx.x; j < m; j += 256) {
      const double wj = p[j] - K * v[j];
      row[j] = row[j] - (vi * wj + wi * v[j]);
    }
  }
}

constexpr int RB = 8;   // row elements loaded together in tridiag_step_kernel
constexpr int64_t kTridiagTwoRows = 1024;   // trailing rows from which a wave takes two rows

// Step k's rank-2 update fused with step k+1's reflector and product, so that
// the trailing block is read and written once per step.  Row k+1 (row 0 of the
// step-k trailing block, the source of reflector k+1) is only read: every
// work-group forms its updated entries itself, with their squared norm in the
// same pass, and stages them in LDS unscaled (m - 1 doubles of dynamic shared
// memory; the scale is applied where the reflector is used).  The rows and columns k+2 .. of A
// (the trailing block of step k+1) are updated in place, one wave per row, and
// each wave then forms its entry of p = tau A22 v for step k+1; column k+1,
// which no later step reads, is left as it is.  p and pv of step k are read
// and those of step k+1 written to separate buffers.  The arithmetic is that of
// house_symv_kernel and rank2_fused_kernel (the reflector's norm summed in
// another order); three barriers per step.
// RW rows of the step-(k+1) block per wave (RW = 2 for large blocks: p and v are
// loaded once for both rows, and the work-group's own reflector is formed for
// twice the rows); nparts = the number of partial sums pv written by the launch
// before (one per work-group)
template <int RW>
__global__ __launch_bounds__(256) void tridiag_step_kernel(double *A, int64_t n, int64_t k,
                                                           double *V, double *tau, double *d,
                                                           double *e, const double *p,
                                                           const double *pv, int64_t nparts,
                                                           double *p1, double *pv1, int *nonfinite) {
  extern __shared__ double vn[];
  __shared__ double red[4], nrm[4], part[4];
  const int64_t m = n - k - 1, m1 = m - 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double *v = V + k * n + k + 1;                 // reflector k, v[0] = 1
  const double *x = A + (k + 1) * n + k + 1;           // row k+1 before the update
  // Every load that does not depend on the sum of the partials is issued before
  // it: the first RB elements of row k+1 with p and v (the reflector's inputs)
  // and the first RB elements of this wave's rows with p and v for them, so that
  // their latencies overlap.  The loops over a row load RB elements (clamped
  // into range) before using any: one memory latency per RB elements.
  double xj[RB], pj[RB], vj[RB];
  auto load_x = [&](int64_t j0) {
#pragma unroll
    for (int t = 0; t < RB; ++t) {
      const int64_t j = min(j0 + 256 * t, m - 1);
      xj[t] = x[j];
      pj[t] = p[j];
      vj[t] = v[j];
    }
  };
  const int64_t jx0 = 1 + threadIdx.x;
  if (jx0 < m) load_x(jx0);
  const double p0 = p[0], v0 = v[0], x0 = x[0];
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wv) * RW;   // first row of the step-(k+1) block
  const bool has_rows = r0 < m1;                            // wave-uniform
  double vi[RW], pi_[RW], aj[RW][RB], qj[RB], uj[RB];
  double *row[RW];
#pragma unroll
  for (int q = 0; q < RW; ++q) {
    const int64_t i = min<int64_t>(r0 + q, m1 - 1) + 1;    // its row in the step-k block
    row[q] = A + (k + 1 + i) * n + k + 1;
  }
  auto load_rows = [&](int64_t j0) {
#pragma unroll
    for (int t = 0; t < RB; ++t) {
      const int64_t j = min(j0 + 64 * t, m - 1);
      qj[t] = p[j];
      uj[t] = v[j];
#pragma unroll
      for (int q = 0; q < RW; ++q) aj[q][t] = row[q][j];
    }
  };
  const int64_t jr0 = 1 + lane;
  if (has_rows) {
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      const int64_t i = min<int64_t>(r0 + q, m1 - 1) + 1;
      vi[q] = v[i];
      pi_[q] = p[i];
    }
    if (jr0 < m) load_rows(jr0);
  }

  double s = 0.0;
  for (int64_t i = threadIdx.x; i < nparts; i += 256) s += pv[i];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) red[wv] = s;
  __syncthreads();
  const double K = 0.5 * tau[k] * (red[0] + red[1] + red[2] + red[3]);
  const double w0 = p0 - K * v0;
  // row k+1 after the update (the unscaled reflector, vn[0] = its first entry)
  // and, in the same pass, its squared norm past the first entry
  double ss = 0.0;
  for (int64_t j0 = jx0; j0 < m; j0 += 256 * RB) {
    if (j0 != jx0) load_x(j0);
#pragma unroll
    for (int t = 0; t < RB; ++t) {
      const int64_t j = j0 + 256 * t;
      if (j < m) {
        const double u = xj[t] - (v0 * (pj[t] - K * vj[t]) + w0 * vj[t]);
        vn[j - 1] = u;
        if (j >= 2) ss += u * u;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) ss += __shfl_down(ss, o, 64);
  if (lane == 0) nrm[wv] = ss;
  __syncthreads();                                     // vn and nrm complete
  // reflector k+1: beta = -sign(alpha) |x|, tau = (beta - alpha)/beta and
  // v = x/(alpha - beta) with v0 = 1 (tau = 0 when the tail of x is 0); v is
  // formed where it is used, vs(i) = i == 0 ? 1 : vn[i] * scale
  const double xn2 = nrm[0] + nrm[1] + nrm[2] + nrm[3], alpha = vn[0];
  double t, scale, beta;
  if (xn2 == 0.0) {
    t = 0.0;
    beta = alpha;
    scale = 0.0;
  } else {
    beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
    t = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  auto vs = [&](int64_t i) -> double { return i == 0 ? 1.0 : vn[i] * scale; };
  if (blockIdx.x == 0) {
    double *vo = V + (k + 1) * n + k + 2;
    for (int64_t i = threadIdx.x; i < m1; i += 256) vo[i] = vs(i);
    if (threadIdx.x == 0) {
      if (!isfinite(beta) || !isfinite(t)) atomicExch(nonfinite, 1);
      tau[k + 1] = t;
      d[k + 1] = x0 - (v0 * w0 + w0 * v0);
      e[k + 1] = beta;
    }
  }
  double pvr = 0.0;
  if (has_rows) {
    const int nr = (int)min<int64_t>(RW, m1 - r0);         // rows of this wave (wave-uniform)
    double wi[RW], acc[RW];
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      wi[q] = pi_[q] - K * vi[q];
      acc[q] = 0.0;
    }
    for (int64_t j0 = jr0; j0 < m; j0 += 64 * RB) {
      if (j0 != jr0) load_rows(j0);
#pragma unroll
      for (int q = 0; q < RW; ++q) {
        if (q >= nr) break;
#pragma unroll
        for (int t = 0; t < RB; ++t) {
          const int64_t j = j0 + 64 * t;
          if (j < m) {
            const double a = aj[q][t] - (vi[q] * (qj[t] - K * uj[t]) + wi[q] * uj[t]);
            row[q][j] = a;
            acc[q] += a * vs(j - 1);
          }
        }
      }
    }
#pragma unroll
    for (int q = 0; q < RW; ++q) {
      if (q >= nr) break;
      double s = acc[q];
      for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
      const double pi = t * s;
      pvr += pi * vs(r0 + q);
      if (lane == 0) p1[r0 + q] = pi;
    }
  }
  if (lane == 0) part[wv] = pvr;
  __syncthreads();
  if (threadIdx.x == 0) pv1[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

__global__ void tail_kernel(const double *A, int64_t n, double *d, double *e) {
  if (threadIdx.x != 0) return;
  if (n >= 2) {
    d[n - 2] = A[(n - 2) * n + n - 2];
    e[n - 2] = A[(n - 1) * n + n - 2];
  }
  d[n - 1] = A[(n - 1) * n + n - 1];
}

// number of eigenvalues of T smaller than x (Sturm count of the LDL^T pivots)
// number of eigenvalues of T below x: the negative pivots of the LDL^T factors
// of T - xI.  1/q is the hardware reciprocal refined by two Newton steps (full
// double accuracy; q is kept away from 0 by pivmin), which halves the dependent
// chain of a step against an IEEE division; only the signs of the pivots count.
__device__ inline double recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return fma(r, fma(-q, r, 1.0), r);
}
__device__ inline int sturm_count(const double *d, const double *e, int64_t n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int64_t i = 1; i < n; ++i) {
    q = (d[i] - x) - e[i - 1] * e[i - 1] * recip(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// lambda[j] = j-th smallest eigenvalue of T, one wave per j: each step the 64
// lanes evaluate Sturm counts at 64 interior points of the bracket, which then
// shrinks by a factor 65 (multisection).
__global__ __launch_bounds__(256) void bisect_kernel(const double *d, const double *e, int64_t n,
                                                     double *lambda, double *tnorm_out) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  double lo = INFINITY, hi = -INFINITY, emax2 = 0.0;
  for (int64_t i = lane; i < n; i += 64) {
    const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    if (i + 1 < n) emax2 = fmax(emax2, e[i] * e[i]);
  }
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
    emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
  }
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pivmin = SAFMIN * fmax(1.0, emax2);
  lo -= 2.0 * EPS * tnorm * n + pivmin;
  hi += 2.0 * EPS * tnorm * n + pivmin;
  for (int it = 0; it < 40; ++it) {
    if (hi - lo <= 2.0 * EPS * fmax(fabs(lo), fabs(hi)) + 4.0 * pivmin) break;
    const double h = (hi - lo) / 65.0;
    const double x = lo + h * (lane + 1);
    const bool above = sturm_count(d, e, n, x, pivmin) > j;     // lambda_j < x
    const unsigned long long mask = __ballot(above);
    if (mask == 0ull) {
      lo = lo + h * 64;                                        // lambda_j in [x_63, hi]
    } else {
      const int t = __ffsll((long long)mask) - 1;               // first point above lambda_j
      const double new_hi = lo + h * (t + 1);
      lo = t > 0 ? lo + h * t : lo;
      hi = new_hi;
    }
  }
  if (lane == 0) {
    lambda[j] = 0.5 * (lo + hi);
    if (j == 0) *tnorm_out = tnorm;
  }
}

__device__ inline double start_value(int64_t i, int64_t j) {
  uint64_t h = (uint64_t)i * 0x9E3779B97F4A7C15ull ^ ((uint64_t)j + 0x632BE59BD9B4E019ull) * 0xBF58476D1CE4E5B9ull;
  h ^= h >> 31;
  h *= 0x94D049BB133111EBull;
  h ^= h >> 29;
  return (double)(h >> 11) * (1.0 / 9007199254740992.0) - 0.5;
}

// Eigenvector of T for lambda[j] by three steps of inverse iteration; thread j
// owns column j of Zt (row-major n x n) and columns j of the factor arrays
// (element i of thread j at [i*n + j], so a wave's accesses are contiguous).
// The LU factorisation of T - lambda I with partial pivoting and both triangular
// solves carry their running values in registers; memory is only written
// (factorisation) or read (solves) once per element.
// The shift is lambda_j - delta, delta = 1e-10 |T|: eigenvalues that are equal to
// working precision (computed values differing by ~1e-14 |T|) are then amplified
// alike, so their vectors stay independent combinations of the common eigenspace
// instead of collapsing onto one eigenvector; an isolated eigenvalue at gap g
// still converges by (delta/g)^3 in three steps.
constexpr int IB = 8;   // rows per block of the pipelined triangular solves

__global__ __launch_bounds__(64) void inverse_iteration_kernel(
    const double *d, const double *e, int64_t n, const double *lambda, const double *tnorm,
    double *Zt, double *dg, double *du, double *du2, double *dl, double *swp) {
  const int64_t j = (int64_t)blockIdx.x * 64 + threadIdx.x;
  if (j >= n) return;
  const double tiny = EPS * fmax(*tnorm, SAFMIN * 1e16);
  const double lam = lambda[j] - 1e-10 * fmax(*tnorm, SAFMIN * 1e16);
#define AT(arr, i) arr[(int64_t)(i) * n + j]
  // factorisation: g = current pivot candidate of row i, u = its superdiagonal
  double g = d[0] - lam, u = n > 1 ? e[0] : 0.0;
  for (int64_t i = 0; i + 1 < n; ++i) {
    const double l = e[i], dn = d[i + 1] - lam, en = i + 2 < n ? e[i + 1] : 0.0;
    if (fabs(g) >= fabs(l)) {
      const double gp = g != 0.0 ? g : tiny;
      const double rg = recip(gp);
      const double f = l * rg;
      AT(dg, i) = rg; AT(dl, i) = f; AT(du, i) = u; AT(swp, i) = 0.0;
      if (i + 2 < n) AT(du2, i) = 0.0;
      g = dn - f * u;
      u = en;
    } else {
      const double rl = recip(l);
      const double f = g * rl;
      AT(dg, i) = rl; AT(dl, i) = f; AT(du, i) = dn; AT(swp, i) = 1.0;
      if (i + 2 < n) AT(du2, i) = en;
      g = u - f * dn;
      u = -f * en;
    }
  }
  AT(dg, n - 1) = recip(g != 0.0 ? g : tiny);   // dg holds the reciprocal pivots
  double nrm = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const double s = start_value(i, j);
    AT(Zt, i) = s;
    nrm += s * s;
  }
  for (int it = 0; it < 3; ++it) {
    const double inv = 1.0 / sqrt(nrm);
    // forward: row interchanges and multipliers (L y = P b).  Both solves run
    // in blocks of IB rows whose operands are loaded one block ahead (rows
    // clamped into range), so the memory latency is paid once per block and
    // not once per row; every row is still loaded before it is overwritten.
    const int64_t nf = n - 1;                 // elimination steps i = 0 .. n-2
    double cur = AT(Zt, 0) * inv;
    {
      double za[IB], sa[IB], la[IB], zb[IB], sb[IB], lb[IB];
      auto fload = [&](int64_t i0, double (&z)[IB], double (&sw)[IB], double (&l)[IB]) {
#pragma unroll
        for (int t = 0; t < IB; ++t) {
          const int64_t i = min(i0 + t, nf - 1);
          z[t] = AT(Zt, i + 1);
          sw[t] = AT(swp, i);
          l[t] = AT(dl, i);
        }
      };
      auto fstep = [&](int64_t i0, const double (&z)[IB], const double (&sw)[IB], const double (&l)[IB]) {
#pragma unroll
        for (int t = 0; t < IB; ++t) {
          const int64_t i = i0 + t;
          if (i < nf) {
            const double nxt = z[t] * inv;
            double bi = cur, bn = nxt;
            if (sw[t] != 0.0) { bi = nxt; bn = cur; }
            AT(Zt, i) = bi;
            cur = bn - l[t] * bi;
          }
        }
      };
      if (nf > 0) fload(0, za, sa, la);
      for (int64_t i0 = 0; i0 < nf; i0 += 2 * IB) {
        if (i0 + IB < nf) fload(i0 + IB, zb, sb, lb);
        fstep(i0, za, sa, la);
        if (i0 + 2 * IB < nf) fload(i0 + 2 * IB, za, sa, la);
        if (i0 + IB < nf) fstep(i0 + IB, zb, sb, lb);
      }
    }
    AT(Zt, n - 1) = cur;
    // backward: U x = y, rows n-1 down to 0
    nrm = 0.0;
    double x1 = 0.0, x2 = 0.0;
    {
      double ya[IB], ua[IB], va[IB], ga[IB], yb[IB], ub[IB], vb[IB], gb[IB];
      auto bload = [&](int64_t i0, double (&y)[IB], double (&u1)[IB], double (&u2)[IB], double (&g)[IB]) {
#pragma unroll
        for (int t = 0; t < IB; ++t) {
          const int64_t i = max(i0 - t, (int64_t)0);
          y[t] = AT(Zt, i);
          u1[t] = AT(du, i);
          u2[t] = AT(du2, i);
          g[t] = AT(dg, i);
        }
      };
      auto bstep = [&](int64_t i0, const double (&y)[IB], const double (&u1)[IB], const double (&u2)[IB],
                       const double (&g)[IB]) {
#pragma unroll
        for (int t = 0; t < IB; ++t) {
          const int64_t i = i0 - t;
          if (i >= 0) {
            double s = y[t];
            if (i + 1 < n) s -= u1[t] * x1;
            if (i + 2 < n) s -= u2[t] * x2;
            const double xi = s * g[t];            // g: reciprocal pivot
            AT(Zt, i) = xi;
            nrm += xi * xi;
            x2 = x1;
            x1 = xi;
          }
        }
      };
      bload(n - 1, ya, ua, va, ga);
      for (int64_t i0 = n - 1; i0 >= 0; i0 -= 2 * IB) {
        if (i0 - IB >= 0) bload(i0 - IB, yb, ub, vb, gb);
        bstep(i0, ya, ua, va, ga);
        if (i0 - 2 * IB >= 0) bload(i0 - 2 * IB, ya, ua, va, ga);
        if (i0 - IB >= 0) bstep(i0 - IB, yb, ub, vb, gb);
      }
    }
    if (!(nrm > 0.0) || !isfinite(nrm)) {  // fall back to a fresh start
      nrm = 0.0;
      for (int64_t i = 0; i < n; ++i) {
        const double s = start_value(i, j + (int64_t)(it + 1) * n);
        AT(Zt, i) = s;
        nrm += s * s;
      }
    }
  }
  const double inv = 1.0 / sqrt(nrm);
  for (int64_t i = 0; i < n; ++i) AT(Zt, i) *= inv;
#undef AT
}

// Back-transformation in blocks of WY_NB reflectors (compact WY form):
// H_k0 H_k0+1 ... H_k1-1 = I - V T V^T, V = [v_k0 .. v_k1-1], T upper triangular
// with T_jj = tau_j and T[0:j, j] = -tau_j T[0:j, 0:j] (V[:, 0:j]^T v_j).
constexpr int WY_NB = 64;
// largest n for the fused tridiagonalisation step (reflector staged in 64 KiB of LDS)
constexpr int64_t kFusedTridiagMax = 8192;

// Vb[i][j] = (v_{k0+j})_i, an n x nb row-major block: zero at and above row
// k0+j, 1 at row k0+j+1
__global__ __launch_bounds__(256) void wy_vblock_kernel(const double *V, int64_t n, int64_t k0,
                                                        int nb, double *Vb) {
  const int64_t total = (int64_t)nb * n;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t i = e / nb, j = e % nb, k = k0 + j;
    Vb[e] = i > k ? V[k * n + i] : 0.0;
  }
}

// G_b[i][j] = v_{k0+i} . v_{k0+j} (i < j) for every block b of WY_NB reflectors
// (k0 = b WY_NB), straight from the rows of V (one wave per pair, grid.y = block;
// v_k is zero up to row k, so the sum runs over rows past k0 + j)
__global__ __launch_bounds__(256) void wy_gram_all_kernel(const double *V, int64_t n, int64_t R,
                                                          double *G) {
  const int64_t b = blockIdx.y, k0 = b * WY_NB;
  const int nb = (int)min<int64_t>(WY_NB, R - k0);
  const int pair = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (pair >= nb * nb) return;
  const int i = pair / nb, j = pair % nb;
  if (i >= j) return;
  const double *vi = V + (k0 + i) * n, *vj = V + (k0 + j) * n;
  double s = 0.0;
  for (int64_t x = k0 + 1 + j + lane; x < n; x += 64) s += vi[x] * vj[x];
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) G[b * WY_NB * WY_NB + i * nb + j] = s;
}

// compact-WY factor T_b of every block (one work-group per block, nb <= 64, in
// LDS): T[j][j] = tau_j and T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j], the operands
// of 8 terms read before any is used (one LDS latency per 8)
__global__ __launch_bounds__(64) void wy_t_all_kernel(const double *G, const double *tau, int64_t R,
                                                      double *T) {
  __shared__ double sT[64][65], sG[64][65];
  const int64_t b = blockIdx.x, k0 = b * WY_NB;
  const int nb = (int)min<int64_t>(WY_NB, R - k0);
  const double *Gb = G + b * WY_NB * WY_NB;
  double *Tb = T + b * WY_NB * WY_NB;
  const int i = threadIdx.x;
  for (int j = 0; j < nb; ++j) {
    if (i < nb) {
      sT[i][j] = 0.0;
      sG[i][j] = i < j ? Gb[i * nb + j] : 0.0;
    }
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    const double tj = tau[k0 + j];
    double s = 0.0;
    if (i < j) {
      for (int l0 = i; l0 < j; l0 += 8) {
        double a[8], g[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int l = min(l0 + u, 63);
          a[u] = sT[i][l];
          g[u] = sG[l][j];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (l0 + u < j) s += a[u] * g[u];
      }
    }
    __syncthreads();
    if (i < j) sT[i][j] = -tj * s;
    if (i == j) sT[j][j] = tj;
    __syncthreads();
  }
  for (int j = 0; j < nb; ++j)
    if (i < nb) Tb[i * nb + j] = sT[i][j];
}

__global__ void clear_ints_kernel(int *p, int count) {
  if (threadIdx.x < count) p[threadIdx.x] = 0;
}

inline unsigned grid_for(int64_t work) {
  const int64_t g = (work + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 8192));
}

struct SyevLayout {
  int64_t n, np, splits;
  size_t a, dg, du, du2, dl, swp, zt, z2, g, m, chol, partial, vec, info, wy, wyt, total;
};

SyevLayout syev_layout(int64_t n) {
  SyevLayout L;
  L.n = n;
  L.np = (n + 63) / 64 * 64;
  L.splits = gemm_tn_splits(n, n, true);
  size_t off = 0;
  auto take = [&](size_t doubles) { size_t o = off; off += (doubles * 8 + 255) / 256 * 256; return o; };
  const size_t nn = (size_t)n * n, npnp = (size_t)L.np * L.np;
  L.a = take(nn);
  L.dg = take(nn); L.du = take(nn); L.du2 = take(nn); L.dl = take(nn); L.swp = take(nn);
  L.zt = take(nn);
  L.z2 = take(nn);
  L.g = take(npnp);
  L.m = take(npnp);
  L.chol = take(chol_rinv_scratch_doubles(n));
  L.partial = take(std::max((size_t)L.splits * nn, (size_t)16 * WY_NB * n));
  L.vec = take(8 * (size_t)n + 8);
  L.info = take(4);
  L.wy = take(3 * (size_t)WY_NB * n + 2 * (size_t)WY_NB * WY_NB);
  L.wyt = take(2 * (size_t)((n + WY_NB - 1) / WY_NB) * WY_NB * WY_NB);   // G and T of every block
  L.total = off;
  return L;
}

}  // namespace

hipError_t launch_clear_ints(int *p, int count, hipStream_t s) {
  hipLaunchKernelGGL(clear_ints_kernel, dim3(1), dim3(64), 0, s, p, count);
  return hipGetLastError();
}

size_t syev_work_bytes(int64_t n) { return n < 1 ? 0 : syev_layout(n).total; }

hipError_t run_syev(int64_t n, const double *Ain, int64_t lda, double *lambda, double *Z,
                    int64_t ldz, void *work, hipStream_t s, int *host_info) {
  const SyevLayout L = syev_layout(n);
  char *w = (char *)work;
  double *A = (double *)(w + L.a), *dg = (double *)(w + L.dg), *du = (double *)(w + L.du);
  double *du2 = (double *)(w + L.du2), *dl = (double *)(w + L.dl), *swp = (double *)(w + L.swp);
  double *Zt = (double *)(w + L.zt), *Z2 = (double *)(w + L.z2), *G = (double *)(w + L.g);
  double *M = (double *)(w + L.m), *chol = (double *)(w + L.chol);
  double *partial = (double *)(w + L.partial), *vec = (double *)(w + L.vec);
  double *tau = vec, *d = vec + n, *e = vec + 2 * n, *p = vec + 3 * n, *pv = vec + 4 * n;
  double *tnorm = vec + 8 * n;
  int *info = (int *)(w + L.info);
  hipError_t err;
  hipLaunchKernelGGL(clear_ints_kernel, dim3(1), dim3(64), 0, s, info, 4);
  hipLaunchKernelGGL(copy_matrix_kernel, dim3(grid_for(n * n)), dim3(256), 0, s, Ain, lda, A, n, n);
  // 1. tridiagonalisation; reflector vectors go to V (rows k, columns k+1..)
  double *V = du2;
  if (n <= kFusedTridiagMax) {
    // one launch per step: step 0's product, then k's update fused with k+1's
    // product (p, pv alternate between two buffers), then the last update
    double *pb[2] = {p, vec + 5 * n}, *pvb[2] = {pv, vec + 6 * n};
    if (n > 2)
      hipLaunchKernelGGL(house_symv_kernel, dim3((unsigned)((n + 2) / 4)), dim3(256), 0, s, A, n,
                         (int64_t)0, V, tau, d, e, pb[0], pvb[0], info + 1);
    int cur = 0;
    int64_t nparts = (n + 2) / 4;                      // partial sums of the launch before
    for (int64_t k = 0; k + 3 < n; ++k, cur ^= 1) {
      const int64_t m1 = n - k - 2;
      if (m1 >= kTridiagTwoRows) {
        const int64_t g = (m1 + 7) / 8;
        hipLaunchKernelGGL(tridiag_step_kernel<2>, dim3((unsigned)g), dim3(256),
                           (unsigned)(m1 * sizeof(double)), s, A, n, k, V, tau, d, e, pb[cur],
                           pvb[cur], nparts, pb[cur ^ 1], pvb[cur ^ 1], info + 1);
        nparts = g;
      } else {
        const int64_t g = (m1 + 3) / 4;
        hipLaunchKernelGGL(tridiag_step_kernel<1>, dim3((unsigned)g), dim3(256),
                           (unsigned)(m1 * sizeof(double)), s, A, n, k, V, tau, d, e, pb[cur],
                           pvb[cur], nparts, pb[cur ^ 1], pvb[cur ^ 1], info + 1);
        nparts = g;
      }
    }
    if (n > 2)
      hipLaunchKernelGGL(rank2_fused_kernel, dim3((unsigned)((2 + 3) / 4)), dim3(256), 0, s, A, n,
                         n - 3, V, tau, pb[cur], pvb[cur]);
  } else {
    for (int64_t k = 0; k + 2 < n; ++k) {
      const int64_t m = n - k - 1;
      hipLaunchKernelGGL(house_symv_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, A, n,
                         k, V, tau, d, e, p, pv, info + 1);
      hipLaunchKernelGGL(rank2_fused_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, s, A, n,
                         k, V, tau, p, pv);
    }
  }
  hipLaunchKernelGGL(tail_kernel, dim3(1), dim3(64), 0, s, A, n, d, e);
  // 2. eigenvalues
  hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, d, e, n,
                     lambda, tnorm);
  // 3. eigenvectors of T
  // V (held in du2) is still needed, so the second superdiagonal of the factors
  // goes to Z2, which is free until the re-orthonormalisation below
  hipLaunchKernelGGL(inverse_iteration_kernel, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s,
                     d, e, n, lambda, tnorm, Zt, dg, du, Z2, dl, swp);
  // 4. Cholesky-QR twice: Zt <- Zt M
  for (int pass = 0; pass < 2; ++pass) {
    double *src = pass == 0 ? Zt : Z2, *dst = pass == 0 ? Z2 : Zt;
    if ((err = launch_gemm_tn_ex(src, n, src, n, n, n, G, L.np, true, false, partial,
                                 (int)L.splits, s)) != hipSuccess) return err;
    if ((err = launch_chol_rinv(G, n, M, chol, info, s)) != hipSuccess) return err;
    if ((err = launch_gemm_nn_ex(src, n, M, L.np, n, n, n, 1.0, dst, n, true, s)) != hipSuccess) return err;
  }
  // 5. back-transformation Z = H_0 ... H_{n-3} Zt, blocks of reflectors from the last:
  //    Z[k0+1:, :] -= V (T (V^T Z[k0+1:, :]))
  hipLaunchKernelGGL(copy_matrix_kernel, dim3(grid_for(n * n)), dim3(256), 0, s, Zt, n, Z, ldz, n);
  {
    const int64_t R = n - 2;                        // reflectors k = 0 .. n-3
    double *Vb = (double *)(w + L.wy), *W = Vb + (int64_t)WY_NB * n, *W2 = Vb + 2 * (int64_t)WY_NB * n;
    double *wpart = partial;                        // split-K partials of W (free here)
    // the T factors of all blocks first (they depend only on V and tau): a few
    // launches instead of a sequence of single-work-group ones
    const int64_t nblk = (R + WY_NB - 1) / WY_NB;
    double *Gall = (double *)(w + L.wyt), *Tall = Gall + nblk * WY_NB * WY_NB;
    if (nblk > 0) {
      hipLaunchKernelGGL(wy_gram_all_kernel, dim3((unsigned)((WY_NB * WY_NB + 3) / 4), (unsigned)nblk),
                         dim3(256), 0, s, V, n, R, Gall);
      hipLaunchKernelGGL(wy_t_all_kernel, dim3((unsigned)nblk), dim3(64), 0, s, Gall, tau, R, Tall);
    }
    for (int64_t k0 = (R > 0 ? (R - 1) / WY_NB * WY_NB : -1); k0 >= 0; k0 -= WY_NB) {
      const int nb = (int)std::min<int64_t>(WY_NB, R - k0);
      const int64_t m = n - k0 - 1;                 // rows touched
      const double *Tw = Tall + (k0 / WY_NB) * WY_NB * WY_NB;
      hipLaunchKernelGGL(wy_vblock_kernel, dim3(grid_for((int64_t)nb * n)), dim3(256), 0, s, V, n, k0, nb, Vb);
      // W = V^T Z[k0+1:, :]   (nb x n), split over the m rows
      const int ws = (int)std::max<int64_t>(1, std::min<int64_t>(16, m / 128));
      if ((err = launch_gemm_tn_general(Vb + (k0 + 1) * nb, nb, Z + (k0 + 1) * ldz, ldz, m, nb, n, W,
                                        n, wpart, ws, s)) != hipSuccess) return err;
      // W2 = T W
      if ((err = launch_gemm_nn_ex(Tw, nb, W, n, nb, nb, n, 1.0, W2, n, false, s)) != hipSuccess) return err;
      // Z[k0+1:, :] -= V W2
      if ((err = launch_gemm_nn_acc(Vb + (k0 + 1) * nb, nb, W2, n, m, nb, n, -1.0, Z + (k0 + 1) * ldz, ldz, s)) != hipSuccess)
        return err;
    }
  }
  if ((err = hipGetLastError()) != hipSuccess) return err;
  if ((err = hipStreamSynchronize(s)) != hipSuccess) return err;
  int h[2] = {0, 0};
  if ((err = hipMemcpy(h, info, sizeof h, hipMemcpyDeviceToHost)) != hipSuccess) return err;
  host_info[0] = h[0];
  host_info[1] = h[1];
  return hipSuccess;
}

}  // namespace ttdft
