// Occupancies and density after the Rayleigh-Ritz step (Sec. 2, Eqs. for the
// electron density, the Fermi-Dirac occupancy and the electron-count
// constraint):
//   f(eps; mu) = 1 / (1 + exp((eps - mu) / kT)),  2 sum_i f(eps_i; mu) = N_e,
//   rho_r = 2 sum_i f_i psi_ri^2   (the diagonal of the density matrix; the
//   off-diagonal entries on the pattern of H come from the sampled product in
//   sddmm.hip with weights 2 f_i).
// mu by bisection on the increasing electron count, in one work-group with
// fixed-order reductions (deterministic).
#include <cmath>

#include "ttdft_internal.h"

namespace ttdft {
namespace {

constexpr int FT = 256;

__device__ inline double wg_reduce(double v, double *red, bool is_max, bool is_min) {
  for (int o = 32; o > 0; o >>= 1) {
    const double u = __shfl_down(v, o, 64);
    v = is_max ? fmax(v, u) : (is_min ? fmin(v, u) : v + u);
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = red[0];
  for (int w = 1; w < FT / 64; ++w) t = is_max ? fmax(t, red[w]) : (is_min ? fmin(t, red[w]) : t + red[w]);
  __syncthreads();
  return t;
}

__device__ inline double occupancy(double eps, double mu, double kT) {
  return 1.0 / (1.0 + exp((eps - mu) / kT));   // exp overflow gives 0, underflow 1
}

__global__ __launch_bounds__(FT) void fermi_kernel(const double *__restrict__ lam, int64_t n, double ne,
                                                   double kT, double *__restrict__ f, double *out) {
  __shared__ double red[FT / 64];
  double lo = INFINITY, hi = -INFINITY, bad = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += FT) {
    const double v = lam[i];
    if (!isfinite(v)) bad = 1.0;
    lo = fmin(lo, v);
    hi = fmax(hi, v);
  }
  lo = wg_reduce(lo, red, false, true);
  hi = wg_reduce(hi, red, true, false);
  bad = wg_reduce(bad, red, true, false);
  if (bad != 0.0) {
    if (threadIdx.x == 0) { out[0] = NAN; out[1] = 1.0; }
    return;
  }
  auto count = [&](double mu) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += FT) s += 2.0 * occupancy(lam[i], mu, kT);
    return wg_reduce(s, red, false, false);
  };
  lo -= kT;
  hi += kT;
  // widen until count(lo) < ne < count(hi); count is increasing in mu and goes
  // from 0 to 2n, and 0 < ne < 2n
  for (int it = 0; it < 64 && count(lo) >= ne; ++it) lo -= (hi - lo);
  for (int it = 0; it < 64 && count(hi) <= ne; ++it) hi += (hi - lo);
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (count(mid) < ne) lo = mid;
    else hi = mid;
  }
  const double mu = 0.5 * (lo + hi);
  for (int64_t i = threadIdx.x; i < n; i += FT) f[i] = occupancy(lam[i], mu, kT);
  if (threadIdx.x == 0) { out[0] = mu; out[1] = 0.0; }
}

// rho_r = 2 sum_c f_c psi_rc^2, one wave per row (fixed-order lane reduction)
__global__ __launch_bounds__(256) void density_kernel(const double *__restrict__ Psi, int64_t ldp,
                                                      const double *__restrict__ f, int64_t rows,
                                                      int64_t n, double *__restrict__ rho) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  const int lane = threadIdx.x & 63;
  const double *row = Psi + r * ldp;
  double s = 0.0;
  for (int64_t c = lane; c < n; c += 64) s = fma(f[c] * row[c], row[c], s);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if (lane == 0) rho[r] = 2.0 * s;
}

}  // namespace

hipError_t run_fermi_level(const double *lambda, int64_t n, double n_electrons, double kT, double *f,
                           double *scratch, hipStream_t s, double *mu, int *nonfinite) {
  hipLaunchKernelGGL(fermi_kernel, dim3(1), dim3(FT), 0, s, lambda, n, n_electrons, kT, f, scratch);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  double out[2];
  if ((e = hipMemcpyAsync(out, scratch, sizeof out, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
  *mu = out[0];
  *nonfinite = out[1] != 0.0;
  return hipSuccess;
}

hipError_t launch_electron_density(const double *Psi, int64_t ldp, const double *f, int64_t rows,
                                   int64_t n, double *rho, hipStream_t s) {
  const int64_t g = (rows + 3) / 4;
  if (g > 0x7fffffff) return hipErrorInvalidConfiguration;
  hipLaunchKernelGGL(density_kernel, dim3((unsigned)g), dim3(256), 0, s, Psi, ldp, f, rows, n, rho);
  return hipGetLastError();
}

}  // namespace ttdft
