// Sampled dense-dense product on the tile pattern of H, for the gradient of the
// Chebyshev filter with respect to the stored entries of H:
//     dH[t](i, j) (+)= coef * sum_c Abar[64*B + i][c] * Yk[64*B' + j][c]
// for every stored tile t = (B, B'), entries outside the true pattern (mask bit
// clear) written as 0.  dH has the layout of H's tile values (the fragment
// order of H's type: tile_pos_16x4 for FP64 / FP32 tiles, tile_pos_16x32 for
// BF16 tiles).  An optional weight
// per vector c multiplies Abar[.][c] (the density matrix on the pattern of H is
// this product with weights 2 f_c and Abar = Yk = Psi).  One work-group owns one tile and sweeps the vector
// dimension in 16-wide panels, both operands staged transposed in LDS
// ([vector][row]) so every matrix-core operand read is 16 consecutive values;
// the panels are double-buffered, the next two (FP64; one for FP32 and BF16)
// loaded into registers while the current one is contracted (one barrier per
// panel).
// FP64 inputs use the f64 16x16x4 op; FP32 and BF16 inputs accumulate in FP32
// on the f32 16x16x4 op.  Each tile is written by one work-group in a fixed
// order, so accumulation over the degree steps is deterministic.  A symmetric
// product (Abar = Yk, the density matrix) computes only the tiles (B, B') with
// B' >= B and writes each result also, transposed, into the mirror tile
// (B', B): half the work.
#include "ttdft_internal.h"

namespace ttdft {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int BK = 16, THREADS = 256;

template <typename TC> struct Op;
template <> struct Op<double> {
  using acc_t = v4d;
  static __device__ inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int t) { return (lane >> 4) + 4 * t; }
};
template <> struct Op<float> {
  using acc_t = v4f;
  static __device__ inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int t) { return 4 * (lane >> 4) + t; }
};

// iterate value in the arithmetic type TC (exact: TC is at least as wide as TX)
template <typename TC, typename TX> __device__ inline TC widen(TX v) { return (TC)v; }
template <> __device__ inline float widen<float, __bf16>(__bf16 v) { return (float)v; }

// TX: storage type of the iterates; TC: arithmetic / output type
template <typename TX, typename TC>
__global__ __launch_bounds__(THREADS) void sddmm_kernel(
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ tcol, int64_t n_block_rows,
    const TX *__restrict__ Abar, int64_t lda, const TX *__restrict__ Yk, int64_t ldb,
    int64_t n_vec, TC coef, TC *__restrict__ dH, const uint64_t *__restrict__ mask,
    int accumulate, const double *__restrict__ colw, int frag32, int sym) {
  using O = Op<TC>;
  __shared__ TC sA[2][BK][64 + 1];
  __shared__ TC sB[2][BK][64 + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t t = blockIdx.x;
  // block row of tile t: the last B with rowptr[B] <= t, by a 64-way search (the
  // 64 lanes test evenly spaced rows and the range shrinks 64-fold per round: two
  // dependent loads at a few thousand block rows)
  int64_t lo = 0, hi = n_block_rows;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) / 64, p = lo + lane * step;
    const bool ok = p < hi && rowptr[p] <= t;
    const uint64_t bal = __ballot(ok);                    // lane 0 (p = lo) always holds
    const int64_t top = lo + (int64_t)(63 - __clzll(bal)) * step;
    hi = min(hi, top + step);
    lo = top;
  }
  const int64_t B = lo, Bc = tcol[t];
  // symmetric product (Abar = Yk): tile (B', B) is the transpose of tile (B, B');
  // the tile with B' > B computes both, the one with B' < B only when its
  // mirror is not stored (the mirror is looked up 64 columns at a time)
  int64_t tm = -1;
  if (sym && Bc != B) {
    const int64_t a = rowptr[Bc], z = rowptr[Bc + 1];
    for (int64_t base = a; base < z; base += 64) {
      const int64_t idx = base + lane;
      const uint64_t hit = __ballot(idx < z && tcol[idx] == B);
      if (hit) {
        tm = base + __ffsll((unsigned long long)hit) - 1;
        break;
      }
    }
    if (Bc < B && tm >= 0) return;
  }
  const TX *Ar = Abar + B * 64 * lda;
  const TX *Br = Yk + Bc * 64 * ldb;

  typename O::acc_t acc[4];
  for (int j = 0; j < 4; ++j) acc[j] = typename O::acc_t{0, 0, 0, 0};
  // 16x16 output blocks of this wave (rows 16w .., columns 16 jb ..) holding no
  // pattern entry are written as 0 below whatever they hold: their products can
  // be skipped
  unsigned live = 0xFu;
  if (sizeof(TC) == 8 && mask) {
    const uint64_t mw = lane < 16 ? mask[t * 64 + 16 * w + lane] : 0ull;
    unsigned lo32 = (unsigned)mw, hi32 = (unsigned)(mw >> 32);
    for (int o = 8; o > 0; o >>= 1) {
      lo32 |= __shfl_xor(lo32, o, 64);
      hi32 |= __shfl_xor(hi32, o, 64);
    }
    live = ((lo32 & 0xFFFFu) ? 1u : 0u) | ((lo32 >> 16) ? 2u : 0u) |
           ((hi32 & 0xFFFFu) ? 4u : 0u) | ((hi32 >> 16) ? 8u : 0u);
    live = __builtin_amdgcn_readfirstlane(live);        // lane 0 holds the OR of rows 0..15
  }

  // panels of BK vectors, double-buffered in LDS; FP64 loads two panels ahead
  // into registers (two register stages), so a panel's loads have two
  // contractions to arrive (columns past n_vec read a clamped, in-range column
  // and are stored as 0)
  constexpr int Q = BK * 64 / THREADS;
  TC ra0[Q], rb0[Q], ra1[Q], rb1[Q];
  auto load = [&](TC *ra, TC *rb, int64_t c0) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int idx = tid + THREADS * q;
      const int r = idx / BK, kk = idx % BK;     // consecutive threads walk the vector index
      const int64_t c = c0 + kk, cc = min(c, n_vec - 1);
      const TC wa = colw ? (TC)colw[cc] : TC(1);
      const TC av = wa * widen<TC, TX>(Ar[(int64_t)r * lda + cc]);
      const TC bv = widen<TC, TX>(Br[(int64_t)r * ldb + cc]);
      ra[q] = c < n_vec ? av : TC(0);
      rb[q] = c < n_vec ? bv : TC(0);
    }
  };
  auto store = [&](const TC *ra, const TC *rb, int buf) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int idx = tid + THREADS * q;
      const int r = idx / BK, kk = idx % BK;
      sA[buf][kk][r] = ra[q];
      sB[buf][kk][r] = rb[q];
    }
  };
  auto contract = [&](int buf) {
    if constexpr (sizeof(TC) == 8) {
      // FP64: the products dominate, so the blocks without pattern entries are skipped
      TC a[BK / 4];
#pragma unroll
      for (int kq = 0; kq < BK; kq += 4) a[kq / 4] = sA[buf][kq + (lane >> 4)][16 * w + (lane & 15)];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        if (!((live >> jb) & 1u)) continue;
#pragma unroll
        for (int kq = 0; kq < BK; kq += 4) {
          const TC b = sB[buf][kq + (lane >> 4)][16 * jb + (lane & 15)];
          acc[jb] = O::mma(a[kq / 4], b, acc[jb]);
        }
      }
    } else {
      // FP32 products are twice as fast and the loads dominate: the plain order
      // measured faster than the skipping one
#pragma unroll
      for (int kq = 0; kq < BK; kq += 4) {
        const TC a = sA[buf][kq + (lane >> 4)][16 * w + (lane & 15)];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
          const TC b = sB[buf][kq + (lane >> 4)][16 * jb + (lane & 15)];
          acc[jb] = O::mma(a, b, acc[jb]);
        }
      }
    }
  };
  const int64_t npanel = (n_vec + BK - 1) / BK;
  if constexpr (sizeof(TC) == 8) {
    // LDS buffer p % 2 holds panel p while it is contracted; register stage
    // (p + 1) % 2 holds panel p + 1 and stage p % 2 receives panel p + 2
    load(ra0, rb0, 0);
    if (npanel > 1) load(ra1, rb1, BK);
    store(ra0, rb0, 0);
    __syncthreads();
    for (int64_t p = 0; p < npanel; p += 2) {
      if (p + 2 < npanel) load(ra0, rb0, (p + 2) * BK);
      contract(0);
      if (p + 1 < npanel) store(ra1, rb1, 1);
      __syncthreads();
      if (p + 1 >= npanel) break;
      if (p + 3 < npanel) load(ra1, rb1, (p + 3) * BK);
      contract(1);
      if (p + 2 < npanel) store(ra0, rb0, 0);
      __syncthreads();
    }
  } else {
    // FP32 products: one register stage (the second one costs half the
    // occupancy, and the loads then bind: measured slower)
    load(ra0, rb0, 0);
    store(ra0, rb0, 0);
    __syncthreads();
    int buf = 0;
    for (int64_t p = 0; p < npanel; ++p) {
      const bool more = p + 1 < npanel;
      if (more) load(ra0, rb0, (p + 1) * BK);
      contract(buf);
      if (more) store(ra0, rb0, buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
  }

  TC *out = dH + t * kTileElems;
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) {
    const int j = 16 * jb + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = 16 * w + O::row(lane, q);
      const bool on = mask ? ((mask[t * 64 + i] >> j) & 1ull) != 0 : true;
      const int pos = frag32 ? tile_pos_16x32(i, j) : tile_pos_16x4(i, j);   // layout of H's tiles
      TC v = coef * acc[jb][q];
      if (accumulate) v += out[pos];
      out[pos] = on ? v : TC(0);
      if (tm >= 0) {
        // entry (j, i) of the mirror tile: the same value
        TC *out2 = dH + tm * kTileElems;
        const bool on2 = mask ? ((mask[tm * 64 + j] >> i) & 1ull) != 0 : true;
        const int pos2 = frag32 ? tile_pos_16x32(j, i) : tile_pos_16x4(j, i);
        TC v2 = coef * acc[jb][q];
        if (accumulate) v2 += out2[pos2];
        out2[pos2] = on2 ? v2 : TC(0);
      }
    }
  }
}

}  // namespace

hipError_t launch_sddmm(const ttdft_bsr &H, const void *Abar, int64_t lda, const void *Bk,
                        int64_t ldb, int64_t n_vec, double coef, void *dH, const uint64_t *mask,
                        bool accumulate, ttdft_dtype xt, hipStream_t s, const double *colw,
                        bool sym) {
  if (H.n_tiles == 0) return hipSuccess;
  const dim3 grid((unsigned)H.n_tiles), block(THREADS);
  const int acc = accumulate ? 1 : 0;
  const int f32o = (H.dtype == TTDFT_BF16 || H.dtype == TTDFT_BF16_SPLIT) ? 1 : 0;
  if (xt == TTDFT_F64)
    hipLaunchKernelGGL((sddmm_kernel<double, double>), grid, block, 0, s, H.tile_rowptr, H.tile_col,
                       H.n_block_rows, (const double *)Abar, lda, (const double *)Bk, ldb, n_vec,
                       coef, (double *)dH, mask, acc, colw, f32o, sym ? 1 : 0);
  else if (xt == TTDFT_F32)
    hipLaunchKernelGGL((sddmm_kernel<float, float>), grid, block, 0, s, H.tile_rowptr, H.tile_col,
                       H.n_block_rows, (const float *)Abar, lda, (const float *)Bk, ldb, n_vec,
                       (float)coef, (float *)dH, mask, acc, colw, f32o, sym ? 1 : 0);
  else
    hipLaunchKernelGGL((sddmm_kernel<__bf16, float>), grid, block, 0, s, H.tile_rowptr, H.tile_col,
                       H.n_block_rows, (const __bf16 *)Abar, lda, (const __bf16 *)Bk, ldb, n_vec,
                       (float)coef, (float *)dH, mask, acc, colw, f32o, sym ? 1 : 0);
  return hipGetLastError();
}

}  // namespace ttdft
