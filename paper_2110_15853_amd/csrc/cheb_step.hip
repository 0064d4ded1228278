// Fused lattice-blocked BSR SpMM + Chebyshev recurrence epilogue for gfx950.
//
// One launch performs one degree step of the scaled three-term recurrence of
// Algorithm 1 (Sec. 3.4):
//     Yout[B, :] = alpha * (sum_{B'} H[B, B'] Yk[B', :] - c * Yk[B, :]) - beta * Yprev[B, :]
// for every 64-row lattice block B.  The sparse-dense product H Yk is the main
// kernel of the filter (Sec. 4); here the dense 64x64 tiles of the blocked H are
// contracted on the matrix cores and the recurrence update is applied in the
// epilogue, so Yk, Yprev and Yout each cross HBM once per step.
//
// Work decomposition: one work-group owns one block row B and one column tile
// of vectors and walks the (at most 27) tiles of B, accumulating in matrix-core
// registers.  Each output element is produced by exactly one work-group, so
// results are deterministic (no atomics).  FP64 and FP32 use the pipelined
// kernel cheb_step_pipe<T>; BF16 tiles use the LDS-staged 16x16x32 bf16 kernel.
#include "ttdft_internal.h"

namespace ttdft {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));



// MFMA 16x16x4 on scalar operands: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// output item t of lane l is D[row(l, t)][l%16].
template <typename T> struct Mfma4;
template <> struct Mfma4<double> {
  using acc_t = v4d;
  static __device__ inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int t) { return (lane >> 4) + 4 * t; }
};
template <> struct Mfma4<float> {
  using acc_t = v4f;
  static __device__ inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lane, int t) { return 4 * (lane >> 4) + t; }
};

// Pipelined FP64 / FP32 path.  8 waves per work-group; the work-group owns block row B and
// 128 vectors, wave w the 64 x 16 output slab of vectors 16w .. 16w+15.
//  - A operand (H tile): double-buffered in LDS in matrix-core fragment order,
//    element H[16*mb + (l & 15)][4*kk + (l >> 4)] of fragment (kk, mb) in its
//    64-slot region (lanes rotated within groups of 16, see store_h); the next
//    tile is fetched into registers while the current one is contracted (one
//    barrier per tile).
//  - B operand (Y_k panel): each wave reads its own 16 vectors straight from
//    global memory into registers, a whole tile (16 k-steps) ahead of use.
constexpr int F64_NV = 128, F64_THREADS = 512, F64_S = 65;   // fragment row stride (+1 pad)
// launch order: column groups of ORDER_CGROUP tiles outermost; each XCD takes runs
// of ORDER_CHUNK consecutive block rows (all column tiles of the group), the 8
// XCDs working on neighbouring runs at the same time
constexpr int ORDER_CGROUP = 16, ORDER_CHUNK = 1;
// column blocks of 16 vectors per wave in the FP64 / FP32 kernel
constexpr int PIPE_CB_F64 = 1, PIPE_CB_F32 = 1;
// waves per SIMD the kernel is compiled for (register budget 512 / waves)
template <typename T, int CB> constexpr int pipe_waves() { return (sizeof(T) == 8 && CB > 1) ? 2 : 4; }

__device__ inline int64_t group_order(int64_t g, int64_t G, int64_t C) {
  // hardware ids go round-robin over 8 XCDs; give each XCD C consecutive logical
  // ids (the column tiles of one block row share that XCD's L2), the 8 XCDs
  // working on neighbouring block rows at the same time
  const int64_t span = 8 * C, full = (G / span) * span;
  if (g >= full) return g;
  return (g / span) * span + (g % 8) * C + (g / 8) % C;
}

// T = double (f64 16x16x4) or float (f32 16x16x4, same operand layouts).
// CB = column blocks of 16 vectors per wave: the work-group covers 8*16*CB
// vectors and each A fragment read from LDS feeds CB matrix-core ops.
template <typename T, int CB>
__global__ __launch_bounds__(F64_THREADS, (pipe_waves<T, CB>())) void cheb_step_pipe(
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ tcol,
    const T *__restrict__ vals, const T *__restrict__ Yk, int64_t ldk,
    const T *__restrict__ Yp, int64_t ldp, T *Yo, int64_t ldo, int64_t n_vec,
    int64_t n_ct, int64_t n_block_rows, int64_t cgroup, int64_t n_wg, T alpha, T c,
    T beta, const uint64_t *__restrict__ frag_mask) {
  using M = Mfma4<T>;
  constexpr int NVW = 16 * CB;            // vectors per wave
  __shared__ T sH[2][16 * 4 * F64_S];
  const int64_t L = group_order(blockIdx.x, n_wg, cgroup * ORDER_CHUNK);
  // logical id -> (column group, block row, column tile inside the group)
  const int64_t per_group = n_block_rows * cgroup;
  const int64_t cg = L / per_group, rem = L % per_group;
  const int64_t B = rem / cgroup;
  const int64_t ct = cg * cgroup + rem % cgroup;
  if (ct >= n_ct) return;        // last group may be partial (whole work-group exits)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t col0 = ct * (8 * NVW) + NVW * w + (lane & 15);   // column of block cb: col0 + 16 cb
  const int krow = lane >> 4;    // row of the 4-row k-step this lane loads

  typename M::acc_t acc[CB][4];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[cb][j] = typename M::acc_t{0, 0, 0, 0};

  const int t_begin = rowptr[B], t_end = rowptr[B + 1];
  T hreg[4], b0[CB][4], b1[CB][4];

  // next H tile: half h (rows 32h .. 32h+31) into registers, then into LDS
  auto load_h = [&](int t, int h) {
    const T *Ht = vals + (int64_t)t * kTileElems + 2048 * h;
#pragma unroll
    for (int q = 0; q < 4; ++q) hreg[q] = Ht[tid + F64_THREADS * q];
  };
  // Fragment lane l = i + 16j lives at slot 16j + ((i + j) mod 16) of its
  // fragment: with the fragment stride of 65 this makes both the row-wise stores
  // below and the fragment reads free of LDS bank conflicts.
  auto store_h = [&](int buf, int h) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = 2048 * h + tid + F64_THREADS * q, r = idx >> 6, cc = idx & 63;
      const int kk = cc >> 2, mb = r >> 4, j = cc & 3;
      const int slot = 16 * j + (((r & 15) + j) & 15);
      sH[buf][(kk * 4 + mb) * F64_S + slot] = hreg[q];
    }
  };
  const int rd_slot = (lane & 48) + (((lane & 15) + (lane >> 4)) & 15);
  // quarter qq (k-steps 4qq .. 4qq+3, panel rows 16qq .. 16qq+15) of the Y_k panel of tile t
  // Columns past n_vec (last column tile) read a clamped, in-range column: an
  // output column of the matrix-core product depends only on its own B column,
  // and those columns are never stored.  Unconditional loads keep the prefetch
  // asynchronous (a per-lane guard makes the compiler wait for each load).
  int64_t colc[CB];
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) colc[cb] = min(col0 + 16 * cb, n_vec - 1);
  auto load_b = [&](int t, int qq, T (&dst)[CB][4]) {
    const T *Xp = Yk + ((int64_t)tcol[t] * 64 + 16 * qq + krow) * ldk;
#pragma unroll
    for (int cb = 0; cb < CB; ++cb)
#pragma unroll
      for (int q = 0; q < 4; ++q) dst[cb][q] = Xp[(int64_t)(4 * q) * ldk + colc[cb]];
  };
  // all-zero 16x4 sub-blocks of the tile (bit clear in fm) are skipped; fm is
  // uniform over the work-group, so the branch costs no divergence.  The four A
  // fragments of a k-step are read from LDS before the branches so the reads are
  // not serialised behind them.
  auto mma_quarter = [&](const T *sA, int qq, const T (&bq)[CB][4], uint64_t fm) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int kk = 4 * qq + q;
      T a[4];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) a[mb] = sA[(kk * 4 + mb) * F64_S + rd_slot];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
        if ((fm >> (kk * 4 + mb)) & 1ull) {
#pragma unroll
          for (int cb = 0; cb < CB; ++cb) acc[cb][mb] = M::op(a[mb], bq[cb][q], acc[cb][mb]);
        }
    }
  };
  auto tile_mask = [&](int t) -> uint64_t { return frag_mask ? frag_mask[t] : ~0ull; };

  // Software pipeline over the block row's tiles: while tile t is contracted from
  // LDS buffer buf, tile t+1 is fetched into registers (H in two halves, stored to
  // the other buffer; the Y_k panel in quarters, each refilled as soon as its
  // quarter of tile t is done).  All loads are unconditional: on the last tile
  // the "next" tile is the last tile again, so no value is undefined on any path
  // and the compiler keeps the loads in flight instead of waiting on them.
  if (t_begin < t_end) {
    T b2[CB][4], b3[CB][4];
    load_b(t_begin, 0, b0);
    load_b(t_begin, 1, b1);
    load_b(t_begin, 2, b2);
    load_b(t_begin, 3, b3);
    load_h(t_begin, 0);
    store_h(0, 0);
    load_h(t_begin, 1);
    store_h(0, 1);
    uint64_t fm = tile_mask(t_begin);
    __syncthreads();
    int buf = 0;
    for (int t = t_begin; t < t_end; ++t) {
      const int tn = min(t + 1, t_end - 1);
      const uint64_t fm_next = tile_mask(tn);
      const T *sA = sH[buf];
      load_h(tn, 0);
      mma_quarter(sA, 0, b0, fm);
      load_b(tn, 0, b0);
      store_h(buf ^ 1, 0);
      mma_quarter(sA, 1, b1, fm);
      load_b(tn, 1, b1);
      load_h(tn, 1);
      mma_quarter(sA, 2, b2, fm);
      load_b(tn, 2, b2);
      store_h(buf ^ 1, 1);
      mma_quarter(sA, 3, b3, fm);
      load_b(tn, 3, b3);
      __syncthreads();
      buf ^= 1;
      fm = fm_next;
    }
  }

  // epilogue: all loads of the 64 x 16 slab first, then the stores
#pragma unroll
  for (int cb = 0; cb < CB; ++cb) {
    const int64_t col = col0 + 16 * cb;
    T yk[4][4], yp[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        yk[mb][q] = Yk[(B * 64 + 16 * mb + M::row(lane, q)) * ldk + colc[cb]];
    if (beta != T(0)) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          yp[mb][q] = Yp[(B * 64 + 16 * mb + M::row(lane, q)) * ldp + colc[cb]];
    } else {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q) yp[mb][q] = T(0);
    }
    if (col < n_vec) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t grow = B * 64 + 16 * mb + M::row(lane, q);
          Yo[grow * ldo + col] = alpha * (acc[cb][mb][q] - c * yk[mb][q]) - beta * yp[mb][q];
        }
    }
  }
}

template <typename TX> __device__ inline float to_f32(TX v);
template <> __device__ inline float to_f32<float>(float v) { return v; }
template <> __device__ inline float to_f32<__bf16>(__bf16 v) { return (float)v; }
template <typename TX> __device__ inline TX from_f32(float v);
template <> __device__ inline float from_f32<float>(float v) { return v; }
template <> __device__ inline __bf16 from_f32<__bf16>(float v) { return (__bf16)v; }

// Pipelined BF16 path: BF16 H tiles, FP32 or BF16 iterates, FP32 accumulation
// on the 16x16x32 bf16 op.  Same decomposition as cheb_step_pipe (8 waves,
// 128 vectors, wave w owns vectors 16w .. 16w+15):
//  - A (H tile, 8 KB): double-buffered in LDS in fragment order, lane l of
//    fragment (kk, mb) holding H[16mb + (l&15)][32kk + 8(l>>4) .. +7] as one
//    16-byte read;
//  - B (Y_k): lane l gathers Y_k[32kk + 8(l>>4) + t][col], t = 0..7, rounds to
//    bf16 and packs them; the next tile's values are fetched during the current
//    tile's contraction.
//  - a 16x32 fragment is skipped when all eight 16x4 sub-blocks it covers are
//    clear in the fragment mask.
template <typename TX>
__global__ __launch_bounds__(F64_THREADS, 4) void cheb_step_bf16_pipe(
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ tcol,
    const __bf16 *__restrict__ vals, const TX *__restrict__ Yk, int64_t ldk,
    const TX *__restrict__ Yp, int64_t ldp, TX *Yo, int64_t ldo, int64_t n_vec, int64_t n_ct,
    int64_t n_block_rows, int64_t cgroup, int64_t n_wg, float alpha, float c, float beta,
    const uint64_t *__restrict__ frag_mask) {
  __shared__ __attribute__((aligned(16))) __bf16 sH[2][2 * 4 * 64 * 8];   // [buf][kk][mb][lane][8]
  const int64_t L = group_order(blockIdx.x, n_wg, cgroup * ORDER_CHUNK);
  const int64_t per_group = n_block_rows * cgroup;
  const int64_t cg = L / per_group, rem = L % per_group;
  const int64_t B = rem / cgroup;
  const int64_t ct = cg * cgroup + rem % cgroup;
  if (ct >= n_ct) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t col = ct * F64_NV + 16 * w + (lane & 15);
  const bool col_ok = col < n_vec;
  const int kgrp = lane >> 4;

  v4f acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = v4f{0, 0, 0, 0};
  const int t_begin = rowptr[B], t_end = rowptr[B + 1];

  // H staging: thread tid moves 8 consecutive bf16 of one tile row (16 bytes)
  v8bf hreg;
  auto load_h = [&](int t) {
    hreg = *reinterpret_cast<const v8bf *>(vals + (int64_t)t * kTileElems + 8 * tid);
  };
  auto store_h = [&](int buf) {
    const int r = tid >> 3, c8 = (tid & 7) * 8;          // row r, columns c8 .. c8+7
    const int kk = c8 >> 5, g = (c8 & 31) >> 3, mb = r >> 4;
    const int fl = (r & 15) + 16 * g;
    *reinterpret_cast<v8bf *>(&sH[buf][((kk * 4 + mb) * 64 + fl) * 8]) = hreg;
  };
  // two register sets for the Y_k values: one being contracted, one being fetched
  TX bA[2][8], bB[2][8];
  auto load_b = [&](int t, TX (&dst)[2][8]) {
    const TX *Xp = Yk + (int64_t)tcol[t] * 64 * ldk + col;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kr = 32 * kk + 8 * kgrp + q;
        dst[kk][q] = col_ok ? Xp[(int64_t)kr * ldk] : TX(0);
      }
  };
  // sub-blocks 4*kk4 + mb, kk4 = 8kk .. 8kk+7, sit at bits 32kk + 4j + mb
  auto mma_tile = [&](int buf, uint64_t fm, const TX (&src)[2][8]) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      v8bf b;
#pragma unroll
      for (int q = 0; q < 8; ++q) b[q] = (__bf16)to_f32<TX>(src[kk][q]);
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        if (((fm >> (32 * kk + mb)) & 0x11111111ull) == 0) continue;
        const v8bf a = *reinterpret_cast<const v8bf *>(&sH[buf][((kk * 4 + mb) * 64 + lane) * 8]);
        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mb], 0, 0, 0);
      }
    }
  };
  auto step = [&](int t, int buf, const TX (&cur)[2][8], TX (&nxt)[2][8]) {
    const bool more = t + 1 < t_end;
    const uint64_t fm = frag_mask ? frag_mask[t] : ~0ull;
    if (more) {
      load_h(t + 1);
      load_b(t + 1, nxt);
    }
    mma_tile(buf, fm, cur);
    if (more) store_h(buf ^ 1);
    __syncthreads();
  };

  if (t_begin < t_end) {
    load_h(t_begin);
    load_b(t_begin, bA);
    store_h(0);
    __syncthreads();
  }
  for (int t = t_begin; t < t_end; t += 2) {
    step(t, 0, bA, bB);
    if (t + 1 < t_end) step(t + 1, 1, bB, bA);
  }

  if (!col_ok) return;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t grow = B * 64 + 16 * mb + 4 * (lane >> 4) + q;
      const float y = to_f32<TX>(Yk[grow * ldk + col]);
      float out = alpha * (acc[mb][q] - c * y);
      if (beta != 0.0f) out -= beta * to_f32<TX>(Yp[grow * ldp + col]);
      Yo[grow * ldo + col] = from_f32<TX>(out);
    }
  }
}

}  // namespace

hipError_t launch_cheb_step(const ttdft_bsr &H, const void *Yk, int64_t ldk, const void *Yp,
                            int64_t ldp, void *Yo, int64_t ldo, int64_t n_vec, double alpha,
                            double c, double beta, ttdft_dtype xt, hipStream_t s) {
  if (H.dtype == TTDFT_F64 || H.dtype == TTDFT_F32) {
    const int cb = H.dtype == TTDFT_F64 ? PIPE_CB_F64 : PIPE_CB_F32;
    const int64_t ctp = (n_vec + 128 * cb - 1) / (128 * cb);
    const int64_t cgroup = std::min<int64_t>(ctp, ORDER_CGROUP);
    const int64_t n_groups = (ctp + cgroup - 1) / cgroup;
    const int64_t wg = n_groups * H.n_block_rows * cgroup;
    if (wg > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (H.dtype == TTDFT_F64)
      hipLaunchKernelGGL((cheb_step_pipe<double, PIPE_CB_F64>), dim3((unsigned)wg), dim3(F64_THREADS),
                         0, s, H.tile_rowptr, H.tile_col, (const double *)H.vals, (const double *)Yk,
                         ldk, (const double *)Yp, ldp, (double *)Yo, ldo, n_vec, ctp,
                         H.n_block_rows, cgroup, wg, alpha, c, beta, H.frag_mask);
    else
      hipLaunchKernelGGL((cheb_step_pipe<float, PIPE_CB_F32>), dim3((unsigned)wg), dim3(F64_THREADS),
                         0, s, H.tile_rowptr, H.tile_col, (const float *)H.vals, (const float *)Yk,
                         ldk, (const float *)Yp, ldp, (float *)Yo, ldo, n_vec, ctp,
                         H.n_block_rows, cgroup, wg, (float)alpha, (float)c, (float)beta,
                         H.frag_mask);
  } else {
    const int64_t ctp = (n_vec + F64_NV - 1) / F64_NV;
    const int64_t cgroup = std::min<int64_t>(ctp, ORDER_CGROUP);
    const int64_t n_groups = (ctp + cgroup - 1) / cgroup;
    const int64_t wg = n_groups * H.n_block_rows * cgroup;
    if (wg > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (xt == TTDFT_F32)
      hipLaunchKernelGGL(cheb_step_bf16_pipe<float>, dim3((unsigned)wg), dim3(F64_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const __bf16 *)H.vals, (const float *)Yk, ldk,
                         (const float *)Yp, ldp, (float *)Yo, ldo, n_vec, ctp, H.n_block_rows,
                         cgroup, wg, (float)alpha, (float)c, (float)beta, H.frag_mask);
    else
      hipLaunchKernelGGL(cheb_step_bf16_pipe<__bf16>, dim3((unsigned)wg), dim3(F64_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const __bf16 *)H.vals, (const __bf16 *)Yk,
                         ldk, (const __bf16 *)Yp, ldp, (__bf16 *)Yo, ldo, n_vec, ctp,
                         H.n_block_rows, cgroup, wg, (float)alpha, (float)c, (float)beta,
                         H.frag_mask);
  }
  return hipGetLastError();
}

}  // namespace ttdft
