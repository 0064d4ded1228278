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
// results are deterministic (no atomics).  FP64 and FP32 tiles use
// cheb_step_mfma<T> (16x16x4 ops, tiles moved to LDS by LDS-DMA); BF16 tiles
// use cheb_step_bf16_pipe (16x16x32 bf16 ops).
//
// Tile values are stored in matrix-core fragment order: element (i, j) of a
// tile at 64*(4*(j/4) + i/16) + 16*(j%4) + i%16, i.e. the 16x4 fragment
// (kk = j/4, mb = i/16) is 64 consecutive values and lane l of the 16x16x4 op
// takes value l of it as its A operand H[16mb + l%16][4kk + l/16].
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

// Work-group shape shared by both kernels: 8 waves, 128 vectors per work-group,
// wave w owning vectors 16w .. 16w+15 of the column tile.
constexpr int F64_NV = 128, F64_THREADS = 512;
// launch order: column groups of ORDER_CGROUP tiles outermost; each XCD takes runs
// of ORDER_CHUNK consecutive block rows (all column tiles of the group), the 8
// XCDs working on neighbouring runs at the same time.  Runs of 4 block rows let
// the rows resident on one XCD share more of their neighbours' Y_k panels in L2
// (measured 3% faster than runs of 1; 8 and longer were slower again).
constexpr int ORDER_CGROUP = 16, ORDER_CHUNK = 4;

__device__ inline int64_t group_order(int64_t g, int64_t G, int64_t C) {
  // hardware ids go round-robin over 8 XCDs; give each XCD C consecutive logical
  // ids (the column tiles of one block row share that XCD's L2), the 8 XCDs
  // working on neighbouring block rows at the same time
  const int64_t span = 8 * C, full = (G / span) * span;
  if (g >= full) return g;
  return (g / span) * span + (g % 8) * C + (g / 8) % C;
}

// ---------------------------------------------------------------------------
// FP64 / FP32 step kernel (T = double: f64 16x16x4 ops; T = float: f32 16x16x4,
// same operand layouts).  Wave w computes the 64 x 16 output slab of vectors
// 16w .. 16w+15 with four 16x16 accumulators.
//  - A operand (H tile): the tile, already in fragment order in memory, is
//    copied to LDS by contiguous 1 KB global_load_lds_dwordx4 transfers (16 bytes
//    per lane, placed at base + 16*lane) without passing through registers; each
//    A read is 64 consecutive values (no bank conflicts, no padding).  Two LDS
//    buffers: the next tile's transfer is issued when the current tile's
//    contraction starts and waited for only before the barrier that ends it.
//  - B operand (Y_k panel): each wave reads its own 16 vectors straight from
//    global memory into registers, a whole tile (16 k-steps) ahead of use.
//  - all-zero 16x4 fragments (clear bits of the fragment mask) are skipped.
typedef __attribute__((address_space(3))) void lds_void_t;

// s_waitcnt vmcnt(N), other counters not waited for (gfx9 encoding)
template <int N> __device__ inline void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// raw buffer load of one value (descriptor word 3 of the gfx9 family: 32-bit
// data, no swizzle); voffset per lane, soffset wave-uniform, both in bytes
constexpr int kBufferWord3 = 0x00020000;
template <typename T> __device__ inline T buffer_load(__amdgpu_buffer_rsrc_t rs, int32_t voff, int32_t soff);
template <> __device__ inline double buffer_load<double>(__amdgpu_buffer_rsrc_t rs, int32_t voff, int32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, 0));
}
template <> __device__ inline float buffer_load<float>(__amdgpu_buffer_rsrc_t rs, int32_t voff, int32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, soff, 0));
}

template <typename T>
__global__ __launch_bounds__(F64_THREADS, 4) void cheb_step_mfma(
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ tcol,
    const T *__restrict__ vals, const T *__restrict__ Yk, int64_t ldk,
    const T *__restrict__ Yp, int64_t ldp, T *Yo, int64_t ldo, int64_t n_vec,
    int64_t n_ct, int64_t n_block_rows, int64_t cgroup, int64_t n_wg, T alpha, T c,
    T beta, const uint64_t *__restrict__ frag_mask) {
  using M = Mfma4<T>;
  constexpr int PER_LANE = 16 / sizeof(T);                 // values per lane per transfer
  constexpr int XFERS = kTileElems / (64 * PER_LANE) / 8;  // transfers per wave per tile
  __shared__ __attribute__((aligned(16))) T sH0[kTileElems];
  __shared__ __attribute__((aligned(16))) T sH1[kTileElems];
  const int64_t L = group_order(blockIdx.x, n_wg, cgroup * ORDER_CHUNK);
  const int64_t per_group = n_block_rows * cgroup;
  const int64_t cg = L / per_group, rem = L % per_group;
  const int64_t B = rem / cgroup;
  const int64_t ct = cg * cgroup + rem % cgroup;
  if (ct >= n_ct) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t col0 = ct * F64_NV + 16 * w + (lane & 15);
  // Columns past n_vec (last column tile) read a clamped, in-range column: an
  // output column of the product depends only on its own B column, and those
  // columns are never stored.  Every load is unconditional, which keeps the
  // prefetch in flight (a per-lane guard makes the compiler wait on each load).
  const int64_t colc = min(col0, n_vec - 1);
  const int krow = lane >> 4;

  typename M::acc_t acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = typename M::acc_t{0, 0, 0, 0};
  const int t_begin = rowptr[B], t_end = rowptr[B + 1];

  // The transfer is written as inline assembly: the compiler then neither orders
  // it against the other loads nor makes barriers wait for every outstanding
  // load on its behalf.  Completion is waited for explicitly (vmcnt counts it;
  // waits the compiler places for other loads can only be stricter than needed).
  auto dma_h = [&](int t, T *dst) {
    const T *src = vals + (int64_t)t * kTileElems + (w * XFERS) * 64 * PER_LANE + PER_LANE * lane;
#pragma unroll
    for (int q = 0; q < XFERS; ++q) {
      const uint32_t lds = (uint32_t)(uintptr_t)(lds_void_t *)(dst + (w * XFERS + q) * 64 * PER_LANE);
      asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                   :
                   : "s"(__builtin_amdgcn_readfirstlane(lds)), "v"(src + q * 64 * PER_LANE)
                   : "memory", "m0");
    }
  };
  T b0[4], b1[4], b2[4], b3[4];
  // Y_k loads are raw buffer loads: the descriptor covers the 64-row panel of
  // tile t (wave-uniform, scalar registers), the per-lane byte offset of row
  // krow, column colc is one 32-bit register and the k-step row offset a scalar,
  // so the 16 loads of a tile need no 64-bit address registers.  Reads past the
  // descriptor's range would return 0 instead of faulting.
  const int32_t yoff = (int32_t)(((int64_t)krow * ldk + colc) * (int64_t)sizeof(T));
  const int32_t panel_bytes = (int32_t)(64 * ldk * (int64_t)sizeof(T));
  auto load_b = [&](int t, int qq, T (&dst)[4]) {
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(Yk + (int64_t)tcol[t] * 64 * ldk), 0, panel_bytes, kBufferWord3);
#pragma unroll
    for (int q = 0; q < 4; ++q)
      dst[q] = buffer_load<T>(rs, yoff, (int32_t)((16 * qq + 4 * q) * ldk * (int64_t)sizeof(T)));
  };
  // the 16 A fragments of a quarter (4 k-steps) are read from LDS before its
  // matrix-core ops, so the LDS latency is paid once per quarter
  auto mma_quarter = [&](const T *sA, int qq, const T (&bq)[4], uint64_t fm) {
    T a[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) a[q][mb] = sA[((4 * qq + q) * 4 + mb) * 64 + lane];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
        if ((fm >> ((4 * qq + q) * 4 + mb)) & 1ull) acc[mb] = M::op(a[q][mb], bq[q], acc[mb]);
  };
  auto tile_mask = [&](int t) -> uint64_t { return frag_mask ? frag_mask[t] : ~0ull; };
  // one tile: contract `cur`, meanwhile move tile tn into `nxt` and its Y_k panel
  // into b0..b3 (each quarter refilled once contracted)
  auto step = [&](int t, const T *cur, T *nxt, uint64_t fm) {
    const int tn = min(t + 1, t_end - 1);   // t may be t_end (empty step)
    dma_h(tn, nxt);
    mma_quarter(cur, 0, b0, fm);
    load_b(tn, 0, b0);
    mma_quarter(cur, 1, b1, fm);
    load_b(tn, 1, b1);
    mma_quarter(cur, 2, b2, fm);
    load_b(tn, 2, b2);
    mma_quarter(cur, 3, b3, fm);
    load_b(tn, 3, b3);
    wait_vmcnt<16>();      // this wave's transfers of tile tn are in LDS
    __syncthreads();
  };

  if (t_begin < t_end) {
    dma_h(t_begin, sH0);
    load_b(t_begin, 0, b0);
    load_b(t_begin, 1, b1);
    load_b(t_begin, 2, b2);
    load_b(t_begin, 3, b3);
    wait_vmcnt<16>();
    __syncthreads();
    // tiles in pairs (the two LDS buffers stay distinct objects, so the compiler
    // can tell the transfer into one from the reads of the other); an odd last
    // tile is paired with an empty step (mask 0: no products)
    uint64_t fm = tile_mask(t_begin);
    for (int t = t_begin; t < t_end; t += 2) {
      const uint64_t fm1 = t + 1 < t_end ? tile_mask(t + 1) : 0ull;
      step(t, sH0, sH1, fm);
      fm = t + 2 < t_end ? tile_mask(t + 2) : 0ull;
      step(t + 1, sH1, sH0, fm1);
    }
  }

  // epilogue: loads first, then the stores
  T yk[4][4], yp[4][4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      yk[mb][q] = Yk[(B * 64 + 16 * mb + M::row(lane, q)) * ldk + colc];
  if (beta != T(0)) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        yp[mb][q] = Yp[(B * 64 + 16 * mb + M::row(lane, q)) * ldp + colc];
  } else {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int q = 0; q < 4; ++q) yp[mb][q] = T(0);
  }
  if (col0 >= n_vec) return;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t grow = B * 64 + 16 * mb + M::row(lane, q);
      Yo[grow * ldo + col0] = alpha * (acc[mb][q] - c * yk[mb][q]) - beta * yp[mb][q];
    }
}

template <typename TX> __device__ inline float to_f32(TX v);
template <> __device__ inline float to_f32<float>(float v) { return v; }
template <> __device__ inline float to_f32<__bf16>(__bf16 v) { return (float)v; }
template <typename TX> __device__ inline TX from_f32(float v);
template <> __device__ inline float from_f32<float>(float v) { return v; }
template <> __device__ inline __bf16 from_f32<__bf16>(float v) { return (__bf16)v; }

// Pipelined BF16 path: BF16 H tiles, FP32 or BF16 iterates, FP32 accumulation
// on the 16x16x32 bf16 op.  Same decomposition as cheb_step_mfma (8 waves,
// 128 vectors, wave w owns vectors 16w .. 16w+15):
//  - A (H tile, 8 KB): double-buffered in LDS in the 16x32 fragment order of
//    the bf16 op, lane l of fragment (kk, mb) holding H[16mb + (l&15)][32kk +
//    8(l>>4) .. +7] as one 16-byte read; each thread loads 16 bytes of the tile
//    (8 rows of one column in the stored 16x4 fragment order) and scatters them;
//  - B (Y_k): lane l gathers Y_k[32kk + 8(l>>4) + t][col], t = 0..7, rounds to
//    bf16 and packs them; the next tile's values are fetched during the current
//    tile's contraction.
//  - a 16x32 fragment is skipped when all eight 16x4 sub-blocks it covers are
//    clear in the fragment mask.
//  - SPLIT (BF16_SPLIT tiles, FP32 iterates): the tile holds hi and lo bf16
//    parts, each iterate value y is split into hi = bf16(y), lo = bf16(y - hi),
//    and every fragment takes the three products hi*hi + hi*lo + lo*hi (the
//    lo*lo term, 2^-16 relative, is dropped).
template <typename TX, bool SPLIT>
__global__ __launch_bounds__(F64_THREADS, 4) void cheb_step_bf16_pipe(
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ tcol,
    const __bf16 *__restrict__ vals, const TX *__restrict__ Yk, int64_t ldk,
    const TX *__restrict__ Yp, int64_t ldp, TX *Yo, int64_t ldo, int64_t n_vec, int64_t n_ct,
    int64_t n_block_rows, int64_t cgroup, int64_t n_wg, float alpha, float c, float beta,
    const uint64_t *__restrict__ frag_mask) {
  constexpr int PARTS = SPLIT ? 2 : 1;
  static_assert(!SPLIT || sizeof(TX) == 4, "split products need FP32 iterates");
  // [buf][part][kk][mb][lane][8]
  __shared__ __attribute__((aligned(16))) __bf16 sH[2][PARTS * 2 * 4 * 64 * 8];
  const int64_t L = group_order(blockIdx.x, n_wg, cgroup * ORDER_CHUNK);
  const int64_t per_group = n_block_rows * cgroup;
  const int64_t cg = L / per_group, rem = L % per_group;
  const int64_t B = rem / cgroup;
  const int64_t ct = cg * cgroup + rem % cgroup;
  if (ct >= n_ct) return;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t col = ct * F64_NV + 16 * w + (lane & 15);
  // columns past n_vec load a clamped in-range column (never stored; an output
  // column depends only on its own B column), so every load is unconditional
  const int64_t colc = min(col, n_vec - 1);
  const int kgrp = lane >> 4;

  v4f acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = v4f{0, 0, 0, 0};
  const int t_begin = rowptr[B], t_end = rowptr[B + 1];

  // H staging: thread tid moves 8 consecutive stored bf16 (16 bytes) per part
  v8bf hreg[PARTS];
  auto load_h = [&](int t) {
#pragma unroll
    for (int pt = 0; pt < PARTS; ++pt)
      hreg[pt] = *reinterpret_cast<const v8bf *>(vals + (int64_t)t * PARTS * kTileElems +
                                                 pt * kTileElems + 8 * tid);
  };
  auto store_h = [&](int buf) {
    // thread tid holds stored values 8 tid .. 8 tid + 7: fragment f = tid / 8 of
    // the 16x4 order, its lanes fl0 .. fl0 + 7, i.e. rows i0 .. i0 + 7 of column j
    const int f = tid >> 3, fl0 = (tid & 7) * 8;
    const int i0 = 16 * (f & 3) + (fl0 & 15), j = 4 * (f >> 2) + (fl0 >> 4);
    const int kk = j >> 5, g = (j & 31) >> 3, e = j & 7, mb = i0 >> 4;
#pragma unroll
    for (int pt = 0; pt < PARTS; ++pt) {
      __bf16 *dst = &sH[buf][pt * kTileElems + ((kk * 4 + mb) * 64 + (i0 & 15) + 16 * g) * 8 + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) dst[8 * u] = hreg[pt][u];
    }
  };
  // two register sets for the Y_k values: one being contracted, one being fetched
  TX bA[2][8], bB[2][8];
  auto load_b = [&](int t, TX (&dst)[2][8]) {
    const TX *Xp = Yk + (int64_t)tcol[t] * 64 * ldk + colc;
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int kr = 32 * kk + 8 * kgrp + q;
        dst[kk][q] = Xp[(int64_t)kr * ldk];
      }
  };
  // sub-blocks 4*kk4 + mb, kk4 = 8kk .. 8kk+7, sit at bits 32kk + 4j + mb
  auto mma_tile = [&](int buf, uint64_t fm, const TX (&src)[2][8]) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      v8bf b, blo;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float y = to_f32<TX>(src[kk][q]);
        b[q] = (__bf16)y;
        if (SPLIT) blo[q] = (__bf16)(y - (float)b[q]);
      }
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        if (((fm >> (32 * kk + mb)) & 0x11111111ull) == 0) continue;
        const v8bf a = *reinterpret_cast<const v8bf *>(&sH[buf][((kk * 4 + mb) * 64 + lane) * 8]);
        acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mb], 0, 0, 0);
        if (SPLIT) {
          const v8bf alo = *reinterpret_cast<const v8bf *>(
              &sH[buf][kTileElems + ((kk * 4 + mb) * 64 + lane) * 8]);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, blo, acc[mb], 0, 0, 0);
          acc[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, b, acc[mb], 0, 0, 0);
        }
      }
    }
  };
  // the last tile fetches itself again as "next": no load is conditional
  auto step = [&](int t, int buf, const TX (&cur)[2][8], TX (&nxt)[2][8]) {
    const int tn = min(t + 1, t_end - 1);
    const uint64_t fm = frag_mask ? frag_mask[t] : ~0ull;
    load_h(tn);
    load_b(tn, nxt);
    mma_tile(buf, fm, cur);
    store_h(buf ^ 1);
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

  // epilogue: loads first, then the stores
  float yk[4][4], yp[4][4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      yk[mb][q] = to_f32<TX>(Yk[(B * 64 + 16 * mb + 4 * (lane >> 4) + q) * ldk + colc]);
  if (beta != 0.0f) {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        yp[mb][q] = to_f32<TX>(Yp[(B * 64 + 16 * mb + 4 * (lane >> 4) + q) * ldp + colc]);
  } else {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int q = 0; q < 4; ++q) yp[mb][q] = 0.0f;
  }
  if (col >= n_vec) return;
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t grow = B * 64 + 16 * mb + 4 * (lane >> 4) + q;
      Yo[grow * ldo + col] = from_f32<TX>(alpha * (acc[mb][q] - c * yk[mb][q]) - beta * yp[mb][q]);
    }
}

}  // namespace

hipError_t launch_cheb_step(const ttdft_bsr &H, const void *Yk, int64_t ldk, const void *Yp,
                            int64_t ldp, void *Yo, int64_t ldo, int64_t n_vec, double alpha,
                            double c, double beta, ttdft_dtype xt, hipStream_t s) {
  if (H.dtype == TTDFT_F64 || H.dtype == TTDFT_F32) {
    const int64_t ctp = (n_vec + F64_NV - 1) / F64_NV;
    const int64_t cgroup = std::min<int64_t>(ctp, ORDER_CGROUP);
    const int64_t n_groups = (ctp + cgroup - 1) / cgroup;
    const int64_t wg = n_groups * H.n_block_rows * cgroup;
    if (wg > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (H.dtype == TTDFT_F64)
      hipLaunchKernelGGL(cheb_step_mfma<double>, dim3((unsigned)wg), dim3(F64_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const double *)H.vals, (const double *)Yk,
                         ldk, (const double *)Yp, ldp, (double *)Yo, ldo, n_vec, ctp,
                         H.n_block_rows, cgroup, wg, alpha, c, beta, H.frag_mask);
    else
      hipLaunchKernelGGL(cheb_step_mfma<float>, dim3((unsigned)wg), dim3(F64_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const float *)H.vals, (const float *)Yk,
                         ldk, (const float *)Yp, ldp, (float *)Yo, ldo, n_vec, ctp,
                         H.n_block_rows, cgroup, wg, (float)alpha, (float)c, (float)beta,
                         H.frag_mask);
  } else {
    const int64_t ctp = (n_vec + F64_NV - 1) / F64_NV;
    const int64_t cgroup = std::min<int64_t>(ctp, ORDER_CGROUP);
    const int64_t n_groups = (ctp + cgroup - 1) / cgroup;
    const int64_t wg = n_groups * H.n_block_rows * cgroup;
    if (wg > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (H.dtype == TTDFT_BF16_SPLIT)
      hipLaunchKernelGGL((cheb_step_bf16_pipe<float, true>), dim3((unsigned)wg), dim3(F64_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const __bf16 *)H.vals, (const float *)Yk, ldk,
                         (const float *)Yp, ldp, (float *)Yo, ldo, n_vec, ctp, H.n_block_rows,
                         cgroup, wg, (float)alpha, (float)c, (float)beta, H.frag_mask);
    else if (xt == TTDFT_F32)
      hipLaunchKernelGGL((cheb_step_bf16_pipe<float, false>), dim3((unsigned)wg), dim3(F64_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const __bf16 *)H.vals, (const float *)Yk, ldk,
                         (const float *)Yp, ldp, (float *)Yo, ldo, n_vec, ctp, H.n_block_rows,
                         cgroup, wg, (float)alpha, (float)c, (float)beta, H.frag_mask);
    else
      hipLaunchKernelGGL((cheb_step_bf16_pipe<__bf16, false>), dim3((unsigned)wg), dim3(F64_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const __bf16 *)H.vals, (const __bf16 *)Yk,
                         ldk, (const __bf16 *)Yp, ldp, (__bf16 *)Yo, ldo, n_vec, ctp,
                         H.n_block_rows, cgroup, wg, (float)alpha, (float)c, (float)beta,
                         H.frag_mask);
  }
  return hipGetLastError();
}

}  // namespace ttdft
