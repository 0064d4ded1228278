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
// Work decomposition: FP64 and FP32 tiles use cheb_step_mfma<T> (16x16x4 ops):
// one work-group owns one block row B and one column tile of vectors and walks
// the (at most 27) tiles of B, accumulating in matrix-core registers, the tiles
// moved to LDS by LDS-DMA.  BF16 tiles use cheb_step_bf16_patch (16x16x32 bf16
// ops): one work-group owns a 2x2x2 patch of block rows and walks the union of
// their tile columns.  Each output element is produced by exactly one
// work-group, so results are deterministic (no atomics).
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
// XCDs working on neighbouring runs at the same time.  A run of 8 block rows is
// one 2x2x2 patch of lattice blocks in the builder's numbering, whose rows
// share most of their neighbours' Y_k panels in L2 (FP64: 15.7 ms per step at
// the full-size workload, against 16.6 ms for runs of 4 and 17.5 ms for runs
// of 2).
constexpr int ORDER_CGROUP = 16, ORDER_CHUNK = 8;

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
  auto load_b = [&](int64_t brow, int qq, T (&dst)[4]) {   // quarter qq of panel brow
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(Yk + brow * 64 * ldk), 0, panel_bytes, kBufferWord3);
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
  // into b0..b3 (each quarter refilled once contracted).  FP64: after the last
  // tile the refill is the work-group's own panel Y_k[B], whose quarters are in
  // the layout of the f64 op's accumulators (row 16 qq + 4 q + l/16 of the panel
  // is item q of accumulator qq), so the epilogue does not wait for it; the f32
  // op's accumulator rows are 4 (l/16) + q, so FP32 loads its values there.
  constexpr bool kOwnPanel = sizeof(T) == 8;
  auto step = [&](int t, const T *cur, T *nxt, uint64_t fm) {
    const int tn = min(t + 1, t_end - 1);
    const int64_t pn = kOwnPanel && t + 1 >= t_end ? B : (int64_t)tcol[tn];
    if (t + 1 < t_end) dma_h(tn, nxt);       // no tile after the last one
    mma_quarter(cur, 0, b0, fm);
    load_b(pn, 0, b0);
    mma_quarter(cur, 1, b1, fm);
    load_b(pn, 1, b1);
    mma_quarter(cur, 2, b2, fm);
    load_b(pn, 2, b2);
    mma_quarter(cur, 3, b3, fm);
    load_b(pn, 3, b3);
    wait_vmcnt<16>();      // this wave's transfers of tile tn are in LDS
    __syncthreads();
  };

  if (t_begin < t_end) {
    dma_h(t_begin, sH0);
    load_b(tcol[t_begin], 0, b0);
    load_b(tcol[t_begin], 1, b1);
    load_b(tcol[t_begin], 2, b2);
    load_b(tcol[t_begin], 3, b3);
    wait_vmcnt<16>();
    __syncthreads();
    // tiles in pairs (the two LDS buffers stay distinct objects, so the compiler
    // can tell the transfer into one from the reads of the other); an odd last
    // tile, already in sH0, takes one step of its own
    uint64_t fm = tile_mask(t_begin);
    int t = t_begin;
    for (; t + 1 < t_end; t += 2) {
      const uint64_t fm1 = tile_mask(t + 1);
      step(t, sH0, sH1, fm);
      fm = t + 2 < t_end ? tile_mask(t + 2) : 0ull;
      step(t + 1, sH1, sH0, fm1);
    }
    if (t < t_end) step(t, sH0, sH1, fm);
  }

  // epilogue: Y_k[B] (FP64: from the last refill, unless the row has no tiles),
  // Y_{k-1}[B], then the stores
  T yk[4][4], yp[4][4];
  if (kOwnPanel && t_begin < t_end) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      yk[0][q] = b0[q];
      yk[1][q] = b1[q];
      yk[2][q] = b2[q];
      yk[3][q] = b3[q];
    }
  } else {
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        yk[mb][q] = Yk[(B * 64 + 16 * mb + M::row(lane, q)) * ldk + colc];
  }
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
template <> __device__ inline __bf16 buffer_load<__bf16>(__amdgpu_buffer_rsrc_t rs, int32_t voff, int32_t soff) {
  return __builtin_bit_cast(__bf16, __builtin_amdgcn_raw_buffer_load_b16(rs, voff, soff, 0));
}

// ---------------------------------------------------------------------------
// BF16 step kernel over patches of block rows: BF16 tiles (or hi + lo pairs),
// FP32 or BF16 iterates, FP32 accumulation on the 16x16x32 bf16 op.
//
// A work-group owns PB_R = 8 consecutive block rows (one 2x2x2 patch of
// lattice blocks in the builder's numbering) and 128 vectors; wave w owns
// vectors 16w .. 16w+15, lane l the vector 16w + l%16 and the rows
// 8(l/16) .. +7 of each 32-row half of a panel.  The patch rows' tiles are
// walked in the order of their block column: the union of the rows' tile
// columns (4x4x4 = 64 blocks for a patch at h <= 4, against 8 x 27 tiles) is
// built in LDS at the start, and each neighbouring Y_k panel is read once per
// union step and contracted with every patch row's tile in that block column.
// The panels (not the 4x smaller tiles) are most of the step's bytes: this cuts
// the panel reads by 27*8/64 (41 -> 16 GB read beyond L2 per launch at the
// full-size workload).  What bounds the step then is the instruction stream of
// each union step (schedule, slot and count bookkeeping, waits) on two waves
// per SIMD that meet at one barrier, not the bytes.
//  - A (H tiles, 16x32 fragment order) moved to LDS by LDS-DMA through a ring
//    of HS tile slots, as far ahead as the ring allows;
//  - B (Y_k panel): FP32 iterates moved to LDS by buffer LDS-DMA (range-checked
//    against the panel) through a ring of PB_YS stages, PB_YS - 1 union steps
//    ahead (a stage is free again once every lane has read its 8 rows of its
//    vector and rounded them to bf16 at the start of its step; SPLIT:
//    hi = bf16(y), lo = bf16(y - hi)); rows padded so the reads hit 64
//    distinct banks; BF16 iterates are read into registers by buffer loads one
//    union step ahead;
//  - completion of each wave's transfers is tracked by counting the memory
//    instructions it issued after the one waited for (the count after each
//    ring slot's and stage's transfer kept in a lane of a register) and waited
//    for with s_waitcnt (a jump over the possible counts) before a barrier;
//  - the tile ids of a refill are read from LDS with one vector read and taken
//    lane by lane, and ring slots are followed by counters (no division);
//  - every 16x32 fragment of a tile is contracted: skipping the empty ones
//    (16% at h = 4) saves matrix-core work, which is not what bounds this step,
//    and costs a scalar test per fragment;
//  - SPLIT: three products hi*hi + hi*lo + lo*hi per fragment.
// Patches with more than PB_CAP tiles (not produced by stencils with h <= 4) are
// walked one block row at a time in chunks of PB_CAP tiles.
constexpr int PB_R = 8, PB_WAVES = 8, PB_THREADS = 64 * PB_WAVES, PB_NV = 16 * PB_WAVES;
// launch order of the patch kernel: column groups of PB_CGROUP column tiles
// outermost; each XCD takes runs of PB_RUN consecutive patches with all column
// tiles of the group (runs of 2, 4 or 8 neighbouring patches, which share half
// of their neighbour panels, with 16, 8 or 4 column tiles, measured no faster)
constexpr int PB_CGROUP = 16, PB_RUN = 1;
constexpr int PB_CAP = 27 * PB_R;
constexpr int PB_YS = 2;                 // Y panel ring stages
constexpr int PB_YCH = 1024 + 16;        // bytes per two-row chunk of an FP32 panel in LDS

// wait until at most k <= n of this wave's memory instructions are outstanding
// (n wave-uniform; a jump to the matching immediate)
__device__ inline void wait_vmcnt_le(int n) {
  switch (n < 0 ? 0 : (n > 40 ? 40 : n)) {
#define TTDFT_WAIT_CASE(k) case k: wait_vmcnt<k>(); break;
    TTDFT_WAIT_CASE(0) TTDFT_WAIT_CASE(1) TTDFT_WAIT_CASE(2) TTDFT_WAIT_CASE(3) TTDFT_WAIT_CASE(4)
    TTDFT_WAIT_CASE(5) TTDFT_WAIT_CASE(6) TTDFT_WAIT_CASE(7) TTDFT_WAIT_CASE(8) TTDFT_WAIT_CASE(9)
    TTDFT_WAIT_CASE(10) TTDFT_WAIT_CASE(11) TTDFT_WAIT_CASE(12) TTDFT_WAIT_CASE(13) TTDFT_WAIT_CASE(14)
    TTDFT_WAIT_CASE(15) TTDFT_WAIT_CASE(16) TTDFT_WAIT_CASE(17) TTDFT_WAIT_CASE(18) TTDFT_WAIT_CASE(19)
    TTDFT_WAIT_CASE(20) TTDFT_WAIT_CASE(21) TTDFT_WAIT_CASE(22) TTDFT_WAIT_CASE(23) TTDFT_WAIT_CASE(24)
    TTDFT_WAIT_CASE(25) TTDFT_WAIT_CASE(26) TTDFT_WAIT_CASE(27) TTDFT_WAIT_CASE(28) TTDFT_WAIT_CASE(29)
    TTDFT_WAIT_CASE(30) TTDFT_WAIT_CASE(31) TTDFT_WAIT_CASE(32) TTDFT_WAIT_CASE(33) TTDFT_WAIT_CASE(34)
    TTDFT_WAIT_CASE(35) TTDFT_WAIT_CASE(36) TTDFT_WAIT_CASE(37) TTDFT_WAIT_CASE(38) TTDFT_WAIT_CASE(39)
    TTDFT_WAIT_CASE(40)
#undef TTDFT_WAIT_CASE
    default: wait_vmcnt<0>();
  }
}

template <typename TX, bool SPLIT>
__global__ __launch_bounds__(PB_THREADS, 1) void cheb_step_bf16_patch(
    const int32_t *__restrict__ rowptr, const int32_t *__restrict__ tcol,
    const __bf16 *__restrict__ vals, const TX *__restrict__ Yk, int64_t ldk,
    const TX *__restrict__ Yp, int64_t ldp, TX *Yo, int64_t ldo, int64_t n_vec, int64_t n_ct,
    int64_t n_block_rows, int64_t cgroup, int64_t n_wg, float alpha, float c, float beta) {
  constexpr bool YDMA = sizeof(TX) == 4;
  constexpr int PARTS = SPLIT ? 2 : 1;
  constexpr int TILE_VALS = 4096 * PARTS;                  // bf16 values per stored tile
  constexpr int XFER = TILE_VALS * 2 / (PB_THREADS * 16);  // 16-byte H transfers per lane per tile
  constexpr int YX = 32 / PB_WAVES;                        // two-row Y transfers per wave per panel
  // H ring slots (tiles): what the LDS leaves beside the Y ring
  constexpr int HS = !YDMA ? 10 : SPLIT ? (PB_YS == 2 ? 5 : 3) : (PB_YS == 2 ? 10 : 6);
  static_assert(HS <= 64 && PB_YS <= 64, "issue counts are kept one per lane");
  static_assert(!SPLIT || sizeof(TX) == 4, "split products need FP32 iterates");
  __shared__ __attribute__((aligned(16))) __bf16 sH[HS][TILE_VALS];
  __shared__ __attribute__((aligned(16))) char sY[YDMA ? PB_YS * 32 * PB_YCH : 16];
  __shared__ int s_val[PB_CAP], s_row[PB_CAP], s_first[PB_CAP], s_seq[PB_CAP];
  __shared__ int s_ucol[PB_CAP + 1], s_ustart[PB_CAP + 1], s_umask[PB_CAP + 1];
  __shared__ int s_rp[PB_R + 1];

  const int64_t n_patch = (n_block_rows + PB_R - 1) / PB_R;
  const int64_t L = group_order(blockIdx.x, n_wg, cgroup * PB_RUN);
  const int64_t per_group = n_patch * cgroup;
  const int64_t cg = L / per_group, rem = L % per_group;
  const int64_t B0 = (rem / cgroup) * PB_R;
  const int64_t ct = cg * cgroup + rem % cgroup;
  if (ct >= n_ct) return;
  const int nrows = (int)min<int64_t>(PB_R, n_block_rows - B0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 4;
  const int64_t col = ct * PB_NV + 16 * w + (lane & 15);
  // a column past n_vec reads a clamped, in-range column (never stored; an output
  // column depends only on its own B column), so every load is unconditional
  const int64_t colc = min(col, n_vec - 1);

  if (tid <= nrows) s_rp[tid] = rowptr[B0 + tid];

  v4f acc[PB_R][4];
#pragma unroll
  for (int i = 0; i < PB_R; ++i)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) acc[i][mb] = v4f{0, 0, 0, 0};

  const int32_t panel_bytes = (int32_t)(64 * ldk * (int64_t)sizeof(TX));

  // ---- H tile t into ring slot st (16 bytes per lane, fragment order kept)
  auto dma_h = [&](int t, int st) {
    const __bf16 *src = vals + (int64_t)t * TILE_VALS + (w * XFER) * 512 + 8 * lane;
#pragma unroll
    for (int q = 0; q < XFER; ++q) {
      const uint32_t lds = (uint32_t)(uintptr_t)(lds_void_t *)(&sH[st][(w * XFER + q) * 512]);
      asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off"
                   :
                   : "s"(__builtin_amdgcn_readfirstlane(lds)), "v"(src + q * 512)
                   : "memory", "m0");
    }
  };
  // ---- FP32 Y panel of block column Bc into ring stage st: two rows per wave
  // transfer (lanes 0-31 row 2ch, lanes 32-63 row 2ch+1, 4 vectors per lane),
  // chunk ch at st*32*PB_YCH + ch*PB_YCH; offsets past the panel read 0
  const int32_t yvoff = (int32_t)((((int64_t)(lane >> 5) + 2 * w) * ldk + ct * PB_NV + 4 * (lane & 31)) *
                                  (int64_t)sizeof(TX));
  auto dma_y = [&](int64_t Bc, int st) {
    if constexpr (YDMA) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(Yk + Bc * 64 * ldk), 0, panel_bytes, kBufferWord3);
#pragma unroll
      for (int q = 0; q < YX; ++q) {
        const int ch = PB_WAVES * q + w;
        const uint32_t lds = (uint32_t)(uintptr_t)(lds_void_t *)(&sY[st * 32 * PB_YCH + ch * PB_YCH]);
        const int32_t so = (int32_t)(2 * PB_WAVES * q * ldk * (int64_t)sizeof(TX));
        asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, %3 offen lds"
                     :
                     : "s"(__builtin_amdgcn_readfirstlane(lds)), "v"(yvoff), "s"(rs), "s"(so)
                     : "memory", "m0");
      }
    }
  };
  // BF16 iterates: the lane's values straight into registers
  const int32_t voff = (int32_t)(((int64_t)8 * g * ldk + colc) * (int64_t)sizeof(TX));
  TX yr[2][8];
  auto load_y_regs = [&](int64_t Bc) {
    if constexpr (!YDMA) {
      const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
          (void *)(Yk + Bc * 64 * ldk), 0, panel_bytes, kBufferWord3);
#pragma unroll
      for (int kk = 0; kk < 2; ++kk)
#pragma unroll
        for (int t = 0; t < 8; ++t)
          yr[kk][t] = buffer_load<TX>(rs, voff, (int32_t)((32 * kk + t) * ldk * (int64_t)sizeof(TX)));
    }
  };
  v8bf bh[2], bl[2];   // [kk]
  auto convert_y = [&](int st) {
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        float v;
        if constexpr (YDMA) {
          const int r = 32 * kk + 8 * g + t;
          v = *reinterpret_cast<const float *>(
              &sY[st * 32 * PB_YCH + (r >> 1) * PB_YCH + (r & 1) * 512 + 4 * (16 * w + (lane & 15))]);
        } else {
          v = to_f32<TX>(yr[kk][t]);
        }
        bh[kk][t] = (__bf16)v;
        if (SPLIT) bl[kk][t] = (__bf16)(v - (float)bh[kk][t]);
      }
  };
  // all A fragments of a tile are read from LDS before its matrix-core ops, so
  // the LDS latency is paid once per tile
  auto mma_tile = [&](v4f (&ac)[4], const __bf16 *sA) {
    v8bf a[8], alo[SPLIT ? 8 : 1];
#pragma unroll
    for (int f = 0; f < 8; ++f) {
      a[f] = *reinterpret_cast<const v8bf *>(sA + f * 512 + 8 * lane);
      if (SPLIT) alo[f] = *reinterpret_cast<const v8bf *>(sA + 4096 + f * 512 + 8 * lane);
    }
    __builtin_amdgcn_sched_barrier(0);   // keep the reads ahead of the ops
#pragma unroll
    for (int kk = 0; kk < 2; ++kk)
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
        const int f = 4 * kk + mb;
        ac[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f], bh[kk], ac[mb], 0, 0, 0);
        if (SPLIT) {
          ac[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[f], bl[kk], ac[mb], 0, 0, 0);
          ac[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo[f], bh[kk], ac[mb], 0, 0, 0);
        }
      }
  };

  __syncthreads();
  const int e_all0 = s_rp[0], e_all1 = s_rp[nrows];
  const bool one_segment = e_all1 - e_all0 <= PB_CAP;
  // segments: the whole patch, or (rare) each block row in chunks of PB_CAP tiles
  const int n_seg_rows = one_segment ? 1 : nrows;
  for (int sr = 0; sr < n_seg_rows; ++sr) {
    const int r0 = one_segment ? e_all0 : s_rp[sr], r1 = one_segment ? e_all1 : s_rp[sr + 1];
    for (int e_begin = r0; e_begin < r1; e_begin += PB_CAP) {
      const int ne = min(PB_CAP, r1 - e_begin);
      // ---- union schedule of this segment (LDS): distinct block columns in
      // ascending order (union steps u) with the patch rows holding a tile there
      // (bit mask) and the first sequence position of the step; the tile
      // sequence in (column, row) order
      for (int e = tid; e < ne; e += PB_THREADS) {
        const int tt = e_begin + e;
        s_val[e] = tcol[tt];
        int i = 0;
        while (i + 1 < nrows && s_rp[i + 1] <= tt) ++i;
        s_row[e] = i;
        s_umask[e] = 0;
      }
      __syncthreads();
      for (int e = tid; e < ne; e += PB_THREADS) {
        const int v = s_val[e];
        int first = 1;
        for (int e2 = 0; e2 < e; ++e2) first &= (s_val[e2] != v);
        s_first[e] = first;
      }
      __syncthreads();
      for (int e = tid; e < ne; e += PB_THREADS) {
        const int v = s_val[e], i = s_row[e];
        int u = 0, pos = 0, before = 0;
        for (int e2 = 0; e2 < ne; ++e2) {
          const int v2 = s_val[e2];
          u += (s_first[e2] && v2 < v);
          before += (v2 < v);
          pos += (v2 < v || (v2 == v && s_row[e2] < i));
        }
        atomicOr(&s_umask[u], 1 << i);
        if (s_first[e]) {
          s_ucol[u] = v;
          s_ustart[u] = before;
        }
        s_seq[pos] = e_begin + e;
      }
      __syncthreads();
      int nu = 0;
      for (int e = 0; e < ne; ++e) nu += s_first[e];
      if (tid == 0) s_ustart[nu] = ne;
      __syncthreads();

      // ---- pipeline at union-step granularity: one wait and one barrier per
      // step.  H tiles go to ring slot (position % HS) as far ahead as the ring
      // allows, the Y_k panel of step u to stage u % PB_YS, PB_YS - 1 steps
      // ahead.  Each wave counts the memory instructions it has issued and keeps
      // the count after each slot's (hc) and stage's (yc) transfer in the lane
      // of that slot or stage, so it waits for exactly those a step needs.
      int issued = 0, next_h = 0, h_slot = 0;   // h_slot = next_h % HS
      int hc = 0, yc = 0;
      auto issue_h_upto = [&](int lim) {     // positions next_h .. lim-1 (at most HS)
        const int cnt = lim - next_h;
        if (cnt <= 0) return;
        const int sq = s_seq[min(next_h + lane, lim - 1)];
        for (int j = 0; j < cnt; ++j) {
          dma_h(__builtin_amdgcn_readlane(sq, j), h_slot);
          issued += XFER;
          hc = lane == h_slot ? issued : hc;
          h_slot = h_slot + 1 == HS ? 0 : h_slot + 1;
        }
        next_h = lim;
      };
      // ring slot of position q, for next_h - HS <= q < next_h
      auto slot_of = [&](int q) {
        const int sl = h_slot - (next_h - q);
        return sl < 0 ? sl + HS : sl;
      };
      auto issue_y = [&](int u, int st) {
        if constexpr (YDMA) {
          dma_y(__builtin_amdgcn_readfirstlane(s_ucol[u]), st);
          issued += YX;
          yc = lane == st ? issued : yc;
        } else {
          load_y_regs(__builtin_amdgcn_readfirstlane(s_ucol[u]));
        }
      };
      issue_h_upto(min(HS, ne));
      constexpr int YAHEAD = YDMA ? PB_YS - 1 : 1;
      for (int u = 0; u < min(YAHEAD, nu); ++u) issue_y(u, u);
      int y_cur = 0;                          // stage of step u
      for (int u = 0; u < nu; ++u) {
        const int s0 = s_ustart[u], s1 = s_ustart[u + 1];
        const int um = __builtin_amdgcn_readfirstlane(s_umask[u]);
        // the step's tiles in chunks of at most HS positions (one chunk unless the
        // step holds more tiles than the ring)
        for (int p = s0; p < s1; p += HS) {
          const int pe = min(s1, p + HS);
          if (next_h < pe) {
            // positions up to pe - 1 take the slots of positions before p, read by
            // the products of the previous chunk or step: wait for every wave
            __syncthreads();
            issue_h_upto(min(p + HS, ne));
          }
          int need = __builtin_amdgcn_readlane(hc, slot_of(pe - 1));
          if constexpr (YDMA) {
            if (p == s0) need = max(need, __builtin_amdgcn_readlane(yc, y_cur));
          }
          wait_vmcnt_le(issued - need);
          __syncthreads();   // the chunk's transfers (every wave's part) are in LDS;
                             // the slots of earlier positions and step u-1's Y stage are free
          if (p == s0) {
            if constexpr (YDMA) {
              if (u + YAHEAD < nu) issue_y(u + YAHEAD, y_cur == 0 ? PB_YS - 1 : y_cur - 1);
              convert_y(y_cur);
            } else {
              convert_y(0);
              if (u + 1 < nu) issue_y(u + 1, 0);
            }
          }
          issue_h_upto(min(p + HS, ne));   // slots of positions < p are free
          const int slot_p = slot_of(p);
          int pos = s0;
#pragma unroll
          for (int i = 0; i < PB_R; ++i) {
            if (!((um >> i) & 1)) continue;
            if (pos >= p && pos < pe) {
              const int sl = slot_p + (pos - p);
              mma_tile(acc[i], sH[sl >= HS ? sl - HS : sl]);
            }
            ++pos;
          }
        }
        if constexpr (YDMA) y_cur = y_cur + 1 == PB_YS ? 0 : y_cur + 1;
      }
      __syncthreads();   // the schedule arrays and slots are reused by the next segment
    }
  }

  // epilogue per block row of the patch: loads first, then the stores
#pragma unroll
  for (int i = 0; i < PB_R; ++i) {
    if (i >= nrows) break;
    const int64_t B = B0 + i;
    float yk[4][4], yp[4][4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        yk[mb][q] = to_f32<TX>(Yk[(B * 64 + 16 * mb + 4 * g + q) * ldk + colc]);
    if (beta != 0.0f) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          yp[mb][q] = to_f32<TX>(Yp[(B * 64 + 16 * mb + 4 * g + q) * ldp + colc]);
    } else {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q) yp[mb][q] = 0.0f;
    }
    if (col < n_vec) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          Yo[(B * 64 + 16 * mb + 4 * g + q) * ldo + col] =
              from_f32<TX>(alpha * (acc[i][mb][q] - c * yk[mb][q]) - beta * yp[mb][q]);
    }
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
    const int64_t ctp = (n_vec + PB_NV - 1) / PB_NV;
    const int64_t cgroup = std::min<int64_t>(ctp, PB_CGROUP);
    const int64_t n_groups = (ctp + cgroup - 1) / cgroup;
    const int64_t n_patch = (H.n_block_rows + PB_R - 1) / PB_R;
    const int64_t wg = n_groups * n_patch * cgroup;
    if (wg > 0x7fffffff) return hipErrorInvalidConfiguration;
    if (H.dtype == TTDFT_BF16_SPLIT)
      hipLaunchKernelGGL((cheb_step_bf16_patch<float, true>), dim3((unsigned)wg), dim3(PB_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const __bf16 *)H.vals, (const float *)Yk, ldk,
                         (const float *)Yp, ldp, (float *)Yo, ldo, n_vec, ctp, H.n_block_rows,
                         cgroup, wg, (float)alpha, (float)c, (float)beta);
    else if (xt == TTDFT_F32)
      hipLaunchKernelGGL((cheb_step_bf16_patch<float, false>), dim3((unsigned)wg), dim3(PB_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const __bf16 *)H.vals, (const float *)Yk, ldk,
                         (const float *)Yp, ldp, (float *)Yo, ldo, n_vec, ctp, H.n_block_rows,
                         cgroup, wg, (float)alpha, (float)c, (float)beta);
    else
      hipLaunchKernelGGL((cheb_step_bf16_patch<__bf16, false>), dim3((unsigned)wg), dim3(PB_THREADS), 0, s,
                         H.tile_rowptr, H.tile_col, (const __bf16 *)H.vals, (const __bf16 *)Yk,
                         ldk, (const __bf16 *)Yp, ldp, (__bf16 *)Yo, ldo, n_vec, ctp,
                         H.n_block_rows, cgroup, wg, (float)alpha, (float)c, (float)beta);
  }
  return hipGetLastError();
}

}  // namespace ttdft
