/*
 * ttdft.h - C ABI of the MI355X (gfx950) Chebyshev-filtered subspace iteration
 * hot path of the Tucker tensor DFT method (Lin & Gavini, arXiv 2110.15853).
 *
 * The operations are those of Algorithm 1 (ChFSI, Sec. 3.4):
 *   step 1  Chebyshev filter      Y = T_m((H - cI)/e) X / T_m((a0 - c)/e)
 *   step 2  orthonormalisation    X_F = Orth(Y)            (Cholesky-QR, FP64)
 *   step 3  subspace projection   H_F = X_F^T H X_F         (FP64, Sec. 4.3)
 *   step 4  dense eigensolve      H_F Q = Q Lambda          (FP64)
 *   step 5  rotation              Psi = X_F Q               (FP64)
 * plus the adjoint of step 1 (gradients with respect to X and to the stored
 * entries of H).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers named "device" point to GPU memory owned by the caller; the
 *   library never frees them and allocates no device memory of its own.
 *   Host pointers are marked "host".
 * - Dense blocks (X, Y, ...) are row-major: element (i, j) is at p[i*ld + j],
 *   with ld >= number of columns.  Rows are in the lattice-blocked order
 *   produced by ttdft_bsr_build (64 rows per 4x4x4 lattice block; padding rows
 *   are zero on input and stay zero).
 * - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 * - Every entry point validates all arguments on the host before any device
 *   work; a failed validation returns an error status and writes nothing.
 * - Entry points marked ASYNC only enqueue work on the stream and report launch
 *   errors (TTDFT_ERR_HIP); the others synchronise the stream before returning.
 * - A thread-local message describing the last error is available from
 *   ttdft_last_error().
 * - Blocks multiplied by H (the filter's iterates, the projection's Q, the
 *   residuals' Psi) are addressed by the step kernel with 32-bit byte offsets
 *   inside 64-row panels: 64 * ld * element size must be at most 2^31 - 1
 *   (ld <= 4,194,303 for FP64), else TTDFT_ERR_SHAPE.
 */
#ifndef TTDFT_H
#define TTDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TTDFT_OK = 0,
  TTDFT_ERR_NULL = 1,           /* a required pointer is NULL                        */
  TTDFT_ERR_SHAPE = 2,          /* sizes / leading dimensions inconsistent           */
  TTDFT_ERR_DTYPE = 3,          /* unsupported dtype or dtype combination            */
  TTDFT_ERR_BOUNDS = 4,         /* filter bounds not finite or not a0 < a < b        */
  TTDFT_ERR_DEGREE = 5,         /* polynomial degree m < 1                           */
  TTDFT_ERR_ALIAS = 6,          /* an output overlaps an input it may not overlap    */
  TTDFT_ERR_WORKSPACE = 7,      /* workspace NULL or smaller than the query result   */
  TTDFT_ERR_NOT_POSDEF = 8,     /* Cholesky breakdown (rank-deficient block)         */
  TTDFT_ERR_NO_CONVERGENCE = 9, /* the dense eigensolver did not converge            */
  TTDFT_ERR_NONFINITE = 10,     /* a non-finite value where a finite one is required */
  TTDFT_ERR_HIP = 11,           /* a HIP runtime call or kernel launch failed        */
  TTDFT_ERR_PATTERN = 12        /* CSR input malformed (unsorted, out of range)      */
} ttdft_status;

/*
 * Element types.  TTDFT_BF16_SPLIT is a tile-value type only: each value h is
 * held as a pair of bf16, hi = bf16(fp32(h)) and lo = bf16(fp32(h) - hi)
 * (round to nearest even), so hi + lo carries 16 significant bits; the step
 * kernel forms the three products hi*hi + hi*lo + lo*hi with the FP32
 * iterates split the same way (bf16x3 on the bf16 matrix cores).
 */
typedef enum { TTDFT_F64 = 0, TTDFT_F32 = 1, TTDFT_BF16 = 2, TTDFT_BF16_SPLIT = 3 } ttdft_dtype;

/*
 * Lattice-blocked BSR matrix (all arrays device, caller-owned).
 * The sparse symmetric Hamiltonian H^L of Sec. 3.3 has entries only between
 * nearby lattice sites (locality of the localized Tucker basis, Sec. 4.1).  Rows
 * are grouped by 4x4x4 lattice blocks into block rows of 64; each stored tile is
 * the dense 64x64 coupling between two blocks.  Site (i, j, k) of the lattice
 * lies in block (i/4, j/4, k/4) at local position
 * 16*(2*((i%4)/2) + (j%4)/2) + 4*(2*(i%2) + j%2) + k%4: sixteen consecutive
 * rows are a 2x2x4 box, four consecutive columns a line along k.  The blocks
 * are numbered by 2x2x2 patches: each complete patch of blocks takes eight
 * consecutive numbers (its blocks in (i, j, k) order, patches in lexicographic
 * order), and the blocks of the incomplete patches at the far faces (an odd
 * number of blocks per axis) come last.  perm from ttdft_bsr_build records the
 * resulting row order.
 */
typedef struct {
  int64_t n_block_rows;        /* number of 64-row blocks; padded row count is 64*n_block_rows */
  int64_t n_tiles;             /* number of stored 64x64 tiles                                 */
  const int32_t *tile_rowptr;  /* device [n_block_rows+1]: tiles of block row B are
                                  tile_rowptr[B] .. tile_rowptr[B+1]-1                         */
  const int32_t *tile_col;     /* device [n_tiles]: block column of each tile, ascending in a row */
  const void *vals;            /* device [n_tiles*4096] values, dtype below, each tile in
                                  the matrix-core fragment order of its type.  F64 and F32:
                                  entry (i, j) of tile t at t*4096 + 64*(4*(j/4) + i/16) +
                                  16*(j%4) + i%16 (the 16x4 sub-block of rows 16*(i/16)..,
                                  columns 4*(j/4).. is 64 consecutive values, column-major
                                  inside).  BF16: at t*4096 + 512*(4*(j/32) + i/16) +
                                  8*(i%16 + 16*((j%32)/8)) + j%8 (the 16x32 fragment of the
                                  bf16 op, 8 consecutive columns of one row per 16 bytes).
                                  BF16_SPLIT: [n_tiles*8192] bf16, tile t = the 4096 hi
                                  values at t*8192 + p, then the 4096 lo values at
                                  t*8192 + 4096 + p (p the BF16 position above)        */
  ttdft_dtype dtype;
  const uint64_t *frag_mask;   /* device [n_tiles] or NULL: bit (4*kk + mb) set when the 16x4
                                  sub-block rows 16mb..16mb+15, columns 4kk..4kk+3 of the tile
                                  holds a stored entry; clear bits are skipped by the
                                  matrix-core contraction.  NULL = contract every sub-block.  */
} ttdft_bsr;

/* ---------------------------------------------------------------- host-side builder */

/*
 * Size query for ttdft_bsr_build.  Input: the natural-order CSR of an N x N
 * matrix on an r x r x r lattice (N = r^3, row index (i*r + j)*r + k), host
 * arrays rowptr[N+1] (int64) and col[nnz] (int32, ascending within each row).
 * Output (host): the number of 64-row blocks and of stored tiles.
 * Errors: TTDFT_ERR_NULL, TTDFT_ERR_SHAPE (r < 1), TTDFT_ERR_PATTERN.
 */
ttdft_status ttdft_bsr_plan(int32_t r, const int64_t *rowptr, const int32_t *col,
                            int64_t *n_block_rows, int64_t *n_tiles);

/*
 * Size query with an explicit tile extent: the number of stored tiles of the
 * blk x blk x blk lattice blocking of the same natural-order CSR (host arrays
 * as for ttdft_bsr_plan).  The kernels are built for blk = 4 (64-row tiles
 * matching the 16x16x4 matrix-core fragments); any other blk returns
 * TTDFT_ERR_SHAPE.  n_tiles_out: host.  The number of block rows is
 * ceil(r/4)^3.  Errors: as ttdft_bsr_plan.
 */
ttdft_status ttdft_bsr_build_size(int32_t r, int32_t blk, const int64_t *rowptr, const int32_t *col,
                                  int64_t *n_tiles_out);

/*
 * Builds the lattice-blocked BSR arrays (all host buffers, caller-allocated
 * with the sizes from ttdft_bsr_plan):
 *   tile_rowptr[n_block_rows+1], tile_col[n_tiles],
 *   vals[n_tiles*4096] of dtype (F64, F32 or BF16; rounding to nearest even), in
 *   the fragment order of ttdft_bsr.vals for that dtype ([n_tiles*8192] for
 *   BF16_SPLIT),
 *   perm[64*n_block_rows]: blocked row -> natural row, or -1 for a padding row,
 *   entry_slot[nnz] (may be NULL): flat index into vals of each CSR entry (of
 *   its hi value for BF16_SPLIT; lo at +4096),
 *   mask[n_tiles*64] (may be NULL): bit j of word (t*64 + i) set when entry
 *   (i, j) of tile t is a stored CSR entry,
 *   frag_mask[n_tiles] (may be NULL): bit (4*kk + mb) set when the 16x4
 *   sub-block (rows 16mb.., columns 4kk..) of tile t holds a stored entry.
 * The lattice is padded to a multiple of 4 per axis with zero rows/columns.
 * Errors: as ttdft_bsr_plan, plus TTDFT_ERR_DTYPE.
 */
ttdft_status ttdft_bsr_build(int32_t r, const int64_t *rowptr, const int32_t *col,
                             const double *val, ttdft_dtype dtype,
                             int32_t *tile_rowptr, int32_t *tile_col, void *vals,
                             int64_t *perm, int64_t *entry_slot, uint64_t *mask,
                             uint64_t *frag_mask);

/* ---------------------------------------------------------------- step 1: Chebyshev filter */

/*
 * One fused degree step of the scaled three-term recurrence of Algorithm 1
 * (Sec. 3.4):  Yout = alpha*(H*Yk - c*Yk) - beta*Yprev.
 * H: F64 with x_dtype F64; F32 with F32; BF16 with F32 or BF16.
 * Yk, Yprev, Yout: device, 64*n_block_rows x n_vec of x_dtype, leading dims ldk,
 * ldp, ldo.  Yprev may be NULL only when beta == 0.  Yout may be Yprev (the
 * update is row-local) but must not overlap Yk.  Accumulation is FP64 for F64
 * and FP32 otherwise.  ASYNC.
 * Errors: NULL, SHAPE, DTYPE, ALIAS, NONFINITE (alpha, c or beta), HIP.
 */
ttdft_status ttdft_cheb_step(const ttdft_bsr *H, const void *Yk, int64_t ldk,
                             const void *Yprev, int64_t ldp, void *Yout, int64_t ldo,
                             int64_t n_vec, double alpha, double c, double beta,
                             ttdft_dtype x_dtype, void *stream);

/* Bytes of workspace ttdft_cheb_filter needs (one 64*n_block_rows x n_vec block). */
size_t ttdft_cheb_filter_workspace(const ttdft_bsr *H, int64_t n_vec, ttdft_dtype x_dtype);

/*
 * Step 1 of Algorithm 1: the degree-m Chebyshev filter with unwanted interval
 * [a, b] (a = upper bound of the wanted spectrum, b = upper bound of the whole
 * spectrum) and scaling point a0 below the wanted spectrum (Sec. 3.4):
 *   Y = T_m((H - cI)/e) X / T_m((a0 - c)/e),  e = (b - a)/2,  c = (b + a)/2,
 * computed by m fused steps (ttdft_cheb_step) with the sigma-scaled
 * coefficients alpha_k, beta_k of Algorithm 1.
 * X (device, read-only) and Y (device, output) are 64*n_block_rows x n_vec of
 * x_dtype; work is a device buffer of ttdft_cheb_filter_workspace bytes.
 * Y must not overlap X or work.  ASYNC.
 * Errors: NULL, SHAPE, DTYPE, BOUNDS (requires a0 < a < b, all finite),
 * DEGREE (m < 1), ALIAS, WORKSPACE, HIP.
 */
ttdft_status ttdft_cheb_filter(const ttdft_bsr *H, const void *X, int64_t ldx, void *Y,
                               int64_t ldy, int64_t n_vec, int32_t m, double a, double b,
                               double a0, ttdft_dtype x_dtype, void *work, size_t work_bytes,
                               void *stream);

/*
 * Step 1 of Algorithm 1 with a precision schedule: the filter of
 * ttdft_cheb_filter (same coefficients, same iterates in x_dtype) where the
 * first m - m_late degree steps take their product with H_early and the last
 * m_late steps with H_late, normally the same Hamiltonian in a cheaper and a
 * more accurate tile format (e.g. BF16 then FP32, or BF16 then BF16_SPLIT, all
 * with F32 iterates).  An error made in an early step is damped in the
 * unwanted directions by the later steps (Sec. 3.4: the filter suppresses the
 * unwanted spectrum), so the accurate format is needed only at the end.  Both
 * matrices must describe the same blocked pattern (same n_block_rows and
 * n_tiles, same tile_rowptr / tile_col content) and each must support
 * x_dtype.  m_late = 0 is ttdft_cheb_filter with H_early, m_late = m with
 * H_late.  work as for ttdft_cheb_filter.  ASYNC.
 * Errors: as ttdft_cheb_filter; SHAPE when the two matrices differ in size;
 * DEGREE when m_late lies outside 0 .. m.
 */
ttdft_status ttdft_cheb_filter_schedule(const ttdft_bsr *H_early, const ttdft_bsr *H_late,
                                        int32_t m_late, const void *X, int64_t ldx, void *Y,
                                        int64_t ldy, int64_t n_vec, int32_t m, double a, double b,
                                        double a0, ttdft_dtype x_dtype, void *work,
                                        size_t work_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the filter of
 * ttdft_cheb_filter with the same arguments except the workspace, which is a
 * fixed device array inside the library of TTDFT_NOALLOC_SCRATCH_BYTES (64 MiB)
 * per GPU, held from the first call on a GPU until the process ends.  The call
 * allocates nothing.  The work block (64*n_block_rows x n_vec of x_dtype,
 * needed for m >= 2) must fit in the array: larger problems are rejected with
 * WORKSPACE before any device work.  The stream must belong to the current
 * device.  Every call on one GPU shares that GPU's array, so calls that overlap
 * in time on one GPU race; calls on one stream, one after another, do not.
 * Results are bitwise those of ttdft_cheb_filter.  ASYNC.
 * Errors: as ttdft_cheb_filter (WORKSPACE when the block exceeds the array),
 * HIP (also when the array's device address cannot be looked up).
 */
#define TTDFT_NOALLOC_SCRATCH_BYTES (64ull << 20)
ttdft_status ttdft_cheb_filter_noalloc(const ttdft_bsr *H, const void *X, int64_t ldx, void *Y,
                                       int64_t ldy, int64_t n_vec, int32_t m, double a, double b,
                                       double a0, ttdft_dtype x_dtype, void *stream);

/* ---------------------------------------------------------------- precision casts */

/*
 * dst = src converted between F64, F32 and BF16 (round to nearest even), for a
 * rows x cols row-major block with leading dims lds / ldd.  Device buffers that
 * must not overlap.  ASYNC.  Errors: NULL, SHAPE, DTYPE, ALIAS, HIP.
 */
ttdft_status ttdft_cast(const void *src, ttdft_dtype src_dtype, int64_t lds, void *dst,
                        ttdft_dtype dst_dtype, int64_t ldd, int64_t rows, int64_t cols,
                        void *stream);

/*
 * FP64 tile values (n_tiles*4096, fragment order, e.g. the vals of an F64
 * ttdft_bsr) to the BF16_SPLIT layout (n_tiles*8192 bf16: per tile the hi
 * values, then the lo values, in the BF16 fragment order), on the device.
 * Same as ttdft_convert_tiles(src, F64, n_tiles, dst, BF16_SPLIT).  src, dst:
 * device, not overlapping.  ASYNC.  Errors: NULL, SHAPE (n_tiles < 0), ALIAS, HIP.
 */
ttdft_status ttdft_split_bf16(const double *src, int64_t n_tiles, void *dst, void *stream);

/*
 * Tile values of a ttdft_bsr converted to another tile type on the device, in
 * the fragment order of the destination type (see ttdft_bsr.vals): F64 or F32
 * source (n_tiles*4096) to F32 (rounded, same order), BF16 (bf16(fp32(h)),
 * reordered) or BF16_SPLIT (hi and lo, reordered; n_tiles*8192 bf16).  The
 * pattern arrays of the source matrix serve the converted one unchanged.
 * src, dst: device, not overlapping.  ASYNC.
 * Errors: NULL, SHAPE (n_tiles < 0), DTYPE (other pairs), ALIAS, HIP.
 */
ttdft_status ttdft_convert_tiles(const void *src, ttdft_dtype src_dtype, int64_t n_tiles, void *dst,
                                 ttdft_dtype dst_dtype, void *stream);

/*
 * Row gather: dst[i, :] = src[perm[i], :] for perm[i] >= 0 and 0 for
 * perm[i] < 0 (moves blocks between natural and lattice-blocked row order).
 * perm: device int64 [rows_dst]; entries must be < rows_src.  8-byte (F64),
 * 4-byte (F32) or 2-byte (BF16) elements.  ASYNC.
 * Errors: NULL, SHAPE, DTYPE, ALIAS, HIP.
 */
ttdft_status ttdft_gather_rows(const void *src, int64_t lds, int64_t rows_src, void *dst,
                               int64_t ldd, int64_t rows_dst, int64_t cols,
                               const int64_t *perm, ttdft_dtype dtype, void *stream);

/* ---------------------------------------------------------------- steps 2-5: Rayleigh-Ritz */

/* Bytes of workspace ttdft_cholqr2 needs for an n_rows x n_vec block. */
size_t ttdft_cholqr2_workspace(int64_t n_rows, int64_t n_vec, ttdft_dtype y_dtype);

/*
 * Step 2 of Algorithm 1 (orthonormalisation of the filtered block), carried
 * out as Cholesky-QR applied twice in FP64 with column scaling:
 *   G = Y^T Y,  D = diag(G)^{1/2},  D^{-1} G D^{-1} = R^T R,  Q = Y D^{-1} R^{-1},
 * then once more on Q.  Q^T Q = I and span(Q) = span(Y).
 * Y: device n_rows x n_vec (F64, F32 or BF16; read in FP64).  Q: device FP64
 * n_rows x n_vec; Q may be Y only when Y is F64 with ldq == ldy, otherwise
 * they must not overlap.  Requires n_rows >= n_vec.  Synchronises the stream
 * (a breakdown must be reported).
 * Errors: NULL, SHAPE, DTYPE, WORKSPACE, ALIAS, NOT_POSDEF (a non-positive
 * pivot: Y numerically rank-deficient in FP64), NONFINITE (Y holds a NaN or
 * Inf), HIP.
 */
ttdft_status ttdft_cholqr2(const void *Y, int64_t ldy, ttdft_dtype y_dtype, int64_t n_rows,
                           int64_t n_vec, double *Q, int64_t ldq, void *work,
                           size_t work_bytes, void *stream);

/* Bytes of workspace ttdft_project needs (H Q, plus split-K partial sums). */
size_t ttdft_project_workspace(const ttdft_bsr *H, int64_t n_vec);

/*
 * Step 3 of Algorithm 1 (subspace projection, Sec. 4.3): A = Q^T (H Q), which
 * is symmetric because H is: the lower-triangular 128 x 128 tiles are formed
 * and mirrored, and inside the diagonal tiles A_ij and A_ji are averaged, so A
 * is written exactly symmetric.  H must be FP64.  Q: device FP64
 * 64*n_block_rows x n_vec (ldq).  A: device FP64 n_vec x n_vec (lda).  ASYNC.
 * Errors: NULL, SHAPE, DTYPE, WORKSPACE, ALIAS, HIP.
 */
ttdft_status ttdft_project(const ttdft_bsr *H, const double *Q, int64_t ldq, int64_t n_vec,
                           double *A, int64_t lda, void *work, size_t work_bytes,
                           void *stream);

/* Bytes of workspace ttdft_syev needs for order n. */
size_t ttdft_syev_workspace(int64_t n);

/*
 * Step 4 of Algorithm 1 (dense eigensolve of the projected matrix):
 * A Z = Z diag(lambda) for a symmetric n x n FP64 matrix A (device, lda; only
 * read), lambda ascending (device [n]), Z orthonormal (device n x n, ldz;
 * column j belongs to lambda[j]).  Householder tridiagonalisation, bisection,
 * inverse iteration, re-orthonormalisation and back-transformation, all on the
 * GPU.  Synchronises the stream.
 * Errors: NULL, SHAPE, WORKSPACE, ALIAS, NO_CONVERGENCE (eigenvector block lost
 * rank), NONFINITE (non-finite entries in A), HIP.
 */
ttdft_status ttdft_syev(int64_t n, const double *A, int64_t lda, double *lambda, double *Z,
                        int64_t ldz, void *work, size_t work_bytes, void *stream);

/*
 * Step 5 of Algorithm 1 (rotation): Psi = X_F Q with X_F device FP64
 * n_rows x n_vec (ldx), Q device FP64 n_vec x n_vec (ldq) and Psi device FP64
 * n_rows x n_vec (ldpsi), Psi overlapping neither input.  ASYNC.
 * Errors: NULL, SHAPE, ALIAS, HIP.
 */
ttdft_status ttdft_rotate(const double *XF, int64_t ldx, int64_t n_rows, int64_t n_vec,
                          const double *Q, int64_t ldq, double *Psi, int64_t ldpsi,
                          void *stream);

/* Bytes of workspace ttdft_rayleigh_ritz needs. */
size_t ttdft_rayleigh_ritz_workspace(const ttdft_bsr *H, int64_t n_vec, ttdft_dtype y_dtype);

/*
 * Steps 2-5 of Algorithm 1 on a filtered block Y (the output of step 1):
 * X_F = Cholesky-QR2(Y); H_F = X_F^T H X_F; H_F Q = Q Lambda; Psi = X_F Q.
 * X_F = Q1 M2 (first pass Q1 = Y M1, second-pass factor M2) is not formed:
 * H_F = M2^T (Q1^T H Q1) M2 and Psi = Q1 (M2 Q), equal up to rounding; after a
 * Cholesky breakdown the shifted Cholesky-QR3 forms X_F explicitly.
 * H must be FP64: the projection stays in FP64 whatever precision the filter
 * used.  Y: device 64*n_block_rows x n_vec of y_dtype.  lambda: device FP64
 * [n_vec], ascending.  Psi: device FP64 64*n_block_rows x n_vec (ldpsi).
 * Synchronises the stream.
 * Errors: NULL, SHAPE, DTYPE, WORKSPACE, ALIAS, NOT_POSDEF, NO_CONVERGENCE,
 * NONFINITE (Y holds a NaN or Inf, or the projected matrix a non-finite
 * value), HIP.
 */
ttdft_status ttdft_rayleigh_ritz(const ttdft_bsr *H, const void *Y, int64_t ldy,
                                 ttdft_dtype y_dtype, int64_t n_vec, double *lambda,
                                 double *Psi, int64_t ldpsi, void *work, size_t work_bytes,
                                 void *stream);

/* ---------------------------------------------------------------- spectrum bound for [a, b] */

/* Bytes of workspace ttdft_lanczos_bounds needs for k steps. */
size_t ttdft_lanczos_workspace(const ttdft_bsr *H, int32_t k);

/*
 * Estimates of both ends of the spectrum of H, for the bounds of the Chebyshev
 * filter (Sec. 3.4 needs an upper bound b of the unwanted spectrum and a
 * scaling point a0 below the wanted one): k steps of the Lanczos process from
 * a seeded random start vector (zero on padding rows), then
 *   bounds[0] = theta_max, the largest eigenvalue of the k x k Lanczos
 *               tridiagonal T_k (a lower estimate of the top of the spectrum),
 *   bounds[1] = theta_max + |beta_{k+1} s_k|, s_k the last component of its
 *               eigenvector (theta_max plus its Ritz residual: the usual estimate),
 *   bounds[2] = theta_max + beta_{k+1} (safeguarded, pessimistic),
 *   bounds[3] = theta_min, the smallest eigenvalue of T_k (an upper estimate of
 *               the bottom of the spectrum).
 * When the process breaks down (some beta_{j+1}, j < k, vanishes relative to
 * the size of T_k: the Krylov space is invariant and its Ritz values need not
 * include the extreme eigenvalues) T is cut at order j + 1 and bounds[1],
 * bounds[2] are raised to at least, and bounds[3] lowered to at most, the
 * Gershgorin bounds max_i (H_ii + r_i) and min_i (H_ii - r_i), r_i = sum over
 * j != i of |H_ij|, which enclose the whole spectrum.  The same widening is
 * applied when k is at least the number of real rows (the Krylov space is then
 * invariant for certain, even where rounding keeps beta from vanishing).
 * H must be FP64.  perm: device int64 [64*n_block_rows] from ttdft_bsr_build
 * (padding rows marked -1).  bounds: host double[4].  Synchronises the stream.
 * Errors: NULL, SHAPE (k outside 1..1000), DTYPE, WORKSPACE, NONFINITE, HIP.
 */
ttdft_status ttdft_lanczos_bounds(const ttdft_bsr *H, const int64_t *perm, int32_t k,
                                  uint64_t seed, double *bounds, void *work, size_t work_bytes,
                                  void *stream);

/* ---------------------------------------------------------------- convergence test */

/* Bytes of workspace ttdft_ritz_residuals needs. */
size_t ttdft_ritz_residuals_workspace(const ttdft_bsr *H, int64_t n_vec);

/*
 * Ritz residual norms res[j] = || H psi_j - lambda_j psi_j ||_2 of the output of
 * steps 2-5 of Algorithm 1 (Sec. 3.4): the subspace iteration is repeated from
 * Psi until they are small enough.  H must be FP64.  Psi: device FP64
 * 64*n_block_rows x n_vec (ldp, blocked row order, zero padding rows);
 * lambda: device FP64 [n_vec]; res: device FP64 [n_vec].  None of them may
 * overlap the workspace or each other (res vs Psi, lambda).  Deterministic
 * (fixed-order reductions).  ASYNC.
 * Errors: NULL, SHAPE, DTYPE, WORKSPACE, ALIAS, HIP.
 */
ttdft_status ttdft_ritz_residuals(const ttdft_bsr *H, const double *Psi, int64_t ldp,
                                  const double *lambda, int64_t n_vec, double *res, void *work,
                                  size_t work_bytes, void *stream);

/* ---------------------------------------------------------------- occupancies and density */

/* Bytes of device workspace ttdft_fermi_level needs (16). */
size_t ttdft_fermi_level_workspace(void);

/*
 * Fermi-Dirac occupancies of the Ritz values (Sec. 2, occupancy and electron
 * count equations): f_i = 1 / (1 + exp((lambda_i - mu) / kT)) with the Fermi
 * energy mu solving 2 sum_i f_i = n_electrons (two electrons per orbital),
 * found by bisection on the increasing count in one work-group (fixed-order
 * sums).  lambda: device FP64 [n]; f: device FP64 [n]; mu: host double.
 * Requires 0 < n_electrons < 2n and 0 < kT < inf (kT in the units of lambda,
 * e.g. Hartree: k_B * 500 K = 1.5834e-3).  Synchronises the stream.
 * Errors: NULL, SHAPE, BOUNDS, WORKSPACE, ALIAS, NONFINITE (a non-finite
 * lambda), HIP.
 */
ttdft_status ttdft_fermi_level(const double *lambda, int64_t n, double n_electrons, double kT,
                               double *f, double *mu, void *work, size_t work_bytes, void *stream);

/*
 * Density matrix of the occupied Ritz vectors on the pattern of H (the
 * electron density of Sec. 2 in a localized basis needs it only where basis
 * functions overlap, which is where H has entries):
 *   P(i, j) of tile t = 2 sum_c f_c Psi[64B + i][c] Psi[64B' + j][c]
 * for every stored tile t = (B, B'), written in the layout of the tile values
 * (fragment order); entries whose mask bit is clear are written as 0 (mask
 * NULL: every tile entry).  H must be FP64 (only its pattern is used).  Psi:
 * device FP64 64*n_block_rows x n_vec (ldp); f: device FP64 [n_vec];
 * P_vals: device FP64 [n_tiles*4096], overlapping none of the inputs.
 * Deterministic.  ASYNC.  Errors: NULL, SHAPE, DTYPE, ALIAS, HIP.
 */
ttdft_status ttdft_density_matrix(const ttdft_bsr *H, const double *Psi, int64_t ldp, const double *f,
                                  int64_t n_vec, double *P_vals, const uint64_t *mask, void *stream);

/*
 * Electron density at the lattice sites (the diagonal of the density matrix):
 * rho[r] = 2 sum_c f_c Psi[r][c]^2 for r < rows.  Psi: device FP64 rows x n_vec
 * (ldp); f: device FP64 [n_vec]; rho: device FP64 [rows], overlapping neither.
 * Deterministic.  ASYNC.  Errors: NULL, SHAPE, ALIAS, HIP.
 */
ttdft_status ttdft_electron_density(const double *Psi, int64_t ldp, const double *f, int64_t rows,
                                    int64_t n_vec, double *rho, void *stream);

/* ---------------------------------------------------------------- adjoint of step 1 */

/*
 * Bytes of workspace ttdft_cheb_filter_backward needs: one block for the
 * reverse sweep plus the stored forward iterates.  ckpt_every = 0 (or 1, 2)
 * stores every iterate Y_1 .. Y_{m-1}; ckpt_every = s >= 3 stores the pairs
 * (Y_{js}, Y_{js+1}) and recomputes the s-2 iterates between them.
 */
size_t ttdft_cheb_filter_backward_workspace(const ttdft_bsr *H, int64_t n_vec, int32_t m,
                                            int32_t ckpt_every, ttdft_dtype x_dtype);

/*
 * Adjoint of ttdft_cheb_filter (step 1 of Algorithm 1, Sec. 3.4) for a loss L
 * with dL/dY = dY.  With Y_0 = X and Y_{k+1} = alpha_k (H - cI) Y_k - beta_k
 * Y_{k-1} the reverse sweep is Ybar_m = dY,
 *   Ybar_k = alpha_k (H - cI) Ybar_{k+1} - beta_{k+1} Ybar_{k+2}  (beta_m = 0),
 * and
 *   dX = Ybar_0  (= p(H) dY, H symmetric),
 *   dH[t](i, j) = sum_k alpha_k <Ybar_{k+1}[row i], Y_k[col j]>  for each stored
 *   entry (i, j) of tile t: the derivative with respect to that entry with all
 *   entries independent (the derivative along a symmetric perturbation of the
 *   pair (i,j), (j,i) is the sum of the two).  Entries whose mask bit is clear
 *   are written as 0.
 * X, dY: device 64*n_block_rows x n_vec of x_dtype (ldx, lddy).  dX: same shape
 * and dtype (lddx), overlapping neither X, dY nor work.  dH_vals: device
 * [n_tiles*4096] in the layout of the tile values of H (the fragment order of
 * H's dtype: 16x4 for F64 / F32 tiles, 16x32 for BF16 tiles), FP64 when
 * x_dtype is F64 and FP32 otherwise.  mask: device
 * [n_tiles*64] from ttdft_bsr_build, or NULL (every tile entry written).  The
 * result does not depend on ckpt_every (bitwise).  ASYNC.
 * Errors: NULL, SHAPE, DTYPE, BOUNDS, DEGREE, ALIAS, WORKSPACE, HIP.
 */
ttdft_status ttdft_cheb_filter_backward(const ttdft_bsr *H, const void *X, int64_t ldx,
                                        const void *dY, int64_t lddy, int64_t n_vec, int32_t m,
                                        double a, double b, double a0, ttdft_dtype x_dtype,
                                        int32_t ckpt_every, void *dX, int64_t lddx,
                                        void *dH_vals, const uint64_t *mask, void *work,
                                        size_t work_bytes, void *stream);

/* ---------------------------------------------------------------- the subspace iteration */

/*
 * Bounds of the next pass of the subspace iteration (Sec. 3.4) from the Ritz
 * values of this one: bounds = {a0', a', b} with a0' the smallest and a' the
 * largest of the n values at lambda (device FP64) and b kept.  Requires
 * a0' < a' < b.  bounds: host double[3].  Synchronises the stream.
 * Errors: NULL, SHAPE (n < 2), BOUNDS (b not finite, or the values do not
 * leave a0' < a' < b), NONFINITE (a non-finite value), HIP.
 */
ttdft_status ttdft_next_bounds(const double *lambda, int64_t n, double b, double *bounds,
                               void *stream);

/* One pass of the subspace iteration, as recorded by ttdft_chfsi_pass / _solve. */
typedef struct {
  int32_t pass;            /* 1-based pass number                                      */
  int32_t m;               /* degree of this attempt                                   */
  int32_t rank_deficient;  /* 1: the filtered block lost rank in FP64 (Cholesky
                              breakdown); the solve repeats the pass at half the degree */
  int32_t reserved;
  double a0, a, b;         /* bounds the filter used                                   */
  double max_residual;     /* largest Ritz residual norm over the lowest n_conv pairs
                              (NaN for a rank-deficient attempt)                        */
  double filter_ms, rr_ms, residual_ms;   /* HIP event times of the three steps       */
} ttdft_chfsi_record;

/* Bytes of workspace ttdft_chfsi_pass needs. */
size_t ttdft_chfsi_pass_workspace(const ttdft_bsr *Hf, const ttdft_bsr *H64, int64_t n_vec,
                                  ttdft_dtype x_dtype);

/*
 * One pass of Algorithm 1 (Sec. 3.4) followed by its convergence test:
 *   Y = ttdft_cheb_filter(Hf, X, m, a, b, a0)   in the precision of Hf / x_dtype,
 *   (lambda, Psi) = ttdft_rayleigh_ritz(H64, Y)  in FP64,
 *   res = ttdft_ritz_residuals(H64, Psi, lambda),
 *   next_bounds = ttdft_next_bounds(lambda, n_vec, b).
 * Hf: the filter's matrix (F64 with x_dtype F64; F32, BF16 or BF16_SPLIT with
 * x_dtype F32); H64: the same blocked matrix in FP64.  bounds: host {a0, a, b}.
 * X: device 64*n_block_rows x n_vec of x_dtype (ldx).  lambda, res: device FP64
 * [n_vec]; Psi: device FP64 64*n_block_rows x n_vec (ldpsi).  record (host, may
 * be NULL) receives m, the bounds, the largest residual over the lowest n_conv
 * pairs and the step times.  next_bounds: host double[3].  Synchronises.
 * Errors: those of the four steps (NOT_POSDEF when the filtered block is
 * rank-deficient in FP64; NONFINITE when it holds a NaN or Inf), NULL, SHAPE,
 * DTYPE, BOUNDS, DEGREE, WORKSPACE.
 */
ttdft_status ttdft_chfsi_pass(const ttdft_bsr *Hf, const ttdft_bsr *H64, const void *X, int64_t ldx,
                              ttdft_dtype x_dtype, int64_t n_vec, int32_t m, const double *bounds,
                              int64_t n_conv, double *lambda, double *Psi, int64_t ldpsi,
                              double *res, ttdft_chfsi_record *record, double *next_bounds,
                              void *work, size_t work_bytes, void *stream);

/* Bytes of workspace ttdft_chfsi_solve needs (lanczos_k = 0 when bounds are given). */
size_t ttdft_chfsi_solve_workspace(const ttdft_bsr *Hf, const ttdft_bsr *H64, int64_t n_vec,
                                   ttdft_dtype x_dtype, int32_t lanczos_k);

/*
 * Algorithm 1 repeated until the Ritz residual norms of the lowest n_conv
 * pairs are at most tol (Sec. 3.4): passes of ttdft_chfsi_pass, each started
 * from the previous pass's Ritz vectors with the bounds it returned.  The
 * first pass uses bounds (host {a0, a, b}) when given, else k = lanczos_k
 * Lanczos steps (ttdft_lanczos_bounds with seed): b = the safeguarded upper
 * bound, a0 = theta_min, a = (theta_min + b) / 2.  The first pass uses degree
 * m_first when m_first > 0, the others m.  An attempt whose filtered block is
 * rank-deficient in FP64 (Cholesky breakdown) is repeated at half the degree
 * (down to 1).  X (device, x_dtype F64 or F32, read only) is the start block;
 * lambda, Psi, res receive the last pass.  history (host, history_cap records,
 * may be NULL when history_cap = 0) receives one record per attempt;
 * *n_records (host) the number of attempts (records beyond history_cap are
 * dropped).  X, Psi and work must not overlap.  Synchronises.
 * Returns TTDFT_OK once converged, TTDFT_ERR_NO_CONVERGENCE after max_passes
 * passes without convergence (outputs hold the last pass), or the error of a step.
 */
ttdft_status ttdft_chfsi_solve(const ttdft_bsr *Hf, const ttdft_bsr *H64, const int64_t *perm,
                               const void *X, int64_t ldx, ttdft_dtype x_dtype, int64_t n_vec,
                               int32_t m, int32_t m_first, double tol, int64_t n_conv,
                               int32_t max_passes, const double *bounds, int32_t lanczos_k,
                               uint64_t seed, double *lambda, double *Psi, int64_t ldpsi,
                               double *res, ttdft_chfsi_record *history, int32_t history_cap,
                               int32_t *n_records, void *work, size_t work_bytes, void *stream);

/* ---------------------------------------------------------------- finiteness check */

/* Bytes of workspace ttdft_check_finite needs (a device counter). */
size_t ttdft_check_finite_workspace(void);

/*
 * Counts the NaN and Inf entries of a rows x cols device block of dtype (F64,
 * F32 or BF16; leading dim ld): *n_nonfinite (host).  Returns
 * TTDFT_ERR_NONFINITE when the count is not zero (for example a filtered block
 * that overflowed), TTDFT_OK otherwise.  Synchronises.
 * Errors: NULL, SHAPE, DTYPE, WORKSPACE, ALIAS, NONFINITE, HIP.
 */
ttdft_status ttdft_check_finite(const void *A, ttdft_dtype dtype, int64_t rows, int64_t cols,
                                int64_t ld, int64_t *n_nonfinite, void *work, size_t work_bytes,
                                void *stream);

/* ---------------------------------------------------------------- diagnostics */

const char *ttdft_status_string(ttdft_status s);
const char *ttdft_last_error(void);
/* Library version string. */
const char *ttdft_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TTDFT_H */
