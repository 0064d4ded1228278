"""Python entry points with the names of the C ABI (include/ttdft.h).

Argument marshalling only: tensors supply device pointers, torch's current
stream supplies the hipStream_t, and every computation runs in libttdft.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from ._lib import BF16, BF16_SPLIT, F32, F64, Bsr

# "bf16x3": tile values as hi + lo bf16 pairs, products hi*hi + hi*lo + lo*hi
DTYPE_CODES = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16, "bf16x3": BF16_SPLIT}
_NP_STORAGE = {F64: np.float64, F32: np.float32, BF16: np.uint16, BF16_SPLIT: np.uint16}
_TILE_VALUES = {F64: 4096, F32: 4096, BF16: 4096, BF16_SPLIT: 8192}   # stored values per tile


def _code(t: torch.Tensor) -> int:
    try:
        return DTYPE_CODES[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported dtype {t.dtype}") from None


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _np_ptr(a):
    return C.c_void_p(a.ctypes.data) if a is not None else C.c_void_p(0)


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("expected a 2-D row-major tensor with unit column stride")
    return t.stride(0)


@dataclass
class BsrMatrix:
    """Lattice-blocked BSR Hamiltonian on the device (see ttdft_bsr)."""
    r: int
    N: int
    n_block_rows: int
    n_tiles: int
    tile_rowptr: torch.Tensor
    tile_col: torch.Tensor
    vals: torch.Tensor          # [n_tiles, 4096] in fragment order (bf16 held as torch.bfloat16)
    perm: torch.Tensor          # blocked row -> natural row or -1 (int64, device)
    inv_perm: torch.Tensor      # natural row -> blocked row (int64, device)
    entry_slot: np.ndarray      # host: flat vals index of each CSR entry
    mask: torch.Tensor          # [n_tiles*64] uint64 stored as int64
    dtype: int
    frag_mask: torch.Tensor = None   # [n_tiles] uint64 stored as int64; None = no skipping
    skip_zero_fragments: bool = True

    @property
    def rows(self) -> int:
        return 64 * self.n_block_rows

    def c_struct(self) -> Bsr:
        fm = self.frag_mask.data_ptr() if (self.frag_mask is not None and self.skip_zero_fragments) else None
        return Bsr(self.n_block_rows, self.n_tiles, self.tile_rowptr.data_ptr(),
                   self.tile_col.data_ptr(), self.vals.data_ptr(), self.dtype, fm)


def bsr_build(indptr, indices, data, r: int, dtype=torch.float64, device="cuda") -> BsrMatrix:
    """ttdft_bsr_plan + ttdft_bsr_build on the host, then copy to the device."""
    indptr = np.ascontiguousarray(indptr, dtype=np.int64)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    data = np.ascontiguousarray(data, dtype=np.float64)
    code = DTYPE_CODES[dtype]
    nbr, nt = C.c_int64(), C.c_int64()
    _lib.call("ttdft_bsr_plan", r, _np_ptr(indptr), _np_ptr(indices), C.byref(nbr), C.byref(nt))
    nbr, nt = nbr.value, nt.value
    tptr = np.empty(nbr + 1, np.int32)
    tcol = np.empty(nt, np.int32)
    vals = np.empty(nt * _TILE_VALUES[code], _NP_STORAGE[code])
    perm = np.empty(nbr * 64, np.int64)
    slot = np.empty(len(data), np.int64)
    mask = np.empty(nt * 64, np.uint64)
    fmask = np.empty(max(nt, 1), np.uint64)
    _lib.call("ttdft_bsr_build", r, _np_ptr(indptr), _np_ptr(indices), _np_ptr(data), code,
              _np_ptr(tptr), _np_ptr(tcol), _np_ptr(vals), _np_ptr(perm), _np_ptr(slot),
              _np_ptr(mask), _np_ptr(fmask))
    N = r ** 3
    inv = np.empty(N, np.int64)
    real = perm >= 0
    inv[perm[real]] = np.nonzero(real)[0]
    tvals = torch.from_numpy(vals.view(np.int16)).view(torch.bfloat16) if code in (BF16, BF16_SPLIT) \
        else torch.from_numpy(vals)
    return BsrMatrix(r=r, N=N, n_block_rows=nbr, n_tiles=nt,
                     tile_rowptr=torch.from_numpy(tptr).to(device),
                     tile_col=torch.from_numpy(tcol).to(device),
                     vals=tvals.reshape(nt, _TILE_VALUES[code]).to(device),
                     perm=torch.from_numpy(perm).to(device),
                     inv_perm=torch.from_numpy(inv).to(device),
                     entry_slot=slot,
                     mask=torch.from_numpy(mask.view(np.int64)).to(device),
                     dtype=code,
                     frag_mask=torch.from_numpy(fmask[:nt].view(np.int64)).to(device))


def gather_rows(src: torch.Tensor, perm: torch.Tensor, rows_dst: int) -> torch.Tensor:
    """ttdft_gather_rows: out[i] = src[perm[i]] (0 where perm[i] < 0)."""
    out = torch.empty((rows_dst, src.shape[1]), dtype=src.dtype, device=src.device)
    _lib.call("ttdft_gather_rows", _ptr(src), _ld(src), src.shape[0], _ptr(out), _ld(out),
              rows_dst, src.shape[1], _ptr(perm), _code(src), _stream())
    return out


def to_blocked(X: torch.Tensor, H: BsrMatrix) -> torch.Tensor:
    """Natural row order (N rows) -> lattice-blocked order (64*n_block_rows rows, zero padding)."""
    if X.shape[0] != H.N:
        raise ValueError("X must have N rows in natural order")
    return gather_rows(X, H.perm, H.rows)


def from_blocked(Y: torch.Tensor, H: BsrMatrix) -> torch.Tensor:
    """Lattice-blocked order -> natural row order (drops padding rows)."""
    if Y.shape[0] != H.rows:
        raise ValueError("Y must have 64*n_block_rows rows")
    return gather_rows(Y, H.inv_perm, H.N)


def cast(src: torch.Tensor, dtype: torch.dtype) -> torch.Tensor:
    """ttdft_cast: precision conversion (round to nearest even)."""
    out = torch.empty(src.shape, dtype=dtype, device=src.device)
    _lib.call("ttdft_cast", _ptr(src), _code(src), _ld(src), _ptr(out), DTYPE_CODES[dtype],
              _ld(out), src.shape[0], src.shape[1], _stream())
    return out


def cheb_step(H: BsrMatrix, Yk: torch.Tensor, Yprev, alpha: float, c: float, beta: float,
              out: torch.Tensor = None) -> torch.Tensor:
    """ttdft_cheb_step: out = alpha*(H Yk - c Yk) - beta*Yprev."""
    if out is None:
        out = torch.empty_like(Yk)
    hs = H.c_struct()
    _lib.call("ttdft_cheb_step", C.byref(hs), _ptr(Yk), _ld(Yk), _ptr(Yprev),
              _ld(Yprev) if Yprev is not None else 0, _ptr(out), _ld(out), Yk.shape[1],
              alpha, c, beta, _code(Yk), _stream())
    return out


def cheb_filter(H: BsrMatrix, X: torch.Tensor, m: int, a: float, b: float, a0: float,
                out: torch.Tensor = None, work: torch.Tensor = None) -> torch.Tensor:
    """ttdft_cheb_filter: Y = T_m((H - cI)/e) X / T_m((a0 - c)/e) on blocked rows."""
    hs = H.c_struct()
    n = X.shape[1]
    code = _code(X)
    need = _lib.load().ttdft_cheb_filter_workspace(C.byref(hs), n, code)
    if out is None:
        out = torch.empty((H.rows, n), dtype=X.dtype, device=X.device)
    if work is None and m >= 2:
        work = torch.empty(need, dtype=torch.uint8, device=X.device)
    _lib.call("ttdft_cheb_filter", C.byref(hs), _ptr(X), _ld(X), _ptr(out), _ld(out), n, m,
              a, b, a0, code, _ptr(work), work.numel() if work is not None else 0, _stream())
    return out


def cheb_filter_schedule(H_early: BsrMatrix, H_late: BsrMatrix, m_late: int, X: torch.Tensor,
                         m: int, a: float, b: float, a0: float, out: torch.Tensor = None,
                         work: torch.Tensor = None) -> torch.Tensor:
    """ttdft_cheb_filter_schedule: the filter with the first m - m_late steps on
    H_early and the last m_late steps on H_late (same pattern, other precision)."""
    he, hl = H_early.c_struct(), H_late.c_struct()
    n = X.shape[1]
    code = _code(X)
    need = _lib.load().ttdft_cheb_filter_workspace(C.byref(he), n, code)
    if out is None:
        out = torch.empty((H_early.rows, n), dtype=X.dtype, device=X.device)
    if work is None and m >= 2:
        work = torch.empty(need, dtype=torch.uint8, device=X.device)
    _lib.call("ttdft_cheb_filter_schedule", C.byref(he), C.byref(hl), m_late, _ptr(X), _ld(X),
              _ptr(out), _ld(out), n, m, a, b, a0, code, _ptr(work),
              work.numel() if work is not None else 0, _stream())
    return out


def cheb_filter_noalloc(H: BsrMatrix, X: torch.Tensor, m: int, a: float, b: float, a0: float,
                        out: torch.Tensor) -> torch.Tensor:
    """ttdft_cheb_filter_noalloc: the filter with the library's fixed device
    scratch as its work block; `out` is caller-provided, nothing is allocated."""
    hs = H.c_struct()
    _lib.call("ttdft_cheb_filter_noalloc", C.byref(hs), _ptr(X), _ld(X), _ptr(out), _ld(out),
              X.shape[1], m, a, b, a0, _code(X), _stream())
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20     # TTDFT_NOALLOC_SCRATCH_BYTES


def _work(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def cholqr2(Y: torch.Tensor, out: torch.Tensor = None) -> torch.Tensor:
    """ttdft_cholqr2: FP64 Cholesky-QR twice (step 2 of Algorithm 1)."""
    rows, n = Y.shape
    if out is None:
        out = torch.empty((rows, n), dtype=torch.float64, device=Y.device)
    need = _lib.load().ttdft_cholqr2_workspace(rows, n, _code(Y))
    w = _work(need, Y.device)
    _lib.call("ttdft_cholqr2", _ptr(Y), _ld(Y), _code(Y), rows, n, _ptr(out), _ld(out), _ptr(w),
              w.numel(), _stream())
    return out


def project(H: BsrMatrix, Q: torch.Tensor) -> torch.Tensor:
    """ttdft_project: Q^T H Q in FP64, exactly symmetric (step 3 of Algorithm 1)."""
    hs = H.c_struct()
    n = Q.shape[1]
    A = torch.empty((n, n), dtype=torch.float64, device=Q.device)
    w = _work(_lib.load().ttdft_project_workspace(C.byref(hs), n), Q.device)
    _lib.call("ttdft_project", C.byref(hs), _ptr(Q), _ld(Q), n, _ptr(A), _ld(A), _ptr(w),
              w.numel(), _stream())
    return A


def syev(A: torch.Tensor):
    """ttdft_syev: eigenvalues (ascending) and eigenvectors of a symmetric FP64 matrix."""
    n = A.shape[0]
    lam = torch.empty(n, dtype=torch.float64, device=A.device)
    Z = torch.empty((n, n), dtype=torch.float64, device=A.device)
    w = _work(_lib.load().ttdft_syev_workspace(n), A.device)
    _lib.call("ttdft_syev", n, _ptr(A), _ld(A), _ptr(lam), _ptr(Z), _ld(Z), _ptr(w), w.numel(),
              _stream())
    return lam, Z


def rotate(XF: torch.Tensor, Q: torch.Tensor) -> torch.Tensor:
    """ttdft_rotate: Psi = X_F Q (step 5 of Algorithm 1)."""
    rows, n = XF.shape
    Psi = torch.empty((rows, n), dtype=torch.float64, device=XF.device)
    _lib.call("ttdft_rotate", _ptr(XF), _ld(XF), rows, n, _ptr(Q), _ld(Q), _ptr(Psi), _ld(Psi),
              _stream())
    return Psi


def rayleigh_ritz(H: BsrMatrix, Y: torch.Tensor, work: torch.Tensor = None):
    """ttdft_rayleigh_ritz: steps 2-5 of Algorithm 1; returns (lambda, Psi)."""
    hs = H.c_struct()
    n = Y.shape[1]
    lam = torch.empty(n, dtype=torch.float64, device=Y.device)
    Psi = torch.empty((H.rows, n), dtype=torch.float64, device=Y.device)
    need = _lib.load().ttdft_rayleigh_ritz_workspace(C.byref(hs), n, _code(Y))
    if work is None or work.numel() < need:
        work = _work(need, Y.device)
    _lib.call("ttdft_rayleigh_ritz", C.byref(hs), _ptr(Y), _ld(Y), _code(Y), n, _ptr(lam),
              _ptr(Psi), _ld(Psi), _ptr(work), work.numel(), _stream())
    return lam, Psi


def rayleigh_ritz_workspace(H: BsrMatrix, n: int, dtype=torch.float64) -> int:
    hs = H.c_struct()
    return int(_lib.load().ttdft_rayleigh_ritz_workspace(C.byref(hs), n, DTYPE_CODES[dtype]))


def cheb_filter_backward(H: BsrMatrix, X: torch.Tensor, dY: torch.Tensor, m: int, a: float,
                         b: float, a0: float, ckpt_every: int = 0, use_mask: bool = True):
    """ttdft_cheb_filter_backward: returns (dX, dH_vals) for dL/dY = dY."""
    hs = H.c_struct()
    n = X.shape[1]
    code = _code(X)
    dX = torch.empty_like(X)
    dH = torch.empty((H.n_tiles, 4096), dtype=torch.float64 if code == F64 else torch.float32,
                     device=X.device)
    need = _lib.load().ttdft_cheb_filter_backward_workspace(C.byref(hs), n, m, ckpt_every, code)
    w = _work(need, X.device)
    _lib.call("ttdft_cheb_filter_backward", C.byref(hs), _ptr(X), _ld(X), _ptr(dY), _ld(dY), n, m,
              a, b, a0, code, ckpt_every, _ptr(dX), _ld(dX), _ptr(dH),
              _ptr(H.mask) if use_mask else C.c_void_p(0), _ptr(w), w.numel(), _stream())
    return dX, dH


class ChebFilter(torch.autograd.Function):
    """Differentiable Chebyshev filter: forward ttdft_cheb_filter, backward
    ttdft_cheb_filter_backward.  Inputs (vals, X) are differentiable; vals must
    be the tensor held by H (its tile layout)."""

    @staticmethod
    def forward(ctx, vals, X, H, m, a, b, a0, ckpt_every):
        if vals.data_ptr() != H.vals.data_ptr():
            raise ValueError("vals must be H.vals")
        ctx.H, ctx.m, ctx.a, ctx.b, ctx.a0, ctx.ckpt = H, m, a, b, a0, ckpt_every
        ctx.save_for_backward(X)
        return cheb_filter(H, X, m, a, b, a0)

    @staticmethod
    def backward(ctx, dY):
        (X,) = ctx.saved_tensors
        dX, dH = cheb_filter_backward(ctx.H, X, dY.contiguous(), ctx.m, ctx.a, ctx.b, ctx.a0,
                                      ctx.ckpt)
        return dH.to(ctx.H.vals.dtype), dX, None, None, None, None, None, None


def cheb_filter_autograd(H: BsrMatrix, X: torch.Tensor, m: int, a: float, b: float, a0: float,
                         ckpt_every: int = 0) -> torch.Tensor:
    """Chebyshev filter that records the adjoint for torch.autograd."""
    return ChebFilter.apply(H.vals, X, H, m, a, b, a0, ckpt_every)


def _slots_16x32(slot16x4: np.ndarray, per_tile: int) -> np.ndarray:
    """Positions of entries given in the 16x4 fragment order of FP64/FP32 tiles,
    in the 16x32 fragment order of BF16 tiles (per_tile values per stored tile;
    the layouts are documented with ttdft_bsr.vals)."""
    t, p = np.divmod(np.asarray(slot16x4, dtype=np.int64), 4096)
    f, q = np.divmod(p, 64)
    i = 16 * (f & 3) + (q & 15)
    j = 4 * (f >> 2) + (q >> 4)
    pos = 512 * (4 * (j >> 5) + (i >> 4)) + 8 * ((i & 15) + 16 * ((j & 31) >> 3)) + (j & 7)
    return t * per_tile + pos


def bsr_astype(H: BsrMatrix, dtype) -> BsrMatrix:
    """The same blocked matrix with its tile values converted on the device by
    ttdft_convert_tiles (round to nearest even; BF16 and bf16x3 tiles in their
    16x32 fragment order); pattern arrays are shared."""
    code = DTYPE_CODES[dtype]
    if code == H.dtype:
        return H
    if H.dtype not in (F64, F32):
        raise ValueError("tile values are converted from FP64 or FP32 tiles")
    slot = H.entry_slot
    if code == BF16_SPLIT:
        vals = torch.empty((H.n_tiles, 8192), dtype=torch.bfloat16, device=H.vals.device)
        slot = _slots_16x32(slot, 8192)                     # position of the hi value
    elif code == BF16:
        vals = torch.empty((H.n_tiles, 4096), dtype=torch.bfloat16, device=H.vals.device)
        slot = _slots_16x32(slot, 4096)
    elif code == F32:
        vals = torch.empty((H.n_tiles, 4096), dtype=torch.float32, device=H.vals.device)
    else:
        raise ValueError("tile values convert to FP32, BF16 or bf16x3")
    _lib.call("ttdft_convert_tiles", _ptr(H.vals), H.dtype, H.n_tiles, _ptr(vals), code, _stream())
    return BsrMatrix(r=H.r, N=H.N, n_block_rows=H.n_block_rows, n_tiles=H.n_tiles,
                     tile_rowptr=H.tile_rowptr, tile_col=H.tile_col, vals=vals, perm=H.perm,
                     inv_perm=H.inv_perm, entry_slot=slot, mask=H.mask, dtype=code,
                     frag_mask=H.frag_mask, skip_zero_fragments=H.skip_zero_fragments)


def chfsi_iteration(Hf: BsrMatrix, H64: BsrMatrix, X: torch.Tensor, m: int, a: float, b: float,
                    a0: float, rr_work: torch.Tensor = None):
    """One pass of Algorithm 1: the filter with Hf (any supported precision) on
    X, then FP64 Rayleigh-Ritz with H64.  Returns (lambda, Psi, filtered Y)."""
    Y = cheb_filter(Hf, X, m, a, b, a0)
    lam, Psi = rayleigh_ritz(H64, Y, work=rr_work)
    return lam, Psi, Y


def updated_bounds(lam: torch.Tensor, b: float):
    """ttdft_next_bounds: the scaling point a0 and the cut a of the next pass
    (the smallest and largest Ritz value of this one; b is kept).  Returns (a0, a)."""
    out = (C.c_double * 3)()
    _lib.call("ttdft_next_bounds", _ptr(lam), lam.numel(), float(b), out, _stream())
    return float(out[0]), float(out[1])


def lanczos_bounds(H: BsrMatrix, k: int = 20, seed: int = 0):
    """ttdft_lanczos_bounds: (theta_max, theta_max + Ritz residual,
    theta_max + beta_{k+1}, theta_min) for an FP64 H."""
    hs = H.c_struct()
    out = (C.c_double * 4)()
    w = _work(_lib.load().ttdft_lanczos_workspace(C.byref(hs), k), H.vals.device)
    _lib.call("ttdft_lanczos_bounds", C.byref(hs), _ptr(H.perm), k, seed, out, _ptr(w),
              w.numel(), _stream())
    return float(out[0]), float(out[1]), float(out[2]), float(out[3])


def ritz_residuals(H: BsrMatrix, Psi: torch.Tensor, lam: torch.Tensor,
                   work: torch.Tensor = None) -> torch.Tensor:
    """ttdft_ritz_residuals: || H psi_j - lambda_j psi_j ||_2 for every column (FP64)."""
    hs = H.c_struct()
    n = Psi.shape[1]
    if Psi.dtype != torch.float64 or lam.dtype != torch.float64:
        raise TypeError("Psi and lambda must be float64")
    res = torch.empty(n, dtype=torch.float64, device=Psi.device)
    if work is None:
        work = _work(_lib.load().ttdft_ritz_residuals_workspace(C.byref(hs), n), Psi.device)
    _lib.call("ttdft_ritz_residuals", C.byref(hs), _ptr(Psi), _ld(Psi), _ptr(lam), n, _ptr(res),
              _ptr(work), work.numel(), _stream())
    return res


def _record_dict(r) -> dict:
    rec = {"pass": r.pass_, "m": r.m, "a0": r.a0, "a": r.a, "b": r.b}
    if r.rank_deficient:
        rec.update(max_residual=None, rank_deficient=True)
    else:
        rec.update(max_residual=r.max_residual, filter_ms=r.filter_ms, rr_ms=r.rr_ms,
                   residual_ms=r.residual_ms)
    return rec


def _x_code(Hf: BsrMatrix) -> int:
    return F64 if Hf.dtype == F64 else F32


def chfsi_pass(Hf: BsrMatrix, H64: BsrMatrix, X: torch.Tensor, m: int, bounds, n_conv: int = None,
               work: torch.Tensor = None):
    """ttdft_chfsi_pass: one pass of Algorithm 1 (filter with Hf, FP64
    Rayleigh-Ritz with H64) and its Ritz residuals.  bounds = (a0, a, b).
    Returns (lambda, Psi, residuals, record dict, next bounds (a0, a, b))."""
    n = X.shape[1]
    n_conv = n if n_conv is None else n_conv
    hf, h64 = Hf.c_struct(), H64.c_struct()
    code = _code(X)
    need = _lib.load().ttdft_chfsi_pass_workspace(C.byref(hf), C.byref(h64), n, code)
    if work is None or work.numel() < need:
        work = _work(need, X.device)
    lam = torch.empty(n, dtype=torch.float64, device=X.device)
    Psi = torch.empty((H64.rows, n), dtype=torch.float64, device=X.device)
    res = torch.empty(n, dtype=torch.float64, device=X.device)
    rec = _lib.ChfsiRecord()
    nxt = (C.c_double * 3)()
    b_in = (C.c_double * 3)(*[float(v) for v in bounds])
    _lib.call("ttdft_chfsi_pass", C.byref(hf), C.byref(h64), _ptr(X), _ld(X), code, n, m, b_in,
              n_conv, _ptr(lam), _ptr(Psi), _ld(Psi), _ptr(res), C.byref(rec), nxt, _ptr(work),
              work.numel(), _stream())
    return lam, Psi, res, _record_dict(rec), (float(nxt[0]), float(nxt[1]), float(nxt[2]))


def chfsi_solve(Hf: BsrMatrix, H64: BsrMatrix, X0: torch.Tensor, m: int, tol: float,
                n_conv: int = None, max_iter: int = 20, m_first: int = None, bounds=None,
                lanczos_k: int = 30, seed: int = 0, history_cap: int = 256):
    """ttdft_chfsi_solve: Algorithm 1 repeated until the Ritz residual norms of
    the lowest n_conv pairs are at most tol (Sec. 3.4), the whole loop in the
    library.  The filter runs with Hf in its precision (FP64 iterates for an
    FP64 Hf, FP32 otherwise; X0 is cast once), the Rayleigh-Ritz step with the
    FP64 H64.  bounds = (a0, a, b) for the first pass, else Lanczos estimates
    (lanczos_k steps, seed).  Returns (lambda, Psi, residuals, history) with one
    history dict per attempt (pass, m, a0, a, b, max_residual and the step
    times; rank-deficient attempts marked).  Without convergence in max_iter
    passes (TTDFT_ERR_NO_CONVERGENCE) the last pass is returned; the history's
    last max_residual shows it.  Other errors raise TtdftError."""
    n = X0.shape[1]
    n_conv = n if n_conv is None else n_conv
    xcode = _x_code(Hf)
    xdt = torch.float64 if xcode == F64 else torch.float32
    X = X0 if X0.dtype == xdt else cast(X0, xdt)
    hf, h64 = Hf.c_struct(), H64.c_struct()
    k = 0 if bounds is not None else lanczos_k
    need = _lib.load().ttdft_chfsi_solve_workspace(C.byref(hf), C.byref(h64), n, xcode, k)
    work = _work(need, X.device)
    lam = torch.empty(n, dtype=torch.float64, device=X.device)
    Psi = torch.empty((H64.rows, n), dtype=torch.float64, device=X.device)
    res = torch.empty(n, dtype=torch.float64, device=X.device)
    hist = (_lib.ChfsiRecord * history_cap)()
    n_rec = C.c_int32(0)
    b_in = (C.c_double * 3)(*[float(v) for v in bounds]) if bounds is not None else None
    lib = _lib.load()
    st = lib.ttdft_chfsi_solve(C.byref(hf), C.byref(h64), _ptr(H64.perm), _ptr(X), _ld(X), xcode, n,
                               m, m_first or 0, float(tol), n_conv, max_iter, b_in, lanczos_k, seed,
                               _ptr(lam), _ptr(Psi), _ld(Psi), _ptr(res), hist, history_cap,
                               C.byref(n_rec), _ptr(work), work.numel(), _stream())
    if st not in (0, 9):            # 9: TTDFT_ERR_NO_CONVERGENCE, outputs hold the last pass
        raise _lib.TtdftError(st, lib.ttdft_last_error().decode())
    history = [_record_dict(hist[i]) for i in range(min(n_rec.value, history_cap))]
    return lam, Psi, res, history


def check_finite(A: torch.Tensor) -> int:
    """ttdft_check_finite: the number of NaN / Inf entries of a 2-D block
    (0 when all are finite)."""
    cnt = C.c_int64(0)
    w = _work(_lib.load().ttdft_check_finite_workspace(), A.device)
    st = _lib.load().ttdft_check_finite(_ptr(A), _code(A), A.shape[0], A.shape[1], _ld(A),
                                        C.byref(cnt), _ptr(w), w.numel(), _stream())
    if st not in (0, 10):
        raise _lib.TtdftError(st, _lib.load().ttdft_last_error().decode())
    return int(cnt.value)


KT_500K_HARTREE = 500.0 * 3.166811563e-6   # k_B T at the paper's smearing temperature, in Hartree


def fermi_level(lam: torch.Tensor, n_electrons: float, kT: float = KT_500K_HARTREE):
    """ttdft_fermi_level: Fermi-Dirac occupancies f and the Fermi energy mu with
    2 sum f = n_electrons.  Returns (f, mu)."""
    if lam.dtype != torch.float64:
        raise TypeError("lambda must be float64")
    f = torch.empty_like(lam)
    mu = C.c_double()
    w = _work(_lib.load().ttdft_fermi_level_workspace(), lam.device)
    _lib.call("ttdft_fermi_level", _ptr(lam), lam.numel(), float(n_electrons), float(kT), _ptr(f),
              C.byref(mu), _ptr(w), w.numel(), _stream())
    return f, mu.value


def density_matrix(H: BsrMatrix, Psi: torch.Tensor, f: torch.Tensor, use_mask: bool = True) -> torch.Tensor:
    """ttdft_density_matrix: 2 sum_c f_c psi_ic psi_jc on the stored tiles of H,
    [n_tiles, 4096] in the layout of the tile values (entry slot of a CSR entry:
    H.entry_slot)."""
    hs = H.c_struct()
    n = Psi.shape[1]
    P_vals = torch.empty((H.n_tiles, 4096), dtype=torch.float64, device=Psi.device)
    _lib.call("ttdft_density_matrix", C.byref(hs), _ptr(Psi), _ld(Psi), _ptr(f), n, _ptr(P_vals),
              _ptr(H.mask) if use_mask else C.c_void_p(0), _stream())
    return P_vals


def electron_density(Psi: torch.Tensor, f: torch.Tensor) -> torch.Tensor:
    """ttdft_electron_density: rho_r = 2 sum_c f_c psi_rc^2 for every row of Psi
    (blocked order for a blocked Psi)."""
    rho = torch.empty(Psi.shape[0], dtype=torch.float64, device=Psi.device)
    _lib.call("ttdft_electron_density", _ptr(Psi), _ld(Psi), _ptr(f), Psi.shape[0], Psi.shape[1],
              _ptr(rho), _stream())
    return rho
