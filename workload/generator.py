"""Seeded generator of Tucker-lattice Hamiltonians and wavefunction blocks.

Recipe (the paper's Al/Si Hamiltonians are not available; this stands in for
them, with the locality described in Sec. 4.1):

* lattice r x r x r, natural row index I = (i*r + j)*r + k (k fastest);
* diagonal H_II ~ U(-2, 10);
* for every unordered pair I != J whose lattice offset d = J - I satisfies
  max(|di|, |dj|, |dk|) <= h:  H_IJ = H_JI = -0.5 * exp(-0.8*|d|) * (1 + 0.1*z),
  z ~ N(0, 1), |d| the Euclidean lattice distance; one draw per pair, mirrored,
  so H is exactly symmetric;
* X ~ N(0, 1) (N x n, row-major), and W ~ N(0, 1) for the adjoint's loss weights.

Random streams: numpy SeedSequence(seed).spawn(3) gives independent PCG64
streams for (H, X, W).  H draws the N diagonal values first, then, for each
positive offset d in lexicographic order, one normal per valid source row I in
increasing I.  X and W are drawn row-major.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def stream_rngs(seed: int):
    """Return the (H, X, W) generators for one seed."""
    ss = np.random.SeedSequence(seed)
    return tuple(np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3))


def positive_offsets(h: int) -> np.ndarray:
    """Lattice offsets d with max|d_x| <= h whose first nonzero entry is > 0,
    in lexicographic order; shape (P, 3), P = ((2h+1)^3 - 1) / 2."""
    rng = np.arange(-h, h + 1)
    di, dj, dk = np.meshgrid(rng, rng, rng, indexing="ij")
    d = np.stack([di.ravel(), dj.ravel(), dk.ravel()], axis=1)
    first = np.where(d[:, 0] != 0, d[:, 0], np.where(d[:, 1] != 0, d[:, 1], d[:, 2]))
    return d[first > 0]


def lattice_hamiltonian(r: int, h: int, seed: int = 0):
    """Sparse symmetric lattice Hamiltonian in natural order, as CSR.

    Returns (indptr int64[N+1], indices int32[nnz], data float64[nnz], N) with
    column indices ascending inside each row.
    """
    if r < 1 or h < 0:
        raise ValueError("need r >= 1 and h >= 0")
    N = r * r * r
    rng_h, _, _ = stream_rngs(seed)
    S = (2 * h + 1) ** 3
    centre = S // 2

    def slot(d):
        return ((d[0] + h) * (2 * h + 1) + (d[1] + h)) * (2 * h + 1) + (d[2] + h)

    I = np.arange(N, dtype=np.int64)
    ci, cj, ck = I // (r * r), (I // r) % r, I % r

    vals = np.zeros((N, S), dtype=np.float64)
    valid = np.zeros((N, S), dtype=bool)
    vals[:, centre] = rng_h.uniform(-2.0, 10.0, size=N)
    valid[:, centre] = True
    for d in positive_offsets(h):
        ok = ((ci + d[0] >= 0) & (ci + d[0] < r) & (cj + d[1] >= 0) & (cj + d[1] < r)
              & (ck + d[2] >= 0) & (ck + d[2] < r))
        src = np.nonzero(ok)[0]
        if src.size == 0:
            continue
        z = rng_h.standard_normal(src.size)
        dist = float(np.sqrt(float(d[0] * d[0] + d[1] * d[1] + d[2] * d[2])))
        v = -0.5 * np.exp(-0.8 * dist) * (1.0 + 0.1 * z)
        dst = src + (int(d[0]) * r * r + int(d[1]) * r + int(d[2]))
        s_pos, s_neg = slot(d), slot(-d)
        vals[src, s_pos] = v
        valid[src, s_pos] = True
        vals[dst, s_neg] = v
        valid[dst, s_neg] = True

    offs = np.array([[a, b, c] for a in range(-h, h + 1) for b in range(-h, h + 1)
                     for c in range(-h, h + 1)], dtype=np.int64)
    lin = offs[:, 0] * r * r + offs[:, 1] * r + offs[:, 2]
    counts = valid.sum(axis=1)
    indptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    rows, slots = np.nonzero(valid)           # row-major: rows ascending, slots ascending
    indices = (rows + lin[slots]).astype(np.int32)
    data = vals[rows, slots]
    return indptr, indices, data, N


def gaussian_block(N: int, n: int, seed: int = 0, stream: str = "X",
                   dtype=np.float64) -> np.ndarray:
    """N x n block of N(0,1) draws, row-major, from the X or W stream.
    dtype float32 draws single-precision normals directly (a different, equally
    seeded sequence; used where the block is held in FP32)."""
    _, rng_x, rng_w = stream_rngs(seed)
    rng = {"X": rng_x, "W": rng_w}[stream]
    return rng.standard_normal((N, n), dtype=dtype)


def conditioned_block(N: int, n: int, seed: int, cond: float) -> np.ndarray:
    """N x n FP64 block G U diag(s) V^T with G ~ N(0,1) (the X stream of the
    seed), U and V random orthogonal n x n matrices and singular factors s
    log-spaced from 1 down to 1/cond, so the block's condition number is about
    cond (G itself is well conditioned for N >> n).  Stands in for a filtered
    block, whose columns are nearly dependent, as an input independent of any
    filter implementation."""
    G = gaussian_block(N, n, seed)
    rng = np.random.default_rng([seed, 1])
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0.0, -np.log10(cond), n)
    return G @ ((U * s[None, :]) @ V.T)


@dataclass(frozen=True)
class WorkloadConfig:
    """One benchmark / parity workload: lattice, block width, degree, bounds."""
    name: str
    r: int
    h: int
    n: int
    m: int
    a: float = 2.0
    b: float = 12.5
    a0: float = -3.0
    seed: int = 0

    @property
    def N(self) -> int:
        return self.r ** 3


CONFIGS = {
    # small parity case
    "lattice20_h3_n64_m10": WorkloadConfig("lattice20_h3_n64_m10", r=20, h=3, n=64, m=10),
    # full-size FP64 filter followed by Cholesky-QR and Rayleigh-Ritz
    "lattice60_h4_n2048_m20": WorkloadConfig("lattice60_h4_n2048_m20", r=60, h=4, n=2048, m=20),
    # adjoint case
    "lattice40_h3_n512_m16": WorkloadConfig("lattice40_h3_n512_m16", r=40, h=3, n=512, m=16),
    # dense-reference adjoint case (lattice not a multiple of 4)
    "lattice10_h3_n16_m16": WorkloadConfig("lattice10_h3_n16_m16", r=10, h=3, n=16, m=16),
    # large mixed-precision step (X held in FP32)
    "lattice90_h3_n8000_m24": WorkloadConfig("lattice90_h3_n8000_m24", r=90, h=3, n=8000, m=24),
    # reduced version of the large step for quick checks (same lattice stencil and degree)
    "lattice30_h3_n512_m24": WorkloadConfig("lattice30_h3_n512_m24", r=30, h=3, n=512, m=24),
}
