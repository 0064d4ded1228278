"""Seeded synthetic inputs shared by the FP64 oracle and the GPU path.

This module generates inputs only: it holds none of the arithmetic of the
Chebyshev filter, the orthonormalisation or the Rayleigh-Ritz step.

The Hamiltonian imitates the structure of the projected Kohn-Sham matrix in a
localized 3-D Tucker basis (Sec. 3.3 and Sec. 4.1 of the paper): a composite
lattice index I = (i, j, k) and entries that decay with lattice distance, so the
matrix is sparse, symmetric and dense only near the diagonal.
"""
from .generator import (  # noqa: F401
    CONFIGS,
    WorkloadConfig,
    lattice_hamiltonian,
    gaussian_block,
    conditioned_block,
    positive_offsets,
    stream_rngs,
)
