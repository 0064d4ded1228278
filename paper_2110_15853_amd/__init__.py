"""MI355X (gfx950) Chebyshev-filtered subspace iteration hot path of the Tucker
tensor DFT method (arXiv 2110.15853): the Chebyshev filter of Algorithm 1
(Sec. 3.4) on a lattice-blocked sparse Hamiltonian, the FP64 Rayleigh-Ritz step
that follows it, and the filter's adjoint.

Every operation runs in the HIP kernels of libttdft.so; this package only
marshals torch tensors (device memory and streams) into the C ABI.
"""
from .api import (  # noqa: F401
    BsrMatrix,
    bsr_build,
    cast,
    cheb_filter,
    cheb_filter_schedule,
    cheb_filter_noalloc,
    NOALLOC_SCRATCH_BYTES,
    cheb_step,
    from_blocked,
    to_blocked,
    DTYPE_CODES,
    ChebFilter,
    bsr_astype,
    chfsi_iteration,
    updated_bounds,
    cheb_filter_autograd,
    cheb_filter_backward,
    cholqr2,
    lanczos_bounds,
    ritz_residuals,
    chfsi_solve,
    chfsi_pass,
    check_finite,
    fermi_level,
    density_matrix,
    electron_density,
    KT_500K_HARTREE,
    gather_rows,
    project,
    rayleigh_ritz,
    rayleigh_ritz_workspace,
    rotate,
    syev,
)
from ._lib import TtdftError, library_path  # noqa: F401
