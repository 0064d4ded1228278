"""FP64 CPU oracle for the Chebyshev-filtered subspace iteration hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this package.  It shares no code with the GPU
library and the GPU library never calls it.

Everything here is plain, slow and FP64 (NumPy / SciPy on the CPU, and the
filter once more in plain C with OpenMP, cheb_filter.c, for the CPU baseline).  Where the
method reaches a result that has a plain definition (the filter is a fixed
polynomial of H applied to X; the Ritz pairs of H on a subspace), the oracle
computes that definition; where it does not (Cholesky-QR as an algorithm), the
oracle follows the steps in the paper's order.
"""
from .chfsi import (  # noqa: F401
    filter_parameters,
    chebyshev_T,
    sigma_sequence,
    cheb_filter,
    cheb_filter_scaled,
    cheb_filter_schedule,
    cheb_filter_adjoint,
    orth,
    cholqr2,
    rayleigh_ritz,
    dense_eigh,
    csr_from_arrays,
    ritz_residuals,
    chfsi,
    fermi_occupancies,
    density_matrix_on_pattern,
    electron_density,
)
from .cfilter import cheb_filter_c  # noqa: F401  (C/OpenMP form of cheb_filter)
