"""Helpers shared by the GPU tests: build a seeded workload on the device and
run the oracle on the same inputs."""
import numpy as np
import pytest

import oracle
import workload

A, B, A0 = 2.0, 12.5, -3.0


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2110_15853_amd as P
    P._lib.load()          # fail loudly when the library is missing
    return torch, P


def make_case(r, h, n, seed=0, dtype=None):
    torch, P = require_gpu()
    dtype = dtype or torch.float64
    ip, ix, d, N = workload.lattice_hamiltonian(r, h, seed)
    Hc = oracle.csr_from_arrays(ip, ix, d, N)
    Hb = P.bsr_build(ip, ix, d, r, dtype=dtype, device="cuda")
    X = workload.gaussian_block(N, n, seed)
    return Hc, Hb, X


def normwise(Y, ref):
    return float(np.linalg.norm(Y - ref) / np.linalg.norm(ref))
