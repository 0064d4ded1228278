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


class RowSlicedCSR:
    """A CSR matrix whose product with a dense block runs as independent row
    slices on a pool of host threads (SciPy's CSR product releases the GIL).
    The product is the same H @ V, only spread over the host's cores, so the
    oracle can take it at the full-size workload in seconds."""

    def __init__(self, H, parts: int = 64, workers: int = None):
        import os
        self.H = H
        self.shape = H.shape
        n = H.shape[0]
        self.bounds = [(n * k // parts, n * (k + 1) // parts) for k in range(parts)]
        self.slices = [H[lo:hi] for lo, hi in self.bounds]
        self.workers = workers or min(16, os.cpu_count() or 1)

    def __matmul__(self, V):
        from concurrent.futures import ThreadPoolExecutor
        V = np.asarray(V)
        out = np.empty((self.shape[0],) + V.shape[1:], dtype=np.result_type(self.H.dtype, V.dtype))

        def run(k):
            lo, hi = self.bounds[k]
            out[lo:hi] = self.slices[k] @ V

        with ThreadPoolExecutor(self.workers) as ex:
            list(ex.map(run, range(len(self.slices))))
        return out
