"""The filter entry point that allocates nothing (ttdft_cheb_filter_noalloc),
called through the C ABI, against ttdft_cheb_filter with a workspace: two calls
in a row on the same GPU, the second on a smaller problem, each bitwise equal
to the workspace entry point (the same kernels in the same order) and within
the FP64 parity bar (1e-12 normwise) of the oracle."""
import ctypes as C

import numpy as np
import pytest

import oracle
import workload
from gpu_common import A, A0, B, normwise, require_gpu

pytestmark = pytest.mark.gpu


def _run_both(r, h, n, m, dtype_name):
    torch, P = require_gpu()
    from paper_2110_15853_amd import _lib
    lib = _lib.load()
    dt = {"f64": torch.float64, "f32": torch.float32}[dtype_name]
    ip, ix, d, N = workload.lattice_hamiltonian(r, h, 0)
    Hb = P.bsr_build(ip, ix, d, r, dtype=dt, device="cuda")
    X = workload.gaussian_block(N, n, 3)
    Xb = P.to_blocked(torch.from_numpy(X).cuda(), Hb).to(dt)
    print(f"no-alloc filter r={r} h={h} n={n} m={m} {dtype_name}: work block "
          f"{Hb.rows * n * Xb.element_size()} bytes", flush=True)
    hs = Hb.c_struct()
    code = P.DTYPE_CODES[dt]
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    Y_ref = torch.full((Hb.rows, n), float("nan"), dtype=dt, device="cuda")
    need = lib.ttdft_cheb_filter_workspace(C.byref(hs), n, code)
    work = torch.empty(need, dtype=torch.uint8, device="cuda")
    _lib.call("ttdft_cheb_filter", C.byref(hs), C.c_void_p(Xb.data_ptr()), n,
              C.c_void_p(Y_ref.data_ptr()), n, n, m, A, B, A0, code, C.c_void_p(work.data_ptr()),
              need, stream)
    Y = torch.full((Hb.rows, n), float("nan"), dtype=dt, device="cuda")
    _lib.call("ttdft_cheb_filter_noalloc", C.byref(hs), C.c_void_p(Xb.data_ptr()), n,
              C.c_void_p(Y.data_ptr()), n, n, m, A, B, A0, code, stream)
    torch.cuda.synchronize()
    assert torch.equal(Y, Y_ref)
    Yn = P.from_blocked(Y.double(), Hb).cpu().numpy()
    if dtype_name == "f64":
        ref = oracle.cheb_filter(oracle.csr_from_arrays(ip, ix, d, N), X, m, A, B, A0)
        assert normwise(Yn, ref) <= 1e-12
    else:
        # FP32 parity bar: the oracle on the FP32-rounded H and X, 4 m 2^-24
        d32 = d.astype(np.float32).astype(np.float64)
        X32 = X.astype(np.float32).astype(np.float64)
        ref = oracle.cheb_filter(oracle.csr_from_arrays(ip, ix, d32, N), X32, m, A, B, A0)
        assert normwise(Yn, ref) <= 4 * m * 2.0 ** -24
    return Hb.rows * n * Xb.element_size()


def test_noalloc_filter_two_calls_second_smaller():
    first = _run_both(20, 3, 64, 10, "f64")        # 8,000 rows x 64: 4 MiB work block
    second = _run_both(12, 2, 24, 7, "f64")        # 1,728 rows x 24: smaller
    assert second < first


def test_noalloc_filter_fp32_and_at_the_limit():
    # FP32 iterates; then a work block of exactly the 64 MiB limit
    # (lattice 16^3 = 64 block rows = 4096 rows, 2048 FP64 vectors)
    _run_both(16, 2, 40, 5, "f32")
    assert _run_both(16, 1, 2048, 2, "f64") == 64 << 20
