"""ctypes binding of the C/OpenMP oracle filter (oracle/cheb_filter.c).

TEST INFRASTRUCTURE ONLY: the tests and the CPU-baseline leg of the benchmark
call it; the GPU library never does.  `build()` compiles oracle/_cheb_filter.so
with gcc (OpenMP); `cheb_filter_c` builds it on first use when it is missing.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cheb_filter.c")
LIB = os.path.join(HERE, "_cheb_filter.so")
_lib = None


def build():
    tmp = LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, SRC], check=True)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        lib = C.CDLL(LIB)
        f = lib.oracle_cheb_filter_csr
        f.restype = C.c_int
        f.argtypes = [C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                      C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.c_double, C.c_double,
                      C.c_double, C.c_int, C.c_int]
        _lib = lib
    return _lib


def cheb_filter_c(H, X, m: int, a: float, b: float, a0: float, threads: int = 0, blk: int = 8):
    """Y = T_m((H - cI)/e) X / T_m(tau) (Sec. 3.4) by the C oracle; H a SciPy CSR
    matrix (FP64), X an n_rows x n_vec array.  threads = 0 keeps OpenMP's default."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[0] != H.shape[0]:
        raise ValueError("X must be n_rows x n_vec")
    ip = np.ascontiguousarray(H.indptr, dtype=np.int64)
    ix = np.ascontiguousarray(H.indices, dtype=np.int32)
    d = np.ascontiguousarray(H.data, dtype=np.float64)
    Y = np.empty_like(X)
    st = _load().oracle_cheb_filter_csr(X.shape[0], ip.ctypes.data, ix.ctypes.data, d.ctypes.data,
                                        X.ctypes.data, X.shape[1], Y.ctypes.data, Y.shape[1],
                                        X.shape[1], m, a, b, a0, blk, threads)
    if st != 0:
        raise ValueError(f"oracle_cheb_filter_csr failed ({st})")
    return Y
