"""ctypes binding of libttdft.so (argument marshalling only).

The library is required: loading fails loudly when it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))

F64, F32, BF16, BF16_SPLIT = 0, 1, 2, 3
STATUS = {0: "TTDFT_OK", 1: "TTDFT_ERR_NULL", 2: "TTDFT_ERR_SHAPE", 3: "TTDFT_ERR_DTYPE",
          4: "TTDFT_ERR_BOUNDS", 5: "TTDFT_ERR_DEGREE", 6: "TTDFT_ERR_ALIAS",
          7: "TTDFT_ERR_WORKSPACE", 8: "TTDFT_ERR_NOT_POSDEF", 9: "TTDFT_ERR_NO_CONVERGENCE",
          10: "TTDFT_ERR_NONFINITE", 11: "TTDFT_ERR_HIP", 12: "TTDFT_ERR_PATTERN"}


class TtdftError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class ChfsiRecord(C.Structure):
    """ttdft_chfsi_record."""
    _fields_ = [("pass_", C.c_int32), ("m", C.c_int32), ("rank_deficient", C.c_int32),
                ("reserved", C.c_int32), ("a0", C.c_double), ("a", C.c_double), ("b", C.c_double),
                ("max_residual", C.c_double), ("filter_ms", C.c_double), ("rr_ms", C.c_double),
                ("residual_ms", C.c_double)]


class Bsr(C.Structure):
    _fields_ = [("n_block_rows", C.c_int64), ("n_tiles", C.c_int64),
                ("tile_rowptr", C.c_void_p), ("tile_col", C.c_void_p),
                ("vals", C.c_void_p), ("dtype", C.c_int), ("frag_mask", C.c_void_p)]


def library_path() -> str:
    return os.path.join(_HERE, "libttdft.so")


_P, _I64, _I32, _D, _SZ, _INT = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_size_t, C.c_int
_BSRP = C.POINTER(Bsr)

# name -> (restype, argtypes); mirrors include/ttdft.h
SIGNATURES = {
    "ttdft_bsr_plan": (_INT, [_I32, _P, _P, _P, _P]),
    "ttdft_bsr_build_size": (_INT, [_I32, _I32, _P, _P, _P]),
    "ttdft_bsr_build": (_INT, [_I32, _P, _P, _P, _INT, _P, _P, _P, _P, _P, _P, _P]),
    "ttdft_cheb_step": (_INT, [_BSRP, _P, _I64, _P, _I64, _P, _I64, _I64, _D, _D, _D, _INT, _P]),
    "ttdft_cheb_filter_workspace": (_SZ, [_BSRP, _I64, _INT]),
    "ttdft_cheb_filter": (_INT, [_BSRP, _P, _I64, _P, _I64, _I64, _I32, _D, _D, _D, _INT, _P,
                                 _SZ, _P]),
    "ttdft_cheb_filter_schedule": (_INT, [_BSRP, _BSRP, _I32, _P, _I64, _P, _I64, _I64, _I32, _D,
                                          _D, _D, _INT, _P, _SZ, _P]),
    "ttdft_cheb_filter_noalloc": (_INT, [_BSRP, _P, _I64, _P, _I64, _I64, _I32, _D, _D, _D, _INT,
                                         _P]),
    "ttdft_cast": (_INT, [_P, _INT, _I64, _P, _INT, _I64, _I64, _I64, _P]),
    "ttdft_gather_rows": (_INT, [_P, _I64, _I64, _P, _I64, _I64, _I64, _P, _INT, _P]),
    "ttdft_cholqr2_workspace": (_SZ, [_I64, _I64, _INT]),
    "ttdft_cholqr2": (_INT, [_P, _I64, _INT, _I64, _I64, _P, _I64, _P, _SZ, _P]),
    "ttdft_project_workspace": (_SZ, [_BSRP, _I64]),
    "ttdft_project": (_INT, [_BSRP, _P, _I64, _I64, _P, _I64, _P, _SZ, _P]),
    "ttdft_syev_workspace": (_SZ, [_I64]),
    "ttdft_syev": (_INT, [_I64, _P, _I64, _P, _P, _I64, _P, _SZ, _P]),
    "ttdft_rotate": (_INT, [_P, _I64, _I64, _I64, _P, _I64, _P, _I64, _P]),
    "ttdft_rayleigh_ritz_workspace": (_SZ, [_BSRP, _I64, _INT]),
    "ttdft_rayleigh_ritz": (_INT, [_BSRP, _P, _I64, _INT, _I64, _P, _P, _I64, _P, _SZ, _P]),
    "ttdft_cheb_filter_backward_workspace": (_SZ, [_BSRP, _I64, _I32, _I32, _INT]),
    "ttdft_cheb_filter_backward": (_INT, [_BSRP, _P, _I64, _P, _I64, _I64, _I32, _D, _D, _D, _INT,
                                          _I32, _P, _I64, _P, _P, _P, _SZ, _P]),
    "ttdft_lanczos_workspace": (_SZ, [_BSRP, _I32]),
    "ttdft_lanczos_bounds": (_INT, [_BSRP, _P, _I32, C.c_uint64, _P, _P, _SZ, _P]),
    "ttdft_ritz_residuals_workspace": (_SZ, [_BSRP, _I64]),
    "ttdft_ritz_residuals": (_INT, [_BSRP, _P, _I64, _P, _I64, _P, _P, _SZ, _P]),
    "ttdft_split_bf16": (_INT, [_P, _I64, _P, _P]),
    "ttdft_convert_tiles": (_INT, [_P, _INT, _I64, _P, _INT, _P]),
    "ttdft_fermi_level_workspace": (_SZ, []),
    "ttdft_fermi_level": (_INT, [_P, _I64, C.c_double, C.c_double, _P, _P, _P, _SZ, _P]),
    "ttdft_density_matrix": (_INT, [_BSRP, _P, _I64, _P, _I64, _P, _P, _P]),
    "ttdft_electron_density": (_INT, [_P, _I64, _P, _I64, _I64, _P, _P]),
    "ttdft_next_bounds": (_INT, [_P, _I64, _D, _P, _P]),
    "ttdft_chfsi_pass_workspace": (_SZ, [_BSRP, _BSRP, _I64, _INT]),
    "ttdft_chfsi_pass": (_INT, [_BSRP, _BSRP, _P, _I64, _INT, _I64, _I32, _P, _I64, _P, _P, _I64,
                                _P, _P, _P, _P, _SZ, _P]),
    "ttdft_chfsi_solve_workspace": (_SZ, [_BSRP, _BSRP, _I64, _INT, _I32]),
    "ttdft_chfsi_solve": (_INT, [_BSRP, _BSRP, _P, _P, _I64, _INT, _I64, _I32, _I32, _D, _I64,
                                 _I32, _P, _I32, C.c_uint64, _P, _P, _I64, _P, _P, _I32, _P, _P,
                                 _SZ, _P]),
    "ttdft_check_finite_workspace": (_SZ, []),
    "ttdft_check_finite": (_INT, [_P, _INT, _I64, _I64, _I64, _P, _P, _SZ, _P]),
    "ttdft_status_string": (C.c_char_p, [_INT]),
    "ttdft_last_error": (C.c_char_p, []),
    "ttdft_version": (C.c_char_p, []),
}

_lib = None


def load():
    """Load libttdft.so once; raises if it has not been built."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} not built: run __graft_entry__.build() "
                              "(python -m paper_2110_15853_amd.build_lib)")
        lib = C.CDLL(path)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def call(name: str, *args):
    """Call an entry point returning ttdft_status; raise TtdftError on failure."""
    lib = load()
    st = getattr(lib, name)(*args)
    if st != 0:
        raise TtdftError(st, lib.ttdft_last_error().decode())
    return st
