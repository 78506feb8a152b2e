"""ctypes declarations of the C ABI in include/leja_logdet.h.

Loads ``libleja_logdet.so`` from this package directory and fails loudly if it
is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
import re

from .build import source_hash  # noqa: F401  (hash of the sources the library is built from)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libleja_logdet.so")


def built_source_hash() -> str:
    """The source hash compiled into the loaded library (ld_version)."""
    m = re.search(r"src=([0-9a-f]+|unknown)", load().ld_version().decode())
    return m.group(1) if m else "unknown"

LD_OK = 0
LD_EINVAL = -1
LD_ECSR = -2
LD_EBREAKDOWN = -3
LD_EWORKSPACE = -4
LD_EHIP = -5
LD_EINDEF = -6
LD_ENOMEM = -7

LD_F32 = 0
LD_F64 = 1
LD_SVAL_CENTER = 0
LD_SVAL_HALF_LMAX = 1
LD_DOT_AUTO = 0
LD_DOT_FORWARD = 1
LD_DOT_SQUARED = 2


class LdCsr(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
        ("dtype", ctypes.c_int32),
    ]


class LdOptions(ctypes.Structure):
    _fields_ = [
        ("s_val_mode", ctypes.c_int32),
        ("block_cols", ctypes.c_int32),
        ("taylor_cap", ctypes.c_int64),
        ("ckpt_stride", ctypes.c_int32),
        ("dot_mode", ctypes.c_int32),
        ("trusted_csr", ctypes.c_int32),
        ("csr_only", ctypes.c_int32),
        ("tile_order", ctypes.c_int32),
        ("probe_dist", ctypes.c_int32),
    ]


class LdStats(ctypes.Structure):
    _fields_ = [
        ("ms_total", ctypes.c_double),
        ("ms_phase1", ctypes.c_double),
        ("ms_qr", ctypes.c_double),
        ("ms_phase23", ctypes.c_double),
        ("ms_adjoint", ctypes.c_double),
        ("bytes_alg", ctypes.c_double),
        ("taylor_terms", ctypes.c_int64),
        ("sigma", ctypes.c_double),
        ("lo", ctypes.c_double),
        ("hi", ctypes.c_double),
        ("k", ctypes.c_int32),
        ("k_G", ctypes.c_int32),
        ("dot_mode_used", ctypes.c_int32),
        ("spmm_launches", ctypes.c_int32),
        ("t_low", ctypes.c_double),
        ("t_res", ctypes.c_double),
        ("ms_steps1", ctypes.c_double),
        ("ms_steps23", ctypes.c_double),
        ("launches1", ctypes.c_int32),
        ("launches23", ctypes.c_int32),
        ("bytes1", ctypes.c_double),
        ("bytes23", ctypes.c_double),
        ("dia_diagonals", ctypes.c_int32),
        ("tile_order_used", ctypes.c_int32),
        ("dia_constant", ctypes.c_int32),
        ("xcd_chunk_rows", ctypes.c_int32),
        ("block_cols1", ctypes.c_int32),
        ("block_cols23", ctypes.c_int32),
        ("ranges23", ctypes.c_int32),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes); every symbol the header declares
SIGNATURES = {
    "ld_default_options": (None, [ctypes.POINTER(LdOptions)]),
    "ld_version": (ctypes.c_char_p, []),
    "ld_error_string": (ctypes.c_char_p, [ctypes.c_int]),
    "ld_last_error_detail": (ctypes.c_char_p, []),
    "ld_leja_points": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]),
    "ld_divided_differences": (ctypes.c_int, [ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int64,
                                              ctypes.POINTER(ctypes.c_double),
                                              ctypes.POINTER(ctypes.c_int64)]),
    "ld_rademacher_host": (ctypes.c_int, [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_int64, ctypes.POINTER(ctypes.c_int8)]),
    "ld_squared_basis_coefficients": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                                     ctypes.POINTER(ctypes.c_double)]),
    "ld_workspace_size": (ctypes.c_int, [ctypes.POINTER(LdCsr), ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(LdOptions),
                                         ctypes.POINTER(ctypes.c_size_t)]),
    "ld_apply_log": (ctypes.c_int, [ctypes.POINTER(LdCsr), ctypes.c_double, ctypes.c_double,
                                    ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.POINTER(LdOptions), ctypes.c_void_p, ctypes.c_size_t,
                                    ctypes.c_void_p]),
    "ld_apply_log_adaptive": (ctypes.c_int, [ctypes.POINTER(LdCsr), ctypes.c_double, ctypes.c_double,
                                             ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(LdOptions),
                                             ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                             ctypes.POINTER(ctypes.c_int32)]),
    "ld_adaptive_workspace_size": (ctypes.c_int, [ctypes.POINTER(LdCsr), ctypes.c_int32, ctypes.c_int32,
                                                  ctypes.POINTER(LdOptions), ctypes.POINTER(ctypes.c_size_t)]),
    "ld_logdet_estimate_adaptive": (ctypes.c_int, [ctypes.POINTER(LdCsr), ctypes.c_double, ctypes.c_double,
                                                   ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
                                                   ctypes.c_uint64, ctypes.POINTER(LdOptions), ctypes.c_void_p,
                                                   ctypes.c_size_t, ctypes.c_void_p,
                                                   ctypes.POINTER(ctypes.c_double),
                                                   ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(LdStats)]),
    "ld_logdet_estimate": (ctypes.c_int, [ctypes.POINTER(LdCsr), ctypes.c_double, ctypes.c_double,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                          ctypes.POINTER(LdOptions), ctypes.c_void_p, ctypes.c_size_t,
                                          ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(LdStats)]),
    "ld_logdet_estimate_noalloc": (ctypes.c_int, [ctypes.POINTER(LdCsr), ctypes.c_double, ctypes.c_double,
                                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                                  ctypes.POINTER(LdOptions), ctypes.c_void_p,
                                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(LdStats)]),
    "ld_logdet_grad": (ctypes.c_int, [ctypes.POINTER(LdCsr), ctypes.c_double, ctypes.c_double,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.POINTER(LdOptions), ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                      ctypes.POINTER(LdStats)]),
    "ld_spectral_bounds": (ctypes.c_int, [ctypes.POINTER(LdCsr), ctypes.c_int32, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


class NativeError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        self.code = code
        super().__init__(f"{where}: {name_of(code)} ({detail})")


def name_of(code: int) -> str:
    return load().ld_error_string(code).decode()


def load():
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"native library {LIB_PATH} is missing; build it with "
                "`python -m paper_2603_02207_amd.build` (there is no fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(code: int, where: str):
    if code != LD_OK:
        detail = load().ld_last_error_detail().decode()
        raise NativeError(code, where, detail)
    return code
