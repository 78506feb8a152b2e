"""Léja + Hutch++ log-determinant estimation on one AMD MI355X (gfx950).

Python binding of the native library (include/leja_logdet.h): argument
marshalling only.  Every step of the estimator runs in the library's HIP
kernels or its host C++ code; PyTorch supplies device memory and the stream.

Main entry points
-----------------
CSR.from_arrays(row_ptr, col_idx, val, n, device)   matrix on the GPU
logdet(A, lmin, lmax, degree, n_matvec, seed)       Alg. 3 estimate of log det A
logdet_noalloc(A, lmin, lmax, degree, n_matvec, seed) the same estimate from the library's
                                                    static scratch (no device allocation)
logdet_with_grad(...)                               estimate and d/d(values)
LogdetFunction / logdet_autograd(values, ...)       torch.autograd wrapper
apply_log(A, lmin, lmax, degree, V)                 P_m(Q~)V + log(sigma)V ~ log(A)V
spectral_bounds(A)                                  Gershgorin interval
leja_points, divided_differences, ...               host-side pieces (no GPU)
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import _native as nat
from ._native import (LD_DOT_AUTO, LD_DOT_FORWARD, LD_DOT_SQUARED, LD_F32, LD_F64,  # noqa: F401
                      LD_SVAL_CENTER, LD_SVAL_HALF_LMAX, NativeError)

__all__ = [
    "CSR", "Options", "logdet", "logdet_adaptive", "logdet_noalloc", "logdet_with_grad", "logdet_autograd",
    "LogdetFunction", "apply_log_adaptive",
    "apply_log", "spectral_bounds", "leja_points", "divided_differences", "rademacher_host",
    "squared_basis_coefficients", "workspace_size", "NativeError", "library_path",
]


def library_path() -> str:
    return nat.LIB_PATH


def _torch():
    import torch

    return torch


@dataclass
class Options:
    s_val_mode: int = LD_SVAL_CENTER
    block_cols: int = 0
    taylor_cap: int = 0
    ckpt_stride: int = 0
    dot_mode: int = LD_DOT_AUTO
    trusted_csr: int = 0
    csr_only: int = 0
    tile_order: int = 0
    probe_dist: int = 0     # 0: Rademacher, 1: Gaussian

    def to_c(self) -> nat.LdOptions:
        o = nat.LdOptions()
        nat.load().ld_default_options(ctypes.byref(o))
        o.s_val_mode = self.s_val_mode
        o.block_cols = self.block_cols
        o.taylor_cap = self.taylor_cap
        o.ckpt_stride = self.ckpt_stride
        o.dot_mode = self.dot_mode
        o.trusted_csr = self.trusted_csr
        o.csr_only = self.csr_only
        o.tile_order = self.tile_order
        o.probe_dist = self.probe_dist
        return o


class CSR:
    """A CSR matrix resident on the GPU (int32 indices, float32 or float64 values)."""

    def __init__(self, row_ptr, col_idx, val, n: int):
        torch = _torch()
        if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32:
            raise TypeError("row_ptr and col_idx must be int32")
        if val.dtype not in (torch.float32, torch.float64):
            raise TypeError("values must be float32 or float64")
        if not (row_ptr.is_cuda and col_idx.is_cuda and val.is_cuda):
            raise TypeError("CSR arrays must live on the GPU")
        self.row_ptr = row_ptr.contiguous()
        self.col_idx = col_idx.contiguous()
        self.val = val.contiguous()
        self.n = int(n)

    @classmethod
    def from_arrays(cls, row_ptr, col_idx, val, n: int, device="cuda", dtype=None):
        torch = _torch()
        dtype = dtype or torch.float32
        return cls(torch.as_tensor(np.asarray(row_ptr, dtype=np.int32), device=device),
                   torch.as_tensor(np.asarray(col_idx, dtype=np.int32), device=device),
                   torch.as_tensor(np.asarray(val), device=device).to(dtype), n)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    @property
    def dtype(self):
        return self.val.dtype

    def with_values(self, val) -> "CSR":
        return CSR(self.row_ptr, self.col_idx, val, self.n)

    def c_struct(self, val=None) -> nat.LdCsr:
        torch = _torch()
        v = self.val if val is None else val
        s = nat.LdCsr()
        s.n = self.n
        s.nnz = self.nnz
        s.row_ptr = self.row_ptr.data_ptr()
        s.col_idx = self.col_idx.data_ptr() if self.nnz else None
        s.val = v.data_ptr() if self.nnz else None
        s.dtype = LD_F64 if v.dtype == torch.float64 else LD_F32
        return s


def _stream_handle(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _opts(options) -> nat.LdOptions:
    return (options or Options()).to_c()


def workspace_size(A: CSR, degree: int, n_matvec: int, want_grad: bool = False, options=None) -> int:
    lib = nat.load()
    c = A.c_struct()
    o = _opts(options)
    b = ctypes.c_size_t(0)
    nat.check(lib.ld_workspace_size(ctypes.byref(c), degree, n_matvec, int(want_grad),
                                    ctypes.byref(o), ctypes.byref(b)), "ld_workspace_size")
    return int(b.value)


def _workspace(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)


def logdet(A: CSR, lmin: float, lmax: float, degree: int, n_matvec: int, seed: int = 0,
           options=None, return_stats: bool = False, workspace=None):
    """Léja + Hutch++ estimate of log det A (Alg. 3); a Python float."""
    lib = nat.load()
    c = A.c_struct()
    o = _opts(options)
    need = workspace_size(A, degree, n_matvec, False, options)
    ws = workspace if workspace is not None and workspace.numel() >= need else _workspace(need, A.val.device)
    out = ctypes.c_double(0.0)
    st = nat.LdStats()
    nat.check(lib.ld_logdet_estimate(ctypes.byref(c), float(lmin), float(lmax), int(degree),
                                     int(n_matvec), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                     ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                     _stream_handle(A.val.device), ctypes.byref(out),
                                     ctypes.byref(st)), "ld_logdet_estimate")
    if return_stats:
        return out.value, st.as_dict()
    return out.value


def logdet_adaptive(A: CSR, lmin: float, lmax: float, max_degree: int, tol: float, n_matvec: int,
                    seed: int = 0, options=None, return_stats: bool = False):
    """Alg. 3 with Alg. 2's stopping rule in each application of log: (estimate,
    degrees), degrees = the degree each column stopped at, for the columns of
    S, Q_b and U in that order (n_matvec entries)."""
    lib = nat.load()
    c = A.c_struct()
    o = _opts(options)
    b = ctypes.c_size_t(0)
    nat.check(lib.ld_adaptive_workspace_size(ctypes.byref(c), int(max_degree), int(n_matvec), ctypes.byref(o),
                                             ctypes.byref(b)), "ld_adaptive_workspace_size")
    ws = _workspace(int(b.value), A.val.device)
    out = ctypes.c_double(0.0)
    st = nat.LdStats()
    degrees = np.zeros(int(n_matvec), dtype=np.int32)
    nat.check(lib.ld_logdet_estimate_adaptive(
        ctypes.byref(c), float(lmin), float(lmax), int(max_degree), float(tol), int(n_matvec),
        ctypes.c_uint64(int(seed) & (2**64 - 1)), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
        _stream_handle(A.val.device), ctypes.byref(out), degrees.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        ctypes.byref(st)), "ld_logdet_estimate_adaptive")
    if return_stats:
        return out.value, degrees, st.as_dict()
    return out.value, degrees


def logdet_noalloc(A: CSR, lmin: float, lmax: float, degree: int, n_matvec: int, seed: int = 0,
                   options=None, return_stats: bool = False):
    """As ``logdet``, from the library's static scratch: no device memory is
    allocated (the estimate's workspace must fit the 64 MiB scratch)."""
    torch = _torch()
    lib = nat.load()
    c = A.c_struct()
    o = _opts(options)
    out = ctypes.c_double(0.0)
    st = nat.LdStats()
    with torch.cuda.device(A.val.device):
        nat.check(lib.ld_logdet_estimate_noalloc(ctypes.byref(c), float(lmin), float(lmax), int(degree),
                                                 int(n_matvec), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                                 ctypes.byref(o), _stream_handle(A.val.device),
                                                 ctypes.byref(out), ctypes.byref(st)),
                  "ld_logdet_estimate_noalloc")
    if return_stats:
        return out.value, st.as_dict()
    return out.value


def logdet_with_grad(A: CSR, lmin: float, lmax: float, degree: int, n_matvec: int, seed: int = 0,
                     options=None, return_stats: bool = False):
    """(estimate, d estimate / d A.val) with probes and interval held fixed."""
    torch = _torch()
    lib = nat.load()
    c = A.c_struct()
    o = _opts(options)
    need = workspace_size(A, degree, n_matvec, True, options)
    ws = _workspace(need, A.val.device)
    grad = torch.empty_like(A.val)
    out = ctypes.c_double(0.0)
    st = nat.LdStats()
    nat.check(lib.ld_logdet_grad(ctypes.byref(c), float(lmin), float(lmax), int(degree),
                                 int(n_matvec), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                 ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                 _stream_handle(A.val.device), ctypes.byref(out),
                                 ctypes.c_void_p(grad.data_ptr()), ctypes.byref(st)), "ld_logdet_grad")
    if return_stats:
        return out.value, grad, st.as_dict()
    return out.value, grad


def _autograd_function():
    torch = _torch()

    class LogdetFunction(torch.autograd.Function):
        """logdet_est(values) with backward = exact derivative of the estimate."""

        @staticmethod
        def forward(ctx, values, A, lmin, lmax, degree, n_matvec, seed, options):
            est, grad = logdet_with_grad(A.with_values(values.detach()), lmin, lmax, degree,
                                         n_matvec, seed, options)
            ctx.save_for_backward(grad)
            return torch.tensor(est, dtype=torch.float64, device=values.device)

        @staticmethod
        def backward(ctx, g):
            (grad,) = ctx.saved_tensors
            return (g.to(grad.dtype) * grad, None, None, None, None, None, None, None)

    return LogdetFunction


_LOGDET_FN = None


def LogdetFunction():
    global _LOGDET_FN
    if _LOGDET_FN is None:
        _LOGDET_FN = _autograd_function()
    return _LOGDET_FN


def logdet_autograd(values, A: CSR, lmin: float, lmax: float, degree: int, n_matvec: int,
                    seed: int = 0, options=None):
    """Differentiable estimate: gradients flow into ``values`` (A's nonzeros)."""
    return LogdetFunction().apply(values, A, lmin, lmax, degree, n_matvec, seed, options)


def apply_log(A: CSR, lmin: float, lmax: float, degree: int, V, options=None):
    """P_m(Q~) V + log(sigma) V ~= log(A) V for an n x ncols block V (row-major)."""
    torch = _torch()
    lib = nat.load()
    V = V.contiguous()
    if V.dtype != A.dtype or V.dim() != 2 or V.shape[0] != A.n:
        raise ValueError("V must be n x ncols with the matrix dtype")
    out = torch.empty_like(V)
    c = A.c_struct()
    o = _opts(options)
    if V.shape[1] == 0:   # nothing to apply; the call still checks its arguments
        nat.check(lib.ld_apply_log(ctypes.byref(c), float(lmin), float(lmax), int(degree), None, None, 0,
                                   ctypes.byref(o), None, 0, _stream_handle(V.device)), "ld_apply_log")
        return out
    b = ctypes.c_size_t(0)
    nat.check(lib.ld_workspace_size(ctypes.byref(c), int(degree), -int(V.shape[1]), 0,
                                    ctypes.byref(o), ctypes.byref(b)), "ld_workspace_size")
    ws = _workspace(int(b.value), V.device)
    nat.check(lib.ld_apply_log(ctypes.byref(c), float(lmin), float(lmax), int(degree),
                               ctypes.c_void_p(V.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                               int(V.shape[1]), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                               ws.numel(), _stream_handle(V.device)), "ld_apply_log")
    return out


def apply_log_adaptive(A: CSR, lmin: float, lmax: float, max_degree: int, tol: float, V, options=None):
    """Alg. 2 with per-column adaptive degree: (log(A) V, degrees), each column
    stopping at the first m with |d_m| ||w_m||_2 <= tol (at most max_degree)."""
    torch = _torch()
    lib = nat.load()
    V = V.contiguous()
    if V.dtype != A.dtype or V.dim() != 2 or V.shape[0] != A.n:
        raise ValueError("V must be n x ncols with the matrix dtype")
    out = torch.empty_like(V)
    ncols = int(V.shape[1])
    degrees = np.zeros(ncols, dtype=np.int32)
    c = A.c_struct()
    o = _opts(options)
    ws = None
    if ncols > 0:
        b = ctypes.c_size_t(0)
        nat.check(lib.ld_workspace_size(ctypes.byref(c), int(max_degree), -ncols, 1, ctypes.byref(o),
                                        ctypes.byref(b)), "ld_workspace_size")
        ws = _workspace(int(b.value), V.device)
    nat.check(lib.ld_apply_log_adaptive(
        ctypes.byref(c), float(lmin), float(lmax), int(max_degree), float(tol),
        ctypes.c_void_p(V.data_ptr() if ncols else None), ctypes.c_void_p(out.data_ptr() if ncols else None),
        ncols, ctypes.byref(o), ctypes.c_void_p(ws.data_ptr() if ws is not None else None),
        ws.numel() if ws is not None else 0, _stream_handle(V.device),
        degrees.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "ld_apply_log_adaptive")
    return out, degrees


def spectral_bounds(A: CSR, lanczos_steps: int = 0):
    """Gershgorin interval (lmin, lmax) computed on the GPU in FP64; with
    ``lanczos_steps`` > 0 the upper end is refined by Lanczos (App. A)."""
    lib = nat.load()
    c = A.c_struct()
    lo, hi = ctypes.c_double(0), ctypes.c_double(0)
    rc = lib.ld_spectral_bounds(ctypes.byref(c), int(lanczos_steps), _stream_handle(A.val.device),
                                ctypes.byref(lo), ctypes.byref(hi))
    if rc == nat.LD_EINDEF:
        return lo.value, hi.value
    nat.check(rc, "ld_spectral_bounds")
    return lo.value, hi.value


# ---- host-side pieces --------------------------------------------------------------------

def leja_points(count: int) -> np.ndarray:
    out = np.zeros(count, dtype=np.float64)
    nat.check(nat.load().ld_leja_points(count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
              "ld_leja_points")
    return out


def divided_differences(lo: float, hi: float, degree: int, s_val_mode: int = LD_SVAL_CENTER,
                        taylor_cap: int = 0):
    d = np.zeros(degree + 1, dtype=np.float64)
    terms = ctypes.c_int64(0)
    nat.check(nat.load().ld_divided_differences(float(lo), float(hi), int(degree), int(s_val_mode),
                                                int(taylor_cap),
                                                d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                                ctypes.byref(terms)), "ld_divided_differences")
    return d, int(terms.value)


def rademacher_host(seed: int, stream: int, n: int, row0: int, nrows: int, col0: int, ncols: int):
    out = np.zeros((nrows, ncols), dtype=np.int8)
    nat.check(nat.load().ld_rademacher_host(ctypes.c_uint64(int(seed) & (2**64 - 1)), stream, n, row0,
                                            nrows, col0, ncols,
                                            out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))),
              "ld_rademacher_host")
    return out


def squared_basis_coefficients(d) -> np.ndarray:
    d = np.ascontiguousarray(d, dtype=np.float64)
    c = np.zeros_like(d)
    nat.check(nat.load().ld_squared_basis_coefficients(
        len(d) - 1, d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "ld_squared_basis_coefficients")
    return c
