"""CPU tests of the native library: exported symbols and its host-side logic.

No GPU is used: only functions that run on the host (Léja table, Alg. 1
divided differences, the probe generator, the squared-basis coefficients,
argument checking) are called.
"""
import ctypes
import math
import os
import re

import mpmath
import numpy as np
import pytest

import paper_2603_02207_amd as ld
from paper_2603_02207_amd import _native as nat
from oracle import divdiff, leja, rng

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "leja_logdet.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ld_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = nat.load()
    names = declared_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
        assert name in nat.SIGNATURES, name
    assert lib.ld_version().decode().startswith("leja_logdet")


def test_library_built_from_these_sources():
    # ld_version carries the hash of the csrc/ and include/ files the library
    # was compiled from; it must be the hash of the files in this tree
    assert nat.built_source_hash() == nat.source_hash()


def test_error_strings():
    lib = nat.load()
    for code in range(0, -8, -1):
        assert lib.ld_error_string(code)
    assert b"LD_EINVAL" in lib.ld_error_string(-1)


def test_leja_table_bit_identical_to_oracle():
    np.testing.assert_array_equal(ld.leja_points(600), leja.fast_leja_vectorised(600))


@pytest.mark.parametrize("lo,hi,m", [(1.0, 17.0, 40), (1.0, 81.0, 80), (1.0, 241.0, 120),
                                     (2.5, 3.0, 30), (1.0, 81.0, 1)])
def test_alg1_divided_differences_match_oracle(lo, hi, m):
    d, terms = ld.divided_differences(lo, hi, m)
    ref = divdiff.exact_dd(lo, hi, leja.fast_leja_vectorised(m + 1))
    assert np.max(np.abs(d - ref)) < 5e-14
    assert terms > 10


def test_alg1_ill_conditioned_interval():
    # condition number 1e5: ~1.8e6 Taylor terms, still at FP64 accuracy
    d, terms = ld.divided_differences(1.0, 1e5, 60)
    ref = divdiff.exact_dd(1.0, 1e5, leja.fast_leja_vectorised(61))
    assert terms > 1e6
    assert np.max(np.abs(d - ref)) < 1e-9 * np.max(np.abs(ref))


@pytest.mark.parametrize("lo,hi,m,cap", [(1.0, 17.0, 40, 2000), (1.0, 81.0, 80, 5000), (2.5, 3.0, 30, 300)])
def test_alg1_half_lmax_variant_matches_oracle(lo, hi, m, cap):
    # s = lambda_max/2 (Sec. 3.1, Tab. 3/4's second variant): the library's
    # Alg. 1 against the oracle's Alg. 1 after the same number of terms
    d, terms = ld.divided_differences(lo, hi, m, ld.LD_SVAL_HALF_LMAX, cap)
    ref, p = divdiff.alg1_dd(lo, hi, leja.fast_leja_vectorised(m + 1), "half_lmax", taylor_cap=cap)
    assert terms == p == cap
    assert np.max(np.abs(d - ref)) < 1e-13 * max(1.0, np.max(np.abs(ref)))
    # and it is not the exact divided differences (the series has not converged)
    exact = divdiff.exact_dd(lo, hi, leja.fast_leja_vectorised(m + 1))
    assert np.max(np.abs(d - exact)) > 1e-6


def test_probe_generator_bit_identical_to_oracle():
    n = 1000
    for seed, stream in ((0, 0), (12345, 1), (2**63 + 7, 0)):
        S = ld.rademacher_host(seed, stream, n, 0, n, 0, 5)
        np.testing.assert_array_equal(S.astype(float), rng.rademacher(seed, stream, n, 5))
    sub = ld.rademacher_host(9, 1, n, 100, 7, 2, 3)
    np.testing.assert_array_equal(sub.astype(float), rng.rademacher(9, 1, n, 5)[100:107, 2:5])


def test_squared_basis_coefficients():
    # independent check: expand both forms in the monomial basis at high precision
    m = 30
    xi = leja.fast_leja_vectorised(m + 2)
    d = divdiff.exact_dd(1.0, 81.0, xi[: m + 1])
    c = ld.squared_basis_coefficients(d)
    mpmath.mp.dps = 60
    X = [mpmath.mpf(float(x)) for x in xi]
    t = [mpmath.mpf(v) / 7 for v in range(-14, 15)]   # sample points in [-2, 2]
    for tt in t:
        pi = [mpmath.mpf(1)]
        for k in range(m + 1):
            pi.append(pi[-1] * (tt - X[k]))
        p_newton = sum(mpmath.mpf(float(d[j])) * pi[j] for j in range(m + 1))
        p_sq = sum(mpmath.mpf(float(c[i])) * (pi[i // 2] ** 2 if i % 2 == 0 else pi[i // 2] * pi[i // 2 + 1])
                   for i in range(m + 1))
        assert abs(float(p_newton - p_sq)) < 1e-12


def test_host_argument_errors():
    lib = nat.load()
    out = np.zeros(4)
    p = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.ld_leja_points(-1, p) == nat.LD_EINVAL
    assert lib.ld_divided_differences(0.0, 2.0, 3, 0, 0, p, None) == nat.LD_EINVAL
    assert lib.ld_divided_differences(2.0, 1.0, 3, 0, 0, p, None) == nat.LD_EINVAL
    assert lib.ld_divided_differences(1.0, 2.0, 3, 7, 0, p, None) == nat.LD_EINVAL
    assert b"lo" in lib.ld_last_error_detail() or lib.ld_last_error_detail()


def test_device_entry_points_reject_bad_arguments_before_any_gpu_work():
    lib = nat.load()
    A = nat.LdCsr()
    A.n, A.nnz, A.dtype = 10, 28, nat.LD_F32
    A.row_ptr = A.col_idx = A.val = 1   # never dereferenced: the checks fail first
    out = ctypes.c_double()
    ws = ctypes.c_size_t()
    o = nat.LdOptions()
    lib.ld_default_options(ctypes.byref(o))

    def est(lmin, lmax, deg, mv):
        return lib.ld_logdet_estimate(ctypes.byref(A), lmin, lmax, deg, mv, 0, ctypes.byref(o), None, 0,
                                      None, ctypes.byref(out), None)

    assert est(-1.0, 2.0, 10, 9) == nat.LD_EINVAL
    assert est(2.0, 1.0, 10, 9) == nat.LD_EINVAL
    assert est(0.5, 2.0, 0, 9) == nat.LD_EINVAL
    assert est(0.5, 2.0, 10, 2) == nat.LD_EINVAL
    assert est(0.5, 2.0, 10, 33) == nat.LD_EINVAL    # k = 11 > n = 10
    A.dtype = 5
    assert est(0.5, 2.0, 10, 9) == nat.LD_EINVAL
    A.dtype = nat.LD_F32
    assert lib.ld_workspace_size(ctypes.byref(A), 10, 9, 0, None, ctypes.byref(ws)) == nat.LD_OK
    assert ws.value > 0
    assert lib.ld_workspace_size(ctypes.byref(A), 0, 9, 0, None, ctypes.byref(ws)) == nat.LD_EINVAL
    A.n = 0
    assert lib.ld_workspace_size(ctypes.byref(A), 10, 9, 0, None, ctypes.byref(ws)) == nat.LD_EINVAL
