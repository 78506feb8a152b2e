"""The estimate entry point that allocates nothing (ld_logdet_estimate_noalloc).

It runs the same kernels as ld_logdet_estimate on the library's static scratch
(a 64 MiB device array per GPU) instead of a caller workspace.  Called through
the C ABI, its result must equal ld_logdet_estimate's on the same arguments,
and the oracle's within the estimator's tolerances; two calls in a row, the
second with a smaller input, check that what the first call left in the
scratch does not leak into the second.
"""
import ctypes

import numpy as np
import pytest

import workloads as w
from oracle import bounds, hutchpp
from tests.gpu_common import random_spd_csr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2603_02207_amd as ld  # noqa: E402
from paper_2603_02207_amd import _native as nat  # noqa: E402

DEV = "cuda:0"


def noalloc(A, lmin, lmax, degree, m_vec, seed, options=None):
    """(return code, estimate, stats) of the C entry point."""
    lib = nat.load()
    c = A.c_struct()
    o = (options or ld.Options()).to_c()
    out = ctypes.c_double(float("nan"))
    st = nat.LdStats()
    stream = ctypes.c_void_p(torch.cuda.current_stream(DEV).cuda_stream)
    rc = lib.ld_logdet_estimate_noalloc(ctypes.byref(c), float(lmin), float(lmax), int(degree), int(m_vec),
                                        ctypes.c_uint64(seed), ctypes.byref(o), stream, ctypes.byref(out),
                                        ctypes.byref(st))
    return rc, out.value, st.as_dict()


def to_gpu(csr, dtype):
    vals = np.asarray(csr[2], dtype=np.float32 if dtype == torch.float32 else np.float64)
    return (ld.CSR.from_arrays(csr[0], csr[1], vals, csr[3], device=DEV, dtype=dtype),
            (csr[0], csr[1], vals.astype(np.float64), csr[3]))


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-5), (torch.float64, 1e-10)])
def test_noalloc_equals_workspace_entry_point_two_calls(dtype, tol):
    # first a larger input (a 5-point grid in diagonal storage, several
    # sketch blocks), then a smaller one (an irregular matrix with long rows
    # on the CSR path, another query count and Gaussian probes)
    cases = [(w.grid_laplacian_2d(160, 0.3), 40, 60, 3, ld.Options()),
             (random_spd_csr(2000, 4, long_rows=2), 30, 21, 5, ld.Options(probe_dist=1))]
    for csr, degree, m_vec, seed, opts in cases:
        A, csr_v = to_gpu(csr, dtype)
        lo, hi = bounds.gershgorin(csr_v)
        lo = max(lo, 0.3)
        rc, est, st = noalloc(A, lo, hi, degree, m_vec, seed, opts)
        assert rc == nat.LD_OK, nat.load().ld_last_error_detail()
        ref_ws = ld.logdet(A, lo, hi, degree, m_vec, seed, options=opts)
        assert est == ref_ws                     # same kernels, same order: the same bits
        ref = hutchpp.logdet_estimate(w.to_scipy(csr_v), lo, hi, degree, m_vec, seed,
                                      probes="gaussian" if opts.probe_dist else "rademacher")
        assert abs(est - ref) < tol * abs(ref)
        assert st["k"] == m_vec // 3 and st["ms_steps1"] == 0.0   # no events were created
        assert ld.workspace_size(A, degree, m_vec, False, opts) <= 64 << 20


def test_noalloc_rejects_inputs_beyond_the_scratch():
    csr = w.grid_laplacian_2d(1024, 0.1)
    A, _ = to_gpu(csr, torch.float32)
    assert ld.workspace_size(A, 80, 60) > 64 << 20
    rc, est, _ = noalloc(A, 0.1, 8.1, 80, 60, 0)
    assert rc == nat.LD_EWORKSPACE
    assert b"static scratch" in nat.load().ld_last_error_detail()
    # a call that fits still works afterwards
    small = w.grid_laplacian_2d(20, 0.5)
    A2, csr_v = to_gpu(small, torch.float64)
    rc, est, _ = noalloc(A2, 0.5, 8.5, 20, 12, 1)
    assert rc == nat.LD_OK and est == ld.logdet(A2, 0.5, 8.5, 20, 12, 1)
