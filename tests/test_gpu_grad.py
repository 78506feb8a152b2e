"""GPU parity of the gradient entry point against the oracle's exact derivative.

The oracle's derivative (oracle/grad.py) is itself pinned to finite
differences of the FP64 estimate; here the HIP reverse sweep is compared
entry by entry, and the GMRF hyperparameter chain rule is checked through
torch.autograd.
"""
import math

import numpy as np
import pytest

import workloads as w
from oracle import bounds, grad as ograd, hutchpp
from tests.gpu_common import assert_cols_close, random_spd_csr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2603_02207_amd as ld  # noqa: E402

DEV = "cuda:0"


def to_gpu(csr, dtype):
    row_ptr, col_idx, val, n = csr
    vals = np.asarray(val, dtype=np.float32 if dtype == torch.float32 else np.float64)
    return ld.CSR.from_arrays(row_ptr, col_idx, vals, n, device=DEV, dtype=dtype), vals.astype(np.float64)


@pytest.mark.parametrize("m_vec,degree,stride", [(12, 20, 0), (30, 40, 1), (30, 40, 7), (9, 13, 5), (4, 11, 0),
                                                 (100, 16, 3)])
def test_grad_small_grid_fp64(m_vec, degree, stride):
    csr = w.grid_laplacian_2d(9, 0.5)
    A, vals = to_gpu(csr, torch.float64)
    est, g = ld.logdet_with_grad(A, 0.5, 8.5, degree, m_vec, 3, options=ld.Options(ckpt_stride=stride))
    ref_est, ref_g = ograd.logdet_grad((csr[0], csr[1], vals, csr[3]), 0.5, 8.5, degree, m_vec, 3)
    assert est == pytest.approx(ref_est, rel=1e-11)
    g = g.cpu().numpy()
    assert np.max(np.abs(g - ref_g)) < 1e-9 * np.max(np.abs(ref_g))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 2e-4)])
def test_grad_irregular(dtype, tol):
    csr = random_spd_csr(300, 5, long_rows=2)
    A, vals = to_gpu(csr, dtype)
    csr_v = (csr[0], csr[1], vals, csr[3])
    lmin, lmax = bounds.gershgorin(csr_v)
    est, g = ld.logdet_with_grad(A, lmin, lmax, 30, 21, 1)
    ref_est, ref_g = ograd.logdet_grad(csr_v, lmin, lmax, 30, 21, 1)
    assert abs(est - ref_est) / abs(ref_est) < (1e-10 if dtype == torch.float64 else 1e-5)
    assert_cols_close(g.double().cpu().numpy(), ref_g, tol)


def test_grad_fp32_grid32():
    csr = w.grid_laplacian_2d(32, 0.5)
    A, vals = to_gpu(csr, torch.float32)
    est, g = ld.logdet_with_grad(A, 0.5, 8.5, 40, 30, 0)
    ref_est, ref_g = ograd.logdet_grad((csr[0], csr[1], vals, csr[3]), 0.5, 8.5, 40, 30, 0)
    assert abs(est - ref_est) / abs(ref_est) < 1e-5
    assert_cols_close(g.double().cpu().numpy(), ref_g, 1e-4)


def gmrf_values(kappa, tau, csr):
    """Values of tau*(kappa^2 I + L) on the grid pattern as a differentiable function."""
    row_ptr, col_idx, val, n = csr
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    diag = torch.tensor(rows == col_idx, device=DEV)
    lap = torch.tensor(np.where(rows == col_idx, 4.0, -1.0), device=DEV, dtype=torch.float64)
    return tau * (lap + kappa ** 2 * diag.to(torch.float64))


def test_autograd_gmrf_hyperparameters():
    N = 12
    csr = w.grid_laplacian_2d(N, 0.1, tau=1.5)
    A, vals = to_gpu(csr, torch.float64)
    kappa = torch.tensor(math.sqrt(0.1), dtype=torch.float64, device=DEV, requires_grad=True)
    tau = torch.tensor(1.5, dtype=torch.float64, device=DEV, requires_grad=True)
    lmin, lmax = 1.5 * 0.1 * 0.999, 1.5 * 8.1
    v = gmrf_values(kappa, tau, csr)
    est = ld.logdet_autograd(v, A, lmin, lmax, 40, 30, 2)
    est.backward()

    def f(kk, tt):
        B = w.grid_laplacian_2d(N, kk * kk, tau=tt)
        return hutchpp.logdet_estimate(w.to_scipy(B), lmin, lmax, 40, 30, 2)

    h = 1e-6
    k0 = math.sqrt(0.1)
    fd_k = (f(k0 + h, 1.5) - f(k0 - h, 1.5)) / (2 * h)
    fd_t = (f(k0, 1.5 + h) - f(k0, 1.5 - h)) / (2 * h)
    assert kappa.grad.item() == pytest.approx(fd_k, rel=1e-6)
    assert tau.grad.item() == pytest.approx(fd_t, rel=1e-6)


def test_grad_gmrf2048_finite_difference_full_size():
    """2048 x 2048 GMRF, degree 100, 32 probes: adjoint vs central FD in tau (FP64 bulk)."""
    N, k2, tau, deg, mv = 2048, 0.1, 1.5, 100, 32
    csr = w.grid_laplacian_2d(N, k2, tau=tau)
    A, vals = to_gpu(csr, torch.float64)
    lmin, lmax = tau * k2 * 0.999, tau * (k2 + 8.0)
    est, g = ld.logdet_with_grad(A, lmin, lmax, deg, mv, 0)
    d_tau = float((g * A.val).sum().item()) / tau
    h = 1e-5 * tau
    ep = ld.logdet(A.with_values(A.val * ((tau + h) / tau)), lmin, lmax, deg, mv, 0)
    em = ld.logdet(A.with_values(A.val * ((tau - h) / tau)), lmin, lmax, deg, mv, 0)
    fd = (ep - em) / (2 * h)
    assert d_tau == pytest.approx(fd, rel=1e-6)
    # diagonal direction (kappa): d/dkappa = 2 kappa tau sum_diag grad
    row_ptr, col_idx = csr[0], csr[1]
    rows = np.repeat(np.arange(csr[3]), np.diff(row_ptr))
    diag = torch.tensor(rows == col_idx, device=DEV)
    kap = math.sqrt(k2)
    d_kap = 2 * kap * tau * float(g[diag].sum().item())
    hk = 1e-6

    def at_kappa(kk):
        return ld.logdet(A.with_values(torch.where(diag, A.val + tau * (kk * kk - k2), A.val)), lmin, lmax,
                         deg, mv, 0)

    fdk = (at_kappa(kap + hk) - at_kappa(kap - hk)) / (2 * hk)
    assert d_kap == pytest.approx(fdk, rel=1e-5)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-9), (torch.float32, 2e-4)])
@pytest.mark.parametrize("stride", [0, 4])
def test_grad_gaussian_probes(dtype, tol, stride):
    # Gaussian S and G (the paper's other probe choice): stored probe blocks
    # in the forward pass and the reverse sweep alike; with checkpoints the
    # sketch's Horner vectors are recomputed from a regenerated S
    csr = random_spd_csr(300, 5, long_rows=2)
    A, vals = to_gpu(csr, dtype)
    csr_v = (csr[0], csr[1], vals, csr[3])
    lmin, lmax = bounds.gershgorin(csr_v)
    est, g = ld.logdet_with_grad(A, lmin, lmax, 30, 21, 6, options=ld.Options(probe_dist=1, ckpt_stride=stride))
    ref_est, ref_g = ograd.logdet_grad(csr_v, lmin, lmax, 30, 21, 6, probes="gaussian")
    assert abs(est - ref_est) / abs(ref_est) < (1e-10 if dtype == torch.float64 else 1e-5)
    assert_cols_close(g.double().cpu().numpy(), ref_g, tol)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 2e-5)])
@pytest.mark.parametrize("degree", [12, 30])
def test_grad_equals_dense_inverse_when_sketch_spans_everything(dtype, tol, degree):
    # k = n = 49 sketch columns: Q_b spans R^n, the residual probes deflate to
    # zero and the estimate is the exact trace of P_m(Q~), whose derivative
    # w.r.t. entry (r, c) is (P_m'(Q~)/sigma)_{cr}.  That is within the
    # interpolant's derivative error max |P_m'(lam) - 1/lam| of the dense
    # (Q^{-1})_{cr} (and equal to it to rounding at degree 30).
    from oracle.newton import NewtonPlan

    csr = w.grid_laplacian_2d(7, 3.0)              # spectrum in [3, 11]
    A, vals = to_gpu(csr, dtype)
    row_ptr, col_idx, _, n = csr
    est, g = ld.logdet_with_grad(A, 3.0, 11.0, degree, 3 * n, 0)
    Q = w.to_scipy((row_ptr, col_idx, vals, n)).toarray()
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    inv_t = np.linalg.inv(Q)[col_idx, rows]
    plan = NewtonPlan(3.0, 11.0, degree)
    lam = np.linspace(3.0, 11.0, 20001)
    t = (lam - plan.c) / plan.gamma
    pi, dpi, dp = np.ones_like(t), np.zeros_like(t), np.zeros_like(t)
    for j in range(degree):
        dpi = pi + (t - plan.xi[j]) * dpi
        pi = pi * (t - plan.xi[j])
        dp += plan.d[j + 1] * dpi
    bound = float(np.max(np.abs(dp / plan.gamma - 1.0 / lam)))
    err = np.abs(g.double().cpu().numpy() - inv_t)
    assert err.max() <= bound + tol * np.abs(inv_t).max(), (err.max(), bound)


def test_grad_gmrf2048_fp32_against_fp64_finite_differences():
    """2048 x 2048 GMRF, degree 100, 32 probes, FP32 bulk: the hyperparameter
    derivatives from the FP32 gradient against central differences of the FP64
    estimate (same probes and interval), 1e-5 relative."""
    N, k2, tau, deg, mv = 2048, 0.1, 1.5, 100, 32
    csr = w.grid_laplacian_2d(N, k2, tau=tau)
    A32, _ = to_gpu(csr, torch.float32)
    A64, vals = to_gpu(csr, torch.float64)
    lmin, lmax = tau * k2 * 0.999, tau * (k2 + 8.0)
    est32, g = ld.logdet_with_grad(A32, lmin, lmax, deg, mv, 0)
    g = g.double()
    rows = np.repeat(np.arange(csr[3]), np.diff(csr[0]))
    diag = torch.tensor(rows == csr[1], device=DEV)
    d_tau = float((g * A32.val.double()).sum().item()) / tau
    kap = math.sqrt(k2)
    d_kap = 2 * kap * tau * float(g[diag].sum().item())
    h = 1e-5 * tau
    fd_tau = (ld.logdet(A64.with_values(A64.val * ((tau + h) / tau)), lmin, lmax, deg, mv, 0)
              - ld.logdet(A64.with_values(A64.val * ((tau - h) / tau)), lmin, lmax, deg, mv, 0)) / (2 * h)
    hk = 1e-6

    def at_kappa(kk):
        return ld.logdet(A64.with_values(torch.where(diag, A64.val + tau * (kk * kk - k2), A64.val)), lmin, lmax,
                         deg, mv, 0)

    fd_kap = (at_kappa(kap + hk) - at_kappa(kap - hk)) / (2 * hk)
    assert abs(est32 - ld.logdet(A64, lmin, lmax, deg, mv, 0)) < 1e-4 * abs(est32)
    assert d_tau == pytest.approx(fd_tau, rel=1e-5)
    assert d_kap == pytest.approx(fd_kap, rel=1e-5)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_grad_both_paths_agree(dtype):
    # The squared-basis path (default) and the Newton-form path (forced by
    # the forward quadratic-form mode) compute the same derivative in
    # different orders: both against the oracle, and the estimate of the
    # squared path equals the estimate entry point's bit for bit.
    csr = random_spd_csr(2000, 8, long_rows=2)
    A, vals = to_gpu(csr, dtype)
    csr_v = (csr[0], csr[1], vals, csr[3])
    lmin, lmax = bounds.gershgorin(csr_v)
    lmin = max(lmin, 0.3)
    ref_est, ref_g = ograd.logdet_grad(csr_v, lmin, lmax, 31, 24, 4)
    tol = 1e-9 if dtype == torch.float64 else 2e-4
    e_sq, g_sq, st_sq = ld.logdet_with_grad(A, lmin, lmax, 31, 24, 4, return_stats=True)
    e_nf, g_nf, st_nf = ld.logdet_with_grad(A, lmin, lmax, 31, 24, 4, options=ld.Options(dot_mode=ld.LD_DOT_FORWARD),
                                            return_stats=True)
    assert st_sq["dot_mode_used"] == ld.LD_DOT_SQUARED and st_nf["dot_mode_used"] == ld.LD_DOT_FORWARD
    assert e_sq == ld.logdet(A, lmin, lmax, 31, 24, 4)
    for e, g in ((e_sq, g_sq), (e_nf, g_nf)):
        assert abs(e - ref_est) < (1e-10 if dtype == torch.float64 else 1e-5) * abs(ref_est)
        assert_cols_close(g.double().cpu().numpy(), ref_g, tol)


def test_grad_gmrf2048_checkpoint_stride_is_exact():
    """2048 x 2048 GMRF, degree 100, 32 probes, FP32: sqrt(m) checkpoints
    (stride 10: the stored vectors recomputed segment by segment) give the
    same gradient, bit for bit, as keeping every vector."""
    N, k2, tau, deg, mv = 2048, 0.1, 1.5, 100, 32
    csr = w.grid_laplacian_2d(N, k2, tau=tau)
    A, _ = to_gpu(csr, torch.float32)
    lmin, lmax = tau * k2 * 0.999, tau * (k2 + 8.0)
    e1, g1 = ld.logdet_with_grad(A, lmin, lmax, deg, mv, 0, options=ld.Options(ckpt_stride=1))
    e10, g10 = ld.logdet_with_grad(A, lmin, lmax, deg, mv, 0, options=ld.Options(ckpt_stride=10))
    assert e1 == e10 and torch.equal(g1, g10)
    assert ld.workspace_size(A, deg, mv, True, ld.Options(ckpt_stride=10)) < \
        0.5 * ld.workspace_size(A, deg, mv, True, ld.Options(ckpt_stride=1))


def test_grad_rejects_a_pattern_without_mirrors():
    # A grid Laplacian plus an explicit zero at (r, r+1) for r at the end of a
    # grid line, whose mirror (r+1, r) is not stored: the same matrix, but the
    # per-entry derivative of the quadratic forms has no mirrored entry to be
    # averaged with.  Both the diagonal storage (offsets still -N, -1, 0, 1, N)
    # and the CSR path refuse the gradient; the estimate is unaffected.
    N = 24
    row_ptr, col_idx, val, n = w.grid_laplacian_2d(N, 0.5)
    r_x = 5 * N + N - 1                       # last point of grid line 5
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    rr = np.concatenate([rows, [r_x]])
    cc = np.concatenate([col_idx, [r_x + 1]])
    vv = np.concatenate([val, [0.0]])
    order = np.lexsort((cc, rr))
    rp2 = np.concatenate([[0], np.cumsum(np.bincount(rr[order], minlength=n))]).astype(np.int32)
    csr = (rp2, cc[order].astype(np.int32), vv[order], n)
    A, _ = to_gpu(csr, torch.float64)
    A_ref, _ = to_gpu((row_ptr, col_idx, val, n), torch.float64)
    est, st = ld.logdet(A, 0.5, 8.5, 20, 12, 1, return_stats=True)
    assert st["dia_diagonals"] == 5
    assert abs(est - ld.logdet(A_ref, 0.5, 8.5, 20, 12, 1)) <= 1e-12 * abs(est)
    for opts in (None, ld.Options(csr_only=1)):
        with pytest.raises(ld.NativeError, match="symmetric sparsity pattern"):
            ld.logdet_with_grad(A, 0.5, 8.5, 20, 12, 1, options=opts)
