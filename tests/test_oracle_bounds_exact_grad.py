"""Pins for the spectral bounds, the exact references and the gradient oracle."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as w
from oracle import bounds, exact, grad, hutchpp


def test_gershgorin_grids():
    assert bounds.gershgorin(w.grid_laplacian_2d(32, 0.5)) == (0.5, 8.5)
    lo, hi = bounds.gershgorin(w.grid_laplacian_3d(6, 0.05))
    assert lo == pytest.approx(0.05, abs=1e-15) and hi == pytest.approx(12.05, abs=1e-14)
    lo, hi = bounds.gershgorin(w.grid_laplacian_2d(16, 0.1, tau=1.5))
    assert lo == pytest.approx(0.15) and hi == pytest.approx(12.15)


def test_gershgorin_contains_spectrum():
    A = w.chung_lu_laplacian(2000, seed=3)
    lo, hi = bounds.gershgorin(A)
    ev = np.linalg.eigvalsh(w.to_scipy(A).toarray())
    assert lo <= ev[0] + 1e-12 and ev[-1] <= hi + 1e-9
    assert lo == pytest.approx(1e-2, abs=1e-9)     # Laplacian rows sum to zero


def test_lanczos_lmax():
    A = w.chung_lu_laplacian(1500, seed=1)
    Q = w.to_scipy(A)
    ev = np.linalg.eigvalsh(Q.toarray())
    est = bounds.lanczos_lmax(Q, 60)
    assert est <= ev[-1] * (1 + 1e-12)
    assert est == pytest.approx(ev[-1], rel=1e-6)


def test_gmrf_theta_closed_form():
    # I + theta*Adj: closed-form eigenvalues and log det against dense algebra
    for N, th in ((7, -0.22), (10, -0.24), (9, 0.1)):
        Q = w.to_scipy(w.gmrf_theta(N, th)).toarray()
        np.testing.assert_allclose(np.sort(exact.gmrf_theta_eigenvalues(N, th)), np.linalg.eigvalsh(Q),
                                   rtol=1e-13, atol=1e-13)
        assert exact.gmrf_theta_logdet(N, th) == pytest.approx(exact.cholesky_logdet(Q), rel=1e-12)
        assert bounds.gershgorin(w.gmrf_theta(N, th)) == pytest.approx((1 - 4 * abs(th), 1 + 4 * abs(th)))


def test_banded_logdet_against_dense():
    for n, seed in ((50, 0), (333, 4)):
        csr = w.pentadiagonal(n, seed)
        Q = w.to_scipy(csr).toarray()
        assert exact.banded_logdet(csr, 2) == pytest.approx(exact.cholesky_logdet(Q), rel=1e-14)
        assert exact.banded_logdet(csr, 5) == pytest.approx(exact.cholesky_logdet(Q), rel=1e-14)
    g = w.grid_laplacian_2d(6, 0.3)                     # bandwidth N
    assert exact.banded_logdet(g, 6) == pytest.approx(exact.grid_logdet_2d(6, 0.3), rel=1e-13)
    with pytest.raises(ValueError):
        exact.banded_logdet(g, 5)


def test_grid_matfun_diag_against_dense():
    import scipy.linalg as sla
    for N, th in ((12, -0.22), (9, 0.15)):
        Q = w.to_scipy(w.gmrf_theta(N, th)).toarray()
        lam = exact.gmrf_theta_eigenvalues(N, th)
        for f, fm in ((np.log, lambda M: sla.logm(M).real), (np.exp, sla.expm)):
            np.testing.assert_allclose(exact.grid_matfun_diag_2d(N, f(lam)), np.diag(fm(Q)), rtol=1e-12,
                                       atol=1e-13)


def test_lanczos_upper_brackets_top_eigenvalue():
    from oracle import rng
    for A, steps in ((w.chung_lu_laplacian(1500, seed=1), 40), (w.grid_laplacian_2d(30, 0.5), 25),
                     (w.pentadiagonal(800, seed=3), 30)):
        Q = w.to_scipy(A)
        n = Q.shape[0]
        ev = np.linalg.eigvalsh(Q.toarray())
        v0 = rng.rademacher(0, 2, n, 1)[:, 0]
        theta, upper = bounds.lanczos_upper(Q, steps, v0)
        assert theta <= ev[-1] * (1 + 1e-12)         # a Ritz value never exceeds lambda_max
        assert upper >= ev[-1] * (1 - 1e-12)         # the residual margin covers the gap
        assert upper <= bounds.gershgorin(A)[1] * 1.5


def test_lanczos_upper_whole_space_is_exact():
    A = w.grid_laplacian_2d(6, 0.3)
    Q = w.to_scipy(A)
    ev = np.linalg.eigvalsh(Q.toarray())
    from oracle import rng
    theta, upper = bounds.lanczos_upper(Q, 36, rng.rademacher(0, 2, 36, 1)[:, 0])
    assert theta == pytest.approx(ev[-1], rel=1e-12)
    assert upper == pytest.approx(ev[-1], rel=1e-10)


def test_closed_form_logdets():
    for N, k2 in ((5, 0.5), (9, 0.1)):
        Q = w.to_scipy(w.grid_laplacian_2d(N, k2, tau=1.5)).toarray()
        assert exact.grid_logdet_2d(N, k2, 1.5) == pytest.approx(exact.cholesky_logdet(Q), rel=1e-13)
    Q3 = w.to_scipy(w.grid_laplacian_3d(6, 0.05)).toarray()
    assert exact.grid_logdet_3d(6, 0.05) == pytest.approx(exact.cholesky_logdet(Q3), rel=1e-13)
    # d/dkappa by central differences of the closed form
    k = math.sqrt(0.1)
    h = 1e-6
    fd = (exact.grid_logdet_2d(9, (k + h) ** 2) - exact.grid_logdet_2d(9, (k - h) ** 2)) / (2 * h)
    assert exact.grid_logdet_2d_dkappa(9, 0.1) == pytest.approx(fd, rel=1e-7)


@pytest.mark.parametrize("seed", [0, 3])
def test_gradient_against_finite_differences(seed):
    A = w.grid_laplacian_2d(8, 0.5)
    est, g = grad.logdet_grad(A, 0.5, 8.5, 20, 12, seed)
    assert est == pytest.approx(hutchpp.logdet_estimate(w.to_scipy(A), 0.5, 8.5, 20, 12, seed), rel=1e-14)
    rng = np.random.default_rng(seed + 10)
    for _ in range(2):
        E = rng.standard_normal(len(A[2]))
        fd = grad.fd_directional(A, E, 0.5, 8.5, 20, 12, seed, 1e-5)
        assert g @ E == pytest.approx(fd, rel=1e-7)
    # a single entry (the sketch-basis term is what makes this match)
    E = np.zeros(len(A[2]))
    E[17] = 1.0
    fd = grad.fd_directional(A, E, 0.5, 8.5, 20, 12, seed, 1e-5)
    assert g[17] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_gradient_gmrf_hyperparameters_and_exact_limit():
    # Q = tau (kappa^2 I + L): d/dtau = <g, val>/tau, d/dkappa = 2 kappa tau sum_diag g.
    N, k2, tau = 10, 0.5, 1.5
    A = w.grid_laplacian_2d(N, k2, tau)
    lmin, lmax = tau * k2 * 0.999, tau * (k2 + 8)
    est, g = grad.logdet_grad(A, lmin, lmax, 40, 60, 1)
    row_ptr, col_idx, val, n = A
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    diag = rows == col_idx
    d_tau = g @ val / tau
    d_kappa = 2 * math.sqrt(k2) * tau * g[diag].sum()

    def est_at(kk, tt):
        B = w.grid_laplacian_2d(N, kk, tt)
        return hutchpp.logdet_estimate(w.to_scipy(B), lmin, lmax, 40, 60, 1)

    h = 1e-5
    fd_tau = (est_at(k2, tau + h) - est_at(k2, tau - h)) / (2 * h)
    k = math.sqrt(k2)
    fd_kappa = (est_at((k + h) ** 2, tau) - est_at((k - h) ** 2, tau)) / (2 * h)
    assert d_tau == pytest.approx(fd_tau, rel=1e-7)
    assert d_kappa == pytest.approx(fd_kappa, rel=1e-7)
    # estimator derivatives approximate the exact ones (n/tau and the closed form)
    assert d_tau == pytest.approx(n / tau, rel=0.05)
    assert d_kappa == pytest.approx(tau * 0 + exact.grid_logdet_2d_dkappa(N, k2), rel=0.1)


def test_gradient_gaussian_probes_against_finite_differences():
    A = w.grid_laplacian_2d(8, 0.5)
    est, g = grad.logdet_grad(A, 0.5, 8.5, 20, 12, 4, probes="gaussian")
    E = np.random.default_rng(21).standard_normal(len(A[2]))
    fd = grad.fd_directional(A, E, 0.5, 8.5, 20, 12, 4, 1e-5, probes="gaussian")
    assert g @ E == pytest.approx(fd, rel=1e-7)


def interpolant_errors(plan, lmin, lmax):
    """max over [lmin, lmax] of |P_m(lam/sigma) + log sigma - log lam| and of
    |d/dlam P_m(lam/sigma) - 1/lam| (Newton form and its derivative by the
    product rule, on a fine grid)."""
    lam = np.linspace(lmin, lmax, 20001)
    t = (lam / plan.sigma - plan.c) / plan.gamma
    pi, dpi = np.ones_like(t), np.zeros_like(t)
    p, dp = np.full_like(t, plan.d[0]), np.zeros_like(t)
    for j in range(plan.degree):
        dpi = pi + (t - plan.xi[j]) * dpi
        pi = pi * (t - plan.xi[j])
        p += plan.d[j + 1] * pi
        dp += plan.d[j + 1] * dpi
    value = np.max(np.abs(p + math.log(plan.sigma) - np.log(lam)))
    deriv = np.max(np.abs(dp / (plan.sigma * plan.gamma) - 1.0 / lam))
    return float(value), float(deriv)


@pytest.mark.parametrize("degree", [12, 20, 40])
def test_gradient_equals_dense_inverse_when_sketch_spans_everything(degree):
    # With k = n sketch columns the basis Q_b spans R^n, the residual probes
    # deflate to zero and the estimate is the exact trace n log sigma +
    # tr P_m(Q~); its derivative w.r.t. the stored entry (r, c) is then
    # (P_m'(Q~)/sigma)_{cr}, which differs from d log det / dQ_rc = (Q^{-1})_{cr}
    # by at most the interpolant's derivative error max |P_m'(lam) - 1/lam|
    # (spectral bound on each entry).
    csr = w.grid_laplacian_2d(7, 3.0)              # n = 49, spectrum in [3, 11]
    row_ptr, col_idx, val, n = csr
    est, g = grad.logdet_grad(csr, 3.0, 11.0, degree, 3 * n, 0)
    Q = w.to_scipy(csr).toarray()
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    inv_t = np.linalg.inv(Q)[col_idx, rows]
    from oracle.newton import NewtonPlan
    value_err, deriv_err = interpolant_errors(NewtonPlan(3.0, 11.0, degree), 3.0, 11.0)
    assert np.max(np.abs(g - inv_t)) <= deriv_err + 1e-12
    assert abs(est - exact.cholesky_logdet(Q)) <= n * value_err + 1e-10
    if degree == 12:   # the bound is not vacuous: a visible polynomial error remains
        assert np.max(np.abs(g - inv_t)) > 1e-3 * deriv_err
