"""Pins for the oracle's Léja + Hutch++ estimator (Alg. 3)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as w
from oracle import exact, hutchpp, rng
from oracle.newton import NewtonPlan


def dense_hutchpp(Qd, lmin, lmax, degree, m_vec, seed):
    """Alg. 3 with F formed densely from the eigendecomposition (independent path)."""
    n = Qd.shape[0]
    plan = NewtonPlan(lmin, lmax, degree)
    lam, Vt = np.linalg.eigh(Qd)
    F = (Vt * plan.eval_scalar(lam)) @ Vt.T
    k, kg = hutchpp.split_queries(m_vec)
    S, G = rng.rademacher(seed, 0, n, k), rng.rademacher(seed, 1, n, kg)
    A, _ = np.linalg.qr(F @ S)
    U = G - A @ (A.T @ G)
    return n * math.log(plan.sigma) + np.trace(A.T @ F @ A) + np.trace(U.T @ F @ U) / kg


def test_cfg_small_closed_form_and_cholesky():
    Q = w.to_scipy(w.grid_laplacian_2d(32, 0.5))
    ex = exact.grid_logdet_2d(32, 0.5)
    assert ex == pytest.approx(exact.cholesky_logdet(Q.toarray()), rel=1e-13)
    # exact-trace mode: only the interpolation error remains (degree 40, [1,17])
    et = hutchpp.exact_trace(exact.grid_eigenvalues_2d(32, 0.5), 0.5, 8.5, 40)
    assert abs(et - ex) / ex < 1e-10


def test_against_dense_path():
    rng_ = np.random.default_rng(2)
    n = 80
    B = sp.random(n, n, density=0.08, random_state=4).toarray()
    Qd = B @ B.T + np.diag(rng_.uniform(0.3, 1.0, n))
    ev = np.linalg.eigvalsh(Qd)
    lmin, lmax = 0.9 * ev[0], 1.1 * ev[-1]
    for seed in (0, 1):
        a = hutchpp.logdet_estimate(sp.csr_matrix(Qd), lmin, lmax, 30, 12, seed)
        b = dense_hutchpp(Qd, lmin, lmax, 30, 12, seed)
        assert a == pytest.approx(b, rel=1e-12)


def test_exact_when_sketch_spans_space():
    # k >= n: the sketch captures all of F, the residual vanishes.
    rng_ = np.random.default_rng(1)
    n = 6
    B = rng_.standard_normal((n, n))
    Qd = B @ B.T + n * np.eye(n)
    ev = np.linalg.eigvalsh(Qd)
    lmin, lmax = 0.9 * ev[0], 1.1 * ev[-1]
    est = hutchpp.logdet_estimate(sp.csr_matrix(Qd), lmin, lmax, 25, 18, 9)
    assert est == pytest.approx(hutchpp.exact_trace(ev, lmin, lmax, 25), rel=1e-12)


def test_basis_invariance():
    Q = w.to_scipy(w.grid_laplacian_2d(12, 0.5))
    O, _ = np.linalg.qr(np.random.default_rng(0).standard_normal((4, 4)))

    def rotated(Y):
        A, _ = np.linalg.qr(Y)
        return A @ O

    a = hutchpp.logdet_estimate(Q, 0.5, 8.5, 30, 12, 5)
    b = hutchpp.logdet_estimate(Q, 0.5, 8.5, 30, 12, 5, orth=rotated)
    assert a == pytest.approx(b, rel=1e-13)


def test_unbiased():
    Q = w.to_scipy(w.grid_laplacian_2d(16, 0.5))
    et = hutchpp.exact_trace(exact.grid_eigenvalues_2d(16, 0.5), 0.5, 8.5, 30)
    hpp = np.array([hutchpp.logdet_estimate(Q, 0.5, 8.5, 30, 12, s) for s in range(60)])
    hut = np.array([hutchpp.hutchinson_estimate(Q, 0.5, 8.5, 30, 12, s) for s in range(60)])
    assert abs(hpp.mean() - et) < 3.5 * hpp.std(ddof=1) / math.sqrt(len(hpp))
    assert abs(hut.mean() - et) < 3.5 * hut.std(ddof=1) / math.sqrt(len(hut))


def test_lower_variance_than_hutchinson_on_decaying_spectrum():
    # Hutch++ removes the top of the spectrum exactly (Sec. 4.1); it beats
    # Hutchinson when log(Q~) is dominated by a few large eigenvalues.
    n = 200
    lam = 1.0 + 1e3 * np.exp(-np.arange(1, n + 1, dtype=float))
    O, _ = np.linalg.qr(np.random.default_rng(7).standard_normal((n, n)))
    Q = sp.csr_matrix((O * lam) @ O.T)
    lmin, lmax = 0.99, 400.0
    et = hutchpp.exact_trace(lam, lmin, lmax, 120)
    hpp = np.array([hutchpp.logdet_estimate(Q, lmin, lmax, 120, 30, s) for s in range(20)])
    hut = np.array([hutchpp.hutchinson_estimate(Q, lmin, lmax, 120, 30, s) for s in range(20)])
    assert hpp.std() < 0.5 * hut.std()
    assert abs(hpp.mean() - et) < 3.5 * hpp.std(ddof=1) / math.sqrt(len(hpp)) + 1e-9 * abs(et)


def test_sigma_split():
    # lmin >= 1 -> sigma = 1; lmin < 1 -> sigma = lmin and n log sigma is added.
    Q = w.to_scipy(w.grid_laplacian_2d(8, 3.0))
    a = hutchpp.logdet_estimate(Q, 3.0, 11.0, 30, 9, 1, return_parts=True)
    assert a["sigma"] == 1.0 and a["lo"] == 3.0
    b = hutchpp.logdet_estimate(Q / 4.0, 0.75, 2.75, 30, 9, 1, return_parts=True)
    assert b["sigma"] == 0.75 and b["lo"] == 1.0
    ex = exact.grid_logdet_2d(8, 3.0)
    # Monte-Carlo error of 9 queries on n = 64: a few units (std ~2)
    assert abs(a["logdet"] - ex) < 8.0
    assert abs(b["logdet"] - (ex - 64 * math.log(4.0))) < 8.0
    # the exact traces of the two polynomials agree with the closed form
    lam = exact.grid_eigenvalues_2d(8, 3.0)
    assert hutchpp.exact_trace(lam, 3.0, 11.0, 30) == pytest.approx(ex, rel=1e-9)
    assert hutchpp.exact_trace(lam / 4, 0.75, 2.75, 30) == pytest.approx(ex - 64 * math.log(4.0), rel=1e-9)


def test_gaussian_probes_exact_span_and_unbiased():
    # The paper's other probe distribution: the same two pins as Rademacher
    # (sketch spanning the space gives the exact trace; mean over seeds).
    rng_ = np.random.default_rng(1)
    n = 6
    B = rng_.standard_normal((n, n))
    Qd = B @ B.T + n * np.eye(n)
    ev = np.linalg.eigvalsh(Qd)
    lmin, lmax = 0.9 * ev[0], 1.1 * ev[-1]
    est = hutchpp.logdet_estimate(sp.csr_matrix(Qd), lmin, lmax, 25, 18, 9, probes="gaussian")
    assert est == pytest.approx(hutchpp.exact_trace(ev, lmin, lmax, 25), rel=1e-12)
    Q = w.to_scipy(w.grid_laplacian_2d(16, 0.5))
    et = hutchpp.exact_trace(exact.grid_eigenvalues_2d(16, 0.5), 0.5, 8.5, 30)
    hpp = np.array([hutchpp.logdet_estimate(Q, 0.5, 8.5, 30, 12, s, probes="gaussian") for s in range(60)])
    assert abs(hpp.mean() - et) < 3.5 * hpp.std(ddof=1) / math.sqrt(len(hpp))
    with pytest.raises(ValueError):
        hutchpp.logdet_estimate(Q, 0.5, 8.5, 30, 12, 0, probes="uniform")
