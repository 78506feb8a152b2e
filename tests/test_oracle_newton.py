"""Pins for the oracle's Newton-Léja recurrence (Alg. 2, mapped form)."""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as w
from oracle import divdiff, exact
from oracle.newton import NewtonPlan, apply_log


def test_polynomial_exactness():
    # With the divided differences of xi^q the Newton form is exactly xi^q, so
    # the recurrence must return T^q V, T = (Q~ - cI)/gamma.
    rng = np.random.default_rng(0)
    n = 50
    B = rng.standard_normal((n, n))
    Q = sp.csr_matrix(B @ B.T / n + 2.0 * np.eye(n))
    ev = np.linalg.eigvalsh(Q.toarray())
    lmin, lmax = 0.9 * ev[0], 1.1 * ev[-1]
    plan = NewtonPlan(lmin, lmax, 12)
    V = rng.standard_normal((n, 3))
    T = (Q.toarray() / plan.sigma - plan.c * np.eye(n)) / plan.gamma
    for q in (0, 1, 2, 5, 12):
        plan.d = divdiff.homogeneous_dd(plan.xi, q)
        ref = np.linalg.matrix_power(T, q) @ V
        np.testing.assert_allclose(plan.apply_poly(Q, V), ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_diagonal_matrix_with_nodes_as_eigenvalues():
    # P_m interpolates log at the nodes, so for Q = diag(sigma*z_i) it returns log exactly.
    lmin, lmax, m = 0.25, 4.0, 24
    plan = NewtonPlan(lmin, lmax, m)
    z = plan.c + plan.gamma * plan.xi             # nodes of Q~ = Q/sigma
    Q = sp.diags(plan.sigma * z).tocsr()
    V = np.eye(m + 1)
    out = apply_log(Q, V, lmin, lmax, m)
    np.testing.assert_allclose(np.diag(out), np.log(plan.sigma * z), rtol=0, atol=1e-12)
    assert np.abs(out - np.diag(np.diag(out))).max() == 0.0


def test_dirichlet_eigenvector():
    N, k2, m = 32, 0.5, 40
    Q = w.to_scipy(w.grid_laplacian_2d(N, k2))
    plan = NewtonPlan(k2, k2 + 8.0, m)
    for a, b in ((1, 1), (7, 20), (32, 32)):
        v = w.dirichlet_sine_vector_2d(N, a, b)[:, None]
        lam = exact.grid_eigenvalue_2d(N, k2, a, b)
        out = plan.apply_poly(Q, v)
        np.testing.assert_allclose(out, plan.eval_scalar(lam) * v, rtol=0, atol=1e-12)
        # and P_m approximates log on the spectrum (interval [1, 17], degree 40)
        assert abs(plan.eval_scalar(lam) - math.log(lam / plan.sigma)) < 1e-9


def test_against_dense_logm():
    rng = np.random.default_rng(3)
    n = 60
    B = rng.standard_normal((n, n))
    Qd = B @ B.T / n + 0.3 * np.eye(n)
    ev = np.linalg.eigvalsh(Qd)
    lmin, lmax = ev[0] * 0.95, ev[-1] * 1.05
    V = rng.standard_normal((n, 4))
    ref = sla.logm(Qd).real @ V
    # interpolation error bound: rho^-m with rho = (sqrt(k)+1)/(sqrt(k)-1)
    kap = lmax / lmin
    rho = (math.sqrt(kap) + 1) / (math.sqrt(kap) - 1)
    m = int(math.ceil(math.log(1e12) / math.log(rho))) + 20
    out = apply_log(sp.csr_matrix(Qd), V, lmin, lmax, m)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-8 * np.abs(ref).max())


def test_geometric_convergence_rate():
    # Proposition (Sec. 3): ||log - P_m||_inf decays like rho^-m.
    lo, hi = 1.0, 17.0
    x = np.linspace(lo, hi, 4001)
    kap = hi / lo
    rho = (math.sqrt(kap) + 1) / (math.sqrt(kap) - 1)
    errs = {}
    for m in (10, 20, 30):
        plan = NewtonPlan(lo, hi, m)
        errs[m] = np.abs(plan.eval_scalar(x) - np.log(x)).max()
    rate = (errs[30] / errs[10]) ** (1 / 20)
    assert rate < 1.15 / rho
    assert errs[30] < errs[20] < errs[10]


def test_dots_match_apply():
    rng = np.random.default_rng(5)
    Q = w.to_scipy(w.grid_laplacian_2d(10, 0.5))
    plan = NewtonPlan(0.5, 8.5, 15)
    X = rng.standard_normal((100, 3))
    s = plan.dots(Q, X)
    np.testing.assert_allclose(plan.d @ s, np.einsum("ij,ij->j", X, plan.apply_poly(Q, X)), rtol=1e-12)


def _sine_mode(N, a, b):
    i = np.arange(1, N + 1)
    return np.outer(np.sin(np.pi * a * i / (N + 1)), np.sin(np.pi * b * i / (N + 1))).ravel()


def test_adaptive_stopping_degree_closed_form():
    # For an eigenvector v of Q with eigenvalue lam, w_m = pi_m(t) v with
    # t = (lam/sigma - c)/gamma, so Alg. 2 stops at the first m with
    # |d_m| |pi_m(t)| ||v|| <= tol and returns P_m(lam/sigma) v (+ log(sigma) v).
    N, k2 = 24, 0.3
    Q = w.to_scipy(w.grid_laplacian_2d(N, k2))
    lmin, lmax = k2, k2 + 8.0
    from oracle.newton import NewtonPlan as NP, apply_log_adaptive
    plan = NP(lmin, lmax, 60)
    modes = [(1, 1), (3, 7), (12, 12), (24, 23)]
    V = np.stack([_sine_mode(N, a, b) for a, b in modes], axis=1)
    lam = np.array([exact.grid_eigenvalue_2d(N, k2, a, b) for a, b in modes])
    t = (lam / plan.sigma - plan.c) / plan.gamma
    norms = np.linalg.norm(V, axis=0)
    # e[m, col] = |d_m| |pi_m(t_col)| ||v_col|| by the scalar product formula
    e = np.empty((61, len(modes)))
    pi = np.ones_like(t)
    for m in range(61):
        e[m] = np.abs(plan.d[m]) * np.abs(pi) * norms
        if m < 60:
            pi = pi * (t - plan.xi[m])
    for tol in (1e-3, 1e-7, 1e-11):
        # expected stop: first m with e <= tol (a tol that sits exactly on some e would be a tie)
        assert np.min(np.abs(np.log(e / tol))) > 1e-6
        want = np.array([next((m for m in range(61) if e[m, c] <= tol), 60) for c in range(len(modes))])
        P, ms = apply_log_adaptive(Q, V, lmin, lmax, 60, tol)
        np.testing.assert_array_equal(ms, want)
        for c in range(len(modes)):
            ref = NP(lmin, lmax, max(int(ms[c]), 1))
            val = ref.d[0] if ms[c] == 0 else ref.eval_scalar(lam[c])
            np.testing.assert_allclose(P[:, c], (val + math.log(plan.sigma)) * V[:, c], rtol=1e-10,
                                       atol=1e-12 * np.abs(V[:, c]).max())
    assert len(set(want.tolist())) > 1          # the columns stopped at different degrees


def test_adaptive_limits():
    rng = np.random.default_rng(5)
    Q = w.to_scipy(w.grid_laplacian_2d(10, 0.5))
    V = rng.standard_normal((100, 3))
    from oracle.newton import NewtonPlan as NP
    plan = NP(0.5, 8.5, 30)
    P, ms = plan.apply_poly_adaptive(Q, V, 0.0)          # never small enough: full degree
    assert (ms == 30).all()
    np.testing.assert_allclose(P, plan.apply_poly(Q, V), rtol=1e-14, atol=1e-14)
    P, ms = plan.apply_poly_adaptive(Q, V, 1e30)         # stops before the first product
    assert (ms == 0).all()
    np.testing.assert_array_equal(P, plan.d[0] * V)
