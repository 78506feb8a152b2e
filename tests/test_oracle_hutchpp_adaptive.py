"""Pins of the oracle's Alg. 3 with Alg. 2's stopping rule (oracle/hutchpp.py
``logdet_estimate_adaptive``): special cases that reduce to other pinned
results, stopping degrees and values from closed-form products on a diagonal
matrix, and the exact log det when the sketch spans the whole space."""
import math

import numpy as np
import scipy.sparse as sp

import workloads as w
from oracle import hutchpp
from oracle.newton import NewtonPlan
from oracle.rng import rademacher


def test_tol_zero_is_the_fixed_degree_estimate():
    # no column ever meets tol = 0: every application runs to the cap, which is
    # Alg. 3 at that degree
    Q = w.to_scipy(w.grid_laplacian_2d(12, 0.4))
    lmin, lmax = 0.4, 8.4
    est, deg = hutchpp.logdet_estimate_adaptive(Q, lmin, lmax, 40, 0.0, 15, seed=3)
    ref = hutchpp.logdet_estimate(Q, lmin, lmax, 40, 15, seed=3)
    assert (deg == 40).all() and deg.size == 15
    assert abs(est - ref) <= 1e-12 * abs(ref)


def test_degree_zero_closed_form():
    # tol above every |d_0| ||x||: every column stops before its first product,
    # so F = d_0 I, the sketch spans span(S), and the estimate is
    # n log(sigma) + d_0 (k + ||(I - P_S) G||_F^2 / k_G)
    Q = w.to_scipy(w.grid_laplacian_2d(9, 0.7))
    n = Q.shape[0]
    lmin, lmax = 0.7, 8.7
    m_vec, seed = 14, 11                  # k = 4, k_G = 6
    est, deg = hutchpp.logdet_estimate_adaptive(Q, lmin, lmax, 30, 1e30, m_vec, seed)
    assert (deg == 0).all()
    k, kg = m_vec // 3, m_vec - 2 * (m_vec // 3)
    S = rademacher(seed, 0, n, k).astype(np.float64)
    G = rademacher(seed, 1, n, kg).astype(np.float64)
    resid = G - S @ np.linalg.lstsq(S, G, rcond=None)[0]
    plan = NewtonPlan(lmin, lmax, 30)
    want = n * math.log(plan.sigma) + plan.d[0] * (k + float((resid ** 2).sum()) / kg)
    assert abs(est - want) <= 1e-12 * abs(want)


def _pi_values(plan, t, m):
    """pi_m(t) = prod_{j<m} (t - xi_j) by direct products."""
    out = np.ones_like(t)
    for j in range(m):
        out = out * (t - plan.xi[j])
    return out


def test_diagonal_matrix_degrees_and_value_from_products():
    # Q = diag(lam): w_m = pi_m(t) * x entrywise, t = (lam/sigma - c)/gamma, so
    # each column's stopping degree is the first m with
    # |d_m| ||pi_m(t) x|| <= tol, and x^T F x = sum_i P_{m_x}(t_i) x_i^2.
    rng = np.random.default_rng(2)
    n = 300
    lam = np.sort(rng.uniform(0.3, 40.0, n))
    Q = sp.diags(lam).tocsr()
    lmin, lmax, cap, m_vec, seed = 0.3, 40.0, 80, 20, 5    # k = 6, k_G = 8
    plan = NewtonPlan(lmin, lmax, cap)
    t = (lam / plan.sigma - plan.c) / plan.gamma
    pis = np.stack([_pi_values(plan, t, m) for m in range(cap + 1)])      # (cap+1) x n
    seen = set()
    for tol in (1e-2, 1e-6, 1e-9):
        parts = hutchpp.logdet_estimate_adaptive(Q, lmin, lmax, cap, tol, m_vec, seed, return_parts=True)
        cols = np.concatenate([parts["S"], parts["A"], parts["U"]], axis=1)
        e = np.abs(plan.d)[:, None] * np.sqrt((pis ** 2) @ (cols ** 2))     # e[m, col]
        assert np.min(np.abs(np.log(e / tol))) > 1e-9                      # no ties with tol
        want = np.array([next((m for m in range(cap + 1) if e[m, c] <= tol), cap) for c in range(cols.shape[1])])
        np.testing.assert_array_equal(parts["degrees"], want)
        seen.update(want.tolist())
        # quadratic forms from the closed-form values P_m(t_i) = sum_j d_j pi_j(t_i)
        pvals = np.cumsum(plan.d[:, None] * pis, axis=0)                   # row m: P_m(t)
        k = m_vec // 3
        A, U = parts["A"], parts["U"]
        t_low = sum(float(pvals[want[k + i]] @ (A[:, i] ** 2)) for i in range(k))
        t_res = sum(float(pvals[want[2 * k + j]] @ (U[:, j] ** 2)) for j in range(U.shape[1])) / U.shape[1]
        ref = n * math.log(plan.sigma) + t_low + t_res
        assert abs(parts["logdet"] - ref) <= 1e-11 * abs(ref)
    assert len(seen) > 3   # columns and tolerances stopped at many different degrees


def test_full_sketch_gives_the_log_determinant():
    # k >= n: Q_b spans R^n, U vanishes, and with every column converged the
    # estimate is tr log(Q) up to the interpolation error at the stop
    Q = w.to_scipy(w.grid_laplacian_2d(5, 0.8))        # n = 25
    n = Q.shape[0]
    lam = np.linalg.eigvalsh(Q.toarray())
    lmin, lmax = 0.8, 8.8
    est, deg = hutchpp.logdet_estimate_adaptive(Q, lmin, lmax, 200, 1e-13, 3 * n, seed=1)
    exact = float(np.sum(np.log(lam)))
    assert abs(est - exact) <= 1e-9 * abs(exact)
    assert deg[n:2 * n].max() < 200                    # the basis columns met tol before the cap
