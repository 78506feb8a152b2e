"""Spectral interval estimates (oracle side).

* ``gershgorin``: the paper estimates [lambda_min, lambda_max] with the
  Gershgorin circle theorem (Sec. 3; Alg. 1/2 step 1; timing note of
  Sec. 5.1): the union of the discs centred at a_ii with radius
  sum_{j != i} |a_ij|, read as the real interval
  [min_i (a_ii - r_i), max_i (a_ii + r_i)].  A non-positive lower bound is
  returned as is (the paper's remark replaces it by some unstated eps > 0;
  the caller must supply a positive lmin).
* ``lanczos_lmax``: the alternative of Appendix A for lambda_max, a few
  Lanczos steps (largest Ritz value of the tridiagonal projection).
* ``lanczos_upper``: the same projection from a given start vector, and the
  largest Ritz value plus its residual norm beta_k |s_k| (s the Ritz vector
  in the Krylov basis): the Ritz value alone is below lambda_max, the sum is
  the usual practical upper bound.

Pinned by: closed-form intervals of the Dirichlet grid Laplacians, dense
eigenvalues of small SPD matrices, and the exact top eigenvalue when the
Krylov space is the whole space (tests/test_oracle_bounds_exact_grad.py).
"""
from __future__ import annotations

import numpy as np


def gershgorin(csr):
    """(lmin, lmax) of a CSR matrix (row_ptr, col_idx, val, n), FP64."""
    row_ptr, col_idx, val, n = csr
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    val = np.asarray(val, dtype=np.float64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    is_diag = rows == col_idx
    diag = np.zeros(n)
    np.add.at(diag, rows[is_diag], val[is_diag])
    radius = np.zeros(n)
    np.add.at(radius, rows[~is_diag], np.abs(val[~is_diag]))
    return float(np.min(diag - radius)), float(np.max(diag + radius))


def lanczos_lmax(Q, steps: int, seed: int = 0):
    """Largest Ritz value after ``steps`` Lanczos steps with full reorthogonalisation."""
    n = Q.shape[0]
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    V = [v]
    alphas, betas = [], []
    w_prev = np.zeros(n)
    beta = 0.0
    for _ in range(min(steps, n)):
        w = Q @ V[-1] - beta * w_prev
        a = float(V[-1] @ w)
        w -= a * V[-1]
        for u in V:                      # full reorthogonalisation
            w -= (u @ w) * u
        alphas.append(a)
        beta = float(np.linalg.norm(w))
        if beta < 1e-14:
            break
        betas.append(beta)
        w_prev = V[-1]
        V.append(w / beta)
    k = len(alphas)
    T = np.diag(alphas) + np.diag(betas[: k - 1], 1) + np.diag(betas[: k - 1], -1)
    return float(np.linalg.eigvalsh(T)[-1])


def lanczos_upper(Q, steps: int, v0):
    """(theta, theta + beta_k |s_k|) after ``steps`` Lanczos steps from v0.

    Full reorthogonalisation; stops early on an invariant subspace (then the
    residual term is zero).
    """
    n = Q.shape[0]
    v = np.asarray(v0, dtype=np.float64)
    v = v / np.linalg.norm(v)
    V = [v]
    alphas, betas = [], []
    beta = 0.0
    k_max = min(steps, n)
    for j in range(k_max):
        w = Q @ V[-1]
        a = float(V[-1] @ w)
        w = w - a * V[-1]
        if j > 0:
            w = w - betas[-1] * V[-2]
        for u in V:                      # full reorthogonalisation
            w = w - (u @ w) * u
        alphas.append(a)
        beta = float(np.linalg.norm(w))
        if j + 1 == k_max or beta <= 1e-14 * max(abs(a), 1.0):
            break
        betas.append(beta)
        V.append(w / beta)
    k = len(alphas)
    T = np.diag(alphas) + np.diag(betas[: k - 1], 1) + np.diag(betas[: k - 1], -1)
    ev, S = np.linalg.eigh(T)
    theta = float(ev[-1])
    return theta, theta + beta * abs(float(S[-1, -1]))
