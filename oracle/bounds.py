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

Pinned by: closed-form intervals of the Dirichlet grid Laplacians and dense
eigenvalues of small random SPD matrices (tests/test_oracle_bounds.py).
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
