"""Exact log-determinants used as references (oracle side).

* Closed forms for the shifted Dirichlet grid Laplacians tau*(kappa2*I + L):
  the 5-point (7-point) Laplacian on an N^d grid has eigenvalues
  sum_axes 4 sin^2(pi a/(2(N+1))), a = 1..N per axis, so
  log det = sum log(tau*(kappa2 + sum_axes 4 sin^2(...))).
* The GMRF precision Q(theta) = I + theta*Adj of Sec. 5.2 on the same grid
  (Adj = 4I - L) has eigenvalues 1 + theta*(4 - mu_a - mu_b), i.e.
  1 + 2 theta (cos(pi a/(N+1)) + cos(pi b/(N+1))).
* Banded Cholesky log det for the pentadiagonal matrices of Sec. 5.1 at full
  size.
* Dense Cholesky log det = 2 sum log diag(chol(Q)) for small n (the paper's
  exact reference is a Cholesky factorisation, Sec. 5).

These are definitions, not approximations; they pin the oracle's estimator.
"""
from __future__ import annotations

import math

import numpy as np


def grid_axis_eigs(N: int) -> np.ndarray:
    a = np.arange(1, N + 1)
    return 4.0 * np.sin(np.pi * a / (2.0 * (N + 1))) ** 2


def grid_eigenvalues_2d(N: int, kappa2: float, tau: float = 1.0) -> np.ndarray:
    mu = grid_axis_eigs(N)
    return (tau * (kappa2 + mu[:, None] + mu[None, :])).reshape(-1)


def grid_eigenvalues_3d(N: int, kappa2: float, tau: float = 1.0) -> np.ndarray:
    mu = grid_axis_eigs(N)
    return (tau * (kappa2 + mu[:, None, None] + mu[None, :, None] + mu[None, None, :])).reshape(-1)


def grid_eigenvalue_2d(N: int, kappa2: float, a: int, b: int, tau: float = 1.0) -> float:
    mu = grid_axis_eigs(N)
    return tau * (kappa2 + mu[a - 1] + mu[b - 1])


def grid_eigenvalue_3d(N: int, kappa2: float, a: int, b: int, c: int, tau: float = 1.0) -> float:
    mu = grid_axis_eigs(N)
    return tau * (kappa2 + mu[a - 1] + mu[b - 1] + mu[c - 1])


def grid_logdet_2d(N: int, kappa2: float, tau: float = 1.0) -> float:
    return math.fsum(np.log(grid_eigenvalues_2d(N, kappa2, tau)).tolist())


def grid_logdet_3d(N: int, kappa2: float, tau: float = 1.0) -> float:
    lam = grid_eigenvalues_3d(N, kappa2, tau)
    return math.fsum(np.log(lam).tolist())


def gmrf_theta_eigenvalues(N: int, theta: float) -> np.ndarray:
    a = np.arange(1, N + 1)
    cs = np.cos(np.pi * a / (N + 1))
    return (1.0 + 2.0 * theta * (cs[:, None] + cs[None, :])).reshape(-1)


def gmrf_theta_logdet(N: int, theta: float) -> float:
    return math.fsum(np.log(gmrf_theta_eigenvalues(N, theta)).tolist())


def grid_matfun_diag_2d(N: int, fvals: np.ndarray) -> np.ndarray:
    """Diagonal of f(Q) for any Q diagonalised by the 2-D Dirichlet sine modes.

    fvals[a-1, b-1] = f(lambda_ab).  The unit eigenvectors are separable,
    u_ab(i, j) = u_a(i) u_b(j) with u_a(i) = sqrt(2/(N+1)) sin(pi a i/(N+1)), so
    f(Q)_(i,j),(i,j) = sum_ab u_a(i)^2 u_b(j)^2 f_ab = (S f S^T)[i, j] with
    S[i, a] = u_a(i)^2.  Returned in grid (row-major) order.
    """
    a = np.arange(1, N + 1)
    S = 2.0 / (N + 1) * np.sin(np.pi * np.outer(a, a) / (N + 1)) ** 2
    return (S @ np.asarray(fvals, dtype=np.float64).reshape(N, N) @ S.T).reshape(-1)


def grid_logdet_2d_dkappa(N: int, kappa2: float, tau: float = 1.0) -> float:
    """d/dkappa of log det tau*(kappa^2 I + L) = sum 2 kappa/(kappa^2 + mu)."""
    mu = grid_eigenvalues_2d(N, kappa2, 1.0) - kappa2
    kappa = math.sqrt(kappa2)
    return math.fsum((2.0 * kappa / (kappa2 + mu)).tolist())


def banded_logdet(csr, bandwidth: int) -> float:
    """log det of a symmetric banded SPD matrix from its banded Cholesky factor.

    csr = (row_ptr, col_idx, val, n) with |i - j| <= bandwidth for every entry;
    the lower band is packed as ab[k, j] = Q[j + k, j] (LAPACK lower banded
    storage) and factored by scipy.linalg.cholesky_banded; log det is
    2 sum log diag(L), summed with math.fsum.  O(n bandwidth^2): used at the
    full size of the paper's pentadiagonal study (Sec. 5.1).
    """
    import scipy.linalg as sla

    row_ptr, col_idx, val, n = csr
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    cols = np.asarray(col_idx, dtype=np.int64)
    if np.any(np.abs(rows - cols) > bandwidth):
        raise ValueError("entry outside the band")
    low = rows >= cols
    ab = np.zeros((bandwidth + 1, n))
    ab[rows[low] - cols[low], cols[low]] = np.asarray(val, dtype=np.float64)[low]
    c = sla.cholesky_banded(ab, lower=True, overwrite_ab=True, check_finite=False)
    return 2.0 * math.fsum(np.log(c[0]).tolist())


def cholesky_logdet(Q_dense) -> float:
    L = np.linalg.cholesky(np.asarray(Q_dense, dtype=np.float64))
    return 2.0 * math.fsum(np.log(np.diag(L)).tolist())
