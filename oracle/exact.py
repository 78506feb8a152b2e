"""Exact log-determinants used as references (oracle side).

* Closed forms for the shifted Dirichlet grid Laplacians tau*(kappa2*I + L):
  the 5-point (7-point) Laplacian on an N^d grid has eigenvalues
  sum_axes 4 sin^2(pi a/(2(N+1))), a = 1..N per axis, so
  log det = sum log(tau*(kappa2 + sum_axes 4 sin^2(...))).
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


def grid_logdet_2d_dkappa(N: int, kappa2: float, tau: float = 1.0) -> float:
    """d/dkappa of log det tau*(kappa^2 I + L) = sum 2 kappa/(kappa^2 + mu)."""
    mu = grid_eigenvalues_2d(N, kappa2, 1.0) - kappa2
    kappa = math.sqrt(kappa2)
    return math.fsum((2.0 * kappa / (kappa2 + mu)).tolist())


def cholesky_logdet(Q_dense) -> float:
    L = np.linalg.cholesky(np.asarray(Q_dense, dtype=np.float64))
    return 2.0 * math.fsum(np.log(np.diag(L)).tolist())
