"""Derivative of the computed Léja-Hutch++ estimate w.r.t. the stored nonzeros.

The paper does not differentiate its estimator; this is the exact derivative
of the number Alg. 3 returns, at fixed probes (S, G) and a fixed interval
(lmin, lmax, sigma), including the dependence of the sketch basis on Q.

With F = P_m(Q~) (symmetric at the base point), Y = F S = A R (QR),
Pr = A A^T, U = (I - Pr) G, c = 1/k_G:

    est = n log sigma + tr(A^T F A) + c tr(U^T F U)
    d est = tr(A^T dF A) + c tr(U^T dF U) + 2 tr(Z^T dF S),
    Z = (I - Pr) X A R^{-T},   X = F - c (F U G^T + G U^T F).

(The dA terms collect into 2 tr(A^T X dA); Q-R perturbation theory gives
dA = (I - Pr) dY R^{-1} + A*Omega with Omega skew, and A^T X A is symmetric,
so only the first part survives.)  Every term has the form tr(L^T dF R);
with the Newton form F = sum_j d_j pi_j(T), T = alpha*Q - (c/gamma)I, the
derivative of pi_j splits at each factor, giving

    d tr(L^T F R) = alpha * sum_{i=0}^{m-1} < lambda_{i+1}, dQ w_i >,
    w_0 = R, w_{i+1} = (T - xi_i) w_i              (forward Newton vectors)
    lambda_m = d_m L, lambda_i = d_i L + (T - xi_i) lambda_{i+1}   (Horner)

so the derivative w.r.t. the stored entry Q[r, col] is
alpha * sum_i sum_columns lambda_{i+1}[r, :] * w_i[col, :], one reverse sweep
over the stacked columns L = [A, sqrt(c) U, 2Z], R = [A, sqrt(c) U, S].

Pinned by: central finite differences of the oracle's own FP64 estimate
(tests/test_oracle_grad.py).  Memory: stores every w_i (small n only).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .hutchpp import logdet_estimate


def logdet_grad(csr, lmin: float, lmax: float, degree: int, m_vec: int, seed: int,
                probes: str = "rademacher"):
    """(estimate, d estimate / d val) for a CSR matrix (row_ptr, col_idx, val, n)."""
    import scipy.sparse as sp

    row_ptr, col_idx, val, n = csr
    Q = sp.csr_matrix((np.asarray(val, dtype=np.float64), col_idx, row_ptr), shape=(n, n))
    parts = logdet_estimate(Q, lmin, lmax, degree, m_vec, seed, return_parts=True, probes=probes)
    plan = parts["plan"]
    A, U, S, G, Y = parts["A"], parts["U"], parts["S"], parts["G"], parts["Y"]
    c = 1.0 / parts["k_G"]
    R = A.T @ Y                                   # Y = A R exactly (A orthonormal)
    FA = plan.apply_poly(Q, A)
    FU = plan.apply_poly(Q, U)
    XA = FA - c * (FU @ (G.T @ A) + G @ (U.T @ FA))
    PXA = XA - A @ (A.T @ XA)
    Z = sla.solve_triangular(R, PXA.T, lower=False).T   # Z^T = R^{-1} (PXA)^T
    Lm = np.hstack([A, math.sqrt(c) * U, 2.0 * Z])
    Rm = np.hstack([A, math.sqrt(c) * U, S])

    m = plan.degree
    W = [Rm]
    for j in range(m):
        W.append(plan.alpha * (Q @ W[-1]) - plan.beta[j] * W[-1])
    rows = np.repeat(np.arange(n), np.diff(np.asarray(row_ptr, dtype=np.int64)))
    cols = np.asarray(col_idx, dtype=np.int64)
    grad = np.zeros(len(cols))
    lam = plan.d[m] * Lm                          # lambda_m
    for i in range(m - 1, -1, -1):
        # contribution of factor i: alpha * <lambda_{i+1}[r], w_i[col]>
        grad += plan.alpha * np.einsum("ij,ij->i", lam[rows], W[i][cols])
        lam = plan.d[i] * Lm + plan.alpha * (Q.T @ lam) - plan.beta[i] * lam
    return parts["logdet"], grad


def fd_directional(csr, direction, lmin, lmax, degree, m_vec, seed, h, probes: str = "rademacher"):
    """Central difference of the FP64 estimate along ``direction`` over the nonzeros."""
    import scipy.sparse as sp

    row_ptr, col_idx, val, n = csr
    val = np.asarray(val, dtype=np.float64)

    def est(v):
        Q = sp.csr_matrix((v, col_idx, row_ptr), shape=(n, n))
        return logdet_estimate(Q, lmin, lmax, degree, m_vec, seed, probes=probes)

    return (est(val + h * direction) - est(val - h * direction)) / (2.0 * h)
