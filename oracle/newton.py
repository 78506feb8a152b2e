"""Newton-Léja action of log on a block of vectors (oracle side, FP64).

Sec. 4 scales the matrix: Q~ = Q/sigma when lambda_min(Q) < 1, else Q~ = Q
(Eq. scaled_sigma_matrix), so that log det Q = n log(sigma) + tr log(Q~).
Reading: sigma is taken from the *input* lower bound, sigma = lmin if
lmin < 1 else 1, and the interval of Q~ is [lo, hi] = [lmin, lmax]/sigma.

Alg. 2 applies the Newton form (Eq. Léja6) of the interpolant of log at the
mapped Léja points z_j = c + gamma*xi_j to v, with w_0 = v, P = d_0 w_0 and
w_{j+1} = (Q~ - z_j I) w_j, P += d_{j+1} w_{j+1}.  Reading: the recurrence is
run in the mapped variable T = (Q~ - cI)/gamma, whose spectrum lies in
[-2, 2], with the xi-variable divided differences d_j = gamma^j log[z_0..z_j]:

    w_{j+1} = (T - xi_j I) w_j = alpha*Q w_j - beta_j w_j,
    alpha = 1/(sigma*gamma),  beta_j = c/gamma + xi_j.

This is the same polynomial P_m(Q~) (each factor carries 1/gamma and each
d_j carries gamma^j), but keeps ||w_j|| bounded.  The degree m is fixed
(the number of matrix products per column) everywhere except in
``apply_poly_adaptive``, which runs Alg. 2's loop: each column grows its own
degree until the last Newton term is small, |d_m| ||w_m||_2 <= tol (reading:
tol is absolute, as printed, with w_m the mapped-form vector; the loop never
goes past the largest degree the Léja points allow).

Pinned by: polynomial exactness with the divided differences of xi^q,
interpolation of log at the nodes for a diagonal matrix with the nodes as
eigenvalues, and closed-form Dirichlet-Laplacian eigenvectors
(tests/test_oracle_newton.py).
"""
from __future__ import annotations

import math

import numpy as np

from .divdiff import alg1_dd, exact_dd, interval_map
from .leja import fast_leja_vectorised


def scaling(lmin: float, lmax: float):
    """sigma and the interval [lo, hi] of Q~ (Eq. scaled_sigma_matrix)."""
    if not (0.0 < lmin < lmax):
        raise ValueError("need 0 < lmin < lmax")
    sigma = lmin if lmin < 1.0 else 1.0
    return sigma, lmin / sigma, lmax / sigma


class NewtonPlan:
    """Everything the recurrence needs for an interval and a degree.

    ``s_mode`` is the scaling value of Alg. 1 (Sec. 3.1).  With the centre
    ("center", the Lemma's optimum) Alg. 1 converges to the divided
    differences of log to FP64 accuracy, so the plan takes their plain
    definition (``exact_dd``).  With "half_lmax" (s = lambda_max/2, the
    paper's other variant) Alg. 1's Taylor series converges only like 1/p at
    xi_0 and the coefficients it returns after ``taylor_cap`` terms are not
    those divided differences: the plan then takes Alg. 1's own output
    (``alg1_dd``), which is what an estimate in that mode computes.
    """

    def __init__(self, lmin: float, lmax: float, degree: int, s_mode: str = "center",
                 taylor_cap: int = 10**8):
        if degree < 1:
            raise ValueError("degree >= 1")
        self.sigma, self.lo, self.hi = scaling(lmin, lmax)
        self.degree = degree
        self.xi = fast_leja_vectorised(degree + 1)
        if s_mode == "center":
            self.d = exact_dd(self.lo, self.hi, self.xi)
        elif s_mode == "half_lmax":
            self.d, self.taylor_terms = alg1_dd(self.lo, self.hi, self.xi, "half_lmax", taylor_cap)
        else:
            raise ValueError(s_mode)
        self.c, self.gamma = interval_map(self.lo, self.hi)
        self.alpha = 1.0 / (self.sigma * self.gamma)
        self.beta = self.c / self.gamma + self.xi[:degree]

    def apply_poly(self, Q, V):
        """P_m(Q~) V by the forward Newton recurrence (Alg. 2, mapped form)."""
        W = np.array(V, dtype=np.float64, copy=True)
        P = self.d[0] * W
        for j in range(self.degree):
            W = self.alpha * (Q @ W) - self.beta[j] * W
            P += self.d[j + 1] * W
        return P

    def apply_poly_adaptive(self, Q, V, tol: float):
        """Alg. 2 per column: (P, m) with m[c] the degree at which column c stopped.

        Column c starts with w_0 = v, P = d_0 w_0, m = 0 and, while
        |d_m| ||w_m||_2 > tol and m < degree, takes w_{m+1} = (T - xi_m) w_m,
        m += 1, P += d_m w_m.
        """
        V = np.asarray(V, dtype=np.float64)
        P = np.empty_like(V)
        ms = np.zeros(V.shape[1], dtype=np.int64)
        for c in range(V.shape[1]):
            w = V[:, c].copy()
            p = self.d[0] * w
            m = 0
            while abs(self.d[m]) * np.linalg.norm(w) > tol and m < self.degree:
                w = self.alpha * (Q @ w) - self.beta[m] * w
                m += 1
                p = p + self.d[m] * w
            P[:, c] = p
            ms[c] = m
        return P, ms

    def dots(self, Q, X):
        """s[j, col] = <X[:, col], w_j[:, col]> for j = 0..m, w_0 = X (DOT form)."""
        W = np.array(X, dtype=np.float64, copy=True)
        out = np.empty((self.degree + 1, X.shape[1]))
        out[0] = np.einsum("ij,ij->j", X, W)
        for j in range(self.degree):
            W = self.alpha * (Q @ W) - self.beta[j] * W
            out[j + 1] = np.einsum("ij,ij->j", X, W)
        return out

    def eval_scalar(self, lam):
        """P_m(lam/sigma) for eigenvalues lam of Q (Newton form, Eq. Léja6)."""
        t = (np.asarray(lam, dtype=np.float64) / self.sigma - self.c) / self.gamma
        acc = np.full_like(t, self.d[0])
        prod = np.ones_like(t)
        for j in range(self.degree):
            prod = prod * (t - self.xi[j])
            acc = acc + self.d[j + 1] * prod
        return acc


def apply_log(Q, V, lmin: float, lmax: float, degree: int, s_mode: str = "center", taylor_cap: int = 10**8):
    """log(Q) V ~= P_m(Q~) V + log(sigma) V."""
    plan = NewtonPlan(lmin, lmax, degree, s_mode, taylor_cap)
    return plan.apply_poly(Q, V) + math.log(plan.sigma) * np.asarray(V, dtype=np.float64)


def apply_log_adaptive(Q, V, lmin: float, lmax: float, max_degree: int, tol: float):
    """(log(Q) V by Alg. 2 with per-column stopping, per-column degrees); the log(sigma) V
    term of the scaling is added after the loop."""
    plan = NewtonPlan(lmin, lmax, max_degree)
    P, ms = plan.apply_poly_adaptive(Q, V, tol)
    return P + math.log(plan.sigma) * np.asarray(V, dtype=np.float64), ms
