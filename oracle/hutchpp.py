"""Léja + Hutch++ log-determinant estimator, Alg. 3 (oracle side, FP64).

Steps (Sec. 4.1, Alg. 3), with F = P_m(Q~) the Léja interpolant of log(Q~):
  1. sigma and Q~ (Eq. scaled_sigma_matrix; input lower bound, see newton.py)
  2. S in {+-1}^{n x k}, k = floor(m_vec/3), from stream 0 of the probe
     generator (Rademacher; or standard normal entries, the paper's other
     choice, with probes="gaussian")
  3. Y = F S  (Eq. eq_lejdetc_onstruction, Alg. 2 per column)
  4. A = orth(Y): Householder QR (any orthonormal basis of span(Y) gives the
     same estimate)
  5. t_low = tr(A^T F A) = sum_i a_i^T F a_i  (Eq. eq_lej_deterministic_part)
  6. G in {+-1}^{n x k_G} (or Gaussian), k_G = m_vec - 2k, from stream 1;
     u_j = (I - A A^T) g_j;  t_res = (1/k_G) sum_j u_j^T F u_j
     (Eq. eq_lej_residual_def; reading: weight 1/k_G, equal to 3/m_vec when 3
     divides m_vec, and the sum index runs over j = 1..k_G)
  7. logdet ~= n log(sigma) + t_low + t_res (Eq. eq_lejdeteq and Alg. 3 output),
     summed with math.fsum.

``logdet_estimate_adaptive`` runs the same steps with Alg. 2's stopping rule
in each application of log (every column its own degree).

``exact_trace`` is the same polynomial traced exactly (n log sigma +
sum_i P_m(lambda_i/sigma)) and isolates the interpolation error from the
Monte-Carlo error.

Pinned by: exactness when k >= n (the sketch spans everything), invariance
to the choice of orthonormal basis, unbiasedness over seeds, closed-form and
Cholesky log-determinants (tests/test_oracle_hutchpp.py); the adaptive form
by its tol = 0 and degree-0 special cases, stopping degrees from closed-form
eigenvector products, and the exact log det at k >= n
(tests/test_oracle_hutchpp_adaptive.py).
"""
from __future__ import annotations

import math

import numpy as np

from .newton import NewtonPlan
from .rng import probes as draw_probes, rademacher


def split_queries(m_vec: int):
    """(k, k_G): sketch width and residual probe count for m_vec queries."""
    if m_vec < 3:
        raise ValueError("m_vec >= 3")
    k = m_vec // 3
    return k, m_vec - 2 * k


def logdet_estimate(Q, lmin: float, lmax: float, degree: int, m_vec: int, seed: int,
                    orth=None, return_parts: bool = False, probes: str = "rademacher",
                    s_mode: str = "center", taylor_cap: int = 10**8):
    """Alg. 3 in FP64 on a scipy sparse (or dense) symmetric Q (s_mode, taylor_cap:
    Alg. 1's scaling value and Taylor cap, see NewtonPlan)."""
    n = Q.shape[0]
    plan = NewtonPlan(lmin, lmax, degree, s_mode, taylor_cap)
    k, k_g = split_queries(m_vec)
    if k > n:
        raise ValueError("sketch wider than the matrix")
    S = draw_probes(probes, seed, 0, n, k)
    G = draw_probes(probes, seed, 1, n, k_g)
    Y = plan.apply_poly(Q, S)
    if orth is None:
        A, _ = np.linalg.qr(Y)               # Householder (LAPACK geqrf/orgqr)
    else:
        A = orth(Y)
    U = G - A @ (A.T @ G)
    s_low = plan.dots(Q, A)                  # (m+1) x k
    s_res = plan.dots(Q, U)                  # (m+1) x k_G
    t_low = math.fsum(float(v) for v in (plan.d[:, None] * s_low).ravel())
    t_res = math.fsum(float(v) for v in (plan.d[:, None] * s_res).ravel()) / k_g
    est = math.fsum([n * math.log(plan.sigma), t_low, t_res])
    if return_parts:
        return dict(logdet=est, t_low=t_low, t_res=t_res, sigma=plan.sigma, lo=plan.lo,
                    hi=plan.hi, k=k, k_G=k_g, Y=Y, A=A, U=U, S=S, G=G, plan=plan)
    return est


def positive_qr(Y):
    """Thin QR basis of Y whose R has a positive diagonal (the unique one for a
    full-rank Y; any orthonormal basis differs from it by an orthogonal factor)."""
    A, R = np.linalg.qr(Y)
    sgn = np.where(np.diag(R) < 0, -1.0, 1.0)
    return A * sgn


def logdet_estimate_adaptive(Q, lmin: float, lmax: float, max_degree: int, tol: float, m_vec: int,
                             seed: int, probes: str = "rademacher", return_parts: bool = False):
    """Alg. 3 with Alg. 2's loop in its three applications of log(Q~) (steps 3,
    5 and 6): every column x gets its own degree m_x (the first m with
    |d_m| ||w_m||_2 <= tol, at most max_degree) and F x = P_{m_x}(Q~) x.

    Reading: with per-column degrees the deterministic term sum_i a_i^T F a_i
    depends on which orthonormal basis A of span(Y) step 4 takes (with one
    common degree it does not); A is the thin QR basis with a positive R
    diagonal, the one CholQR also produces.  Column signs change neither a
    column's degree nor its quadratic form.
    Returns (estimate, degrees) with degrees = [S (k), A (k), U (k_G)].
    """
    n = Q.shape[0]
    plan = NewtonPlan(lmin, lmax, max_degree)
    k, k_g = split_queries(m_vec)
    if k > n:
        raise ValueError("sketch wider than the matrix")
    S = draw_probes(probes, seed, 0, n, k)
    G = draw_probes(probes, seed, 1, n, k_g)
    Y, deg_s = plan.apply_poly_adaptive(Q, S, tol)          # step 3
    A = positive_qr(Y)                                     # step 4
    FA, deg_a = plan.apply_poly_adaptive(Q, A, tol)         # step 5
    U = G - A @ (A.T @ G)                                  # step 6
    FU, deg_u = plan.apply_poly_adaptive(Q, U, tol)
    t_low = math.fsum(float(v) for v in (A * FA).ravel())
    t_res = math.fsum(float(v) for v in (U * FU).ravel()) / k_g
    est = math.fsum([n * math.log(plan.sigma), t_low, t_res])
    degrees = np.concatenate([deg_s, deg_a, deg_u])
    if return_parts:
        return dict(logdet=est, degrees=degrees, t_low=t_low, t_res=t_res, sigma=plan.sigma, Y=Y, A=A, U=U,
                    S=S, G=G, plan=plan)
    return est, degrees


def hutchinson_estimate(Q, lmin: float, lmax: float, degree: int, m_vec: int, seed: int):
    """Plain Hutchinson (Eq. Léja8) with the same polynomial: all queries on stream 1."""
    n = Q.shape[0]
    plan = NewtonPlan(lmin, lmax, degree)
    G = rademacher(seed, 1, n, m_vec)
    s = plan.dots(Q, G)
    tr = math.fsum(float(v) for v in (plan.d[:, None] * s).ravel()) / m_vec
    return n * math.log(plan.sigma) + tr


def exact_trace(eigenvalues, lmin: float, lmax: float, degree: int):
    """n log(sigma) + tr P_m(Q~) from the eigenvalues of Q."""
    lam = np.asarray(eigenvalues, dtype=np.float64)
    plan = NewtonPlan(lmin, lmax, degree)
    vals = plan.eval_scalar(lam)
    return math.fsum([lam.size * math.log(plan.sigma)] + [float(v) for v in vals])
