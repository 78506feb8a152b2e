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

``exact_trace`` is the same polynomial traced exactly (n log sigma +
sum_i P_m(lambda_i/sigma)) and isolates the interpolation error from the
Monte-Carlo error.

Pinned by: exactness when k >= n (the sketch spans everything), invariance
to the choice of orthonormal basis, unbiasedness over seeds, closed-form and
Cholesky log-determinants (tests/test_oracle_hutchpp.py).
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
