"""Divided differences of log at mapped Léja points (oracle side).

Notation (Sec. 3.1, Eqs. z_mapping, eq_centre, eq_gamma): the spectral
interval [lo, hi] of the scaled matrix Q~ is the image of [-2, 2] under
z = c + gamma*xi with c = (lo+hi)/2 and gamma = (hi-lo)/4.  The Newton
coefficients used by the recurrence are the divided differences of
g(xi) = log(c + gamma*xi) at the Léja points xi_0..xi_m, i.e.

    d_j = g[xi_0, ..., xi_j] = gamma^j * log[z_0, ..., z_j].

These are what the paper's Alg. 1 returns: with the lower bidiagonal Léja
matrix Q^_m of Eq. eq_leja_matrix (xi on the diagonal, ones below) and
Q_m = c*I + gamma*Q^_m, the first column of log(Q_m) holds exactly these
divided differences.  (Reading: Alg. 1 step 5 has the "+" sign; the "-" in
the text just before Eq. eq_leja_matrix is taken as a misprint, and so is the
"/2" for gamma in Alg. 1/2 step 3 against Eq. eq_gamma.)

Three independent computations:

* ``exact_dd``    -- the plain definition: the divided-difference recursion
  of Eq. Léja7 carried out in high-precision decimal arithmetic (mpmath), then
  rounded to FP64.  This is the oracle's value.
* ``alg1_dd``     -- the paper's Alg. 1 in FP64: log(Q_m)e_1 =
  (log(s)I + sum_{k=1}^p (-1)^{k+1} W^k/k) e_1 with W = (Q_m - sI)/s, the
  Taylor order p chosen adaptively (reading: stop once the largest term is
  below 2^-60 of the largest accumulated entry, after at least 10 terms).
  The scaling value s is the centre c (the Lemma of Sec. 3.1) or lambda_max/2.
* ``integral_dd`` -- from log z = int_0^inf (1/(1+t) - 1/(z+t)) dt, whose
  j-th divided difference (j >= 1) is (-1)^(j+1) int_0^inf dt/prod_i (z_i+t);
  evaluated by the trapezoid rule in u = ln t in log-space (no cancellation).

``homogeneous_dd`` gives the divided differences of xi^q (complete homogeneous
symmetric polynomials), used to pin the recurrence by polynomial exactness.

Pinned by: agreement of the three computations (tests/test_oracle_divdiff.py),
closed forms d_0 = log(hi) at xi_0 = 2 and d_1, the interpolation property
P_m(xi_i) = g(xi_i), and the Lemma's optimal scaling value.
"""
from __future__ import annotations

import math

import mpmath
import numpy as np


def interval_map(lo: float, hi: float):
    """(c, gamma) of Eqs. eq_centre and eq_gamma, in FP64."""
    c = (lo + hi) / 2.0
    gamma = (hi - lo) / 4.0
    return c, gamma


def exact_dd(lo: float, hi: float, xi, dps: int | None = None) -> np.ndarray:
    """d_j = g[xi_0..xi_j], g(xi) = log(c + gamma*xi), by Eq. Léja7 in high precision."""
    xi = [float(x) for x in xi]
    m1 = len(xi)
    if dps is None:
        dps = max(120, 4 * m1 + 60)
    c, gamma = interval_map(lo, hi)
    with mpmath.workdps(dps):
        X = [mpmath.mpf(x) for x in xi]
        C, G = mpmath.mpf(c), mpmath.mpf(gamma)
        # table[j] holds g[xi_j .. xi_{j+level}] for the current level
        table = [mpmath.log(C + G * x) for x in X]
        out = [table[0]]
        for level in range(1, m1):
            table = [(table[j + 1] - table[j]) / (X[j + level] - X[j]) for j in range(m1 - level)]
            out.append(table[0])
        return np.array([float(v) for v in out], dtype=np.float64)


def scaling_value(lo: float, hi: float, mode: str = "center") -> float:
    """s_val of Sec. 3.1: the centre c (optimal, Lemma) or lambda_max/2."""
    if mode == "center":
        return (lo + hi) / 2.0
    if mode == "half_lmax":
        return hi / 2.0
    raise ValueError(mode)


def alg1_dd(lo: float, hi: float, xi, s_mode: str = "center", taylor_cap: int = 10**8,
            rel_stop: float = 2.0**-60):
    """The paper's Alg. 1 in FP64; returns (d, p) with p the Taylor order used."""
    xi = np.asarray(xi, dtype=np.float64)
    c, gamma = interval_map(lo, hi)
    s = scaling_value(lo, hi, s_mode)
    diag = (c + gamma * xi - s) / s          # diagonal of W = (Q_m - sI)/s
    sub = gamma / s                          # sub-diagonal of W
    v = np.zeros_like(xi)
    v[0] = 1.0                               # e_1
    acc = np.zeros_like(xi)
    acc[0] = math.log(s)
    p = 0
    for k in range(1, taylor_cap + 1):
        w = diag * v
        w[1:] += sub * v[:-1]
        v = w
        term = v * (((-1.0) ** (k + 1)) / k)
        acc += term
        p = k
        if k > 10 and np.max(np.abs(term)) <= rel_stop * np.max(np.abs(acc)):
            break
    return acc, p


def integral_dd(lo: float, hi: float, xi, h: float = 0.02) -> np.ndarray:
    """Divided differences from the integral representation of log (independent pin)."""
    xi = np.asarray(xi, dtype=np.float64)
    c, gamma = interval_map(lo, hi)
    z = c + gamma * xi
    m1 = len(z)
    out = np.empty(m1)
    out[0] = math.log(z[0])
    u = np.arange(math.log(z.min()) - 45.0, math.log(z.max()) + 60.0, h)
    t = np.exp(u)
    # log of prod_{i<=j} (z_i + t), cumulative over j
    cum = np.cumsum(np.log(z[None, :] + t[:, None]), axis=1)
    for j in range(1, m1):
        a = u - cum[:, j]                    # log of the integrand in u (dt = t du)
        amax = a.max()
        logint = amax + math.log(h * np.sum(np.exp(a - amax)))
        logd = logint + j * math.log(gamma)
        out[j] = (-1.0) ** (j + 1) * math.exp(logd) if logd < 700 else math.inf
    return out


def homogeneous_dd(xi, q: int) -> np.ndarray:
    """Divided differences of x^q at xi_0..xi_j: h_{q-j}(xi_0..xi_j) (0 for j > q)."""
    xi = [mpmath.mpf(float(x)) for x in xi]
    m1 = len(xi)
    out = np.zeros(m1)
    with mpmath.workdps(60):
        for j in range(min(m1, q + 1)):
            # h_r(x_0..x_j) by the recursion h_r(x_0..x_j) = h_r(x_0..x_{j-1}) + x_j h_{r-1}(x_0..x_j)
            r = q - j
            h = [mpmath.mpf(1)] + [mpmath.mpf(0)] * r      # over x_0 only: h_t = x_0^t
            for t in range(1, r + 1):
                h[t] = xi[0] ** t
            for i in range(1, j + 1):
                for t in range(1, r + 1):
                    h[t] = h[t] + xi[i] * h[t - 1]
            out[j] = float(h[r])
    return out
