"""Pins for the divided differences of log (Sec. 3.1, Alg. 1, Eq. Léja7)."""
import math

import numpy as np
import pytest

from oracle import divdiff, leja
from oracle.newton import NewtonPlan

XI = leja.fast_leja_vectorised(161)
CASES = [(1.0, 17.0, 40), (1.0, 81.0, 80), (1.0, 241.0, 120), (1.0, 8.3e5, 150), (2.5, 3.0, 30)]


@pytest.mark.parametrize("lo,hi,m", CASES)
def test_exact_against_integral_representation(lo, hi, m):
    e = divdiff.exact_dd(lo, hi, XI[: m + 1])
    i = divdiff.integral_dd(lo, hi, XI[: m + 1])
    np.testing.assert_allclose(i, e, rtol=2e-11, atol=0)


@pytest.mark.parametrize("lo,hi,m", CASES[:3] + CASES[4:])
def test_alg1_reaches_exact(lo, hi, m):
    e = divdiff.exact_dd(lo, hi, XI[: m + 1])
    a, p = divdiff.alg1_dd(lo, hi, XI[: m + 1], "center")
    assert np.max(np.abs(a - e)) < 1e-13
    # Taylor order grows like log(2^-60)/log(r), r = (hi-lo)/(hi+lo)  (Lemma)
    r = (hi - lo) / (hi + lo)
    assert p < 1.2 * (60 * math.log(2) / -math.log(r)) + 20


def truncated_taylor_dd(lo, hi, xi, p, dps=80):
    """Divided differences (Eq. Léja7, high precision) of f_p(c + gamma*xi),
    f_p(z) = log s + sum_{k=1}^p (-1)^(k+1) ((z-s)/s)^k / k with s = hi/2:
    the polynomial whose value at the Léja bidiagonal matrix Alg. 1 forms after
    p Taylor terms, so that its first column holds these divided differences."""
    import mpmath

    with mpmath.workdps(dps):
        c, g = mpmath.mpf(lo + hi) / 2, mpmath.mpf(hi - lo) / 4
        s = mpmath.mpf(hi) / 2
        X = [mpmath.mpf(float(x)) for x in xi]
        vals = []
        for x in X:
            w = (c + g * x - s) / s
            acc, pw = mpmath.log(s), mpmath.mpf(1)
            for k in range(1, p + 1):
                pw *= w
                acc += (pw / k) if k % 2 else -(pw / k)
            vals.append(acc)
        out, table = [vals[0]], vals
        for level in range(1, len(X)):
            table = [(table[j + 1] - table[j]) / (X[j + level] - X[j]) for j in range(len(X) - level)]
            out.append(table[0])
        return np.array([float(v) for v in out])


@pytest.mark.parametrize("lo,hi,m,p", [(1.0, 17.0, 40, 3000), (1.0, 81.0, 24, 1500), (2.5, 3.0, 30, 500)])
def test_alg1_half_lmax_equals_truncated_taylor_divided_differences(lo, hi, m, p):
    # Sec. 3.1 with s = lambda_max/2: after p terms Alg. 1 returns the divided
    # differences of the truncated Taylor polynomial of log about s (no
    # convergence test can stop it earlier: xi_0 sits on the Taylor disc's
    # boundary), computed here independently by Eq. Léja7's recursion.
    a, terms = divdiff.alg1_dd(lo, hi, XI[: m + 1], "half_lmax", taylor_cap=p)
    assert terms == p
    ref = truncated_taylor_dd(lo, hi, XI[: m + 1], p)
    assert np.max(np.abs(a - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("p", [1, 2, 7, 100, 2001])
def test_alg1_half_lmax_first_coefficient_closed_form(p):
    # At xi_0 = 2 (z_0 = lambda_max) the Taylor variable is (z_0 - s)/s = 1, so
    # d_0 = log(s) + S_p with S_p the p-th partial sum of the alternating
    # harmonic series, S_p = log 2 + ((-1)^(p+1)/2) (psi((p+2)/2) - psi((p+1)/2)).
    import mpmath

    lo, hi = 1.0, 17.0
    a, _ = divdiff.alg1_dd(lo, hi, XI[:5], "half_lmax", taylor_cap=p)
    Sp = mpmath.log(2) + (-1) ** (p + 1) * (mpmath.digamma((p + 2) / mpmath.mpf(2))
                                            - mpmath.digamma((p + 1) / mpmath.mpf(2))) / 2
    assert a[0] == pytest.approx(math.log(hi / 2) + float(Sp), abs=1e-13)
    # and the error against log(lambda_max) decays like 1/(2p)
    if p > 50:
        assert abs(a[0] - math.log(hi)) == pytest.approx(1 / (2 * p), rel=2 / p)


def test_newton_plan_half_lmax_takes_alg1():
    plan = NewtonPlan(0.5, 8.5, 30, "half_lmax", 1000)
    a, _ = divdiff.alg1_dd(1.0, 17.0, XI[:31], "half_lmax", taylor_cap=1000)
    np.testing.assert_array_equal(plan.d, a)
    with pytest.raises(ValueError):
        NewtonPlan(0.5, 8.5, 30, "lambda_min")


def test_alg1_half_lmax_converges_slowly():
    # s = lambda_max/2 puts xi_0 = 2 on the boundary |w| = 1 of the Taylor
    # disc: the error decays only like 1/p.
    e = divdiff.exact_dd(1.0, 17.0, XI[:41])
    a, p = divdiff.alg1_dd(1.0, 17.0, XI[:41], "half_lmax", taylor_cap=2000)
    assert p == 2000
    err = np.max(np.abs(a - e))
    assert 1e-6 < err < 1e-2


def test_closed_form_first_coefficients():
    lo, hi = 1.0, 17.0
    d = divdiff.exact_dd(lo, hi, XI[:4])
    c, g = divdiff.interval_map(lo, hi)
    assert d[0] == pytest.approx(math.log(hi), rel=1e-15)       # xi_0 = 2 -> z_0 = hi
    z0, z1 = c + 2 * g, c - 2 * g
    assert d[1] == pytest.approx(g * (math.log(z1) - math.log(z0)) / (z1 - z0), rel=1e-14)


def test_precision_of_exact_recursion():
    e1 = divdiff.exact_dd(1.0, 8.3e5, XI[:151])
    e2 = divdiff.exact_dd(1.0, 8.3e5, XI[:151], dps=1200)
    np.testing.assert_array_equal(e1, e2)


@pytest.mark.parametrize("lo,hi,m", CASES)
def test_interpolation_at_nodes(lo, hi, m):
    plan = NewtonPlan(lo, hi, m)            # lmin = lo >= 1 -> sigma = 1
    z = plan.c + plan.gamma * plan.xi
    np.testing.assert_allclose(plan.eval_scalar(z), np.log(z), rtol=0, atol=5e-13 * max(1, math.log(hi)))


def test_homogeneous_dd_of_monomials():
    # Divided differences of x^q: 1 at order q, 0 above, h_{q-j} below.
    for q in range(6):
        d = divdiff.homogeneous_dd(XI[:8], q)
        assert d[q] == 1.0
        assert np.all(d[q + 1:] == 0.0)
    d = divdiff.homogeneous_dd(XI[:3], 2)    # x^2 at 2, -2, 0: [4, 0, 1]
    assert list(d) == [4.0, 0.0, 1.0]


def test_lemma_optimal_scaling():
    lo, hi = 1.0, 81.0
    s_grid = np.linspace(0.5, 100.0, 20001)
    D = np.maximum(np.abs(lo / s_grid - 1), np.abs(hi / s_grid - 1))
    s_best = s_grid[np.argmin(D)]
    assert s_best == pytest.approx(divdiff.scaling_value(lo, hi, "center"), abs=0.01)
    assert D.min() == pytest.approx((hi - lo) / (hi + lo), abs=1e-4)
