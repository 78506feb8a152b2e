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
