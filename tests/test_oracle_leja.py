"""Pins for the oracle's fast Léja points on [-2, 2] (Sec. 3, Eq. Léja5)."""
import math

import numpy as np

from oracle import leja


def test_first_points_fixed_by_extremal_property():
    xi = leja.fast_leja(5)
    # xi_0 = right end (lambda_max); max |x-2| on [-2,2] at -2; max 4-x^2 at 0;
    # |x|(4-x^2) is maximal at +-2/sqrt(3), the midpoint candidates +-1 tie and
    # the larger one is taken; then only -1 remains on the left side.
    assert list(xi) == [2.0, -2.0, 0.0, 1.0, -1.0]


def test_vectorised_equals_plain():
    np.testing.assert_array_equal(leja.fast_leja(160), leja.fast_leja_vectorised(160))


def test_points_distinct_dyadic_in_interval_and_nested():
    xi = leja.fast_leja_vectorised(600)
    assert np.all(np.abs(xi) <= 2.0)
    assert len(np.unique(xi)) == len(xi)
    for x in xi:
        assert (x * 2.0**60) == math.floor(x * 2.0**60)   # dyadic, exact in FP64
    np.testing.assert_array_equal(leja.fast_leja_vectorised(100), xi[:100])


def test_near_extremal_against_continuous_maximum():
    # Fast Léja restricts Eq. Léja5's maximum to midpoint candidates; the
    # chosen product must stay close to the continuous maximum.
    xi = leja.fast_leja_vectorised(65)
    xs = np.linspace(-2.0, 2.0, 200001)
    for j in range(1, 65):
        prod_c = np.ones_like(xs)
        for k in range(j):
            prod_c *= np.abs(xs - xi[k])
        pj = leja.leja_product(xi[j], xi[:j])
        assert pj <= prod_c.max() * (1 + 1e-9)
        assert pj >= 0.8 * prod_c.max()
        if j < 2:
            continue
        # and it is the best midpoint candidate (brute force)
        s = np.sort(xi[:j])
        cands = 0.5 * (s[:-1] + s[1:])
        best = max(leja.leja_product(c, xi[:j]) for c in cands)
        assert pj >= best * (1 - 1e-12)


def test_capacity_of_interval():
    # Léja points are asymptotically distributed like Chebyshev points: the
    # j-th root of the Léja product tends to the capacity of [-2,2], which is 1.
    xi = leja.fast_leja_vectorised(321)
    roots = [leja.leja_product(xi[j], xi[:j]) ** (1.0 / j) for j in (10, 40, 80, 160, 320)]
    assert all(a > b for a, b in zip(roots, roots[1:]))
    assert 1.0 < roots[-1] < 1.02
    assert roots[0] < 1.3
