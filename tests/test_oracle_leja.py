"""Pins for the oracle's fast Léja points on [-2, 2] (Sec. 3, Eq. Léja5)."""
import math
from fractions import Fraction

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


def test_first_sixteen_points():
    # The first points worked by hand from Eq. Léja5 over midpoint candidates:
    # after 2, -2, 0 the product |x| |4 - x^2| ties at +-1 (larger x first);
    # after {2, -2, 0, 1, -1} the product |x| |4 - x^2| |x^2 - 1| is even and
    # ties at +-1.5 (3.28125) above +-0.5 (1.40625); on the symmetric set
    # {0, +-1, +-1.5, +-2} the best midpoints are +-0.5 (2.8125 against
    # 2.3262 at +-1.75), and so on; the later entries follow from the same
    # rule in exact arithmetic (next test).
    want = [2, -2, 0, 1, -1, 1.5, -1.5, 0.5, -1.75, 1.75, -0.5, 1.875, -1.875, 1.25, -1.25, 0.25]
    assert list(leja.fast_leja(16)) == want
    assert list(leja.fast_leja_vectorised(16)) == want


def test_exact_arithmetic_brute_force():
    # The same greedy rule in exact rational arithmetic: every candidate
    # product is exact, ties are exact equalities (broken towards the larger
    # x), so the FP64 products and the relative tie tolerance of the oracle
    # must reproduce this sequence.
    pts = [Fraction(2), Fraction(-2)]
    while len(pts) < 96:
        srt = sorted(pts)
        cands = [(a + b) / 2 for a, b in zip(srt, srt[1:])]
        best = None
        for x in cands:
            prod = Fraction(1)
            for q in pts:
                prod *= abs(x - q)
            if best is None or prod > best[0] or (prod == best[0] and x > best[1]):
                best = (prod, x)
        pts.append(best[1])
    np.testing.assert_array_equal(leja.fast_leja_vectorised(96), np.array([float(x) for x in pts]))
