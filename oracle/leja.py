"""Real fast Léja points on [-2, 2] (oracle side).

The paper interpolates log at Léja points generated once on the fixed
interval [-2, 2] (Sec. 3.1) and mapped to the spectral interval.  Léja points
are defined greedily (Sec. 3, Eq. Léja5): xi_0 is an end point (the paper
starts from the right end, lambda_max, i.e. +2 here) and each next point
maximises the product of distances to all earlier points over the interval.
The paper computes them with the *fast* Léja algorithm of Baglama, Calvetti
and Reichel (1998), which searches that maximum only over the midpoints of
adjacent points already chosen.

This oracle does exactly that, by brute force:
  * xi_0 = +2, xi_1 = -2 (the maximiser of |x - 2| on [-2, 2]);
  * for j >= 2 the candidates are the midpoints of adjacent chosen points
    (sorted), and xi_j is the candidate with the largest product
    prod_{k<j} |x - xi_k|, each product formed in FP64 in index order k;
  * products equal to within a relative 1e-12 are a tie, broken towards the
    larger x (a reading: the paper states no tie rule).
All points are dyadic rationals, hence exact in FP64.

Pinned by: the Léja extremal property against a dense search of the
continuous maximum (Eq. Léja5) for the first points, exactness of the first
points fixed by symmetry, nestedness, the capacity limit
(prod |xi_j - xi_k|)^(1/j) -> 1 = capacity of [-2, 2]
(tests/test_oracle_leja.py).
"""
from __future__ import annotations

import numpy as np

TIE_RTOL = 1e-12


def leja_product(x: float, pts) -> float:
    """prod_k |x - pts[k]| in FP64, in the order given."""
    p = 1.0
    for q in pts:
        p *= abs(x - q)
    return p


def _pick(cands, prods):
    """Index of the winning candidate: the largest product, ties (relative
    TIE_RTOL) broken towards the larger x."""
    pmax = max(prods)
    best = None
    for i, (x, p) in enumerate(zip(cands, prods)):
        if p >= pmax * (1.0 - TIE_RTOL) and (best is None or x > cands[best]):
            best = i
    return best


def fast_leja(count: int) -> np.ndarray:
    """First ``count`` fast Léja points on [-2, 2], xi_0 = +2."""
    if count <= 0:
        return np.zeros(0)
    pts = [2.0, -2.0][:count]
    while len(pts) < count:
        s = sorted(pts)
        cands = [(s[i] + s[i + 1]) / 2.0 for i in range(len(s) - 1)]
        prods = [leja_product(x, pts) for x in cands]
        pts.append(cands[_pick(cands, prods)])
    return np.array(pts, dtype=np.float64)


def fast_leja_vectorised(count: int) -> np.ndarray:
    """Same sequence as ``fast_leja`` with the candidate products vectorised.

    Used for long tables; ``fast_leja`` is the plain reference for it.
    """
    if count <= 0:
        return np.zeros(0)
    pts = np.zeros(count)
    pts[0] = 2.0
    if count > 1:
        pts[1] = -2.0
    for j in range(2, count):
        s = np.sort(pts[:j])
        cands = 0.5 * (s[:-1] + s[1:])
        prods = np.ones_like(cands)
        for k in range(j):  # index order, as in leja_product
            prods *= np.abs(cands - pts[k])
        pts[j] = cands[_pick(list(cands), list(prods))]
    return pts
