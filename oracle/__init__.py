"""FP64 CPU oracle for the Léja-point + Hutch++ log-determinant estimator.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
implementation of what the GPU library computes, written from the paper
("Novel technique based on Léja Points Approximation for Log-determinant
Estimation of Large matrices", arXiv 2603.02207).  Only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import it; the library
and its Python binding never do, and it shares no code with them.

Modules
-------
rng       counter-based SplitMix64 Rademacher probes (published generator)
leja      fast real Léja points on [-2, 2]                     (Sec. 3, Eq. Léja5)
divdiff   divided differences of log: exact definition (Eq. Léja7 in high
          precision), the paper's scaled Taylor matrix function (Alg. 1), and
          an integral representation used as an independent pin
newton    Newton-Léja action P_m(Q~)v (Alg. 2, mapped form)
hutchpp   Léja + Hutch++ estimator (Alg. 3) and its exact-trace mode
bounds    Gershgorin interval (Sec. 3) and Lanczos lambda_max (App. A)
exact     closed-form Dirichlet-Laplacian log-determinants, dense Cholesky
grad      derivative of the computed estimate w.r.t. the stored nonzeros

Pinning status of each function is stated in its module docstring; a function
with no independent pin says "parity unpinned".
"""
from . import rng, leja, divdiff, newton, hutchpp, bounds, exact, grad  # noqa: F401
