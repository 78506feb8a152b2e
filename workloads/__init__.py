"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds input data: sparse SPD matrices in CSR form and a few
structured probe vectors.  It holds none of the estimator's arithmetic (no
Léja points, divided differences, Newton recurrence, sketching or traces), so
that both the CPU oracle and the GPU path can take their inputs from here
without sharing any of the method.

Matrices stand in for the paper's workloads (Section 5): the paper measures on
SuiteSparse matrices and on synthetic pentadiagonal and 2-D GMRF precision
matrices; the grid Laplacians and the Chung-Lu graph Laplacian below are the
synthetic stand-ins with the sizes of the benchmark configurations.

Every generator returns ``(row_ptr int32[n+1], col_idx int32[nnz], val
float64[nnz], n)`` with sorted column indices inside each row.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "grid_laplacian_2d",
    "grid_laplacian_3d",
    "chung_lu_laplacian",
    "pentadiagonal",
    "gmrf_theta",
    "dirichlet_sine_vector_2d",
    "dirichlet_sine_vector_3d",
    "to_scipy",
    "CONFIGS",
]


def _assemble(n, rows, cols, vals):
    """COO (rows, cols, vals) -> CSR with sorted columns (duplicates kept separate)."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz does not fit int32 indices")
    return row_ptr.astype(np.int32), cols.astype(np.int32), vals, n


def grid_laplacian_2d(N: int, kappa2: float, tau: float = 1.0):
    """tau * (kappa2*I + L), L the 5-point Dirichlet Laplacian on an N x N grid.

    Row-major grid order (index = i*N + j).  Diagonal tau*(4+kappa2),
    off-diagonals -tau.  This is the GMRF precision of the paper's
    maximum-likelihood study (Section 5.2) with a Dirichlet boundary.
    """
    n = N * N
    idx = np.arange(n, dtype=np.int64)
    i, j = idx // N, idx % N
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, tau * (4.0 + kappa2))]
    for di, dj in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ii, jj = i + di, j + dj
        ok = (ii >= 0) & (ii < N) & (jj >= 0) & (jj < N)
        rows.append(idx[ok])
        cols.append((ii * N + jj)[ok])
        vals.append(np.full(int(ok.sum()), -tau))
    return _assemble(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def grid_laplacian_3d(N: int, kappa2: float, tau: float = 1.0):
    """tau * (kappa2*I + L3), L3 the 7-point Dirichlet Laplacian on an N^3 grid.

    Index = (i*N + j)*N + k.  Diagonal tau*(6+kappa2), off-diagonals -tau.
    """
    n = N * N * N
    idx = np.arange(n, dtype=np.int64)
    i, j, k = idx // (N * N), (idx // N) % N, idx % N
    rows = [idx]
    cols = [idx]
    vals = [np.full(n, tau * (6.0 + kappa2))]
    for d in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
        ii, jj, kk = i + d[0], j + d[1], k + d[2]
        ok = (ii >= 0) & (ii < N) & (jj >= 0) & (jj < N) & (kk >= 0) & (kk < N)
        rows.append(idx[ok])
        cols.append(((ii * N + jj) * N + kk)[ok])
        vals.append(np.full(int(ok.sum()), -tau))
    return _assemble(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def chung_lu_laplacian(n: int, seed: int = 0, beta: float = 2.5, mean_degree: float = 16.0,
                       delta: float = 1e-2, permute: bool = False):
    """Weighted graph Laplacian of a Chung-Lu power-law graph, plus delta*I.

    Expected-degree weights w_i ~ (i+1)^(-1/(beta-1)), scaled to the requested
    mean degree and capped at sqrt(n*mean_degree).  n*mean_degree/2 endpoint
    pairs are drawn i.i.d. with probability proportional to w (seeded),
    self-loops are dropped, duplicate edges merged (weights summed), and each
    edge gets a weight U(0.5, 1.5).  Rows come hubs first; ``permute`` applies
    a seeded random relabelling instead.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x5EED]))
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (beta - 1.0))
    w *= mean_degree * n / w.sum()
    np.minimum(w, np.sqrt(n * mean_degree), out=w)
    p = w / w.sum()
    m_edges = int(n * mean_degree // 2)
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    a = np.searchsorted(cdf, rng.random(m_edges), side="right")
    b = np.searchsorted(cdf, rng.random(m_edges), side="right")
    np.minimum(a, n - 1, out=a)
    np.minimum(b, n - 1, out=b)
    ew = rng.uniform(0.5, 1.5, size=m_edges)
    keep = a != b
    a, b, ew = a[keep], b[keep], ew[keep]
    lo_, hi_ = np.minimum(a, b).astype(np.int64), np.maximum(a, b).astype(np.int64)
    key = lo_ * n + hi_
    uniq, inv = np.unique(key, return_inverse=True)
    wsum = np.bincount(inv, weights=ew)
    u, v = uniq // n, uniq % n
    if permute:
        perm = rng.permutation(n)
        u, v = perm[u], perm[v]
    deg = np.bincount(u, weights=wsum, minlength=n) + np.bincount(v, weights=wsum, minlength=n)
    idx = np.arange(n, dtype=np.int64)
    rows = np.concatenate([idx, u, v])
    cols = np.concatenate([idx, v, u])
    vals = np.concatenate([deg + delta, -wsum, -wsum])
    return _assemble(n, rows, cols, vals)


def gmrf_theta(N: int, theta: float):
    """Q(theta) = I + theta * Adj on an N x N grid, Adj the 4-nearest-neighbour adjacency.

    The GMRF precision of the paper's maximum-likelihood study (Sec. 5.2):
    unit diagonal, theta on the four neighbours; Dirichlet boundary (a border
    node has fewer neighbours).  Its spectrum lies in [1 - 4|theta|, 1 + 4|theta|].
    Same pattern and order as ``grid_laplacian_2d``; since L = 4I - Adj this is
    (1 + 4 theta) I - theta L.
    """
    row_ptr, col_idx, _, n = grid_laplacian_2d(N, 0.0)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    val = np.where(col_idx == rows, 1.0, float(theta))
    return row_ptr, col_idx, val, n


def pentadiagonal(n: int, seed: int = 0):
    """Symmetric pentadiagonal SPD matrix of the paper's synthetic study (Section 5.1).

    Five diagonals (offsets 0, +-1, +-2) filled with U(0,1) entries, the matrix
    symmetrised (Q + Q^T) and shifted by n*I.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x9E7A]))
    d0, d1, d2 = rng.random(n), rng.random(n - 1), rng.random(n - 2)
    dm1, dm2 = rng.random(n - 1), rng.random(n - 2)
    idx = np.arange(n, dtype=np.int64)
    rows = [idx, idx[:-1], idx[:-2], idx[1:], idx[2:]]
    cols = [idx, idx[1:], idx[2:], idx[:-1], idx[:-2]]
    # (Q + Q^T): upper entry (i, i+k) = u_k[i] + l_k[i], mirrored below.
    s1, s2 = d1 + dm1, d2 + dm2
    vals = [2.0 * d0 + n, s1, s2, s1, s2]
    return _assemble(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def dirichlet_sine_vector_2d(N: int, a: int, b: int):
    """Eigenvector (a, b) of the 5-point Dirichlet Laplacian, 1 <= a, b <= N.

    v[i*N + j] = sin(pi*a*(i+1)/(N+1)) * sin(pi*b*(j+1)/(N+1)).
    """
    s_a = np.sin(np.pi * a * np.arange(1, N + 1) / (N + 1))
    s_b = np.sin(np.pi * b * np.arange(1, N + 1) / (N + 1))
    return np.outer(s_a, s_b).reshape(-1)


def dirichlet_sine_vector_3d(N: int, a: int, b: int, c: int):
    """Eigenvector (a, b, c) of the 7-point Dirichlet Laplacian on an N^3 grid."""
    t = np.arange(1, N + 1) / (N + 1)
    s_a, s_b, s_c = (np.sin(np.pi * q * t) for q in (a, b, c))
    return np.einsum("i,j,k->ijk", s_a, s_b, s_c).reshape(-1)


def to_scipy(csr):
    """(row_ptr, col_idx, val, n) -> scipy.sparse.csr_matrix (float64)."""
    import scipy.sparse as sp

    row_ptr, col_idx, val, n = csr
    return sp.csr_matrix((np.asarray(val, dtype=np.float64), col_idx, row_ptr), shape=(n, n))


# Benchmark and parity workloads: (generator, kwargs, Gershgorin interval,
# degree, number of matrix-vector queries m_vec).
CONFIGS = {
    "grid32_k0.5": dict(kind="grid2d", N=32, kappa2=0.5, degree=40, m_vec=30),
    "grid1024_k0.1": dict(kind="grid2d", N=1024, kappa2=0.1, degree=80, m_vec=60),
    "grid128c_k0.05": dict(kind="grid3d", N=128, kappa2=0.05, degree=120, m_vec=96),
    "chunglu_4M": dict(kind="chunglu", n=1 << 22, degree=150, m_vec=64),
    "gmrf2048": dict(kind="grid2d", N=2048, kappa2=0.1, tau=1.5, degree=100, m_vec=32),
    # Sec. 5.2's GMRF, I + theta*Adj on 5000 x 5000 at the hidden theta = -0.22
    # (spectrum [0.12, 1.88]); the sweep over theta uses the same pattern
    "gmrf5000_theta": dict(kind="gmrf_theta", N=5000, theta=-0.22, degree=80, m_vec=30),
    # Sec. 5.1's pentadiagonal matrices at their largest size; the spectrum sits in
    # [n - 8, n + 10], so a low degree already interpolates log to rounding level
    "penta_1e7": dict(kind="penta", n=10_000_000, degree=8, m_vec=30),
}

# the theta values of the likelihood sweep over the paper's range [-0.25, 0]
GMRF_THETAS = (-0.24, -0.22, -0.2, -0.16, -0.12, -0.08, -0.04)


def build(name: str, **override):
    """Build the matrix of a named workload (``CONFIGS``); keyword overrides allowed."""
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    kind = cfg["kind"]
    if kind == "grid2d":
        return grid_laplacian_2d(cfg["N"], cfg["kappa2"], cfg.get("tau", 1.0))
    if kind == "grid3d":
        return grid_laplacian_3d(cfg["N"], cfg["kappa2"], cfg.get("tau", 1.0))
    if kind == "chunglu":
        return chung_lu_laplacian(cfg["n"], seed=cfg.get("seed", 0), permute=cfg.get("permute", False))
    if kind == "penta":
        return pentadiagonal(cfg["n"], seed=cfg.get("seed", 0))
    if kind == "gmrf_theta":
        return gmrf_theta(cfg["N"], cfg["theta"])
    raise ValueError(kind)
