"""Helpers shared by the GPU tests (inputs only; no arithmetic of the method)."""
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def golden(name):
    path = os.path.join(HERE, "golden", f"{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def random_spd_csr(n, seed, density=0.02, long_rows=0, shift=0.5):
    """Seeded sparse SPD matrix (symmetric, diagonally dominant) with ragged rows.

    ``long_rows`` rows are made dense-ish to exercise long-row handling.
    """
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    B = sp.random(n, n, density=density, random_state=rng, data_rvs=lambda k: rng.uniform(-1, 1, k))
    B = sp.triu(B, 1)
    if long_rows:
        rows = rng.choice(n, size=long_rows, replace=False)
        extra = sp.coo_matrix((rng.uniform(-0.2, 0.2, long_rows * (n // 2)),
                               (np.repeat(rows, n // 2), rng.integers(0, n, long_rows * (n // 2)))),
                              shape=(n, n))
        B = B + sp.triu(extra, 1)
    S = (B + B.T).tocsr()
    S.sum_duplicates()
    radius = np.asarray(abs(S).sum(axis=1)).ravel()
    Q = (S + sp.diags(radius + shift + rng.uniform(0, 1, n))).tocsr()
    Q.sort_indices()
    return (Q.indptr.astype(np.int32), Q.indices.astype(np.int32), Q.data.astype(np.float64), n)


def nine_point_grid(N, seed):
    """Seeded SPD 9-point stencil on an N x N grid (row-major points).

    Random symmetric weights on the eight neighbours (varying values, so the
    diagonal storage keeps them), diagonal = sum of the row's |weights| + 0.5.
    """
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    n = N * N
    idx = np.arange(n)
    i, j = idx // N, idx % N
    rows, cols, vals = [], [], []
    for di, dj in ((0, 1), (1, -1), (1, 0), (1, 1)):   # one of each mirrored pair
        ii, jj = i + di, j + dj
        ok = (ii >= 0) & (ii < N) & (jj >= 0) & (jj < N)
        wgt = -rng.uniform(0.2, 1.0, int(ok.sum()))
        rows += [idx[ok], (ii * N + jj)[ok]]
        cols += [(ii * N + jj)[ok], idx[ok]]
        vals += [wgt, wgt]
    B = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    radius = np.asarray(abs(B).sum(axis=1)).ravel()
    Q = (B + sp.diags(radius + 0.5)).tocsr()
    Q.sort_indices()
    return (Q.indptr.astype(np.int32), Q.indices.astype(np.int32), Q.data.astype(np.float64), n)



def assert_cols_close(out, ref, tol):
    """Element by element: |out - ref| <= tol * max|ref[:, c]| for every entry of
    every column c (a 1-D array is one column)."""
    out = np.asarray(out, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert out.shape == ref.shape, (out.shape, ref.shape)
    if ref.ndim == 1:
        out, ref = out[:, None], ref[:, None]
    scale = np.abs(ref).max(axis=0)
    err = np.abs(out - ref) / np.where(scale > 0, scale, 1.0)
    worst = float(err.max()) if err.size else 0.0
    where = np.unravel_index(int(err.argmax()), err.shape) if err.size else None
    assert worst <= tol, f"largest element error {worst:.3e} (tolerance {tol:.1e}) at row, column {where}"
