"""GPU parity of Alg. 2 with its adaptive degree (ld_apply_log_adaptive) against the oracle.

The stopping test compares |d_m| ||w_m||_2 with tol.  The two sides compute
||w_m|| from different roundings of the same vectors, so every tolerance used
here is first checked to sit well away (relative margin 1e-3 on the oracle's
sequence) from every e_m a column passes before it stops; then the degrees
must agree exactly.
"""
import math

import numpy as np
import pytest

import workloads as w
from oracle import exact, newton
from tests.gpu_common import assert_cols_close, golden, random_spd_csr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2603_02207_amd as ld  # noqa: E402

DEV = "cuda:0"


def to_gpu(csr, dtype):
    row_ptr, col_idx, val, n = csr
    vals = np.asarray(val, dtype=np.float32 if dtype == torch.float32 else np.float64)
    return ld.CSR.from_arrays(row_ptr, col_idx, vals, n, device=DEV, dtype=dtype), vals.astype(np.float64)


def e_sequence(plan, Q, V):
    """e[m, col] = |d_m| ||w_m|| of the forward recurrence, m = 0..degree (oracle arithmetic)."""
    W = np.array(V, dtype=np.float64, copy=True)
    e = np.empty((plan.degree + 1, V.shape[1]))
    e[0] = abs(plan.d[0]) * np.linalg.norm(W, axis=0)
    for j in range(plan.degree):
        W = plan.alpha * (Q @ W) - plan.beta[j] * W
        e[j + 1] = abs(plan.d[j + 1]) * np.linalg.norm(W, axis=0)
    return e


def clear_of_ties(e, tol, margin=1e-3):
    """True when no column meets an e_m within `margin` (relative) of tol up to where it stops."""
    for c in range(e.shape[1]):
        for m in range(e.shape[0]):
            if abs(e[m, c] / tol - 1.0) < margin:
                return False
            if e[m, c] <= tol:
                break
    return True


@pytest.mark.parametrize("dtype,vtol", [(torch.float64, 1e-11), (torch.float32, 2e-5)])
def test_adaptive_dirichlet_eigenvectors_full_size(dtype, vtol):
    # 1024 x 1024 grid: w_m = pi_m(t) v, so each column's stopping degree and
    # value follow from the closed-form eigenvalue alone.
    N, k2, M = 1024, 0.1, 120
    A, _ = to_gpu(w.grid_laplacian_2d(N, k2), dtype)
    plan = newton.NewtonPlan(k2, k2 + 8.0, M)
    modes = [(1, 1), (3, 700), (300, 40), (512, 200), (1000, 1024)]
    V = np.stack([w.dirichlet_sine_vector_2d(N, a, b) for a, b in modes], axis=1)
    Vd = torch.tensor(V, dtype=dtype, device=DEV)
    Vin = Vd.double().cpu().numpy()
    lam = np.array([exact.grid_eigenvalue_2d(N, k2, a, b) for a, b in modes])
    t = (lam / plan.sigma - plan.c) / plan.gamma
    e = np.empty((M + 1, len(modes)))
    pi = np.ones_like(t)
    for m in range(M + 1):
        e[m] = np.abs(plan.d[m]) * np.abs(pi) * np.linalg.norm(Vin, axis=0)
        if m < M:
            pi = pi * (t - plan.xi[m])
    seen = set()
    for tol in (1e-2, 3e-5, 1e-8):
        assert clear_of_ties(e, tol)
        want = [next((m for m in range(M + 1) if e[m, c] <= tol), M) for c in range(len(modes))]
        out, deg = ld.apply_log_adaptive(A, k2, k2 + 8.0, M, tol, Vd)
        assert deg.tolist() == want, (tol, deg.tolist(), want)
        seen.update(want)
        out = out.double().cpu().numpy()
        for c in range(len(modes)):
            val = plan.d[0] if want[c] == 0 else newton.NewtonPlan(k2, k2 + 8.0, want[c]).eval_scalar(lam[c])
            ref = (val + math.log(plan.sigma)) * Vin[:, c]
            assert_cols_close(out[:, c], ref, vtol)
    assert len(seen) >= 4   # the columns stop at many different degrees


@pytest.mark.parametrize("dtype,vtol", [(torch.float64, 1e-11), (torch.float32, 3e-5)])
@pytest.mark.parametrize("ncols", [5, 70])
def test_adaptive_matches_oracle_irregular(dtype, vtol, ncols):
    # random diagonally dominant SPD matrix with near-dense rows (long-row path);
    # 70 columns run as two chunks of at most 64
    csr = random_spd_csr(3000, 11, long_rows=3)
    A, vals = to_gpu(csr, dtype)
    Q = w.to_scipy((csr[0], csr[1], vals, csr[3]))
    lo, hi = 0.5, 1.02 * float(np.abs(Q).sum(axis=1).max())
    M = 60
    plan = newton.NewtonPlan(lo, hi, M)
    rng = np.random.default_rng(ncols)
    V = rng.standard_normal((csr[3], ncols)) * rng.uniform(0.1, 10.0, ncols)
    Vd = torch.tensor(V, dtype=dtype, device=DEV)
    Vin = Vd.double().cpu().numpy()
    e = e_sequence(plan, Q, Vin)
    used = 0
    for tol in np.geomspace(1e-1, 1e-9, 17):
        if not clear_of_ties(e, tol):
            continue
        out, deg = ld.apply_log_adaptive(A, lo, hi, M, float(tol), Vd)
        ref, rdeg = newton.apply_log_adaptive(Q, Vin, lo, hi, M, float(tol))
        np.testing.assert_array_equal(deg, rdeg)
        assert_cols_close(out.double().cpu().numpy(), ref, vtol)
        used += 1
        if used == 4:
            break
    assert used >= 3


def test_adaptive_limits_and_errors():
    csr = w.grid_laplacian_2d(40, 0.5)
    A, vals = to_gpu(csr, torch.float64)
    V = torch.tensor(np.random.default_rng(2).standard_normal((1600, 6)), device=DEV)
    # tol = 0: every column runs to the cap, i.e. the fixed-degree interpolant
    out, deg = ld.apply_log_adaptive(A, 0.5, 8.5, 30, 0.0, V)
    assert (deg == 30).all()
    fixed = ld.apply_log(A, 0.5, 8.5, 30, V)
    torch.testing.assert_close(out, fixed, rtol=1e-12, atol=1e-12)
    # tol above every |d_0| ||v||: no product at all
    out, deg = ld.apply_log_adaptive(A, 0.5, 8.5, 30, 1e30, V)
    assert (deg == 0).all()
    plan = newton.NewtonPlan(0.5, 8.5, 30)
    # d_0 from Alg. 1 (library) and from the exact recursion (oracle) agree to ~1e-14
    torch.testing.assert_close(out, (plan.d[0] + math.log(plan.sigma)) * V, rtol=1e-13, atol=1e-13)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(ld.NativeError):
            ld.apply_log_adaptive(A, 0.5, 8.5, 30, bad, V)
    out, deg = ld.apply_log_adaptive(A, 0.5, 8.5, 30, 1e-6, V[:, :0])
    assert out.shape == (1600, 0) and deg.shape == (0,)


# ---- Alg. 3 with Alg. 2's stopping rule (ld_logdet_estimate_adaptive) ----------

def estimator_margins_ok(plan, Q, parts, tol, margin=1e-3):
    """clear_of_ties for the columns of S, Q_b and U the oracle's estimate used."""
    return all(clear_of_ties(e_sequence(plan, Q, parts[key]), tol, margin) for key in ("S", "A", "U"))


@pytest.mark.parametrize("dtype,rtol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
@pytest.mark.parametrize("case", ["grid", "irregular", "blocks", "gaussian"])
def test_adaptive_estimate_against_oracle(case, dtype, rtol):
    # same probes, same stopping rule: identical per-column degrees and the
    # oracle's estimate; "blocks" forces 4-column blocks (several sketch and
    # quadratic-form blocks, a ragged last one), "irregular" has near-dense rows
    if case == "irregular":
        csr = random_spd_csr(3000, 17, long_rows=3)
    else:
        csr = w.grid_laplacian_2d(48, 0.3)
    A, vals = to_gpu(csr, dtype)
    Q = w.to_scipy((csr[0], csr[1], vals, csr[3]))
    lo = 0.3 if case != "irregular" else 0.5
    hi = 1.02 * float(np.abs(Q).sum(axis=1).max())
    M, m_vec, seed = 70, 31, 4
    probes = "gaussian" if case == "gaussian" else "rademacher"
    opts = ld.Options(block_cols=4 if case == "blocks" else 0,
                      probe_dist=1 if case == "gaussian" else 0)   # 1: Gaussian, 0: Rademacher
    used = 0
    for tol in np.geomspace(1e-1, 1e-9, 9) * math.sqrt(csr[3]):
        parts = hutchpp_adaptive(Q, lo, hi, M, float(tol), m_vec, seed, probes)
        if not estimator_margins_ok(parts["plan"], Q, parts, float(tol)):
            continue
        est, deg = ld.logdet_adaptive(A, lo, hi, M, float(tol), m_vec, seed, options=opts)
        np.testing.assert_array_equal(deg, parts["degrees"])
        assert abs(est - parts["logdet"]) <= rtol * abs(parts["logdet"]), (tol, est, parts["logdet"])
        used += 1
        if used == 3:
            break
    assert used >= 2


def hutchpp_adaptive(Q, lo, hi, M, tol, m_vec, seed, probes):
    from oracle import hutchpp
    return hutchpp.logdet_estimate_adaptive(Q, lo, hi, M, tol, m_vec, seed, probes=probes, return_parts=True)


def test_adaptive_estimate_special_cases():
    csr = w.grid_laplacian_2d(30, 0.5)
    A, _ = to_gpu(csr, torch.float64)
    # tol = 0: every application runs to the cap (the fixed degree, forward form)
    est, deg = ld.logdet_adaptive(A, 0.5, 8.5, 40, 0.0, 30, 2)
    assert (deg == 40).all()
    fixed = ld.logdet(A, 0.5, 8.5, 40, 30, 2)
    assert abs(est - fixed) <= 1e-11 * abs(fixed)
    # tol above every |d_0| ||x||: no products, F = d_0 I
    est, deg, st = ld.logdet_adaptive(A, 0.5, 8.5, 40, 1e30, 30, 2, return_stats=True)
    assert (deg == 0).all() and st["launches1"] == 0 and st["launches23"] == 0
    from oracle import hutchpp
    Q = w.to_scipy(csr)
    ref, rdeg = hutchpp.logdet_estimate_adaptive(Q, 0.5, 8.5, 40, 1e30, 30, 2)
    assert abs(est - ref) <= 1e-12 * abs(ref)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(ld.NativeError):
            ld.logdet_adaptive(A, 0.5, 8.5, 40, bad, 30, 2)
    with pytest.raises(ld.NativeError):
        ld.logdet_adaptive(A, 0.5, 8.5, 40, 1e-6, 2, 2)      # n_matvec < 3


@pytest.mark.parametrize("dtype,rtol", [(torch.float64, 1e-10), (torch.float32, 1e-6)])
def test_adaptive_estimate_gmrf2048_full_size(dtype, rtol):
    # the 2048^2 GMRF (cap 100, 32 queries) against the stored oracle run, whose
    # stopping decisions all sit at least 1e-3 (relative) away from tol
    g = golden("gmrf2048_adaptive")
    if g is None:
        pytest.skip("no stored value")
    assert g["stop_margin"] > 1e-3
    A, _ = to_gpu(w.build("gmrf2048"), dtype)
    est, deg = ld.logdet_adaptive(A, g["lmin"], g["lmax"], g["max_degree"], g["tol"], g["m_vec"], g["seed"])
    np.testing.assert_array_equal(deg, g["degrees"])
    assert abs(est - g["logdet"]) <= rtol * abs(g["logdet"])
