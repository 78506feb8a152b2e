"""The GMRF of the paper's maximum-likelihood study, Q(theta) = I + theta*Adj (Sec. 5.2).

* Small grid: the HIP estimate against the oracle on identical probes.
* Full size (5000 x 5000, n = 25e6, about 1.25e8 stored entries): the sine
  eigenvectors through ld_apply_log against the closed-form P_m(lambda/sigma),
  and the estimate against its expectation n log(sigma) + sum_i P_m(lambda_i/sigma)
  within 6 standard deviations of Rademacher Hutchinson on the residual
  (stored closed-form values, tests/golden/gmrf5000_theta_sweep.json); that
  expectation equals the exact log det to about 1e-12 here.
"""
import math

import numpy as np
import pytest

import workloads as w
from oracle import bounds, exact, hutchpp, newton
from tests.gpu_common import assert_cols_close, golden

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2603_02207_amd as ld  # noqa: E402

DEV = "cuda:0"


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
@pytest.mark.parametrize("theta", [-0.22, -0.08])
def test_small_grid_against_oracle(dtype, tol, theta):
    csr = w.gmrf_theta(48, theta)
    npd = np.float32 if dtype == torch.float32 else np.float64
    vals = np.asarray(csr[2], dtype=npd)
    A = ld.CSR.from_arrays(csr[0], csr[1], vals, csr[3], device=DEV, dtype=dtype)
    csr_v = (csr[0], csr[1], vals.astype(np.float64), csr[3])
    lmin, lmax = bounds.gershgorin(csr_v)
    glo, ghi = ld.spectral_bounds(A)
    assert glo == pytest.approx(lmin, rel=1e-12) and ghi == pytest.approx(lmax, rel=1e-12)
    est = ld.logdet(A, lmin, lmax, 80, 30, 0)
    ref = hutchpp.logdet_estimate(w.to_scipy(csr_v), lmin, lmax, 80, 30, 0)
    assert abs(est - ref) / abs(ref) < tol


@pytest.fixture(scope="module")
def full_pattern():
    N = w.CONFIGS["gmrf5000_theta"]["N"]
    row_ptr, col_idx, val, n = w.gmrf_theta(N, -0.22)
    A = ld.CSR.from_arrays(row_ptr, col_idx, val.astype(np.float32), n, device=DEV, dtype=torch.float32)
    diag = torch.tensor(val == 1.0, device=DEV)
    return N, A, diag


def test_full_size_sine_modes(full_pattern):
    N, A, diag = full_pattern
    theta = -0.22
    lmin, lmax = ld.spectral_bounds(A)
    plan = newton.NewtonPlan(lmin, lmax, 80)
    modes = [(1, 1), (17, 4000), (2500, 2400), (5000, 4999)]   # away from lambda = 1 (a = N+1-b)
    V = torch.tensor(np.stack([w.dirichlet_sine_vector_2d(N, a, b) for a, b in modes], axis=1),
                     dtype=torch.float32, device=DEV)
    out = ld.apply_log(A, lmin, lmax, 80, V).double().cpu().numpy()
    Vin = V.double().cpu().numpy()
    lam = exact.gmrf_theta_eigenvalues(N, theta).reshape(N, N)
    for i, (a, b) in enumerate(modes):
        scal = float(plan.eval_scalar(lam[a - 1, b - 1])) + math.log(plan.sigma)
        ref = scal * Vin[:, i]
        assert_cols_close(out[:, i], ref, 2e-5)


@pytest.mark.parametrize("theta", [-0.22, -0.08])
def test_full_size_estimate_within_hutchinson_error(full_pattern, theta):
    N, A, diag = full_pattern
    g = golden("gmrf5000_theta_sweep")["results"][repr(theta)]
    At = A.with_values(torch.where(diag, torch.ones_like(A.val), torch.full_like(A.val, theta)))
    lmin, lmax = ld.spectral_bounds(At)
    assert lmin == pytest.approx(g["lmin"], rel=1e-6) and lmax == pytest.approx(g["lmax"], rel=1e-6)
    est = ld.logdet(At, lmin, lmax, 80, 30, 0)
    z = (est - g["expectation"]) / g["sd_hutchinson"]
    assert abs(z) < 6.0, (theta, est, g["expectation"], z)
    assert abs(g["expectation"] - g["logdet_exact"]) < 1e-9 * abs(g["logdet_exact"])


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_full_size_row_ranges_cover_every_row(full_pattern, dtype):
    # At 25e6 rows each persistent workgroup of the quadratic-form step would
    # walk about 170 tiles in FP32 (340 in FP64), so with XCD bands the step runs as several launches
    # over consecutive row ranges that add to the same partial sums; with
    # interleaved tiles it is one launch.  The recurrence vectors are per-row
    # results (the same bits in both orders) and the FP64 column sums differ
    # only in grouping, so the two estimates agree to FP64 rounding: a row
    # range skipped or taken twice would move the estimate by a large share.
    N, A, diag = full_pattern
    if dtype == torch.float64:   # the same pattern and values in FP64 (2-wide vectors, its own tiles)
        A = A.with_values(A.val.double())
    lmin, lmax = ld.spectral_bounds(A)
    e_b, s_b = ld.logdet(A, lmin, lmax, 80, 30, 0, options=ld.Options(tile_order=1), return_stats=True)
    e_i, s_i = ld.logdet(A, lmin, lmax, 80, 30, 0, options=ld.Options(tile_order=2), return_stats=True)
    assert s_b["tile_order_used"] == 1 and s_i["tile_order_used"] == 2
    assert s_b["block_cols23"] == 20 and s_b["dot_mode_used"] == 2
    assert s_b["ranges23"] > 1 and s_i["ranges23"] == 1
    assert abs(e_b - e_i) <= 1e-10 * abs(e_i), (e_b, e_i)
    g = golden("gmrf5000_theta_sweep")["results"][repr(-0.22)]
    assert abs((e_b - g["expectation"]) / g["sd_hutchinson"]) < 6.0
