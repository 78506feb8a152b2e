"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: FP64 bulk 1e-10 relative; FP32 bulk 1e-4 relative on the
estimate (the target), with tighter checks where the arithmetic allows.
"""
import math

import numpy as np
import pytest

import workloads as w
from oracle import bounds, exact, hutchpp, newton
from tests.gpu_common import assert_cols_close, golden, nine_point_grid, random_spd_csr

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


def rel(a, b):
    return abs(a - b) / abs(b)


def test_loaded_library_matches_sources():
    # the library this GPU run loaded was built from the sources in this tree
    from paper_2603_02207_amd import _native as nat

    assert nat.built_source_hash() == nat.source_hash(), (nat.built_source_hash(), nat.source_hash())


# ---------------------------------------------------------------- apply_log

@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 2e-5)])
@pytest.mark.parametrize("ncols", [1, 3, 8, 20, 33])
def test_apply_log_random_block(dtype, tol, ncols):
    csr = w.grid_laplacian_2d(37, 0.5)          # n = 1369: several tiles plus a ragged tail
    A, vals = to_gpu(csr, dtype)
    rng = np.random.default_rng(ncols)
    V = rng.standard_normal((csr[3], ncols))
    Vd = torch.tensor(V, dtype=dtype, device=DEV)
    Vin = Vd.double().cpu().numpy()
    out = ld.apply_log(A, 0.5, 8.5, 40, Vd).double().cpu().numpy()
    Q = w.to_scipy((csr[0], csr[1], vals, csr[3]))
    ref = newton.apply_log(Q, Vin, 0.5, 8.5, 40)
    assert_cols_close(out, ref, tol)


def test_apply_log_block_width_invariance_bitwise():
    csr = w.grid_laplacian_2d(30, 0.5)
    A, _ = to_gpu(csr, torch.float32)
    V = torch.tensor(np.random.default_rng(0).standard_normal((900, 24)), dtype=torch.float32, device=DEV)
    full = ld.apply_log(A, 0.5, 8.5, 30, V)
    for b in (4, 8, 12):
        part = ld.apply_log(A, 0.5, 8.5, 30, V, options=ld.Options(block_cols=b))
        assert torch.equal(full, part)
    # each column alone gives the same bits as inside the block
    one = ld.apply_log(A, 0.5, 8.5, 30, V[:, 5:6].contiguous())
    assert torch.equal(one[:, 0], full[:, 5])


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_apply_log_dirichlet_eigenvectors_full_size(dtype, tol):
    # 1024 x 1024 grid, degree 80: P_m(Q~)v = P_m(lambda/sigma) v for the sine eigenvectors.
    N, k2, m = 1024, 0.1, 80
    csr = w.grid_laplacian_2d(N, k2)
    A, _ = to_gpu(csr, dtype)
    plan = newton.NewtonPlan(k2, k2 + 8.0, m)
    modes = [(1, 1), (3, 700), (512, 513), (1024, 1024)]
    V = np.stack([w.dirichlet_sine_vector_2d(N, a, b) for a, b in modes], axis=1)
    Vd = torch.tensor(V, dtype=dtype, device=DEV)
    out = ld.apply_log(A, k2, k2 + 8.0, m, Vd).double().cpu().numpy()
    Vin = Vd.double().cpu().numpy()
    for i, (a, b) in enumerate(modes):
        lam = exact.grid_eigenvalue_2d(N, k2, a, b)
        scal = float(plan.eval_scalar(lam)) + math.log(plan.sigma)
        ref = scal * Vin[:, i]
        assert_cols_close(out[:, i], ref, tol)


def test_apply_log_empty_block_and_degree_one():
    csr = w.grid_laplacian_2d(8, 0.5)
    A, vals = to_gpu(csr, torch.float64)
    V = torch.zeros((64, 0), dtype=torch.float64, device=DEV)
    assert ld.apply_log(A, 0.5, 8.5, 10, V).shape == (64, 0)
    V = torch.tensor(np.random.default_rng(1).standard_normal((64, 2)), device=DEV)
    out = ld.apply_log(A, 0.5, 8.5, 1, V).cpu().numpy()
    ref = newton.apply_log(w.to_scipy((csr[0], csr[1], vals, 64)), V.cpu().numpy(), 0.5, 8.5, 1)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13)


# ---------------------------------------------------------------- estimator

@pytest.mark.parametrize("seed", range(5))
def test_estimate_grid32_against_oracle(seed):
    g = golden("grid32_k0.5")
    csr = w.grid_laplacian_2d(32, 0.5)
    A64, _ = to_gpu(csr, torch.float64)
    A32, vals32 = to_gpu(csr, torch.float32)
    ref = g["results"][str(seed)]["logdet"]
    e64 = ld.logdet(A64, 0.5, 8.5, 40, 30, seed)
    assert rel(e64, ref) < 1e-10
    e32 = ld.logdet(A32, 0.5, 8.5, 40, 30, seed)
    assert rel(e32, ref) < 1e-4
    # against the oracle run on the FP32-rounded values: FP32 arithmetic error only
    ref32 = hutchpp.logdet_estimate(w.to_scipy((csr[0], csr[1], vals32, csr[3])), 0.5, 8.5, 40, 30, seed)
    assert rel(e32, ref32) < 1e-5


@pytest.mark.parametrize("mode", [ld.LD_DOT_FORWARD, ld.LD_DOT_SQUARED])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_estimate_dot_modes(mode, dtype, tol):
    csr = w.grid_laplacian_2d(45, 0.3)        # n = 2025, ragged against every tile size
    A, vals = to_gpu(csr, dtype)
    lmin, lmax = bounds.gershgorin(csr)
    for deg, mv in ((33, 21), (40, 30)):       # odd and even degree
        est, st = ld.logdet(A, lmin, lmax, deg, mv, 3, options=ld.Options(dot_mode=mode), return_stats=True)
        assert st["dot_mode_used"] == mode
        ref = hutchpp.logdet_estimate(w.to_scipy((csr[0], csr[1], vals, csr[3])), lmin, lmax, deg, mv, 3)
        assert rel(est, ref) < tol


@pytest.mark.parametrize("dtype,widths", [(torch.float32, (4, 8, 12, 16, 20)), (torch.float64, (2, 4, 6))])
def test_estimate_block_cols_invariance(dtype, widths):
    # narrow sketch blocks on the diagonal storage read their signs from the
    # byte planes when the block lies in one byte of the sign word (every
    # block at 4 and 8 FP32 columns, 2 and 4 FP64; some at 12 and 6), the
    # 64-bit words otherwise (16 and 20 take all k = 16 columns): the same
    # estimate to the grouping of the FP64 sums
    csr = w.grid_laplacian_2d(40, 0.5)
    A, _ = to_gpu(csr, dtype)
    base = ld.logdet(A, 0.5, 8.5, 30, 48, 1)
    for b in widths:
        e, st = ld.logdet(A, 0.5, 8.5, 30, 48, 1, options=ld.Options(block_cols=b), return_stats=True)
        assert st["block_cols1"] == min(b, 16) and st["dia_constant"] == 1
        assert rel(e, base) < 1e-12, b
    # deterministic repeat
    assert ld.logdet(A, 0.5, 8.5, 30, 48, 1) == base


@pytest.mark.parametrize("n,long_rows,seed", [(700, 0, 0), (1500, 3, 1), (333, 1, 2)])
@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
def test_estimate_irregular_sparsity(n, long_rows, seed, dtype, tol):
    csr = random_spd_csr(n, seed, long_rows=long_rows)
    A, vals = to_gpu(csr, dtype)
    csr_v = (csr[0], csr[1], vals, n)
    lmin, lmax = bounds.gershgorin(csr_v)
    est = ld.logdet(A, lmin, lmax, 50, 24, seed)
    ref = hutchpp.logdet_estimate(w.to_scipy(csr_v), lmin, lmax, 50, 24, seed)
    assert rel(est, ref) < tol


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
@pytest.mark.parametrize("permute", [False, True])
def test_estimate_power_law_hub_rows(dtype, tol, permute):
    # hub rows far above the long-row threshold, both row orders
    csr = w.chung_lu_laplacian(30000, seed=2, permute=permute)
    assert np.diff(csr[0]).max() > 200
    A, vals = to_gpu(csr, dtype)
    csr_v = (csr[0], csr[1], vals, csr[3])
    lmin, lmax = bounds.gershgorin(csr_v)
    Q = w.to_scipy(csr_v)
    for mode in (ld.LD_DOT_FORWARD, ld.LD_DOT_SQUARED):
        est = ld.logdet(A, lmin, lmax, 40, 24, 5, options=ld.Options(dot_mode=mode))
        ref = hutchpp.logdet_estimate(Q, lmin, lmax, 40, 24, 5)
        assert rel(est, ref) < tol, mode
    V = np.random.default_rng(0).standard_normal((csr[3], 6))
    out = ld.apply_log(A, lmin, lmax, 30, torch.tensor(V, dtype=dtype, device=DEV)).double().cpu().numpy()
    refv = newton.apply_log(Q, torch.tensor(V, dtype=dtype).double().numpy(), lmin, lmax, 30)
    assert_cols_close(out, refv, 1e-10 if dtype == torch.float64 else 1e-5)


@pytest.mark.parametrize("m_vec", [3, 4, 5, 32, 100, 192])
def test_estimate_query_counts(m_vec):
    # k = floor(m_vec/3) sketch columns and k_G = m_vec - 2k residual probes:
    # the fewest queries, counts not divisible by three, and the widest
    # sketch allowed (k = k_G = 64: the MFMA cross products, quadratic forms
    # in two column blocks).  FP64 against the oracle; FP32 against the oracle
    # run on the FP32-rounded values.
    csr = random_spd_csr(2500, 11, long_rows=1)
    for dtype, tol in ((torch.float64, 1e-10), (torch.float32, 2e-5)):
        A, vals = to_gpu(csr, dtype)
        csr_v = (csr[0], csr[1], vals, csr[3])
        lo, hi = bounds.gershgorin(csr_v)
        lo = max(lo, 0.2)
        est, st = ld.logdet(A, lo, hi, 30, m_vec, 4, return_stats=True)
        assert st["k"] == m_vec // 3 and st["k_G"] == m_vec - 2 * (m_vec // 3)
        ref = hutchpp.logdet_estimate(w.to_scipy(csr_v), lo, hi, 30, m_vec, 4)
        assert rel(est, ref) < tol, (dtype, est, ref)
    with pytest.raises(ld.NativeError):   # k_G = 66 > 64
        ld.logdet(A, lo, hi, 30, 194, 4)


def test_estimate_small_and_sigma_one():
    # lmin >= 1 (sigma = 1), tiny n with k close to n
    csr = w.grid_laplacian_2d(4, 3.0)
    A, vals = to_gpu(csr, torch.float64)
    est = ld.logdet(A, 3.0, 11.0, 25, 30, 0)
    ref = hutchpp.logdet_estimate(w.to_scipy((csr[0], csr[1], vals, 16)), 3.0, 11.0, 25, 30, 0)
    assert rel(est, ref) < 1e-10


def test_estimate_grid1024_full_size():
    g = golden("grid1024_k0.1")
    if g is None:
        pytest.skip("oracle value for the 1024 x 1024 grid not generated")
    csr = w.grid_laplacian_2d(1024, 0.1)
    ref = g["results"]["0"]["logdet"]
    A32, _ = to_gpu(csr, torch.float32)
    e32 = ld.logdet(A32, g["lmin"], g["lmax"], g["degree"], g["m_vec"], 0)
    assert rel(e32, ref) < 1e-4
    A64, _ = to_gpu(csr, torch.float64)
    e64 = ld.logdet(A64, g["lmin"], g["lmax"], g["degree"], g["m_vec"], 0)
    assert rel(e64, ref) < 1e-10


def test_estimate_pentadiagonal_1e7_full_size():
    # Sec. 5.1's pentadiagonal study at its largest size (n = 1e7): parity with the
    # oracle's estimate on the same probes, and the exact log det by banded
    # Cholesky within the estimator's own error.  For Q ~ n I the Monte-Carlo
    # error is dominated by log(lambda) * (||u_j||^2 - n) of the deflated
    # residual probes, ||u_j||^2 = n - ||Q_b^T g_j||^2 with ||Q_b^T g_j||^2 ~ chi^2_k,
    # so sd ~ log(lmax) sqrt(2k/k_G); six of those bound |estimate - exact|.
    g = golden("penta_1e7")
    csr = w.build("penta_1e7")
    k, kg = g["m_vec"] // 3, g["m_vec"] - 2 * (g["m_vec"] // 3)
    sd = math.log(g["lmax"]) * math.sqrt(2.0 * k / kg)
    ref = g["results"]["0"]["logdet"]
    A64, _ = to_gpu(csr, torch.float64)
    e64 = ld.logdet(A64, g["lmin"], g["lmax"], g["degree"], g["m_vec"], 0)
    assert rel(e64, ref) < 1e-12
    assert abs(e64 - g["logdet_exact"]) < 6 * sd
    del A64
    A32, _ = to_gpu(csr, torch.float32)
    lo, hi = ld.spectral_bounds(A32)
    assert lo == pytest.approx(g["lmin_f32_values"], rel=1e-12) and hi == pytest.approx(g["lmax_f32_values"], rel=1e-12)
    e32 = ld.logdet(A32, lo, hi, g["degree"], g["m_vec"], 0)
    assert rel(e32, ref) < 1e-7
    assert abs(e32 - g["logdet_exact_f32_values"]) < 6 * sd


# ---------------------------------------------------------------- bounds and errors

def test_spectral_bounds_match_oracle():
    for csr in (w.grid_laplacian_2d(50, 0.1), w.grid_laplacian_3d(9, 0.05), random_spd_csr(500, 4, long_rows=2)):
        for dtype in (torch.float64, torch.float32):
            A, vals = to_gpu(csr, dtype)
            lo, hi = ld.spectral_bounds(A)
            rlo, rhi = bounds.gershgorin((csr[0], csr[1], vals, csr[3]))
            assert lo == pytest.approx(rlo, rel=1e-12, abs=1e-12)
            assert hi == pytest.approx(rhi, rel=1e-12)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_lanczos_upper_bound(dtype):
    # Appendix A's Lanczos refinement of lambda_max: the device result must lie
    # between the true top eigenvalue and Gershgorin's bound, and agree with the
    # oracle's Ritz value + residual from the same start vector.
    from oracle import rng
    cases = ((w.chung_lu_laplacian(1500, seed=1), 40), (w.grid_laplacian_2d(30, 0.5), 25),
             (w.pentadiagonal(800, seed=3), 30), (random_spd_csr(600, 4, long_rows=2), 20))
    for csr, steps in cases:
        A, vals = to_gpu(csr, dtype)
        csr_v = (csr[0], csr[1], vals, csr[3])
        Q = w.to_scipy(csr_v)
        top = np.linalg.eigvalsh(Q.toarray())[-1]
        g_lo, g_hi = bounds.gershgorin(csr_v)
        lo, hi = ld.spectral_bounds(A, lanczos_steps=steps)
        assert lo == pytest.approx(g_lo, rel=1e-12, abs=1e-12)
        assert top * (1 - 1e-9) <= hi <= g_hi * (1 + 1e-12)
        theta, upper = bounds.lanczos_upper(Q, steps, rng.rademacher(0, 2, csr[3], 1)[:, 0])
        # the refinement runs in FP64 on the (FP32-rounded) values in both cases
        assert hi == pytest.approx(min(upper, g_hi), rel=1e-8)
    with pytest.raises(ld.NativeError):
        ld.spectral_bounds(A, lanczos_steps=10**6)


def test_invalid_csr_is_rejected():
    csr = w.grid_laplacian_2d(6, 0.5)
    bad_cols = csr[1].copy()
    bad_cols[10] = 999                        # out of range
    A = ld.CSR.from_arrays(csr[0], bad_cols, csr[2], 36, device=DEV)
    with pytest.raises(ld.NativeError) as e:
        ld.logdet(A, 0.5, 8.5, 10, 9, 0)
    assert e.value.code == -2
    unsorted = csr[1].copy()
    unsorted[[0, 1]] = unsorted[[1, 0]]
    A = ld.CSR.from_arrays(csr[0], unsorted, csr[2], 36, device=DEV)
    with pytest.raises(ld.NativeError):
        ld.apply_log(A, 0.5, 8.5, 10, torch.ones((36, 2), device=DEV))
    bad_ptr = csr[0].copy()
    bad_ptr[5] = 10**6
    A = ld.CSR.from_arrays(bad_ptr, csr[1], csr[2], 36, device=DEV)
    with pytest.raises(ld.NativeError):
        ld.spectral_bounds(A)


def test_cholqr_breakdown_is_reported():
    # n = 3 and k = 3: pick a seed whose 3 x 3 sketch is singular (two equal or
    # opposite columns), so Y = F S is rank deficient.
    from oracle import rng

    seed = next(s for s in range(200) if abs(np.linalg.det(rng.rademacher(s, 0, 3, 3))) < 0.5)
    row_ptr = np.array([0, 1, 2, 3], dtype=np.int32)
    col_idx = np.array([0, 1, 2], dtype=np.int32)
    A = ld.CSR.from_arrays(row_ptr, col_idx, np.array([2.0, 3.0, 5.0]), 3, device=DEV, dtype=torch.float64)
    with pytest.raises(ld.NativeError) as e:
        ld.logdet(A, 1.5, 6.0, 10, 9, seed)
    assert e.value.code == -3


def test_workspace_too_small():
    csr = w.grid_laplacian_2d(8, 0.5)
    A, _ = to_gpu(csr, torch.float32)
    ws = torch.empty(16, dtype=torch.uint8, device=DEV)
    import ctypes
    from paper_2603_02207_amd import _native as nat

    c = A.c_struct()
    out = ctypes.c_double()
    rc = nat.load().ld_logdet_estimate(ctypes.byref(c), 0.5, 8.5, 10, 9, 0, None, ctypes.c_void_p(ws.data_ptr()),
                                       16, None, ctypes.byref(out), None)
    assert rc == nat.LD_EWORKSPACE
    # a workspace that is large enough but not 256-byte aligned is refused
    need = ld.workspace_size(A, 10, 9)
    big = torch.empty(need + 512, dtype=torch.uint8, device=DEV)
    rc = nat.load().ld_logdet_estimate(ctypes.byref(c), 0.5, 8.5, 10, 9, 0, None,
                                       ctypes.c_void_p(big.data_ptr() + 8), need, None, ctypes.byref(out), None)
    assert rc == nat.LD_EINVAL and b"aligned" in nat.load().ld_last_error_detail()
    rc = nat.load().ld_logdet_estimate(ctypes.byref(c), 0.5, 8.5, 10, 9, 0, None,
                                       ctypes.c_void_p(big.data_ptr() + 256), need, None, ctypes.byref(out), None)
    assert rc == nat.LD_OK


# ---------------------------------------------------------------- the other workloads at full size

@pytest.mark.parametrize("name,tol32", [("grid128c_k0.05", 1e-4), ("gmrf2048", 1e-4), ("chunglu_1M", 1e-4)])
def test_estimate_full_size_workloads(name, tol32):
    g = golden(name)
    if g is None:
        pytest.skip(f"oracle value for {name} not generated")
    csr = w.build(g["workload"], **g["overrides"])
    ref = g["results"]["0"]["logdet"]
    A32, _ = to_gpu(csr, torch.float32)
    A64, _ = to_gpu(csr, torch.float64)
    lo, hi = ld.spectral_bounds(A64)
    assert lo == pytest.approx(g["lmin"], rel=1e-12) and hi == pytest.approx(g["lmax"], rel=1e-12)
    e32, st = ld.logdet(A32, g["lmin"], g["lmax"], g["degree"], g["m_vec"], 0, return_stats=True)
    assert rel(e32, ref) < tol32, (e32, ref, st["dot_mode_used"])
    e64, st64 = ld.logdet(A64, g["lmin"], g["lmax"], g["degree"], g["m_vec"], 0, return_stats=True)
    assert rel(e64, ref) < 1e-10
    # column blocks whose two step buffers (2 n elem bytes per column) fit
    # 170 MB with the matrix as stored: 8 FP32 / 4 FP64 columns at n = 2^21,
    # 4 / 2 at n = 2^22 (constant diagonals); the power-law graph's blocks
    # follow its CSR bytes and are not asserted here
    blocks = {"grid128c_k0.05": ((8, 8), (4, 4)), "gmrf2048": ((4, 4), (2, 2)), "chunglu_1M": (None, None)}[name]
    for stats, want in ((st, blocks[0]), (st64, blocks[1])):
        if want:
            assert (stats["block_cols1"], stats["block_cols23"]) == want
            assert stats["xcd_chunk_rows"] == 0   # the blocks run from the cache: contiguous bands
    if name == "grid128c_k0.05":
        # one 64-column block streams from HBM: XCD bands in chunks of a plane / 8
        e1, s1 = ld.logdet(A32, g["lmin"], g["lmax"], g["degree"], g["m_vec"], 0,
                           options=ld.Options(block_cols=64), return_stats=True)
        assert s1["block_cols23"] == 64 and s1["xcd_chunk_rows"] == 128 * 128 // 8
        assert rel(e1, ref) < tol32


# ---------------------------------------------------------------- diagonal storage

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_diagonal_storage_matches_csr_bitwise(dtype):
    # Stencil and banded matrices are gathered from the diagonal storage, with
    # the offsets in column order: the same products summed in the same order
    # as the CSR path, hence bit-identical results.  Constant-coefficient
    # stencils keep one value per diagonal (presence bits per row); a grid
    # with one diagonal entry changed and the random pentadiagonal matrix
    # keep the stored values, as does a 9-point stencil with random weights
    # (nine diagonals: the widest gather of the diagonal storage).
    g2 = w.grid_laplacian_2d(96, 0.3)
    bumped = np.array(g2[2], dtype=np.float64, copy=True)
    r_b = 4321
    bumped[g2[0][r_b] + list(g2[1][g2[0][r_b]:g2[0][r_b + 1]]).index(r_b)] += 0.5
    for csr, lo, hi, const in ((g2, 0.3, 8.3, 1), (w.grid_laplacian_3d(20, 0.2), 0.2, 12.2, 1),
                               ((g2[0], g2[1], bumped, g2[3]), 0.3, 8.8, 0),
                               (w.pentadiagonal(5000, 1), None, None, 0), (nine_point_grid(61, 4), None, None, 0)):
        A, vals = to_gpu(csr, dtype)
        if lo is None:
            lo, hi = bounds.gershgorin((csr[0], csr[1], vals, csr[3]))
        est_d, st_d = ld.logdet(A, lo, hi, 30, 24, 5, return_stats=True)
        est_c, st_c = ld.logdet(A, lo, hi, 30, 24, 5, options=ld.Options(csr_only=1), return_stats=True)
        rows = np.repeat(np.arange(csr[3]), np.diff(csr[0]))
        assert st_d["dia_diagonals"] == len(np.unique(np.asarray(csr[1]) - rows))
        assert st_d["dia_constant"] == const
        assert st_c["dia_diagonals"] == 0 and st_c["dia_constant"] == 0
        assert est_d == est_c
        V = torch.tensor(np.random.default_rng(3).standard_normal((csr[3], 6)), dtype=dtype, device=DEV)
        assert torch.equal(ld.apply_log(A, lo, hi, 25, V), ld.apply_log(A, lo, hi, 25, V, ld.Options(csr_only=1)))
        # the gradient: the same recurrence vectors and estimate; the FP64
        # per-entry sums of the two sweep kernels are added in another order
        e1, g1 = ld.logdet_with_grad(A, lo, hi, 12, 9, 2)
        e2, g2 = ld.logdet_with_grad(A, lo, hi, 12, 9, 2, options=ld.Options(csr_only=1))
        assert e1 == e2
        assert_cols_close(g1.double().cpu().numpy(), g2.double().cpu().numpy(),
                          1e-13 if dtype == torch.float64 else 2e-7)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 2e-5)])
def test_nine_point_stencil_against_oracle(dtype, tol):
    # nine diagonals with varying values (the widest diagonal-storage gather),
    # a grid ragged against the row tiles; estimate and Horner apply
    csr = nine_point_grid(45, 7)
    A, vals = to_gpu(csr, dtype)
    csr_v = (csr[0], csr[1], vals, csr[3])
    lo, hi = bounds.gershgorin(csr_v)
    est, st = ld.logdet(A, lo, hi, 30, 24, 2, return_stats=True)
    assert st["dia_diagonals"] == 9 and st["dia_constant"] == 0
    Q = w.to_scipy(csr_v)
    assert rel(est, hutchpp.logdet_estimate(Q, lo, hi, 30, 24, 2)) < tol
    V = np.random.default_rng(5).standard_normal((csr[3], 5))
    out = ld.apply_log(A, lo, hi, 25, torch.tensor(V, dtype=dtype, device=DEV)).double().cpu().numpy()
    ref = newton.apply_log(Q, torch.tensor(V, dtype=dtype).double().numpy(), lo, hi, 25)
    assert_cols_close(out, ref, tol)


def test_diagonal_storage_falls_back_to_csr():
    # one entry off the stencil's diagonals, and an irregular matrix: CSR path
    row_ptr, col_idx, val, n = w.grid_laplacian_2d(40, 0.5)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    keep_r, keep_c, keep_v = list(rows), list(col_idx), list(val)
    keep_r += [0, 777]
    keep_c += [777, 0]
    keep_v += [-0.25, -0.25]
    order = np.lexsort((keep_c, keep_r))
    r2, c2, v2 = np.asarray(keep_r)[order], np.asarray(keep_c)[order], np.asarray(keep_v)[order]
    rp2 = np.concatenate([[0], np.cumsum(np.bincount(r2, minlength=n))]).astype(np.int32)
    for csr in ((rp2, c2.astype(np.int32), v2, n), random_spd_csr(900, 2, long_rows=1)):
        A, vals = to_gpu(csr, torch.float64)
        lo, hi = bounds.gershgorin((csr[0], csr[1], vals, csr[3]))
        lo = max(lo, 0.1)
        est, st = ld.logdet(A, lo, hi, 20, 12, 1, return_stats=True)
        assert st["dia_diagonals"] == 0
        ref = hutchpp.logdet_estimate(w.to_scipy((csr[0], csr[1], vals, csr[3])), lo, hi, 20, 12, 1)
        assert rel(est, ref) < 1e-10


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 2e-5)])
def test_tile_orders_agree_with_oracle(dtype, tol):
    # Both row-tile orders of the Newton-step launches: the recurrence vectors
    # are per-row results (bit-identical), the quadratic forms regroup their
    # workgroup sums (same value to rounding); both against the oracle.  A
    # 3-D stencil (diagonal storage) and an irregular matrix with long rows
    # (CSR path), several hundred tiles each.
    for csr in (w.grid_laplacian_3d(40, 0.2), random_spd_csr(60000, 9, long_rows=3)):
        A, vals = to_gpu(csr, dtype)
        csr_v = (csr[0], csr[1], vals, csr[3])
        lo, hi = bounds.gershgorin(csr_v)
        lo = max(lo, 0.2)
        ref = hutchpp.logdet_estimate(w.to_scipy(csr_v), lo, hi, 30, 24, 4)
        V = torch.tensor(np.random.default_rng(8).standard_normal((csr[3], 7)), dtype=dtype, device=DEV)
        outs = []
        for order in (1, 2):
            o = ld.Options(tile_order=order)
            est = ld.logdet(A, lo, hi, 30, 24, 4, options=o)
            assert rel(est, ref) < tol, (order, est, ref)
            outs.append(ld.apply_log(A, lo, hi, 25, V, o))
        assert torch.equal(outs[0], outs[1])
        # the gradient call: its sweeps are per-row work that does not depend
        # on the tile order (bit-identical); its estimate regroups its sums
        e1, g1 = ld.logdet_with_grad(A, lo, hi, 12, 9, 2, options=ld.Options(tile_order=1))
        e2, g2 = ld.logdet_with_grad(A, lo, hi, 12, 9, 2, options=ld.Options(tile_order=2))
        assert rel(e1, e2) < 1e-12 and torch.equal(g1, g2)
    with pytest.raises(ld.NativeError):
        ld.logdet(A, lo, hi, 30, 24, 4, options=ld.Options(tile_order=3))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-11), (torch.float32, 2e-5)])
def test_chunked_xcd_bands_for_3d_grids(dtype, tol):
    # A 64^3 grid: the plane neighbours (4096 rows away) of a contiguous band
    # would not stay in an XCD's L2 at 64 columns, so the quadratic forms cut
    # the bands into chunks of 512 rows dealt to the XCDs in turn.  The
    # recurrence vectors are per-row results (bit-identical to the other
    # orders), the quadratic forms regroup their sums; both against the oracle.
    csr = w.grid_laplacian_3d(64, 0.2)
    A, vals = to_gpu(csr, dtype)
    csr_v = (csr[0], csr[1], vals, csr[3])
    lo, hi = bounds.gershgorin(csr_v)
    ref = hutchpp.logdet_estimate(w.to_scipy(csr_v), lo, hi, 24, 96, 3)
    est, st = ld.logdet(A, lo, hi, 24, 96, 3, return_stats=True)
    assert st["tile_order_used"] == 1 and st["xcd_chunk_rows"] == 512
    assert rel(est, ref) < tol, (est, ref)
    for order in (1, 2):   # explicit bands are the chunked bands here; interleaved never chunks
        e, so = ld.logdet(A, lo, hi, 24, 96, 3, options=ld.Options(tile_order=order), return_stats=True)
        assert so["xcd_chunk_rows"] == (512 if order == 1 else 0)
        assert rel(e, ref) < tol
    V = torch.tensor(np.random.default_rng(2).standard_normal((csr[3], 32)), dtype=dtype, device=DEV)
    out_b = ld.apply_log(A, lo, hi, 20, V, ld.Options(tile_order=1))
    out_i = ld.apply_log(A, lo, hi, 20, V, ld.Options(tile_order=2))
    assert torch.equal(out_b, out_i)
    refv = newton.apply_log(w.to_scipy(csr_v), V.double().cpu().numpy(), lo, hi, 20)
    assert_cols_close(out_b.double().cpu().numpy(), refv, 1e-12 if dtype == torch.float64 else 2e-5)


def test_tile_order_follows_band_balance():
    # auto: XCD bands for a stencil, interleaved tiles for a power-law graph
    # whose hubs come first (most entries in the first row band); the estimate
    # matches the oracle either way.
    for csr, want in ((w.grid_laplacian_2d(300, 0.5), 1), (w.chung_lu_laplacian(1 << 16), 2)):
        A, vals = to_gpu(csr, torch.float64)
        csr_v = (csr[0], csr[1], vals, csr[3])
        lo, hi = bounds.gershgorin(csr_v)
        lo = max(lo, 1e-2)
        est, st = ld.logdet(A, lo, hi, 30, 24, 2, return_stats=True)
        assert st["tile_order_used"] == want
        forced = ld.logdet(A, lo, hi, 30, 24, 2, options=ld.Options(tile_order=3 - want), return_stats=True)[1]
        assert forced["tile_order_used"] == 3 - want
        ref = hutchpp.logdet_estimate(w.to_scipy(csr_v), lo, hi, 30, 24, 2)
        assert rel(est, ref) < 1e-10


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 2e-5)])
def test_gaussian_probes_against_oracle(dtype, tol):
    # Gaussian probe entries from the same counter generator (Box-Muller in
    # FP64 on both sides): a stencil in diagonal storage with several sketch
    # blocks, and an irregular matrix with long rows; the sketch goes
    # through the stored-probe Horner step, the deflation through the
    # general cross product.
    cases = ((w.grid_laplacian_2d(200, 0.3), 48, dict(block_cols=8)),
             (random_spd_csr(20000, 9, long_rows=3), 30, {}))
    for csr, m_vec, extra in cases:
        A, vals = to_gpu(csr, dtype)
        csr_v = (csr[0], csr[1], vals, csr[3])
        lo, hi = bounds.gershgorin(csr_v)
        lo = max(lo, 0.3)
        est, st = ld.logdet(A, lo, hi, 30, m_vec, 7, options=ld.Options(probe_dist=1, **extra), return_stats=True)
        ref = hutchpp.logdet_estimate(w.to_scipy(csr_v), lo, hi, 30, m_vec, 7, probes="gaussian")
        assert rel(est, ref) < tol, (est, ref)
        if dtype == torch.float64:   # not the Rademacher estimate
            assert rel(est, hutchpp.logdet_estimate(w.to_scipy(csr_v), lo, hi, 30, m_vec, 7)) > 1e-8
    with pytest.raises(ld.NativeError):
        ld.logdet(A, lo, hi, 30, 24, 4, options=ld.Options(probe_dist=2))


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 2e-5)])
def test_estimate_parts_against_oracle(dtype, tol):
    # The two traces of Alg. 3 (steps 5 and 6) separately, so that errors in
    # the sketch basis and in the deflated residual cannot cancel in the sum;
    # both quadratic-form modes.
    for csr in (w.grid_laplacian_2d(70, 0.4), random_spd_csr(12000, 7, long_rows=2)):
        A, vals = to_gpu(csr, dtype)
        csr_v = (csr[0], csr[1], vals, csr[3])
        lo, hi = bounds.gershgorin(csr_v)
        lo = max(lo, 0.4)
        ref = hutchpp.logdet_estimate(w.to_scipy(csr_v), lo, hi, 36, 30, 11, return_parts=True)
        scale = abs(ref["logdet"])
        for mode in (ld.LD_DOT_FORWARD, ld.LD_DOT_SQUARED):
            est, st = ld.logdet(A, lo, hi, 36, 30, 11, options=ld.Options(dot_mode=mode), return_stats=True)
            assert st["dot_mode_used"] == mode
            assert abs(st["t_low"] - ref["t_low"]) < tol * scale, (mode, st["t_low"], ref["t_low"])
            assert abs(st["t_res"] - ref["t_res"]) < tol * scale, (mode, st["t_res"], ref["t_res"])
            assert rel(est, ref["logdet"]) < tol


def test_profile_line_on_request(capfd, monkeypatch):
    # LD_PROFILE=1: one phase-breakdown line per estimate on stderr; the
    # estimate itself is unchanged
    csr = w.grid_laplacian_2d(40, 0.5)
    A, _ = to_gpu(csr, torch.float32)
    quiet = ld.logdet(A, 0.5, 8.5, 20, 12, 1)
    capfd.readouterr()
    monkeypatch.setenv("LD_PROFILE", "1")
    loud = ld.logdet(A, 0.5, 8.5, 20, 12, 1)
    err = capfd.readouterr().err
    assert "ld_profile: estimate n=1600 degree=20 m_vec=12" in err and "storage diagonal" in err
    assert loud == quiet
    monkeypatch.setenv("LD_PROFILE", "0")
    ld.logdet(A, 0.5, 8.5, 20, 12, 1)
    assert "ld_profile" not in capfd.readouterr().err


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_half_lmax_scaling_value_against_oracle(dtype, tol):
    # Alg. 1 with s = lambda_max/2 (Sec. 3.1, the second variant of Tab. 3/4):
    # the Taylor series has not converged after taylor_cap terms, so the
    # coefficients (and the estimate) differ from the s = c ones; the oracle
    # runs its own Alg. 1 with the same cap.  Estimate and Horner apply, a
    # stencil in diagonal storage and an irregular matrix with long rows.
    for csr, deg, mv, cap in ((w.grid_laplacian_2d(32, 0.5), 40, 30, 3000),
                              (random_spd_csr(3000, 6, long_rows=2), 30, 24, 800)):
        A, vals = to_gpu(csr, dtype)
        csr_v = (csr[0], csr[1], vals, csr[3])
        lo, hi = bounds.gershgorin(csr_v)
        lo = max(lo, 0.5)
        Q = w.to_scipy(csr_v)
        opts = ld.Options(s_val_mode=ld.LD_SVAL_HALF_LMAX, taylor_cap=cap)
        est, st = ld.logdet(A, lo, hi, deg, mv, 2, options=opts, return_stats=True)
        assert st["taylor_terms"] == cap
        ref = hutchpp.logdet_estimate(Q, lo, hi, deg, mv, 2, s_mode="half_lmax", taylor_cap=cap)
        assert rel(est, ref) < tol, (est, ref)
        if dtype == torch.float64:   # a different number from the s = c estimate (FP64 parity is ~1e-12)
            assert rel(est, hutchpp.logdet_estimate(Q, lo, hi, deg, mv, 2)) > 1e-10
        V = np.random.default_rng(4).standard_normal((csr[3], 5))
        Vd = torch.tensor(V, dtype=dtype, device=DEV)
        out = ld.apply_log(A, lo, hi, deg, Vd, options=opts).double().cpu().numpy()
        refv = newton.apply_log(Q, Vd.double().cpu().numpy(), lo, hi, deg, s_mode="half_lmax", taylor_cap=cap)
        assert_cols_close(out, refv, 1e-12 if dtype == torch.float64 else 2e-5)
