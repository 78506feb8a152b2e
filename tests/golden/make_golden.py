"""Write the stored oracle values that the GPU tests compare against.

Calls only the FP64 oracle (``oracle/``) and the shared input generators
(``workloads``).  Usage:  python tests/golden/make_golden.py [name ...]
Each entry is written to tests/golden/<name>.json together with the inputs
that define it (workload, interval, degree, queries, seed).
"""
from __future__ import annotations

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402
from oracle import bounds, exact, hutchpp, newton  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# name -> (workload, overrides, seeds)
ENTRIES = {
    "grid32_k0.5": ("grid32_k0.5", {}, list(range(5))),
    "grid1024_k0.1": ("grid1024_k0.1", {}, [0]),
    "gmrf2048": ("gmrf2048", {}, [0]),
    "grid128c_k0.05": ("grid128c_k0.05", {}, [0]),
    "chunglu_1M": ("chunglu_4M", {"n": 1 << 20}, [0]),
    "penta_1e7": ("penta_1e7", {}, [0]),
}


def make(name: str):
    wl, over, seeds = ENTRIES[name]
    cfg = dict(workloads.CONFIGS[wl])
    cfg.update(over)
    csr = workloads.build(wl, **over)
    Q = workloads.to_scipy(csr)
    lmin, lmax = bounds.gershgorin(csr)
    out = dict(workload=wl, overrides=over, n=int(csr[3]), nnz=int(len(csr[1])), lmin=lmin, lmax=lmax,
               degree=cfg["degree"], m_vec=cfg["m_vec"], results={})
    if cfg["kind"] == "penta":   # exact references by banded Cholesky, FP64 values and FP32-rounded values
        v32 = np.asarray(csr[2], dtype=np.float32).astype(np.float64)
        out["logdet_exact"] = exact.banded_logdet(csr, 2)
        out["logdet_exact_f32_values"] = exact.banded_logdet((csr[0], csr[1], v32, csr[3]), 2)
        out["lmin_f32_values"], out["lmax_f32_values"] = bounds.gershgorin((csr[0], csr[1], v32, csr[3]))
    for s in seeds:
        t = time.perf_counter()
        parts = hutchpp.logdet_estimate(Q, lmin, lmax, cfg["degree"], cfg["m_vec"], s, return_parts=True)
        out["results"][str(s)] = dict(logdet=parts["logdet"], t_low=parts["t_low"], t_res=parts["t_res"],
                                      seconds=time.perf_counter() - t)
        print(name, s, parts["logdet"], f"{time.perf_counter() - t:.1f}s", flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


def make_gmrf_theta_sweep(name="gmrf5000_theta_sweep"):
    """Closed-form references for the theta sweep of Sec. 5.2 at full size (N = 5000).

    For each theta: the exact log det; the estimator's expectation
    n log(sigma) + sum_i P_m(lambda_i / sigma) (Hutch++ is unbiased for the
    trace of the polynomial); and a bound on its standard deviation,
    sqrt(2 sum_i P_m(lambda_i/sigma)^2 / k_G) (Rademacher Hutchinson on the
    deflated residual, whose Frobenius norm is at most that of P_m).  Also the
    standard deviation of plain Hutchinson with k_G Rademacher probes,
    sqrt(2 (||F||_F^2 - sum_i F_ii^2) / k_G), F = P_m(Q~), whose diagonal
    comes from the separable sine eigenvectors (exact.grid_matfun_diag_2d).
    The interval is Gershgorin's, [1 - 4|theta|, 1 + 4|theta|].
    """
    cfg = workloads.CONFIGS["gmrf5000_theta"]
    N, degree, m_vec = cfg["N"], cfg["degree"], cfg["m_vec"]
    n = N * N
    k_g = m_vec - 2 * (m_vec // 3)
    out = dict(workload="gmrf5000_theta", N=N, n=n, degree=degree, m_vec=m_vec, results={})
    for th in workloads.GMRF_THETAS:
        t = time.perf_counter()
        lmin, lmax = 1.0 - 4.0 * abs(th), 1.0 + 4.0 * abs(th)
        lam = exact.gmrf_theta_eigenvalues(N, th)
        plan = newton.NewtonPlan(lmin, lmax, degree)
        pm = plan.eval_scalar(lam)
        fdiag = exact.grid_matfun_diag_2d(N, pm)
        off = float(np.sum(pm * pm) - np.sum(fdiag * fdiag))
        out["results"][repr(th)] = dict(
            theta=th, lmin=lmin, lmax=lmax, logdet_exact=exact.gmrf_theta_logdet(N, th),
            expectation=n * float(np.log(plan.sigma)) + float(np.sum(pm)),
            sd_bound=float(np.sqrt(2.0 * np.sum(pm * pm) / k_g)),
            sd_hutchinson=float(np.sqrt(2.0 * max(off, 0.0) / k_g)), seconds=time.perf_counter() - t)
        print(name, th, out["results"][repr(th)], flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


def stop_margin(plan, Q, X, degrees, tol):
    """Smallest |e_m / tol - 1| over the columns of X and the m up to each
    column's stop, e_m = |d_m| ||w_m||_2 of the forward recurrence: how far the
    stopping decisions sit from a tie with tol."""
    W = np.array(X, dtype=np.float64, copy=True)
    worst = np.inf
    for m in range(int(np.max(degrees)) + 1):
        if m > 0:
            W = plan.alpha * (Q @ W) - plan.beta[m - 1] * W
        e = abs(plan.d[m]) * np.linalg.norm(W, axis=0)
        live = np.asarray(degrees) >= m
        if live.any():
            worst = min(worst, float(np.min(np.abs(e[live] / tol - 1.0))))
    return worst


def make_adaptive(name="gmrf2048_adaptive", wl="gmrf2048", tol_per_sqrt_n=1e-7, seed=0):
    """Alg. 3 with Alg. 2's stopping rule (absolute tol = tol_per_sqrt_n * sqrt(n),
    the norm of a Rademacher probe times tol_per_sqrt_n) at the workload's
    degree as the cap: estimate, every column's degree, and the stopping margin."""
    cfg = dict(workloads.CONFIGS[wl])
    csr = workloads.build(wl)
    Q = workloads.to_scipy(csr)
    n = int(csr[3])
    lmin, lmax = bounds.gershgorin(csr)
    tol = tol_per_sqrt_n * float(np.sqrt(n))
    t = time.perf_counter()
    parts = hutchpp.logdet_estimate_adaptive(Q, lmin, lmax, cfg["degree"], tol, cfg["m_vec"], seed,
                                             return_parts=True)
    secs = time.perf_counter() - t
    k = parts["A"].shape[1]
    deg = parts["degrees"]
    margin = min(stop_margin(parts["plan"], Q, parts["S"], deg[:k], tol),
                 stop_margin(parts["plan"], Q, parts["A"], deg[k:2 * k], tol),
                 stop_margin(parts["plan"], Q, parts["U"], deg[2 * k:], tol))
    out = dict(workload=wl, n=n, nnz=int(len(csr[1])), lmin=lmin, lmax=lmax, max_degree=cfg["degree"],
               m_vec=cfg["m_vec"], seed=seed, tol=tol, logdet=parts["logdet"], t_low=parts["t_low"],
               t_res=parts["t_res"], degrees=[int(x) for x in deg], stop_margin=margin, seconds=secs)
    print(name, parts["logdet"], sorted(set(out["degrees"])), f"margin {margin:.2e}", f"{secs:.1f}s", flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    names = sys.argv[1:] or list(ENTRIES) + ["gmrf5000_theta_sweep", "gmrf2048_adaptive"]
    for nm in names:
        if nm == "gmrf5000_theta_sweep":
            make_gmrf_theta_sweep()
        elif nm == "gmrf2048_adaptive":
            make_adaptive()
        else:
            make(nm)
