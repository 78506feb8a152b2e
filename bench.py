#!/usr/bin/env python3
"""Throughput of the Léja + Hutch++ log-determinant estimator on one MI355X.

One "step" is one complete estimate (Alg. 3: sketch recurrence, CholQR2,
deflation, quadratic-form recurrence, combination) on the default workload:
the 5-point Dirichlet Laplacian of a 1024 x 1024 grid plus 0.1 I (n = 1,048,576,
nnz = 5,238,784), Léja degree 80, 60 Rademacher queries, FP32 bulk arithmetic
with FP64 scalars and reductions.  Inputs are resident in HBM before timing;
the probes are generated inside each estimate.

Prints one JSON line: the estimate rate (value), the roofline of the dominant
recurrence kernel from HIP events in the library, the FP64-bulk rate, parity
against the stored FP64 oracle value on the oracle's own interval, the rate of
the same workload on the CSR path (no diagonal storage), the bytes of the
step kernels against the plain per-step bytes of the method, an HBM-bound
record (the 2048 x 2048 GMRF, degree 100, 32 queries, whose blocks do not fit
the Infinity Cache) with its dominant kernel against 8 TB/s and against a
1 GiB device copy measured in the same run, and a CPU baseline (the oracle
itself, one full estimate on the host).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "logdet estimates/sec & SpMM HBM GB/s at ≤1e-4 rel err, FP32 vs FP64, 1 GPU"
HBM_PEAK_GBS = 8000.0
INFINITY_CACHE_BYTES = 256e6   # MI355X last-level (MALL) cache: a launch below this can run from it
LARGE_WORKLOADS = {           # extra records of the default line
    "gmrf2048": "gmrf2048",        # the 2048^2 GMRF: column blocks that fit the Infinity Cache
    "hbm_bound": "gmrf5000_theta",  # n = 2.5e7: no block fits the cache, the steps stream from HBM
}


def parse():
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="grid1024_k0.1")
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--block-cols", type=int, default=0)
    p.add_argument("--dot-mode", choices=["auto", "forward", "squared"], default="auto")
    p.add_argument("--probe-dist", choices=["rademacher", "gaussian"], default="rademacher",
                   help="distribution of the probe entries (Alg. 3 step 2)")
    p.add_argument("--tile-order", choices=["auto", "bands", "interleaved"], default="auto",
                   help="row-tile order of the Newton-step launches (default: XCD bands unless the entries "
                        "crowd into a few row bands)")
    p.add_argument("--row-order", choices=["natural", "rcm", "degree", "random"], default="natural",
                   help="relabel the matrix rows before upload (symmetric permutation P A P^T): reverse "
                        "Cuthill-McKee, descending row length, or a seeded random order; the estimate is the "
                        "same up to the probes' row assignment")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-extras", action="store_true",
                   help="default workload only: leave out the CSR-path rate and the HBM-bound record")
    p.add_argument("--grad", action="store_true",
                   help="also time the gradient entry point against the estimate alone")
    p.add_argument("--calibrate-copy", action="store_true",
                   help="only run a 1 GiB device-to-device copy (reference for the memory counters)")
    p.add_argument("--adaptive-tol", type=float, default=0.0,
                   help="also time Alg. 2's adaptive loop (ld_apply_log_adaptive) on k Rademacher columns "
                        "with tol = this value times sqrt(n) (the norm of a probe), against the fixed degree")
    p.add_argument("--sweep", action="store_true",
                   help="only the theta sweep of the 5000 x 5000 GMRF I + theta*Adj (Sec. 5.2): one FP32 "
                        "estimate per theta against the closed-form log det, one JSON line")
    p.add_argument("--stats-summary", metavar="DIR",
                   help="only print a markdown table of the rocprofv3 --kernel-trace --stats CSV under DIR")
    p.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                          "COPY_WRITE_DIR"),
                   help="only print the copy-calibrated FETCH_SIZE/WRITE_SIZE bytes per launch of every kernel "
                        "from four rocprofv3 --pmc CSV directories (the workload's run under each counter, "
                        "then the --calibrate-copy run under each), with the current source hash")
    p.add_argument("--bench-log", metavar="FILE",
                   help="with --traffic-summary: the bench JSON line of the profiled run (algorithmic bytes)")
    p.add_argument("--all", action="store_true",
                   help="one JSON line per workload (FP32 and FP64, no CPU baseline), about 2 s of "
                        "timed work per precision each")
    return p.parse_args()


def calibrate_copy():
    """A plain copy of known size: the yardstick for the FETCH_SIZE/WRITE_SIZE counters."""
    import torch

    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")   # 1 GiB
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / 5
    print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                      "GBps": 2 * src.numel() * 4 / dt / 1e9}), flush=True)


def describe(name, cfg, n, nnz):
    if cfg["kind"] == "grid2d":
        shape = f"5-point Dirichlet Laplacian {cfg['N']}x{cfg['N']} grid"
        shift = f"{cfg.get('tau', 1.0)}*(L + {cfg['kappa2']} I)" if cfg.get("tau") else f"L + {cfg['kappa2']} I"
    elif cfg["kind"] == "grid3d":
        shape = f"7-point Dirichlet Laplacian {cfg['N']}^3 grid"
        shift = f"L + {cfg['kappa2']} I"
    elif cfg["kind"] == "penta":
        shape = "pentadiagonal Q + Q^T + n I with U(0,1) diagonals (Sec. 5.1)"
        shift = f"seed {cfg.get('seed', 0)}"
    elif cfg["kind"] == "gmrf_theta":
        shape = f"GMRF precision I + theta*Adj (4 neighbours) on a {cfg['N']}x{cfg['N']} grid"
        shift = f"theta = {cfg['theta']}"
    else:
        shape = "Chung-Lu power-law graph Laplacian (exponent 2.5, mean degree 16)"
        shift = "Lap + 0.01 I"
    return f"{name}: {shape}, {shift}, n={n}, nnz={nnz}, Leja degree {cfg['degree']}, {cfg['m_vec']} Rademacher queries"


def time_estimates(ld, A, lmin, lmax, degree, m_vec, seed, opts, steps, warmup):
    import torch

    ws = torch.empty(ld.workspace_size(A, degree, m_vec, False, opts), dtype=torch.uint8, device=A.val.device)
    for _ in range(warmup):
        ld.logdet(A, lmin, lmax, degree, m_vec, seed, options=opts, workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    est = None
    for _ in range(steps):
        est, stats = ld.logdet(A, lmin, lmax, degree, m_vec, seed, options=opts, workspace=ws,
                               return_stats=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return est, stats, dt


def theta_sweep(args):
    """log det Q(theta), Q = I + theta*Adj on 5000 x 5000, for the thetas of the stored sweep."""
    import numpy as np
    import torch

    import paper_2603_02207_amd as ld
    import workloads
    from tests.gpu_common import golden

    cfg = workloads.CONFIGS["gmrf5000_theta"]
    N, degree, m_vec = cfg["N"], cfg["degree"], cfg["m_vec"]
    row_ptr, col_idx, val, n = workloads.gmrf_theta(N, workloads.GMRF_THETAS[0])
    A = ld.CSR.from_arrays(row_ptr, col_idx, val.astype(np.float32), n, device="cuda:0", dtype=torch.float32)
    diag = torch.tensor(val == 1.0, device="cuda:0")
    g = golden("gmrf5000_theta_sweep")
    opts = ld.Options(trusted_csr=1)
    rows = []
    t_all = time.perf_counter()
    for th in workloads.GMRF_THETAS:
        At = A.with_values(torch.where(diag, torch.ones_like(A.val), torch.full_like(A.val, th)))
        lmin, lmax = ld.spectral_bounds(At)
        est, st, dt = time_estimates(ld, At, lmin, lmax, degree, m_vec, args.seed, opts, 3, 1)
        r = g["results"][repr(th)] if g else None
        row = {"theta": th, "lmin": lmin, "lmax": lmax, "estimate_f32": est, "ms_per_estimate": dt / 3 * 1e3}
        if r is not None:
            row.update(logdet_exact=r["logdet_exact"], rel_err_vs_exact=abs(est - r["logdet_exact"]) /
                       abs(r["logdet_exact"]), z=(est - r["expectation"]) / r["sd_hutchinson"])
        rows.append(row)
    ms = [r["ms_per_estimate"] for r in rows]
    return {"metric": "theta sweep of log det Q(theta), GMRF of Sec. 5.2", "workload":
            describe("gmrf5000_theta", cfg, n, int(len(col_idx))), "n": n, "nnz": int(len(col_idx)),
            "degree": degree, "m_vec": m_vec, "dtype": "f32", "estimates_per_s": 1e3 / float(np.mean(ms)),
            "sweep_seconds": time.perf_counter() - t_all, "points": rows}


def time_adaptive(ld, A, lmin, lmax, degree, ncols, rel_tol, n, nnz, reps=5):
    """Alg. 2's adaptive loop against the fixed-degree apply on the same Rademacher block."""
    import numpy as np
    import torch

    g = torch.Generator(device="cpu").manual_seed(1)
    V = (torch.randint(0, 2, (n, ncols), generator=g, dtype=torch.int8) * 2 - 1).to(A.val.device, A.dtype)
    tol = rel_tol * math.sqrt(n)
    out = {}
    for name, fn in (("adaptive", lambda: ld.apply_log_adaptive(A, lmin, lmax, degree, tol, V)),
                     ("fixed", lambda: (ld.apply_log(A, lmin, lmax, degree, V), None))):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            _, deg = fn()
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t) / reps
        if deg is not None:
            degs = np.asarray(deg)
    mx = int(degs.max())                                        # steps launched: until a poll sees all stopped
    steps = min(degree, next(p for p in (1, 2, 4) if p >= mx) if mx <= 4 else -(-mx // 8) * 8)
    step_bytes = 8.0 * nnz + 4.0 * (n + 1) + 16.0 * n * ncols   # A + read w, write w, read and write P
    return {"tol": tol, "tol_over_sqrt_n": rel_tol, "columns": ncols, "max_degree": degree,
            "degree_min": int(degs.min()), "degree_median": float(np.median(degs)), "degree_max": int(degs.max()),
            "ms_adaptive": out["adaptive"] * 1e3, "ms_fixed_degree_horner": out["fixed"] * 1e3,
            "steps_launched": steps, "adaptive_GBps": steps * step_bytes / out["adaptive"] / 1e9}


def time_adaptive_estimate(ld, A, lmin, lmax, degree, m_vec, seed, rel_tol, n, s_fixed, reps=3):
    """Alg. 3 with Alg. 2's stopping rule (tol = rel_tol * sqrt(n), the degree as the
    cap) against the fixed-degree estimate of the same call."""
    import numpy as np
    import torch

    tol = rel_tol * math.sqrt(n)
    ld.logdet_adaptive(A, lmin, lmax, degree, tol, m_vec, seed)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        est, deg, st = ld.logdet_adaptive(A, lmin, lmax, degree, tol, m_vec, seed, return_stats=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    k = st["k"]
    return {"tol": tol, "tol_over_sqrt_n": rel_tol, "max_degree": degree, "estimate": est,
            "ms_per_estimate": dt * 1e3, "over_fixed_degree": dt / s_fixed,
            "degrees_sketch": sorted(set(int(x) for x in deg[:k])),
            "degrees_basis": sorted(set(int(x) for x in deg[k:2 * k])),
            "degrees_residual": sorted(set(int(x) for x in deg[2 * k:])),
            "newton_steps": [st["launches1"], st["launches23"]],
            "note": "forward Newton form with the accumulator (Alg. 2 as printed), no Horner or squared basis"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(csr, lmin, lmax, degree, m_vec, seed):
    """The FP64 oracle, one complete estimate of the same workload on the host."""
    from threadpoolctl import threadpool_info

    import workloads
    from oracle import hutchpp

    Q = workloads.to_scipy(csr)
    blas = [(i.get("internal_api"), i.get("num_threads")) for i in threadpool_info()]
    threads = max([t for _, t in blas if t] or [1])
    t = time.perf_counter()
    hutchpp.logdet_estimate(Q, lmin, lmax, degree, m_vec, seed)
    full = time.perf_counter() - t
    return {
        "value": 1.0 / full,
        "unit": "logdet estimates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"one complete FP64 oracle estimate (NumPy/SciPy, Alg. 3 with Léja points and the "
                   f"divided differences computed in the call) of the same workload at Leja degree {degree} "
                   f"with all {m_vec} queries: {full:.1f} s. Host: {os.cpu_count()} logical CPUs "
                   f"({cpu_model()}); BLAS pools {blas} (the dense QR and block products may use them, "
                   f"SciPy's CSR x dense product runs on one thread). The GPU library caches its Léja "
                   f"table and Alg. 1 results across calls, so its timed estimates exclude them (the "
                   f"'host_alg1_ms' field gives one uncached Alg. 1 call)."),
    }


# counter-measured bytes per launch, one summary per workload (written by
# `bench.py --traffic-summary`), used while the library sources are unchanged
TRAFFIC_PROFILE = "profiles/step_kernel_{workload}_traffic.md"
# the step kernels of the two phases, as rocprofv3 names them (template
# argument 3 = step kind: 0 sketch with probe signs, 3 / 2 quadratic forms)
KERNEL_PREFIXES = {
    ("sketch_horner", "step_kernel"): ("step_kernel<float, 4, 0, false",),
    ("sketch_horner", "dia_flat_kernel"): ("dia_flat_kernel<float, 4, 0,",),
    ("quadform", "step_kernel"): ("step_kernel<float, 4, 3, false", "step_kernel<float, 4, 2, false"),
}


def step_kernel_name(tag: str, st) -> str:
    """Kernel of a phase's Newton steps: on diagonal storage the sketch's
    steps (no column sums) take the one-chunk-per-thread kernel."""
    return "dia_flat_kernel" if tag == "sketch_horner" and st.get("dia_diagonals") else "step_kernel"


def source_hash() -> str:
    from paper_2603_02207_amd.build import source_hash as h

    return h()


def traffic_blob(workload: str):
    path = os.path.join(ROOT, TRAFFIC_PROFILE.format(workload=workload))
    if not os.path.exists(path):
        return None
    text = open(path).read()
    try:
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (IndexError, ValueError):
        return None
    return blob if blob.get("source_hash") == source_hash() else None   # else the kernels changed since


def measured_traffic(tag: str, workload: str, kernel: str):
    """Counter-measured bytes per launch of a step kernel, if taken on the current sources."""
    blob = traffic_blob(workload)
    if blob is None:
        return None
    for name, mb in blob.get("traffic_MB_per_launch", {}).items():
        if any(name.startswith(p) for p in KERNEL_PREFIXES.get((tag, kernel), ())):
            return mb * 1e6
    return None


def copy_GBps(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """A plain device-to-device copy of `nbytes` (read + write bytes / time)."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes / dt / 1e9


def method_bytes_per_estimate(n, nnz, degree, k, kg, elem=4):
    """The method's plain bytes per estimate: each Newton step reads the CSR
    matrix once (values + int32 indices + row pointers); the sketch step
    reads and writes the block and reads and writes the accumulator of
    Alg. 2 (16 B per element in FP32), the quadratic-form step reads and
    writes the block and reads X (12 B per element); m steps each."""
    a = (elem + 4.0) * nnz + 4.0 * (n + 1)
    return degree * ((a + 4.0 * elem * n * k) + (a + 3.0 * elem * n * (k + kg)))


def short_kernel_name(name: str) -> str:
    """`void ld::(anonymous namespace)::k<T, ...>(args)` -> `k<T, ...>`."""
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    name = name.replace("ld::(anonymous namespace)::", "")
    if name.startswith("ld::"):
        name = name[4:]
    depth = 0
    for i, ch in enumerate(name):          # drop the argument list (outside template brackets)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def find_csv(d: str, suffix: str) -> str:
    import glob

    hits = sorted(glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True))
    if not hits:
        raise SystemExit(f"no *{suffix} under {d}")
    return hits[0]


def stats_summary(d: str) -> str:
    import csv

    rows = list(csv.DictReader(open(find_csv(d, "kernel_stats.csv"))))
    out = ["| kernel | calls | avg us | total ms | % |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {short_kernel_name(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def counter_means(d: str):
    """Mean counter value (KiB) per dispatch of each kernel."""
    import csv
    from collections import defaultdict

    per = defaultdict(lambda: defaultdict(float))   # kernel -> dispatch -> value (summed over instances)
    for r in csv.DictReader(open(find_csv(d, "counter_collection.csv"))):
        per[short_kernel_name(r["Kernel_Name"])][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: sum(v.values()) / len(v) for k, v in per.items()}


def traffic_summary(dirs, bench_log=None) -> str:
    fetch, write, cfetch, cwrite = (counter_means(d) for d in dirs)
    copy_kib = (1 << 30) / 1024.0
    ck = max(cfetch, key=lambda k: cfetch[k] if "copy" in k else -1)
    f_scale, w_scale = copy_kib / cfetch[ck], copy_kib / cwrite[ck]
    alg = {}
    if bench_log:
        line = [l for l in open(bench_log) if l.startswith("{")][-1]
        for tag, rec in json.loads(line).get("kernels", {}).items():
            alg[tag] = rec
    lines = [f"Scale factors from the 1 GiB copy ({copy_kib:.0f} KiB read and written): FETCH_SIZE reads "
             f"{cfetch[ck]:.1f} KiB -> x{f_scale:.4f}; WRITE_SIZE reads {cwrite[ck]:.1f} KiB -> x{w_scale:.4f}.",
             "", f"Library source hash: {source_hash()}", "",
             "| kernel | read MB/launch (scaled) | write MB/launch (scaled) | total MB/launch | algorithmic MB | "
             "total / algorithmic |", "|---|---|---|---|---|---|"]
    blob = {}
    for k in sorted(set(fetch) | set(write)):
        if k.startswith("at::") or k.startswith("__amd"):   # torch's copy and runtime fills
            continue
        r = fetch.get(k, 0.0) * f_scale * 1024 / 1e6
        w = write.get(k, 0.0) * w_scale * 1024 / 1e6
        a = ""
        ratio = ""
        for tag, rec in alg.items():
            prefixes = KERNEL_PREFIXES.get((tag, rec["kernel"]), ())
            # a library launch of a step kernel may be several dispatches over row ranges
            if any(k.startswith(p.replace(", false", "")) for p in prefixes):
                r, w = (x * rec.get("dispatches_per_launch", 1) for x in (r, w))
            # (a step kernel's first-step variant, ", true, ...", is not the phase's typical launch)
            if any(k.startswith(p) for p in prefixes) and not (k.startswith("step_kernel") and ", true," in k):
                a = f"{rec['bytes_per_launch'] / 1e6:.1f}"
                ratio = f"{(r + w) / (rec['bytes_per_launch'] / 1e6):.2f}"
        lines.append(f"| {k[:160]} | {r:.1f} | {w:.1f} | {r + w:.1f} | {a} | {ratio} |")
        blob[k] = round(r + w, 3)
    lines += ["", "Machine-readable (bench.py reads it while the source hash matches):", "", "```json",
              json.dumps({"source_hash": source_hash(), "traffic_MB_per_launch": blob}), "```"]
    return "\n".join(lines)


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.stats_summary:
        print(stats_summary(args.stats_summary))
        return
    if args.traffic_summary:
        print(traffic_summary(args.traffic_summary, args.bench_log))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on exactly one GPU; --gpus must be 1 "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.sweep:
        print(json.dumps(theta_sweep(args)), flush=True)
        return
    if not args.all:
        # the default line carries the CSR-path rate and the HBM-bound record too
        args.extras = args.workload == "grid1024_k0.1" and not args.no_extras
        out = run_workload(args, args.workload, args.steps)
        if args.extras:
            torch.cuda.empty_cache()
            for key, name in LARGE_WORKLOADS.items():
                out[key] = large_record(args, name)
                torch.cuda.empty_cache()
        print(json.dumps(out), flush=True)
        return
    args.extras = False
    for name in workloads.CONFIGS:
        args.no_cpu_baseline = True
        out = run_workload(args, name, None)
        print(json.dumps(out), flush=True)
        torch.cuda.empty_cache()


def relabel(csr, order):
    """P A P^T for a row order: reverse Cuthill-McKee, descending row length, or random (seed 0)."""
    import numpy as np
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee

    import workloads

    Q = workloads.to_scipy(csr)
    if order == "rcm":
        perm = reverse_cuthill_mckee(Q, symmetric_mode=True)
    elif order == "degree":
        perm = np.argsort(-np.diff(csr[0]), kind="stable")
    else:
        perm = np.random.default_rng(0).permutation(csr[3])
    P = sp.csr_matrix(Q[perm][:, perm])
    P.sort_indices()
    return P.indptr.astype(np.int32), P.indices.astype(np.int32), P.data, P.shape[0]


def kernel_records(st):
    """Per-phase step-kernel records from the library's HIP-event timings."""
    kernels = {}
    for tag, ms, nl, by in (("sketch_horner", st["ms_steps1"], st["launches1"], st["bytes1"]),
                            ("quadform", st["ms_steps23"], st["launches23"], st["bytes23"])):
        if nl:
            avg_s = ms / 1e3 / nl
            kernels[tag] = {"kernel": step_kernel_name(tag, st), "launches": nl, "avg_us": avg_s * 1e6,
                            "bytes_per_launch": by / nl,
                            "GBps": by / nl / avg_s / 1e9, "total_ms": ms,
                            # kernel dispatches per library launch (row ranges of a streaming step)
                            "dispatches_per_launch": st.get("ranges23", 1) if tag == "quadform" else 1}
    return kernels


def run_workload(args, workload, steps):
    """One bench record for `workload`; steps=None: as many as fit about 2 s."""
    import numpy as np
    import torch

    import paper_2603_02207_amd as ld
    import workloads
    from tests.gpu_common import golden

    dev = "cuda:0"
    args.workload = workload
    cfg = dict(workloads.CONFIGS[args.workload])
    csr = workloads.build(args.workload)
    reorder_s = 0.0
    if args.row_order != "natural":
        t = time.perf_counter()
        csr = relabel(csr, args.row_order)
        reorder_s = time.perf_counter() - t
    row_ptr, col_idx, val, n = csr
    nnz = int(len(col_idx))
    degree, m_vec = cfg["degree"], cfg["m_vec"]
    mode = {"auto": ld.LD_DOT_AUTO, "forward": ld.LD_DOT_FORWARD, "squared": ld.LD_DOT_SQUARED}[args.dot_mode]

    A32 = ld.CSR.from_arrays(row_ptr, col_idx, val, n, device=dev, dtype=torch.float32)
    g = golden(args.workload)
    if g is not None and g.get("degree") == degree and g.get("m_vec") == m_vec and cfg["kind"] != "penta":
        # the oracle's own interval (Gershgorin of the FP64 values): the estimates
        # below and the stored oracle value then share every input but the FP32
        # rounding of the matrix values
        lmin, lmax = g["lmin"], g["lmax"]
        bounds_from = "oracle (Gershgorin of the FP64 values)"
    else:
        lmin, lmax = ld.spectral_bounds(A32)           # Gershgorin on the device (also checks the CSR)
        bounds_from = "Gershgorin on the device"
    A64 = ld.CSR.from_arrays(row_ptr, col_idx, val, n, device=dev, dtype=torch.float64)
    tiles = {"auto": 0, "bands": 1, "interleaved": 2}[args.tile_order]
    opts = ld.Options(block_cols=args.block_cols, dot_mode=mode, trusted_csr=1, tile_order=tiles,
                      probe_dist={"rademacher": 0, "gaussian": 1}[args.probe_dist])
    t = time.perf_counter()
    ld.logdet(A32, lmin, lmax, degree, m_vec, args.seed)   # validated call
    torch.cuda.synchronize()
    if steps is None:
        steps = int(min(20, max(3, 2.0 / max(time.perf_counter() - t, 1e-3))))
    args.steps = steps

    est32, st, dt = time_estimates(ld, A32, lmin, lmax, degree, m_vec, args.seed, opts, args.steps,
                                   args.warmup)
    value = args.steps / dt

    # dominant recurrence kernel, timed by HIP events on the launch stream
    kernels = kernel_records(st)
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    achieved = kernels[dom]["GBps"]
    traffic = (measured_traffic(dom, args.workload, kernels[dom]["kernel"])
               if args.block_cols == 0 and args.dot_mode == "auto" else None)
    total_bytes = st["bytes1"] + st["bytes23"]
    total_ms = st["ms_steps1"] + st["ms_steps23"]
    # a launch whose bytes fit the Infinity Cache streams (largely) from it:
    # its GB/s is then not an HBM bandwidth
    in_cache = kernels[dom]["bytes_per_launch"] <= INFINITY_CACHE_BYTES
    method = method_bytes_per_estimate(n, nnz, degree, st["k"], st["k_G"])

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "logdet estimates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": describe(args.workload, cfg, n, nnz),
            "degree": degree,
            "m_vec": m_vec,
            "k": st["k"],
            "k_G": st["k_G"],
            "lmin": lmin,
            "lmax": lmax,
            "bounds": bounds_from,
            "dot_mode": {1: "forward", 2: "squared"}[st["dot_mode_used"]],
            "matrix_storage": ((f"diagonal ({st['dia_diagonals']} diagonals" +
                                (", one value each, presence bits per row)" if st.get("dia_constant") else ")"))
                               if st.get("dia_diagonals") else "csr"),
            "block_cols": args.block_cols,
            "column_blocks": {"sketch": st["block_cols1"], "quadform": st["block_cols23"]},
            "tile_order": {1: "bands", 2: "interleaved"}[st["tile_order_used"]],
            "probes": args.probe_dist,
            "seed": args.seed,
            "row_order": args.row_order + (f" (host relabelling {reorder_s:.1f} s, before upload)"
                                           if args.row_order != "natural" else ""),
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "infinity_cache" if in_cache else "hbm",
            "kernel": f"{kernels[dom]['kernel']} ({dom})",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "alg_bytes_per_launch": kernels[dom]["bytes_per_launch"],
            "working_set": (f"{kernels[dom]['bytes_per_launch'] / 1e6:.0f} MB per launch "
                            + ("<= the 256 MB Infinity Cache: the blocks stream from the cache, so frac "
                               "against the HBM peak is not an HBM efficiency (hbm_bound: a workload whose "
                               "blocks cannot fit it)" if in_cache
                               else "> the 256 MB Infinity Cache: the blocks stream from HBM")),
        },
        "spmm_recurrence_GBps": total_bytes / (total_ms / 1e3) / 1e9,
        "kernels": kernels,
        "alg_bytes": {
            "implementation_GB_per_estimate": total_bytes / 1e9,
            "method_GB_per_estimate": method / 1e9,
            "reformulation_factor": method / total_bytes,
            "note": ("method: Alg. 2 forward steps over the CSR matrix (8 B per entry + row pointers) for the "
                     "sketch (16 B per block element: read and write the block and the accumulator) and the "
                     "quadratic forms (12 B: read and write the block, read X), m steps each; "
                     "implementation: the sketch in Horner order (8 B per element + one sign word per row), "
                     "the quadratic forms in the squared Newton basis (ceil(m/2) steps, 8 B per element) and "
                     "the matrix in diagonal storage when it has one (presence bits only for constant "
                     "diagonals)"),
        },
        "phase_ms": {"sketch": st["ms_phase1"], "cholqr_deflation": st["ms_qr"], "quadform": st["ms_phase23"]},
        "estimate_f32": est32,
    }

    if cfg["kind"] == "penta":        # banded-Cholesky log det of the same values (stored)
        gp = golden(args.workload)
        if gp is not None and "logdet_exact_f32_values" in gp:
            out["parity_exact"] = {"logdet_exact_f32_values": gp["logdet_exact_f32_values"],
                                   "rel_err_f32_vs_exact": abs(est32 - gp["logdet_exact_f32_values"]) /
                                   abs(gp["logdet_exact_f32_values"])}
    if cfg["kind"] == "gmrf_theta":   # closed form of the stored sweep (exact log det, expectation, sd)
        gs = golden("gmrf5000_theta_sweep")
        r = gs["results"].get(repr(cfg["theta"])) if gs and gs["N"] == cfg["N"] else None
        if r is not None:
            out["parity"] = {"logdet_exact": r["logdet_exact"], "expectation": r["expectation"],
                             "rel_err_f32_vs_exact": abs(est32 - r["logdet_exact"]) / abs(r["logdet_exact"])}
            if args.probe_dist == "rademacher":   # the stored sd is Rademacher Hutchinson's
                out["parity"]["z_f32"] = (est32 - r["expectation"]) / r["sd_hutchinson"]
    ref = None
    if (g is not None and args.probe_dist == "rademacher" and str(args.seed) in g["results"]
            and g["degree"] == degree and bounds_from.startswith("oracle")):   # stored values: Rademacher
        ref = g["results"][str(args.seed)]["logdet"]
        out["parity"] = {"oracle_fp64": ref, "rel_err_f32": abs(est32 - ref) / abs(ref)}

    if not args.no_fp64:
        k64 = max(2, args.steps // 4)
        est64, st64, dt64 = time_estimates(ld, A64, lmin, lmax, degree, m_vec, args.seed, opts, k64, 1)
        out["fp64"] = {"value": k64 / dt64, "ms_per_step": dt64 / k64 * 1e3, "estimate": est64,
                       "spmm_recurrence_GBps": (st64["bytes1"] + st64["bytes23"]) /
                       ((st64["ms_steps1"] + st64["ms_steps23"]) / 1e3) / 1e9}
        if ref is not None:
            out["parity"]["rel_err_f64"] = abs(est64 - ref) / abs(ref)
        out["parity_f32_vs_f64"] = abs(est32 - est64) / abs(est64)

    if args.grad:
        k_g = max(2, args.steps // 4)
        ld.logdet_with_grad(A32, lmin, lmax, degree, m_vec, args.seed, options=opts)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k_g):
            _, _, stg = ld.logdet_with_grad(A32, lmin, lmax, degree, m_vec, args.seed, options=opts,
                                            return_stats=True)
        torch.cuda.synchronize()
        dtg = (time.perf_counter() - t) / k_g
        t_est = dt / args.steps * 1e3
        out["gradient"] = {"ms_estimate_and_gradient": dtg * 1e3, "ms_estimate": t_est,
                           "ms_gradient_part": stg["ms_adjoint"],
                           "call_over_estimate": dtg * 1e3 / t_est,
                           "extra_over_estimate": (dtg * 1e3 - t_est) / t_est,
                           "path": {2: "squared Newton basis", 1: "Newton form"}[stg["dot_mode_used"]],
                           "ckpt_stride": "auto (every stored vector kept when they fit 64 GiB)",
                           "workspace_GB": ld.workspace_size(A32, degree, m_vec, True, opts) / 1e9}
        # the estimate in the gradient's layout (one column block per phase):
        # its default blocks may run from the Infinity Cache, the gradient's
        # stored vectors cannot
        o_one = ld.Options(block_cols=64, dot_mode=mode, trusted_csr=1, tile_order=tiles)
        _, st_one, dt_one = time_estimates(ld, A32, lmin, lmax, degree, m_vec, args.seed, o_one, k_g, 1)
        t_one = dt_one / k_g * 1e3
        out["gradient"]["one_block_estimate"] = {
            "column_blocks": {"sketch": st_one["block_cols1"], "quadform": st_one["block_cols23"]},
            "ms_estimate": t_one, "call_over_estimate": dtg * 1e3 / t_one}
        # sqrt(m) checkpoints: a fraction of the memory, segments recomputed
        s_ck = max(1, math.ceil(math.sqrt(degree)))
        o_ck = ld.Options(block_cols=args.block_cols, dot_mode=mode, trusted_csr=1, tile_order=tiles,
                          ckpt_stride=s_ck)
        ld.logdet_with_grad(A32, lmin, lmax, degree, m_vec, args.seed, options=o_ck)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k_g):
            ld.logdet_with_grad(A32, lmin, lmax, degree, m_vec, args.seed, options=o_ck)
        torch.cuda.synchronize()
        dtc = (time.perf_counter() - t) / k_g
        out["gradient"]["sqrt_m_checkpoints"] = {
            "ckpt_stride": s_ck, "ms_estimate_and_gradient": dtc * 1e3, "call_over_estimate": dtc * 1e3 / t_est,
            "workspace_GB": ld.workspace_size(A32, degree, m_vec, True, o_ck) / 1e9}

    if args.adaptive_tol > 0:
        out["apply_log_adaptive"] = time_adaptive(ld, A32, lmin, lmax, degree, st["k"], args.adaptive_tol, n,
                                                  nnz)
        out["logdet_adaptive"] = time_adaptive_estimate(ld, A32, lmin, lmax, degree, m_vec, args.seed,
                                                        args.adaptive_tol, n, dt / args.steps)

    if args.extras:
        # the same workload on the CSR path (no diagonal storage): the general SpMM kernels
        o_csr = ld.Options(block_cols=args.block_cols, dot_mode=mode, trusted_csr=1, tile_order=tiles,
                           csr_only=1)
        k_c = max(3, args.steps // 2)
        e_c, st_c, dt_c = time_estimates(ld, A32, lmin, lmax, degree, m_vec, args.seed, o_csr, k_c, 1)
        kc = kernel_records(st_c)
        out["csr_only"] = {"value": k_c / dt_c, "ms_per_step": dt_c / k_c * 1e3, "estimate": e_c,
                           "matrix_storage": "csr" if not st_c["dia_diagonals"] else "diagonal",
                           "kernels": kc,
                           "spmm_recurrence_GBps": (st_c["bytes1"] + st_c["bytes23"]) /
                           ((st_c["ms_steps1"] + st_c["ms_steps23"]) / 1e3) / 1e9}
        # one Alg. 1 call that misses the library's cache (an interval not used before)
        t = time.perf_counter()
        ld.divided_differences(1.0, (lmax / lmin) * (1.0 + 1e-9 * (1 + time.time() % 1)), degree)
        out["host_alg1_ms"] = (time.perf_counter() - t) * 1e3

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline((row_ptr, col_idx, np.asarray(val), n), lmin, lmax, degree,
                                           m_vec, args.seed)
    return out


def large_record(args, name):
    """A large workload in FP32: estimates/s, its dominant step kernel against
    8 TB/s and against a 1 GiB copy measured here, whether its launches fit the
    Infinity Cache, and counter bytes if taken on the current sources."""
    import torch

    import paper_2603_02207_amd as ld
    import workloads

    cfg = dict(workloads.CONFIGS[name])
    row_ptr, col_idx, val, n = workloads.build(name)
    nnz = int(len(col_idx))
    A = ld.CSR.from_arrays(row_ptr, col_idx, val, n, device="cuda:0", dtype=torch.float32)
    del row_ptr, col_idx, val
    lmin, lmax = ld.spectral_bounds(A)
    opts = ld.Options(trusted_csr=1)
    est, st, dt = time_estimates(ld, A, lmin, lmax, cfg["degree"], cfg["m_vec"], args.seed, opts, 5, 1)
    kernels = kernel_records(st)
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    for tag, rec in kernels.items():
        t = measured_traffic(tag, name, rec["kernel"])
        rec["traffic_bytes_per_launch"] = t
        rec["traffic_over_alg"] = t / rec["bytes_per_launch"] if t else None
    del A
    torch.cuda.empty_cache()
    copy = copy_GBps()
    return {
        "workload": describe(name, cfg, n, nnz),
        "dtype": "f32",
        "value": 5 / dt,
        "unit": "logdet estimates/s",
        "ms_per_estimate": dt / 5 * 1e3,
        "estimate_f32": est,
        "matrix_storage": ((f"diagonal ({st['dia_diagonals']} diagonals" +
                            (", one value each)" if st.get("dia_constant") else ")"))
                           if st.get("dia_diagonals") else "csr"),
        "column_blocks": {"sketch": st["block_cols1"], "quadform": st["block_cols23"]},
        "dominant_kernel": f"{kernels[dom]['kernel']} ({dom})",
        "bound": "infinity_cache" if kernels[dom]["bytes_per_launch"] <= INFINITY_CACHE_BYTES else "hbm",
        "avg_us": kernels[dom]["avg_us"],
        "alg_bytes_per_launch": kernels[dom]["bytes_per_launch"],
        "achieved_GBps": kernels[dom]["GBps"],
        "frac_of_8TBps": kernels[dom]["GBps"] / HBM_PEAK_GBS,
        "copy_1GiB_GBps": copy,
        "frac_of_copy": kernels[dom]["GBps"] / copy,
        "traffic_bytes_per_launch": kernels[dom]["traffic_bytes_per_launch"],
        "kernels": kernels,
        "spmm_recurrence_GBps": (st["bytes1"] + st["bytes23"]) / ((st["ms_steps1"] + st["ms_steps23"]) / 1e3) / 1e9,
    }


if __name__ == "__main__":
    main()
