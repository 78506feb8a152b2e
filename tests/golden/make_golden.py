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
from oracle import bounds, hutchpp  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# name -> (workload, overrides, seeds)
ENTRIES = {
    "grid32_k0.5": ("grid32_k0.5", {}, list(range(5))),
    "grid1024_k0.1": ("grid1024_k0.1", {}, [0]),
    "gmrf2048": ("gmrf2048", {}, [0]),
    "grid128c_k0.05": ("grid128c_k0.05", {}, [0]),
    "chunglu_1M": ("chunglu_4M", {"n": 1 << 20}, [0]),
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
    for s in seeds:
        t = time.perf_counter()
        parts = hutchpp.logdet_estimate(Q, lmin, lmax, cfg["degree"], cfg["m_vec"], s, return_parts=True)
        out["results"][str(s)] = dict(logdet=parts["logdet"], t_low=parts["t_low"], t_res=parts["t_res"],
                                      seconds=time.perf_counter() - t)
        print(name, s, parts["logdet"], f"{time.perf_counter() - t:.1f}s", flush=True)
    with open(os.path.join(HERE, f"{name}.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(ENTRIES):
        make(nm)
