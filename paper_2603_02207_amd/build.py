"""Build the native library ``libleja_logdet.so`` for gfx950 with hipcc.

Usage:  python -m paper_2603_02207_amd.build   (or python paper_2603_02207_amd/build.py)
The shared object is written next to this file, so it travels with the tree.
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libleja_logdet.so")
SOURCES = ["host_math.cpp", "kernels.hip", "api.hip"]

HIPCC_FLAGS = [
    "-O3",
    "-std=c++17",
    "--offload-arch=gfx950",
    "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def source_files():
    """The files the library is built from: csrc/* and include/*.h (sorted relative paths)."""
    out = []
    for sub, keep in ((os.path.join("paper_2603_02207_amd", "csrc"), lambda f: True),
                      ("include", lambda f: f.endswith(".h"))):
        d = os.path.join(ROOT, sub)
        out += [os.path.join(sub, f) for f in os.listdir(d) if keep(f) and os.path.isfile(os.path.join(d, f))]
    return sorted(out)


def source_hash() -> str:
    """First 16 hex digits of SHA-256 over (path, contents) of every source file."""
    h = hashlib.sha256()
    for rel in source_files():
        h.update(rel.replace(os.sep, "/").encode() + b"\0")
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
        h.update(b"\0")
    return h.hexdigest()[:16]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    # the library reports the hash of the sources it was built from (ld_version)
    ident = ["-DLD_SOURCE_HASH=\"" + source_hash() + "\""]
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, jobs = [], []
    for src in SOURCES:   # the three translation units compile in parallel
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc()] + HIPCC_FLAGS + ident + inc + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        objs.append(obj)
    for src, proc in jobs:
        out, _ = proc.communicate()
        msgs = "\n".join(l for l in out.splitlines() if "packed-fp32-ops" not in l)
        if proc.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{msgs}")
        if verbose and msgs.strip():
            print(msgs)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
