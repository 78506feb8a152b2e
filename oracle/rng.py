"""Rademacher (and Gaussian) probes from a counter-based SplitMix64 generator (oracle side).

The paper draws the sketch S and the residual probes with i.i.d. entries of
+1/-1 with probability 1/2 (Sec. 4.1; Alg. 3 step 2) and fixes no generator.
Both this oracle and the GPU library implement the same published generator so
that they see identical probes: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014;
reference C code by S. Vigna).  Its i-th output (i = 1, 2, ...) from state s0 is
mix(s0 + i*0x9E3779B97F4A7C15), with the mixing function

    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
    z ^= z >> 27; z *= 0x94D049BB133111EB;
    z ^= z >> 31.

Layout of the probe stream (a reading of an unspecified point):
    key(seed, stream)   = output number (stream+1) of SplitMix64(seed)
    entry(row, col)     = +1 if the top bit of output number (col*n + row + 1)
                          of SplitMix64(key) is 0, else -1.
Stream 0 is the sketch S, stream 1 the residual probes G.  Entries depend only
on (seed, stream, n, row, col), not on any blocking.

Gaussian probes (the paper's alternative to Rademacher, Alg. 3 step 2; no
generator fixed either) use the same outputs, one per entry (a reading): with
x = output number (col*n + row + 1) of SplitMix64(key),
    u1 = ((x >> 32) + 1/2) / 2^32,  u2 = ((x mod 2^32) + 1/2) / 2^32,
    entry(row, col) = sqrt(-2 ln u1) * cos(2 pi u2)          (Box-Muller),
evaluated in FP64.

Pinned by: the published SplitMix64 test vector (outputs for seed 1234567),
balance/independence statistics, and for the Gaussian entries a
Kolmogorov-Smirnov test against the standard normal, its moments and
column independence (tests/test_oracle_rng.py).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def mix(z):
    """SplitMix64 output function on a uint64 array (wrapping arithmetic)."""
    z = np.array(z, dtype=np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= M1
        z ^= z >> np.uint64(27)
        z *= M2
        z ^= z >> np.uint64(31)
    return z


def splitmix64_outputs(state: int, count: int, start: int = 1):
    """Outputs number start .. start+count-1 of SplitMix64 seeded with ``state``."""
    i = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(state) + i * GOLDEN
    return mix(z)


def stream_key(seed: int, stream: int) -> int:
    return int(splitmix64_outputs(int(seed) & 0xFFFFFFFFFFFFFFFF, 1, start=stream + 1)[0])


def rademacher(seed: int, stream: int, n: int, ncols: int) -> np.ndarray:
    """n x ncols float64 matrix of +-1 entries (column-major index col*n + row)."""
    key = stream_key(seed, stream)
    out = np.empty((n, ncols), dtype=np.float64)
    for c in range(ncols):
        x = splitmix64_outputs(key, n, start=c * n + 1)
        out[:, c] = np.where((x >> np.uint64(63)) != 0, -1.0, 1.0)
    return out


def gaussian(seed: int, stream: int, n: int, ncols: int) -> np.ndarray:
    """n x ncols float64 standard normal entries (Box-Muller on one output per entry)."""
    key = stream_key(seed, stream)
    out = np.empty((n, ncols), dtype=np.float64)
    two32 = float(2 ** 32)
    for c in range(ncols):
        x = splitmix64_outputs(key, n, start=c * n + 1)
        u1 = ((x >> np.uint64(32)).astype(np.float64) + 0.5) / two32
        u2 = ((x & np.uint64(0xFFFFFFFF)).astype(np.float64) + 0.5) / two32
        out[:, c] = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return out


def probes(kind: str, seed: int, stream: int, n: int, ncols: int) -> np.ndarray:
    """Probe block of the given distribution: "rademacher" or "gaussian"."""
    if kind == "rademacher":
        return rademacher(seed, stream, n, ncols)
    if kind == "gaussian":
        return gaussian(seed, stream, n, ncols)
    raise ValueError(f"unknown probe distribution {kind!r}")
