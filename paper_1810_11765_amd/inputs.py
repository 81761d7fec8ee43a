"""Seeded synthetic inputs for the SMMO workloads.

This module only produces starting states and instance lists from a seed; it
holds none of the allocator's or the workloads' arithmetic.  The GPU path and
the CPU oracle both start from what it returns.

Randomness is SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): ``splitmix64(x)``
is the first output of the generator seeded with ``x`` (add the golden gamma,
then the 64-bit finalizer).  A draw keyed on (seed, step, id, stream) is
``ctr = sm(sm(sm(seed ^ (stream << 56)) ^ step) ^ id)``; ``u24(h) = h >> 40``
and ``U01(h) = u24(h) * 2**-24`` (exact in float32).

The paper's own benchmark inputs are described only on its project wiki
(Sec. 6); these generators stand in for them with the shapes of Table 1's
apps (game of life, wa-tor, collision/n-body, Linux Scalability).
"""
from __future__ import annotations

import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x) -> np.ndarray:
    """First SplitMix64 output for each seed in ``x`` (uint64, wrapping)."""
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def ctr(seed: int, step: int, ids, stream: int) -> np.ndarray:
    """Counter-based draw keyed on (seed, step, id, stream)."""
    h = splitmix64(np.uint64(seed) ^ (np.uint64(stream) << np.uint64(56)))
    h = splitmix64(h ^ np.uint64(step))
    return splitmix64(h ^ np.asarray(ids, dtype=np.uint64))


def u24(h) -> np.ndarray:
    return (np.asarray(h, dtype=np.uint64) >> np.uint64(40)).astype(np.int64)


def u01(h) -> np.ndarray:
    return u24(h).astype(np.float32) * np.float32(1.0 / 16777216.0)


def threshold(p: float) -> int:
    """Bernoulli(p) is ``u24 < threshold(p)``."""
    return int(round(p * 16777216.0))


# ---------------------------------------------------------------- workloads

def alloc_bench_initial(seed: int, nthreads: int, per_thread: int):
    """Alloc microbench start: thread t creates ids 4t+k with x, v ~ U[0,1)."""
    ids = np.arange(nthreads * per_thread, dtype=np.int32)
    x = u01(ctr(seed, 0, ids, 0))
    v = u01(ctr(seed, 0, ids, 1))
    return ids, x, v


def life_initial(seed: int, width: int, height: int, density: float = 0.3) -> np.ndarray:
    """Alive grid (uint8, row-major, cell id y*width + x) with the given density."""
    c = np.arange(width * height, dtype=np.uint64)
    return (u24(ctr(seed, 0, c, 0)) < threshold(density)).astype(np.uint8)


def wator_initial(seed: int, width: int, height: int, fish: float = 0.20, shark: float = 0.05):
    """Kind grid: 0 empty, 1 fish, 2 shark (uint8, row-major)."""
    c = np.arange(width * height, dtype=np.uint64)
    u = u24(ctr(seed, 0, c, 0))
    tf, ts = threshold(fish), threshold(fish + shark)
    kind = np.zeros(width * height, dtype=np.uint8)
    kind[u < tf] = 1
    kind[(u >= tf) & (u < ts)] = 2
    return kind


def nbody_initial(seed: int, n: int):
    """Bodies uniform in the unit disk, lognormal(0, 0.5) masses, at rest.

    Drawn in double on the host (rho = sqrt(u1), theta = 2*pi*u2; Box-Muller
    for the normal), then rounded to float32 once.  Returns x, y, vx, vy, m.
    """
    i = np.arange(n, dtype=np.uint64)
    u1 = u24(ctr(seed, 0, i, 0)).astype(np.float64) / 16777216.0
    u2 = u24(ctr(seed, 0, i, 1)).astype(np.float64) / 16777216.0
    u3 = u24(ctr(seed, 0, i, 2)).astype(np.float64) / 16777216.0
    u4 = u24(ctr(seed, 0, i, 3)).astype(np.float64) / 16777216.0
    rho = np.sqrt(u1)
    th = 2.0 * math.pi * u2
    z = np.sqrt(-2.0 * np.log(1.0 - u3)) * np.cos(2.0 * math.pi * u4)
    x = (rho * np.cos(th)).astype(np.float32)
    y = (rho * np.sin(th)).astype(np.float32)
    m = np.exp(0.5 * z).astype(np.float32)
    zero = np.zeros(n, dtype=np.float32)
    return x, y, zero.copy(), zero.copy(), m


def serving_instances(seed: int, count: int, rate: float = 50.0, lo: int = 64, hi: int = 1024):
    """Instance list for the batched/serving form.

    Side log-uniform in [lo, hi): floor(lo * (hi/lo)**U); per-instance seed;
    Poisson arrivals with exponential gaps -ln(1-U)/rate seconds.
    Returns (sides int32, seeds uint64, arrival times float64).
    """
    i = np.arange(count, dtype=np.uint64)
    us = u24(ctr(seed, 0, i, 7)).astype(np.float64) / 16777216.0
    sides = np.floor(lo * (hi / lo) ** us).astype(np.int32)
    seeds = ctr(seed, 0, i, 8)
    ua = u24(ctr(seed, 0, i, 9)).astype(np.float64) / 16777216.0
    gaps = -np.log(1.0 - ua) / rate
    return sides, seeds, np.cumsum(gaps)
