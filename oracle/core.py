"""ctypes wrapper of oracle.c (test infrastructure only).

Builds the library with gcc on first use if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        u64, i64, i32, u32, f32 = C.c_uint64, C.c_int64, C.c_int32, C.c_uint32, C.c_float
        P = C.c_void_p
        L.or_splitmix64.argtypes = [u64]; L.or_splitmix64.restype = u64
        L.or_ctr.argtypes = [u64, u64, u64, u64]; L.or_ctr.restype = u64
        L.or_c1_round.argtypes = [u64, u32, i64, P, P, P]; L.or_c1_round.restype = i64
        L.or_c2_run.argtypes = [i32, i32, i32, P, P]; L.or_c2_run.restype = None
        L.or_c3_run.argtypes = [i32, i32, u64, i32, i32, i32, i32, i32, P, P, P, P]
        L.or_c3_run.restype = None
        L.or_c4_step.argtypes = [i64, P, P, P, P, P, P, f32, f32, f32, P]; L.or_c4_step.restype = i64
        L.or_c4_accel.argtypes = [i64, P, P, P, f32, i64, P, P, P]; L.or_c4_accel.restype = None
        L.or_threads.argtypes = []; L.or_threads.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]; L.or_set_threads.restype = None
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().or_threads())


def set_threads(n: int) -> None:
    lib().or_set_threads(n)


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def splitmix64(x: int) -> int:
    return int(lib().or_splitmix64(C.c_uint64(x & (2**64 - 1))))


def ctr(seed: int, step: int, ident: int, stream: int) -> int:
    return int(lib().or_ctr(seed & (2**64 - 1), step, ident, stream))


# ------------------------------------------------------- alloc microbench

def c1_round(seed: int, r: int, ids: np.ndarray, x: np.ndarray, v: np.ndarray) -> int:
    """One round (sweep do-all + churn do-all) in place; arrays sorted by id."""
    assert ids.dtype == np.int32 and x.dtype == np.float32 and v.dtype == np.float32
    return int(lib().or_c1_round(seed, r, len(ids), _p(ids), _p(x), _p(v)))


def c1_run(seed: int, ids, x, v, rounds: int):
    ids, x, v = ids.copy(), x.copy(), v.copy()
    order = np.argsort(ids, kind="stable")
    ids, x, v = ids[order].copy(), x[order].copy(), v[order].copy()
    states = []
    for r in range(rounds):
        c1_round(seed, r, ids, x, v)
        states.append((ids.copy(), x.copy(), v.copy()))
    return states


# ------------------------------------------------------------ Life-like grid

def c2_run(alive0: np.ndarray, width: int, height: int, steps: int):
    """Returns (alive grid uint8, agent age per cell int32, -1 = no agent)."""
    alive = np.ascontiguousarray(alive0, dtype=np.uint8).copy()
    age = np.empty(width * height, dtype=np.int32)
    lib().or_c2_run(width, height, steps, _p(alive), _p(age))
    return alive, age


# ------------------------------------------------------------ predator-prey

def c3_run(kind0: np.ndarray, width: int, height: int, seed: int, steps: int,
           fish_breed: int = 3, shark_breed: int = 8, eat_gain: int = 4, shark_e0: int = 4,
           with_counts: bool = False):
    """Returns (kind, age, energy) per cell [, counts (steps, 6): fish, sharks after the
    step, fish eaten, sharks starved, fish born, sharks born]."""
    kind = np.ascontiguousarray(kind0, dtype=np.uint8).copy()
    n = width * height
    age = np.zeros(n, dtype=np.int32)
    energy = np.where(kind == 2, shark_e0, 0).astype(np.int32)
    counts = np.zeros((max(steps, 1), 6), dtype=np.int64)
    lib().or_c3_run(width, height, seed & (2**64 - 1), steps, fish_breed, shark_breed, eat_gain,
                    shark_e0, _p(kind), _p(age), _p(energy), _p(counts))
    if with_counts:
        return kind, age, energy, counts[:steps]
    return kind, age, energy


# ----------------------------------------------------------------- n-body

def c4_step(ids, x, y, vx, vy, m, G=1e-6, dt=1e-3, merge_dist=1e-4):
    """One step (merge, force, move); returns new arrays (survivors, by id) and #pairs."""
    arrs = [np.ascontiguousarray(a).copy() for a in (ids, x, y, vx, vy, m)]
    assert arrs[0].dtype == np.int32 and all(a.dtype == np.float32 for a in arrs[1:])
    npairs = np.zeros(1, dtype=np.int64)
    n = lib().or_c4_step(len(arrs[0]), *[_p(a) for a in arrs], G, dt, merge_dist, _p(npairs))
    return tuple(a[:n].copy() for a in arrs), int(npairs[0])


def c4_accel(x, y, m, sel, G=1e-6):
    x, y, m = (np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, m))
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    ax = np.zeros(len(sel), dtype=np.float32)
    ay = np.zeros(len(sel), dtype=np.float32)
    lib().or_c4_accel(len(x), _p(x), _p(y), _p(m), G, len(sel), _p(sel), _p(ax), _p(ay))
    return ax, ay


def c4_run_grid(ids, x, y, vx, vy, m, steps, G=1e-6, dt=1e-3, merge_dist=1e-4, cell=1.0 / 1024,
                checkpoints=(), on_checkpoint=None):
    """`steps` whole steps (grid merge, force, move) of a large state; after
    each step listed in `checkpoints`, on_checkpoint(step, arrays) is called
    with the survivors (ascending id).  Returns the final arrays."""
    L = lib()
    if not hasattr(L, "_step_grid_sig"):
        L.or_c4_step_grid.argtypes = [C.c_int64] + [C.c_void_p] * 6 + [C.c_float] * 3 + [C.c_double, C.c_void_p]
        L.or_c4_step_grid.restype = C.c_int64
        L._step_grid_sig = True
    arrs = [np.ascontiguousarray(a).copy() for a in (ids, x, y, vx, vy, m)]
    assert arrs[0].dtype == np.int32 and all(a.dtype == np.float32 for a in arrs[1:])
    n = len(arrs[0])
    npairs = np.zeros(1, dtype=np.int64)
    for s in range(1, steps + 1):
        n = L.or_c4_step_grid(n, *[_p(a) for a in arrs], G, dt, merge_dist, cell, _p(npairs))
        if on_checkpoint is not None and s in checkpoints:
            on_checkpoint(s, tuple(a[:n] for a in arrs))
    return tuple(a[:n].copy() for a in arrs)


def c4_merge_grid(ids, x, y, vx, vy, m, merge_dist=1e-4, cell=1.0 / 1024):
    """Merge phase only (grid candidates, same float test); returns survivors and #pairs."""
    L = lib()
    if not hasattr(L, "_merge_sig"):
        L.or_c4_merge_grid.argtypes = [C.c_int64] + [C.c_void_p] * 6 + [C.c_float, C.c_double, C.c_void_p]
        L.or_c4_merge_grid.restype = C.c_int64
        L._merge_sig = True
    arrs = [np.ascontiguousarray(a).copy() for a in (ids, x, y, vx, vy, m)]
    npairs = np.zeros(1, dtype=np.int64)
    n = L.or_c4_merge_grid(len(arrs[0]), *[_p(a) for a in arrs], merge_dist, cell, _p(npairs))
    return tuple(a[:n].copy() for a in arrs), int(npairs[0])
