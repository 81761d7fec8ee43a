"""Shared helpers of the GPU tests (test code only)."""
from __future__ import annotations

import sys

import numpy as np

from oracle import heapcheck


def say(*a):
    """Name the case before a GPU step, flushed, so a crash log shows it."""
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def check_heap(heap, expect_live=None):
    """Raw-dump invariants (H1-H6) plus status 0; returns the checker's summary."""
    st = heap.status()
    assert st == 0, f"device status {st:#x}"
    raw = heapcheck.RawHeap(heap.dump_raw())
    summary = heapcheck.check(raw)
    if expect_live is not None:
        assert summary["live"] == list(expect_live), (summary["live"], expect_live)
    for t in range(len(summary["live"])):
        assert heap.live_count(t) == summary["live"][t]
    return summary


def bits_equal(a: np.ndarray, b: np.ndarray) -> bool:
    a = np.ascontiguousarray(a)
    b = np.ascontiguousarray(b)
    if a.shape != b.shape:
        return False
    return np.array_equal(a.view(np.uint8), b.view(np.uint8))


def wator_check(w, steps_done, oracle_state):
    """Predator-prey state of workload `w` equals the oracle's (bit-exact),
    the occupancy grid agrees with the live objects, and the heap is sound."""
    kind, age, energy = w.state()
    ok, oa, oe = oracle_state
    assert np.array_equal(kind, ok), f"occupancy differs after {steps_done} steps"
    assert np.array_equal(age[kind > 0], oa[ok > 0]), f"ages differ after {steps_done} steps"
    assert np.array_equal(energy[kind == 2], oe[ok == 2]), f"energies differ after {steps_done} steps"
    assert np.array_equal(w.occ_kind(), kind), "occupancy grid disagrees with the live objects"
    return check_heap(w.heap, expect_live=[int((ok == 1).sum()), int((ok == 2).sum())])
