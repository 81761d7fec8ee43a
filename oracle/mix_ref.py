"""Oracle of the two-class churn test method (test infrastructure only).

Definition (the method's contract in the C-ABI header): in round r, a do-all
over class A and then one over class B (or, with B a subclass of A, one do-all
over A that covers both, `run_subtree`); each visited object computes
h = splitmix64(seed ^ id ^ (r << 32)); if h is odd it is destroyed and a
replacement with id' = ((r+1) << 18) | (id & 0x3FFFF) is created in class B
when bit 1 of h is set, else in class A.  A do-all visits the objects of its
class that exist when it starts.  Placement is not part of the result.
"""
from __future__ import annotations

import numpy as np

from . import core

M64 = (1 << 64) - 1


def run(seed: int, ids_a, ids_b, rounds: int):
    """Returns [(sorted ids of A, sorted ids of B) after each round]."""
    a = sorted(int(i) for i in ids_a)
    b = sorted(int(i) for i in ids_b)
    out = []
    for r in range(rounds):
        for phase in ("a", "b"):
            src = a if phase == "a" else b
            keep, to_a, to_b = [], [], []
            for i in src:
                h = core.splitmix64((seed ^ i ^ (r << 32)) & M64)
                if h & 1:
                    nid = ((r + 1) << 18) | (i & 0x3FFFF)
                    (to_b if (h >> 1) & 1 else to_a).append(nid)
                else:
                    keep.append(i)
            if phase == "a":
                a = sorted(keep + to_a)
                b = sorted(b + to_b)
            else:
                b = sorted(keep + to_b)
                a = sorted(a + to_a)
        out.append((np.array(a, dtype=np.int32), np.array(b, dtype=np.int32)))
    return out


def run_subtree(seed: int, ids_a, ids_b, rounds: int):
    """B is a subclass of A: each round is one do-all over A, which visits the
    objects of A and of B that exist when it starts (Sec. 2.1) and none that
    it creates.  Returns [(sorted ids of A, sorted ids of B) after each round]."""
    a = sorted(int(i) for i in ids_a)
    b = sorted(int(i) for i in ids_b)
    out = []
    for r in range(rounds):
        new_a, new_b = [], []
        for src, keep in ((a, new_a), (b, new_b)):
            for i in src:
                h = core.splitmix64((seed ^ i ^ (r << 32)) & M64)
                if h & 1:
                    nid = ((r + 1) << 18) | (i & 0x3FFFF)
                    (new_b if (h >> 1) & 1 else new_a).append(nid)
                else:
                    keep.append(i)
        a, b = sorted(new_a), sorted(new_b)
        out.append((np.array(a, dtype=np.int32), np.array(b, dtype=np.int32)))
    return out
