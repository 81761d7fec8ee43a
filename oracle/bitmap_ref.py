"""Sequential hierarchical bitmap (test infrastructure only).

Sec. 4.1.1: a bitmap of N bits is an array of ceil(N/W) containers of W bits
plus, if N > W, a nested bitmap of ceil(N/W) bits whose bit i is the OR of
container i ("container consistency").  The paper uses W = 64; its worked
example (figure "bitmap_clear_example") uses W = 4, so W is a parameter here.

Operations follow Sec. 4.1.2 and Alg. 3/4/5 in a single thread: ``set`` /
``clear`` change the bit and, when they set the first or clear the last bit of
a container, update the nested bitmap with the non-try form; ``try_find_set``
descends from the top level.  ``trace`` records every (level, op, pos) that
reaches a container, so the cascade of the worked example can be checked.
"""
from __future__ import annotations


class HBitmap:
    def __init__(self, nbits: int, width: int = 64, level: int = 0, trace=None):
        assert nbits >= 1 and width >= 2
        self.n = nbits
        self.w = width
        self.level = level
        self.ncont = (nbits + width - 1) // width
        self.cont = [0] * self.ncont
        self.trace = trace if trace is not None else []
        self.nested = HBitmap(self.ncont, width, level + 1, self.trace) if nbits > width else None

    # -- helpers
    def _popc(self, v: int) -> int:
        return bin(v).count("1")

    def get(self, pos: int) -> int:
        return (self.cont[pos // self.w] >> (pos % self.w)) & 1

    # -- Alg. 3 (try_clear) and its non-try / set counterparts
    def try_clear(self, pos: int) -> bool:
        self.trace.append((self.level, "clear", pos))
        cid, off = divmod(pos, self.w)
        mask = 1 << off
        prev = self.cont[cid]
        self.cont[cid] = prev & ~mask
        success = (prev & mask) != 0
        if success and self.nested is not None and self._popc(prev) == 1:
            self.nested.clear(cid)
        return success

    def clear(self, pos: int) -> None:
        # sequentially the bit must be set, otherwise the concurrent form would spin forever
        assert self.try_clear(pos), f"clear({pos}) on a cleared bit at level {self.level}"

    def try_set(self, pos: int) -> bool:
        self.trace.append((self.level, "set", pos))
        cid, off = divmod(pos, self.w)
        mask = 1 << off
        prev = self.cont[cid]
        self.cont[cid] = prev | mask
        success = (prev & mask) == 0
        if success and self.nested is not None and prev == 0:
            self.nested.set(cid)
        return success

    def set(self, pos: int) -> None:
        assert self.try_set(pos), f"set({pos}) on a set bit at level {self.level}"

    # -- Alg. 4
    def try_find_set(self):
        if self.nested is not None:
            cid = self.nested.try_find_set()
            if cid is None:
                return None
        else:
            cid = 0
        c = self.cont[cid]
        if c == 0:
            return None
        off = (c & -c).bit_length() - 1
        return cid * self.w + off

    # clear(): find and clear any set bit (loop until a find fails or a clear succeeds)
    def clear_any(self):
        while True:
            i = self.try_find_set()
            if i is None:
                return None
            if self.try_clear(i):
                return i

    # -- Alg. 5 (sequential): indices of all set bits, ascending
    def indices(self):
        selected = self.nested.indices() if self.nested is not None else [0]
        out = []
        for cid in selected:
            c = self.cont[cid]
            for k in range(self.w):
                if (c >> k) & 1:
                    out.append(cid * self.w + k)
        return out

    # -- Definition "Consistency" (App. A.5)
    def consistent(self) -> bool:
        if self.nested is None:
            return True
        for i in range(self.ncont):
            if (self.cont[i] != 0) != bool(self.nested.get(i)):
                return False
        return self.nested.consistent()

    def levels(self):
        """Containers of every level, bottom first."""
        out, b = [], self
        while b is not None:
            out.append(list(b.cont))
            b = b.nested
        return out
