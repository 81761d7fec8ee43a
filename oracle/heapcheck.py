"""Invariant checker over a raw heap dump (test infrastructure only).

Reads the byte format the C-ABI documents for its raw metadata dump (a
little-endian header of 64-bit fields, then per-block type ids, allocation
words, iteration words and the block bitmaps) and checks the invariants the
paper states for a quiescent heap, i.e. between kernels (Sec. 4.1.1: "the
bitmap is guaranteed to be in a consistent state ... at the end of a GPU
kernel"):

  H1 container consistency of every level of every block bitmap
     (Sec. 4.1.1 and App. A.5, Definition "Consistency")
  H2 no bit beyond the bitmap's size is set, and the unused words between
     the words of a level (the layout's word stride) are zero
  H3 every block is either free or allocated to exactly one class
     (Sec. 3.4: free bitmap, one allocation bitmap per class)
  H4 a free block's allocation word is all ones (Alg. 9, invalidated; a
     never-used block is created that way too)
  H5 an allocated block has the class's type id and its slots N..63 set
     (App. A.1); it holds at least one object (empty blocks are deleted, Alg. 2)
  H6 active[T] <=> allocated[T] and not full (Sec. 3.4: active means allocated
     and non-full; "active => allocated")
Returns the per-class live object counts (popcount of the allocation words
without the padding slots).
"""
from __future__ import annotations

import struct

import numpy as np

ONES = np.uint64(0xFFFFFFFFFFFFFFFF)
MAGIC = 0x504145484F4D4D53
MAX_CLASSES = 16
MAX_FIELDS = 16
MAX_LEVELS = 6


class RawHeap:
    """Parsed raw metadata dump."""

    def __init__(self, buf: bytes | np.ndarray):
        b = bytes(buf) if not isinstance(buf, bytes) else buf
        q = lambda off: struct.unpack_from("<Q", b, off)[0]
        self.magic = q(0)
        if self.magic != MAGIC:
            raise ValueError(f"bad magic {self.magic:#x}")
        self.version = q(8)
        self.M = q(16)
        self.ncls = q(24)
        self.block_bytes = q(32)
        self.nlevels = q(40)
        self.level_words = [q(48 + 8 * i) for i in range(MAX_LEVELS)][: self.nlevels]
        self.level_off = [q(96 + 8 * i) for i in range(MAX_LEVELS)][: self.nlevels]
        self.bitmap_words = q(144)
        (self.off_status, self.off_type, self.off_alloc, self.off_iter, self.off_bitmaps,
         self.off_scratch, self.scratch_bytes, self.off_data, self.total_bytes) = (
            q(152 + 8 * i) for i in range(9))
        self.capacity = [q(224 + 8 * i) for i in range(MAX_CLASSES)][: self.ncls]
        self.nfields = [q(352 + 8 * i) for i in range(MAX_CLASSES)][: self.ncls]
        fb = np.frombuffer(b, dtype="<u4", count=MAX_CLASSES * MAX_FIELDS, offset=480)
        fo = np.frombuffer(b, dtype="<u4", count=MAX_CLASSES * MAX_FIELDS, offset=1504)
        self.field_bytes = fb.reshape(MAX_CLASSES, MAX_FIELDS)[: self.ncls]
        self.field_off = fo.reshape(MAX_CLASSES, MAX_FIELDS)[: self.ncls]
        self.tune_flags, self.lookups, self.force_fail_ppm = struct.unpack_from("<III", b, 2528)
        # format 2 spaces the words of a level `bitmap_stride` words apart
        self.stride = struct.unpack_from("<I", b, 2540)[0] if self.version >= 2 else 1
        if self.stride < 1:
            raise ValueError("bitmap word stride 0")
        # 1 + superclass id per class (0: none)
        self.superclass = list(struct.unpack_from("<16I", b, 2544))[: self.ncls]
        M = self.M
        self.status = struct.unpack_from("<I", b, self.off_status)[0]
        self.counters = np.frombuffer(b, dtype="<u8", count=16, offset=self.off_status + 64)
        self.type = np.frombuffer(b, dtype="<u4", count=M, offset=self.off_type)
        self.alloc = np.frombuffer(b, dtype="<u8", count=M, offset=self.off_alloc)
        self.iter = np.frombuffer(b, dtype="<u8", count=M, offset=self.off_iter)
        nb = 1 + 2 * self.ncls
        self.bm = np.frombuffer(b, dtype="<u8", count=nb * self.bitmap_words, offset=self.off_bitmaps)

    # bitmap b: 0 free, 1+T allocated[T], 1+ncls+T active[T]
    def level(self, b: int, l: int) -> np.ndarray:
        base = b * self.bitmap_words + self.level_off[l]
        return np.ascontiguousarray(self.bm[base: base + self.level_words[l] * self.stride: self.stride])

    def level_gaps(self, b: int, l: int) -> np.ndarray:
        """The unused words between the words of level l of bitmap b."""
        base = b * self.bitmap_words + self.level_off[l]
        span = self.bm[base: base + self.level_words[l] * self.stride].reshape(-1, self.stride)
        return span[:, 1:].ravel()

    def bits(self, b: int) -> np.ndarray:
        """Level-0 bits of bitmap b as a bool array of length M."""
        w = self.level(b, 0)
        bits = np.unpackbits(w.view(np.uint8), bitorder="little").astype(bool)
        return bits[: self.M]


def _pad(n: int) -> np.uint64:
    return np.uint64(0) if n >= 64 else np.uint64((0xFFFFFFFFFFFFFFFF << n) & 0xFFFFFFFFFFFFFFFF)


def _popcount64(a: np.ndarray) -> np.ndarray:
    return np.unpackbits(np.ascontiguousarray(a, dtype="<u8").view(np.uint8)).reshape(-1, 64).sum(1) \
        if len(a) else np.zeros(0, dtype=np.int64)


def check(raw: RawHeap) -> dict:
    """Assert H1-H6; return {'live': [per class], 'blocks': [per class], 'free': n}."""
    M, ncls = raw.M, raw.ncls
    nbm = 1 + 2 * ncls
    # H1 / H2
    for b in range(nbm):
        nbits = M
        for l in range(raw.nlevels):
            w = raw.level(b, l)
            assert len(w) == (nbits + 63) // 64, (b, l, len(w), nbits)
            bits = np.unpackbits(w.view(np.uint8), bitorder="little").astype(bool)
            assert not bits[nbits:].any(), f"bitmap {b} level {l}: bits beyond size {nbits} set"
            gaps = np.nonzero(raw.level_gaps(b, l))[0]
            assert len(gaps) == 0, f"bitmap {b} level {l}: unused words between its words are set {gaps[:8]}"
            if l + 1 < raw.nlevels:
                up = raw.level(b, l + 1)
                upbits = np.unpackbits(up.view(np.uint8), bitorder="little").astype(bool)[: len(w)]
                nz = w != 0
                bad = np.nonzero(nz != upbits)[0]
                assert len(bad) == 0, f"bitmap {b}: level {l+1} inconsistent with level {l} at {bad[:8]}"
            else:
                assert len(w) == 1, "top level must be a single word"
            nbits = len(w)
    free = raw.bits(0)
    alloc_bits = [raw.bits(1 + t) for t in range(ncls)]
    active_bits = [raw.bits(1 + ncls + t) for t in range(ncls)]
    # H3
    owners = free.astype(np.int64) + sum(a.astype(np.int64) for a in alloc_bits)
    bad = np.nonzero(owners != 1)[0]
    assert len(bad) == 0, f"blocks neither free nor allocated to exactly one class: {bad[:8]}"
    # H4
    bad = np.nonzero(free & (raw.alloc != ONES))[0]
    assert len(bad) == 0, f"free blocks whose allocation word is not all ones: {bad[:8]}"
    live, blocks = [], []
    for t in range(ncls):
        a = alloc_bits[t]
        idx = np.nonzero(a)[0]
        pad = _pad(int(raw.capacity[t]))
        words = raw.alloc[idx]
        # H5
        bad = idx[raw.type[idx] != t]
        assert len(bad) == 0, f"class {t}: blocks with a foreign type id {bad[:8]}"
        bad = idx[(words & pad) != pad]
        assert len(bad) == 0, f"class {t}: padding slots not set in blocks {bad[:8]}"
        bad = idx[words == pad]
        assert len(bad) == 0, f"class {t}: empty allocated blocks {bad[:8]}"
        # H6
        full = words == ONES
        act = active_bits[t][idx]
        bad = idx[act == full]
        assert len(bad) == 0, f"class {t}: active bit disagrees with fill state at {bad[:8]}"
        stray = np.nonzero(active_bits[t] & ~a)[0]
        assert len(stray) == 0, f"class {t}: active but not allocated {stray[:8]}"
        live.append(int(_popcount64(words & ~pad).sum()))
        blocks.append(int(len(idx)))
    return {"live": live, "blocks": blocks, "free": int(free.sum())}


def fragmentation(raw: RawHeap) -> float:
    """F = sum over allocated blocks of unused slots / sum of capacities (Sec. 6.3)."""
    used = cap = 0
    for t in range(raw.ncls):
        idx = np.nonzero(raw.bits(1 + t))[0]
        n = int(raw.capacity[t])
        pad = _pad(n)
        used += int(_popcount64(raw.alloc[idx] & ~pad).sum())
        cap += n * len(idx)
    return 0.0 if cap == 0 else (cap - used) / cap
