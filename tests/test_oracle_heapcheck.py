"""Pins of the raw-heap invariant checker (oracle/heapcheck.py).

A small heap dump is assembled here by hand in the byte format the C-ABI
documents for its raw metadata dump (header of 64-bit fields, per-block type
ids, allocation and iteration words, then the block bitmaps free /
allocated[T] / active[T], each level after level).  The consistent dump must
pass; each dump below corrupts exactly one invariant and must be rejected
with that invariant's message, so that none of the checks is vacuous:

  H1 container consistency of the levels (Sec. 4.1.1; App. A.5)
  H2 no bit beyond the bitmap's size; the unused words between the words of
     a level (the layout's word stride) are zero
  H3 a block is free or allocated to exactly one class (Sec. 3.4)
  H4 a free block's allocation word is all ones (Alg. 9, invalidated)
  H5 an allocated block has its class's type, padding slots set, >= 1 object
     (App. A.1; Alg. 2 deletes empty blocks)
  H6 active[T] <=> allocated[T] and not full, active => allocated (Sec. 3.4)
"""
import struct

import numpy as np
import pytest

from oracle import heapcheck

ONES = (1 << 64) - 1


def _pad(n):
    return 0 if n >= 64 else (ONES << n) & ONES


class Dump:
    """A quiescent heap of M blocks and the classes' capacities, turned into
    raw dump bytes.  blocks[b] = (class or None, allocation word)."""

    def __init__(self, M=130, caps=(64, 42), stride=16):
        self.M, self.caps, self.stride = M, list(caps), stride
        self.blocks = [(None, ONES)] * M
        self.type_override = {}
        self.extra_bits = []           # (bitmap, level, bit index) toggled after derivation
        self.gap_words = []            # (bitmap, level, word index, offset 1..stride-1, value)

    def levels(self):
        words, n = [], self.M
        while True:
            w = (n + 63) // 64
            words.append(w)
            if w == 1:
                return words
            n = w

    def bitmaps(self):
        """Level-0 bits of free, allocated[T], active[T] derived from the blocks."""
        nc = len(self.caps)
        bits = np.zeros((1 + 2 * nc, self.M), dtype=bool)
        for b, (t, w) in enumerate(self.blocks):
            if t is None:
                bits[0, b] = True
            else:
                bits[1 + t, b] = True
                bits[1 + nc + t, b] = w != ONES
        return bits

    def to_bytes(self):
        M, nc = self.M, len(self.caps)
        lw = self.levels()
        loff, off = [], 0
        for w in lw:
            loff.append(off)
            off += (w + 7) // 8 * 8 * self.stride
        bitmap_words = (off + 31) // 32 * 32
        p = 4096
        off_status = p; p += 256
        off_type = p; p = (p + 4 * M + 255) // 256 * 256
        off_alloc = p; p = (p + 8 * M + 255) // 256 * 256
        off_iter = p; p = (p + 8 * M + 255) // 256 * 256
        off_bitmaps = p; p = (p + 8 * bitmap_words * (1 + 2 * nc) + 255) // 256 * 256
        off_scratch = p; scratch = 1024 + 4 * M; p += scratch
        off_data = (p + 4095) // 4096 * 4096
        buf = bytearray(off_data)
        hdr = [heapcheck.MAGIC, 2, M, nc, 768, len(lw)]
        struct.pack_into("<6Q", buf, 0, *hdr)
        struct.pack_into("<6Q", buf, 48, *(lw + [0] * (6 - len(lw))))
        struct.pack_into("<6Q", buf, 96, *(loff + [0] * (6 - len(loff))))
        struct.pack_into("<Q", buf, 144, bitmap_words)
        struct.pack_into("<9Q", buf, 152, off_status, off_type, off_alloc, off_iter, off_bitmaps, off_scratch,
                         scratch, off_data, off_data)
        struct.pack_into("<16Q", buf, 224, *(self.caps + [0] * (16 - nc)))
        struct.pack_into("<16Q", buf, 352, *([1] * nc + [0] * (16 - nc)))
        struct.pack_into("<I", buf, 2540, self.stride)
        for b, (t, w) in enumerate(self.blocks):
            ty = 0xFFFFFFFF if t is None else t
            ty = self.type_override.get(b, ty)
            struct.pack_into("<I", buf, off_type + 4 * b, ty)
            struct.pack_into("<Q", buf, off_alloc + 8 * b, w)
        bits = self.bitmaps()
        for bm in range(1 + 2 * nc):
            lv = [bits[bm].copy()]
            for l in range(1, len(lw)):
                prev = lv[-1]
                up = np.zeros(lw[l - 1], dtype=bool)
                for i in range(lw[l - 1]):
                    up[i] = prev[64 * i: 64 * i + 64].any()
                lv.append(up)
            for (xb, xl, xi) in self.extra_bits:
                if xb == bm:
                    if xi >= len(lv[xl]):
                        lv[xl] = np.concatenate([lv[xl], np.zeros(xi + 1 - len(lv[xl]), dtype=bool)])
                    lv[xl][xi] = not lv[xl][xi]
            for l, v in enumerate(lv):
                for i in range(lw[l]):
                    word = 0
                    for k in range(64):
                        if 64 * i + k < len(v) and v[64 * i + k]:
                            word |= 1 << k
                    struct.pack_into("<Q", buf, off_bitmaps + 8 * (bm * bitmap_words + loff[l] + i * self.stride),
                                     word)
        for (bm, l, i, k, v) in self.gap_words:
            struct.pack_into("<Q", buf, off_bitmaps + 8 * (bm * bitmap_words + loff[l] + i * self.stride + k), v)
        return bytes(buf)

    def check(self):
        return heapcheck.check(heapcheck.RawHeap(self.to_bytes()))


def consistent():
    """130 blocks (levels 3 + 1 words): class 0 (N = 64) and class 1 (N = 42)
    blocks, some full, some partly used; the rest free."""
    d = Dump()
    d.blocks[0] = (0, ONES)                               # full class-0 block
    d.blocks[1] = (0, 0b1011)                             # 3 objects
    d.blocks[2] = (0, 0b1)                                # 1 object
    d.blocks[65] = (1, _pad(42) | 0b1)                    # 1 object
    d.blocks[66] = (1, ONES)                              # full class-1 block
    d.blocks[129] = (0, 1 << 63)                          # last block of the heap
    return d


def test_consistent_dump_passes_and_counts():
    s = consistent().check()
    assert s["live"] == [64 + 3 + 1 + 1, 1 + 42]
    assert s["blocks"] == [4, 2]
    assert s["free"] == 130 - 6


@pytest.mark.parametrize("stride", [1, 2, 16])
def test_word_stride_is_read_from_the_header(stride):
    # the same heap laid out with its bitmap words 1, 2 or 16 words apart
    # decodes to the same bitmaps and counts
    d = consistent()
    d.stride = stride
    raw = heapcheck.RawHeap(d.to_bytes())
    assert raw.stride == stride
    assert raw.bits(1)[[0, 1, 2, 129]].all() and raw.bits(2)[[65, 66]].all()
    assert heapcheck.check(raw)["live"] == [64 + 3 + 1 + 1, 1 + 42]


def test_format_1_dump_is_dense():
    d = consistent()
    d.stride = 1
    b = bytearray(d.to_bytes())
    struct.pack_into("<Q", b, 8, 1)             # format 1 has no stride field
    struct.pack_into("<I", b, 2540, 0)
    assert heapcheck.RawHeap(bytes(b)).stride == 1
    assert heapcheck.check(heapcheck.RawHeap(bytes(b)))["blocks"] == [4, 2]


def test_h2_set_word_between_level_words_is_rejected():
    d = consistent()
    d.gap_words.append((3, 0, 1, 5, 1 << 3))    # active[0], level 0: a word between words 1 and 2
    with pytest.raises(AssertionError, match="unused words"):
        d.check()


def test_h1_level1_bit_without_children_is_rejected():
    d = consistent()
    d.extra_bits.append((0, 1, 1))        # free bitmap: clear the level-1 bit of word 1 (it has free blocks)
    with pytest.raises(AssertionError, match="inconsistent"):
        d.check()


def test_h1_level1_bit_over_empty_word_is_rejected():
    d = consistent()
    d.extra_bits.append((2, 1, 0))        # allocated[1]: word 0 holds no class-1 block; set its level-1 bit
    with pytest.raises(AssertionError, match="inconsistent"):
        d.check()


def test_h2_bit_beyond_size_is_rejected():
    d = consistent()
    d.extra_bits.append((0, 0, 130))      # free bitmap, level 0: bit 130 of a 130-block heap
    with pytest.raises(AssertionError, match="beyond size"):
        d.check()


def test_h3_block_free_and_allocated_is_rejected():
    d = consistent()
    d.extra_bits.append((0, 0, 1))        # block 1 (class 0) also free; its level-0 word already has free bits
    with pytest.raises(AssertionError, match="exactly one class"):
        d.check()


def test_h3_block_in_no_bitmap_is_rejected():
    d = consistent()
    d.extra_bits.append((0, 0, 100))      # free block 100 taken out of the free bitmap
    with pytest.raises(AssertionError, match="exactly one class"):
        d.check()


def test_h4_free_block_with_live_slots_is_rejected():
    d = consistent()
    d.blocks[10] = (None, ONES & ~1)
    with pytest.raises(AssertionError, match="not all ones"):
        d.check()


def test_h5_foreign_type_is_rejected():
    d = consistent()
    d.type_override[1] = 1
    with pytest.raises(AssertionError, match="foreign type"):
        d.check()


def test_h5_padding_slot_cleared_is_rejected():
    d = consistent()
    d.blocks[65] = (1, (_pad(42) & ~(1 << 50)) | 0b1)
    with pytest.raises(AssertionError, match="padding"):
        d.check()


def test_h5_empty_allocated_block_is_rejected():
    d = consistent()
    d.blocks[65] = (1, _pad(42))
    with pytest.raises(AssertionError, match="empty allocated"):
        d.check()


def test_h6_full_block_marked_active_is_rejected():
    d = consistent()
    d.extra_bits.append((3, 0, 0))        # active[0]: block 0 is full; its word already has active blocks
    with pytest.raises(AssertionError, match="active bit disagrees"):
        d.check()


def test_h6_partial_block_not_active_is_rejected():
    d = consistent()
    d.extra_bits.append((3, 0, 1))        # active[0]: clear block 1 (3 objects, not full; block 2 stays active)
    with pytest.raises(AssertionError, match="active bit disagrees"):
        d.check()


def test_h6_active_but_not_allocated_is_rejected():
    d = consistent()
    d.extra_bits.append((4, 0, 100))      # active[1]: free block 100 (word 1 already holds active block 65)
    with pytest.raises(AssertionError, match="active but not allocated"):
        d.check()
