"""CPU tests of the C-ABI library: it loads, exports every declared symbol,
and its host-side logic (layout, sizes, argument checks, handles) matches the
paper's formulas as restated by the oracle.  No kernel is launched."""
import ctypes as C
import os
import re
import subprocess

import pytest

from oracle import heapcheck, layout_ref
from paper_1810_11765_amd import smmo as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "smmo.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(smmo_\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 20
    L = C.CDLL(S.LIB_PATH)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", S.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (smmo_\w+)", out))
    assert set(names) <= exported


WORKLOAD_CLASSES = [
    [[4, 4, 4]],                 # alloc microbench
    [[4, 4, 1], [4, 4]],         # Life: Cell, Agent
    [[4, 4], [4, 4, 4]],         # Wa-Tor: Fish, Shark
    [[4] * 5],                   # n-body
    [[1, 2], [8, 8, 8, 8], [4]],
    [[1], [8] * 8],              # exactly 64x
]


@pytest.mark.parametrize("classes", WORKLOAD_CLASSES)
def test_layout_matches_capacity_formula(classes):
    block, per = layout_ref.layout(classes)
    for t, (n, offs) in enumerate(per):
        lay = S.layout_of(classes, t)
        assert lay.capacity == n
        assert lay.block_bytes == block
        assert list(lay.field_offset[: len(offs)]) == offs
        assert list(lay.field_bytes[: len(offs)]) == classes[t]


@pytest.mark.parametrize("block_objects", [1, 21, 32, 63])
@pytest.mark.parametrize("classes", WORKLOAD_CLASSES[:4])
def test_layout_with_fewer_objects_per_block_matches_the_formula(classes, block_objects):
    try:
        block, per = layout_ref.layout(classes, block_objects=block_objects)
    except ValueError:                                   # a class too big for this capacity:
        with pytest.raises(S.SmmoError):                 # the library refuses it too
            S.layout_of(classes, 0, block_objects)
        return
    for t, (n, offs) in enumerate(per):
        lay = S.layout_of(classes, t, block_objects)
        assert lay.capacity == n and lay.block_bytes == block
        assert list(lay.field_offset[: len(offs)]) == offs


def test_block_objects_out_of_range_is_rejected():
    for bad in (0, 65):
        with pytest.raises(S.SmmoError):
            S.heap_bytes([[4]], 16, bad)


def test_layout_with_subclasses_by_hand():
    """Base {i32, i32}; Sub: Base + {f64}; Leaf: Sub + nothing; Tiny {i8, i8}.
    Sizes 8, 16, 16, 2: capacities 64*2 // size = 16, 8, 8, 64; SOA arrays of
    the inherited fields first, each 128-B aligned."""
    specs = [([4, 4], None), ([8], 0), ([], 1), ([1, 1], None)]
    full = layout_ref.flatten(specs)
    assert full == [[4, 4], [4, 4, 8], [4, 4, 8], [1, 1]]
    block, per = layout_ref.layout(full)
    assert per == [(16, [0, 128]), (8, [0, 128, 256]), (8, [0, 128, 256]), (64, [0, 128])]
    assert block == 384
    classes = [{"fields": own, "super": sup} if sup is not None else own for own, sup in specs]
    for t, (n, offs) in enumerate(per):
        lay = S.layout_of(classes, t)
        assert lay.capacity == n and lay.block_bytes == block
        assert list(lay.field_offset[: len(offs)]) == offs
        assert list(lay.field_bytes[: lay.nfields]) == full[t]
    assert S.full_fields(classes) == full


def test_layout_rejects_bad_subclasses():
    for bad in ([[4], {"fields": [4], "super": 1}],                  # superclass not a smaller id
                [[4], {"fields": [4], "super": 5}],
                [[4] * 10, {"fields": [4] * 7, "super": 0}],        # 17 fields in all
                [{"fields": [], "super": None}]):                   # no field at all
        with pytest.raises(S.SmmoError):
            S.layout_of(bad, len(bad) - 1)


def test_layout_rejects_bad_classes():
    for bad in ([[1], [8] * 9], [[3]], [[]], [[4]] * 17):
        with pytest.raises(S.SmmoError):
            S.layout_of(bad, 0)


def test_heap_bytes_and_header_struct_offsets(tmp_path):
    # bytes grow with blocks by exactly block_bytes (data) + per-block words
    b1 = S.heap_bytes([[4, 4, 4]], 4096)
    b2 = S.heap_bytes([[4, 4, 4]], 8192)
    assert b2 - b1 >= 4096 * (768 + 20)
    # the checker's parser offsets agree with the C struct layout
    prog = str(tmp_path / "hdr_offsets")
    src = prog + ".c"
    with open(src, "w") as f:
        f.write('#include <stdio.h>\n#include <stddef.h>\n#include "smmo.h"\n'
                '#define P(x) printf("%zu ", offsetof(smmo_raw_header, x));\n'
                "int main(){P(magic)P(num_blocks)P(ncls)P(block_bytes)P(nlevels)P(level_words)P(level_off)"
                "P(bitmap_words)P(off_status)P(off_type)P(off_alloc)P(off_iter)P(off_bitmaps)P(off_scratch)"
                "P(scratch_bytes)P(off_data)P(total_bytes)P(capacity)P(nfields)P(field_bytes)P(field_off)"
                "P(tune_flags)P(lookups)P(force_fail_ppm)P(bitmap_stride)P(superclass)return 0;}\n")
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), src, "-o", prog], check=True)
    got = [int(v) for v in subprocess.run([prog], capture_output=True, text=True).stdout.split()]
    assert got == [0, 16, 24, 32, 40, 48, 96, 144, 152, 160, 168, 176, 184, 192, 200, 208, 216, 224, 352, 480,
                   1504, 2528, 2532, 2536, 2540, 2544]
    assert heapcheck.MAGIC == 0x504145484F4D4D53


def test_handle_encoding():
    L = S.lib()
    for cls, blk, slot in ((0, 0, 0), (3, 12345, 63), (15, (1 << 44) - 1, 7)):
        r = L.smmo_ref_make(cls, blk, slot)
        assert r != 0
        assert (L.smmo_ref_class(r), L.smmo_ref_block(r), L.smmo_ref_slot(r)) == (cls, blk, slot)
        assert int(S.ref_class(r)) == cls


def test_strerror_codes():
    L = S.lib()
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert L.smmo_strerror(code)


def test_arena_first_fit_and_merging():
    """The arena is host-side bookkeeping over a device range: exercise it on
    a fake base address (no device access happens)."""
    L = S._bind_batch()
    base = 0x7f0000000000
    h = C.c_void_p()
    assert L.smmo_arena_create(C.c_void_p(base), 1 << 20, C.byref(h)) == 0
    ptrs = []
    for n in (1000, 256, 70000, 1):
        p = C.c_void_p()
        assert L.smmo_arena_alloc(h, n, C.byref(p)) == 0
        assert p.value % 256 == 0 and base <= p.value < base + (1 << 20)
        ptrs.append((p.value, (n + 255) // 256 * 256))
    spans = sorted(ptrs)
    for (a, na), (b, nb) in zip(spans, spans[1:]):
        assert a + na <= b                                  # no overlap
    big = C.c_void_p()
    assert L.smmo_arena_alloc(h, 1 << 20, C.byref(big)) == -3   # does not fit
    for p, _ in ptrs:
        assert L.smmo_arena_free(h, C.c_void_p(p)) == 0
    free, largest = C.c_uint64(), C.c_uint64()
    L.smmo_arena_stats(h, C.byref(free), C.byref(largest))
    assert free.value == largest.value == 1 << 20              # fully merged again
    assert L.smmo_arena_free(h, C.c_void_p(base + 12345)) == -1
    L.smmo_arena_destroy(h)
