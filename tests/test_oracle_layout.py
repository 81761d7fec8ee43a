"""Pins of block capacity and SOA layout (Sec. 3.2; arrays 128-byte aligned)."""
import pytest

from oracle import layout_ref as L


def test_smallest_class_has_capacity_64():
    for classes in ([[4]], [[4, 4, 4]], [[1, 1], [8, 8, 8]], [[8], [4, 4, 1]]):
        sizes = [sum(c) for c in classes]
        s = sizes.index(min(sizes))
        assert L.capacity(classes, s) == 64


def test_workload_layouts_by_hand():
    # alloc microbench {i32 id, f32 x, f32 v}: 12 B, N = 64, arrays 256 B each
    assert L.layout([[4, 4, 4]]) == (768, [(64, [0, 256, 512])])
    # Life: Agent {i32, i32} = 8 B -> 64; Cell {i32, i32, i8} = 9 B -> floor(512/9) = 56
    # Cell arrays: 224 -> 256, 224 -> 256, 56 -> 128  => 640 B; Agent 2 x 256 = 512
    assert L.layout([[4, 4, 1], [4, 4]]) == (640, [(56, [0, 256, 512]), (64, [0, 256])])
    # Wa-Tor: Fish 8 B -> 64 (512 B); Shark 12 B -> floor(512/12) = 42, arrays 168 -> 256
    assert L.layout([[4, 4], [4, 4, 4]]) == (768, [(64, [0, 256]), (42, [0, 256, 512])])
    # N-body: 5 x f32 = 20 B -> 64, 5 x 256 = 1280 B
    assert L.layout([[4] * 5]) == (1280, [(64, [0, 256, 512, 768, 1024])])


def test_class_more_than_64x_bigger_is_rejected():
    with pytest.raises(ValueError):
        L.capacity([[1], [8] * 9], 1)          # 72 B vs 1 B
    assert L.capacity([[1], [8] * 8], 1) == 1   # exactly 64 x


def test_block_capacity_parameter_by_hand():
    """With 32 objects per block for the smallest class (the autotuner's
    other layout): Wa-Tor Fish 8 B -> 32 (arrays 128 B), Shark 12 B ->
    floor(256/12) = 21 (arrays 84 -> 128 B); block = 3 x 128 = 384 B.  With
    one object per block every class of size <= the smallest holds 1."""
    assert L.layout([[4, 4], [4, 4, 4]], block_objects=32) == (384, [(32, [0, 128]), (21, [0, 128, 256])])
    assert L.layout([[4, 4, 1], [4, 4]], block_objects=32) == (384, [(28, [0, 128, 256]), (32, [0, 128])])
    assert L.capacity([[4]], 0, block_objects=1) == 1
    with pytest.raises(ValueError):
        L.capacity([[1], [8] * 5], 1, block_objects=32)     # 40 B vs 1 B > 32x
