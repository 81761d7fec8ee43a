"""Block capacity and SOA layout (test infrastructure only).

Sec. 3.2: with s the smallest class, N_T = floor(64 * size(T_s) / size(T));
a block of the smallest class holds 64 objects; a class more than 64 times
bigger than the smallest cannot be stored.  size(T) is the sum of its field
sizes: only SOA arrays are aligned, not objects (Sec. 6.2).  Each SOA array
starts on a 128-byte boundary (the vector / cache-line granule of Sec. 2.3),
arrays follow the declaration order, and every block has the byte size of the
largest class layout so that all blocks are alike (Sec. 3).
"""
from __future__ import annotations


def align(v: int, a: int) -> int:
    return (v + a - 1) // a * a


def flatten(specs):
    """Full field lists of classes given as (own field sizes, superclass id or
    None): a subclass's objects hold the superclass's fields first, then its
    own (Sec. 3.2, the data segment starts with the inherited SOA arrays)."""
    out = []
    for own, sup in specs:
        out.append((list(out[sup]) if sup is not None else []) + list(own))
    return out


def capacity(classes, t: int, block_objects: int = 64) -> int:
    """N_T; with block_objects B < 64 the smallest class holds B objects per
    block instead of 64 and the formula scales the others the same way."""
    sizes = [sum(c) for c in classes]
    n = (block_objects * min(sizes)) // sizes[t]
    if n < 1:
        raise ValueError("class more than %dx bigger than the smallest class" % block_objects)
    return n


def layout(classes, align_bytes: int = 128, block_objects: int = 64):
    """classes: list of lists of field byte sizes.

    Returns (block_bytes, [(capacity, [field offsets])...]).
    """
    out = []
    block = 0
    for t, fields in enumerate(classes):
        n = capacity(classes, t, block_objects)
        offs, cur = [], 0
        for f in fields:
            offs.append(cur)
            cur += align(n * f, align_bytes)
        out.append((n, offs))
        block = max(block, cur)
    return block, out
