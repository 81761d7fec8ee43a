"""Object-slot bitmap rules of one block (test infrastructure only).

Every block has a 64-bit object allocation bitmap (Sec. 3.1).  A block of
capacity N < 64 keeps its slots N..63 set to 1 for its whole life (App. A.1).
The paper prints the rules for N = 64:
  reserve (Alg. 6):      FULL iff popc(before) = 63
  deallocate (Alg. 7):   EMPTY iff popc(before) = 1, FIRST iff popc(before) = 64
  invalidate (Alg. 9):   succeeds iff before = 0; otherwise it rolls back with
                         AND before, and retries if the block became empty.
For general N the same events are stated on the word itself:
  pad(N)   = the bits N..63
  FULL     the word becomes all ones because of this operation
  FIRST    the word was all ones before a deallocation
  EMPTY    after a deallocation only pad(N) remains
  invalid. succeeds iff before = pad(N)
Multi-slot forms (allocation request coalescing, Sec. 4.2) reserve or free a
mask in one operation; a deallocation can be FIRST and EMPTY at once.
"""
from __future__ import annotations

ONES = (1 << 64) - 1


def pad(n: int) -> int:
    assert 1 <= n <= 64
    return ONES & ~((1 << n) - 1)


def initialized(n: int) -> int:
    """Allocation word right after initialize_block (Alg. 8)."""
    return pad(n)


def reserve_one(word: int):
    """Alg. 6 run by one thread with no contention: (new_word, pos or None, full)."""
    free = ~word & ONES
    if free == 0:
        return word, None, False
    pos = (free & -free).bit_length() - 1
    before = word
    word = before | (1 << pos)
    return word, pos, word == ONES


def reserve_mask(word: int, mask: int):
    """Coalesced reservation of ``mask``: (new_word, got, full)."""
    before = word
    word = before | mask
    got = mask & ~before & ONES
    return word, got, (word == ONES and got != 0)


def deallocate(word: int, mask: int, n: int):
    """Free ``mask``: (new_word, first, empty).  Precondition: mask live."""
    assert mask and (word & mask) == mask and (mask & pad(n)) == 0
    before = word
    word = before & ~mask & ONES
    return word, before == ONES, word == pad(n)


def invalidate(word: int, n: int):
    """Invalidation without contention: (new_word, success)."""
    before = word
    if before == ONES:
        return word, False
    if before == pad(n):
        return ONES, True
    return before, False          # rolled back: AND with before restores the word


def live_slots(word: int, n: int) -> int:
    return bin(word & ~pad(n) & ONES).count("1")
