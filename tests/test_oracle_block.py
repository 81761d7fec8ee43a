"""Pins of the block allocation-word rules (Alg. 6, 7, 8, 9; App. A.1-A.2)."""
import random

from oracle import block_ref as B

ONES = (1 << 64) - 1


def popc(v):
    return bin(v).count("1")


def test_capacity_64_reduces_to_printed_popcount_rules():
    rnd = random.Random(3)
    for _ in range(20000):
        word = rnd.getrandbits(64)
        if rnd.random() < 0.1:
            word = ONES & ~(1 << rnd.randrange(64))        # one free slot left
        # Alg. 6: FULL iff popc(before) = 63
        new, pos, full = B.reserve_one(word)
        if pos is None:
            assert word == ONES
        else:
            assert full == (popc(word) == 63)
            assert (word >> pos) & 1 == 0 and new == word | (1 << pos)
        # Alg. 7: EMPTY iff popc(before)=1, FIRST iff popc(before)=64
        live = word
        if live:
            slot = rnd.choice([i for i in range(64) if (live >> i) & 1])
            after, first, empty = B.deallocate(live, 1 << slot, 64)
            assert empty == (popc(live) == 1)
            assert first == (popc(live) == 64)
            assert after == live & ~(1 << slot)
        # Alg. 9: invalidation succeeds iff before = 0
        after, ok = B.invalidate(word, 64)
        assert ok == (word == 0)
        assert after == (ONES if ok else word)


def test_general_capacity_bruteforce():
    rnd = random.Random(4)
    for n in (1, 2, 42, 56, 63, 64):
        pad = B.pad(n)
        assert popc(pad) == 64 - n and pad & ((1 << n) - 1) == 0
        assert B.initialized(n) == pad
        for _ in range(3000):
            live = rnd.getrandbits(n) if n < 64 else rnd.getrandbits(64)
            word = pad | live
            # reservation of an arbitrary mask: full iff the word becomes all ones now
            mask = rnd.getrandbits(64) & ~pad & ONES
            new, got, full = B.reserve_mask(word, mask)
            free_before = [i for i in range(n) if not (word >> i) & 1]
            assert got == sum(1 << i for i in free_before if (mask >> i) & 1)
            assert full == (got != 0 and all((new >> i) & 1 for i in range(64)))
            # deallocation of a nonempty subset of the live slots
            if live:
                bits = [i for i in range(n) if (live >> i) & 1]
                sub = rnd.sample(bits, rnd.randint(1, len(bits)))
                m = sum(1 << i for i in sub)
                after, first, empty = B.deallocate(word, m, n)
                assert first == (len(bits) == n)           # block was full
                assert empty == (len(sub) == len(bits))    # no live slot left
                assert B.live_slots(after, n) == len(bits) - len(sub)
            # invalidation succeeds iff no live slot
            after, ok = B.invalidate(word, n)
            assert ok == (live == 0)


def test_capacity_one_block_is_first_and_empty():
    after, first, empty = B.deallocate(B.pad(1) | 1, 1, 1)
    assert first and empty and after == B.pad(1)
