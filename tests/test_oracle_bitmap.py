"""Pins of the sequential hierarchical bitmap (Sec. 4.1, Alg. 3-5, App. A.5)."""
import random

from oracle.bitmap_ref import HBitmap


def test_worked_example_clear_cascade():
    # Figure "bitmap_clear_example": 32 bits, container size 4.  clear(18)
    # clears the last bit of container 4, which clears bit 4 of the nested
    # bitmap, the last bit of its container 1, which clears bit 1 one level up.
    b = HBitmap(32, width=4)
    for pos in (1, 2, 7, 13, 18):          # bits 16, 17, 19 and 20..31 stay clear
        b.set(pos)
    assert b.consistent()
    assert b.levels()[1:] == [[0b1011, 0b0001], [0b11]]   # L1: containers 0,1,3 and 4
    b.trace.clear()
    b.clear(18)
    assert b.trace == [(0, "clear", 18), (1, "clear", 4), (2, "clear", 1)]
    assert b.consistent()
    assert b.levels() == [[0b0110, 0b1000, 0, 0b0010, 0, 0, 0, 0], [0b1011, 0], [0b01]]


def test_set_first_propagates_and_not_otherwise():
    b = HBitmap(32, width=4)
    b.set(18)
    assert b.trace == [(0, "set", 18), (1, "set", 4), (2, "set", 1)]
    b.trace.clear()
    b.set(17)                               # not the first bit of container 4
    assert b.trace == [(0, "set", 17)]


def test_levels_geometry_64():
    for n, nlev in ((1, 1), (64, 1), (65, 2), (4096, 2), (4097, 3), (2**18, 3), (2**18 + 1, 4)):
        b = HBitmap(n)
        assert len(b.levels()) == nlev, n
        assert len(b.levels()[-1]) == 1


def test_try_find_set_and_indices_bruteforce():
    rnd = random.Random(1)
    for n in (1, 5, 64, 65, 300, 4100):
        b = HBitmap(n, width=64)
        ref = set()
        for _ in range(3 * n):
            p = rnd.randrange(n)
            if p in ref:
                b.clear(p); ref.remove(p)
            else:
                b.set(p); ref.add(p)
            if rnd.random() < 0.05:
                assert b.consistent()
        assert b.consistent()
        assert b.indices() == sorted(ref)
        f = b.try_find_set()
        assert (f is None) == (not ref) and (f is None or f in ref)


def test_clear_any_drains_every_bit_once():
    b = HBitmap(300, width=8)
    for p in range(0, 300, 7):
        b.set(p)
    got = []
    while True:
        i = b.clear_any()
        if i is None:
            break
        got.append(i)
    assert sorted(got) == list(range(0, 300, 7))
    assert b.consistent() and b.levels()[-1] == [0]


def test_legal_multiset_final_state_is_the_set_surplus():
    # App. A.5, Lemma: a legal multiset of set/clear ops leaves every L0 bit at
    # initial + set-surplus and every level consistent, in any order.
    rnd = random.Random(7)
    for trial in range(40):
        n, w = rnd.choice([(64, 4), (200, 4), (1000, 64), (5000, 64)])
        init = {p for p in range(n) if rnd.random() < 0.3}
        ops = []
        for p in range(n):
            s = rnd.choice([-1, 0, 0, 1])
            if (p in init and s == 1) or (p not in init and s == -1):
                s = 0
            extra = rnd.randrange(3) if s == 0 and rnd.random() < 0.2 else 0
            ops += [("set", p)] * (max(s, 0) + extra) + [("clear", p)] * (max(-s, 0) + extra)
        # any order in which no op would have to wait forever: run set/clear
        # pairs so that the bit never needs to be set twice in a row
        rnd.shuffle(ops)
        b = HBitmap(n, width=w)
        for p in init:
            b.set(p)
        pending = list(ops)
        while pending:
            progressed = False
            for i, (op, p) in enumerate(pending):
                if (op == "set") != bool(b.get(p)):
                    (b.set if op == "set" else b.clear)(p)
                    pending.pop(i)
                    progressed = True
                    break
            assert progressed, "legal multiset must always let one op progress"
        want = set(init)
        for op, p in ops:
            pass
        surplus = {}
        for op, p in ops:
            surplus[p] = surplus.get(p, 0) + (1 if op == "set" else -1)
        want = {p for p in range(n) if (p in init) + surplus.get(p, 0) == 1}
        assert set(b.indices()) == want
        assert b.consistent()
