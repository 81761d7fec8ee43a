"""Pins of the two-class churn oracle (oracle/mix_ref.py) by an independent
per-lineage formulation: every object is the current member of one lineage
(id & 0x3FFFF), and a do-all visits the objects of its classes that exist when
it starts (Sec. 2.1).  With two do-alls per round (A, then B), an object that
the A do-all moves into B is visited again by the B do-all of the same round;
with one do-all over a class and its subclass, every lineage moves at most
once per round."""
import numpy as np
import pytest

from oracle import core, mix_ref

M64 = (1 << 64) - 1


def _step(seed, r, cls, i):
    h = core.splitmix64((seed ^ i ^ (r << 32)) & M64)
    if h & 1:
        return ("b" if (h >> 1) & 1 else "a", ((r + 1) << 18) | (i & 0x3FFFF)), True
    return (cls, i), False


def _lineages(seed, ids_a, ids_b, rounds, subtree):
    state = {int(i) & 0x3FFFF: ("a", int(i)) for i in ids_a}
    state.update({int(i) & 0x3FFFF: ("b", int(i)) for i in ids_b})
    out = []
    for r in range(rounds):
        for lin, (c, i) in list(state.items()):
            (c2, i2), moved = _step(seed, r, c, i)
            if not subtree and c == "a" and moved and c2 == "b":
                (c2, i2), _ = _step(seed, r, c2, i2)      # the B do-all of this round sees it
            state[lin] = (c2, i2)
        a = sorted(i for c, i in state.values() if c == "a")
        b = sorted(i for c, i in state.values() if c == "b")
        out.append((a, b))
    return out


@pytest.mark.parametrize("seed", [1, 42, 7])
@pytest.mark.parametrize("subtree", [False, True])
def test_mix_oracle_equals_per_lineage_formulation(seed, subtree):
    ids_a, ids_b = range(0, 300), range(300, 520)
    fn = mix_ref.run_subtree if subtree else mix_ref.run
    got = fn(seed, ids_a, ids_b, 8)
    want = _lineages(seed, ids_a, ids_b, 8, subtree)
    for (ga, gb), (wa, wb) in zip(got, want):
        assert ga.tolist() == wa and gb.tolist() == wb
        assert len(ga) + len(gb) == 520                   # one object per lineage
        lin = np.concatenate([ga, gb]) & 0x3FFFF
        assert np.unique(lin).size == 520


def test_mix_two_phases_differ_from_one_subtree_do_all():
    """The two readings must differ somewhere (else the pin above is weak)."""
    a = mix_ref.run(42, range(0, 300), range(300, 520), 3)
    b = mix_ref.run_subtree(42, range(0, 300), range(300, 520), 3)
    assert any(x[0].tolist() != y[0].tolist() for x, y in zip(a, b))
