"""GPU tests of subclassing (Sec. 3.2: a subclass's objects hold the
inherited SOA arrays first) and of the do-all over a class and its subclasses
(Sec. 2.1: parallel_do<T> runs on the objects of T and of its subtypes that
exist at launch, one kernel per type), through the C-ABI."""
import numpy as np
import pytest

from helpers import check_heap, say
from oracle import mix_ref

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def S():
    from paper_1810_11765_amd import smmo
    return smmo


# Base {i32 id, f32 x, f32 v}; Sub: Base + {f64 w}; Leaf: Sub + {}; Other {i32 id}
CLASSES = [[4, 4, 4], {"fields": [8], "super": 0}, {"fields": [], "super": 1}, [4]]
COUNTS = [700, 333, 129, 250]            # ragged: 34 + 28 + 11 + 4 blocks (capacities 21, 12, 12, 64)


def _populate(h):
    smmo = S()
    start = 0
    for t, n in enumerate(COUNTS):
        ids = torch.arange(start, start + n, dtype=torch.int32, device="cuda")
        x = torch.arange(n, dtype=torch.float32, device="cuda") * 0.25
        v = torch.ones(n, dtype=torch.float32, device="cuda")
        w = torch.full((n,), 2.5, dtype=torch.float64, device="cuda")
        srcs = [ids, x, v, w][: len(h.classes[t])]
        h.parallel_new(t, n, smmo.CTOR_ARRAYS, smmo.ctor_arrays(srcs))
        start += n
    return np.cumsum([0] + COUNTS)


@pytest.mark.parametrize("blocks", [128, 300_000])      # flat scan; level-1 block list
def test_do_all_over_class_visits_its_subclasses_once(blocks):
    say("subclass visit", blocks)
    smmo = S()
    h = smmo.Heap(CLASSES, blocks)
    assert h.classes == [[4, 4, 4], [4, 4, 4, 8], [4, 4, 4, 8], [4]]
    edges = _populate(h)
    assert h.status() == 0
    total = int(edges[-1])
    for root, covered in ((0, (0, 1, 2)), (1, (1, 2)), (2, (2,)), (3, (3,))):
        visits = torch.zeros(total, dtype=torch.int32, device="cuda")
        h.parallel_do(root, smmo.M_VISIT, smmo.VisitArgs(visits.data_ptr()))
        got = visits.cpu().numpy()
        want = np.zeros(total, dtype=np.int32)
        for t in covered:
            want[edges[t]:edges[t + 1]] = 1
        assert np.array_equal(got, want), f"do-all over class {root}"
    # inherited fields keep their indices in the subclass
    ids, x, v, w = h.dump_objects(1, [np.int32, np.float32, np.float32, np.float64])
    o = np.argsort(ids)
    assert np.array_equal(ids[o], np.arange(edges[1], edges[2]))
    assert np.array_equal(x[o], np.arange(COUNTS[1], dtype=np.float32) * 0.25)
    assert (v == 1).all() and (w == 2.5).all()
    check_heap(h, expect_live=COUNTS)


def test_axpy_over_class_and_subclasses():
    say("subclass axpy")
    smmo = S()
    h = smmo.Heap(CLASSES, 128)
    _populate(h)
    assert h.status() == 0
    h.parallel_do(0, smmo.M_AXPY, smmo.AxpyArgs(0.5, 1, 2, 0))
    for t in (0, 1, 2):
        fields = h.dump_objects(t, [np.int32, np.float32, np.float32] + ([np.float64] if t else []))
        ids, x, v = fields[:3]
        assert np.array_equal(v, np.float32(1) + np.float32(0.5) * x), f"class {t}"
    (oid,) = h.dump_objects(3, [np.int32])
    assert oid.size == COUNTS[3]


@pytest.mark.parametrize("blocks,flags", [(64, 0), (96, 8), (300_000, 0)])
def test_churn_over_class_and_subclass_matches_oracle(blocks, flags):
    """Each round one do-all over A covers A and its subclass B; objects it
    re-creates in A or B are not visited by the same do-all."""
    say("subclass churn", blocks, flags)
    smmo = S()
    seed = 5
    h = smmo.Heap([[4], {"fields": [4], "super": 0}], blocks)
    h.set_tuning(flags, 5, 200000)
    lineages = 1200
    half = 700
    ids = torch.arange(lineages, dtype=torch.int32, device="cuda")
    h.parallel_alloc(0, half, 1, smmo.CTOR_ARRAYS, smmo.ctor_arrays([ids[:half]]))
    h.parallel_alloc(1, lineages - half, 1, smmo.CTOR_ARRAYS, smmo.ctor_arrays([ids[half:], None]))
    want = mix_ref.run_subtree(seed, range(half), range(half, lineages), 10)
    for r in range(10):
        h.parallel_do(0, smmo.M_MIX, smmo.MixArgs(seed, r, 0, 1, 0))
        a = np.sort(h.dump_objects(0, [np.int32])[0])
        b = np.sort(h.dump_objects(1, [np.int32, np.int32])[0])
        assert np.array_equal(a, want[r][0]) and np.array_equal(b, want[r][1]), f"round {r}"
    check_heap(h, expect_live=[len(want[-1][0]), len(want[-1][1])])


def test_nbody_methods_refuse_a_class_with_subclasses():
    smmo = S()
    h = smmo.Heap([[4] * 5, {"fields": [4], "super": 0}], 16)
    with pytest.raises(smmo.SmmoError, match="subclasses"):
        h.parallel_do(0, smmo.M_NBODY_MOVE, smmo.NbodyArgs())


@pytest.mark.parametrize("blocks", [128, 300_000])      # flat scan; level-1 block list
def test_do_all_from_snapshot_skips_later_objects(blocks):
    """smmo_snapshot then smmo_parallel_do_snapshot: objects created after the
    snapshot, in the class or a subclass, are not visited; the recorded ones
    are visited once."""
    say("snapshot do-all", blocks)
    smmo = S()
    h = smmo.Heap(CLASSES, blocks)
    edges = _populate(h)
    first = int(edges[-1])
    h.snapshot(0)
    extra = [90, 45]                                    # more objects of class 0 and of its subclass 1
    start = first
    for t, n in enumerate(extra):
        ids = torch.arange(start, start + n, dtype=torch.int32, device="cuda")
        srcs = [ids, None, None, None][: len(h.classes[t])]
        h.parallel_new(t, n, smmo.CTOR_ARRAYS, smmo.ctor_arrays(srcs))
        start += n
    assert h.status() == 0
    visits = torch.zeros(start, dtype=torch.int32, device="cuda")
    h.parallel_do(0, smmo.M_VISIT, smmo.VisitArgs(visits.data_ptr()), from_snapshot=True)
    got = visits.cpu().numpy()
    want = np.zeros(start, dtype=np.int32)
    for t in (0, 1, 2):
        want[edges[t]:edges[t + 1]] = 1
    assert np.array_equal(got, want)
    visits.zero_()
    h.parallel_do(0, smmo.M_VISIT, smmo.VisitArgs(visits.data_ptr()))     # live now: everything in the subtree
    want[first:] = 1
    assert np.array_equal(visits.cpu().numpy(), want)
    with pytest.raises(smmo.SmmoError, match="snapshot"):
        h.parallel_do(0, smmo.M_AXPY, smmo.AxpyArgs(0.5, 1, 2, 0), from_snapshot=True)
    check_heap(h, expect_live=[COUNTS[0] + extra[0], COUNTS[1] + extra[1], COUNTS[2], COUNTS[3]])
