"""GPU parity of the allocator path (heap create, parallel_new, device-side
allocation with request coalescing, do-all sweep and churn, destruction)
against the CPU oracle, through the C-ABI.  Bit-exact: every value here is an
integer or an FP32 result of one rounding that both sides form identically."""
import numpy as np
import pytest

from helpers import bits_equal, check_heap, say
from oracle import core, mix_ref
from paper_1810_11765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1810_11765_amd import smmo  # noqa: F401  (fails loudly if the library is missing)


def S():
    from paper_1810_11765_amd import smmo
    return smmo


def W():
    from paper_1810_11765_amd import workloads
    return workloads


@pytest.mark.parametrize("M", [1, 63, 64, 65, 4096, 4097, 262145])
def test_heap_create_is_consistent_and_empty(M):
    say("create", M)
    h = S().Heap([[4, 4, 1], [4, 4]], M)
    s = check_heap(h, expect_live=[0, 0])
    assert s["free"] == M and s["blocks"] == [0, 0]


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4096])
def test_parallel_new_dense_ascending(n):
    say("parallel_new", n)
    smmo = S()
    h = smmo.Heap([[4, 4, 4]], 64)
    ids = torch.arange(n, dtype=torch.int32, device="cuda")
    h.parallel_new(0, n, smmo.CTOR_ARRAYS, smmo.ctor_arrays([ids, None, ids]))
    got_id, x, v = h.dump_objects(0, [np.int32, np.float32, np.int32])
    assert np.array_equal(got_id, np.arange(n))           # block order = id order
    assert (x == 0).all() and np.array_equal(v, np.arange(n))
    refs = h.dump_refs(0)
    blocks = (refs >> np.uint64(6)) & np.uint64((1 << 44) - 1)
    assert np.array_equal(blocks, np.arange(n) // 64)     # lowest blocks, dense
    s = check_heap(h, expect_live=[n])
    assert s["blocks"] == [(n + 63) // 64]


def test_parallel_new_oom_creates_nothing():
    say("parallel_new oom")
    smmo = S()
    h = smmo.Heap([[4]], 4)
    with pytest.raises(smmo.SmmoError):
        h.parallel_new(0, 5 * 64, smmo.CTOR_ZERO)        # more blocks than the heap has
    h.parallel_new(0, 3 * 64 + 5, smmo.CTOR_ZERO)
    h.parallel_new(0, 64, smmo.CTOR_ZERO)                 # only 0 blocks left: device OOM
    assert h.status() & smmo.STATUS_OOM
    h.clear_status()
    s = check_heap(h, expect_live=[3 * 64 + 5])
    assert s["free"] == 0


def _oracle_states(seed, nthreads, per, rounds):
    ids, x, v = inputs.alloc_bench_initial(seed, nthreads, per)
    return core.c1_run(seed, ids, x, v, rounds)


@pytest.mark.parametrize("seed", [42, 7, 1234])
def test_alloc_microbench_parity(seed):
    """65,536 threads x 4 device allocations into exactly 4096 x 64 slots,
    then 10 rounds of sweep + churn; live set bit-exact after every round."""
    say("alloc microbench", seed)
    wl = W().AllocBench(seed=seed)
    wl.initial_alloc()
    ids, x, v = wl.state()
    i0, x0, v0 = wl.init_arrays
    assert np.array_equal(ids, i0) and bits_equal(x, x0) and bits_equal(v, v0)
    s = check_heap(wl.heap, expect_live=[262144])
    assert s["blocks"] == [4096] and s["free"] == 0           # 100% fill, no OOM
    want = _oracle_states(seed, 65536, 4, 10)
    for r in range(10):
        say("alloc microbench round", seed, r)
        wl.round(r)
        ids, x, v = wl.state()
        wi, wx, wv = want[r]
        assert np.array_equal(ids, wi), f"round {r}: live ids differ"
        assert bits_equal(x, wx) and bits_equal(v, wv), f"round {r}: field values differ"
        check_heap(wl.heap, expect_live=[262144])


@pytest.mark.parametrize("seed", [42, 7])
def test_alloc_microbench_through_the_device_api_header(seed):
    """The churn round written against include/smmo_device.h only
    (smmo_alloc, smmo_destroy_self, smmo_field; SMMO_M_CHURN_API): the same
    microbenchmark, bit-exact against the oracle after every round, on heaps
    of 4,096 blocks (exactly full) and of 4,500 blocks (spare blocks)."""
    smmo = S()
    for blocks in (4096, 4500):
        say("alloc microbench via device API", seed, blocks)
        wl = W().AllocBench(seed=seed, num_blocks=blocks)
        wl.initial_alloc()
        want = _oracle_states(seed, 65536, 4, 6)
        for r in range(6):
            wl.sweep()
            wl.heap.parallel_do(0, smmo.M_CHURN_API, smmo.ChurnArgs(seed, r, 0))
            ids, x, v = wl.state()
            wi, wx, wv = want[r]
            assert np.array_equal(ids, wi), f"round {r}: live ids differ"
            assert bits_equal(x, wx) and bits_equal(v, wv), f"round {r}: field values differ"
            check_heap(wl.heap, expect_live=[262144])


@pytest.mark.parametrize("seed", [42, 5])
def test_capacity_one_class_churn_matches_oracle(seed):
    """A class of capacity 1 (44-byte objects next to a 1-byte class: N =
    floor(64 * 1 / 44) = 1): every allocation takes a whole block and every
    destruction is both FIRST and EMPTY (App. A.1 / Alg. 7), so the block is
    set active and then invalidated and freed at once.  The alloc microbench
    rounds (sweep + churn) on it, bit-exact against the oracle."""
    smmo = S()
    nthreads, per, rounds = 1000, 2, 4
    classes = [[1], [4, 4, 4, 8, 8, 8, 8]]
    h = smmo.Heap(classes, nthreads * per + 130)
    assert h.capacity(1) == 1 and h.capacity(0) == 64
    ids, x, v = inputs.alloc_bench_initial(seed, nthreads, per)
    src = [torch.from_numpy(a).cuda() for a in (ids, x, v)] + [None] * 4
    say("capacity 1 alloc", seed)
    h.parallel_alloc(1, nthreads, per, smmo.CTOR_ARRAYS, smmo.ctor_arrays(src))
    s = check_heap(h, expect_live=[0, nthreads * per])
    assert s["blocks"] == [0, nthreads * per]
    want = _oracle_states(seed, nthreads, per, rounds)
    dt = [np.int32, np.float32, np.float32] + [np.uint64] * 4
    for r in range(rounds):
        say("capacity 1 round", seed, r)
        h.parallel_do(1, smmo.M_AXPY, smmo.AxpyArgs(0.5, 1, 2, 0))
        h.parallel_do(1, smmo.M_CHURN, smmo.ChurnArgs(seed, r, 0))
        gi, gx, gv = h.dump_objects(1, dt)[:3]
        o = np.argsort(gi, kind="stable")
        wi, wx, wv = want[r]
        assert np.array_equal(gi[o], wi), f"round {r}: live ids differ"
        assert bits_equal(gx[o], wx) and bits_equal(gv[o], wv), f"round {r}: field values differ"
        s = check_heap(h, expect_live=[0, nthreads * per])
        assert s["blocks"] == [0, nthreads * per]


@pytest.mark.parametrize("blocks,rounds", [(1, 2000), (96, 2000), (4099, 200), (65536, 40)])
def test_publication_order_message_passing(blocks, rounds):
    """smmo_check_publish_order: the allocator's block initialization
    (type, then the word once the type store has completed) against its
    reservation (OR on the word, then the type): writer waves re-initialize
    blocks round after round while reader waves on every XCD OR into random
    blocks and read the type; no reader may see a word newer than the type.
    Bounded: no wave waits for another."""
    import ctypes as C
    say("publish order", blocks, rounds)
    L = S().lib()
    L.smmo_check_publish_order.argtypes = [C.c_void_p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_void_p,
                                           C.c_void_p]
    L.smmo_check_publish_order.restype = C.c_int
    nbytes = (20 * blocks + 7) // 8 * 8
    buf = torch.empty(nbytes // 8, dtype=torch.int64, device="cuda")
    out = torch.full((4,), 7, dtype=torch.int64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    S().check(L.smmo_check_publish_order(buf.data_ptr(), nbytes, blocks, rounds, 5, out.data_ptr(), stream))
    samples, fresh, bad, first = out.cpu().tolist()
    assert bad == 0, f"{bad} readers saw a newer word than type (first: block {first >> 32}, type {first & 0xFFFFFFFF})"
    assert samples > 0 and fresh > samples // 2, (samples, fresh)
    # the writers ran to completion: every block ends at the last round
    words = buf[:blocks].cpu().numpy().view(np.uint64) >> np.uint64(32)
    types = buf.cpu().numpy().view(np.uint32)[4 * blocks:5 * blocks]
    assert (words == rounds).all() and (types == rounds).all()
    with pytest.raises(S().SmmoError):
        S().check(L.smmo_check_publish_order(buf.data_ptr(), nbytes - 8, blocks + 1, rounds, 5, out.data_ptr(), stream))


@pytest.mark.parametrize("block_objects,fraction,seed", [(64, 0.5, 1), (64, 1.0, 2), (32, 0.6, 3)])
def test_destroy_by_handle_across_blocks(block_objects, fraction, seed):
    """Destroys whose lanes hold handles of many blocks and of two classes at
    once (a random permutation of every live handle, 64 to a wave): each
    block group's deallocation goes out as one lane-parallel atomic, and only
    the groups that need it take Alg. 2's state update (a full block becomes
    active, an emptied block is invalidated and freed; with 32 objects per
    block both classes have padding slots).  Afterwards every heap invariant
    holds, each class has exactly its survivors, and a full destroy leaves
    every block free (App. A.1, Alg. 2, 7, 9)."""
    say(f"destroy by handle across blocks: {block_objects} objects per block, fraction {fraction}")
    H = S().Heap([[4, 4, 4], [8, 8, 8, 8]], 8192, block_objects=block_objects)
    H.parallel_alloc(0, 8192, 8, S().CTOR_NONE)
    H.parallel_alloc(1, 4096, 8, S().CTOR_NONE)
    r0, r1 = H.dump_refs(0), H.dump_refs(1)
    assert len(r0) == 8192 * 8 and len(r1) == 4096 * 8
    refs = np.concatenate([r0, r1])
    perm = np.random.default_rng(seed).permutation(len(refs))
    k = int(len(refs) * fraction)
    gone = np.ascontiguousarray(refs[perm[:k]])
    H.parallel_destroy(torch.from_numpy(gone.view(np.int64)).cuda(), k, 1)
    keep = set(refs[perm[k:]].tolist())
    left0 = int((S().ref_class(refs[perm[k:]]) == 0).sum())
    summary = check_heap(H, expect_live=[left0, len(keep) - left0])
    assert set(H.dump_refs(0).tolist()) | set(H.dump_refs(1).tolist()) == keep
    if fraction == 1.0:
        assert summary["blocks"] == [0, 0] and summary["free"] == 8192
    H.close()


def test_every_live_object_visited_exactly_once():
    say("visit")
    smmo = S()
    wl = W().AllocBench(seed=5, num_blocks=512, nthreads=4096, per_thread=6)
    wl.initial_alloc()
    for r in range(3):
        wl.round(r)
    visits = torch.zeros(11 << 18, dtype=torch.int32, device="cuda")
    wl.heap.parallel_do(0, smmo.M_VISIT, smmo.VisitArgs(visits.data_ptr()))
    ids, _, _ = wl.state()
    vis = visits.cpu().numpy()
    assert (vis[ids] == 1).all()
    assert vis.sum() == len(ids) == 4096 * 6


def test_destroy_all_frees_every_block():
    say("destroy all")
    smmo = S()
    wl = W().AllocBench(seed=3, num_blocks=300, nthreads=4000, per_thread=3)
    wl.initial_alloc()
    wl.round(0)
    wl.heap.parallel_do(0, smmo.M_DESTROY_ALL)
    s = check_heap(wl.heap, expect_live=[0])
    assert s["free"] == 300


@pytest.mark.parametrize("flags,lookups,ppm", [
    (0, 5, 0),
    (1, 5, 0),            # no rotation
    (2, 5, 0),            # no coalescing: one slot per reservation
    (3, 1, 0),            # neither, single lookup
    (8, 5, 300000),       # 30% forced lookup failures: extra slow paths
    (8, 2, 900000),
])
def test_microbench_under_tuning_and_faults(flags, lookups, ppm):
    """Ragged sizes (4000 threads x 3 into 200 blocks, ~94% full) with the
    allocator switched to the ablation / fault-injection paths."""
    say("tuning", flags, lookups, ppm)
    smmo = S()
    seed = 11
    wl = W().AllocBench(seed=seed, num_blocks=200, nthreads=4000, per_thread=3)
    wl.heap.set_tuning(flags | smmo.TUNE_STATS, lookups, ppm)
    wl.initial_alloc()
    want = _oracle_states(seed, 4000, 3, 6)
    for r in range(6):
        wl.round(r)
        ids, x, v = wl.state()
        assert np.array_equal(ids, want[r][0]) and bits_equal(v, want[r][2])
        check_heap(wl.heap, expect_live=[12000])
    st = wl.heap.stats()
    assert st["alloc_obj"] == 12000 + sum(int((want[r][0] >> 18 == r + 1).sum()) for r in range(6))
    if flags & 8:
        assert st["find_fail"] > 0
    if flags & 2:
        assert st["reserve_atomic"] >= st["alloc_obj"]       # one atomic per object


@pytest.mark.parametrize("blocks,lineages,flags", [(16, 300, 0), (48, 1000, 0), (48, 1000, 8), (12, 200, 1)])
def test_two_class_churn_type_changes(blocks, lineages, flags):
    """Objects hop between two classes of different capacity (64 and 32) on a
    tiny heap, so freed blocks change type under concurrent allocation."""
    say("mix", blocks, lineages, flags)
    smmo = S()
    seed = 99
    h = smmo.Heap([[4], [4, 4]], blocks)
    h.set_tuning(flags | smmo.TUNE_STATS, 5, 200000)
    ids = torch.arange(lineages, dtype=torch.int32, device="cuda")
    half = lineages // 2
    h.parallel_alloc(0, half, 1, smmo.CTOR_ARRAYS, smmo.ctor_arrays([ids[:half]]))
    h.parallel_alloc(1, lineages - half, 1, smmo.CTOR_ARRAYS, smmo.ctor_arrays([ids[half:], None]))
    want = mix_ref.run(seed, range(half), range(half, lineages), 12)
    for r in range(12):
        for cls in (0, 1):
            h.parallel_do(cls, smmo.M_MIX, smmo.MixArgs(seed, r, 0, 1, 0))
        a = np.sort(h.dump_objects(0, [np.int32])[0])
        b = np.sort(h.dump_objects(1, [np.int32, np.int32])[0])
        assert np.array_equal(a, want[r][0]) and np.array_equal(b, want[r][1]), f"round {r}"
        check_heap(h, expect_live=[len(want[r][0]), len(want[r][1])])
    st = h.stats()
    print("[stats]", st, flush=True)
    assert st["block_init"] > 0


@pytest.mark.parametrize("drivers,blocks,lanes,iters,flags", [
    (64 * 256, 256 + 16, 1, 200, 0),      # 256 waves, one allocation each, into 16 blocks
    (64 * 256, 256 + 12, 1, 200, 1),      # same without rotation
    (64 * 512, 512 + 40, 2, 100, 0),      # 512 waves, two lanes each (coalesced pairs)
    (64 * 128, 128 + 8, 1, 300, 8),       # forced lookup failures: extra slow paths
    (64 * 256, 256 + 10, 1, 60, 16),      # paused picks: blocks change type under a pick
])
def test_allocation_storm_forces_rollbacks(drivers, blocks, lanes, iters, flags):
    """Many waves allocate and free in the same few blocks at once: blocks
    empty, are invalidated and re-initialized to the other class while other
    waves hold stale picks.  Afterwards nothing of either class is left, the
    heap is consistent and no bounded retry gave up."""
    say("storm", drivers, blocks, lanes, iters, flags)
    smmo = S()
    h = smmo.Heap([[4], [4], [4, 4]], blocks)         # drivers, class a (cap 64), class b (cap 32)
    h.set_tuning(flags | smmo.TUNE_STATS, 5, 250000)
    h.parallel_new(0, drivers, smmo.CTOR_ZERO)
    h.parallel_do(0, smmo.M_STRESS, smmo.StressArgs(7, iters, lanes, 1, 2))
    st = h.stats()
    print("[stats]", st, flush=True)
    s = check_heap(h, expect_live=[drivers, 0, 0])
    assert s["free"] == blocks - drivers // 64
    waves = drivers // 64
    assert st["alloc_obj"] == st["free_obj"] == waves * lanes * iters
    assert st["block_free"] > 0
    if flags & 16:
        assert st["type_rollback"] > 0        # the Alg. 1 rollback path really ran
