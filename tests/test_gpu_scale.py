"""GPU tests of the allocator's measurement paths through the C-ABI:

* big heaps, where the do-all, the iteration snapshot and the live count go
  through level 1 of the allocated bitmap (Sec. 6.5) -- predator-prey results
  bit-exact against the oracle with and without that skip;
* the allocator variants of the ablations (no rotation, no request
  coalescing, r = 1..8 lookups, Sec. 6.3) -- placement changes, results do
  not;
* the occupancy / fragmentation query against the raw-dump checker;
* raw allocation without constructor and device-side destroy by handle
  (the raw allocation benchmark of Sec. 6.4).
"""
import numpy as np
import pytest

from helpers import check_heap, say, wator_check
from oracle import core, heapcheck

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")


def S():
    from paper_1810_11765_amd import smmo
    return smmo


def W():
    from paper_1810_11765_amd import workloads
    return workloads


def _occupancy_matches_dump(heap, summary):
    occ = heap.occupancy()
    raw = heapcheck.RawHeap(heap.dump_raw())
    assert occ["used"] == summary["live"]
    assert occ["blocks"] == summary["blocks"]
    assert occ["slots"] == [b * heap.capacity(t) for t, b in enumerate(summary["blocks"])]
    assert abs(occ["F"] - heapcheck.fragmentation(raw)) < 1e-12
    return occ


# 270,000 blocks: 4,219 level-0 words, above the block-list threshold of 4,096
@pytest.mark.parametrize("flat", [False, True])
def test_wator_big_heap_parity(flat):
    say("wator big heap", "flat" if flat else "block list")
    w = W().WaTor(seed=11, width=193, height=97, num_blocks=270_000)
    if flat:
        w.heap.set_tuning(S().TUNE_FLAT_ENUM)
    w.populate()
    for s in range(1, 81):
        w.step()
        if s in (1, 80):
            summary = wator_check(w, s, core.c3_run(w.kind0, 193, 97, 11, s))
    _occupancy_matches_dump(w.heap, summary)


VARIANTS = [("default", 0, 5), ("noshift", 1, 5), ("nocoal", 2, 5), ("nocoal-noshift", 3, 5),
            ("r1", 0, 1), ("r2", 0, 2), ("r3", 0, 3), ("r8", 0, 8), ("rotated-start", 64, 5)]


@pytest.mark.parametrize("name,flags,lookups", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_wator_allocator_variants_parity(name, flags, lookups):
    say("wator variant", name)
    w = W().WaTor(seed=21, width=160, height=144, num_blocks=1024)
    w.heap.set_tuning(flags, lookups)
    w.populate()
    for _ in range(60):
        w.step()
    summary = wator_check(w, 60, core.c3_run(w.kind0, 160, 144, 21, 60))
    occ = _occupancy_matches_dump(w.heap, summary)
    assert 0.0 <= occ["F"] < 1.0


def _aligned_heap(classes, num_blocks, fill):
    nbytes = S().heap_bytes(classes, num_blocks)
    buf = torch.full((nbytes + 4096,), fill, dtype=torch.uint8, device="cuda")
    base = buf.data_ptr() + (-buf.data_ptr()) % 256
    return buf, S().Heap(classes, num_blocks, dev_ptr=base)


def test_raw_alloc_untouched_then_destroy_by_handle():
    say("raw alloc / destroy")
    classes = [[8] * 8]                                   # one 64-byte class, N = 64
    buf, h = _aligned_heap(classes, 64, 0xAB)
    nthreads, per = 1000, 3                               # ragged last wave
    refs = torch.zeros(nthreads * per, dtype=torch.int64, device="cuda")
    h.parallel_alloc(0, nthreads, per, S().CTOR_NONE, S().ctor_none(refs))
    r = refs.cpu().numpy().view(np.uint64)
    assert (r != 0).all() and np.unique(r).size == r.size
    assert (S().ref_class(r) == 0).all()
    summary = check_heap(h, expect_live=[nthreads * per])
    fields = h.dump_objects(0, [np.uint64] * 8)
    assert all((f == np.uint64(0xABABABABABABABAB)).all() for f in fields), "object memory was written"
    _occupancy_matches_dump(h, summary)
    h.parallel_destroy(refs, nthreads, per)
    summary = check_heap(h, expect_live=[0])
    assert summary["free"] == 64 and summary["blocks"] == [0]
    h.close()
    del buf


def test_raw_alloc_oom_gives_null_handles():
    say("raw alloc oom")
    classes = [[8] * 8]
    buf, h = _aligned_heap(classes, 8, 0)                 # 512 slots
    nthreads, per = 300, 2                                # 600 requests
    refs = torch.zeros(nthreads * per, dtype=torch.int64, device="cuda")
    h.parallel_alloc(0, nthreads, per, S().CTOR_NONE, S().ctor_none(refs))
    assert h.status() & S().STATUS_OOM
    r = refs.cpu().numpy().view(np.uint64)
    got = r[r != 0]
    assert np.unique(got).size == got.size
    assert got.size == 512, "every slot of the heap is handed out before OOM"
    h.clear_status()
    check_heap(h, expect_live=[512])
    assert h.occupancy()["F"] == 0.0
    h.parallel_destroy(refs, nthreads, per)             # null handles are skipped
    summary = check_heap(h, expect_live=[0])
    assert summary["free"] == 8
    h.close()
    del buf


def test_raw_alloc_full_size_then_destroy():
    """16,384 threads x 64 objects of 64 B in a 1 GiB heap, then destroy all."""
    say("raw alloc 16384 x 64")
    ls = W().LinuxScalability()
    ls.alloc(64)
    assert ls.heap.status() == 0
    assert ls.heap.live_count(0) == 16384 * 64
    r = ls.refs[: 16384 * 64].cpu().numpy().view(np.uint64)
    assert (r != 0).all() and np.unique(r).size == r.size
    ls.free(64)
    assert ls.heap.live_count(0) == 0
    occ = ls.heap.occupancy()
    assert occ["blocks"] == [0] and ls.heap.status() == 0


def test_atomic_probe_sets_every_bit_it_targets():
    """The atomic-throughput reference kernel: thread t ORs bit (t + r) & 63
    into word (t / lanes) % nwords for r < rounds."""
    say("atomic probe")
    S_ = S()
    for lanes, nwords, nthreads, rounds in ((1, 1000, 3000, 2), (64, 7, 64 * 20 + 5, 3)):
        words = torch.zeros(nwords, dtype=torch.int64, device="cuda")
        S_.atomic_probe(words, lanes, nthreads, rounds)
        got = words.cpu().numpy().view(np.uint64)
        want = np.zeros(nwords, dtype=np.uint64)
        for t in range(nthreads):
            for r in range(rounds):
                want[(t // lanes) % nwords] |= np.uint64(1) << np.uint64((t + r) & 63)
        assert np.array_equal(got, want)


@pytest.mark.parametrize("M", [1, 2, 65, 4097, 262145])
def test_empty_class_and_fill_to_capacity_twice(M):
    """Degenerate cases on heaps of one to 262,145 blocks (one bitmap level up
    to three, flat scan and level-1 block list): zero-sized operations, a
    do-all over a class with no object, then device allocation of every slot
    of one class and destruction by handle, twice (the second round re-uses
    invalidated blocks)."""
    say("edges", M)
    S_ = S()
    h = S_.Heap([[4, 4, 4], [8]], M)                      # capacities 42 and 64
    cap = h.capacity(0) * M
    visits = torch.zeros(8, dtype=torch.int32, device="cuda")
    h.parallel_do(0, S_.M_VISIT, S_.VisitArgs(visits.data_ptr()))
    h.parallel_do(1, S_.M_DESTROY_ALL)
    refs = torch.zeros(cap, dtype=torch.int64, device="cuda")
    h.parallel_new(0, 0)
    h.parallel_alloc(0, 0, 1)
    h.parallel_destroy(refs, 0, 1)
    assert int(visits.sum()) == 0 and h.live_count(0) == 0 and h.live_count(1) == 0
    occ = h.occupancy()
    assert occ["blocks"] == [0, 0] and occ["F"] == 0.0
    for _ in range(2):
        refs.zero_()
        h.parallel_alloc(0, cap, 1, S_.CTOR_NONE, S_.ctor_none(refs))
        r = refs.cpu().numpy().view(np.uint64)
        assert (r != 0).all() and np.unique(r).size == cap
        summary = check_heap(h, expect_live=[cap, 0])
        assert summary["free"] == 0 and h.occupancy()["F"] == 0.0
        h.parallel_destroy(refs, cap, 1)
        summary = check_heap(h, expect_live=[0, 0])
        assert summary["free"] == M


LAUNCHES = [dict(), dict(doall_waves_per_cu=1, doall_units=64), dict(doall_waves_per_cu=64, doall_units=1 << 20),
            dict(list_min_words=1), dict(sweep_waves_per_cu=1, sweep_groups=1), dict(sweep_groups=2)]


@pytest.mark.parametrize("launch", LAUNCHES, ids=[str(i) for i in range(len(LAUNCHES))])
def test_launch_shapes_do_not_change_results(launch):
    """Extreme launch shapes (one wave per CU, 64-bit units, a block list even
    for a small heap, a one-wave sweep): predator-prey equals the oracle and
    the sweep gives the same values."""
    say("launch", launch)
    S_ = S()
    w = W().WaTor(seed=31, width=96, height=80, num_blocks=512)
    w.heap.set_launch(**launch)
    got = w.heap.get_launch()
    assert all(got[k] == v for k, v in launch.items())
    w.populate()
    for _ in range(40):
        w.step()
    wator_check(w, 40, core.c3_run(w.kind0, 96, 80, 31, 40))
    h = S_.Heap([[4, 4, 4]], 300)
    h.set_launch(**launch)
    n = 300 * 64 - 5
    x = torch.arange(n, dtype=torch.float32, device="cuda") * 0.25
    h.parallel_new(0, n, S_.CTOR_ARRAYS, S_.ctor_arrays([None, x, None]))
    for _ in range(3):
        h.parallel_do(0, S_.M_AXPY, S_.AxpyArgs(0.5, 1, 2, 0))
    ids, xv, v = h.dump_objects(0, [np.int32, np.float32, np.float32])
    xs = np.arange(n, dtype=np.float32) * np.float32(0.25)
    want = np.zeros(n, dtype=np.float32)
    for _ in range(3):
        want = want + np.float32(0.5) * xs
    assert np.array_equal(v, want)
    # the same sweep through the generic do-all kernel, after destroying a
    # third of the objects (holes in blocks)
    refs = torch.from_numpy(h.dump_refs(0).astype(np.int64)[::3].copy()).cuda()
    h.parallel_destroy(refs, refs.numel(), 1)
    h.parallel_do(0, S_.M_AXPY_GENERIC, S_.AxpyArgs(0.5, 1, 2, 0))
    ids, xv, v = h.dump_objects(0, [np.int32, np.float32, np.float32])
    keep = np.ones(n, dtype=bool)
    keep[::3] = False
    assert np.array_equal(v, (want + np.float32(0.5) * xs)[keep])


def test_launch_shape_rejects_out_of_range():
    S_ = S()
    h = S_.Heap([[4]], 8)
    for bad in (dict(doall_waves_per_cu=65), dict(doall_units=63), dict(sweep_groups=3), dict(sweep_waves_per_cu=2000)):
        with pytest.raises(S_.SmmoError):
            h.set_launch(**bad)
    assert h.get_launch() == {"doall_waves_per_cu": 32, "doall_units": 16384, "list_min_words": 4096,
                              "sweep_waves_per_cu": 128, "sweep_groups": 4}


def test_timing_hook_records_the_kernel_alone():
    """smmo_time_next_doall: the next do-all kernel records the two events at
    its own start and end; its duration is positive and within the events
    recorded around the call, and the do-all's result is unchanged."""
    say("timing hook")
    S_ = S()
    h = S_.Heap([[4, 4, 4]], 256)
    n = 256 * 21 - 7
    ids = torch.arange(n, dtype=torch.int32, device="cuda")
    h.parallel_new(0, n, S_.CTOR_ARRAYS, S_.ctor_arrays([ids, None, None]))
    for _ in range(2):                                   # the hook applies to one launch only
        visits = torch.zeros(n, dtype=torch.int32, device="cuda")
        outer_a, outer_b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        h.time_next_doall(a, b)
        outer_a.record()
        h.parallel_do(0, S_.M_VISIT, S_.VisitArgs(visits.data_ptr()))
        outer_b.record()
        torch.cuda.synchronize()
        own, around = a.elapsed_time(b), outer_a.elapsed_time(outer_b)
        assert 0.0 < own <= around + 1e-3, (own, around)
        assert (visits.cpu().numpy() == 1).all()
    visits.zero_()
    h.parallel_do(0, S_.M_VISIT, S_.VisitArgs(visits.data_ptr()))  # no pending request: a plain launch
    assert (visits.cpu().numpy() == 1).all()


def test_timing_request_is_dropped_by_other_calls_and_taken_by_the_sweep():
    """A pending smmo_time_next_doall request belongs to the next do-all call:
    another entry point in between (a live count) drops it, so the later
    do-all leaves the events where they were; the streaming sweep and the
    n-body force kernel take a request like the generic do-all."""
    say("timing request scope")
    S_ = S()
    h = S_.Heap([[4, 4, 4]], 256)
    n = 256 * 64
    h.parallel_new(0, n, S_.CTOR_ZERO)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h.time_next_doall(a, b)                      # the binding records both once to create them
    torch.cuda._sleep(50_000_000)                # tens of ms between those records and the do-all
    mark = torch.cuda.Event(enable_timing=True)
    mark.record()
    assert h.live_count(0) == n                  # drops the request
    h.parallel_do(0, S_.M_AXPY, S_.AxpyArgs(0.5, 1, 2, 0))
    torch.cuda.synchronize()
    assert a.elapsed_time(mark) > 1.0, "the do-all after another call recorded a dropped request"
    # taken by the sweep itself
    a2, b2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h.time_next_doall(a2, b2)
    o1, o2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    o1.record()
    h.parallel_do(0, S_.M_AXPY, S_.AxpyArgs(0.5, 1, 2, 0))
    o2.record()
    torch.cuda.synchronize()
    own, around = a2.elapsed_time(b2), o1.elapsed_time(o2)
    assert 0.0 < own <= around + 1e-3, (own, around)


@pytest.mark.parametrize("lanes", [1, 8, 37, 64])
def test_spawn_partial_requests_create_exactly_the_requested_objects(lanes):
    """SMMO_M_SPAWN: the first `lanes` slots of every driver block each create
    one object (partial wave requests sharing active blocks): exactly that
    many objects exist afterwards, in a consistent heap, and destroy-all
    removes them all."""
    say("spawn", lanes)
    S_ = S()
    D = 300
    n = D * 64 - 20                                   # a partial last block
    h = S_.Heap([[4], [4]], D + (D * lanes + 63) // 64 + 16)
    h.parallel_new(0, n, S_.CTOR_ZERO)
    h.parallel_do(0, S_.M_SPAWN, S_.SpawnArgs(1, lanes))
    want = (D - 1) * lanes + min(lanes, 64 - 20)
    s = check_heap(h, expect_live=[n, want])
    h.parallel_do(1, S_.M_DESTROY_ALL)
    check_heap(h, expect_live=[n, 0])
