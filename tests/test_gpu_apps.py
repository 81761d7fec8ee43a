"""GPU parity of the SMMO application workloads (Life-like grid with agents,
predator-prey grid) against the CPU oracle, through the C-ABI.  Integer
workloads: bit-exact."""
import numpy as np
import pytest

from helpers import check_heap, say, wator_check as _wator_check
from oracle import core
from paper_1810_11765_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1810_11765_amd import smmo  # noqa: F401


def W():
    from paper_1810_11765_amd import workloads
    return workloads


def _life_check(g, W_, H_, steps_done):
    alive, ages = g.state()
    oa, oage = core.c2_run(g.alive0, W_, H_, steps_done)
    assert np.array_equal(alive, oa), f"alive grid differs after {steps_done} steps"
    assert np.array_equal(ages, oage), f"agent ages differ after {steps_done} steps"
    check_heap(g.heap, expect_live=[W_ * H_, int(oa.sum())])


@pytest.mark.parametrize("seed", [42, 7, 1234])
def test_life_full_size_parity(seed):
    """512 x 512 torus, density 0.3, 200 steps (16,384-block heap)."""
    say("life 512", seed)
    g = W().LifeGrid(seed=seed)
    g.populate()
    _life_check(g, 512, 512, 0)
    for s in range(1, 201):
        g.step()
        if s in (1, 2, 50):
            say("life step", s)
            _life_check(g, 512, 512, s)
    _life_check(g, 512, 512, 200)


def test_life_full_size_parity_with_the_tuned_shape():
    """The launch shape and active-block lookups the bench uses for the
    Life-like headline (autotuner's cache), 200 steps at full size."""
    import os
    from paper_1810_11765_amd import smmo as S
    from paper_1810_11765_amd import tune
    path = os.path.join(os.path.dirname(S.__file__), "tuned_launch.json")
    shape = tune.load(path, "life-like 512x512 200 steps")
    if shape is None:
        pytest.skip("no tuned shape for this device")
    say("life tuned", shape)
    g = W().LifeGrid(seed=42)
    g.heap.set_launch(**{k: v for k, v in shape.items() if k in S.LAUNCH_FIELDS})
    g.heap.set_tuning(0, shape.get("lookups", 5), 0)
    g.populate()
    for _ in range(200):
        g.step()
    _life_check(g, 512, 512, 200)


def _tuned_life(seed=42):
    import os
    from paper_1810_11765_amd import smmo as S
    from paper_1810_11765_amd import tune
    path = os.path.join(os.path.dirname(S.__file__), "tuned_launch.json")
    shape = tune.load(path, "life-like 512x512 200 steps") or {}
    g = W().LifeGrid(seed=seed)
    g.heap.set_launch(**{k: v for k, v in shape.items() if k in S.LAUNCH_FIELDS})
    g.heap.set_tuning(0, shape.get("lookups", 5), 0)
    return g


@pytest.mark.parametrize("seed", [42, 7])
def test_life_concurrent_phases_parity(seed):
    """The agent phase on a second stream, concurrent with the commit phase
    (snapshot of the agents while plan runs): same state as the oracle."""
    say("life concurrent", seed)
    g = _tuned_life(seed)
    g.populate()
    side = torch.cuda.Stream()
    for s in range(1, 201):
        g.step(side_stream=side)
        if s in (1, 2, 50):
            torch.cuda.synchronize()
            _life_check(g, 512, 512, s)
    torch.cuda.synchronize()
    _life_check(g, 512, 512, 200)


def test_life_concurrent_phases_in_a_graph():
    """100 concurrent-phase steps captured once in a HIP graph over two
    streams, replayed twice with host dumps in between: the state equals the
    oracle's after 100 and after 200 steps."""
    say("life concurrent graph")
    g = _tuned_life(42)
    g.populate()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    cap, side = torch.cuda.Stream(), torch.cuda.Stream()
    with torch.cuda.stream(cap):
        with torch.cuda.graph(graph, stream=cap):
            for _ in range(100):
                g.step(stream=cap, side_stream=side)
    torch.cuda.synchronize()
    _life_check(g, 512, 512, 0)                      # capture ran nothing
    for rep in (1, 2):
        graph.replay()
        torch.cuda.synchronize()
        _life_check(g, 512, 512, 100 * rep)
    del graph


@pytest.mark.parametrize("Wd,Hd,blocks", [(37, 23, 64), (130, 7, 64), (64, 64, 128)])
def test_life_ragged_parity(Wd, Hd, blocks):
    say("life ragged", Wd, Hd)
    g = W().LifeGrid(seed=3, width=Wd, height=Hd, num_blocks=blocks)
    g.populate()
    for s in range(60):
        g.step()
    _life_check(g, Wd, Hd, 60)


def test_life_textbook_glider_on_gpu():
    W_ = H_ = 16
    a0 = np.zeros(W_ * H_, dtype=np.uint8)
    for x, y in [(1, 0), (2, 1), (0, 2), (1, 2), (2, 2)]:
        a0[y * W_ + x] = 1
    g = W().LifeGrid(width=W_, height=H_, num_blocks=16, alive0=a0)
    g.populate()
    for _ in range(4):
        g.step()
    alive, ages = g.state()
    want = np.zeros_like(a0)
    for x, y in [(2, 1), (3, 2), (1, 3), (2, 3), (3, 3)]:
        want[y * W_ + x] = 1
    assert np.array_equal(alive, want)


@pytest.mark.parametrize("seed", [42, 7, 1234])
def test_wator_full_size_parity(seed):
    """1024 x 1024 torus, 20% fish, 5% sharks, 500 steps (32,768-block heap)."""
    say("wator 1024", seed)
    w = W().WaTor(seed=seed)
    w.populate()
    assert np.array_equal(w.kind0, inputs.wator_initial(seed, 1024, 1024))
    for s in range(1, 501):
        w.step()
        if s in (1, 25, 500):
            say("wator step", s)
            _wator_check(w, s, core.c3_run(w.kind0, 1024, 1024, seed, s))


@pytest.mark.parametrize("Wd,Hd,blocks,seed", [(97, 61, 256, 5), (16, 200, 128, 6), (8, 8, 8, 7)])
def test_wator_ragged_parity(Wd, Hd, blocks, seed):
    say("wator ragged", Wd, Hd)
    w = W().WaTor(seed=seed, width=Wd, height=Hd, num_blocks=blocks)
    w.populate()
    for s in range(120):
        w.step()
    _wator_check(w, 120, core.c3_run(w.kind0, Wd, Hd, seed, 120))


@pytest.mark.parametrize("blocks", [256, 300000])
def test_plan_phase_records_the_snapshot_of_its_class(blocks):
    """A plan do-all (creates and destroys nothing) records its class's
    snapshot in passing: right after it, every allocated fish block's
    iteration word equals its live slots, in a flat-scanned and in a
    block-listed heap; the step then continues (the move phase uses it) and
    30 steps still equal the oracle."""
    from oracle import heapcheck
    from paper_1810_11765_amd import smmo as S
    say("recorded snapshot", blocks)
    w = W().WaTor(seed=9, width=97, height=61, num_blocks=blocks)
    w.populate()
    for _ in range(3):
        w.step()
    w.t += 1
    w.args.step = w.t
    w.heap.parallel_do(w.FISH, S.M_WATOR_FISH_PLAN, w.args)
    raw = heapcheck.RawHeap(w.heap.dump_raw())
    fish = raw.bits(1 + w.FISH)
    pad = np.uint64((0xFFFFFFFFFFFFFFFF << raw.capacity[w.FISH]) & 0xFFFFFFFFFFFFFFFF) \
        if raw.capacity[w.FISH] < 64 else np.uint64(0)
    assert fish.any()
    assert np.array_equal(raw.iter[fish], raw.alloc[fish] & ~pad)
    w.heap.parallel_do(w.FISH, S.M_WATOR_FISH_MOVE, w.args)
    w.heap.parallel_do(w.SHARK, S.M_WATOR_SHARK_PLAN, w.args)
    w.heap.parallel_do(w.SHARK, S.M_WATOR_SHARK_MOVE, w.args)
    for _ in range(26):
        w.step()
    _wator_check(w, 30, core.c3_run(w.kind0, 97, 61, 9, 30))


@pytest.mark.parametrize("bo,blocks", [(32, 65536), (16, 131072)])
def test_wator_parity_with_fewer_objects_per_block(bo, blocks):
    """The layout knob: bo objects per block of the smallest class (fish
    blocks hold bo fish, shark blocks bo * 8 // 12), at the same heap bytes
    as the 64-object default.  1024 x 1024, seed 3, 60 steps."""
    say("wator block objects", bo, blocks)
    w = W().WaTor(seed=3, num_blocks=blocks, block_objects=bo)
    assert w.heap.layout(0).capacity == bo and w.heap.layout(1).capacity == bo * 8 // 12
    w.populate()
    for s in range(60):
        w.step()
    _wator_check(w, 60, core.c3_run(w.kind0, 1024, 1024, 3, 60))
