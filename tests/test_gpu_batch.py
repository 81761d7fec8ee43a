"""GPU parity of the batched and served predator-prey forms: every instance's
result is the oracle's for its own size and seed, alone or in the mix, with
both batch forms (one launch per phase, one persistent kernel), graph replay
and continuous admission."""
import numpy as np
import pytest

from helpers import say
from oracle import core

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1810_11765_amd import smmo  # noqa: F401


def SV():
    from paper_1810_11765_amd import serve
    return serve


def S():
    from paper_1810_11765_amd import smmo
    return smmo


def _check(results, reqs, steps):
    assert sorted(results) == sorted(r.rid for r in reqs)
    for r in reqs:
        (kind, age, energy), status = results[r.rid]
        assert status == 0, f"request {r.rid}: device status {status:#x}"
        ok, oa, oe = core.c3_run(r.kind0, r.side, r.side, r.seed, steps)
        assert np.array_equal(kind, ok), f"request {r.rid} (side {r.side}): occupancy differs"
        assert np.array_equal(age[kind > 0], oa[ok > 0]), f"request {r.rid}: ages differ"
        assert np.array_equal(energy[kind == 2], oe[ok == 2]), f"request {r.rid}: energies differ"


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("per_launch,graph", [(1, False), (7, False), (1, True), (10, True)])
def test_batched_instances_match_oracle(per_launch, graph, mode):
    say("batched", per_launch, graph, mode)
    sv = SV()
    reqs = sv.make_requests(seed=5, count=12, lo=12, hi=100)
    arena = S().Arena(sv.arena_bytes_for(reqs))
    results, dt, _ = sv.run_batched(reqs, 40, arena, per_launch=per_launch, graph=graph, mode=mode)
    _check(results, reqs, 40)
    free, largest = arena.stats()
    assert free == largest                                   # every range returned and merged


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("wg_per_cu", [1, 2])
def test_batched_smaller_grid_matches_oracle(wg_per_cu, mode):
    """Both batch forms on 1 or 2 workgroups per CU (the autotuner's knob):
    same results."""
    say("batched grid", wg_per_cu, mode)
    sv = SV()
    reqs = sv.make_requests(seed=15, count=12, lo=12, hi=100)
    arena = S().Arena(sv.arena_bytes_for(reqs))
    results, dt, grid = sv.run_batched(reqs, 40, arena, per_launch=3, graph=False, wg_per_cu=wg_per_cu, mode=mode)
    assert grid == 256 * wg_per_cu or grid < 256 * wg_per_cu      # capped by residency
    _check(results, reqs, 40)


def test_batched_with_the_tuned_shape_matches_oracle():
    """The launch shape the bench uses for config 5 (autotuner's cache):
    workgroups per CU, steps per launch and active-block lookups."""
    import os
    from paper_1810_11765_amd import tune
    path = os.path.join(os.path.dirname(SV().__file__), "tuned_launch.json")
    shape = tune.load(path, "predator-prey batched 256 instances 200 steps")
    if shape is None:
        pytest.skip("no tuned shape for this device")
    say("batched tuned", shape)
    sv = SV()
    reqs = sv.make_requests(seed=17, count=24, lo=16, hi=160)
    bo = shape.get("block_objects", 64)
    arena = S().Arena(sv.arena_bytes_for(reqs, bo))
    results, dt, grid = sv.run_batched(reqs, 50, arena, per_launch=shape["steps_per_launch"], graph=True,
                                       wg_per_cu=shape["wg_per_cu"], lookups=shape.get("lookups", 5),
                                       block_objects=bo, mode=shape.get("mode", 0))
    _check(results, reqs, 50)


def test_batched_and_served_with_32_object_blocks_match_oracle():
    """Every instance's heap laid out with 32 objects per fish block (the
    autotuner's other layout candidate), batched and served."""
    say("batched 32-object blocks")
    sv = SV()
    reqs = sv.make_requests(seed=19, count=10, lo=16, hi=140)
    arena = S().Arena(sv.arena_bytes_for(reqs, 32))
    results, dt, grid = sv.run_batched(reqs, 40, arena, per_launch=4, graph=True, block_objects=32)
    _check(results, reqs, 40)
    out = sv.serve(reqs, 40, arena, time_scale=1.0, block_objects=32)
    _check(out["results"], reqs, 40)


def test_plain_one_by_one_matches_oracle():
    say("plain")
    sv = SV()
    reqs = sv.make_requests(seed=6, count=6, lo=12, hi=80)
    arena = S().Arena(sv.arena_bytes_for(reqs))
    results, dt = sv.run_plain(reqs, 30, arena)
    _check(results, reqs, 30)


def test_serving_continuous_admission_matches_oracle():
    """Requests arrive while others run (arrivals compressed 20x); each result
    equals the oracle's for the instance alone."""
    say("serve")
    sv = SV()
    reqs = sv.make_requests(seed=8, count=16, lo=16, hi=128)
    arena = S().Arena(sv.arena_bytes_for(reqs))
    out = sv.serve(reqs, 30, arena, time_scale=0.05)
    _check(out["results"], reqs, 30)
    assert len(out["latency_ms"]) == 16 * 30                # every instance-step timed
    assert out["latency_ms"].min() > 0


def test_serving_with_a_batching_window_matches_oracle():
    """Launches at most every 10 ms: instances wait for the tick, results and
    step counts are unchanged, every request reports its completion time, and
    a request never completes before its steps could have run."""
    say("serve window")
    sv = SV()
    reqs = sv.make_requests(seed=12, count=12, lo=16, hi=96)
    arena = S().Arena(sv.arena_bytes_for(reqs))
    out = sv.serve(reqs, 30, arena, time_scale=0.05, steps_per_tick=10, tick_s=0.01)
    _check(out["results"], reqs, 30)
    assert len(out["latency_ms"]) == 12 * 30
    assert len(out["completion_s"]) == 12
    assert out["completion_s"].min() >= 0.015                 # 3 launches, at least 2 ticks apart


def test_serving_waits_for_memory():
    """An arena that holds only a few instances at once: later requests wait
    for earlier ones to leave, and all results still match."""
    say("serve small arena")
    sv = SV()
    reqs = sv.make_requests(seed=9, count=10, lo=40, hi=64)
    need = sv.arena_bytes_for(reqs)
    arena = S().Arena(need // 3)
    out = sv.serve(reqs, 20, arena, time_scale=0.0)         # all arrive at once
    _check(out["results"], reqs, 20)
    assert len(out["admit_delay_s"]) == 10 and out["admit_delay_s"].max() > 0


def test_batched_three_level_bitmaps_match_oracle():
    """Instances large enough for three-level block bitmaps (more than 4,096
    blocks: sides 400 and 512) next to small ones, batched (graph replay) and
    served: the top-down and level-0-probe searches of the batch kernels
    against the oracle."""
    sv = SV()
    from paper_1810_11765_amd import inputs
    from paper_1810_11765_amd.workloads import wator_blocks
    reqs = []
    for rid, (side, seed) in enumerate([(512, 101), (400, 102), (70, 103), (33, 104)]):
        k0 = inputs.wator_initial(seed, side, side)
        reqs.append(sv.Request(rid, side, seed, 0.01 * rid, k0))
    assert wator_blocks(reqs[0].kind0) > 4096 and wator_blocks(reqs[1].kind0) > 4096
    arena = S().Arena(sv.arena_bytes_for(reqs))
    say("batched 3-level", [r.side for r in reqs])
    results, dt, _ = sv.run_batched(reqs, 50, arena, per_launch=5, graph=True)
    _check(results, reqs, 50)
    say("served 3-level")
    out = sv.serve(reqs, 50, arena, time_scale=1.0)
    _check(out["results"], reqs, 50)


def test_config_5_batched_and_served_against_oracle_goldens():
    """The configuration as stated: 256 instances of seed 42, side log-uniform
    in [64, 1024), 200 steps each, batched (graph replay, the bench's launch
    shape, and the other batch form) and served (Poisson arrivals at 50/s).  Every
    instance's final state hashes to the value the oracle stored in
    tests/golden (written by tests/golden/make_goldens.py from oracle/ only)."""
    import os
    from golden.make_goldens import BATCH_FILE, read_batch, wator_hash
    from paper_1810_11765_amd import tune
    if not os.path.exists(BATCH_FILE):
        pytest.fail("golden values missing: run python tests/golden/make_goldens.py batch")
    golden = read_batch()
    sv = SV()
    reqs = sv.make_requests(seed=42, count=256)
    assert sorted(golden) == [r.rid for r in reqs]
    for r in reqs:
        assert golden[r.rid][:2] == (r.side, r.seed)
    shape = {"wg_per_cu": 0, "steps_per_launch": 1, "lookups": 5, "block_objects": 64, "mode": 0}
    path = os.path.join(os.path.dirname(sv.__file__), "tuned_launch.json")
    shape.update(tune.load(path, "predator-prey batched 256 instances 200 steps") or {})
    bo = shape["block_objects"]
    arena = S().Arena(sv.arena_bytes_for(reqs, bo))

    def check(results, what):
        bad = []
        for r in reqs:
            (kind, age, energy), status = results[r.rid]
            assert status == 0, f"{what}: request {r.rid} device status {status:#x}"
            if wator_hash(kind, age, energy) != golden[r.rid][2]:
                bad.append((r.rid, r.side))
        assert not bad, f"{what}: {len(bad)} instances differ from the oracle, e.g. {bad[:5]}"

    say("config 5 batched", shape)
    results, dt, _ = sv.run_batched(reqs, 200, arena, per_launch=shape["steps_per_launch"], graph=True,
                                    wg_per_cu=shape["wg_per_cu"], lookups=shape["lookups"], block_objects=bo,
                                    mode=shape["mode"])
    check(results, "batched")
    other = 1 - shape["mode"]
    say("config 5 batched, mode", other)
    results, dt, _ = sv.run_batched(reqs, 200, arena, per_launch=10, graph=True, block_objects=bo, mode=other)
    check(results, "batched, other form")
    say("config 5 served")
    out = sv.serve(reqs, 200, arena, time_scale=1.0, wg_per_cu=shape["wg_per_cu"], lookups=shape["lookups"],
                   steps_per_tick=shape["steps_per_launch"], block_objects=bo, mode=shape["mode"])
    check(out["results"], "served")


@pytest.mark.parametrize("mode", [0, 1])
def test_captured_batch_graph_replayed_several_times_matches_oracle(mode):
    """smmo_batch_capture_graph: one launch group of 5 steps captured once and
    replayed six times, with eager work (state dumps) and synchronizations
    between the replays; after every replay each instance equals the oracle
    at 5, 10, ... 30 steps.  Once the instance set changes, the graph is
    refused instead of being replayed with a stale schedule."""
    sv = SV()
    S_ = S()
    reqs = sv.make_requests(seed=11, count=6, lo=16, hi=90)
    arena = S_.Arena(sv.arena_bytes_for(reqs))
    fleet = sv.Fleet(arena, 8, mode=mode)
    for r in reqs:
        assert fleet.admit(r, 30)
    stream = torch.cuda.Stream()
    say("capture batch graph")
    g = fleet.batch.capture_graph(1, 5, stream=stream)
    torch.cuda.synchronize()
    for rep in range(1, 7):
        say("replay", rep)
        g.launch(stream=stream)
        torch.cuda.synchronize()
        fleet.advanced(5)
        for slot, (r, w) in fleet.live.items():
            kind, age, energy = w.state()
            ok, oa, oe = core.c3_run(r.kind0, r.side, r.side, r.seed, 5 * rep)
            assert np.array_equal(kind, ok), f"replay {rep}, request {r.rid}: occupancy differs"
            assert np.array_equal(age[kind > 0], oa[ok > 0]), f"replay {rep}, request {r.rid}: ages differ"
            assert np.array_equal(energy[kind == 2], oe[ok == 2]), f"replay {rep}, request {r.rid}: energies differ"
    assert (fleet.batch.remaining()[:len(reqs)] == 0).all()
    done = fleet.harvest()                       # removes every instance: the graph is now stale
    assert len(done) == len(reqs) and all(st == 0 for _, _, st in done)
    with pytest.raises(S_.SmmoError):
        g.launch(stream=stream)
    g.close()
    fleet.close()


def test_batch_graph_capture_rejects_the_null_stream():
    S_ = S()
    arena = S_.Arena(1 << 22)
    b = S_.Batch(arena, 4)
    import ctypes as C
    out = C.c_void_p()
    rc = S_.lib().smmo_batch_capture_graph(b.h, 1, 1, None, C.byref(out))
    assert rc == -1 and not out.value
    with pytest.raises(S_.SmmoError):
        b.set_mode(2)
    b.close()
