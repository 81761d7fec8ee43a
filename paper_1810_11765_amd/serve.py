"""Batched and served predator-prey instances.

Three ways to advance a set of independent instances (each its own heap and
grids carved from one arena):

* plain      one instance after the other through the per-phase C-ABI calls
             (four do-alls and two snapshots per step, one launch each);
* batched    all instances admitted up front, every step advanced for all of
             them at once (smmo_batch_step: one launch per phase, or one
             persistent launch for several steps), optionally replayed from
             a captured HIP graph;
* served     continuous batching: requests arrive over time (Poisson), are
             admitted between steps when the arena has room for their heap
             and grids, advance together with whatever else is running, and
             leave when done; per instance-step latency is recorded.

Only orchestration lives here; every object operation runs in libsmmo.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import inputs
from . import smmo as S
from .workloads import WaTor, wator_blocks


@dataclass
class Request:
    rid: int
    side: int
    seed: int
    arrival: float
    kind0: np.ndarray = field(repr=False, default=None)


def make_requests(seed: int = 42, count: int = 256, rate: float = 50.0, lo: int = 64, hi: int = 1024):
    sides, seeds, arrivals = inputs.serving_instances(seed, count, rate, lo, hi)
    out = []
    for i in range(count):
        s = int(sides[i])
        out.append(Request(i, s, int(seeds[i]), float(arrivals[i]), inputs.wator_initial(int(seeds[i]), s, s)))
    return out


def arena_bytes_for(reqs, block_objects: int = 64) -> int:
    """Arena size that holds every request at once (plus batch tables: the
    persistent kernel's barrier words take ~8.5 KB per slot)."""
    tot = (1 << 22) + 9 * 1024 * len(reqs)
    for r in reqs:
        n = r.side * r.side
        tot += S.heap_bytes(WaTor.CLASSES, wator_blocks(r.kind0, block_objects), block_objects) + 16 * n + 4096
    return tot


def instance_state(w: WaTor):
    """(kind, age, energy) per cell of a finished instance."""
    return w.state()


class Fleet:
    """A batch plus the instances it runs.  The host counts every instance's
    remaining steps itself (the batch advances each by min(steps,
    remaining)), so finding finished instances needs no device readback; the
    device's own count is checked once, when an instance leaves."""

    def __init__(self, arena: S.Arena, max_instances: int = 256, lookups: int = 5, block_objects: int = 64,
                 mode: int = S.BATCH_PHASED):
        self.arena = arena
        self.batch = S.Batch(arena, max_instances)
        self.batch.set_mode(mode)
        self.lookups = lookups              # active-block lookups r of every instance heap
        self.block_objects = block_objects  # objects per block of the smallest class (layout)
        self.live = {}                      # slot -> (request, WaTor)
        self.left = {}                      # slot -> steps still to run

    def admit(self, req: Request, steps: int, stream=None) -> bool:
        try:
            w = WaTor(seed=req.seed, width=req.side, height=req.side, num_blocks=None, kind0=req.kind0,
                      arena=self.arena, block_objects=self.block_objects)
        except S.SmmoError:
            return False                    # no room in the arena yet
        if self.lookups != 5:
            w.heap.set_tuning(0, self.lookups, 0, stream=stream)
        w.populate(stream)
        slot = self.batch.add(w.heap, w.args, steps, stream)
        self.live[slot] = (req, w)
        self.left[slot] = steps
        return True

    def step(self, steps: int, stream=None) -> None:
        self.batch.step(steps, stream)
        self.advanced(steps)

    def advanced(self, steps: int) -> None:
        """Account for `steps` steps run on the batch (by step() or a graph replay)."""
        for slot in self.left:
            self.left[slot] = max(0, self.left[slot] - steps)

    def finished(self) -> bool:
        return any(v == 0 for v in self.left.values())

    def harvest(self, stream=None):
        """Finished instances: (request, state, status); their memory is released."""
        done = []
        slots = [s for s in self.live if self.left[s] == 0]
        if not slots:
            return done
        rem = self.batch.remaining(stream)
        for slot in slots:
            assert rem[slot] == 0, f"slot {slot}: the device still counts {rem[slot]} steps"
            req, w = self.live.pop(slot)
            del self.left[slot]
            done.append((req, instance_state(w), w.heap.status()))
            self.batch.remove(slot)
            w.release()
        return done

    def close(self):
        for req, w in self.live.values():
            w.release()
        self.live.clear()
        self.batch.close()


def run_plain(reqs, steps: int, arena: S.Arena, block_objects: int = 64):
    """One instance at a time, per-phase launches.  Returns (results, seconds)."""
    results = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        w = WaTor(seed=r.seed, width=r.side, height=r.side, num_blocks=None, kind0=r.kind0, arena=arena,
                  block_objects=block_objects)
        w.populate()
        for _ in range(steps):
            w.step()
        results[r.rid] = (instance_state(w), w.heap.status())
        w.release()
    torch.cuda.synchronize()
    return results, time.perf_counter() - t0


def run_batched(reqs, steps: int, arena: S.Arena, per_launch: int = 1, graph: bool = False, wg_per_cu: int = 0,
                lookups: int = 5, block_objects: int = 64, mode: int = S.BATCH_PHASED):
    """All instances admitted, then `steps` steps of the batch (`per_launch`
    steps per smmo_batch_step call, wg_per_cu workgroups per CU, 0 = the batch
    form's default; `lookups` active-block lookups per allocation; `mode` phased or
    persistent).  Returns (results, seconds of the stepping, grid
    workgroups)."""
    fleet = Fleet(arena, max(len(reqs), 1), lookups=lookups, block_objects=block_objects, mode=mode)
    fleet.batch.set_grid(wg_per_cu)
    for r in reqs:
        assert fleet.admit(r, steps), "arena too small for the whole batch"
    torch.cuda.synchronize()
    launches = (steps + per_launch - 1) // per_launch
    if graph:
        # every launch captured by the library into one HIP graph, replayed once
        s = torch.cuda.Stream()
        g = fleet.batch.capture_graph(launches, per_launch, stream=s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.launch(stream=s)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        g.close()
        fleet.advanced(launches * per_launch)
    else:
        t0 = time.perf_counter()
        for _ in range(launches):
            fleet.step(per_launch)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
    grid = fleet.batch.grid()
    results = {req.rid: (st, status) for req, st, status in fleet.harvest()}
    assert not fleet.live, "instances left unfinished"
    fleet.close()
    return results, dt, grid


def serve(reqs, steps: int, arena: S.Arena, time_scale: float = 1.0, max_instances: int = 256,
          wg_per_cu: int = 0, lookups: int = 5, steps_per_tick: int = 10, block_objects: int = 64,
          tick_s: float = 0.0, mode: int = S.BATCH_PHASED):
    """Continuous batching over arrivals (arrival times scaled by time_scale):
    between launches, arrived requests are admitted while the arena has room;
    each tick advances every live instance by up to `steps_per_tick` steps
    (one smmo_batch_step on wg_per_cu workgroups per CU, 0 = the form's default,
    in `mode`); finished instances leave and free their memory.  With tick_s > 0 a
    launch starts at most every tick_s seconds (a batching window: instances
    wait for the next tick, so each launch carries more of them, for fewer
    GPU-seconds and a longer time to completion); 0 launches back to back
    while anything is live.

    Returns dict with results per request, per instance-step latencies (ms:
    the launch's GPU time over its steps, one entry per live instance and
    step), per-request completion times (s, arrival to finished), wall
    seconds, busy seconds (GPU time of the launches), the mean number of live
    instances per step run, admission host times (ms, outside the latencies)
    and admission delays."""
    fleet = Fleet(arena, max(1, min(max_instances, len(reqs))), lookups=lookups, block_objects=block_objects,
                  mode=mode)
    fleet.batch.set_grid(wg_per_cu)
    pending = deque(sorted(reqs, key=lambda r: r.arrival))
    lat, admit_delay, admit_ms, done_s, results = [], [], [], [], {}
    busy, steps_run = 0.0, 0
    next_tick = 0.0
    t0 = time.perf_counter()
    while pending or fleet.live:
        now = time.perf_counter() - t0
        while pending and pending[0].arrival * time_scale <= now:
            ta = time.perf_counter()
            if not fleet.admit(pending[0], steps):
                if not fleet.live:
                    raise S.SmmoError(f"request {pending[0].rid} does not fit in the empty arena")
                break                                   # wait until memory frees up
            admit_ms.append((time.perf_counter() - ta) * 1e3)
            admit_delay.append(now - pending[0].arrival * time_scale)
            pending.popleft()
        if fleet.live and now >= next_tick:
            next_tick = now + tick_s
            k = min(steps_per_tick, min(fleet.left.values()))      # stop when the first instance ends
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fleet.step(k)
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b)
            busy += ms * 1e-3
            steps_run += k
            lat.extend([ms / k] * (len(fleet.live) * k))
            finished = fleet.harvest()
            t_done = time.perf_counter() - t0
            for req, st, status in finished:
                results[req.rid] = (st, status)
                done_s.append(t_done - req.arrival * time_scale)
        else:
            wake = next_tick if fleet.live else float("inf")
            if pending and pending[0].arrival * time_scale > now:       # (an arrived one waits for memory)
                wake = min(wake, pending[0].arrival * time_scale)
            time.sleep(max(0.0, wake - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    fleet.close()
    return {"results": results, "latency_ms": np.array(lat), "wall_s": wall, "busy_s": busy,
            "mean_live": len(lat) / max(1, steps_run), "completion_s": np.array(done_s),
            "admit_ms": np.array(admit_ms), "admit_delay_s": np.array(admit_delay)}
