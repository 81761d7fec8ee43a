"""Benchmark of the SMMO hot path on one MI355X.

Workload (the headline config): Life-like grid, 512 x 512 torus, Cell
{int32 x, int32 y, int8 alive} objects and Agent {int32 cell, int32 age}
objects created on birth and destroyed on death (B3/S23), initial density 0.3,
16,384-block heap.  One step = the three do-alls of the workload
(Cell::plan, Agent::step with destruction, Cell::commit with allocation),
each enumerating its class from the block bitmaps.  The timed region is steps
1..K of a freshly populated grid; the warm-up runs W steps on a separate
grid first.

Printed: one JSON line.  value = steps/s; roofline = the dominant kernel's
algorithmic bytes per launch over its event-timed duration; cpu_baseline =
the CPU oracle on the host.  Two sub-measurements of the same hot path are
attached: the alloc microbench (alloc+destroy Mobj/s) and the do-all sweep at
a heap six times the size of the Infinity Cache (GB/s vs HBM peak).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "alloc+destroy Mobj/s; parallel_do GB/s (% HBM peak); app steps/s plain vs batched"
TUNED_LAUNCH = os.path.join(ROOT, "paper_1810_11765_amd", "tuned_launch.json")
HBM_PEAK_GBS = 8000.0
CLOCK_HZ = 2.4e9                  # MI355X peak engine clock
SERVE_STEPS_PER_TICK = 10         # steps per launch while serving (an instance's 200 steps in 20 ticks)
SIMDS = 256 * 4                   # compute units x SIMDs per unit
HOLD_CYCLES = 1 << 28           # spin-kernel length that holds the stream while launches are queued


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-sub", action="store_true", help="skip the alloc / sweep / batch sub-measurements")
    p.add_argument("--no-batch", action="store_true", help="skip the plain-vs-batched sub-measurement")
    p.add_argument("--sweep-blocks", type=int, default=1 << 21)
    p.add_argument("--calib-copy", action="store_true",
                   help="also run a plain 1 GiB device copy 5 times (reference for HBM byte counters)")
    p.add_argument("--suite", choices=["ablation", "linux-scalability", "heap-size", "autotune", "nbody", "batch"],
                   help="run one of the allocator studies instead of the headline and print its JSON line")
    p.add_argument("--suite-steps", type=int, default=None, help="predator-prey steps of a suite run")
    p.add_argument("--tune-cache", default=None, help="JSON cache the autotune suite writes "
                   "(default: paper_1810_11765_amd/tuned_launch.json, which the batch sub-measurement reads)")
    return p.parse_args()


class Timer:
    """HIP events on torch's current stream, which is the stream every
    library call of this benchmark is queued on."""

    def __init__(self, torch):
        self.torch = torch
        self.spans = {}

    def run(self, name, fn):
        t = self.torch
        a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        self.spans.setdefault(name, []).append((a, b))

    def ms(self, name):
        return [a.elapsed_time(b) for a, b in self.spans.get(name, [])]


def life_bench(torch, workloads, steps, warmup):
    from paper_1810_11765_amd import smmo as S
    from paper_1810_11765_amd import tune
    # launch shape found by the autotuner for this workload on this device
    # (bench.py --suite autotune), if the package holds one
    shape = tune.load(TUNED_LAUNCH, "life-like 512x512 200 steps") or {}
    launch = {k: v for k, v in shape.items() if k in S.LAUNCH_FIELDS}
    lookups = shape.get("lookups", 5)

    def grid():
        g = workloads.LifeGrid(seed=42)
        g.heap.set_launch(**launch)
        g.heap.set_tuning(0, lookups, 0)
        return g
    if warmup:
        g0 = grid()
        g0.populate()
        for _ in range(warmup):
            g0.step()
        torch.cuda.synchronize()
        del g0
    # eager: K whole steps launched one do-all at a time
    ge = grid()
    ge.populate()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ge.step()
    torch.cuda.synchronize()
    ms_eager = (time.perf_counter() - t0) * 1e3 / steps
    # timed region: the same K steps captured once in a HIP graph (capture runs
    # nothing), then replayed from the freshly populated state
    g = grid()
    g.populate()
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph, stream=side):
            for _ in range(steps):
                g.step(stream=side)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graph.replay()
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / steps
    status = g.heap.status()
    same = all((a == b).all() for a, b in zip(g.state(), ge.state()))
    del graph
    # per-kernel durations: the same K steps again from a fresh grid.  Each
    # do-all kernel is dispatched with a pair of HIP events on its stream that
    # the dispatch itself records when the kernel starts and ends
    # (smmo_time_next_doall), so an event pair measures the kernel alone, as
    # the kernel trace does.  A spin kernel first holds the stream while the
    # host queues every launch, so the GPU then runs them back to back.
    g2 = grid()
    g2.populate()
    torch.cuda.synchronize()
    hold_start = torch.cuda.Event()
    torch.cuda._sleep(HOLD_CYCLES)
    hold_start.record()
    own = {"plan": [], "agent": [], "commit": []}

    def timed(name, cls, method):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g2.heap.time_next_doall(a, b)
        g2.heap.parallel_do(cls, method, g2.args)
        own[name].append((a, b))
    for _ in range(steps):
        timed("plan", g2.CELL, S.M_LIFE_PLAN)
        timed("agent", g2.AGENT, S.M_LIFE_AGENT)
        timed("commit", g2.CELL, S.M_LIFE_COMMIT)
    queued_ahead = not hold_start.query()            # the spin was still running when the last launch was queued
    torch.cuda.synchronize()
    names = ("plan", "agent", "commit")
    own_ms = {k: [a.elapsed_time(b) for a, b in own[k]] for k in names}
    per = {k: sum(own_ms[k]) / steps for k in names}
    return ms_step, per, status, {"eager_steps_s": round(1e3 / ms_eager, 2), "graph_equals_eager": bool(same),
                                  "launch": g.heap.get_launch(), "lookups": lookups, "events_queued_ahead": queued_ahead,
                                  "kernel_max_ms": {k: round(max(own_ms[k]), 5) for k in names}}


def roofline_for(per_ms):
    """Dominant kernel of the step and its algorithmic-bytes roofline.

    Algorithmic bytes per launch (unique data a launch must move at least):
      plan   per cell: x, y (8) + alive read (1) + alive write (1) + its entry of
             the cell -> handle table (8, read by its 8 neighbours) = 18 B
      commit per cell: x, y (8) + alive read/write (2) = 10 B (+ 8 B per birth)
      agent  per agent: cell, age (8) + age write (4) + table entry (8) + alive (1)
    The dominant kernel is the one with the largest share of the step (kernel
    durations recorded by the dispatches themselves) (the commit, whose births run the allocator: a chain of dependent
    agent-scope round trips, so it sits far below this bound).
    """
    name = max(per_ms, key=per_ms.get)
    cells = 512 * 512
    bytes_per = {"plan": 18.0 * cells, "commit": 10.0 * cells, "agent": 21.0 * cells * 0.3}
    kernel = {"plan": "k_doall<MLifePlan>", "agent": "k_doall<MLifeAgent>", "commit": "k_doall<MLifeCommit>"}[name]
    ms = per_ms[name]
    achieved = bytes_per[name] / (ms * 1e-3) / 1e9
    return name, {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": measured_traffic(kernel),
                  "kernel": kernel, "ms_per_launch": round(ms, 5), "bytes_per_launch": int(bytes_per[name])}


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs recorded in paper_1810_11765_amd/hbm_traffic.json (each counter scaled by
    its reading on a plain copy of known size), or None when that record was
    taken on different kernel sources."""
    path = os.path.join(ROOT, "paper_1810_11765_amd", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    from paper_1810_11765_amd.counters import kernel_source_hash
    if rec.get("source_sha256") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


def alloc_sub(torch, workloads):
    """Alloc microbench at its stated size: 65,536 threads x 4 device
    allocations, then churn rounds (each ~131k destroys + ~131k allocs)."""
    from paper_1810_11765_amd import smmo as S
    wl = workloads.AllocBench(seed=42)
    tm = Timer(torch)
    tm.run("alloc", wl.initial_alloc)
    for r in range(10):
        wl.sweep()
        tm.run("churn", lambda: wl.churn(r))
    torch.cuda.synchronize()
    # object counts of the same (deterministic) run, from the device counters
    # of a second run with counting switched on (counting adds atomics, so it
    # stays out of the timed run)
    wl2 = workloads.AllocBench(seed=42)
    wl2.heap.set_tuning(S.TUNE_STATS, 5, 0)
    wl2.initial_alloc()
    for r in range(10):
        wl2.round(r)
    st = wl2.heap.stats()
    churn_objs = (st["alloc_obj"] - 262144) + st["free_obj"]
    alloc_ms = tm.ms("alloc")[0]
    churn_ms = sum(tm.ms("churn"))
    return {"initial_alloc_mobj_s": round(262144 / (alloc_ms * 1e-3) / 1e6, 2),
            "churn_alloc_destroy_mobj_s": round(churn_objs / (churn_ms * 1e-3) / 1e6, 2),
            "churn_ms_per_round": round(churn_ms / 10, 4), "objects_per_round": churn_objs // 10,
            "reservation_ors_per_allocated_object": round(st["reserve_atomic"] / st["alloc_obj"], 4),
            "status": wl.heap.status()}


def atomic_ceiling(torch):
    """Reference rates of 64-bit agent-scope atomic ORs on this GPU: every
    lane on its own word (2^24 words), and a whole wavefront on one word."""
    from paper_1810_11765_amd import smmo as S
    words = torch.zeros(1 << 24, dtype=torch.int64, device="cuda")
    out = {}
    for name, lpw in (("distinct_words", 1), ("one_word_per_wave", 64)):
        nthreads, rounds = 1 << 24, 16
        for _ in range(2):
            S.atomic_probe(words, lpw, nthreads, rounds)
        tm = Timer(torch)
        for _ in range(5):
            tm.run("p", lambda: S.atomic_probe(words, lpw, nthreads, rounds))
        torch.cuda.synchronize()
        ms = sorted(tm.ms("p"))[2]
        out[name + "_gops_s"] = round(nthreads * rounds / (ms * 1e-3) / 1e9, 2)
    del words
    return out


def alloc_scaled_sub(torch):
    """Device allocation at scale: 2^22 threads x 4 allocations of the
    alloc-microbench class into a 2^18-block heap (16,777,216 objects, every
    slot), objects untouched; then every object destroys itself (one do-all).
    Atomics per object from a second run with the device counters on."""
    from paper_1810_11765_amd import smmo as S
    res = {}
    for counted in (False, True):
        h = S.Heap([[4, 4, 4]], 1 << 18)
        if counted:
            h.set_tuning(S.TUNE_STATS, 5, 0)
        tm = Timer(torch)
        tm.run("alloc", lambda: h.parallel_alloc(0, 1 << 22, 4, S.CTOR_NONE))
        torch.cuda.synchronize()
        live = h.live_count(0)
        tm.run("destroy", lambda: h.parallel_do(0, S.M_DESTROY_ALL))
        torch.cuda.synchronize()
        if counted:
            st = h.stats()
            res["reservation_ors_per_object"] = round(st["reserve_atomic"] / max(st["alloc_obj"], 1), 4)
            res["blocks_initialized"] = st["block_init"]
        else:
            a, d = tm.ms("alloc")[0], tm.ms("destroy")[0]
            res.update({"objects": live, "alloc_ms": round(a, 4), "destroy_ms": round(d, 4),
                        "alloc_mobj_s": round(live / (a * 1e-3) / 1e6, 1),
                        "destroy_mobj_s": round(live / (d * 1e-3) / 1e6, 1),
                        "left_after_destroy": h.live_count(0), "status": h.status()})
        h.close()
    return res


def alloc_partial_sub(torch):
    """Allocation at scale with partial wave requests (contended reservations
    in shared active blocks): 2^16 blocks of driver objects; in every block the
    first L slots each create one object of a second class (one do-all,
    SMMO_M_SPAWN), L = 1, 8, 32, so each wave asks for L slots and 64 / L
    waves share a fresh active block; then every spawned object destroys
    itself.  Atomics per object from a second run with the counters on."""
    from paper_1810_11765_amd import smmo as S
    D = 1 << 16
    out = {"driver_blocks": D}
    for L in (1, 8, 32):
        row = {}
        for counted in (False, True):
            h = S.Heap([[4], [4]], D + (D * L + 63) // 64 + 1024)
            h.parallel_new(0, D * 64, S.CTOR_NONE)
            if counted:
                h.set_tuning(S.TUNE_STATS, 5, 0)
            torch.cuda.synchronize()
            tm = Timer(torch)
            tm.run("spawn", lambda: h.parallel_do(0, S.M_SPAWN, S.SpawnArgs(1, L)))
            torch.cuda.synchronize()
            live = h.live_count(1)
            tm.run("destroy", lambda: h.parallel_do(1, S.M_DESTROY_ALL))
            torch.cuda.synchronize()
            if counted:
                st = h.stats()
                row["atomic_ors_per_object"] = round(st["reserve_atomic"] / max(st["alloc_obj"], 1), 4)
                row["reserve_fail_per_object"] = round(st["reserve_fail"] / max(st["alloc_obj"], 1), 4)
                row["blocks_initialized"] = st["block_init"]
            else:
                a, d = tm.ms("spawn")[0], tm.ms("destroy")[0]
                row.update({"objects": live, "spawn_ms": round(a, 4), "destroy_ms": round(d, 4),
                            "alloc_mobj_s": round(live / (a * 1e-3) / 1e6, 1),
                            "destroy_mobj_s": round(live / (d * 1e-3) / 1e6, 1),
                            "left_after_destroy": h.live_count(1), "status": h.status()})
            h.close()
        out[f"lanes_{L}"] = row
    return out


def nbody_sub(torch, workloads, steps=2):
    """N-body with merging at 262,144 bodies: per-phase event times of
    `steps` steps after one warm-up step; interactions/s of the all-pairs
    force (device_do) and its FP32 rate at 14 flops per interaction (the
    correctly rounded sqrt and division counted as one flop each) against the
    157.3 TFLOP/s vector peak; and the force's issue bound: the VALU issue
    cost of its instruction kinds measured by smmo_valu_probe, applied to its
    instruction mix."""
    from paper_1810_11765_amd import smmo as S
    nb = workloads.NBody(seed=42)
    nb.populate()
    nb.step()
    tm = Timer(torch)
    for _ in range(steps):
        tm.run("merge", nb.merge)
        tm.run("force", lambda: nb.phase(S.M_NBODY_FORCE))
        tm.run("move", lambda: nb.phase(S.M_NBODY_MOVE))
    torch.cuda.synchronize()
    n = nb.heap.live_count(0)
    f = sum(tm.ms("force")) / steps
    inter = n * (n - 1)
    tf = 14.0 * inter / (f * 1e-3) / 1e12
    status = nb.heap.status()
    del nb
    # issue cost of the force kernel's instruction kinds (smmo_valu_probe at 8
    # waves per SIMD): cycles one SIMD spends per wave-instruction, and the
    # force kernel's time if every SIMD issued its instructions back to back
    # at those costs (mix per interaction from the SQ_INSTS_VALU counter run:
    # 29.1 VALU lane-instructions, one square root and one reciprocal among
    # them, the rest priced as fmac)
    import ctypes as C
    L = S.lib()
    L.smmo_valu_probe.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p]
    L.smmo_valu_probe.restype = C.c_int
    wgs, iters = 2048, 20000
    out = torch.empty(wgs * 256, dtype=torch.float32, device="cuda")
    cyc = {}
    for kind, name in ((0, "add"), (1, "fmac"), (2, "sqrt"), (3, "rcp")):
        t = Timer(torch)
        for _ in range(3):
            t.run(name, lambda: S.check(L.smmo_valu_probe(out.data_ptr(), kind, wgs, iters,
                                                          C.c_void_p(torch.cuda.current_stream().cuda_stream))))
        torch.cuda.synchronize()
        ms = min(t.ms(name))
        cyc[name] = ms * 1e-3 * CLOCK_HZ * SIMDS / (wgs * 4 * iters * 8)
    per_inter = (29.1 - 2) * cyc["fmac"] + cyc["sqrt"] + cyc["rcp"]     # SIMD cycles per wave-interaction
    bound_ms = inter / 64 * per_inter / (SIMDS * CLOCK_HZ) * 1e3
    return {"bodies_live": n, "ms_per_step": round((sum(tm.ms("merge")) + sum(tm.ms("force")) + sum(tm.ms("move"))) / steps, 3),
            "force_ms": round(f, 3), "merge_ms": round(sum(tm.ms("merge")) / steps, 3),
            "interactions_per_s": round(inter / (f * 1e-3), 1), "fp32_tflops_at_14_per_interaction": round(tf, 2),
            "fp32_vector_peak_frac": round(tf / 157.3, 4),
            "valu_cycles_per_wave_instruction": {k: round(v, 3) for k, v in cyc.items()},
            "force_issue_bound_ms": round(bound_ms, 2), "force_frac_of_issue_bound": round(bound_ms / f, 3),
            "status": status}


def sweep_sub(torch, nblocks):
    """parallel_do sweep v += 0.5*x over nblocks x 64 objects of 12 B."""
    from paper_1810_11765_amd import smmo as S
    from paper_1810_11765_amd import tune
    h = S.Heap([[4, 4, 4]], nblocks)
    h.set_launch(**(tune.load(TUNED_LAUNCH, "sweep 2^21 blocks") or {}))
    n = nblocks * 64
    h.parallel_new(0, n, S.CTOR_ZERO)
    args = S.AxpyArgs(0.5, 1, 2, 0)
    for _ in range(3):
        h.parallel_do(0, S.M_AXPY, args)
    tm = Timer(torch)
    for _ in range(20):
        tm.run("sweep", lambda: h.parallel_do(0, S.M_AXPY, args))
    torch.cuda.synchronize()
    ms = sorted(tm.ms("sweep"))[len(tm.ms("sweep")) // 2]
    gbs = 12.0 * n / (ms * 1e-3) / 1e9
    # the same sweep through the generic do-all kernel (one wave per block,
    # lane = slot): what a method without a streaming form gets
    gen_args = S.AxpyArgs(0.5, 1, 2, 0)
    for _ in range(2):
        h.parallel_do(0, S.M_AXPY_GENERIC, gen_args)
    tmg = Timer(torch)
    for _ in range(10):
        tmg.run("g", lambda: h.parallel_do(0, S.M_AXPY_GENERIC, gen_args))
    torch.cuda.synchronize()
    ms_gen = sorted(tmg.ms("g"))[5]
    gbs_gen = 12.0 * n / (ms_gen * 1e-3) / 1e9
    # about half of the objects destroyed at random (fixed seed): the sweep
    # still streams whole block segments, so its algorithmic rate (live bytes
    # only) shows what fragmentation costs
    gen = torch.Generator(device="cuda")
    gen.manual_seed(42)
    idx = torch.nonzero(torch.rand(n, device="cuda", generator=gen) < 0.5).flatten()
    refs = idx | (1 << 56)                     # fresh heap: object i sits in block i/64, slot i%64
    del idx
    h.parallel_destroy(refs, refs.numel(), 1)
    del refs
    live_half = h.live_count(0)
    for _ in range(3):
        h.parallel_do(0, S.M_AXPY, args)
    tm2 = Timer(torch)
    for _ in range(20):
        tm2.run("sweep", lambda: h.parallel_do(0, S.M_AXPY, args))
    torch.cuda.synchronize()
    ms_half = sorted(tm2.ms("sweep"))[10]
    status = h.status()
    h_launch = h.get_launch()
    del h
    # reference: the vendor elementwise kernel on the same access mix (two
    # 512 MiB float reads, one 512 MiB write), i.e. what plain arrays reach
    a = torch.empty(1 << 27, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    c = torch.ones_like(a)
    for _ in range(3):
        torch.add(b, c, alpha=0.5, out=a)
    ref = Timer(torch)
    for _ in range(20):
        ref.run("ref", lambda: torch.add(b, c, alpha=0.5, out=a))
    torch.cuda.synchronize()
    ref_ms = sorted(ref.ms("ref"))[10]
    ref_gbs = 3.0 * a.numel() * 4 / (ref_ms * 1e-3) / 1e9
    del a, b, c
    return {"objects": n, "bytes_per_sweep": 12 * n, "ms_median": round(ms, 4), "gbs": round(gbs, 1),
            "launch": {k: v for k, v in h_launch.items() if k.startswith("sweep")},
            "kernel": "k_doall_axpy<%d>" % h_launch["sweep_groups"],
            "traffic": measured_traffic("k_doall_axpy<%d>@2^21" % h_launch["sweep_groups"]),
            "plain_array_reference_gbs": round(ref_gbs, 1),
            "fraction_of_plain_array_reference": round(gbs / ref_gbs, 3),
            "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
            "generic_doall": {"kernel": "k_doall<MAxpy>", "ms_median": round(ms_gen, 4), "gbs": round(gbs_gen, 1),
                              "hbm_frac": round(gbs_gen / HBM_PEAK_GBS, 4),
                              "fraction_of_streaming": round(gbs_gen / gbs, 3)},
            "half_fill": {"live_objects": live_half, "ms_median": round(ms_half, 4),
                          "algorithmic_gbs": round(12.0 * live_half / (ms_half * 1e-3) / 1e9, 1),
                          "field_segment_gbs": round(12.0 * n / (ms_half * 1e-3) / 1e9, 1)},
            "status": status}


def batch_sub(torch, steps=200, count=256):
    """Predator-prey instances of log-uniform side in [64, 1024): plain (one by
    one, per-phase launches) vs batched (one launch per phase for every
    instance, or one persistent kernel; graph replay) vs
    served (Poisson arrivals at 50/s, continuous admission; again with
    batching windows of 20 and 50 ms, and with the arrivals 10x and 100x
    faster).
    Results are compared instance by instance between all forms."""
    import numpy as np
    from paper_1810_11765_amd import serve as sv
    from paper_1810_11765_amd import smmo as S
    from paper_1810_11765_amd import tune
    reqs = sv.make_requests(seed=42, count=count)
    arena = S.Arena(sv.arena_bytes_for(reqs))
    inst_steps = count * steps
    # launch shape found by the autotuner for this workload on this device
    # (bench.py --suite autotune), if the package holds one
    tuned = {"wg_per_cu": 0, "steps_per_launch": 1, "lookups": 5, "block_objects": 64, "mode": S.BATCH_PHASED}
    tuned.update(tune.load(TUNED_LAUNCH, "predator-prey batched %d instances %d steps" % (count, steps)) or {})
    if tuned["block_objects"] != 64:
        del arena
        arena = S.Arena(max(sv.arena_bytes_for(reqs, b) for b in (64, tuned["block_objects"])))
    plain, t_plain = sv.run_plain(reqs, steps, arena)
    base, t_base, grid_base = sv.run_batched(reqs, steps, arena, per_launch=1, graph=True)
    batched, t_batch, grid = sv.run_batched(reqs, steps, arena, per_launch=tuned["steps_per_launch"], graph=True,
                                            wg_per_cu=tuned["wg_per_cu"], lookups=tuned["lookups"],
                                            block_objects=tuned["block_objects"], mode=tuned["mode"])
    # the other batch form at its best measured shape (10 steps per launch)
    other_mode = 1 - tuned["mode"]
    other, t_other, grid_other = sv.run_batched(reqs, steps, arena, per_launch=10, graph=True, mode=other_mode,
                                                block_objects=tuned["block_objects"])
    served = sv.serve(reqs, steps, arena, time_scale=1.0, wg_per_cu=tuned["wg_per_cu"], lookups=tuned["lookups"],
                      steps_per_tick=SERVE_STEPS_PER_TICK, block_objects=tuned["block_objects"],
                      mode=tuned["mode"])
    # the same requests arriving 10x and 100x faster: more instances live at
    # once, so each launch has more work for the same step latency
    faster = {ts: sv.serve(reqs, steps, arena, time_scale=ts, wg_per_cu=tuned["wg_per_cu"],
                           lookups=tuned["lookups"], steps_per_tick=SERVE_STEPS_PER_TICK,
                           block_objects=tuned["block_objects"], mode=tuned["mode"]) for ts in (0.1, 0.01)}
    # config 5's arrivals again, with batching windows of 20 and 50 ms between launches
    windowed = {w: sv.serve(reqs, steps, arena, time_scale=1.0, wg_per_cu=tuned["wg_per_cu"], lookups=tuned["lookups"],
                            steps_per_tick=SERVE_STEPS_PER_TICK, block_objects=tuned["block_objects"], tick_s=w,
                            mode=tuned["mode"])
                for w in (0.02, 0.05)}
    runs = ([batched, base, other, served["results"]] + [f["results"] for f in windowed.values()] +
            [f["results"] for f in faster.values()])
    same = all(all(all(np.array_equal(a, b) for a, b in zip(plain[r.rid][0], run[r.rid][0])) for run in runs)
               for r in reqs)
    status = max([plain[r.rid][1] for r in reqs] + [run[r.rid][1] for run in runs for r in reqs])
    lat = served["latency_ms"]
    by_rate = [{"arrivals_per_s": round(50.0 / ts), "busy_s": round(f["busy_s"], 3),
                "busy_over_batched": round(f["busy_s"] / t_batch, 2), "mean_live_instances": round(f["mean_live"], 1),
                "p50_step_ms": round(float(np.percentile(f["latency_ms"], 50)), 4)}
               for ts, f in [(1.0, served)] + sorted(faster.items(), reverse=True)]
    return {"instances": count, "steps": steps, "cells_total": int(sum(r.side * r.side for r in reqs)),
            "plain_steps_s": round(inst_steps / t_plain, 1),
            "batched_graph_steps_s": round(inst_steps / t_batch, 1),
            "batched_launch_shape": dict(tuned, workgroups=grid),
            "batched_default_shape_steps_s": round(inst_steps / t_base, 1),
            "batched_default_workgroups": grid_base,
            "batched_other_form": {"mode": ("phased", "persistent")[other_mode], "steps_per_launch": 10,
                                   "steps_s": round(inst_steps / t_other, 1), "workgroups": grid_other},
            "batched_over_plain": round(t_plain / t_batch, 2),
            "served_wall_s": round(served["wall_s"], 3), "served_busy_s": round(served["busy_s"], 3),
            "served_steps_s": round(inst_steps / served["wall_s"], 1),
            "served_p50_step_ms": round(float(np.percentile(lat, 50)), 4),
            "served_p99_step_ms": round(float(np.percentile(lat, 99)), 4),
            "served_max_admit_delay_s": round(float(served["admit_delay_s"].max()), 4),
            "served_steps_per_launch": SERVE_STEPS_PER_TICK,
            "served_busy_over_batched": round(served["busy_s"] / t_batch, 2),
            "served_admission_ms_p50_p99": [round(float(np.percentile(served["admit_ms"], q)), 3) for q in (50, 99)],
            "served_mean_live_instances": round(served["mean_live"], 1),
            "served_completion_s_p50_p99": [round(float(np.percentile(served["completion_s"], q)), 3) for q in (50, 99)],
            "served_with_window": [{"window_ms": round(w * 1e3), "busy_s": round(f["busy_s"], 3),
                                    "busy_over_batched": round(f["busy_s"] / t_batch, 2),
                                    "mean_live_instances": round(f["mean_live"], 1),
                                    "completion_s_p50_p99": [round(float(np.percentile(f["completion_s"], q)), 3)
                                                             for q in (50, 99)],
                                    "wall_s": round(f["wall_s"], 3)} for w, f in windowed.items()],
            "served_by_arrival_rate": by_rate,
            "identical_results": bool(same), "status": int(status)}


def _progress(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _wator_same(w, oracle_state):
    import numpy as np
    kind, age, energy = w.state()
    ok, oa, oe = oracle_state
    return bool(np.array_equal(kind, ok) and np.array_equal(age[kind > 0], oa[ok > 0]) and
                np.array_equal(energy[kind == 2], oe[ok == 2]))


ABLATION_VARIANTS = [("default", 0, 5), ("rotated-start", 64, 5), ("noshift", 1, 5), ("nocoal", 2, 5),
                     ("nocoal-noshift", 3, 5), ("r1", 0, 1), ("r2", 0, 2), ("r3", 0, 3), ("r5", 0, 5), ("r8", 0, 8)]


ABLATION_BLOCKS = 65536


def ablation_suite(torch, workloads, steps):
    """Predator-prey 1024 x 1024 (seed 42) under each allocator variant of
    Sec. 6.3: the paper's rotated-start search (rotated-start), rotation off
    (noshift), request coalescing off (nocoal), both,
    and r = 1..8 active-block lookups.  Per variant: step time (events around
    each step), fragmentation F every 10 steps (occupancy query, outside the
    timed spans) and whether the final state equals the oracle's.  The heap
    has 65,536 blocks, twice the workload's own: without rotation F reaches
    about 0.86 during the population peak, which would exhaust 32,768 blocks
    and turn the comparison into one of out-of-memory handling."""
    from oracle import core
    from paper_1810_11765_amd import smmo as S
    seed, side = 42, 1024
    kind0 = None
    out = {}
    for name, flags, lookups in ABLATION_VARIANTS:
        _progress("ablation", name)
        w = workloads.WaTor(seed=seed, width=side, height=side, kind0=kind0, num_blocks=ABLATION_BLOCKS)
        kind0 = w.kind0
        w.heap.set_tuning(flags, lookups, 0)
        w.populate()
        tm = Timer(torch)
        F = []
        for st in range(1, steps + 1):
            tm.run("step", w.step)
            if st % 10 == 0:
                F.append(round(w.heap.occupancy()["F"], 5))
        torch.cuda.synchronize()
        ms = tm.ms("step")
        st = w.heap.stats()
        out[name] = {"flags": flags, "lookups": lookups, "ms_per_step": round(sum(ms) / len(ms), 5),
                     "ms_total": round(sum(ms), 3), "ms_max_step": round(max(ms), 3), "F_every_10_steps": F,
                     "F_mean_last_100": round(sum(F[-10:]) / len(F[-10:]), 5), "status": w.heap.status(),
                     "guards": {k: st[k] for k in ("guard_alloc", "guard_spin", "guard_inval", "oom")},
                     "_w": w}
    _progress("ablation oracle")
    ref = core.c3_run(kind0, side, side, seed, steps)
    for name in out:
        w = out[name].pop("_w")
        out[name]["identical_to_oracle"] = _wator_same(w, ref)
        w.heap.close()
    return {"workload": f"predator-prey {side}x{side} torus, seed {seed}, {ABLATION_BLOCKS}-block heap, {steps} steps",
            "variants": out}


def linux_scalability_suite(torch, workloads):
    """Raw allocation (Sec. 6.4): 16,384 threads each allocate n 64-byte
    objects without touching them (one kernel), then destroy them by handle
    (a second kernel); the heap's whole device footprint is 1 GiB.  n from 1
    to 1024; the paper's measure is (alloc + destroy time) / n."""
    from paper_1810_11765_amd import smmo as S
    ls = workloads.LinuxScalability()
    cap = ls.num_blocks * 64
    out = {"workload": "16384 threads x n allocations of a 64-byte class, heap footprint 1 GiB",
           "num_blocks": ls.num_blocks, "slots": cap, "heap_bytes": S.heap_bytes(ls.CLASSES, ls.num_blocks)}
    for mode, flags in (("default", 0),):
        rows = []
        n = 1
        while n <= 1024:
            _progress("linux-scalability", mode, "n", n)
            reps = 3 if n < 1024 else 1
            a_ms, f_ms = [], []
            live = left = status = 0
            for _ in range(reps):
                ls.heap.reset()
                ls.heap.set_tuning(flags, 5, 0)
                tm = Timer(torch)
                tm.run("alloc", lambda: ls.alloc(n))
                torch.cuda.synchronize()
                live = ls.heap.live_count(0)
                status = ls.heap.status()
                tm.run("free", lambda: ls.free(n))
                torch.cuda.synchronize()
                left = ls.heap.live_count(0)
                a_ms += tm.ms("alloc")
                f_ms += tm.ms("free")
                ls.heap.clear_status()
            a, f = sorted(a_ms)[len(a_ms) // 2], sorted(f_ms)[len(f_ms) // 2]
            rows.append({"n": n, "alloc_ms": round(a, 4), "destroy_ms": round(f, 4),
                         "total_ms_over_n": round((a + f) / n, 5),
                         "ns_per_alloc": round(a * 1e6 / (16384 * n), 4),
                         "ns_per_destroy": round(f * 1e6 / (16384 * n), 4),
                         "live_after_alloc": live, "requested": 16384 * n, "left_after_destroy": left,
                         "oom": bool(status & S.STATUS_OOM)})
            n *= 2
        out[mode] = {"utilization_at_1024": round(rows[-1]["live_after_alloc"] * 64 / (1 << 30), 5), "rows": rows}
    return out


def blocks_for_bytes(classes, total: int) -> int:
    from paper_1810_11765_amd import smmo as S
    lo, hi = 1, total // 64 + 1
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if S.heap_bytes(classes, mid) <= total:
            lo = mid
        else:
            hi = mid - 1
    return lo


def heap_size_suite(torch, workloads, steps):
    """Predator-prey 1024 x 1024 (seed 42) in its own 32,768-block heap and in
    heaps of 1 to 64 GiB (Sec. 6.5): step time with the level-1 skip
    (default; a heap under 4,096 level-0 words is always scanned flat) and
    with every level-0 word scanned (flat), and whether the final state
    equals the oracle's."""
    from oracle import core
    from paper_1810_11765_amd import smmo as S
    seed, side = 42, 1024
    kind0 = None
    rows = []
    for gib in (0, 1, 2, 4, 8, 16, 32, 64):
        # 0: the workload's own 32,768-block heap (25 MiB), the reference row
        nb = 32768 if gib == 0 else blocks_for_bytes(workloads.WaTor.CLASSES, gib << 30)
        row = {"heap_gib": gib, "num_blocks": nb}
        for mode in ("hierarchical", "flat"):
            _progress("heap-size", gib, mode)
            w = workloads.WaTor(seed=seed, width=side, height=side, num_blocks=nb, kind0=kind0)
            kind0 = w.kind0
            if mode == "flat":
                w.heap.set_tuning(S.TUNE_FLAT_ENUM, 5, 0)
            w.populate()
            tm = Timer(torch)
            for _ in range(steps):
                tm.run("step", w.step)
            torch.cuda.synchronize()
            ms = tm.ms("step")
            row[mode] = {"ms_per_step": round(sum(ms) / len(ms), 5), "status": w.heap.status(), "_w": w}
            if mode == "hierarchical":
                row[mode]["F_end"] = round(w.heap.occupancy()["F"], 5)
            if gib == 0 and mode == "hierarchical":
                _progress("heap-size oracle")
                ref = core.c3_run(kind0, side, side, seed, steps)
            row[mode]["identical_to_oracle"] = _wator_same(w, ref)
            row[mode].pop("_w")
            w.heap.close()
            del w
            torch.cuda.empty_cache()
        rows.append(row)
    return {"workload": f"predator-prey {side}x{side} torus, seed {seed}, {steps} steps", "rows": rows}


def autotune_suite(torch, workloads, cache):
    """The autotuner (paper_1810_11765_amd/tune.py) on four workloads:
    the batched predator-prey form of config 5 (batch form, workgroups per
    CU, steps per launch, active-block lookups r, objects per block), predator-prey 1024 x 1024 with per-phase launches (objects
    per block, r, do-all grid cap and unit count), the Life-like step (r,
    do-all grid cap and unit count) and the 2^21-block sweep (grid and
    blocks in flight).  Every candidate's result is compared with the
    default shape's."""
    import numpy as np
    from paper_1810_11765_amd import serve as sv
    from paper_1810_11765_amd import smmo as S
    from paper_1810_11765_amd import tune
    out = {"arch": tune.device_arch()}

    # batched predator-prey (config 5: 256 instances x 200 steps), graph replay;
    # objects per block of the smallest class is a layout knob (the bitmap
    # fan-out stays 64: one bit per lane of a 64-wide wavefront)
    reqs = sv.make_requests(seed=42, count=256)
    arena = S.Arena(max(sv.arena_bytes_for(reqs, b) for b in (64, 32)))

    def batched(cfg):
        _progress("autotune batched", cfg)
        res, dt, grid = sv.run_batched(reqs, 200, arena, per_launch=cfg["steps_per_launch"], graph=True,
                                       wg_per_cu=cfg["wg_per_cu"], lookups=cfg["lookups"],
                                       block_objects=cfg["block_objects"], mode=cfg["mode"])
        return dt, res

    def same_states(a, b):
        return all(all(np.array_equal(x, y) for x, y in zip(a[k][0], b[k][0])) and a[k][1] == b[k][1] == 0
                   for k in a)
    rec = tune.search(batched, {"mode": [S.BATCH_PHASED, S.BATCH_PERSISTENT], "wg_per_cu": [0, 8, 24, 32, 2],
                                "steps_per_launch": [1, 2, 5, 10], "lookups": [5, 3, 8, 12],
                                "block_objects": [64, 32]}, reps=2, equal=same_states)
    tune.save(cache, "predator-prey batched 256 instances 200 steps", rec)
    out["batched"] = {k: rec[k] for k in ("default", "default_s", "best", "best_s", "speedup")}
    out["batched"]["rejected"] = sum(not t["same_result"] for t in rec["trials"])
    del arena

    # predator-prey 1024 x 1024 (config 3), plain per-phase launches, 100 steps
    kind0 = workloads.inputs.wator_initial(42, 1024, 1024, 0.20, 0.05)

    def wator(cfg):
        _progress("autotune predator-prey", cfg)
        b = cfg["block_objects"]
        w = workloads.WaTor(seed=42, width=1024, height=1024, kind0=kind0, num_blocks=32768 * 64 // b,
                            block_objects=b)
        w.heap.set_launch(**{k: v for k, v in cfg.items() if k in S.LAUNCH_FIELDS})
        w.heap.set_tuning(0, cfg["lookups"], 0)
        w.populate()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(100):
            w.step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = (w.state(), w.heap.status())
        w.release()
        return dt, st

    def same_wator(a, b):
        return all(np.array_equal(x, y) for x, y in zip(a[0], b[0])) and a[1] == b[1] == 0
    rec = tune.search(wator, {"block_objects": [64, 32], "lookups": [5, 3, 8], "doall_waves_per_cu": [32, 24, 48, 64],
                              "doall_units": [16384, 4096, 65536]}, reps=3, equal=same_wator)
    tune.save(cache, "predator-prey 1024x1024 100 steps", rec)
    out["predator_prey"] = {k: rec[k] for k in ("default", "default_s", "best", "best_s", "speedup")}
    out["predator_prey"]["rejected"] = sum(not t["same_result"] for t in rec["trials"])

    # Life-like step: 200 steps, graph replay of the whole run
    def life(cfg):
        _progress("autotune life", cfg)
        g = workloads.LifeGrid(seed=42)
        g.heap.set_launch(**{k: v for k, v in cfg.items() if k in S.LAUNCH_FIELDS})
        g.heap.set_tuning(0, cfg["lookups"], 0)
        g.populate()
        torch.cuda.synchronize()
        graph, side = torch.cuda.CUDAGraph(), torch.cuda.Stream()
        with torch.cuda.stream(side):
            with torch.cuda.graph(graph, stream=side):
                for _ in range(200):
                    g.step(stream=side)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        graph.replay()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = g.state()
        del graph
        return dt, (st, g.heap.status())

    def same_life(a, b):
        return all(np.array_equal(x, y) for x, y in zip(a[0], b[0])) and a[1] == b[1] == 0
    rec = tune.search(life, {"lookups": [5, 3, 8, 12, 16], "doall_waves_per_cu": [32, 16, 24, 48, 64],
                             "doall_units": [16384, 4096, 8192, 32768, 65536]}, reps=5, equal=same_life)
    tune.save(cache, "life-like 512x512 200 steps", rec)
    out["life"] = {k: rec[k] for k in ("default", "default_s", "best", "best_s", "speedup")}
    out["life"]["rejected"] = sum(not t["same_result"] for t in rec["trials"])

    # sweep at 2^21 blocks (timing) with the result checked on a 2^14-block heap
    big = S.Heap([[4, 4, 4]], 1 << 21)
    big.parallel_new(0, (1 << 21) * 64, S.CTOR_ZERO)
    small = S.Heap([[4, 4, 4]], 1 << 14)
    n_small = (1 << 14) * 64 - 77
    xs = torch.arange(n_small, dtype=torch.float32, device="cuda") * 0.125
    args = S.AxpyArgs(0.5, 1, 2, 0)

    def sweep(cfg):
        _progress("autotune sweep", cfg)
        big.set_launch(**cfg)
        for _ in range(2):
            big.parallel_do(0, S.M_AXPY, args)
        tm = Timer(torch)
        for _ in range(10):
            tm.run("s", lambda: big.parallel_do(0, S.M_AXPY, args))
        torch.cuda.synchronize()
        small.reset()
        small.set_launch(**cfg)
        small.parallel_new(0, n_small, S.CTOR_ARRAYS, S.ctor_arrays([None, xs, None]))
        small.parallel_do(0, S.M_AXPY, args)
        small.parallel_do(0, S.M_AXPY, args)
        return sorted(tm.ms("s"))[5] * 1e-3, small.dump_objects(0, [np.int32, np.float32, np.float32])[2]

    rec = tune.search(sweep, {"sweep_waves_per_cu": [128, 32, 64, 256], "sweep_groups": [4, 1, 2]}, reps=1,
                      equal=lambda a, b: bool(np.array_equal(a, b)))
    tune.save(cache, "sweep 2^21 blocks", rec)
    out["sweep"] = {k: rec[k] for k in ("default", "default_s", "best", "best_s", "speedup")}
    out["sweep"]["best_gbs"] = round(12.0 * (1 << 27) / rec["best_s"] / 1e9, 1)
    out["sweep"]["rejected"] = sum(not t["same_result"] for t in rec["trials"])
    out["cache"] = cache
    return out


def run_suite(args, torch, workloads):
    if args.suite == "ablation":
        res = ablation_suite(torch, workloads, args.suite_steps or 500)
    elif args.suite == "linux-scalability":
        res = linux_scalability_suite(torch, workloads)
    elif args.suite == "autotune":
        res = autotune_suite(torch, workloads, args.tune_cache or TUNED_LAUNCH)
    elif args.suite == "nbody":
        res = {"workload": "n-body with merging, 262,144 bodies, seed 42", **nbody_sub(torch, workloads)}
    elif args.suite == "batch":
        res = batch_suite(torch)
    else:
        res = heap_size_suite(torch, workloads, args.suite_steps or 100)
    if args.calib_copy:
        res["calib_copy_bytes"] = calib_copy(torch)
    print(json.dumps({"suite": args.suite, **res}), flush=True)


def calib_copy(torch):
    """A plain 1 GiB device copy, 5 times: the reference the HBM byte
    counters are scaled by."""
    a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda").fill_(1)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    return 1 << 30


def batch_suite(torch, steps=200, count=256):
    """Only the batched run of the 256 predator-prey instances (the tuned
    launch shape, graph replay; the kernels the batch counters and trace
    profiles cover), checked instance by instance against the default shape's
    run."""
    import numpy as np
    from paper_1810_11765_amd import serve as sv
    from paper_1810_11765_amd import smmo as S
    from paper_1810_11765_amd import tune
    reqs = sv.make_requests(seed=42, count=count)
    tuned = {"wg_per_cu": 0, "steps_per_launch": 1, "lookups": 5, "block_objects": 64, "mode": S.BATCH_PHASED}
    tuned.update(tune.load(TUNED_LAUNCH, "predator-prey batched %d instances %d steps" % (count, steps)) or {})
    arena = S.Arena(max(sv.arena_bytes_for(reqs, b) for b in (64, tuned["block_objects"])))
    base, t_base, _ = sv.run_batched(reqs, steps, arena, per_launch=1, graph=True)
    res, dt, grid = sv.run_batched(reqs, steps, arena, per_launch=tuned["steps_per_launch"], graph=True,
                                   wg_per_cu=tuned["wg_per_cu"], lookups=tuned["lookups"],
                                   block_objects=tuned["block_objects"], mode=tuned["mode"])
    same = all(all(np.array_equal(x, y) for x, y in zip(res[k][0], base[k][0])) for k in base)
    status = max(r[1] for r in res.values())
    return {"workload": f"predator-prey, {count} instances of side 64-1023, {steps} steps, batched", "launch": tuned,
            "workgroups": grid, "ms": round(dt * 1e3, 2), "instance_steps_s": round(count * steps / dt, 1),
            "default_shape_ms": round(t_base * 1e3, 2), "identical_to_default_shape": bool(same), "status": status}


def cpu_baseline():
    """The CPU oracle's Life run on whole 200-step runs of the same 512 x 512
    workload: on every OpenMP thread the host gives it (the per-cell loops of
    the oracle split over threads), then on one thread; each repeated until
    about 8 s of wall time."""
    import os
    from oracle import core
    from paper_1810_11765_amd import inputs
    a0 = inputs.life_initial(42, 512, 512)

    def rate():
        steps = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < 8.0:
            core.c2_run(a0, 512, 512, 200)
            steps += 200
        return steps, time.perf_counter() - t0
    threads = core.threads()
    steps_mt, dt_mt = rate()
    core.set_threads(1)
    steps_1, dt_1 = rate()
    core.set_threads(threads)
    cpu = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(steps_mt / dt_mt, 2), "unit": "steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{steps_mt // 200} full runs of 200 steps of the 512x512 Life-like grid on {threads} threads, "
                      f"then {steps_1 // 200} on one",
            "single_thread_value": round(steps_1 / dt_1, 2), "host_cpus": os.cpu_count(), "cpu_model": cpu}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    from paper_1810_11765_amd import smmo, workloads
    smmo.lib()                                   # fail loudly if the library is missing
    if args.suite:
        run_suite(args, torch, workloads)
        return
    _progress("life-like grid")
    ms_step, per, status, life_extra = life_bench(torch, workloads, args.steps, args.warmup)
    kname, roof = roofline_for(per)
    full_run = None
    if args.steps != 200:
        # the whole 200-step run of the configuration, measured the same way
        ms200, per200, st200, _ = life_bench(torch, workloads, 200, 0)
        full_run = {"steps_s": round(1e3 / ms200, 2), "ms_per_step": round(ms200, 5),
                    "kernel_ms_per_step": {k: round(v, 5) for k, v in per200.items()},
                    "roofline": roofline_for(per200)[1], "device_status": st200}
    out = {
        "metric": METRIC,
        "value": round(1e3 / ms_step, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "life-like grid 512x512 torus, density 0.3, 16384-block heap, "
                               "Cell{i32,i32,i8} + Agent{i32,i32}: steps 1..%d of the 200-step run" % args.steps,
                   "seed": 42, "mode": "hip-graph replay of steps 1..%d from the freshly populated grid" % args.steps},
        "kernel_ms_per_step": {k: round(v, 5) for k, v in per.items()},
        "life_eager": life_extra,
        "full_run_200_steps": full_run,
        "roofline": roof,
        "device_status": status,
    }
    if not args.no_sub:
        _progress("alloc microbench")
        out["alloc_microbench"] = alloc_sub(torch, workloads)
        _progress("atomic reference")
        out["atomic_reference"] = atomic_ceiling(torch)
        _progress("alloc at scale")
        out["alloc_scaled"] = alloc_scaled_sub(torch)
        _progress("alloc at scale, partial requests")
        out["alloc_scaled_partial"] = alloc_partial_sub(torch)
        _progress("sweep")
        out["sweep"] = sweep_sub(torch, args.sweep_blocks)
        _progress("n-body")
        out["nbody"] = nbody_sub(torch, workloads)
        if not args.no_batch:
            _progress("predator-prey plain vs batched vs served")
            out["predator_prey_plain_vs_batched"] = batch_sub(torch)
    if args.calib_copy:
        out["calib_copy_bytes"] = calib_copy(torch)
    if not args.no_cpu_baseline:
        _progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
