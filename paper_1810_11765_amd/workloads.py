"""Host drivers of the SMMO workloads: set up heaps and issue the C-ABI calls.

Each driver only uploads seeded starting states (paper_1810_11765_amd.inputs)
and sequences parallel_new / parallel_alloc / parallel_do; every object
operation runs in libsmmo's kernels.
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs
from . import smmo as S

INT32_MAX = 2**31 - 1


def _dev(a: np.ndarray, device="cuda") -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


class AllocBench:
    """Alloc microbench: one class {int32 id, f32 x, f32 v}; `nthreads` threads
    allocate `per_thread` objects each, then rounds of sweep + churn."""

    CLASSES = [[4, 4, 4]]

    def __init__(self, seed=42, num_blocks=4096, nthreads=65536, per_thread=4, device="cuda"):
        self.seed, self.nthreads, self.per_thread = seed, nthreads, per_thread
        self.heap = S.Heap(self.CLASSES, num_blocks, device=device)
        ids, x, v = inputs.alloc_bench_initial(seed, nthreads, per_thread)
        self.init_arrays = (ids, x, v)
        self._src = [_dev(ids, device), _dev(x, device), _dev(v, device)]
        self._sweep_args = S.AxpyArgs(0.5, 1, 2, 0)

    def initial_alloc(self, stream=None):
        self.heap.parallel_alloc(0, self.nthreads, self.per_thread, S.CTOR_ARRAYS,
                                 S.ctor_arrays(self._src), stream=stream)

    def initial_new(self, stream=None):
        """Same objects through parallel_new (dense placement)."""
        self.heap.parallel_new(0, self.nthreads * self.per_thread, S.CTOR_ARRAYS,
                               S.ctor_arrays(self._src), stream=stream)

    def sweep(self, stream=None):
        self.heap.parallel_do(0, S.M_AXPY, self._sweep_args, stream=stream)

    def churn(self, r: int, stream=None):
        self.heap.parallel_do(0, S.M_CHURN, S.ChurnArgs(self.seed, r, 0), stream=stream)

    def round(self, r: int, stream=None):
        self.sweep(stream)
        self.churn(r, stream)

    def state(self):
        ids, x, v = self.heap.dump_objects(0, [np.int32, np.float32, np.float32])
        o = np.argsort(ids, kind="stable")
        return ids[o], x[o], v[o]


class LinuxScalability:
    """Raw allocation benchmark (Sec. 6.4): one class of 64-byte objects
    (eight 8-byte fields, N = 64, 4 KiB blocks) in a heap whose whole device
    footprint is `heap_total` bytes; `nthreads` threads each allocate n
    objects without touching them, a second kernel destroys them."""

    CLASSES = [[8] * 8]

    def __init__(self, nthreads=16384, heap_total=1 << 30, max_per_thread=1024, device="cuda"):
        self.nthreads = nthreads
        # the most blocks whose heap (metadata + scratch + data) fits heap_total
        lo, hi = 1, heap_total // 4096 + 1
        while lo < hi:
            mid = (lo + hi + 1) // 2
            if S.heap_bytes(self.CLASSES, mid) <= heap_total:
                lo = mid
            else:
                hi = mid - 1
        self.num_blocks = lo
        self.heap = S.Heap(self.CLASSES, lo, device=device)
        self.refs = torch.zeros(nthreads * max_per_thread, dtype=torch.int64, device=device)
        self._args = S.ctor_none(self.refs)

    def alloc(self, n: int, stream=None):
        self.heap.parallel_alloc(0, self.nthreads, n, S.CTOR_NONE, self._args, stream=stream)

    def free(self, n: int, stream=None):
        self.heap.parallel_destroy(self.refs, self.nthreads, n, stream=stream)

    def data_bytes(self) -> int:
        return self.num_blocks * 64 * 64


class LifeGrid:
    """Life-like grid: Cell {int32 x, int32 y, int8 alive} (class 0) and
    Agent {int32 cell, int32 age} (class 1) on a width x height torus."""

    CLASSES = [[4, 4, 1], [4, 4]]
    CELL, AGENT = 0, 1

    def __init__(self, seed=42, width=512, height=512, num_blocks=16384, density=0.3, device="cuda",
                 alive0: np.ndarray | None = None):
        self.W, self.H = width, height
        self.heap = S.Heap(self.CLASSES, num_blocks, device=device)
        n = width * height
        self.alive0 = inputs.life_initial(seed, width, height, density) if alive0 is None else alive0
        c = np.arange(n, dtype=np.int32)
        self._x = _dev((c % width).astype(np.int32), device)
        self._y = _dev((c // width).astype(np.int32), device)
        self._a = _dev(self.alive0.astype(np.uint8), device)
        self.cell_ref = torch.zeros(n, dtype=torch.int64, device=device)
        alive_ids = np.nonzero(self.alive0)[0].astype(np.int32)
        self._agent_cell = _dev(alive_ids, device)
        self.n_alive0 = len(alive_ids)
        self.args = S.LifeArgs(self.cell_ref.data_ptr(), width, height, self.CELL, self.AGENT)

    def populate(self, stream=None):
        self.heap.parallel_new(self.CELL, self.W * self.H, S.CTOR_ARRAYS,
                               S.ctor_arrays([self._x, self._y, self._a], ref_out=self.cell_ref), stream=stream)
        if self.n_alive0:
            self.heap.parallel_new(self.AGENT, self.n_alive0, S.CTOR_ARRAYS,
                                   S.ctor_arrays([self._agent_cell, None]), stream=stream)

    def step(self, stream=None, side_stream=None):
        """One step: Cell::plan, Agent::step, Cell::commit, in this order.

        With side_stream, the agent phase runs on side_stream at the same time
        as the commit phase on `stream`: the agents to visit are recorded
        (snapshot) on side_stream while plan runs, commit waits for that
        record, so the agents it creates are not visited, and the agent phase
        reads the next state from bit 1 of the alive byte, which commit leaves
        unchanged.  The two phases touch no common field, so the result is
        that of the sequential order."""
        if side_stream is None:
            self.heap.parallel_do(self.CELL, S.M_LIFE_PLAN, self.args, stream=stream)
            self.heap.parallel_do(self.AGENT, S.M_LIFE_AGENT, self.args, stream=stream)
            self.heap.parallel_do(self.CELL, S.M_LIFE_COMMIT, self.args, stream=stream)
            return
        if (self.heap.num_blocks + 63) // 64 >= self.heap.get_launch()["list_min_words"]:
            raise ValueError("concurrent phases need a heap below the block-list threshold (shared list buffer)")
        main = stream if stream is not None else torch.cuda.current_stream()
        side_stream.wait_stream(main)
        self.heap.snapshot(self.AGENT, stream=side_stream)
        recorded = torch.cuda.Event()
        recorded.record(side_stream)
        self.heap.parallel_do(self.CELL, S.M_LIFE_PLAN, self.args, stream=main)
        side_stream.wait_stream(main)
        self.heap.parallel_do(self.AGENT, S.M_LIFE_AGENT, self.args, stream=side_stream, from_snapshot=True)
        main.wait_event(recorded)
        self.heap.parallel_do(self.CELL, S.M_LIFE_COMMIT, self.args, stream=main)
        main.wait_stream(side_stream)

    def state(self):
        """(alive grid uint8, agent age per cell with -1 where none)."""
        x, y, a = self.heap.dump_objects(self.CELL, [np.int32, np.int32, np.uint8])
        alive = np.zeros(self.W * self.H, dtype=np.uint8)
        alive[y.astype(np.int64) * self.W + x] = a & 1          # bit 0: the state (bit 1: next)
        cell, age = self.heap.dump_objects(self.AGENT, [np.int32, np.int32])
        ages = np.full(self.W * self.H, -1, dtype=np.int32)
        assert len(np.unique(cell)) == len(cell), "two agents on one cell"
        ages[cell] = age
        return alive, ages


def wator_blocks(kind0: np.ndarray, block_objects: int = 64) -> int:
    """Heap blocks for a predator-prey instance: room for every cell holding
    an object of the largest class (capacity 42 with 64 objects per block of
    the smallest class, floor(block_objects * 8 / 12) in general) plus 50% for
    fragmentation, plus 64.  The oracle shows the population peaking at up to
    ~3.15x its initial size under these rules, so "2x the initial object
    count" runs out of blocks; this bound holds at any population."""
    n = int(kind0.size)
    cap = (block_objects * 8) // 12
    return (3 * n + 2 * cap - 1) // (2 * cap) + 64


class WaTor:
    """Predator-prey grid: Fish {int32 pos, int32 age} (class 0) and Shark
    {int32 pos, int32 age, int32 energy} (class 1) on a width x height torus."""

    CLASSES = [[4, 4], [4, 4, 4]]
    FISH, SHARK = 0, 1

    def __init__(self, seed=42, width=1024, height=1024, num_blocks=32768, fish=0.20, shark=0.05,
                 fish_breed=3, shark_breed=8, eat_gain=4, shark_e0=4, device="cuda",
                 kind0: np.ndarray | None = None, arena: "S.Arena | None" = None, block_objects: int = 64):
        self.seed, self.W, self.H = seed, width, height
        self.params = dict(fish_breed=fish_breed, shark_breed=shark_breed, eat_gain=eat_gain, shark_e0=shark_e0)
        n = width * height
        self.kind0 = inputs.wator_initial(seed, width, height, fish, shark) if kind0 is None else kind0
        self.arena, self.region = arena, None
        if num_blocks is None:
            num_blocks = wator_blocks(self.kind0, block_objects)
        if arena is None:
            self.heap = S.Heap(self.CLASSES, num_blocks, device=device, block_objects=block_objects)
            self.occ = torch.zeros(n, dtype=torch.int64, device=device)
            self.claim = torch.full((n,), INT32_MAX, dtype=torch.int32, device=device)
            self.want = torch.zeros(n, dtype=torch.int32, device=device)
        else:
            # one arena range: heap, then the three grids
            hb = (S.heap_bytes(self.CLASSES, num_blocks, block_objects) + 255) // 256 * 256
            gb = (8 * n + 255) // 256 * 256 + 2 * ((4 * n + 255) // 256 * 256)
            self.region = arena.alloc(hb + gb)
            self.heap = S.Heap(self.CLASSES, num_blocks, dev_ptr=self.region, block_objects=block_objects)
            p = self.region + hb
            self.occ = arena.view(p, n, torch.int64); p += (8 * n + 255) // 256 * 256
            self.claim = arena.view(p, n, torch.int32); p += (4 * n + 255) // 256 * 256
            self.want = arena.view(p, n, torch.int32)
            self.occ.zero_()
            self.claim.fill_(INT32_MAX)
        self.num_blocks = num_blocks
        fpos = np.nonzero(self.kind0 == 1)[0].astype(np.int32)
        spos = np.nonzero(self.kind0 == 2)[0].astype(np.int32)
        self._f = [_dev(fpos, device), None]
        self._s = [_dev(spos, device), None, _dev(np.full(len(spos), shark_e0, np.int32), device)]
        self.nf0, self.ns0 = len(fpos), len(spos)
        self.args = S.WatorArgs(self.occ.data_ptr(), self.claim.data_ptr(), self.want.data_ptr(),
                                seed & (2**64 - 1), width, height, 0, fish_breed, shark_breed, eat_gain,
                                shark_e0, self.FISH, self.SHARK, 0)
        self.t = 0

    def release(self):
        """Give an arena-backed instance's memory back to the arena."""
        self.heap.close()
        if self.region is not None:
            self.arena.free(self.region)
            self.region = None

    def populate(self, stream=None):
        if self.nf0:
            self.heap.parallel_new(self.FISH, self.nf0, S.CTOR_ARRAYS,
                                   S.ctor_arrays(self._f, ref_out=self.occ, ref_index=self._f[0]), stream=stream)
        if self.ns0:
            self.heap.parallel_new(self.SHARK, self.ns0, S.CTOR_ARRAYS,
                                   S.ctor_arrays(self._s, ref_out=self.occ, ref_index=self._s[0]), stream=stream)

    def step(self, stream=None):
        self.t += 1
        self.args.step = self.t
        self.heap.parallel_do(self.FISH, S.M_WATOR_FISH_PLAN, self.args, stream=stream)
        self.heap.parallel_do(self.FISH, S.M_WATOR_FISH_MOVE, self.args, stream=stream)
        self.heap.parallel_do(self.SHARK, S.M_WATOR_SHARK_PLAN, self.args, stream=stream)
        self.heap.parallel_do(self.SHARK, S.M_WATOR_SHARK_MOVE, self.args, stream=stream)

    def state(self):
        """(kind, age, energy) per cell, as the oracle reports them."""
        n = self.W * self.H
        kind = np.zeros(n, dtype=np.uint8)
        age = np.zeros(n, dtype=np.int32)
        energy = np.zeros(n, dtype=np.int32)
        fp, fa = self.heap.dump_objects(self.FISH, [np.int32, np.int32])
        sp, sa, se = self.heap.dump_objects(self.SHARK, [np.int32, np.int32, np.int32])
        for p in (fp, sp):
            assert len(np.unique(p)) == len(p), "two agents on one cell"
        assert len(np.intersect1d(fp, sp)) == 0, "fish and shark on one cell"
        kind[fp] = 1; age[fp] = fa
        kind[sp] = 2; age[sp] = sa; energy[sp] = se
        return kind, age, energy

    def occ_kind(self) -> np.ndarray:
        """Kind per cell as the occupancy grid records it (0 empty, 1+class)."""
        occ = self.occ.cpu().numpy().view(np.uint64)
        return np.where(occ == 0, 0, S.ref_class(occ) + 1).astype(np.uint8)


class NBody:
    """N-body with merging: Body {f32 x, f32 y, f32 vx, f32 vy, f32 m}, created
    by one parallel_new on a fresh heap, so a body's creation index is its key
    block*64 + slot."""

    CLASSES = [[4, 4, 4, 4, 4]]

    def __init__(self, seed=42, n=262144, G=1e-6, dt=1e-3, merge_dist=1e-4, hash_bits=21, pair_cap=4096,
                 device="cuda", init=None):
        self.n = n
        M = (n + 63) // 64
        self.heap = S.Heap(self.CLASSES, M, device=device)
        arrs = inputs.nbody_initial(seed, n) if init is None else init
        self.init = tuple(np.ascontiguousarray(a, dtype=np.float32) for a in arrs)
        self._src = [_dev(a, device) for a in self.init]
        self.head = torch.full((1 << hash_bits,), -1, dtype=torch.int32, device=device)
        self.next = torch.empty(M * 64, dtype=torch.int32, device=device)
        self.lab = torch.empty(M * 64, dtype=torch.int32, device=device)
        self.merged = torch.zeros(M * 64, dtype=torch.uint8, device=device)
        self.pairs = torch.empty(2 * pair_cap, dtype=torch.int32, device=device)
        self.npairs = torch.zeros(1, dtype=torch.int32, device=device)
        self.args = S.NbodyArgs(self.head.data_ptr(), self.next.data_ptr(), self.lab.data_ptr(),
                                self.merged.data_ptr(), self.pairs.data_ptr(), self.npairs.data_ptr(),
                                hash_bits, pair_cap, G, dt, merge_dist, 1024.0)

    def populate(self, stream=None):
        self.heap.parallel_new(0, self.n, S.CTOR_ARRAYS, S.ctor_arrays(self._src), stream=stream)

    def phase(self, method, stream=None):
        self.heap.parallel_do(0, method, self.args, stream=stream)

    def merge(self, stream=None):
        for m in S.NBODY_PHASES[:4]:
            self.phase(m, stream)

    def force_move(self, stream=None):
        for m in S.NBODY_PHASES[4:]:
            self.phase(m, stream)

    def step(self, stream=None):
        for m in S.NBODY_PHASES:
            self.phase(m, stream)

    def state(self):
        """(ids, x, y, vx, vy, m) of the survivors in ascending id."""
        x, y, vx, vy, m = self.heap.dump_objects(0, [np.float32] * 5)
        refs = self.heap.dump_refs(0)
        key = ((refs >> np.uint64(6)) & np.uint64((1 << 44) - 1)) * np.uint64(64) + (refs & np.uint64(63))
        return key.astype(np.int32), x, y, vx, vy, m
