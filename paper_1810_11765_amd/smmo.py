"""ctypes binding of libsmmo.so (include/smmo.h): argument marshalling only.

Every operation runs in the library's HIP kernels; torch supplies the device
buffer a heap lives in and the stream calls are queued on.  Importing this
module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsmmo.so")

MAX_CLASSES = 16
MAX_FIELDS = 16

# constructors
CTOR_ZERO = 0
CTOR_ARRAYS = 1
CTOR_NONE = 2
# methods
M_AXPY = 0
M_DESTROY_ALL = 1
M_VISIT = 2
M_CHURN = 3
M_MIX = 4
M_CHURN_API = 6
M_AXPY_GENERIC = 7
M_SPAWN = 8
M_LIFE_PLAN = 10
M_LIFE_AGENT = 11
M_LIFE_COMMIT = 12
M_WATOR_FISH_PLAN = 20
M_WATOR_FISH_MOVE = 21
M_WATOR_SHARK_PLAN = 22
M_WATOR_SHARK_MOVE = 23
# status bits
STATUS_OOM = 1
STATUS_RETRY = 2
STATUS_CORRUPT = 4
# tuning flags
TUNE_NO_ROTATE = 1
TUNE_NO_COALESCE = 2
TUNE_STATS = 4
TUNE_FORCE_FAIL = 8
TUNE_FLAT_ENUM = 32
TUNE_ROTATED_START = 64
BATCH_PHASED, BATCH_PERSISTENT = 0, 1          # smmo_batch_set_mode
COUNTERS = ["alloc_obj", "free_obj", "block_init", "block_free", "inval_rollback", "type_rollback",
            "find_fail", "reserve_fail", "spin", "reserve_atomic", "guard_alloc", "guard_spin", "guard_inval",
            "oom"]


class ClassDesc(C.Structure):
    _fields_ = [("nfields", C.c_uint32), ("field_bytes", C.POINTER(C.c_uint8)), ("superclass", C.c_uint32)]


class Layout(C.Structure):
    _fields_ = [("capacity", C.c_uint32), ("nfields", C.c_uint32), ("block_bytes", C.c_uint64),
                ("field_bytes", C.c_uint32 * MAX_FIELDS), ("field_offset", C.c_uint32 * MAX_FIELDS)]


class Launch(C.Structure):
    """smmo_launch: per-heap launch shape (0 = default)."""
    _fields_ = [("doall_waves_per_cu", C.c_uint32), ("doall_units", C.c_uint32), ("list_min_words", C.c_uint32),
                ("sweep_waves_per_cu", C.c_uint32), ("sweep_groups", C.c_uint32)]


LAUNCH_FIELDS = [f for f, _ in Launch._fields_]


class CtorNone(C.Structure):
    _fields_ = [("ref_out", C.c_void_p)]


class CtorArrays(C.Structure):
    _fields_ = [("src", C.c_void_p * MAX_FIELDS), ("ref_out", C.c_void_p), ("ref_index", C.c_void_p)]


class AxpyArgs(C.Structure):
    _fields_ = [("a", C.c_float), ("fx", C.c_uint32), ("fy", C.c_uint32), ("pad", C.c_uint32)]


class SpawnArgs(C.Structure):
    _fields_ = [("cls", C.c_uint32), ("lanes", C.c_uint32)]


class VisitArgs(C.Structure):
    _fields_ = [("visits", C.c_void_p)]


class ChurnArgs(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("round", C.c_uint32), ("pad", C.c_uint32)]


class MixArgs(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("round", C.c_uint32), ("cls_a", C.c_uint32), ("cls_b", C.c_uint32),
                ("pad", C.c_uint32)]


class LifeArgs(C.Structure):
    _fields_ = [("cell_ref", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32),
                ("cell_cls", C.c_uint32), ("agent_cls", C.c_uint32)]


class WatorArgs(C.Structure):
    _fields_ = [("occ", C.c_void_p), ("claim", C.c_void_p), ("want", C.c_void_p), ("seed", C.c_uint64),
                ("width", C.c_int32), ("height", C.c_int32), ("step", C.c_int32),
                ("fish_breed", C.c_int32), ("shark_breed", C.c_int32), ("eat_gain", C.c_int32),
                ("shark_e0", C.c_int32), ("fish_cls", C.c_uint32), ("shark_cls", C.c_uint32),
                ("pad", C.c_uint32)]


class SmmoError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SmmoError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                            "or python paper_1810_11765_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P, u32, u64, i = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
        sig = {
            "smmo_heap_bytes": ([P, u32, u64, P], i),
            "smmo_heap_create": ([P, u32, u64, P, u64, P, P], i),
            "smmo_heap_destroy": ([P], i),
            "smmo_heap_reset": ([P, P], i),
            "smmo_class_layout": ([P, u32, P], i),
            "smmo_layout_compute": ([P, u32, u32, P], i),
            "smmo_heap_bytes_ex": ([P, u32, u64, u32, P], i),
            "smmo_heap_create_ex": ([P, u32, u64, u32, P, u64, P, P], i),
            "smmo_layout_compute_ex": ([P, u32, u32, u32, P], i),
            "smmo_set_tuning": ([P, u32, u32, u32, P], i),
            "smmo_parallel_new": ([P, u32, u64, u32, P, u64, P], i),
            "smmo_parallel_alloc": ([P, u32, u64, u32, u32, P, u64, P], i),
            "smmo_parallel_do": ([P, u32, u32, P, u64, P], i),
            "smmo_parallel_do_snapshot": ([P, u32, u32, P, u64, P], i),
            "smmo_parallel_do_static_scratch": ([P, u32, u32, P, u64, P], i),
            "smmo_snapshot": ([P, u32, P], i),
            "smmo_time_next_doall": ([P, P, P], i),
            "smmo_parallel_destroy": ([P, P, u64, u32, P], i),
            "smmo_occupancy": ([P, P, P, P, P], i),
            "smmo_atomic_probe": ([P, u64, u32, u64, u32, P], i),
            "smmo_set_launch": ([P, P], i),
            "smmo_get_launch": ([P, P], i),
            "smmo_live_count": ([P, u32, P, P], i),
            "smmo_dump_objects": ([P, u32, P, u64, P, P], i),
            "smmo_dump_refs": ([P, u32, P, u64, P, P], i),
            "smmo_raw_bytes": ([P, P], i),
            "smmo_dump_raw": ([P, P, u64, P], i),
            "smmo_status": ([P, P, P], i),
            "smmo_clear_status": ([P, P], i),
            "smmo_stats": ([P, P, u32, P], i),
            "smmo_ref_make": ([u32, u64, u32], u64),
            "smmo_ref_class": ([u64], u32),
            "smmo_ref_block": ([u64], u64),
            "smmo_ref_slot": ([u64], u32),
            "smmo_strerror": ([i], C.c_char_p),
            "smmo_last_error": ([], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(rc: int) -> None:
    if rc != 0:
        L = lib()
        raise SmmoError(f"{L.smmo_strerror(rc).decode()} ({rc}): {L.smmo_last_error().decode()}")


def class_spec(c):
    """(own field sizes, superclass id or None) of a class given either as a
    list of field byte sizes or as {"fields": [...], "super": id}."""
    if isinstance(c, dict):
        return list(c.get("fields", [])), c.get("super")
    return list(c), None


def full_fields(classes):
    """Every class's field sizes, inherited fields first."""
    out = []
    for c in classes:
        own, sup = class_spec(c)
        out.append((list(out[sup]) if sup is not None else []) + own)
    return out


def _descs(classes):
    specs = [class_spec(c) for c in classes]
    arrs = [(C.c_uint8 * max(len(own), 1))(*own) for own, _ in specs]
    descs = (ClassDesc * len(classes))()
    for d, a, (own, sup) in zip(descs, arrs, specs):
        d.nfields = len(own)
        d.field_bytes = C.cast(a, C.POINTER(C.c_uint8))
        d.superclass = 0 if sup is None else sup + 1
    return descs, arrs


def layout_of(classes, cls: int, block_objects: int = 64) -> Layout:
    """Layout of class `cls` computed by the library without a heap."""
    descs, _keep = _descs(classes)
    out = Layout()
    check(lib().smmo_layout_compute_ex(descs, len(classes), block_objects, cls, C.byref(out)))
    return out


def heap_bytes(classes, num_blocks: int, block_objects: int = 64) -> int:
    descs, _keep = _descs(classes)
    out = C.c_uint64()
    check(lib().smmo_heap_bytes_ex(descs, len(classes), num_blocks, block_objects, C.byref(out)))
    return out.value


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _blob(args):
    if args is None:
        return None, 0
    return C.c_void_p(C.addressof(args)), C.sizeof(args)


class Heap:
    """A heap of `num_blocks` blocks for `classes` (lists of field byte sizes,
    or {"fields": [...], "super": id} for a subclass) inside one torch uint8
    device tensor owned by this object.  `classes` holds every class's full
    field list afterwards, inherited fields first."""

    def __init__(self, classes, num_blocks: int, device="cuda", stream=None, dev_ptr: int | None = None,
                 block_objects: int = 64):
        import torch
        self.specs = list(classes)
        self.classes = full_fields(self.specs)
        self.num_blocks = num_blocks
        self.block_objects = block_objects
        nbytes = heap_bytes(self.specs, num_blocks, block_objects)
        if dev_ptr is None:
            # 4 KiB slack so the buffer can be aligned to 256 bytes
            self.buf = torch.empty(nbytes + 4096, dtype=torch.uint8, device=device)
            base = self.buf.data_ptr()
            self.base = base + (-base) % 256
        else:
            self.buf = None                      # memory owned by the caller (an arena range)
            self.base = dev_ptr
        self.nbytes = nbytes
        descs, _keep = _descs(self.specs)
        h = C.c_void_p()
        check(lib().smmo_heap_create_ex(descs, len(self.classes), num_blocks, block_objects, C.c_void_p(self.base),
                                        nbytes, _stream(stream), C.byref(h)))
        self.h = h
        self.layouts = [self.layout(t) for t in range(len(self.classes))]

    def close(self):
        if getattr(self, "h", None):
            lib().smmo_heap_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- queries
    def layout(self, cls: int) -> Layout:
        out = Layout()
        check(lib().smmo_class_layout(self.h, cls, C.byref(out)))
        return out

    def capacity(self, cls: int) -> int:
        return self.layouts[cls].capacity

    def live_count(self, cls: int, stream=None) -> int:
        out = C.c_uint64()
        check(lib().smmo_live_count(self.h, cls, C.byref(out), _stream(stream)))
        return out.value

    def status(self, stream=None) -> int:
        out = C.c_uint32()
        check(lib().smmo_status(self.h, C.byref(out), _stream(stream)))
        return out.value

    def clear_status(self, stream=None) -> None:
        check(lib().smmo_clear_status(self.h, _stream(stream)))

    def stats(self, stream=None) -> dict:
        out = (C.c_uint64 * 16)()
        check(lib().smmo_stats(self.h, out, 16, _stream(stream)))
        return {k: int(out[i]) for i, k in enumerate(COUNTERS)}

    def set_tuning(self, flags: int = 0, lookups: int = 5, force_fail_ppm: int = 0, stream=None) -> None:
        check(lib().smmo_set_tuning(self.h, flags, lookups, force_fail_ppm, _stream(stream)))

    def reset(self, stream=None) -> None:
        check(lib().smmo_heap_reset(self.h, _stream(stream)))

    def set_launch(self, **fields) -> None:
        """Launch shape of this heap's kernels (smmo_launch fields; omitted or 0 =
        default).  Results do not depend on it."""
        unknown = set(fields) - set(LAUNCH_FIELDS)
        assert not unknown, f"unknown launch fields {unknown}"
        check(lib().smmo_set_launch(self.h, C.byref(Launch(**fields))))

    def get_launch(self) -> dict:
        out = Launch()
        check(lib().smmo_get_launch(self.h, C.byref(out)))
        return {f: getattr(out, f) for f in LAUNCH_FIELDS}

    # -- operations
    def parallel_new(self, cls: int, n: int, ctor: int = CTOR_ZERO, args=None, stream=None) -> None:
        p, nb = _blob(args)
        check(lib().smmo_parallel_new(self.h, cls, n, ctor, p, nb, _stream(stream)))

    def parallel_alloc(self, cls: int, nthreads: int, per_thread: int, ctor: int = CTOR_ZERO, args=None,
                       stream=None) -> None:
        p, nb = _blob(args)
        check(lib().smmo_parallel_alloc(self.h, cls, nthreads, per_thread, ctor, p, nb, _stream(stream)))

    def parallel_destroy(self, refs, nthreads: int, per_thread: int = 1, stream=None) -> None:
        """Thread t destroys refs[t*per_thread + k], k < per_thread (device uint64 tensor)."""
        assert refs.numel() >= nthreads * per_thread and refs.element_size() == 8 and refs.is_contiguous()
        check(lib().smmo_parallel_destroy(self.h, refs.data_ptr(), nthreads, per_thread, _stream(stream)))

    def occupancy(self, stream=None) -> dict:
        """Per-class used slots, slots and blocks, and the fragmentation F (Sec. 6.3)."""
        n = len(self.classes)
        used, slots, blocks = (C.c_uint64 * n)(), (C.c_uint64 * n)(), (C.c_uint64 * n)()
        check(lib().smmo_occupancy(self.h, used, slots, blocks, _stream(stream)))
        u, sl, b = list(used), list(slots), list(blocks)
        return {"used": u, "slots": sl, "blocks": b, "F": (1.0 - sum(u) / sum(sl)) if sum(sl) else 0.0}

    def parallel_do(self, cls: int, method: int, args=None, stream=None, from_snapshot: bool = False,
                    static_scratch: bool = False) -> None:
        """Run `method` on every live object of `cls` and its subclasses; with
        from_snapshot, on the objects recorded by the last snapshot(cls); with
        static_scratch, through smmo_parallel_do_static_scratch."""
        p, nb = _blob(args)
        assert not (from_snapshot and static_scratch)
        fn = (lib().smmo_parallel_do_snapshot if from_snapshot else
              lib().smmo_parallel_do_static_scratch if static_scratch else lib().smmo_parallel_do)
        check(fn(self.h, cls, method, p, nb, _stream(stream)))

    def time_next_doall(self, start, stop) -> None:
        """Make the next do-all kernel record torch events `start` and `stop`
        (enable_timing=True) at its own start and end."""
        for e in (start, stop):
            if e.cuda_event == 0:                  # torch creates the HIP event on first record
                e.record()
        check(lib().smmo_time_next_doall(self.h, C.c_void_p(start.cuda_event), C.c_void_p(stop.cuda_event)))

    def snapshot(self, cls: int, stream=None) -> None:
        """Record the objects of `cls` (and subclasses) live now, for a later
        parallel_do(..., from_snapshot=True)."""
        check(lib().smmo_snapshot(self.h, cls, _stream(stream)))

    # -- dumps (synchronize)
    def dump_objects(self, cls: int, dtypes, stream=None):
        """Live objects of `cls` as a list of numpy arrays, one per field."""
        n = self.live_count(cls, stream)
        bufs = [np.zeros(max(n, 1), dtype=dt) for dt in dtypes]
        assert [b.itemsize for b in bufs] == self.classes[cls], "dtype sizes must match the field sizes"
        ptrs = (C.c_void_p * MAX_FIELDS)(*[b.ctypes.data for b in bufs])
        got = C.c_uint64()
        check(lib().smmo_dump_objects(self.h, cls, ptrs, n, C.byref(got), _stream(stream)))
        assert got.value == n, (got.value, n)
        return [b[:n] for b in bufs]

    def dump_refs(self, cls: int, stream=None) -> np.ndarray:
        n = self.live_count(cls, stream)
        out = np.zeros(max(n, 1), dtype=np.uint64)
        got = C.c_uint64()
        check(lib().smmo_dump_refs(self.h, cls, out.ctypes.data, n, C.byref(got), _stream(stream)))
        return out[: got.value]

    def dump_raw(self, stream=None) -> bytes:
        nb = C.c_uint64()
        check(lib().smmo_raw_bytes(self.h, C.byref(nb)))
        buf = np.zeros(nb.value, dtype=np.uint8)
        check(lib().smmo_dump_raw(self.h, buf.ctypes.data, nb.value, _stream(stream)))
        return buf.tobytes()


def atomic_probe(words, lanes_per_word: int, nthreads: int, rounds: int, stream=None) -> None:
    """Atomic-throughput reference kernel (see smmo_atomic_probe) on a device
    int64 tensor `words`."""
    assert words.element_size() == 8 and words.is_contiguous()
    check(lib().smmo_atomic_probe(words.data_ptr(), words.numel(), lanes_per_word, nthreads, rounds,
                                  _stream(stream)))


def ctor_none(ref_out=None) -> CtorNone:
    """Argument blob of CTOR_NONE: object memory untouched, handle i -> ref_out[i]."""
    return CtorNone(None if ref_out is None else ref_out.data_ptr())


def ctor_arrays(srcs, ref_out=None, ref_index=None) -> CtorArrays:
    """Argument blob of CTOR_ARRAYS from device tensors (None = zero field)."""
    a = CtorArrays()
    for f, t in enumerate(srcs):
        a.src[f] = None if t is None else t.data_ptr()
    a.ref_out = None if ref_out is None else ref_out.data_ptr()
    a.ref_index = None if ref_index is None else ref_index.data_ptr()
    return a


def ref_class(ref) -> np.ndarray:
    return (np.asarray(ref, dtype=np.uint64) >> np.uint64(56)).astype(np.int64) - 1


M_NBODY_INSERT = 30
M_NBODY_PAIRS = 31
M_NBODY_RESOLVE = 32
M_NBODY_REAP = 33
M_NBODY_FORCE = 34
M_NBODY_MOVE = 35
NBODY_PHASES = (M_NBODY_INSERT, M_NBODY_PAIRS, M_NBODY_RESOLVE, M_NBODY_REAP, M_NBODY_FORCE, M_NBODY_MOVE)


class NbodyArgs(C.Structure):
    _fields_ = [("head", C.c_void_p), ("next", C.c_void_p), ("lab", C.c_void_p), ("merged", C.c_void_p),
                ("pairs", C.c_void_p), ("npairs", C.c_void_p), ("hash_bits", C.c_uint32),
                ("pair_cap", C.c_uint32), ("G", C.c_float), ("dt", C.c_float), ("merge_dist", C.c_float),
                ("inv_cell", C.c_float)]


M_STRESS = 5


class StressArgs(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("iters", C.c_uint32), ("lanes", C.c_uint32), ("cls_a", C.c_uint32),
                ("cls_b", C.c_uint32)]
TUNE_SLOW_PICK = 16


def _bind_batch():
    L = lib()
    P, u32, u64, i = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
    sig = {
        "smmo_arena_create": ([P, u64, P], i), "smmo_arena_destroy": ([P], i),
        "smmo_arena_alloc": ([P, u64, P], i), "smmo_arena_free": ([P, P], i),
        "smmo_arena_stats": ([P, P, P], i),
        "smmo_batch_create": ([P, u32, P], i), "smmo_batch_destroy": ([P], i),
        "smmo_batch_add_wator": ([P, P, P, u32, P, P], i), "smmo_batch_remove": ([P, u32], i),
        "smmo_batch_step": ([P, u32, P], i), "smmo_batch_remaining": ([P, P, P], i),
        "smmo_batch_grid": ([P, P], i), "smmo_batch_set_grid": ([P, u32], i),
        "smmo_batch_set_mode": ([P, u32], i),
        "smmo_batch_capture_graph": ([P, u32, u32, P, P], i), "smmo_batch_graph_launch": ([P, P], i),
        "smmo_batch_graph_destroy": ([P], i),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    return L


class Arena:
    """Range allocator (in the library) over one torch device buffer."""

    def __init__(self, nbytes: int, device="cuda"):
        import torch
        L = _bind_batch()
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        h = C.c_void_p()
        check(L.smmo_arena_create(C.c_void_p(self.buf.data_ptr()), nbytes + 256, C.byref(h)))
        self.h = h

    def alloc(self, nbytes: int) -> int:
        p = C.c_void_p()
        check(lib().smmo_arena_alloc(self.h, nbytes, C.byref(p)))
        return p.value

    def try_alloc(self, nbytes: int):
        p = C.c_void_p()
        rc = lib().smmo_arena_alloc(self.h, nbytes, C.byref(p))
        return p.value if rc == 0 else None

    def free(self, ptr: int) -> None:
        check(lib().smmo_arena_free(self.h, C.c_void_p(ptr)))

    def stats(self):
        f, big = C.c_uint64(), C.c_uint64()
        check(lib().smmo_arena_stats(self.h, C.byref(f), C.byref(big)))
        return f.value, big.value

    def view(self, ptr: int, count: int, dtype):
        """torch view of `count` elements of `dtype` at device address ptr."""
        import torch
        off = ptr - self.buf.data_ptr()
        nbytes = count * torch.empty((), dtype=dtype).element_size()
        return self.buf[off: off + nbytes].view(dtype)

    def close(self):
        if getattr(self, "h", None):
            lib().smmo_arena_destroy(self.h)
            self.h = None


class Batch:
    """Persistent-kernel batch of predator-prey instances (see smmo.h)."""

    def __init__(self, arena: Arena, max_instances: int = 256):
        L = _bind_batch()
        h = C.c_void_p()
        check(L.smmo_batch_create(arena.h, max_instances, C.byref(h)))
        self.h = h
        self.max_instances = max_instances

    def add(self, heap, args: "WatorArgs", steps: int, stream=None) -> int:
        slot = C.c_uint32()
        check(lib().smmo_batch_add_wator(self.h, heap.h, C.byref(args), steps, _stream(stream), C.byref(slot)))
        return slot.value

    def remove(self, slot: int) -> None:
        check(lib().smmo_batch_remove(self.h, slot))

    def step(self, steps: int = 1, stream=None) -> None:
        check(lib().smmo_batch_step(self.h, steps, _stream(stream)))

    def remaining(self, stream=None) -> np.ndarray:
        out = np.zeros(self.max_instances, dtype=np.uint32)
        check(lib().smmo_batch_remaining(self.h, out.ctypes.data, _stream(stream)))
        return out

    def capture_graph(self, launches: int, steps_per_launch: int = 1, stream=None) -> "BatchGraph":
        """smmo_batch_capture_graph on `stream` (a created stream; torch's current
        stream when None, which must then not be the null stream)."""
        g = C.c_void_p()
        check(lib().smmo_batch_capture_graph(self.h, launches, steps_per_launch, _stream(stream), C.byref(g)))
        return BatchGraph(g)

    def grid(self) -> int:
        g = C.c_uint32()
        check(lib().smmo_batch_grid(self.h, C.byref(g)))
        return g.value

    def set_grid(self, wg_per_cu: int = 0) -> None:
        """Workgroups per CU of the batch's launches (0 = the mode's default)."""
        check(lib().smmo_batch_set_grid(self.h, wg_per_cu))

    def set_mode(self, mode: int) -> None:
        """BATCH_PHASED (one launch per phase, the default) or BATCH_PERSISTENT."""
        check(lib().smmo_batch_set_mode(self.h, mode))

    def close(self):
        if getattr(self, "h", None):
            lib().smmo_batch_destroy(self.h)
            self.h = None


class BatchGraph:
    """An instantiated HIP graph of batch steps (smmo_batch_capture_graph)."""

    def __init__(self, handle):
        self.h = handle

    def launch(self, stream=None) -> None:
        check(lib().smmo_batch_graph_launch(self.h, _stream(stream)))

    def close(self):
        if getattr(self, "h", None):
            lib().smmo_batch_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
