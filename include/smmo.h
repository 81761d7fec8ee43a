/*
 * smmo.h — C-ABI of the MI355X SMMO object heap (DynaSOAr method).
 *
 * Method: Springer & Masuhara, "DynaSOAr: A Parallel Memory Allocator for
 * Object-oriented Programming on GPUs with Efficient Memory Access", ECOOP
 * 2019 (arXiv 1810.11765).  Sec. 2.1 lists the operations this library
 * exports: parallel_do, parallel_new, device-side new / destroy, device_do.
 *
 * Conventions for every entry point
 *  - Return 0 on success or a negative SMMO_E* code; smmo_last_error() gives a
 *    message for the calling thread's last failure.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call is asynchronous on that stream unless it says "synchronizes".
 *  - Device pointers are addresses in the current HIP device's memory; host
 *    pointers are ordinary process memory.  No call allocates device memory:
 *    the caller hands in one device buffer per heap and owns it.
 *  - Handles (smmo_heap*) are not thread-safe; one stream per heap at a time.
 */
#ifndef SMMO_H
#define SMMO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ limits ---- */
#define SMMO_MAX_CLASSES 16       /* class ids 0..15 (the paper's 8-bit type id, Sec. 3.3) */
#define SMMO_MAX_FIELDS 16        /* fields per class */
#define SMMO_MAX_LEVELS 6         /* bitmap levels: 64^6 blocks */
#define SMMO_ARGS_MAX 256         /* bytes of a method / constructor argument blob */

/* ------------------------------------------------------------ errors ---- */
#define SMMO_OK 0
#define SMMO_EINVAL (-1)          /* bad descriptor, class id, method id or size */
#define SMMO_ETOOSMALL (-2)       /* dev_bytes below smmo_heap_bytes() */
#define SMMO_ENOMEM_DEVICE (-3)   /* the heap ran out of blocks (sticky status) */
#define SMMO_ERETRY (-4)          /* a bounded retry loop gave up (sticky status) */
#define SMMO_EHIP (-5)            /* a HIP runtime call failed; see smmo_last_error() */
#define SMMO_ECORRUPT (-6)        /* a precondition violation was detected on the device */
#define SMMO_ENOTBUILT (-7)       /* requested kernel variant not compiled in */

/* Sticky device status bits (smmo_status). */
#define SMMO_STATUS_OOM 1u        /* an allocation found no active and no free block */
#define SMMO_STATUS_RETRY 2u      /* a spinning bitmap set/clear exceeded its bound */
#define SMMO_STATUS_CORRUPT 4u    /* e.g. destroy of a slot that is not live */

/* ------------------------------------------------------------- types ---- */

/* One class: the byte sizes of the fields it introduces, in declaration
 * order (each 1, 2, 4 or 8), and its direct superclass.  A subclass's objects
 * hold the superclass's fields first (inherited, same field indices), then
 * its own (Sec. 3.2: inherited SOA arrays first), so a method written for a
 * class runs unchanged on its subclasses.  A subclass may introduce no field
 * (nfields 0, field_bytes NULL); every class has 1..SMMO_MAX_FIELDS fields
 * in all.  Blocks hold objects of exactly one class; allocated[T] and
 * active[T] index T's own blocks only (Sec. 3.4). */
typedef struct smmo_class_desc {
    uint32_t nfields;
    const uint8_t* field_bytes;   /* host array of nfields sizes */
    uint32_t superclass;          /* 0: none; else 1 + the superclass's id, which
                                     must be smaller than this class's id */
} smmo_class_desc;

/* Layout of one class inside a block (Sec. 3.2; SOA arrays 128-B aligned). */
typedef struct smmo_layout {
    uint32_t capacity;                       /* N_T = floor(64*size(T_s)/size(T)) */
    uint32_t nfields;
    uint64_t block_bytes;                    /* bytes of every block's data segment */
    uint32_t field_bytes[SMMO_MAX_FIELDS];
    uint32_t field_offset[SMMO_MAX_FIELDS];  /* byte offset of the field's SOA array */
} smmo_layout;

typedef struct smmo_heap smmo_heap;          /* opaque host handle */

/*
 * Raw heap metadata, the first bytes of the device buffer and of
 * smmo_dump_raw's output.  All integers little-endian.  Byte offsets are from
 * the start of the device buffer.
 *   type[M]   uint32 block type id (0xFFFFFFFF: never initialized)
 *   alloc[M]  uint64 object allocation bitmap of each block (Sec. 3.1)
 *   iter[M]   uint64 object iteration bitmap of each block (Sec. 3.1)
 *   bitmaps   uint64 words; bitmap b (0 = free, 1+T = allocated[T],
 *             1+ncls+T = active[T], Sec. 3.4) starts at word b*bitmap_words;
 *             its level l (0 = containers of block bits) starts
 *             level_off[l] words further and has level_words[l] words,
 *             word k of the level at level_off[l] + k*bitmap_stride (16:
 *             every word on a 128-B line of its own, so that the atomics of
 *             different words never queue on one line; the words between
 *             are unused and zero).
 *             Bit i of level l+1 is the OR of word i of level l (Sec. 4.1.1).
 *   data      block b's data segment is at off_data + b*block_bytes.
 */
#define SMMO_MAGIC 0x504145484F4D4D53ull /* "SMMOHEAP" in little-endian bytes */
typedef struct smmo_raw_header {
    uint64_t magic;
    uint64_t version;                        /* 2 */
    uint64_t num_blocks;                     /* M */
    uint64_t ncls;
    uint64_t block_bytes;
    uint64_t nlevels;
    uint64_t level_words[SMMO_MAX_LEVELS];
    uint64_t level_off[SMMO_MAX_LEVELS];
    uint64_t bitmap_words;
    uint64_t off_status;                     /* uint32 status, then uint64 counters[16] at +64 */
    uint64_t off_type;
    uint64_t off_alloc;
    uint64_t off_iter;
    uint64_t off_bitmaps;
    uint64_t off_scratch;
    uint64_t scratch_bytes;
    uint64_t off_data;                       /* = raw dump size */
    uint64_t total_bytes;
    uint64_t capacity[SMMO_MAX_CLASSES];
    uint64_t nfields[SMMO_MAX_CLASSES];
    uint32_t field_bytes[SMMO_MAX_CLASSES][SMMO_MAX_FIELDS];
    uint32_t field_off[SMMO_MAX_CLASSES][SMMO_MAX_FIELDS];
    uint32_t tune_flags;                     /* SMMO_TUNE_* */
    uint32_t lookups;                        /* active-block lookup attempts r (Sec. 4.2) */
    uint32_t force_fail_ppm;                 /* fault injection rate of try_find_set */
    uint32_t bitmap_stride;                  /* words between consecutive words of a bitmap level */
    uint32_t superclass[SMMO_MAX_CLASSES];   /* as in smmo_class_desc (0: none) */
} smmo_raw_header;

/* Device counters (SMMO_TUNE_STATS), uint64 at off_status + 64. */
enum smmo_counter {
    SMMO_CNT_ALLOC_OBJ = 0,     /* objects allocated by the device allocator */
    SMMO_CNT_FREE_OBJ,          /* objects destroyed */
    SMMO_CNT_BLOCK_INIT,        /* slow paths: blocks initialized (Alg. 1 slow path) */
    SMMO_CNT_BLOCK_FREE,        /* successful invalidations (Alg. 9) */
    SMMO_CNT_INVAL_ROLLBACK,    /* invalidation rollbacks */
    SMMO_CNT_TYPE_ROLLBACK,     /* reservations rolled back after a type change */
    SMMO_CNT_FIND_FAIL,         /* active-block lookups that failed */
    SMMO_CNT_RESERVE_FAIL,      /* reservations that got no slot */
    SMMO_CNT_SPIN,              /* retries of spinning set/clear */
    SMMO_CNT_RESERVE_ATOMIC,    /* atomic ORs on allocation bitmaps */
    /* the next four are counted whether or not SMMO_TUNE_STATS is set */
    SMMO_CNT_GUARD_ALLOC,       /* allocations abandoned at the retry bound (SMMO_STATUS_RETRY) */
    SMMO_CNT_GUARD_SPIN,        /* bitmap set/clear spins abandoned at their bound (SMMO_STATUS_RETRY) */
    SMMO_CNT_GUARD_INVAL,       /* invalidations abandoned at their bound (SMMO_STATUS_RETRY) */
    SMMO_CNT_OOM,               /* wave allocation requests that ended in OOM */
    SMMO_CNT_NUM = 16
};

/* Tuning / ablation / fault-injection flags (smmo_set_tuning). */
#define SMMO_TUNE_NO_ROTATE 1u      /* plain find-first-set (paper's "-NoShift") */
#define SMMO_TUNE_NO_COALESCE 2u    /* one slot per reservation ("-NoCoal") */
#define SMMO_TUNE_STATS 4u          /* maintain device counters */
#define SMMO_TUNE_FORCE_FAIL 8u     /* try_find_set fails force_fail_ppm / 1e6 of the time */
#define SMMO_TUNE_SLOW_PICK 16u     /* pause ~20 us between picking an active block and
                                       reserving in it (widens the race window of App. A.3) */
#define SMMO_TUNE_ROTATED_START 64u /* bitmap lookups use the paper's rotated find-first-set
                                       (start at a wave- and retry-dependent bit) instead of
                                       picking one of the word's set bits uniformly */
#define SMMO_TUNE_FLAT_ENUM 32u     /* do-all, snapshot and live count scan every level-0
                                       word even in big heaps (no level-1 skip) */

/* -------------------------------------------------- heap management ---- */

/* Bytes of device memory a heap of `num_blocks` blocks for these classes
 * needs (metadata + scratch + data).  Classes: 1..SMMO_MAX_CLASSES, each with
 * 1..SMMO_MAX_FIELDS fields; no class may be more than 64x the smallest
 * (Sec. 3.2).  num_blocks: 1..2^32 (block ids are kept in 32 bits by the
 * enumeration lists).  Errors: SMMO_EINVAL. */
int smmo_heap_bytes(const smmo_class_desc* cls, uint32_t ncls, uint64_t num_blocks,
                    uint64_t* bytes_out);

/* Create a heap of `num_blocks` equal blocks (Sec. 3) inside the caller's
 * device buffer `dev_mem` (256-B aligned, `dev_bytes` >= smmo_heap_bytes()).
 * Enqueues the initialization on `stream`: every block free, every allocation
 * word all ones ("invalidated", so a stale pick fails), bitmaps consistent.
 * The caller keeps ownership of dev_mem and must keep it alive until
 * smmo_heap_destroy.  Errors: SMMO_EINVAL, SMMO_ETOOSMALL, SMMO_EHIP. */
int smmo_heap_create(const smmo_class_desc* cls, uint32_t ncls, uint64_t num_blocks,
                     void* dev_mem, uint64_t dev_bytes, void* stream, smmo_heap** out);

/* The same with a block capacity other than the paper's: block_objects
 * (1..64) objects per block for the smallest class, N_T = floor(block_objects
 * * size(T_s) / size(T)) for the others (Sec. 3.2 with 64 replaced; slots
 * from N_T to 63 of a block's allocation word stay set as padding, App. A.1).
 * A layout parameter the autotuner searches; results of a workload do not
 * depend on it.  block_objects = 64 is smmo_heap_bytes / smmo_heap_create.
 * Errors as those, and SMMO_EINVAL for block_objects outside 1..64 or a class
 * more than block_objects times the smallest. */
int smmo_heap_bytes_ex(const smmo_class_desc* cls, uint32_t ncls, uint64_t num_blocks, uint32_t block_objects,
                       uint64_t* bytes_out);
int smmo_heap_create_ex(const smmo_class_desc* cls, uint32_t ncls, uint64_t num_blocks, uint32_t block_objects,
                        void* dev_mem, uint64_t dev_bytes, void* stream, smmo_heap** out);

/* Free the host handle (never the device buffer).  NULL is accepted. */
int smmo_heap_destroy(smmo_heap* heap);

/* Re-initialize the heap to the empty state (all objects dropped). */
int smmo_heap_reset(smmo_heap* heap, void* stream);

/* Layout of class `cls` (host-side, no device access). */
int smmo_class_layout(const smmo_heap* heap, uint32_t cls, smmo_layout* out);

/* Same layout computed from the class descriptors alone, without a heap
 * (host-side only).  Errors: SMMO_EINVAL. */
int smmo_layout_compute(const smmo_class_desc* cls, uint32_t ncls, uint32_t which, smmo_layout* out);
int smmo_layout_compute_ex(const smmo_class_desc* cls, uint32_t ncls, uint32_t block_objects, uint32_t which,
                           smmo_layout* out);

/* Tuning: flags SMMO_TUNE_*, lookups = active-block lookup attempts before
 * the slow path (paper default 5; 1..64), force_fail_ppm for SMMO_TUNE_FORCE_FAIL.
 * Enqueued on `stream`. */
int smmo_set_tuning(smmo_heap* heap, uint32_t flags, uint32_t lookups, uint32_t force_fail_ppm,
                    void* stream);

/* ----------------------------------------------------- constructors ---- */
/* ctor_id values.  A constructor runs on each new object right after its slot
 * is reserved; `i` is the object's index in the creating call (Sec. 2.1:
 * parallel_new passes 0..n-1). */
#define SMMO_CTOR_ZERO 0u           /* all fields zero; args unused */
#define SMMO_CTOR_ARRAYS 1u         /* fields from device arrays, see below */
#define SMMO_CTOR_NONE 2u           /* object memory untouched (the raw allocation
                                       benchmark of Sec. 6.4); see smmo_ctor_none */

/* Argument blob of SMMO_CTOR_ARRAYS: field f of object i = src[f][i] (src[f]
 * NULL: zero).  If ref_out is non-NULL the new handle is stored at
 * ref_out[ref_index ? ref_index[i] : i].  All pointers are device pointers. */
typedef struct smmo_ctor_arrays {
    const void* src[SMMO_MAX_FIELDS];
    uint64_t* ref_out;
    const int32_t* ref_index;
} smmo_ctor_arrays;

/* Argument blob of SMMO_CTOR_NONE (may be omitted: args NULL, 0 bytes): if
 * ref_out is non-NULL the new handle of object i is stored at ref_out[i]
 * (device pointer); the object's fields are never written. */
typedef struct smmo_ctor_none {
    uint64_t* ref_out;
} smmo_ctor_none;

/* ---------------------------------------------------------- methods ---- */
/* method_id values for smmo_parallel_do.  A method runs once on every object
 * of the class that is live when the do-all starts (Sec. 2.1, Sec. 3.1);
 * objects it creates are not visited by the same do-all; it may destroy
 * `this` and objects of other classes only. */
#define SMMO_M_AXPY 0u              /* f32 fields: y += a*x           (smmo_axpy_args)  */
#define SMMO_M_DESTROY_ALL 1u       /* every object destroys itself   (no args)         */
#define SMMO_M_VISIT 2u             /* visits[id field 0] += 1        (smmo_visit_args) */
#define SMMO_M_CHURN 3u             /* alloc microbench round         (smmo_churn_args) */
#define SMMO_M_MIX 4u               /* two-class churn (test method)  (smmo_mix_args)   */
#define SMMO_M_STRESS 5u            /* alloc/destroy storm (test)     (smmo_stress_args) */
#define SMMO_M_CHURN_API 6u         /* SMMO_M_CHURN written against smmo_device.h only      */
#define SMMO_M_SPAWN 8u             /* lanes < a.lanes of every block each create one object of
                                       class a.cls, fields untouched (smmo_spawn_args): partial
                                       wave requests sharing active blocks */
#define SMMO_M_AXPY_GENERIC 7u      /* SMMO_M_AXPY through the generic do-all kernel (one
                                       wave per block, lane = slot), not the streaming one */
#define SMMO_M_LIFE_PLAN 10u        /* Cell: next state, B3/S23       (smmo_life_args)  */
#define SMMO_M_LIFE_AGENT 11u       /* Agent: die or age              (smmo_life_args)  */
#define SMMO_M_LIFE_COMMIT 12u      /* Cell: birth of agents, commit  (smmo_life_args)  */
#define SMMO_M_WATOR_FISH_PLAN 20u  /* Fish: age, choose and claim    (smmo_wator_args) */
#define SMMO_M_WATOR_FISH_MOVE 21u  /* Fish: move, breed              (smmo_wator_args) */
#define SMMO_M_WATOR_SHARK_PLAN 22u /* Shark: age, choose and claim   (smmo_wator_args) */
#define SMMO_M_WATOR_SHARK_MOVE 23u /* Shark: move, eat, breed, starve(smmo_wator_args) */
#define SMMO_M_NBODY_INSERT 30u     /* Body: enter the cell hash grid (smmo_nbody_args) */
#define SMMO_M_NBODY_PAIRS 31u      /* Body: list close pairs         (smmo_nbody_args) */
#define SMMO_M_NBODY_RESOLVE 32u    /* class phase: merge components  (smmo_nbody_args) */
#define SMMO_M_NBODY_REAP 33u       /* Body: merged bodies destroy themselves, grid reset */
#define SMMO_M_NBODY_FORCE 34u      /* Body: all-pairs force via device_do, v += a*dt   */
#define SMMO_M_NBODY_MOVE 35u       /* Body: x += v*dt                                  */

/* y += a*x on float32 fields fx, fy of the class (one rounding: a*x is formed
 * first, then added). */
typedef struct smmo_axpy_args { float a; uint32_t fx; uint32_t fy; uint32_t pad; } smmo_axpy_args;

/* Test method: atomically increments visits[field0 (int32)]. */
typedef struct smmo_visit_args { uint32_t* visits; } smmo_visit_args;

/* SMMO_M_SPAWN: objects of class `cls` created by the first `lanes` (1..64)
 * slots of every visited block that hold a live object. */
typedef struct smmo_spawn_args { uint32_t cls; uint32_t lanes; } smmo_spawn_args;
/* Alloc microbench round `round` on class {int32 id, f32 x, f32 v}: each
 * object with splitmix64(seed ^ id ^ round) odd destroys itself and allocates
 * a replacement id' = ((round+1) << 18) | (id & 0x3FFFF) with
 * x' = U01(ctr(seed, round+1, id', 0)), v' = U01(ctr(seed, round+1, id', 1)). */
typedef struct smmo_churn_args { uint64_t seed; uint32_t round; uint32_t pad; } smmo_churn_args;

/* Two-class churn on classes whose field 0 is an int32 id (test method that
 * makes blocks change type while other waves allocate): with
 * h = splitmix64(seed ^ id ^ (round << 32)), an object with h odd destroys
 * itself and allocates a replacement id' = ((round+1) << 18) | (id & 0x3FFFF)
 * in class cls_b if bit 1 of h is set, else in cls_a.  Other fields: zero. */
typedef struct smmo_mix_args {
    uint64_t seed;
    uint32_t round;
    uint32_t cls_a, cls_b;
    uint32_t pad;
} smmo_mix_args;

/* Allocation storm (test method that forces the races of App. A.3-A.4):
 * every wave of the do-all runs `iters` rounds; in round k the lanes whose
 * slot is below `lanes` allocate one object each, in cls_b if bit 0 of
 * splitmix64(seed ^ (key << 20) ^ k) is set else in cls_a, write the
 * allocating object's key into field 0, and destroy it again in the same
 * round.  The driver objects are not changed.  Classes a and b need an int32
 * field 0; at the end no object of either class remains. */
typedef struct smmo_stress_args {
    uint64_t seed;
    uint32_t iters, lanes;
    uint32_t cls_a, cls_b;
} smmo_stress_args;

/* Life-like grid on a width x height torus.  Cell {int32 x, int32 y, int8
 * alive}: alive bit 0 = current, bit 1 = next (plan sets bit 1; commit copies
 * it into bit 0 and leaves bit 1 as it is, so the agent phase, which reads
 * bit 1, sees the same value before and after the commit of its cell and may
 * run concurrently with the commit phase).  Agent {int32 cell, int32 age}.
 * cell_ref[c] is the handle of cell c = y*width + x (device array). */
typedef struct smmo_life_args {
    const uint64_t* cell_ref;
    int32_t width, height;
    uint32_t cell_cls, agent_cls;
} smmo_life_args;

/* Predator-prey grid on a width x height torus.  Fish {int32 pos, int32 age},
 * Shark {int32 pos, int32 age, int32 energy}.  occ[c] is the handle on cell c
 * (0 = empty); claim[c] must be INT32_MAX before a plan phase and is restored
 * by the matching move phase; want[c] is scratch.  step is 1-based. */
typedef struct smmo_wator_args {
    uint64_t* occ;
    int32_t* claim;
    int32_t* want;
    uint64_t seed;
    int32_t width, height;
    int32_t step;
    int32_t fish_breed, shark_breed, eat_gain, shark_e0;
    uint32_t fish_cls, shark_cls;
    uint32_t pad;
} smmo_wator_args;

/* N-body with merging (the collision app of Sec. 1 and Table 1) on a class
 * Body {f32 x, f32 y, f32 vx, f32 vy, f32 m} created by one parallel_new, so
 * that ascending (block, slot) order is ascending creation index; the body's
 * key is block*64 + slot.  One step = INSERT, PAIRS, RESOLVE, REAP, FORCE,
 * MOVE, all with the same argument blob:
 *  INSERT   put each body into a hashed uniform grid (cell 1/inv_cell)
 *  PAIRS    list every pair closer than merge_dist (sqrtf of the squared
 *           distance, compared with <), lower key first
 *  RESOLVE  join the pairs into connected components; the lowest key keeps
 *           its position and gets m = sum m_k, v = (sum m_k v_k) / m, both
 *           summed in ascending key; every other member is marked merged
 *  REAP     merged bodies destroy themselves (Listing 1, step_6_delete_merged)
 *  FORCE    a_i = sum over live j != i in ascending key of
 *           s*(x_j - x_i, y_j - y_i), s = (G*m_j) / (d2*sqrtf(d2)),
 *           d2 = dx*dx + dy*dy (device_do over all bodies, Sec. 2.1); v += a*dt
 *  MOVE     x += v*dt
 * Scratch arrays are caller device memory: head[1 << hash_bits] (all -1 and
 * npairs 0 before the first step; every step leaves them so), next, lab and
 * merged with num_blocks*64 entries (merged all 0), pairs[2*pair_cap].  More
 * than pair_cap close pairs in one step sets SMMO_STATUS_CORRUPT. */
typedef struct smmo_nbody_args {
    int32_t* head;
    int32_t* next;
    int32_t* lab;
    uint8_t* merged;
    int32_t* pairs;
    uint32_t* npairs;
    uint32_t hash_bits;
    uint32_t pair_cap;
    float G, dt, merge_dist, inv_cell;
} smmo_nbody_args;

/* -------------------------------------------------------- operations ---- */

/* parallel_new<T>(n) (Sec. 2.1): create n objects of class `cls`; object i
 * gets constructor index i.  Placement: the lowest free blocks in ascending
 * order, filled densely (object i at block rank i / N_T, slot i mod N_T).
 * Sets SMMO_STATUS_OOM (and creates nothing) if too few blocks are free.
 * args: the constructor's blob (copied; <= SMMO_ARGS_MAX bytes). */
int smmo_parallel_new(smmo_heap* heap, uint32_t cls, uint64_t n, uint32_t ctor_id,
                      const void* args, uint64_t args_bytes, void* stream);

/* Device-side allocation from a kernel of `nthreads` threads, each calling
 * new(d_allocator) T `per_thread` times in sequence (Sec. 2.1 "new"; the
 * allocation microbenchmarks of Sec. 6.4).  Object of thread t, call k gets
 * constructor index t*per_thread + k.  Allocation uses Alg. 1 with request
 * coalescing per wavefront (Sec. 4.2). */
int smmo_parallel_alloc(smmo_heap* heap, uint32_t cls, uint64_t nthreads, uint32_t per_thread,
                        uint32_t ctor_id, const void* args, uint64_t args_bytes, void* stream);

/* Device-side destruction from a kernel of `nthreads` threads, thread t
 * calling destroy(refs[t*per_thread + k]) for k = 0..per_thread-1 in sequence
 * (Sec. 2.1 "destroy"; Alg. 2), the mirror of smmo_parallel_alloc.  refs is a
 * device array of nthreads*per_thread handles; 0 (null) entries are skipped.
 * Destructions of one wave that hit the same block are combined into one
 * atomic update.  Every non-null handle must name a live object and appear at
 * most once; this is not checked beyond flagging SMMO_STATUS_CORRUPT when a
 * slot is freed twice. */
int smmo_parallel_destroy(smmo_heap* heap, const uint64_t* refs, uint64_t nthreads, uint32_t per_thread,
                          void* stream);

/* parallel_do<T, method> (Sec. 2.1, Sec. 3.7): run `method_id` on every live
 * object of class `cls` and of its subclasses (transitively), one kernel per
 * class in ascending class id.  Objects the method creates, in any of these
 * classes, are not visited by the same call: with subclasses, the iteration
 * words of every class are taken before the first kernel.  A method destroys
 * no object of these classes other than the one it runs on.  The n-body
 * methods take a class without subclasses.  args: the method's blob
 * (<= SMMO_ARGS_MAX bytes). */
int smmo_parallel_do(smmo_heap* heap, uint32_t cls, uint32_t method_id, const void* args,
                     uint64_t args_bytes, void* stream);

/* The iteration snapshot of Sec. 3.1 on its own: for `cls` and its
 * subclasses, record the objects live now (each allocated block's iteration
 * word <- its allocation word).  With smmo_parallel_do_snapshot this splits a
 * do-all into "fix the objects to visit" and "visit them", so that another
 * do-all that creates objects of `cls` can run between the two, or at the
 * same time as the second on another stream, without its objects being
 * visited.  Asynchronous on `stream`. */
int smmo_snapshot(smmo_heap* heap, uint32_t cls, void* stream);

/* smmo_parallel_do over the objects recorded by the last smmo_snapshot of
 * `cls` (and its subclasses) instead of those live at launch; objects created
 * since the snapshot are not visited.  Between the snapshot and the end of
 * this call no recorded object may be destroyed except by this call's own
 * method (as in any do-all, on itself), and no snapshot of these classes may
 * be taken.  Every method that smmo_parallel_do runs through the generic
 * do-all is accepted; SMMO_M_AXPY and the n-body methods give SMMO_EINVAL.
 * Calls on one heap that run at the same time on different streams share
 * the heap's block-list buffer: at most one of them may build a block list
 * (do-alls of heaps with at least list_min_words level-0 words, smmo_launch),
 * so for concurrent do-alls on such heaps raise list_min_words or set
 * SMMO_TUNE_FLAT_ENUM. */
int smmo_parallel_do_snapshot(smmo_heap* heap, uint32_t cls, uint32_t method_id, const void* args,
                              uint64_t args_bytes, void* stream);

/* smmo_parallel_do for callers that cannot allocate device memory or have
 * no spare heap scratch (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the same do-all, but every block list it
 * builds (big heaps' level-1 enumeration, the ordered list of the n-body
 * force) and its counters live in one static device array of the library,
 * 4 MiB + 1 KiB, allocated with the code object (no hipMalloc, hipFree or
 * allocating library call).  Limit: heaps of at most 1,048,576 blocks
 * (SMMO_EINVAL above).  The array is per GPU and shared by every call on
 * that GPU and kept between calls: calls of this entry point that overlap on
 * one GPU (other streams, other threads) race and must not be issued; the
 * counters a call needs are cleared by its own kernels.  Otherwise as
 * smmo_parallel_do, whose calls it may follow or precede on the stream. */
int smmo_parallel_do_static_scratch(smmo_heap* heap, uint32_t cls, uint32_t method_id, const void* args,
                                    uint64_t args_bytes, void* stream);

/* Measurement hook: the method kernel of the NEXT call of smmo_parallel_do
 * or smmo_parallel_do_snapshot on this heap (its first method kernel when the
 * class has subclasses; the streaming kernel of SMMO_M_AXPY; the force kernel
 * of SMMO_M_NBODY_FORCE; not a snapshot or block-list pass) is dispatched with
 * hipExtLaunchKernelGGL so that `start_event` and `stop_event` (hipEvent_t
 * handles owned by the caller, created with timing enabled) record when the
 * kernel itself starts and ends; hipEventElapsedTime then gives its duration
 * without the queueing around it.  The request is consumed by that call
 * whatever it launches (a call that fails validation, or a method without a
 * timed kernel such as SMMO_M_NBODY_RESOLVE, records nothing), and every
 * other entry point taking this heap drops a pending request, so a request
 * never attaches to a later, unrelated kernel.  The events must stay valid
 * until that do-all call has returned; null events cancel a pending request.
 * A measurement aid; it changes no result. */
int smmo_time_next_doall(smmo_heap* heap, void* start_event, void* stop_event);

/* Live objects of class `cls`.  Synchronizes the stream. */
int smmo_live_count(smmo_heap* heap, uint32_t cls, uint64_t* out, void* stream);

/* Slot occupancy per class (Sec. 6.3, the fragmentation measure): for each
 * class c < ncls, used[c] = live objects, slots[c] = N_c times blocks[c],
 * blocks[c] = blocks allocated to c.  Fragmentation F = 1 - sum(used) /
 * sum(slots).  Host arrays of ncls entries.  Synchronizes the stream. */
int smmo_occupancy(smmo_heap* heap, uint64_t* used, uint64_t* slots, uint64_t* blocks, void* stream);

/* Copy every live object of `cls` to host SOA arrays (host_field_bufs[f] has
 * room for `cap` values of field f), in block order then slot order; *n_out
 * = number of live objects (copying stops at cap).  Synchronizes. */
int smmo_dump_objects(smmo_heap* heap, uint32_t cls, void* const* host_field_bufs, uint64_t cap,
                      uint64_t* n_out, void* stream);

/* Handles of every live object of `cls`, in the same order as
 * smmo_dump_objects, to host memory.  Synchronizes. */
int smmo_dump_refs(smmo_heap* heap, uint32_t cls, uint64_t* host_refs, uint64_t cap,
                   uint64_t* n_out, void* stream);

/* Bytes of the raw metadata region (header, status, block words, bitmaps). */
int smmo_raw_bytes(const smmo_heap* heap, uint64_t* out);

/* Copy the raw metadata region (smmo_raw_header first) to host_buf
 * (`bytes` >= smmo_raw_bytes).  Synchronizes. */
int smmo_dump_raw(smmo_heap* heap, void* host_buf, uint64_t bytes, void* stream);

/* Sticky SMMO_STATUS_* bits.  Synchronizes. */
int smmo_status(smmo_heap* heap, uint32_t* flags_out, void* stream);

/* Clear the status bits and the counters. */
int smmo_clear_status(smmo_heap* heap, void* stream);

/* Copy `n` (<= SMMO_CNT_NUM) device counters to host.  Synchronizes. */
int smmo_stats(smmo_heap* heap, uint64_t* out, uint32_t n, void* stream);

/* ---------------------------------------------------- arena and batch ---- */
/* An arena is a host-side range allocator over one caller device buffer
 * (256-B granules, first fit); it lets many heaps and their workload arrays
 * live in one allocation and be admitted and released at run time.  It never
 * touches device memory itself. */
typedef struct smmo_arena smmo_arena;
int smmo_arena_create(void* dev_mem, uint64_t bytes, smmo_arena** out);
int smmo_arena_destroy(smmo_arena* arena);
/* *dev_out = a 256-B aligned range of `bytes`; SMMO_ENOMEM_DEVICE if no
 * free range is large enough. */
int smmo_arena_alloc(smmo_arena* arena, uint64_t bytes, void** dev_out);
int smmo_arena_free(smmo_arena* arena, void* dev_ptr);
int smmo_arena_stats(const smmo_arena* arena, uint64_t* free_bytes, uint64_t* largest_free);

/* A batch advances many independent predator-prey instances (each its own
 * heap and grids, see smmo_wator_args) together: each instance gets a share
 * of the workgroups proportional to its grid (at most one wave per block of
 * its heap), in one of two forms (smmo_batch_set_mode):
 *  SMMO_BATCH_PHASED (default): one launch per phase of a step (fish plan,
 *    fish move, shark plan, shark move) for every instance at once; the
 *    kernel boundaries separate the phases.
 *  SMMO_BATCH_PERSISTENT: ONE persistent kernel launch per call for all the
 *    call's steps; an instance's four phases per step are separated by
 *    barriers among its own workgroups only (every workgroup resident).
 * Both give the same results.  The batch's device tables live in `arena`. */
#define SMMO_BATCH_PHASED 0u
#define SMMO_BATCH_PERSISTENT 1u
typedef struct smmo_batch smmo_batch;
int smmo_batch_create(smmo_arena* arena, uint32_t max_instances, smmo_batch** out);
int smmo_batch_destroy(smmo_batch* batch);     /* returns its tables to the arena */
/* Add an instance that runs `steps` more steps; args.step is ignored (the
 * batch counts steps from 1).  `heap` must outlive the instance.
 * Synchronizes the stream.  *slot_out identifies the instance. */
int smmo_batch_add_wator(smmo_batch* batch, smmo_heap* heap, const smmo_wator_args* args, uint32_t steps,
                         void* stream, uint32_t* slot_out);
int smmo_batch_remove(smmo_batch* batch, uint32_t slot);
/* Advance every instance by min(steps, its remaining steps).  Asynchronous,
 * no host synchronization and no memset.  If the instance set or grid changed
 * since the last call, the schedule is uploaded first, in stream order from
 * pinned staging (not under stream capture: capture with
 * smmo_batch_capture_graph, which uploads before it captures).  Calls on one
 * batch must use one stream at a time. */
int smmo_batch_step(smmo_batch* batch, uint32_t steps, void* stream);
/* Capture `launches` launch groups of `steps_per_launch` steps each (the
 * work of that many smmo_batch_step calls) into a HIP graph and
 * instantiate it: the alloc -> do-all -> dealloc step of every admitted
 * instance, replayed with one graph launch (Sec. 2.1's do-alls, batched).
 * `stream` must be a created stream (not the null stream); nothing runs during
 * the capture.  If the instance set or grid changed since the last step, the
 * schedule is uploaded first (synchronously, outside the capture).  The
 * captured kernels read the batch's tables at replay time, so a graph may be
 * replayed only while the batch keeps the instance set and grid it was
 * captured with: smmo_batch_graph_launch refuses it (SMMO_EINVAL) after
 * smmo_batch_add_wator, smmo_batch_remove, smmo_batch_set_grid or
 * smmo_batch_set_mode.  Each replay
 * advances every instance by min(launches * steps_per_launch, its remaining
 * steps).  The graph holds no device memory of its own besides what the HIP
 * runtime keeps for an instantiated graph; free it with
 * smmo_batch_graph_destroy before the batch. */
typedef struct smmo_batch_graph smmo_batch_graph;
int smmo_batch_capture_graph(smmo_batch* batch, uint32_t launches, uint32_t steps_per_launch, void* stream,
                             smmo_batch_graph** out);
/* Replay a captured graph on `stream` (asynchronous). */
int smmo_batch_graph_launch(smmo_batch_graph* graph, void* stream);
int smmo_batch_graph_destroy(smmo_batch_graph* graph);
/* Remaining steps of every slot (0xFFFFFFFF for an empty slot), to host
 * memory of max_instances entries.  Synchronizes. */
int smmo_batch_remaining(smmo_batch* batch, uint32_t* out, void* stream);
/* Workgroups of the batch's launches (the grid of the current mode). */
int smmo_batch_grid(const smmo_batch* batch, uint32_t* workgroups);
/* Use wg_per_cu workgroups per CU.  0 selects the mode's default: 16 for the
 * phased form (its kernels need no co-residency, so the grid may exceed what
 * is resident at once; at most 32), every workgroup that can be resident for
 * the persistent kernel (which is also its most).  Larger values are capped.
 * The schedule is rebuilt at the next step.  Results do not depend on it. */
int smmo_batch_set_grid(smmo_batch* batch, uint32_t wg_per_cu);
/* SMMO_BATCH_PHASED or SMMO_BATCH_PERSISTENT (SMMO_EINVAL otherwise); the
 * grid follows the mode's occupancy and the schedule is rebuilt at the next
 * step.  Results do not depend on it. */
int smmo_batch_set_mode(smmo_batch* batch, uint32_t mode);

/* ------------------------------------------------------ launch shape ---- */

/* Launch shape of a heap's kernels.  The paper leaves the do-all's thread
 * count to hand tuning (Sec. 3.7); here it is a per-heap setting that an
 * autotuner can search.  Results do not depend on it.  A zero field selects
 * the built-in default. */
typedef struct smmo_launch {
    uint32_t doall_waves_per_cu;   /* do-all grid cap in waves per CU: 1..64 (default 32) */
    uint32_t doall_units;          /* units of block bits a flat do-all is cut into, at most
                                      (64 bits per level-0 word) x 64: 64..2^20 (default 16384) */
    uint32_t list_min_words;       /* level-0 words from which a do-all enumerates through
                                      level 1 (block list): 1..2^32-1 (default 4096) */
    uint32_t sweep_waves_per_cu;   /* streaming sweep (SMMO_M_AXPY) grid in waves per CU:
                                      1..1024 (default 128) */
    uint32_t sweep_groups;         /* groups of four blocks in flight per sweep wave: 1, 2 or 4
                                      (default 4) */
} smmo_launch;

/* Set the launch shape (fields 0: defaults); out-of-range fields: SMMO_EINVAL
 * and nothing changes.  Host-side only; takes effect for later launches. */
int smmo_set_launch(smmo_heap* heap, const smmo_launch* launch);
/* The effective launch shape (defaults filled in). */
int smmo_get_launch(const smmo_heap* heap, smmo_launch* out);

/* ------------------------------------------------------- measurement ---- */

/* Atomic-throughput reference for the allocator (not part of the method):
 * nthreads device threads each perform `rounds` 64-bit atomic ORs (agent
 * scope, relaxed, value returned and consumed) on words[(t / lanes_per_word)
 * % nwords] — lanes_per_word 1: every lane its own word; 64: a whole
 * wavefront on one word, the pattern of an uncoalesced allocation.  `words`
 * is a device array of nwords uint64 (contents are overwritten).
 * lanes_per_word: 1..64.  Asynchronous on `stream`. */
int smmo_atomic_probe(uint64_t* words, uint64_t nwords, uint32_t lanes_per_word, uint64_t nthreads,
                      uint32_t rounds, void* stream);

/* VALU issue-cost reference for the n-body force kernel (not part of the
 * method): `workgroups` workgroups of 256 threads each run eight independent
 * chains of `iters` instructions of one kind per lane, all operands in
 * vector registers (kind 0: FP32 add, 1: FP32 multiply-add into the chain,
 * 2: hardware square root, 3: hardware reciprocal) and store one float per
 * thread into out (a device array of workgroups * 256 floats).
 * Time it with events: wave-instructions = workgroups * 4 * iters * 8.
 * kind > 3, workgroups 0 or a null out: SMMO_EINVAL.  Asynchronous. */
int smmo_valu_probe(float* out, uint32_t kind, uint32_t workgroups, uint32_t iters, void* stream);

/* Self-check of the arithmetic the n-body force kernel uses on its fast
 * path (device_do, Sec. 2.1: correctly rounded sqrt and division where
 * operands lie in ranges that need no scaling).  Adds to counts_dev[0] (a
 * device uint64[2], cleared first) the float bit patterns in
 * [lo_bits, hi_bits) whose fast square root differs from the correctly
 * rounded one, and to counts_dev[1] the quotients that differ among `pairs`
 * pseudo-random operand pairs from the fast ranges (seeded).  Both must be 0;
 * the tests run it over the whole range [2^-40, 2^40). Asynchronous. */
int smmo_check_force_arith(uint32_t lo_bits, uint32_t hi_bits, uint64_t pairs, uint64_t seed, uint64_t* counts_dev,
                           void* stream);

/* Message-passing check of the order the allocator relies on when a block is
 * re-initialized (Alg. 8, App. A.3): a reservation that sees a block's new
 * allocation word must read the block's new type.  Runs the allocator's own
 * block initialization and reservation code on a scratch block table:
 * writer waves re-initialize each of `blocks` blocks `rounds` times (round
 * k: type k, then the word k << 32), reader waves (on every XCD, the writers
 * on others) OR a bit into random blocks' words and then read their types;
 * a type older than the round the OR returned is a violation.  Every wave
 * runs a bounded number of iterations and waits for no other wave; readers
 * stop soon after the first violation.
 * dev_buf: device buffer of at least 20 * blocks bytes rounded up to a
 * multiple of 8, 8-byte aligned (overwritten).  counts_dev: device uint64[4], cleared first, then
 * [0] samples, [1] samples that saw a re-initialized word, [2] violations
 * (must be 0), [3] the first violation as block << 32 | type read.
 * blocks >= 1; 1 <= rounds < 2^31.  SMMO_EINVAL otherwise.  Asynchronous. */
int smmo_check_publish_order(void* dev_buf, uint64_t buf_bytes, uint32_t blocks, uint32_t rounds, uint64_t seed,
                             uint64_t* counts_dev, void* stream);

/* Handle layout: bits 56-63 class id + 1, bits 6-49 block, bits 0-5 slot;
 * 0 is the null handle.  Host-side helpers. */

uint64_t smmo_ref_make(uint32_t cls, uint64_t block, uint32_t slot);
uint32_t smmo_ref_class(uint64_t ref);
uint64_t smmo_ref_block(uint64_t ref);
uint32_t smmo_ref_slot(uint64_t ref);

const char* smmo_strerror(int code);
const char* smmo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SMMO_H */
