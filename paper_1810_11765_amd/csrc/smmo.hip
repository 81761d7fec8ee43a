// Host side of the SMMO heap C-ABI (include/smmo.h): heap layout, argument
// checking, kernel dispatch.  Every compute step runs in the kernels of
// kernels.h / methods.h; this file only lays out memory and launches them.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "batch.h"
#include "device_api.h"
#include "methods.h"
#include "methods_api.h"
#include "nbody.h"

#include <map>
#include <mutex>

using namespace smmo;

// Default launch shape (smmo_launch).  Sweep: 128 waves per CU (beyond the
// resident limit, workgroups wait for a slot) x 4 groups of four blocks in
// flight measured best on MI355X with non-temporal field access (one L0 word
// per wave at 2^21 blocks).
constexpr smmo_launch kDefaultLaunch = {32, 16384, 4096, 128, 4};

struct smmo_heap {
    smmo_raw_header hdr;   // host copy of the device header
    DevHeap dev;           // kernel-argument view
    uint8_t* base;         // caller's device buffer
    uint64_t bytes;
    smmo_launch launch;    // effective launch shape
    uint32_t cus;          // compute units of the device
    hipEvent_t time_start = nullptr, time_stop = nullptr;   // smmo_time_next_doall, pending
    hipEvent_t armed_start = nullptr, armed_stop = nullptr; // taken by the current do-all call
    uint8_t* stage = nullptr;   // scratch of the current call when not the heap's own (static-scratch calls)
    // The class whose block list the heap's scratch holds and is still
    // current (-1: none): a do-all whose method creates and destroys nothing
    // leaves every class's blocks as they were, so the next list of the same
    // class is the same list.  Every call that may change blocks, or write
    // the scratch list, resets it; a heap in a batch (changed by the batch
    // kernel behind the host's back) never caches.
    int32_t list_cls = -1;
    // The class whose iteration words equal its allocation words, recorded
    // in passing by the last do-all of a method that creates and destroys
    // nothing (-1: none); reset with list_cls by every call that may change
    // blocks.  A do-all that needs the class's snapshot then skips k_snapshot.
    int32_t snap_cls = -1;
    bool in_batch = false;
};

// a call that may change blocks (or write the scratch list): the cached block
// list and the recorded snapshot are no longer current
inline void blocks_changed(smmo_heap* H) {
    H->list_cls = -1;
    H->snap_cls = -1;
}

// Static device scratch of smmo_parallel_do_static_scratch (see below):
// counters (1 KiB), then up to kStaticListBlocks block ids.
constexpr uint64_t kStaticListBlocks = 1ull << 20;
constexpr uint64_t kStaticScratchBytes = 1024 + 4 * kStaticListBlocks;
static __device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

// A timing request (smmo_time_next_doall) belongs to the next do-all call on
// the heap: that call arms it for its method kernel, and every other entry
// point, or a do-all call that launches no timed kernel, drops it.
struct TimingScope {
    smmo_heap* H;
    explicit TimingScope(smmo_heap* h, bool take) : H(h) {
        if (!H) return;
        if (take) { H->armed_start = H->time_start; H->armed_stop = H->time_stop; }
        H->time_start = H->time_stop = nullptr;
    }
    ~TimingScope() { if (H) H->armed_start = H->armed_stop = nullptr; }
};

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(SMMO_EHIP, "%s: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

#define LAUNCH_CHECK(name)                                                            \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess) return fail(SMMO_EHIP, "%s launch: %s", name, hipGetErrorString(e_)); \
    } while (0)

inline uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }
constexpr uint64_t kScratchHead = 1024;                 // bytes of scratch counters
inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }
inline unsigned grid_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

// Layout of every class (Sec. 3.2): a class's fields are its superclass's
// (inherited, first) followed by its own; N_T = floor(B * size(T_s) /
// size(T)) with B = objects per block of the smallest class (the paper's 64,
// the width of a block's allocation word; fewer leaves the upper bits as
// padding); SOA arrays in field order, each starting on a 128-B boundary;
// every block has the size of the largest class layout.
int compute_layout(const smmo_class_desc* cls, uint32_t ncls, uint64_t M, smmo_raw_header* hdr,
                   uint32_t block_objects = 64) {
    if (!cls || ncls == 0 || ncls > SMMO_MAX_CLASSES) return fail(SMMO_EINVAL, "ncls must be 1..%d", SMMO_MAX_CLASSES);
    if (block_objects < 1 || block_objects > 64) return fail(SMMO_EINVAL, "block_objects must be 1..64");
    if (M == 0 || M > (1ull << 32)) return fail(SMMO_EINVAL, "num_blocks must be 1..2^32");
    std::memset(hdr, 0, sizeof *hdr);
    uint64_t size[SMMO_MAX_CLASSES];
    uint64_t smin = ~0ull;
    for (uint32_t t = 0; t < ncls; ++t) {
        const uint32_t sup = cls[t].superclass;
        if (sup > t) return fail(SMMO_EINVAL, "class %u: superclass must be a smaller class id", t);
        if (cls[t].nfields > SMMO_MAX_FIELDS || (cls[t].nfields && !cls[t].field_bytes))
            return fail(SMMO_EINVAL, "class %u: nfields must be 0..%d with a field array", t, SMMO_MAX_FIELDS);
        uint32_t nf = 0;
        if (sup) {                                         // inherited fields first
            nf = (uint32_t)hdr->nfields[sup - 1];
            for (uint32_t f = 0; f < nf; ++f) hdr->field_bytes[t][f] = hdr->field_bytes[sup - 1][f];
        }
        if (nf + cls[t].nfields == 0 || nf + cls[t].nfields > SMMO_MAX_FIELDS)
            return fail(SMMO_EINVAL, "class %u: 1..%d fields in all, inherited included", t, SMMO_MAX_FIELDS);
        for (uint32_t f = 0; f < cls[t].nfields; ++f) {
            uint32_t b = cls[t].field_bytes[f];
            if (b != 1 && b != 2 && b != 4 && b != 8)
                return fail(SMMO_EINVAL, "class %u field %u: size %u not 1/2/4/8", t, f, b);
            hdr->field_bytes[t][nf++] = b;
        }
        hdr->nfields[t] = nf;
        hdr->superclass[t] = sup;
        size[t] = 0;
        for (uint32_t f = 0; f < nf; ++f) size[t] += hdr->field_bytes[t][f];
        smin = std::min(smin, size[t]);
    }
    uint64_t block = 0;
    for (uint32_t t = 0; t < ncls; ++t) {
        uint64_t n = block_objects * smin / size[t];
        if (n < 1)
            return fail(SMMO_EINVAL, "class %u is more than %ux the smallest class", t, block_objects);
        hdr->capacity[t] = n;
        uint64_t off = 0;
        for (uint32_t f = 0; f < hdr->nfields[t]; ++f) {
            hdr->field_off[t][f] = (uint32_t)off;
            off += align_up(n * hdr->field_bytes[t][f], 128);
        }
        block = std::max(block, off);
    }
    hdr->magic = SMMO_MAGIC;
    hdr->version = 2;
    hdr->bitmap_stride = (uint32_t)kBmStride;
    hdr->num_blocks = M;
    hdr->ncls = ncls;
    hdr->block_bytes = block;
    // bitmap geometry: level 0 has one bit per block, each next level one bit
    // per word of the level below, up to a single top word
    uint64_t nbits = M, off = 0;
    uint32_t l = 0;
    for (;;) {
        if (l >= SMMO_MAX_LEVELS) return fail(SMMO_EINVAL, "too many blocks for %d bitmap levels", SMMO_MAX_LEVELS);
        uint64_t words = (nbits + 63) / 64;
        hdr->level_words[l] = words;
        hdr->level_off[l] = off;
        off += align_up(words, 8) * kBmStride;
        ++l;
        if (words == 1) break;
        nbits = words;
    }
    hdr->nlevels = l;
    hdr->bitmap_words = align_up(off, 32);
    // sections of the device buffer
    uint64_t p = 4096;                                     // header
    hdr->off_status = p;       p += 256;
    hdr->off_type = p;         p = align_up(p + 4 * M, 256);
    hdr->off_alloc = p;        p = align_up(p + 8 * M, 256);
    hdr->off_iter = p;         p = align_up(p + 8 * M, 256);
    hdr->off_bitmaps = p;      p = align_up(p + 8 * hdr->bitmap_words * (1 + 2 * (uint64_t)ncls), 256);
    hdr->off_scratch = p;
    // counters (1 KiB), then a block list R (4 B per block)
    hdr->scratch_bytes = align_up(kScratchHead + 4 * M, 256);
    p += hdr->scratch_bytes;
    hdr->off_data = align_up(p, 4096);
    hdr->total_bytes = hdr->off_data + M * block;
    hdr->tune_flags = 0;
    hdr->lookups = 5;                                      // Sec. 6.3: r = 5 by default
    hdr->force_fail_ppm = 0;
    return SMMO_OK;
}

void fill_dev(smmo_heap* H) {
    const smmo_raw_header& h = H->hdr;
    DevHeap& d = H->dev;
    std::memset(&d, 0, sizeof d);
    uint8_t* b = H->base;
    d.data = b + h.off_data;
    d.alloc = reinterpret_cast<uint64_t*>(b + h.off_alloc);
    d.iter = reinterpret_cast<uint64_t*>(b + h.off_iter);
    d.type = reinterpret_cast<uint32_t*>(b + h.off_type);
    d.bm = reinterpret_cast<uint64_t*>(b + h.off_bitmaps);
    d.status = reinterpret_cast<uint32_t*>(b + h.off_status);
    d.counters = reinterpret_cast<unsigned long long*>(b + h.off_status + 64);
    d.scratch = b + h.off_scratch;
    d.hdr = reinterpret_cast<const smmo_raw_header*>(b);
    d.M = h.num_blocks;
    d.block_bytes = h.block_bytes;
    d.bitmap_words = h.bitmap_words;
    for (int l = 0; l < SMMO_MAX_LEVELS; ++l) {
        d.level_off[l] = h.level_off[l];
        d.level_words[l] = h.level_words[l];
    }
    d.nlevels = (uint32_t)h.nlevels;
    d.ncls = (uint32_t)h.ncls;
    d.tune = h.tune_flags;
    d.lookups = h.lookups;
    d.force_fail_ppm = h.force_fail_ppm;
    for (uint32_t t = 0; t < h.ncls; ++t) {
        uint64_t n = h.capacity[t];
        d.cls_cap[t] = (uint32_t)n;
        d.cls_pad[t] = n >= 64 ? 0ull : (~0ull << n);
    }
}

int init_device(smmo_heap* H, hipStream_t s) {
    const smmo_raw_header& h = H->hdr;
    HIP_TRY(hipMemcpyAsync(H->base, &H->hdr, sizeof H->hdr, hipMemcpyHostToDevice, s));
    k_init_blocks<<<grid_for(h.num_blocks, 256), 256, 0, s>>>(H->dev);
    LAUNCH_CHECK("k_init_blocks");
    uint64_t nw = h.bitmap_words * (1 + 2 * h.ncls);
    k_init_bitmaps<<<grid_for(nw, 256), 256, 0, s>>>(H->dev, nw);
    LAUNCH_CHECK("k_init_bitmaps");
    HIP_TRY(hipStreamSynchronize(s));                      // the header copy reads host memory
    return SMMO_OK;
}

uint8_t* scratch_base(smmo_heap* H) { return H->stage ? H->stage : H->dev.scratch; }
unsigned long long* scratch_counter(smmo_heap* H, int i) {
    return reinterpret_cast<unsigned long long*>(scratch_base(H)) + i;
}
// scratch counters: 0 parallel_new's found, 1 live count, 2 n-body's found,
// 3 block-list length, 8.. occupancy (3 per class).  R is the block list of
// whichever call ran last on the heap's stream (calls on one heap are
// stream-ordered).
uint32_t* scratch_R(smmo_heap* H) { return reinterpret_cast<uint32_t*>(scratch_base(H) + kScratchHead); }

// ------------------------------------------------- static scratch ----
// `scratch` (top of the file) is the device memory
// smmo_parallel_do_static_scratch stages its block lists in instead of the
// heap's scratch region, laid out like it (kScratchHead bytes of counters,
// then the list).  Each GPU the library runs on holds one copy until the
// process ends; every call on a GPU shares it.
static_assert(kStaticScratchBytes == kScratchHead + 4 * kStaticListBlocks, "static scratch layout");

// The array's device address on the current GPU, taken once per device with
// hipGetSymbolAddress (in host code the array's name is not a device
// address).
std::mutex g_static_mu;
std::map<int, uint8_t*> g_static_ptr;
int static_scratch(uint8_t** out) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_static_mu);
    auto it = g_static_ptr.find(dev);
    if (it == g_static_ptr.end()) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SMMO_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        it = g_static_ptr.emplace(dev, static_cast<uint8_t*>(p)).first;
    }
    *out = it->second;
    return SMMO_OK;
}

// Routes a call's scratch to another buffer for its duration.
struct StageScope {
    smmo_heap* H;
    StageScope(smmo_heap* h, uint8_t* p) : H(h) { H->stage = p; }
    ~StageScope() { H->stage = nullptr; }
};

// Big heaps: list the blocks of allocated[cls] via level 1 into R, so that
// the passes after it cost the class's blocks, not the heap's size.
// Returns false (nothing launched) when the heap is scanned flat.
bool build_block_list(smmo_heap* H, uint32_t cls, hipStream_t s, int* rc) {
    *rc = SMMO_OK;
    if (H->hdr.nlevels < 2 || H->hdr.level_words[0] < H->launch.list_min_words || (H->dev.tune & SMMO_TUNE_FLAT_ENUM))
        return false;
    if (!H->stage && !H->in_batch && H->list_cls == (int32_t)cls) return true;   // still current
    unsigned long long* cnt = scratch_counter(H, 3);
    k_fill_u64<<<1, 64, 0, s>>>(cnt, 1, 0);
    if (hipGetLastError() != hipSuccess) { *rc = fail(SMMO_EHIP, "k_fill_u64 launch"); return false; }
    k_enum_blocks<<<grid_for(H->hdr.level_words[1], 4 * kEnumPerWave), 256, 0, s>>>(H->dev, bm_allocated(cls),
                                                                                    scratch_R(H), cnt);
    if (hipGetLastError() != hipSuccess) { *rc = fail(SMMO_EHIP, "k_enum_blocks launch"); return false; }
    H->list_cls = H->stage ? -1 : (int32_t)cls;
    return true;
}

// Methods that create and destroy no object (and do not write the scratch
// list): a do-all of one of them keeps the cached block list.
bool method_keeps_blocks(uint32_t method_id) {
    switch (method_id) {
        case SMMO_M_AXPY: case SMMO_M_AXPY_GENERIC: case SMMO_M_VISIT: case SMMO_M_LIFE_PLAN:
        case SMMO_M_WATOR_FISH_PLAN: case SMMO_M_WATOR_SHARK_PLAN: case SMMO_M_NBODY_INSERT:
        case SMMO_M_NBODY_PAIRS: case SMMO_M_NBODY_RESOLVE: case SMMO_M_NBODY_MOVE:
            return true;
        default:
            return false;
    }
}

// grid of the list-form thread-per-block passes: at most 32 waves per CU,
// grid-stride beyond
unsigned list_grid(const smmo_heap* H) {
    const uint64_t threads = std::min<uint64_t>(H->hdr.num_blocks, (uint64_t)H->cus * 32 * 64);
    return grid_for(threads, 256);
}

int check_heap_cls(const smmo_heap* H, uint32_t cls) {
    if (!H) return fail(SMMO_EINVAL, "null heap");
    if (cls >= H->hdr.ncls) return fail(SMMO_EINVAL, "class %u out of range (%llu classes)", cls,
                                        (unsigned long long)H->hdr.ncls);
    return SMMO_OK;
}

template <class A>
int unpack_args(A& a, const void* args, uint64_t bytes, const char* what) {
    std::memset(&a, 0, sizeof a);
    if (bytes == 0 && args == nullptr) return SMMO_OK;
    if (bytes != sizeof(A) || !args)
        return fail(SMMO_EINVAL, "%s: argument blob of %llu bytes, expected %zu", what,
                    (unsigned long long)bytes, sizeof(A));
    std::memcpy(&a, args, sizeof a);
    return SMMO_OK;
}

// units of 64 >> s_log2 block bits so that small heaps still spread over
// enough waves (launch.doall_units); big heaps get whole words per unit and
// a grid capped at launch.doall_waves_per_cu
void doall_geometry(const smmo_heap* H, uint32_t& s_log2, uint64_t& nunits, unsigned& grid) {
    const uint64_t W0 = H->hdr.level_words[0];
    const uint64_t target = H->launch.doall_units;
    s_log2 = 0;
    while (s_log2 < 6 && (W0 << s_log2) < target) ++s_log2;
    nunits = W0 << s_log2;
    const uint64_t waves = std::min<uint64_t>(nunits, (uint64_t)H->cus * H->launch.doall_waves_per_cu);
    grid = (unsigned)((waves + 3) / 4);
}

// `cls` and its subclasses, transitively, in ascending id (a superclass has
// a smaller id than its subclasses)
uint32_t subtree(const smmo_heap* H, uint32_t cls, uint32_t* out) {
    bool in[SMMO_MAX_CLASSES] = {};
    uint32_t n = 0;
    for (uint32_t t = cls; t < H->hdr.ncls; ++t) {
        const uint32_t sup = H->hdr.superclass[t];
        in[t] = t == cls || (sup && in[sup - 1]);
        if (in[t]) out[n++] = t;
    }
    return n;
}

// One do-all kernel on one class; with snap_here, the class's snapshot first
// (unless a do-all recorded it since the class's blocks last changed); with
// kRecord, the kernel records it.
template <class M, bool kSnap, bool kRecord = false>
int launch_doall_one(smmo_heap* H, uint32_t cls, const typename M::Args& a, bool snap_here, hipStream_t s) {
    int rc = SMMO_OK;
    const bool list = build_block_list(H, cls, s, &rc);
    if (rc) return rc;
    const uint32_t* R = list ? scratch_R(H) : nullptr;
    const unsigned long long* nR = list ? scratch_counter(H, 3) : nullptr;
    if (snap_here && !(H->snap_cls == (int32_t)cls && !H->in_batch)) {
        if (list) k_snapshot<<<list_grid(H), 256, 0, s>>>(H->dev, cls, R, nR);
        else k_snapshot<<<grid_for(H->hdr.num_blocks, 256), 256, 0, s>>>(H->dev, cls, nullptr, nullptr);
        LAUNCH_CHECK("k_snapshot");
    }
    uint32_t s_log2;
    uint64_t nunits;
    unsigned grid;
    doall_geometry(H, s_log2, nunits, grid);
    if (list) {
        // the list length is known on the device only: the kernel sizes its
        // runs to at most 16,384 of them; the grid covers that many waves or
        // one per listed block, whichever is less, at most 32 waves per CU
        nunits = 0;
        grid = (unsigned)((std::min<uint64_t>(std::min<uint64_t>(H->hdr.num_blocks, 16384),
                                              (uint64_t)H->cus * H->launch.doall_waves_per_cu) + 3) / 4);
    }
    if (H->armed_start || H->armed_stop) {
        // the kernel's own start and end, recorded by the dispatch itself
        hipExtLaunchKernelGGL((k_doall<M, kSnap, kRecord>), dim3(grid), dim3(kBlockThreads), 0, s, H->armed_start,
                              H->armed_stop, 0, H->dev, cls, s_log2, nunits, R, nR, a);
        H->armed_start = H->armed_stop = nullptr;
    } else {
        k_doall<M, kSnap, kRecord><<<grid, kBlockThreads, 0, s>>>(H->dev, cls, s_log2, nunits, R, nR, a);
    }
    LAUNCH_CHECK("k_doall");
    if (kRecord) H->snap_cls = (int32_t)cls;
    return SMMO_OK;
}

int snapshot_class(smmo_heap* H, uint32_t cls, hipStream_t s) {
    int rc = SMMO_OK;
    const bool list = build_block_list(H, cls, s, &rc);
    if (rc) return rc;
    if (list) k_snapshot<<<list_grid(H), 256, 0, s>>>(H->dev, cls, scratch_R(H), scratch_counter(H, 3));
    else k_snapshot<<<grid_for(H->hdr.num_blocks, 256), 256, 0, s>>>(H->dev, cls, nullptr, nullptr);
    LAUNCH_CHECK("k_snapshot");
    return SMMO_OK;
}

template <class M>
int launch_doall(smmo_heap* H, uint32_t cls, const void* args, uint64_t bytes, hipStream_t s,
                 bool from_snapshot = false) {
    typename M::Args a;
    int rc = unpack_args(a, args, bytes, "parallel_do");
    if (rc) return rc;
    uint32_t cl[SMMO_MAX_CLASSES];
    const uint32_t n = subtree(H, cls, cl);
    if (from_snapshot) {                  // the iteration words of an earlier smmo_snapshot
        for (uint32_t i = 0; i < n; ++i)
            if ((rc = launch_doall_one<M, true>(H, cl[i], a, false, s))) return rc;
        return SMMO_OK;
    }
    if (n == 1) return launch_doall_one<M, M::kSnapshot, RecordsSnapshot<M>::value>(H, cls, a, M::kSnapshot, s);
    // class and subclasses (Sec. 2.1): one kernel per class, every class's
    // iteration words taken before the first, so no kernel visits objects an
    // earlier one created
    for (uint32_t i = 0; i < n; ++i)
        if ((rc = snapshot_class(H, cl[i], s))) return rc;
    for (uint32_t i = 0; i < n; ++i)
        if ((rc = launch_doall_one<M, true>(H, cl[i], a, false, s))) return rc;
    return SMMO_OK;
}

int check_nbody(const smmo_heap* H, uint32_t cls, const smmo_nbody_args& a) {
    if (H->hdr.nfields[cls] != 5) return fail(SMMO_EINVAL, "n-body: class needs 5 float32 fields");
    for (int f = 0; f < 5; ++f)
        if (H->hdr.field_bytes[cls][f] != 4) return fail(SMMO_EINVAL, "n-body: class needs 5 float32 fields");
    if (H->hdr.num_blocks * 64 > (uint64_t)INT32_MAX) return fail(SMMO_EINVAL, "n-body: keys exceed int32");
    if (!a.head || !a.next || !a.lab || !a.merged || !a.pairs || !a.npairs)
        return fail(SMMO_EINVAL, "n-body: null scratch array");
    if (a.hash_bits < 1 || a.hash_bits > 30) return fail(SMMO_EINVAL, "n-body: hash_bits must be 1..30");
    if (!(a.inv_cell > 0.0f) || !(a.merge_dist * a.inv_cell <= 1.0f))
        return fail(SMMO_EINVAL, "n-body: grid cell must be at least merge_dist");
    return SMMO_OK;
}

int launch_nbody(smmo_heap* H, uint32_t cls, uint32_t method, const void* args, uint64_t bytes, hipStream_t s) {
    smmo_nbody_args a;
    int rc = unpack_args(a, args, bytes, "n-body");
    if (rc) return rc;
    uint32_t cl[SMMO_MAX_CLASSES];
    if (subtree(H, cls, cl) != 1) return fail(SMMO_EINVAL, "n-body methods take a class without subclasses");
    rc = check_nbody(H, cls, a);
    if (rc) return rc;
    switch (method) {
        case SMMO_M_NBODY_INSERT: return launch_doall<MNbInsert>(H, cls, args, bytes, s);
        case SMMO_M_NBODY_PAIRS: return launch_doall<MNbPairs>(H, cls, args, bytes, s);
        case SMMO_M_NBODY_REAP: return launch_doall<MNbReap>(H, cls, args, bytes, s);
        case SMMO_M_NBODY_MOVE: return launch_doall<MNbMove>(H, cls, args, bytes, s);
        case SMMO_M_NBODY_RESOLVE:
            k_nbody_resolve<<<1, 1024, 0, s>>>(H->dev, cls, a);
            LAUNCH_CHECK("k_nbody_resolve");
            return SMMO_OK;
        case SMMO_M_NBODY_FORCE:
            k_enum<<<1, 1024, 0, s>>>(H->dev, bm_allocated(cls), H->hdr.num_blocks, scratch_R(H),
                                       scratch_counter(H, 2));
            LAUNCH_CHECK("k_enum");
            hipExtLaunchKernelGGL(k_nbody_force, dim3(grid_for(H->hdr.num_blocks, 4)), dim3(256), 0, s,
                                  H->armed_start, H->armed_stop, 0, H->dev, cls, scratch_R(H), scratch_counter(H, 2), a);
            H->armed_start = H->armed_stop = nullptr;
            LAUNCH_CHECK("k_nbody_force");
            return SMMO_OK;
        default: return fail(SMMO_EINVAL, "unknown n-body method %u", method);
    }
}

template <class C>
int launch_new(smmo_heap* H, uint32_t cls, uint64_t n, const void* args, uint64_t bytes, hipStream_t s) {
    typename C::Args a;
    int rc = unpack_args(a, args, bytes, "parallel_new");
    if (rc) return rc;
    const uint64_t N = H->hdr.capacity[cls];
    const uint64_t nb = (n + N - 1) / N;
    if (nb > H->hdr.num_blocks) return fail(SMMO_EINVAL, "parallel_new: %llu objects need %llu blocks, heap has %llu",
                                            (unsigned long long)n, (unsigned long long)nb,
                                            (unsigned long long)H->hdr.num_blocks);
    k_enum<<<1, 1024, 0, s>>>(H->dev, bm_free(), nb, scratch_R(H), scratch_counter(H, 0));
    LAUNCH_CHECK("k_enum");
    k_new_fill<C><<<grid_for(nb * 64, kBlockThreads), kBlockThreads, 0, s>>>(H->dev, cls, n, scratch_R(H),
                                                                              scratch_counter(H, 0), a);
    LAUNCH_CHECK("k_new_fill");
    return SMMO_OK;
}

template <class C>
int launch_alloc(smmo_heap* H, uint32_t cls, uint64_t nthreads, uint32_t per, const void* args, uint64_t bytes,
                 hipStream_t s) {
    typename C::Args a;
    int rc = unpack_args(a, args, bytes, "parallel_alloc");
    if (rc) return rc;
    k_alloc<C><<<grid_for(nthreads, kBlockThreads), kBlockThreads, 0, s>>>(H->dev, cls, nthreads, per, a);
    LAUNCH_CHECK("k_alloc");
    return SMMO_OK;
}

}  // namespace

extern "C" {

int smmo_heap_bytes(const smmo_class_desc* cls, uint32_t ncls, uint64_t num_blocks, uint64_t* bytes_out) {
    return smmo_heap_bytes_ex(cls, ncls, num_blocks, 64, bytes_out);
}

int smmo_heap_bytes_ex(const smmo_class_desc* cls, uint32_t ncls, uint64_t num_blocks, uint32_t block_objects,
                       uint64_t* bytes_out) {
    smmo_raw_header h;
    int rc = compute_layout(cls, ncls, num_blocks, &h, block_objects);
    if (rc) return rc;
    if (!bytes_out) return fail(SMMO_EINVAL, "null bytes_out");
    *bytes_out = h.total_bytes;
    return SMMO_OK;
}

int smmo_heap_create(const smmo_class_desc* cls, uint32_t ncls, uint64_t num_blocks, void* dev_mem,
                     uint64_t dev_bytes, void* stream, smmo_heap** out) {
    return smmo_heap_create_ex(cls, ncls, num_blocks, 64, dev_mem, dev_bytes, stream, out);
}

int smmo_heap_create_ex(const smmo_class_desc* cls, uint32_t ncls, uint64_t num_blocks, uint32_t block_objects,
                        void* dev_mem, uint64_t dev_bytes, void* stream, smmo_heap** out) {
    if (!out || !dev_mem) return fail(SMMO_EINVAL, "null out or dev_mem");
    if (reinterpret_cast<uintptr_t>(dev_mem) % 256) return fail(SMMO_EINVAL, "dev_mem must be 256-B aligned");
    smmo_heap* H = new smmo_heap();
    int rc = compute_layout(cls, ncls, num_blocks, &H->hdr, block_objects);
    if (rc) { delete H; return rc; }
    if (dev_bytes < H->hdr.total_bytes) {
        unsigned long long need = H->hdr.total_bytes;
        delete H;
        return fail(SMMO_ETOOSMALL, "dev_bytes %llu < required %llu", (unsigned long long)dev_bytes, need);
    }
    H->base = static_cast<uint8_t*>(dev_mem);
    H->bytes = dev_bytes;
    H->launch = kDefaultLaunch;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
            delete H;
            return fail(SMMO_EHIP, "cannot query the device's compute units");
        }
        H->cus = (uint32_t)cus;
    }
    fill_dev(H);
    rc = init_device(H, S(stream));
    if (rc) { delete H; return rc; }
    *out = H;
    return SMMO_OK;
}

int smmo_set_launch(smmo_heap* heap, const smmo_launch* l) {
    if (!heap || !l) return fail(SMMO_EINVAL, "null argument");
    smmo_launch v = *l;
    if (!v.doall_waves_per_cu) v.doall_waves_per_cu = kDefaultLaunch.doall_waves_per_cu;
    if (!v.doall_units) v.doall_units = kDefaultLaunch.doall_units;
    if (!v.list_min_words) v.list_min_words = kDefaultLaunch.list_min_words;
    if (!v.sweep_waves_per_cu) v.sweep_waves_per_cu = kDefaultLaunch.sweep_waves_per_cu;
    if (!v.sweep_groups) v.sweep_groups = kDefaultLaunch.sweep_groups;
    if (v.doall_waves_per_cu > 64) return fail(SMMO_EINVAL, "doall_waves_per_cu must be 1..64");
    if (v.doall_units < 64 || v.doall_units > (1u << 20)) return fail(SMMO_EINVAL, "doall_units must be 64..2^20");
    if (v.sweep_waves_per_cu > 1024) return fail(SMMO_EINVAL, "sweep_waves_per_cu must be 1..1024");
    if (v.sweep_groups != 1 && v.sweep_groups != 2 && v.sweep_groups != 4)
        return fail(SMMO_EINVAL, "sweep_groups must be 1, 2 or 4");
    heap->launch = v;
    return SMMO_OK;
}

int smmo_get_launch(const smmo_heap* heap, smmo_launch* out) {
    if (!heap || !out) return fail(SMMO_EINVAL, "null argument");
    *out = heap->launch;
    return SMMO_OK;
}

int smmo_heap_destroy(smmo_heap* heap) {
    delete heap;
    return SMMO_OK;
}

int smmo_heap_reset(smmo_heap* heap, void* stream) {
    TimingScope timing(heap, false);
    if (heap) blocks_changed(heap);
    if (!heap) return fail(SMMO_EINVAL, "null heap");
    return init_device(heap, S(stream));
}

int smmo_class_layout(const smmo_heap* heap, uint32_t cls, smmo_layout* out) {
    int rc = check_heap_cls(heap, cls);
    if (rc) return rc;
    if (!out) return fail(SMMO_EINVAL, "null out");
    std::memset(out, 0, sizeof *out);
    out->capacity = (uint32_t)heap->hdr.capacity[cls];
    out->nfields = (uint32_t)heap->hdr.nfields[cls];
    out->block_bytes = heap->hdr.block_bytes;
    for (uint32_t f = 0; f < out->nfields; ++f) {
        out->field_bytes[f] = heap->hdr.field_bytes[cls][f];
        out->field_offset[f] = heap->hdr.field_off[cls][f];
    }
    return SMMO_OK;
}

int smmo_layout_compute(const smmo_class_desc* cls, uint32_t ncls, uint32_t which, smmo_layout* out) {
    return smmo_layout_compute_ex(cls, ncls, 64, which, out);
}

int smmo_layout_compute_ex(const smmo_class_desc* cls, uint32_t ncls, uint32_t block_objects, uint32_t which,
                           smmo_layout* out) {
    smmo_heap tmp;
    int rc = compute_layout(cls, ncls, 1, &tmp.hdr, block_objects);
    if (rc) return rc;
    return smmo_class_layout(&tmp, which, out);
}

int smmo_set_tuning(smmo_heap* heap, uint32_t flags, uint32_t lookups, uint32_t force_fail_ppm, void* stream) {
    TimingScope timing(heap, false);
    if (!heap) return fail(SMMO_EINVAL, "null heap");
    if (lookups < 1 || lookups > 64) return fail(SMMO_EINVAL, "lookups must be 1..64");
    if (force_fail_ppm > 1000000) return fail(SMMO_EINVAL, "force_fail_ppm must be <= 1e6");
    heap->hdr.tune_flags = flags;
    heap->hdr.lookups = lookups;
    heap->hdr.force_fail_ppm = force_fail_ppm;
    heap->dev.tune = flags;
    heap->dev.lookups = lookups;
    heap->dev.force_fail_ppm = force_fail_ppm;
    // keep the device header (dumped by smmo_dump_raw) in step
    const size_t off = offsetof(smmo_raw_header, tune_flags);
    HIP_TRY(hipMemcpyAsync(heap->base + off, reinterpret_cast<uint8_t*>(&heap->hdr) + off, 12,
                           hipMemcpyHostToDevice, S(stream)));
    HIP_TRY(hipStreamSynchronize(S(stream)));
    return SMMO_OK;
}

int smmo_parallel_new(smmo_heap* heap, uint32_t cls, uint64_t n, uint32_t ctor_id, const void* args,
                      uint64_t args_bytes, void* stream) {
    TimingScope timing(heap, false);
    if (heap) blocks_changed(heap);
    int rc = check_heap_cls(heap, cls);
    if (rc) return rc;
    if (n == 0) return SMMO_OK;
    switch (ctor_id) {
        case SMMO_CTOR_ZERO: return launch_new<CtorZero>(heap, cls, n, args, args_bytes, S(stream));
        case SMMO_CTOR_ARRAYS: return launch_new<CtorArrays>(heap, cls, n, args, args_bytes, S(stream));
        case SMMO_CTOR_NONE: return launch_new<CtorNone>(heap, cls, n, args, args_bytes, S(stream));
        default: return fail(SMMO_EINVAL, "unknown ctor_id %u", ctor_id);
    }
}

int smmo_parallel_alloc(smmo_heap* heap, uint32_t cls, uint64_t nthreads, uint32_t per_thread, uint32_t ctor_id,
                        const void* args, uint64_t args_bytes, void* stream) {
    TimingScope timing(heap, false);
    if (heap) blocks_changed(heap);
    int rc = check_heap_cls(heap, cls);
    if (rc) return rc;
    if (nthreads == 0 || per_thread == 0) return SMMO_OK;
    switch (ctor_id) {
        case SMMO_CTOR_ZERO:
            return launch_alloc<CtorZero>(heap, cls, nthreads, per_thread, args, args_bytes, S(stream));
        case SMMO_CTOR_ARRAYS:
            return launch_alloc<CtorArrays>(heap, cls, nthreads, per_thread, args, args_bytes, S(stream));
        case SMMO_CTOR_NONE:
            return launch_alloc<CtorNone>(heap, cls, nthreads, per_thread, args, args_bytes, S(stream));
        default: return fail(SMMO_EINVAL, "unknown ctor_id %u", ctor_id);
    }
}

int smmo_parallel_destroy(smmo_heap* heap, const uint64_t* refs, uint64_t nthreads, uint32_t per_thread,
                          void* stream) {
    TimingScope timing(heap, false);
    if (heap) blocks_changed(heap);
    if (!heap) return fail(SMMO_EINVAL, "null heap");
    if (nthreads == 0 || per_thread == 0) return SMMO_OK;
    if (!refs) return fail(SMMO_EINVAL, "null refs");
    if (nthreads > (1ull << 40)) return fail(SMMO_EINVAL, "nthreads too large");
    k_destroy<<<grid_for(nthreads, kBlockThreads), kBlockThreads, 0, S(stream)>>>(heap->dev, refs, nthreads,
                                                                                 per_thread);
    LAUNCH_CHECK("k_destroy");
    return SMMO_OK;
}

static int parallel_do(smmo_heap* heap, uint32_t cls, uint32_t method_id, const void* args, uint64_t args_bytes,
                       void* stream, bool from_snapshot) {
    TimingScope timing(heap, true);
    int rc = check_heap_cls(heap, cls);
    if (rc) return rc;
    hipStream_t s = S(stream);
    if (from_snapshot && (method_id == SMMO_M_AXPY || (method_id >= SMMO_M_NBODY_INSERT && method_id <= SMMO_M_NBODY_MOVE)))
        return fail(SMMO_EINVAL, "method %u has no snapshot form", method_id);
    switch (method_id) {
        case SMMO_M_AXPY: {
            smmo_axpy_args a;
            rc = unpack_args(a, args, args_bytes, "axpy");
            if (rc) return rc;
            if (a.fx >= heap->hdr.nfields[cls] || a.fy >= heap->hdr.nfields[cls] ||
                heap->hdr.field_bytes[cls][a.fx] != 4 || heap->hdr.field_bytes[cls][a.fy] != 4)
                return fail(SMMO_EINVAL, "axpy: fields must be 4-byte fields of the class");
            // creates and destroys nothing: one streaming kernel per class
            uint32_t cl[SMMO_MAX_CLASSES];
            const uint32_t n = subtree(heap, cls, cl);
            const uint64_t nwords = heap->hdr.level_words[0];
            const uint64_t waves = std::min<uint64_t>(nwords, (uint64_t)heap->cus * heap->launch.sweep_waves_per_cu);
            const unsigned grid = (unsigned)((waves + 3) / 4);
            for (uint32_t i = 0; i < n; ++i) {
                hipEvent_t e0 = heap->armed_start, e1 = heap->armed_stop;
                heap->armed_start = heap->armed_stop = nullptr;
                switch (heap->launch.sweep_groups) {
                    case 1: hipExtLaunchKernelGGL((k_doall_axpy<1>), dim3(grid), dim3(kBlockThreads), 0, s, e0, e1, 0,
                                                  heap->dev, cl[i], nwords, a); break;
                    case 2: hipExtLaunchKernelGGL((k_doall_axpy<2>), dim3(grid), dim3(kBlockThreads), 0, s, e0, e1, 0,
                                                  heap->dev, cl[i], nwords, a); break;
                    default: hipExtLaunchKernelGGL((k_doall_axpy<4>), dim3(grid), dim3(kBlockThreads), 0, s, e0, e1, 0,
                                                   heap->dev, cl[i], nwords, a); break;
                }
                LAUNCH_CHECK("k_doall_axpy");
            }
            return SMMO_OK;
        }
        case SMMO_M_AXPY_GENERIC: {
            smmo_axpy_args a;
            rc = unpack_args(a, args, args_bytes, "axpy");
            if (rc) return rc;
            if (a.fx >= heap->hdr.nfields[cls] || a.fy >= heap->hdr.nfields[cls] ||
                heap->hdr.field_bytes[cls][a.fx] != 4 || heap->hdr.field_bytes[cls][a.fy] != 4)
                return fail(SMMO_EINVAL, "axpy: fields must be 4-byte fields of the class");
            return launch_doall<MAxpy>(heap, cls, args, args_bytes, s, from_snapshot);
        }
        case SMMO_M_DESTROY_ALL: return launch_doall<MDestroyAll>(heap, cls, nullptr, 0, s, from_snapshot);
        case SMMO_M_SPAWN: {
            smmo_spawn_args a;
            rc = unpack_args(a, args, args_bytes, "spawn");
            if (rc) return rc;
            uint32_t cl[SMMO_MAX_CLASSES];
            const uint32_t n = subtree(heap, cls, cl);
            bool other = a.cls < heap->hdr.ncls;
            for (uint32_t i = 0; i < n; ++i) other = other && a.cls != cl[i];
            if (!other || a.lanes < 1 || a.lanes > 64)
                return fail(SMMO_EINVAL, "spawn: a class outside the do-all's, lanes 1..64");
            return launch_doall<MSpawn>(heap, cls, args, args_bytes, s, from_snapshot);
        }
        case SMMO_M_VISIT: return launch_doall<MVisit>(heap, cls, args, args_bytes, s, from_snapshot);
        case SMMO_M_CHURN: return launch_doall<MChurn>(heap, cls, args, args_bytes, s, from_snapshot);
        case SMMO_M_CHURN_API: {
            if (heap->hdr.nfields[cls] != 3 || heap->hdr.field_bytes[cls][0] != 4 || heap->hdr.field_bytes[cls][1] != 4 ||
                heap->hdr.field_bytes[cls][2] != 4)
                return fail(SMMO_EINVAL, "churn (device API): class needs fields {int32, float32, float32}");
            return launch_doall<MChurnApi>(heap, cls, args, args_bytes, s, from_snapshot);
        }
        case SMMO_M_MIX: {
            smmo_mix_args a;
            rc = unpack_args(a, args, args_bytes, "mix");
            if (rc) return rc;
            if (a.cls_a >= heap->hdr.ncls || a.cls_b >= heap->hdr.ncls || heap->hdr.field_bytes[a.cls_a][0] != 4 ||
                heap->hdr.field_bytes[a.cls_b][0] != 4 || heap->hdr.field_bytes[cls][0] != 4)
                return fail(SMMO_EINVAL, "mix: classes need an int32 field 0");
            return launch_doall<MMix>(heap, cls, args, args_bytes, s, from_snapshot);
        }
        case SMMO_M_STRESS: {
            smmo_stress_args a;
            rc = unpack_args(a, args, args_bytes, "stress");
            if (rc) return rc;
            uint32_t cl[SMMO_MAX_CLASSES];
            const uint32_t n = subtree(heap, cls, cl);
            bool other = a.cls_a < heap->hdr.ncls && a.cls_b < heap->hdr.ncls;
            for (uint32_t i = 0; i < n; ++i) other = other && a.cls_a != cl[i] && a.cls_b != cl[i];
            if (!other || heap->hdr.field_bytes[a.cls_a][0] != 4 || heap->hdr.field_bytes[a.cls_b][0] != 4 ||
                a.lanes > 64)
                return fail(SMMO_EINVAL, "stress: two classes outside the do-all's with an int32 field 0, lanes <= 64");
            return launch_doall<MStress>(heap, cls, args, args_bytes, s, from_snapshot);
        }
        case SMMO_M_LIFE_PLAN: return launch_doall<MLifePlan>(heap, cls, args, args_bytes, s, from_snapshot);
        case SMMO_M_LIFE_AGENT: return launch_doall<MLifeAgent>(heap, cls, args, args_bytes, s, from_snapshot);
        case SMMO_M_LIFE_COMMIT: return launch_doall<MLifeCommit>(heap, cls, args, args_bytes, s, from_snapshot);
        case SMMO_M_WATOR_FISH_PLAN: return launch_doall<MFishPlan>(heap, cls, args, args_bytes, s, from_snapshot);
        case SMMO_M_WATOR_FISH_MOVE: return launch_doall<MFishMove>(heap, cls, args, args_bytes, s, from_snapshot);
        case SMMO_M_WATOR_SHARK_PLAN: return launch_doall<MSharkPlan>(heap, cls, args, args_bytes, s, from_snapshot);
        case SMMO_M_WATOR_SHARK_MOVE: return launch_doall<MSharkMove>(heap, cls, args, args_bytes, s, from_snapshot);
        case SMMO_M_NBODY_INSERT:
        case SMMO_M_NBODY_PAIRS:
        case SMMO_M_NBODY_RESOLVE:
        case SMMO_M_NBODY_REAP:
        case SMMO_M_NBODY_FORCE:
        case SMMO_M_NBODY_MOVE: return launch_nbody(heap, cls, method_id, args, args_bytes, s);
        default: return fail(SMMO_EINVAL, "unknown method_id %u", method_id);
    }
}

// a do-all call, then the block-list cache kept or dropped by its method
static int parallel_do_call(smmo_heap* heap, uint32_t cls, uint32_t method_id, const void* args,
                            uint64_t args_bytes, void* stream, bool from_snapshot) {
    const int rc = parallel_do(heap, cls, method_id, args, args_bytes, stream, from_snapshot);
    if (heap && !method_keeps_blocks(method_id)) blocks_changed(heap);
    return rc;
}

int smmo_parallel_do(smmo_heap* heap, uint32_t cls, uint32_t method_id, const void* args, uint64_t args_bytes,
                     void* stream) {
    return parallel_do_call(heap, cls, method_id, args, args_bytes, stream, false);
}

int smmo_parallel_do_snapshot(smmo_heap* heap, uint32_t cls, uint32_t method_id, const void* args,
                              uint64_t args_bytes, void* stream) {
    return parallel_do_call(heap, cls, method_id, args, args_bytes, stream, true);
}

int smmo_parallel_do_static_scratch(smmo_heap* heap, uint32_t cls, uint32_t method_id, const void* args,
                                    uint64_t args_bytes, void* stream) {
    if (!heap) return fail(SMMO_EINVAL, "null heap");
    if (heap->hdr.num_blocks > kStaticListBlocks)
        return fail(SMMO_EINVAL, "parallel_do_static_scratch: %llu blocks, the static scratch lists at most %llu",
                    (unsigned long long)heap->hdr.num_blocks, (unsigned long long)kStaticListBlocks);
    uint8_t* p = nullptr;
    int rc = static_scratch(&p);
    if (rc) return rc;
    StageScope stage(heap, p);
    return parallel_do_call(heap, cls, method_id, args, args_bytes, stream, false);
}

int smmo_time_next_doall(smmo_heap* heap, void* start_event, void* stop_event) {
    if (!heap) return fail(SMMO_EINVAL, "null heap");
    heap->time_start = static_cast<hipEvent_t>(start_event);
    heap->time_stop = static_cast<hipEvent_t>(stop_event);
    return SMMO_OK;
}

int smmo_snapshot(smmo_heap* heap, uint32_t cls, void* stream) {
    TimingScope timing(heap, false);
    int rc = check_heap_cls(heap, cls);
    if (rc) return rc;
    uint32_t cl[SMMO_MAX_CLASSES];
    const uint32_t n = subtree(heap, cls, cl);
    for (uint32_t i = 0; i < n; ++i)
        if ((rc = snapshot_class(heap, cl[i], S(stream)))) return rc;
    return SMMO_OK;
}

int smmo_live_count(smmo_heap* heap, uint32_t cls, uint64_t* out, void* stream) {
    TimingScope timing(heap, false);
    int rc = check_heap_cls(heap, cls);
    if (rc) return rc;
    if (!out) return fail(SMMO_EINVAL, "null out");
    hipStream_t s = S(stream);
    unsigned long long* c = scratch_counter(heap, 1);
    k_fill_u64<<<1, 64, 0, s>>>(c, 1, 0);
    LAUNCH_CHECK("k_fill_u64");
    const bool list = build_block_list(heap, cls, s, &rc);
    if (rc) return rc;
    if (list)
        k_live_count<<<list_grid(heap), 256, 0, s>>>(heap->dev, cls, scratch_R(heap), scratch_counter(heap, 3), c);
    else
        k_live_count<<<grid_for(heap->hdr.num_blocks, 256), 256, 0, s>>>(heap->dev, cls, nullptr, nullptr, c);
    LAUNCH_CHECK("k_live_count");
    unsigned long long v = 0;
    HIP_TRY(hipMemcpyAsync(&v, c, sizeof v, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *out = v;
    return SMMO_OK;
}

int smmo_atomic_probe(uint64_t* words, uint64_t nwords, uint32_t lanes_per_word, uint64_t nthreads, uint32_t rounds,
                      void* stream) {
    if (!words || nwords == 0) return fail(SMMO_EINVAL, "atomic probe: null or empty word array");
    if (lanes_per_word < 1 || lanes_per_word > 64) return fail(SMMO_EINVAL, "lanes_per_word must be 1..64");
    if (nthreads == 0 || rounds == 0) return SMMO_OK;
    if (nthreads > (1ull << 32)) return fail(SMMO_EINVAL, "nthreads too large");
    k_atomic_probe<<<grid_for(nthreads, kBlockThreads), kBlockThreads, 0, S(stream)>>>(
        reinterpret_cast<unsigned long long*>(words), nwords, lanes_per_word, nthreads, rounds);
    LAUNCH_CHECK("k_atomic_probe");
    return SMMO_OK;
}

int smmo_valu_probe(float* out, uint32_t kind, uint32_t workgroups, uint32_t iters, void* stream) {
    if (!out || kind > 3 || workgroups == 0) return fail(SMMO_EINVAL, "valu probe: null output, kind > 3 or no workgroups");
    k_valu_probe<<<workgroups, 256, 0, S(stream)>>>(out, kind, iters, 1.0000001f);
    LAUNCH_CHECK("k_valu_probe");
    return SMMO_OK;
}

int smmo_check_force_arith(uint32_t lo_bits, uint32_t hi_bits, uint64_t pairs, uint64_t seed, uint64_t* counts_dev,
                           void* stream) {
    if (!counts_dev) return fail(SMMO_EINVAL, "check_force_arith: null output");
    if (hi_bits < lo_bits || hi_bits > 0x7F800000u) return fail(SMMO_EINVAL, "check_force_arith: bad bit range");
    hipStream_t s = S(stream);
    k_fill_u64<<<1, 64, 0, s>>>(reinterpret_cast<unsigned long long*>(counts_dev), 2, 0);
    LAUNCH_CHECK("k_fill_u64");
    k_check_force_arith<<<4096, 256, 0, s>>>(lo_bits, hi_bits, pairs, seed,
                                             reinterpret_cast<unsigned long long*>(counts_dev));
    LAUNCH_CHECK("k_check_force_arith");
    return SMMO_OK;
}

int smmo_check_publish_order(void* dev_buf, uint64_t buf_bytes, uint32_t blocks, uint32_t rounds, uint64_t seed,
                             uint64_t* counts_dev, void* stream) {
    if (!dev_buf || !counts_dev) return fail(SMMO_EINVAL, "check_publish_order: null argument");
    if (blocks == 0 || rounds == 0 || rounds >= (1u << 31))
        return fail(SMMO_EINVAL, "check_publish_order: blocks %u, rounds %u out of range", blocks, rounds);
    const uint64_t words = (20ull * blocks + 7) / 8;
    if (reinterpret_cast<uintptr_t>(dev_buf) % 8 || buf_bytes < 8 * words)
        return fail(SMMO_EINVAL, "check_publish_order: buffer of %llu bytes (8-aligned, %llu needed)",
                    (unsigned long long)buf_bytes, (unsigned long long)(8 * words));
    hipStream_t s = S(stream);
    // table: alloc words, iteration words, then types
    DevHeap h;
    std::memset(&h, 0, sizeof h);
    h.alloc = reinterpret_cast<uint64_t*>(dev_buf);
    h.iter = h.alloc + blocks;
    h.type = reinterpret_cast<uint32_t*>(h.iter + blocks);
    h.M = blocks;
    k_fill_u64<<<grid_for(words, 256), 256, 0, s>>>(reinterpret_cast<unsigned long long*>(dev_buf), words, 0);
    LAUNCH_CHECK("k_fill_u64");
    k_fill_u64<<<1, 64, 0, s>>>(reinterpret_cast<unsigned long long*>(counts_dev), 4, 0);
    LAUNCH_CHECK("k_fill_u64");
    k_check_publish<<<2048, 256, 0, s>>>(h, blocks, rounds, seed, reinterpret_cast<unsigned long long*>(counts_dev));
    LAUNCH_CHECK("k_check_publish");
    return SMMO_OK;
}

int smmo_occupancy(smmo_heap* heap, uint64_t* used, uint64_t* slots, uint64_t* blocks, void* stream) {
    TimingScope timing(heap, false);
    if (!heap) return fail(SMMO_EINVAL, "null heap");
    if (!used || !slots || !blocks) return fail(SMMO_EINVAL, "null output array");
    hipStream_t s = S(stream);
    const uint32_t nc = (uint32_t)heap->hdr.ncls;
    unsigned long long* c = scratch_counter(heap, 8);
    k_fill_u64<<<1, 64, 0, s>>>(c, 3 * nc, 0);
    LAUNCH_CHECK("k_fill_u64");
    k_occupancy<<<grid_for(heap->hdr.num_blocks, 256), 256, 0, s>>>(heap->dev, c);
    LAUNCH_CHECK("k_occupancy");
    unsigned long long v[3 * SMMO_MAX_CLASSES];
    HIP_TRY(hipMemcpyAsync(v, c, 3 * nc * sizeof v[0], hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (uint32_t t = 0; t < nc; ++t) {
        used[t] = v[3 * t];
        slots[t] = v[3 * t + 1];
        blocks[t] = v[3 * t + 2];
    }
    return SMMO_OK;
}

// host-side walk over a copy of the metadata and data (introspection, not the
// hot path)
// Append the live objects of `cls` in blocks [first, last] (block-major,
// slot-minor) from host copies of their allocation words and data segments.
static void dump_range(const smmo_raw_header& h, uint32_t cls, const uint64_t* l0, uint64_t first, uint64_t last,
                       const uint64_t* alloc, const uint8_t* data, void* const* bufs, uint64_t* refs, uint64_t cap,
                       uint64_t& n) {
    const uint64_t N = h.capacity[cls];
    const uint64_t valid = N >= 64 ? ~0ull : ((1ull << N) - 1);
    for (uint64_t b = first; b <= last; ++b) {
        if (!((l0[(b >> 6) * kBmStride] >> (b & 63)) & 1)) continue;
        uint64_t w = alloc[b - first] & valid;
        const uint8_t* blk = data + (b - first) * h.block_bytes;
        while (w) {
            uint32_t slot = (uint32_t)__builtin_ctzll(w);
            w &= w - 1;
            if (n < cap) {
                if (refs) refs[n] = make_ref(cls, b, slot);
                if (bufs)
                    for (uint32_t f = 0; f < h.nfields[cls]; ++f) {
                        if (!bufs[f]) continue;
                        uint32_t fb = h.field_bytes[cls][f];
                        std::memcpy(static_cast<uint8_t*>(bufs[f]) + n * fb, blk + h.field_off[cls][f] + slot * fb, fb);
                    }
            }
            ++n;
        }
    }
}

static int dump_walk(smmo_heap* heap, uint32_t cls, void* const* bufs, uint64_t* refs, uint64_t cap,
                     uint64_t* n_out, void* stream) {
    TimingScope timing(heap, false);
    int rc = check_heap_cls(heap, cls);
    if (rc) return rc;
    if (!n_out) return fail(SMMO_EINVAL, "null n_out");
    const smmo_raw_header& h = heap->hdr;
    hipStream_t s = S(stream);
    const uint64_t W0 = h.level_words[0];
    const uint64_t l0_off = h.off_bitmaps + 8 * ((1 + cls) * h.bitmap_words + h.level_off[0]);
    uint64_t n = 0;
    if (h.total_bytes <= (256ull << 20)) {
        // small heap: one copy of the whole buffer
        std::vector<uint8_t> raw(h.total_bytes);
        HIP_TRY(hipMemcpyAsync(raw.data(), heap->base, h.total_bytes, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        dump_range(h, cls, reinterpret_cast<const uint64_t*>(raw.data() + l0_off), 0, h.num_blocks - 1,
                   reinterpret_cast<const uint64_t*>(raw.data() + h.off_alloc), raw.data() + h.off_data, bufs, refs,
                   cap, n);
        *n_out = n;
        return SMMO_OK;
    }
    // big heap: level 0 of allocated[cls], then only the runs of blocks it
    // names (close runs merged), so the copy is the class's size, not the heap's
    std::vector<uint64_t> l0(W0 * kBmStride);
    HIP_TRY(hipMemcpyAsync(l0.data(), heap->base + l0_off, 8 * W0 * kBmStride, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<std::pair<uint64_t, uint64_t>> runs;       // [first, last] block
    for (uint64_t i = 0; i < W0; ++i)
        for (uint64_t w = l0[i * kBmStride]; w; w &= w - 1) {
            const uint64_t b = (i << 6) | (uint64_t)__builtin_ctzll(w);
            if (!runs.empty() && b <= runs.back().second + 8) runs.back().second = b;
            else runs.push_back({b, b});
        }
    std::vector<uint64_t> alloc;
    std::vector<uint8_t> data;
    for (const auto& r : runs) {
        const uint64_t nb = r.second - r.first + 1;
        alloc.resize(nb);
        data.resize(nb * h.block_bytes);
        HIP_TRY(hipMemcpyAsync(alloc.data(), heap->base + h.off_alloc + 8 * r.first, 8 * nb, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(data.data(), heap->base + h.off_data + r.first * h.block_bytes, nb * h.block_bytes,
                               hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        dump_range(h, cls, l0.data(), r.first, r.second, alloc.data(), data.data(), bufs, refs, cap, n);
    }
    *n_out = n;
    return SMMO_OK;
}

int smmo_dump_objects(smmo_heap* heap, uint32_t cls, void* const* host_field_bufs, uint64_t cap, uint64_t* n_out,
                      void* stream) {
    return dump_walk(heap, cls, host_field_bufs, nullptr, cap, n_out, stream);
}

int smmo_dump_refs(smmo_heap* heap, uint32_t cls, uint64_t* host_refs, uint64_t cap, uint64_t* n_out,
                   void* stream) {
    return dump_walk(heap, cls, nullptr, host_refs, cap, n_out, stream);
}

int smmo_raw_bytes(const smmo_heap* heap, uint64_t* out) {
    if (!heap || !out) return fail(SMMO_EINVAL, "null argument");
    *out = heap->hdr.off_data;
    return SMMO_OK;
}

int smmo_dump_raw(smmo_heap* heap, void* host_buf, uint64_t bytes, void* stream) {
    TimingScope timing(heap, false);
    if (!heap || !host_buf) return fail(SMMO_EINVAL, "null argument");
    if (bytes < heap->hdr.off_data)
        return fail(SMMO_EINVAL, "dump_raw: %llu bytes < %llu", (unsigned long long)bytes,
                    (unsigned long long)heap->hdr.off_data);
    hipStream_t s = S(stream);
    HIP_TRY(hipMemcpyAsync(host_buf, heap->base, heap->hdr.off_data, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SMMO_OK;
}

int smmo_status(smmo_heap* heap, uint32_t* flags_out, void* stream) {
    TimingScope timing(heap, false);
    if (!heap || !flags_out) return fail(SMMO_EINVAL, "null argument");
    hipStream_t s = S(stream);
    HIP_TRY(hipMemcpyAsync(flags_out, heap->dev.status, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SMMO_OK;
}

int smmo_clear_status(smmo_heap* heap, void* stream) {
    TimingScope timing(heap, false);
    if (!heap) return fail(SMMO_EINVAL, "null argument");
    hipStream_t s = S(stream);
    // status word and counters: 256 bytes = 32 words, written by a kernel
    k_fill_u64<<<1, 64, 0, s>>>(reinterpret_cast<unsigned long long*>(heap->dev.status), 32, 0);
    LAUNCH_CHECK("k_fill_u64");
    return SMMO_OK;
}

int smmo_stats(smmo_heap* heap, uint64_t* out, uint32_t n, void* stream) {
    TimingScope timing(heap, false);
    if (!heap || !out || n > SMMO_CNT_NUM) return fail(SMMO_EINVAL, "bad argument");
    hipStream_t s = S(stream);
    HIP_TRY(hipMemcpyAsync(out, heap->dev.counters, 8ull * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SMMO_OK;
}

// ------------------------------------------------------------- arena ----
}  // extern "C"

struct smmo_arena {
    uint8_t* base;
    uint64_t bytes;
    std::map<uint64_t, uint64_t> free_ranges;   // offset -> size
    std::map<uint64_t, uint64_t> used;          // offset -> size
};

struct smmo_batch {
    smmo_arena* arena;
    uint32_t max_inst;
    uint32_t grid;                              // persistent workgroups in use
    uint32_t grid_max;                          // the largest grid of either mode (tables sized for it)
    uint32_t grid_bar;                          // the persistent kernel's largest grid (barrier words sized for it)
    uint32_t cus, per_cu;                       // compute units, workgroups per CU of the current grid
    uint32_t per_cu_mode[2];                    // most workgroups per CU of each mode
    uint32_t mode;                              // SMMO_BATCH_PHASED or SMMO_BATCH_PERSISTENT
    uint32_t wg_req = 0;                        // requested workgroups per CU (0: the mode's default)
    uint8_t* dev;                               // device tables (from the arena)
    BatchDesc* d_desc;
    BatchProg* d_prog;
    BatchSched* d_sched;
    int32_t* d_wg_inst;
    uint32_t* d_bar;
    std::vector<int> used;                      // slot in use
    std::vector<uint64_t> weight;               // grid cells of each slot
    std::vector<uint32_t> cap;                  // most workgroups a slot's instance can use
    std::vector<uint64_t> w0;                   // level-0 bitmap words of a slot's heap
    uint8_t* h_stage = nullptr;                 // pinned staging of the schedule tables
    hipEvent_t stage_done = nullptr;            // the last upload from the staging has completed
    bool dirty;
    uint64_t generation = 0;                    // bumped whenever the instance set or grid changes
};

struct smmo_batch_graph {
    hipGraphExec_t exec;
    smmo_batch* batch;
    uint64_t generation;                        // the batch's generation at capture
};

extern "C" {

int smmo_arena_create(void* dev_mem, uint64_t bytes, smmo_arena** out) {
    if (!dev_mem || !out || bytes < 256) return fail(SMMO_EINVAL, "arena: bad arguments");
    smmo_arena* A = new smmo_arena();
    uint64_t skew = (256 - reinterpret_cast<uintptr_t>(dev_mem) % 256) % 256;
    A->base = static_cast<uint8_t*>(dev_mem) + skew;
    A->bytes = (bytes - skew) / 256 * 256;
    A->free_ranges[0] = A->bytes;
    *out = A;
    return SMMO_OK;
}

int smmo_arena_destroy(smmo_arena* arena) {
    delete arena;
    return SMMO_OK;
}

int smmo_arena_alloc(smmo_arena* A, uint64_t bytes, void** dev_out) {
    if (!A || !dev_out || bytes == 0) return fail(SMMO_EINVAL, "arena_alloc: bad arguments");
    const uint64_t need = align_up(bytes, 256);
    for (auto it = A->free_ranges.begin(); it != A->free_ranges.end(); ++it) {
        if (it->second < need) continue;
        const uint64_t off = it->first, size = it->second;
        A->free_ranges.erase(it);
        if (size > need) A->free_ranges[off + need] = size - need;
        A->used[off] = need;
        *dev_out = A->base + off;
        return SMMO_OK;
    }
    return fail(SMMO_ENOMEM_DEVICE, "arena: no free range of %llu bytes", (unsigned long long)need);
}

int smmo_arena_free(smmo_arena* A, void* dev_ptr) {
    if (!A || !dev_ptr) return fail(SMMO_EINVAL, "arena_free: bad arguments");
    const uint64_t off = static_cast<uint8_t*>(dev_ptr) - A->base;
    auto u = A->used.find(off);
    if (u == A->used.end()) return fail(SMMO_EINVAL, "arena_free: pointer was not allocated here");
    uint64_t start = off, size = u->second;
    A->used.erase(u);
    auto next = A->free_ranges.lower_bound(start);
    if (next != A->free_ranges.end() && next->first == start + size) {   // merge with the next range
        size += next->second;
        A->free_ranges.erase(next);
    }
    auto prev = A->free_ranges.lower_bound(start);
    if (prev != A->free_ranges.begin()) {
        --prev;
        if (prev->first + prev->second == start) {                         // merge with the previous
            start = prev->first;
            size += prev->second;
            A->free_ranges.erase(prev);
        }
    }
    A->free_ranges[start] = size;
    return SMMO_OK;
}

int smmo_arena_stats(const smmo_arena* A, uint64_t* free_bytes, uint64_t* largest_free) {
    if (!A) return fail(SMMO_EINVAL, "null arena");
    uint64_t tot = 0, big = 0;
    for (auto& kv : A->free_ranges) {
        tot += kv.second;
        big = std::max(big, kv.second);
    }
    if (free_bytes) *free_bytes = tot;
    if (largest_free) *largest_free = big;
    return SMMO_OK;
}

// ------------------------------------------------------------- batch ----
// workgroups per CU of the phase kernels: at most, and by default
constexpr uint32_t kPhasedMaxPerCu = 32, kPhasedDefaultPerCu = 16;

static uint32_t default_per_cu(const smmo_batch* B) {
    return B->mode == SMMO_BATCH_PHASED ? kPhasedDefaultPerCu : B->per_cu_mode[SMMO_BATCH_PERSISTENT];
}

int smmo_batch_create(smmo_arena* arena, uint32_t max_inst, smmo_batch** out) {
    if (!arena || !out || max_inst == 0 || max_inst > 65536) return fail(SMMO_EINVAL, "batch: bad arguments");
    int dev = 0, cus = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int per_cu_phased = 0;
    {
        int o[4];
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o[0], (k_batch_phase<MFishPlan, false, true>), 256, 0));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o[1], (k_batch_phase<MFishMove, false, false>), 256, 0));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o[2], (k_batch_phase<MSharkPlan, true, true>), 256, 0));
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&o[3], (k_batch_phase<MSharkMove, true, false>), 256, 0));
        per_cu_phased = std::min(std::min(o[0], o[1]), std::min(o[2], o[3]));
    }
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch_wator, 256, 0));
    if (per_cu < 1 || per_cu_phased < 1) return fail(SMMO_EHIP, "batch kernels cannot be resident");
    if (per_cu > (int)kPhasedMaxPerCu) per_cu = (int)kPhasedMaxPerCu;
    smmo_batch* B = new smmo_batch();
    B->arena = arena;
    B->max_inst = max_inst;
    // the persistent kernel needs every workgroup resident at once for the
    // instance barriers: its grid is the occupancy the runtime reports.  The
    // phase kernels need no co-residency, so their grid may exceed it: more
    // workgroups give every instance more waves and keep the CUs busy while
    // others finish (config 5: 401 ms at the 5 resident per CU, 333 at 16, 326
    // at 32); the tables are sized for the larger grid
    B->cus = (uint32_t)cus;
    B->per_cu_mode[SMMO_BATCH_PHASED] = kPhasedMaxPerCu;
    B->per_cu_mode[SMMO_BATCH_PERSISTENT] = (uint32_t)per_cu;
    B->mode = SMMO_BATCH_PHASED;
    B->per_cu = default_per_cu(B);
    B->grid = (uint32_t)cus * B->per_cu;
    B->grid_max = (uint32_t)cus * std::max((uint32_t)per_cu, kPhasedMaxPerCu);
    B->grid_bar = (uint32_t)cus * (uint32_t)per_cu;
    const uint64_t bytes = align_up(sizeof(BatchDesc) * max_inst, 256) + align_up(sizeof(BatchProg) * max_inst, 256) +
                           align_up(sizeof(BatchSched) * max_inst, 256) + align_up(4ull * B->grid_max, 256) +
                           align_up(4ull * max_inst * bar_words(B->grid_bar), 256);
    void* p = nullptr;
    int rc = smmo_arena_alloc(arena, bytes, &p);
    if (rc) { delete B; return rc; }
    uint8_t* q = static_cast<uint8_t*>(p);
    B->dev = q;
    B->d_desc = reinterpret_cast<BatchDesc*>(q);        q += align_up(sizeof(BatchDesc) * max_inst, 256);
    B->d_prog = reinterpret_cast<BatchProg*>(q);        q += align_up(sizeof(BatchProg) * max_inst, 256);
    B->d_sched = reinterpret_cast<BatchSched*>(q);      q += align_up(sizeof(BatchSched) * max_inst, 256);
    B->d_wg_inst = reinterpret_cast<int32_t*>(q);       q += align_up(4ull * B->grid_max, 256);
    B->d_bar = reinterpret_cast<uint32_t*>(q);
    B->used.assign(max_inst, 0);
    B->weight.assign(max_inst, 0);
    B->cap.assign(max_inst, 0);
    B->w0.assign(max_inst, 0);
    {
        void* hp = nullptr;
        const uint64_t stage_bytes = sizeof(BatchSched) * max_inst + 4ull * B->grid_max;
        if (hipHostMalloc(&hp, stage_bytes, hipHostMallocDefault) != hipSuccess || !hp) {
            smmo_arena_free(arena, B->dev);
            delete B;
            return fail(SMMO_EHIP, "batch: pinned staging of %llu bytes", (unsigned long long)stage_bytes);
        }
        B->h_stage = static_cast<uint8_t*>(hp);
        if (hipEventCreateWithFlags(&B->stage_done, hipEventDisableTiming) != hipSuccess) {
            (void)hipHostFree(hp);
            smmo_arena_free(arena, B->dev);
            delete B;
            return fail(SMMO_EHIP, "batch: event creation");
        }
    }
    B->dirty = true;
    std::vector<BatchProg> prog(max_inst, BatchProg{0, 0});
    HIP_TRY(hipMemcpy(B->d_prog, prog.data(), sizeof(BatchProg) * max_inst, hipMemcpyHostToDevice));
    *out = B;
    return SMMO_OK;
}

int smmo_batch_destroy(smmo_batch* B) {
    if (!B) return SMMO_OK;
    if (B->stage_done) {
        (void)hipEventSynchronize(B->stage_done);
        (void)hipEventDestroy(B->stage_done);
    }
    if (B->h_stage) (void)hipHostFree(B->h_stage);
    smmo_arena_free(B->arena, B->dev);
    delete B;
    return SMMO_OK;
}

int smmo_batch_add_wator(smmo_batch* B, smmo_heap* heap, const smmo_wator_args* args, uint32_t steps,
                         void* stream, uint32_t* slot_out) {
    if (!B || !heap || !args || !slot_out) return fail(SMMO_EINVAL, "batch_add: null argument");
    if (args->fish_cls >= heap->hdr.ncls || args->shark_cls >= heap->hdr.ncls)
        return fail(SMMO_EINVAL, "batch_add: class out of range");
    uint32_t slot = 0;
    while (slot < B->max_inst && B->used[slot]) ++slot;
    if (slot == B->max_inst) return fail(SMMO_ENOMEM_DEVICE, "batch_add: all %u slots in use", B->max_inst);
    BatchDesc d;
    std::memset(&d, 0, sizeof d);
    d.h = heap->dev;
    d.a = *args;
    d.a.step = 0;
    BatchProg pr{steps, 0};
    hipStream_t s = S(stream);
    HIP_TRY(hipMemcpyAsync(&B->d_desc[slot], &d, sizeof d, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(&B->d_prog[slot], &pr, sizeof pr, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    heap->in_batch = true;                      // the batch kernels change its blocks from now on
    blocks_changed(heap);
    B->used[slot] = 1;
    B->weight[slot] = (uint64_t)args->width * (uint64_t)args->height;
    // one wave per block of the instance's heap at most (units of one block)
    B->cap[slot] = (uint32_t)std::max<uint64_t>(1, (heap->hdr.num_blocks + 3) / 4);
    B->w0[slot] = heap->hdr.level_words[0];
    B->dirty = true;
    ++B->generation;
    *slot_out = slot;
    return SMMO_OK;
}

int smmo_batch_remove(smmo_batch* B, uint32_t slot) {
    if (!B || slot >= B->max_inst || !B->used[slot]) return fail(SMMO_EINVAL, "batch_remove: bad slot");
    B->used[slot] = 0;
    B->weight[slot] = 0;
    B->dirty = true;
    ++B->generation;
    return SMMO_OK;
}

// Workgroups per instance proportional to its cells (at least one each), but
// no more than it can use: every workgroup of an instance takes part in its
// four barriers per step, and each arrival and departure writes back and
// invalidates that XCD's L2, so idle workgroups cost time.  The tables are
// uploaded in stream order from pinned staging (no host synchronization of
// the stream); the staging is reused only once its previous upload is done.
static int batch_schedule(smmo_batch* B, hipStream_t s) {
    HIP_TRY(hipEventSynchronize(B->stage_done));
    BatchSched* sched = reinterpret_cast<BatchSched*>(B->h_stage);
    int32_t* wg = reinterpret_cast<int32_t*>(B->h_stage + sizeof(BatchSched) * B->max_inst);
    for (uint32_t i = 0; i < B->grid; ++i) wg[i] = -1;
    uint64_t total = 0;
    uint32_t n = 0;
    for (uint32_t i = 0; i < B->max_inst; ++i) {
        sched[i] = BatchSched{0, 0, 0, 0};
        if (B->used[i]) { total += B->weight[i]; ++n; }
    }
    if (n > B->grid) return fail(SMMO_EINVAL, "batch: %u instances but only %u workgroups", n, B->grid);
    uint32_t next = 0;
    const uint32_t spare = B->grid - n;                    // beyond one each
    for (uint32_t i = 0; i < B->max_inst; ++i) {
        if (!B->used[i]) continue;
        const uint32_t extra = total ? (uint32_t)((double)spare * (double)B->weight[i] / (double)total) : 0;
        const uint32_t cnt = std::min(1 + extra, std::max(1u, B->cap[i]));
        // the coarsest unit (at most 8 blocks) that still gives every wave
        // of the instance four units of its heap to take
        uint32_t ul = kBatchUnitLog2Max;
        while (ul > 0 && (B->w0[i] << (6 - ul)) < 4ull * 4 * cnt) --ul;
        sched[i] = BatchSched{next, cnt, ul, 0};
        for (uint32_t k = 0; k < cnt; ++k) wg[next + k] = (int32_t)i;
        next += cnt;
    }
    HIP_TRY(hipMemcpyAsync(B->d_sched, sched, sizeof(BatchSched) * B->max_inst, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(B->d_wg_inst, wg, 4ull * B->grid, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(B->stage_done, s));
    B->dirty = false;
    return SMMO_OK;
}

// The launches of one group of `steps` steps, in the batch's mode.
static int batch_launch(smmo_batch* B, uint32_t steps, hipStream_t s) {
    if (B->mode == SMMO_BATCH_PHASED) {
        // one launch per phase of each step; the boundaries order the phases
        for (uint32_t st = 0; st < steps; ++st) {
            k_batch_phase<MFishPlan, false, true><<<B->grid, 256, 0, s>>>(B->d_desc, B->d_prog, B->d_sched,
                                                                          B->d_wg_inst, st);
            k_batch_phase<MFishMove, false, false><<<B->grid, 256, 0, s>>>(B->d_desc, B->d_prog, B->d_sched,
                                                                           B->d_wg_inst, st);
            k_batch_phase<MSharkPlan, true, true><<<B->grid, 256, 0, s>>>(B->d_desc, B->d_prog, B->d_sched,
                                                                          B->d_wg_inst, st);
            k_batch_phase<MSharkMove, true, false><<<B->grid, 256, 0, s>>>(B->d_desc, B->d_prog, B->d_sched,
                                                                           B->d_wg_inst, st);
        }
        LAUNCH_CHECK("k_batch_phase");
        k_batch_advance<<<grid_for(B->max_inst, 256), 256, 0, s>>>(B->d_prog, B->max_inst, steps);
        LAUNCH_CHECK("k_batch_advance");
        return SMMO_OK;
    }
    // one persistent launch: the instance barrier counters are cleared by a
    // kernel (not a memset, so the pair can be captured and replayed)
    const uint32_t stride = bar_words(B->grid_bar);
    const uint64_t bar_u64 = ((uint64_t)B->max_inst * stride + 1) / 2;
    k_fill_u64<<<grid_for(bar_u64, 256), 256, 0, s>>>(reinterpret_cast<unsigned long long*>(B->d_bar), bar_u64, 0);
    LAUNCH_CHECK("k_fill_u64");
    k_batch_wator<<<B->grid, 256, 0, s>>>(B->d_desc, B->d_prog, B->d_sched, B->d_wg_inst, B->d_bar, stride, steps);
    LAUNCH_CHECK("k_batch_wator");
    return SMMO_OK;
}

static int batch_prepare(smmo_batch* B, hipStream_t s) {
    if (!B->dirty) return SMMO_OK;
    return batch_schedule(B, s);
}

int smmo_batch_step(smmo_batch* B, uint32_t steps, void* stream) {
    if (!B) return fail(SMMO_EINVAL, "null batch");
    if (steps == 0) return SMMO_OK;
    hipStream_t s = S(stream);
    int rc = batch_prepare(B, s);
    if (rc) return rc;
    return batch_launch(B, steps, s);
}

int smmo_batch_capture_graph(smmo_batch* B, uint32_t launches, uint32_t steps_per_launch, void* stream,
                             smmo_batch_graph** out) {
    if (!B || !out) return fail(SMMO_EINVAL, "batch_capture_graph: null argument");
    if (!stream) return fail(SMMO_EINVAL, "batch_capture_graph: capture needs a created stream, not the null stream");
    if (launches == 0 || steps_per_launch == 0) return fail(SMMO_EINVAL, "batch_capture_graph: nothing to capture");
    hipStream_t s = S(stream);
    int rc = batch_prepare(B, s);
    if (rc) return rc;
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    for (uint32_t i = 0; i < launches && rc == SMMO_OK; ++i) rc = batch_launch(B, steps_per_launch, s);
    hipGraph_t graph = nullptr;
    const hipError_t e_end = hipStreamEndCapture(s, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e_end != hipSuccess || !graph)
        return fail(SMMO_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e_end));
    hipGraphExec_t exec = nullptr;
    const hipError_t e_inst = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e_inst != hipSuccess) return fail(SMMO_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e_inst));
    *out = new smmo_batch_graph{exec, B, B->generation};
    return SMMO_OK;
}

int smmo_batch_graph_launch(smmo_batch_graph* g, void* stream) {
    if (!g) return fail(SMMO_EINVAL, "null batch graph");
    if (g->batch->generation != g->generation)
        return fail(SMMO_EINVAL, "batch graph: the batch's instances or grid changed since the capture");
    HIP_TRY(hipGraphLaunch(g->exec, S(stream)));
    return SMMO_OK;
}

int smmo_batch_graph_destroy(smmo_batch_graph* g) {
    if (!g) return SMMO_OK;
    const hipError_t e = hipGraphExecDestroy(g->exec);
    delete g;
    if (e != hipSuccess) return fail(SMMO_EHIP, "hipGraphExecDestroy: %s", hipGetErrorString(e));
    return SMMO_OK;
}

int smmo_batch_remaining(smmo_batch* B, uint32_t* out, void* stream) {
    if (!B || !out) return fail(SMMO_EINVAL, "null argument");
    std::vector<BatchProg> prog(B->max_inst);
    hipStream_t s = S(stream);
    HIP_TRY(hipMemcpyAsync(prog.data(), B->d_prog, sizeof(BatchProg) * B->max_inst, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < B->max_inst; ++i) out[i] = B->used[i] ? prog[i].remaining : 0xFFFFFFFFu;
    return SMMO_OK;
}

int smmo_batch_grid(const smmo_batch* B, uint32_t* workgroups) {
    if (!B || !workgroups) return fail(SMMO_EINVAL, "null argument");
    *workgroups = B->grid;
    return SMMO_OK;
}

int smmo_batch_set_grid(smmo_batch* B, uint32_t wg_per_cu) {
    if (!B) return fail(SMMO_EINVAL, "null batch");
    B->wg_req = wg_per_cu;
    const uint32_t most = B->per_cu_mode[B->mode];
    const uint32_t w = wg_per_cu == 0 ? default_per_cu(B) : (wg_per_cu > most ? most : wg_per_cu);
    B->per_cu = w;
    B->grid = B->cus * w;
    B->dirty = true;
    ++B->generation;
    return SMMO_OK;
}

int smmo_batch_set_mode(smmo_batch* B, uint32_t mode) {
    if (!B) return fail(SMMO_EINVAL, "null batch");
    if (mode != SMMO_BATCH_PHASED && mode != SMMO_BATCH_PERSISTENT) return fail(SMMO_EINVAL, "batch: unknown mode %u", mode);
    B->mode = mode;
    return smmo_batch_set_grid(B, B->wg_req);
}

uint64_t smmo_ref_make(uint32_t cls, uint64_t block, uint32_t slot) { return make_ref(cls, block, slot); }
uint32_t smmo_ref_class(uint64_t ref) { return ref_cls(ref); }
uint64_t smmo_ref_block(uint64_t ref) { return ref_block(ref); }
uint32_t smmo_ref_slot(uint64_t ref) { return ref_slot(ref); }

const char* smmo_strerror(int code) {
    switch (code) {
        case SMMO_OK: return "ok";
        case SMMO_EINVAL: return "invalid argument";
        case SMMO_ETOOSMALL: return "device buffer too small";
        case SMMO_ENOMEM_DEVICE: return "heap out of blocks";
        case SMMO_ERETRY: return "retry bound exceeded";
        case SMMO_EHIP: return "HIP runtime error";
        case SMMO_ECORRUPT: return "heap corruption detected";
        case SMMO_ENOTBUILT: return "variant not built";
        default: return "unknown error";
    }
}

const char* smmo_last_error(void) { return g_err.c_str(); }

}  // extern "C"
