// Device-side basics of the SMMO heap for gfx950 (CDNA4, wave64).
//
// Heap model (DynaSOAr, Sec. 3): M equal blocks; each block has a 64-bit
// object allocation bitmap, a 64-bit object iteration bitmap and a type id
// (kept here in three per-block arrays indexed by block id, so every block's
// words sit at a location that is a function of its id only), followed by an
// SOA data segment.  Block bitmaps (free / allocated[T] / active[T], Sec. 3.4)
// are hierarchical bitmaps of 64-bit containers (Sec. 4.1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smmo.h"

namespace smmo {

constexpr uint64_t kOnes = ~0ull;
constexpr uint64_t kFail = ~0ull;
constexpr uint32_t kNoType = 0xFFFFFFFFu;
constexpr uint32_t kWave = 64;
// Bitmap word k of a level sits kBmStride words after word k-1: one word per
// 128-B line.  Agent-scope atomics are performed past the L2 and queue per
// line, and the few words of a level-0 active bitmap take every lookup and
// every full/non-full transition of their class; on their own lines they
// no longer wait on each other's atomics.  (-DSMMO_BM_STRIDE=1 builds the
// dense layout for comparison.)
#ifndef SMMO_BM_STRIDE
#define SMMO_BM_STRIDE 16
#endif
constexpr uint64_t kBmStride = SMMO_BM_STRIDE;

// Everything a kernel needs to address the heap; passed by value.
struct DevHeap {
    uint8_t* data;                 // M * block_bytes
    uint64_t* alloc;               // [M] object allocation words
    uint64_t* iter;                // [M] object iteration words
    uint32_t* type;                // [M] block type ids
    uint64_t* bm;                  // all block-bitmap words
    uint32_t* status;              // sticky SMMO_STATUS_* bits
    unsigned long long* counters;  // SMMO_CNT_*
    uint8_t* scratch;              // enumeration / counting scratch
    const smmo_raw_header* hdr;    // field layout table (device copy)
    uint64_t M;
    uint64_t block_bytes;
    uint64_t bitmap_words;
    uint64_t level_off[SMMO_MAX_LEVELS];
    uint64_t level_words[SMMO_MAX_LEVELS];
    uint32_t nlevels;
    uint32_t ncls;
    uint32_t tune;
    uint32_t lookups;
    uint32_t force_fail_ppm;
    uint32_t pad0;
    uint64_t cls_pad[SMMO_MAX_CLASSES];  // slots >= capacity (always 1 in the word)
    uint32_t cls_cap[SMMO_MAX_CLASSES];
};

// Bitmap ids inside the bitmap area.
__host__ __device__ inline uint32_t bm_free() { return 0; }
__host__ __device__ inline uint32_t bm_allocated(uint32_t t) { return 1 + t; }
__host__ __device__ inline uint32_t bm_active(const DevHeap& h, uint32_t t) { return 1 + h.ncls + t; }

// ------------------------------------------------------------- atomics ----
// All heap-word atomics are agent (device) scope: the 8 XCDs of the chip
// have separate L2s, so the workgroup/XCD scopes would not order them.
__device__ inline uint64_t at_or(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t at_and(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_and(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t at_or_acq(uint64_t* p, uint64_t v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t at_load(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t at_load32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void at_store(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every memory operation this wave has issued has completed.  An
// agent-scope store is complete once it has reached the device coherence
// point, so agent-scope accesses issued after the wait, from any XCD, are
// ordered after it.  This is the ordering Alg. 8's fence provides between a
// block's type and its allocation word.  A C++ release store would add a
// write-back of this XCD's whole L2, which only plain stores need; the words
// it orders here are all agent-scope atomics.  (vmcnt(0); the expcnt and
// lgkmcnt fields are left at their maximum, i.e. not waited on.)
__device__ inline void wait_mem_complete() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);      // no compiler motion across the wait
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// Agent-scope store ordered after this wave's earlier agent-scope accesses.
__device__ inline void at_store_ordered(uint64_t* p, uint64_t v) {
    wait_mem_complete();
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void at_store32(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void set_status(const DevHeap& h, uint32_t bits) {
    __hip_atomic_fetch_or(h.status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void count(const DevHeap& h, uint32_t which, uint64_t n = 1) {
    if (h.tune & SMMO_TUNE_STATS)
        __hip_atomic_fetch_add(&h.counters[which], (unsigned long long)n, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
}
// A bound was hit: count it (always) and raise `bits` in the status word.
__device__ inline void guard_hit(const DevHeap& h, uint32_t which, uint32_t bits) {
    __hip_atomic_fetch_add(&h.counters[which], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    set_status(h, bits);
}
__device__ inline bool status_has(const DevHeap& h, uint32_t bits) {
    return (__hip_atomic_load(h.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bits) != 0;
}
__device__ inline void backoff() { __builtin_amdgcn_s_sleep(2); }

// ---------------------------------------------------------- wave prims ----
__device__ inline uint32_t lane_id() { return __lane_id(); }
__device__ inline uint64_t ballot(bool p) { return __ballot(p); }
// number of set bits of m strictly below this lane
__device__ inline uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ inline uint32_t readlane32(uint32_t v, uint32_t l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, (int)l);
}
__device__ inline uint64_t readlane64(uint64_t v, uint32_t l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, (int)l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), (int)l);
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t wave_or(uint64_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}
__device__ inline uint32_t wave_add(uint32_t v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------- bit tricks ----
__device__ inline uint32_t popc64(uint64_t v) { return (uint32_t)__popcll(v); }
__device__ inline uint32_t ctz64(uint64_t v) { return (uint32_t)__builtin_ctzll(v); }
__device__ inline uint64_t rotr64(uint64_t v, uint32_t r) {
    r &= 63;
    return r ? (v >> r) | (v << (64 - r)) : v;
}
__device__ inline uint64_t rotl64(uint64_t v, uint32_t r) {
    r &= 63;
    return r ? (v << r) | (v >> (64 - r)) : v;
}
// Position of the n-th (0-based) set bit of v; requires n < popc(v).
// Binary search over popcounts instead of clearing n low bits one by one.
__device__ inline uint32_t nth_set_bit(uint64_t v, uint32_t n) {
    uint32_t pos = 0;
#pragma unroll
    for (uint32_t w = 32; w >= 1; w >>= 1) {
        uint32_t c = popc64(v & ((1ull << w) - 1));
        if (n >= c) { n -= c; v >>= w; pos += w; }
    }
    return pos;
}
// Mask of the lowest k set bits of v (all of v when popc(v) <= k).
__device__ inline uint64_t lowest_k_bits(uint64_t v, uint32_t k) {
    if (popc64(v) <= k) return v;
    if (k == 0) return 0;
    uint32_t p = nth_set_bit(v, k);     // first bit NOT taken
    return v & ((1ull << p) - 1);
}

// -------------------------------------------------- wave-uniform ops ----
// The allocator's bookkeeping (bitmap searches, block words) runs on the
// whole wave with wave-uniform values: the compiler keeps them in scalar
// registers and works on them with the scalar unit's 64-bit instructions,
// instead of spending a full vector instruction per step on one lane.  A
// heap word is read by every active lane at the same address (a single
// memory request) and broadcast; an atomic is performed once, by the first
// active lane.  These functions are also correct with one active lane.
__device__ inline uint32_t first_lane() { return ctz64(__builtin_amdgcn_read_exec()); }
__device__ inline bool is_first_lane() { return lane_id() == first_lane(); }
// the first active lane's value, as a wave-uniform value
__device__ inline uint32_t uni32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ inline uint64_t uni64(uint64_t v) {
    const uint32_t lo = uni32((uint32_t)v), hi = uni32((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
__device__ inline uint64_t w_load(const uint64_t* p) { return uni64(at_load(p)); }
__device__ inline uint32_t w_load32(const uint32_t* p) { return uni32(at_load32(p)); }
__device__ inline uint64_t w_or(uint64_t* p, uint64_t v) {
    uint64_t r = 0;
    if (is_first_lane()) r = at_or(p, v);
    return uni64(r);
}
__device__ inline uint64_t w_and(uint64_t* p, uint64_t v) {
    uint64_t r = 0;
    if (is_first_lane()) r = at_and(p, v);
    return uni64(r);
}
__device__ inline void w_set_status(const DevHeap& h, uint32_t bits) {
    if (is_first_lane()) set_status(h, bits);
}
__device__ inline void w_count(const DevHeap& h, uint32_t which, uint64_t n = 1) {
    if ((h.tune & SMMO_TUNE_STATS) && is_first_lane()) count(h, which, n);
}
__device__ inline void w_guard_hit(const DevHeap& h, uint32_t which, uint32_t bits) {
    if (is_first_lane()) guard_hit(h, which, bits);
}
__device__ inline bool w_status_has(const DevHeap& h, uint32_t bits) { return (w_load32(h.status) & bits) != 0; }

// ------------------------------------------------------------------ RNG ----
// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): first output for seed x.
__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
// Draw keyed on (seed, step, id, stream).
__host__ __device__ inline uint64_t ctr_draw(uint64_t seed, uint64_t step, uint64_t id, uint64_t stream) {
    return splitmix64(splitmix64(splitmix64(seed ^ (stream << 56)) ^ step) ^ id);
}
__host__ __device__ inline float unit_float(uint64_t h) {
    return (float)(uint32_t)(h >> 40) * (1.0f / 16777216.0f);
}

// --------------------------------------------------------------- handles ----
// bits 56-63 class id + 1, bits 6-49 block, bits 0-5 slot; 0 = null.
__host__ __device__ inline uint64_t make_ref(uint32_t cls, uint64_t block, uint32_t slot) {
    return ((uint64_t)(cls + 1) << 56) | (block << 6) | (uint64_t)slot;
}
__host__ __device__ inline uint32_t ref_cls(uint64_t r) { return (uint32_t)(r >> 56) - 1u; }
__host__ __device__ inline uint64_t ref_block(uint64_t r) { return (r >> 6) & ((1ull << 44) - 1); }
__host__ __device__ inline uint32_t ref_slot(uint64_t r) { return (uint32_t)(r & 63); }

// Address of field f of the object in (block, slot) of class cls.
__device__ inline uint8_t* field_addr(const DevHeap& h, uint32_t cls, uint64_t block, uint32_t slot,
                                      uint32_t f) {
    return h.data + block * h.block_bytes + h.hdr->field_off[cls][f] + slot * h.hdr->field_bytes[cls][f];
}
template <class F>
__device__ inline F& field_of(const DevHeap& h, uint64_t ref, uint32_t f) {
    uint32_t c = ref_cls(ref);
    return *reinterpret_cast<F*>(h.data + ref_block(ref) * h.block_bytes + h.hdr->field_off[c][f] +
                                 ref_slot(ref) * sizeof(F));
}

}  // namespace smmo
