// Object allocation and deallocation (DynaSOAr Sec. 3.5-3.6, Alg. 1, 2, 6-9,
// App. A), re-shaped for wave64.
//
// The paper coalesces the allocation requests of a warp into one leader
// thread (Sec. 4.2, after XMalloc).  Here the unit is the 64-lane wavefront:
//   * one ballot collects the requesting lanes of a class,
//   * the wave reserves as many slots as it can in one block with a single
//     64-bit atomic OR (the block's allocation word holds all 64 slots, one
//     per lane) and moves on to further blocks for the rest,
//   * every lane takes its slot as the n-th set bit of the reserved mask,
//     n = its rank among the requesting lanes (mbcnt).
// Destruction groups the lanes of a wave by block and frees each group with
// one atomic AND.  The bookkeeping runs wave-uniform (dev.h): every atomic
// once per wave, the bit manipulation on the scalar unit, and no spin ever
// waits on a lane of the same wave.
//
// Slots >= capacity N_T stay set for the life of a block (App. A.1); the
// capacity-64 rules of Alg. 6/7/9 are applied to the word itself:
//   FULL   the reservation turned the word into all ones
//   FIRST  the word was all ones before a deallocation
//   EMPTY  only the padding bits remain after a deallocation
//   invalidation succeeds iff the word was exactly the padding.
#pragma once

#include "bitmap.h"

namespace smmo {

// Bounds of the allocator's retry loops.  A wave gives up an allocation
// after kOomRounds rounds that find neither an active block nor any free
// block (the free bitmap's top word empty: OOM; the bound is large because a
// wave can also lose every freed block to others for a while: with 512 waves
// churning two classes through 40 spare blocks, 4,096 such rounds were once
// exceeded with free blocks coming and going), or after kAllocIters
// iterations in all (RETRY: a livelock guard that contention alone does not
// reach).  Once the status word holds OOM or RETRY, later requests give up
// after a few rounds instead.
constexpr uint32_t kOomRounds = 1u << 14;
constexpr uint32_t kAllocIters = 1u << 18;

// initialize_block<T> (Alg. 8): type and iteration word first, then, once
// both stores have completed, the allocation word.  A reservation that sees
// the new word therefore reads the new type (see alloc_piece).  The zeroed
// iteration word keeps a block re-initialized during a do-all out of it.
// No plain store of this wave needs to be visible before the word: a new
// object's fields are written after its reservation, and no method reads
// fields written in the same do-all (phases are separate kernels, each
// ending with a release).
// With `word` the allocation word starts as given instead of the padding
// (all ones: a block whose every slot goes to the caller).
__device__ inline void initialize_block(const DevHeap& h, uint32_t cls, uint64_t bid, uint64_t word) {
    if (is_first_lane()) {
        at_store32(&h.type[bid], cls);
        at_store(&h.iter[bid], 0);
        at_store_ordered(&h.alloc[bid], word);
    }
}

// The reader's half of that order: an OR on a block's allocation word, after
// which (the OR has returned before the next load is issued: its result is
// broadcast first) block_type reads the type at the device coherence point,
// so it is at least as new as the initialization that wrote the word the OR
// saw.  Reservations and invalidations both use this pair.
__device__ inline uint64_t reserve_or(const DevHeap& h, uint64_t bid, uint64_t mask) {
    const uint64_t before = w_or(&h.alloc[bid], mask);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return before;
}
__device__ inline uint32_t block_type(const DevHeap& h, uint64_t bid) { return w_load32(&h.type[bid]); }

// invalidate(bid) (Alg. 9, iterative).  True if this call took the block
// from "empty" to "invalidated"; the caller then frees it.
// The OR is relaxed: every word it races with is an agent-scope atomic, and
// the type is read with a device-scope load after the OR has returned.  No
// plain store into the block's data can be pending in this do-all, since a
// method writes no field of an object destroyed in the same do-all, and
// earlier do-alls are separate kernels.
__device__ inline bool invalidate_block(const DevHeap& h, uint64_t bid) {
    bid = uni64(bid);
    for (uint32_t tries = 0; tries < kSpinLimit; ++tries) {
        const uint64_t before = reserve_or(h, bid, kOnes);
        if (before == kOnes) return false;          // nothing invalidated
        const uint32_t t = block_type(h, bid);
        if (t >= h.ncls) { w_set_status(h, SMMO_STATUS_CORRUPT); return false; }
        const uint64_t pad = h.cls_pad[t];
        if (before == pad) return true;             // every slot was free
        w_count(h, SMMO_CNT_INVAL_ROLLBACK);
        // roll back exactly the bits this call set (the zeros of `before`)
        const uint64_t before_rb = w_and(&h.alloc[bid], before);
        // a thread that freed a slot in between saw a full block (FIRST) and
        // waits to set active[t]; perform the deferred deactivation for it
        if (before_rb != kOnes) bm_clear(h, bm_active(h, t), bid);
        if ((before_rb & before) != pad) return false;
        // emptied again while invalidated: try once more
    }
    w_guard_hit(h, SMMO_CNT_GUARD_INVAL, SMMO_STATUS_RETRY);
    return false;
}

// Alg. 2's block state update after a deallocation of `mask` from block
// `bid` of class T whose AND returned `before` (wave-uniform arguments).
__device__ inline void dealloc_update(const DevHeap& h, uint32_t T, uint64_t bid, uint64_t mask, uint64_t before) {
    T = uni32(T);
    bid = uni64(bid);
    mask = uni64(mask);
    before = uni64(before);
    if ((before & mask) != mask) w_set_status(h, SMMO_STATUS_CORRUPT);   // double free
    const bool first = before == kOnes;
    const bool empty = (before & ~mask) == h.cls_pad[T];
    if (first) bm_set(h, bm_active(h, T), bid);
    if (empty && invalidate_block(h, bid)) {
        const uint32_t t = w_load32(&h.type[bid]);
        bm_clear(h, bm_active(h, t), bid);
        bm_clear(h, bm_allocated(t), bid);
        bm_set(h, bm_free(), bid);
        w_count(h, SMMO_CNT_BLOCK_FREE);
    }
}

// Block::deallocate for a mask of slots of class-T objects, then the state update.
__device__ inline void dealloc_mask(const DevHeap& h, uint32_t T, uint64_t bid, uint64_t mask) {
    T = uni32(T);
    bid = uni64(bid);
    mask = uni64(mask);
    dealloc_update(h, T, bid, mask, w_and(&h.alloc[bid], ~mask));
}

// One piece of a coalesced allocation (Alg. 1 + Alg. 6), wave-uniform: find
// an active block of class `cls` (r lookups, then the slow path), and reserve
// up to `want` free slots of it with one atomic OR.  Returns the reserved
// mask (never 0) and the block in bid_out; returns 0 on OOM.
__device__ __forceinline__ uint64_t alloc_piece(const DevHeap& h, uint32_t cls, uint32_t want, uint64_t& seed,
                                       uint64_t& bid_out) {
    cls = uni32(cls);
    want = uni32(want);
    seed = uni64(seed);
    uint32_t empty_rounds = 0;
    const bool rotate = !(h.tune & SMMO_TUNE_NO_ROTATE);
    if (h.tune & SMMO_TUNE_NO_COALESCE) want = 1;
    const bool whole = want >= h.cls_cap[cls];
    for (uint32_t iters = 0;; ++iters) {
        if (iters > kAllocIters) {                        // livelock guard: never hang a kernel
            w_guard_hit(h, SMMO_CNT_GUARD_ALLOC, SMMO_STATUS_RETRY);
            return 0;
        }
        if (iters >= 64 && (iters & 63) == 0 && w_status_has(h, SMMO_STATUS_RETRY)) return 0;
        uint64_t bid = kFail;
        for (uint32_t a = 0; a < h.lookups; ++a) {
            seed = splitmix64(seed);
            // a whole-block request mostly finds no active block: the plain
            // search fails at the top word in one round trip
            bid = whole ? bm_try_find_set(h, bm_active(h, cls), seed)
                        : bm_try_find_set_dense(h, bm_active(h, cls), seed);
            if (bid != kFail) break;
            w_count(h, SMMO_CNT_FIND_FAIL);
            // a request for a whole block or more fills a fresh block by
            // itself, so retrying the lookup cannot save a block: one miss
            // sends it to the slow path
            if (whole) break;
        }
        if (bid == kFail) {                               // slow path
            bid = bm_clear_any(h, bm_free(), seed);
            if (bid == kFail) {
                // only a round that finds the free bitmap empty counts
                // towards OOM; a miss caused by contention is retried (up
                // to the livelock guard above)
                if (bm_top_empty(h, bm_free()) &&
                    (++empty_rounds > kOomRounds || (empty_rounds > 2 && w_status_has(h, SMMO_STATUS_OOM)))) {
                    w_guard_hit(h, SMMO_CNT_OOM, SMMO_STATUS_OOM);
                    return 0;
                }
                backoff();
                continue;
            }
            w_count(h, SMMO_CNT_BLOCK_INIT);
            if (whole) {
                // the whole block goes to this request: it starts full and
                // never becomes active (no other wave can find it before
                // allocated[cls] lists it, and by then it is full), which
                // saves the reservation and two active-bitmap updates
                initialize_block(h, cls, bid, kOnes);
                bm_set(h, bm_allocated(cls), bid);
                bid_out = bid;
                return ~h.cls_pad[cls];
            }
            initialize_block(h, cls, bid, h.cls_pad[cls]);
            bm_set(h, bm_allocated(cls), bid);
            bm_set(h, bm_active(h, cls), bid);
        }
        if (h.tune & SMMO_TUNE_SLOW_PICK)                 // fault injection: widen the pick/reserve window
            for (int i = 0; i < 8; ++i) __builtin_amdgcn_s_sleep(127);
        // Block::reserve, coalesced: take up to `want` zero bits, rotated start
        const uint64_t freeb = ~w_load(&h.alloc[bid]);
        if (!freeb) { w_count(h, SMMO_CNT_RESERVE_FAIL); continue; }
        seed = splitmix64(seed);
        const uint32_t rot = rotate ? (uint32_t)seed & 63 : 0;
        const uint64_t mask = rotl64(lowest_k_bits(rotr64(freeb, rot), want), rot);
        // The type read below must see the type written before the word this
        // OR observed was re-initialized (Alg. 8's fence).  The writer
        // stores the word only after its type store has completed at the
        // device coherence point (initialize_block); here the OR has
        // returned before the type load is issued (its address is uniform
        // and the load follows the broadcast of the OR's result), and the
        // type load is a device-scope load, so it reads at the device
        // coherence point, where the type already is.  An acquire on the OR
        // would also invalidate this CU's caches on every reservation, which
        // more than doubled the allocating do-alls' time on MI355X.
        const uint64_t before = reserve_or(h, bid, mask);
        w_count(h, SMMO_CNT_RESERVE_ATOMIC);
        const uint64_t got = mask & ~before;
        if (!got) { w_count(h, SMMO_CNT_RESERVE_FAIL); continue; }
        const uint32_t t = block_type(h, bid);
        if (t >= h.ncls) { w_set_status(h, SMMO_STATUS_CORRUPT); continue; }
        if ((before | got) == kOnes) bm_clear(h, bm_active(h, t), bid);   // this call filled it
        if (t != cls) {                                   // block changed type: roll back
            w_count(h, SMMO_CNT_TYPE_ROLLBACK);
            dealloc_mask(h, t, bid, got);
            continue;
        }
        bid_out = bid;
        return got;
    }
}

// Wave-collective allocation: every active lane of the wave must call this
// with the same `cls` and `wave_seed`; lanes with want=true receive a handle
// (0 on OOM).
__device__ __forceinline__ uint64_t wave_alloc(const DevHeap& h, uint32_t cls, bool want, uint64_t wave_seed) {
    const uint64_t req = ballot(want);
    if (!req) return 0;
    const uint32_t k = popc64(req);
    const uint32_t rank = lanes_below(req);
    uint64_t seed = uni64(wave_seed);
    uint64_t mine = 0;
    uint32_t taken = 0;
    while (taken < k) {                       // wave-uniform loop
        uint64_t bid = 0;
        const uint64_t got = alloc_piece(h, cls, k - taken, seed, bid);
        if (!got) break;                      // OOM: remaining lanes get null
        const uint32_t n = popc64(got);
        if (want && rank >= taken && rank < taken + n)
            mine = make_ref(cls, bid, nth_set_bit(got, rank - taken));
        taken += n;
    }
    w_count(h, SMMO_CNT_ALLOC_OBJ, taken);
    return mine;
}

// Wave-collective destruction of arbitrary handles (any classes, any blocks).
__device__ inline void wave_destroy(const DevHeap& h, uint64_t ref, bool want) {
    want = want && ref != 0;
    uint64_t pending = ballot(want);
    if (!pending) return;
    const uint32_t lane = lane_id();
    // group the lanes by block: the lowest lane of a group holds its mask
    uint64_t my_mask = 0, leaders = 0;
    while (pending) {
        const uint32_t leader = ctz64(pending);
        const uint64_t lref = readlane64(ref, leader);
        const bool in = ((pending >> lane) & 1) && ref_block(ref) == ref_block(lref);
        const uint64_t grp = ballot(in);
        const uint64_t mask = wave_or(in ? (1ull << ref_slot(ref)) : 0ull);
        if (lane == leader) my_mask = mask;
        leaders |= 1ull << leader;
        w_count(h, SMMO_CNT_FREE_OBJ, popc64(grp));
        pending &= ~grp;
    }
    // the groups' ANDs touch different blocks: one per leader lane, all in flight together
    const bool lead = (leaders >> lane) & 1;
    uint64_t before = 0;
    if (lead) before = at_and(&h.alloc[ref_block(ref)], ~my_mask);
    // a group needs the state update when the block was full (first free
    // slot), may now hold only its padding (the slots left form a run at the
    // top of the word: a superset of "empty" that needs no per-lane class),
    // or when the AND found a slot already free
    const uint64_t left = before & ~my_mask;
    const uint64_t inv = ~left;
    const bool first = lead && before == kOnes;
    const bool full_update = lead && ((inv & (inv + 1)) == 0 || (before & my_mask) != my_mask);
    // a group whose only update is FIRST sets its block's active bit here, all
    // such groups in one atomic (their level-0 words are independent);
    // Alg. 3's set goes on one level up only for a word that was empty, and
    // a bit found still set (another wave's clear pending) takes the
    // spinning form below
    const bool quick = first && !full_update;
    const uint64_t blk = ref_block(ref);
    const uint64_t bit = 1ull << (blk & 63);
    uint64_t prev0 = bit;
    if (quick) prev0 = at_or(bm_word(h, bm_active(h, ref_cls(ref)), 0, blk >> 6), bit);
    const bool settle = quick && (prev0 == 0 || (prev0 & bit));
    // the rest runs wave-uniform, one group at a time
    for (uint64_t todo = ballot(full_update || settle); todo; todo &= todo - 1) {
        const uint32_t l = ctz64(todo);
        const uint64_t r = readlane64(ref, l);
        const uint32_t T = ref_cls(r);
        const uint64_t b = ref_block(r);
        if (!((readlane64((uint64_t)quick, l)) & 1)) {
            dealloc_update(h, T, b, readlane64(my_mask, l), readlane64(before, l));
        } else if (readlane64(prev0, l) == 0) {
            bm_set_from(h, bm_active(h, T), 1, b >> 6);          // the word was empty: its parent bit
        } else {
            bm_set_from(h, bm_active(h, T), 0, b);               // the bit was still set: spin as Alg. 3
        }
    }
}

// Wave-collective destruction of `this` in a do-all where lane = slot of one
// block: the wave's mask is the ballot itself.
__device__ inline void wave_destroy_self(const DevHeap& h, uint32_t cls, uint64_t bid, bool want) {
    const uint64_t mask = ballot(want);
    if (!mask) return;
    dealloc_mask(h, cls, bid, mask);
    w_count(h, SMMO_CNT_FREE_OBJ, popc64(mask));
}

// Bounded message-passing check of initialize_block against reserve_or /
// block_type on a scratch table (smmo_check_publish_order).  Workgroups
// alternate roles, so writers and readers share every XCD (a workgroup runs
// on XCD blockIdx mod 8) and a reader's random blocks are mostly written on
// other XCDs.  out: [0] samples, [1] re-initialized words seen, [2]
// violations, [3] first violation (block << 32 | type).
__global__ __launch_bounds__(256) void k_check_publish(DevHeap h, uint32_t blocks, uint32_t rounds, uint64_t seed,
                                                        unsigned long long* out) {
    const uint32_t rank = (blockIdx.x >> 1) * (blockDim.x >> 6) + (threadIdx.x >> 6);   // wave within its role
    const uint32_t nrole = (gridDim.x >> 1) * (blockDim.x >> 6);
    if ((blockIdx.x & 1) == 0) {
        for (uint32_t k = 1; k <= rounds; ++k)
            for (uint64_t b = rank; b < blocks; b += nrole) initialize_block(h, k, b, (uint64_t)k << 32);
        return;
    }
    uint64_t s = uni64(splitmix64(seed ^ ((uint64_t)rank << 20)));
    unsigned long long samples = 0, fresh = 0;
    const uint64_t n = 2ull * rounds * ((blocks + nrole - 1) / nrole);
    for (uint64_t j = 0; j < n; ++j) {
        if ((j & 63) == 0 && w_load(reinterpret_cast<const uint64_t*>(&out[2])) != 0) break;
        s = splitmix64(s);
        const uint64_t b = s % blocks;
        const uint64_t before = reserve_or(h, b, 1ull << (j & 31));
        const uint32_t t = block_type(h, b);
        const uint32_t k = (uint32_t)(before >> 32);
        ++samples;
        fresh += k != 0;
        if (t < k) {
            if (is_first_lane()) {
                atomicAdd(&out[2], 1ull);
                atomicCAS(&out[3], 0ull, (unsigned long long)((b << 32) | t));
            }
            break;
        }
    }
    if (is_first_lane()) {
        atomicAdd(&out[0], samples);
        atomicAdd(&out[1], fresh);
    }
}

}  // namespace smmo
