// Lock-free hierarchical bitmap (DynaSOAr Sec. 4.1, Alg. 3 and 4, App. A.5).
//
// A bitmap of M bits is ceil(M/64) 64-bit containers plus, if that is more
// than one word, a nested bitmap whose bit i is the OR of container i.  Every
// level is eventually consistent with the one below: the operation that sets
// the first bit or clears the last bit of a container is responsible for the
// parent bit and updates it with the spinning (non-try) form (Sec. 4.1.3).
//
// On gfx950 these functions run wave-uniform (dev.h): the whole wave, or a
// single lane of it, executes them on values that are the same in every
// active lane, and each atomic is performed once.  So a spin never waits on
// another lane of its own wave, which a wave64 could not schedule (lanes of
// a wave share one program counter), and the bit manipulation runs on the
// scalar unit.  Arguments are made uniform on entry (the first active lane's
// value).  Every spin is bounded: past kSpinLimit it raises SMMO_STATUS_RETRY and gives
// up, so a kernel always terminates even on a corrupted heap; once the status
// word holds RETRY (the run is already invalid) spins give up early, so the
// kernel ends soon after the first bound is hit.
#pragma once

#include "dev.h"

namespace smmo {

constexpr uint32_t kSpinLimit = 1u << 18;

__device__ inline uint64_t* bm_word(const DevHeap& h, uint32_t b, uint32_t level, uint64_t idx) {
    return h.bm + (uint64_t)b * h.bitmap_words + h.level_off[level] + idx * kBmStride;
}

// set(pos) from `level` upwards: switch the bit 0 -> 1, retrying while it is
// still 1 (a pending clear of another wave); a set-first continues one level up.
__device__ inline void bm_set_from(const DevHeap& h, uint32_t b, uint32_t level, uint64_t pos) {
    b = uni32(b);
    pos = uni64(pos);
    for (uint32_t l = uni32(level); l < h.nlevels; ++l) {
        uint64_t* w = bm_word(h, b, l, pos >> 6);
        const uint64_t bit = 1ull << (pos & 63);
        uint64_t prev = w_or(w, bit);
        uint32_t spins = 0;
        while (prev & bit) {
            if (++spins > kSpinLimit) { w_guard_hit(h, SMMO_CNT_GUARD_SPIN, SMMO_STATUS_RETRY); return; }
            if ((spins & 255) == 0 && w_status_has(h, SMMO_STATUS_RETRY)) return;
            w_count(h, SMMO_CNT_SPIN);
            backoff();
            prev = w_or(w, bit);
        }
        if (prev != 0) return;          // not the first bit of the container
        pos >>= 6;
    }
}

// clear(pos) from `level` upwards (spinning form).
__device__ inline void bm_clear_from(const DevHeap& h, uint32_t b, uint32_t level, uint64_t pos) {
    b = uni32(b);
    pos = uni64(pos);
    for (uint32_t l = uni32(level); l < h.nlevels; ++l) {
        uint64_t* w = bm_word(h, b, l, pos >> 6);
        const uint64_t bit = 1ull << (pos & 63);
        uint64_t prev = w_and(w, ~bit);
        uint32_t spins = 0;
        while (!(prev & bit)) {
            if (++spins > kSpinLimit) { w_guard_hit(h, SMMO_CNT_GUARD_SPIN, SMMO_STATUS_RETRY); return; }
            if ((spins & 255) == 0 && w_status_has(h, SMMO_STATUS_RETRY)) return;
            w_count(h, SMMO_CNT_SPIN);
            backoff();
            prev = w_and(w, ~bit);
        }
        if (prev != bit) return;        // container still has other bits (popc(prev) > 1)
        pos >>= 6;
    }
}

__device__ inline void bm_set(const DevHeap& h, uint32_t b, uint64_t pos) { bm_set_from(h, b, 0, pos); }
__device__ inline void bm_clear(const DevHeap& h, uint32_t b, uint64_t pos) { bm_clear_from(h, b, 0, pos); }

// try_clear(pos) (Alg. 3): one atomic AND; true if this call cleared the bit.
__device__ inline bool bm_try_clear(const DevHeap& h, uint32_t b, uint64_t pos) {
    b = uni32(b);
    pos = uni64(pos);
    uint64_t* w = bm_word(h, b, 0, pos >> 6);
    const uint64_t bit = 1ull << (pos & 63);
    const uint64_t prev = w_and(w, ~bit);
    if (!(prev & bit)) return false;
    if (prev == bit && h.nlevels > 1) bm_clear_from(h, b, 1, pos >> 6);
    return true;
}

// A set bit of w (w != 0) chosen uniformly by the 32 random bits r: the
// spreading that Sec. 4.2's bitmap rotation provides.
__device__ inline uint32_t pick_set_bit(uint64_t w, uint32_t r) {
    return nth_set_bit(w, (uint32_t)(((uint64_t)r * popc64(w)) >> 32));
}

// The paper's spreading (Sec. 4.2): the find-first-set starts at a bit that
// depends on the wave and the retry (the word rotated right by r & 63), so
// that waves spread over a word's set bits (SMMO_TUNE_ROTATED_START).
__device__ inline uint32_t pick_rotated(uint64_t w, uint32_t r) {
    const uint32_t rot = r & 63;
    return (ctz64(rotr64(w, rot)) + rot) & 63;
}
// the set bit of w (w != 0) a lookup takes, by the heap's tuning
__device__ inline uint32_t pick_bit(const DevHeap& h, uint64_t w, uint32_t r) {
    if (h.tune & SMMO_TUNE_NO_ROTATE) return ctz64(w);
    if (h.tune & SMMO_TUNE_ROTATED_START) return pick_rotated(w, r);
    return pick_set_bit(w, r);
}

// try_find_set() (Alg. 4), top-down from the single top word.  Where the
// paper rotates the start of each level's find-first-set (Sec. 4.2), this
// picks one of the word's set bits uniformly: the same spreading of waves
// over the bits, without favouring bits that follow a long run of zeros.
// `seed` gives different random bits per level; it depends on the wave and
// changes per retry.  Without rotation (ablation), the first set bit.
__device__ inline uint64_t bm_try_find_set(const DevHeap& h, uint32_t b, uint64_t seed) {
    b = uni32(b);
    seed = uni64(seed);
    if (h.tune & SMMO_TUNE_FORCE_FAIL) {
        if ((uint32_t)(splitmix64(seed) % 1000000u) < h.force_fail_ppm) return kFail;
    }
    uint64_t idx = 0;
    for (int l = (int)h.nlevels - 1; l >= 0; --l) {
        const uint64_t w = w_load(bm_word(h, b, (uint32_t)l, idx));
        if (!w) return kFail;
        idx = (idx << 6) | pick_bit(h, w, (uint32_t)(seed >> (6 * l)));
    }
    return idx;
}

// try_find_set() for a bitmap expected to be dense at level 0 (the active
// blocks of a class): with three or more levels, two random level-0 words are
// read first, by two lanes in one round trip (instead of one per level), and a
// set bit of a non-empty one is returned; only if both are empty does the
// top-down search run.  A set bit found this way is as valid as one found
// top-down (both come from reads that may be stale).
__device__ inline uint64_t bm_try_find_set_dense(const DevHeap& h, uint32_t b, uint64_t seed) {
    b = uni32(b);
    seed = uni64(seed);
    if (!(h.tune & (SMMO_TUNE_NO_ROTATE | SMMO_TUNE_FORCE_FAIL)) && h.nlevels >= 3 &&
        __builtin_amdgcn_read_exec() == kOnes) {
        const uint64_t r = splitmix64(seed ^ 0x5bd1e995ull);
        const uint32_t lane = lane_id();
        const uint64_t j = lane < 2 ? (((uint64_t)(uint32_t)(r >> (32 * lane)) * h.level_words[0]) >> 32) : 0;
        const uint64_t wl = lane < 2 ? at_load(bm_word(h, b, 0, j)) : 0;
        const uint64_t nz = ballot(wl != 0);
        if (nz) {
            const uint32_t i = nz == 3 ? (uint32_t)(seed >> 63) : ctz64(nz);
            return (readlane64(j, i) << 6) | pick_bit(h, readlane64(wl, i), (uint32_t)seed);
        }
    }
    return bm_try_find_set(h, b, seed);
}

// clear(): find and clear any set bit; kFail if a lookup finds none.  A
// lost race for the bit found backs off before the next lookup.
__device__ inline uint64_t bm_clear_any(const DevHeap& h, uint32_t b, uint64_t& seed) {
    seed = uni64(seed);
    for (uint32_t tries = 0; tries < 64; ++tries) {
        seed = splitmix64(seed);
        const uint64_t i = bm_try_find_set(h, b, seed);
        if (i == kFail) return kFail;
        if (bm_try_clear(h, b, i)) return i;
        backoff();
    }
    return kFail;
}

// The top word of bitmap b is empty, i.e. no bit is set (up to the sets and
// clears in flight).  A lookup that fails while the top word still has bits
// met a stale upper-level bit: contention, not an empty bitmap.
__device__ inline bool bm_top_empty(const DevHeap& h, uint32_t b) {
    return w_load(bm_word(h, uni32(b), h.nlevels - 1, 0)) == 0;
}

}  // namespace smmo
