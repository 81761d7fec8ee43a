// Kernels of the SMMO heap: heap initialization, iteration snapshot,
// parallel do-all, parallel_new, device-side allocation, live counting.
#pragma once

#include "alloc.h"

namespace smmo {

constexpr uint32_t kBlockThreads = 256;   // 4 waves per workgroup

__device__ inline uint64_t global_wave() {
    return ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
}
__device__ inline uint64_t wave_seed(uint64_t a, uint64_t b) {
    return splitmix64((a << 24) ^ b ^ 0x5deece66dull);
}

// ------------------------------------------------------------------ init ----
// Per-block words: type none, allocation word all ones (Q: a never-used block
// looks invalidated, so a stale pick fails), iteration word 0.
__global__ void k_init_blocks(DevHeap h) {
    uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= h.M) return;
    h.type[b] = kNoType;
    h.alloc[b] = kOnes;
    h.iter[b] = 0;
}

// Bitmap words: free = all M bits set (every level consistent), allocated[*]
// and active[*] empty.  One thread per word of the bitmap area.
__global__ void k_init_bitmaps(DevHeap h, uint64_t nwords_total) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nwords_total) return;
    uint64_t b = i / h.bitmap_words, off = i % h.bitmap_words;
    uint64_t v = 0;
    if (b == bm_free()) {
        uint64_t nbits = h.M;
#pragma unroll
        for (uint32_t l = 0; l < SMMO_MAX_LEVELS; ++l) {
            if (l < h.nlevels && off >= h.level_off[l] && off < h.level_off[l] + h.level_words[l] * kBmStride &&
                (off - h.level_off[l]) % kBmStride == 0) {
                uint64_t k = (off - h.level_off[l]) / kBmStride;
                uint64_t lo = k * 64;
                v = nbits >= lo + 64 ? kOnes : (nbits > lo ? ((1ull << (nbits - lo)) - 1) : 0);
            }
            nbits = h.level_words[l];
        }
    }
    h.bm[i] = v;
    if (i == 0) {
        *h.status = 0;
        for (int c = 0; c < SMMO_CNT_NUM; ++c) h.counters[c] = 0;
    }
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n, uint64_t v) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------- hierarchical enumeration ----
// Block ids of every set bit of bitmap `bmid`, found through level 1 (Alg. 5 /
// Sec. 4.1.5: level-0 words whose level-1 bit is clear are never read),
// appended in any order to R[]; *count must be 0 on entry.  Each wave
// takes kEnumPerWave consecutive level-1 words (their loads in flight
// together), lane l reading child word 64j + l of each; a workgroup reserves
// its range of R with one atomic (the reservations of one counter queue at
// the memory side, one per arriving request).  Used for big heaps so that a
// do-all costs the class's blocks, not the heap's size (Sec. 6.5).
constexpr uint32_t kEnumPerWave = 8;
__global__ __launch_bounds__(256) void k_enum_blocks(DevHeap h, uint32_t bmid, uint32_t* R,
                                                     unsigned long long* count) {
    __shared__ uint32_t wave_total[4];
    __shared__ unsigned long long wg_base;
    const uint32_t lane = lane_id(), wv = threadIdx.x >> 6;
    const uint64_t nw1 = h.level_words[1];
    const uint64_t j0 = ((uint64_t)blockIdx.x * 4 + wv) * kEnumPerWave;
    uint64_t w0[kEnumPerWave];
    uint32_t n = 0;
#pragma unroll
    for (uint32_t k = 0; k < kEnumPerWave; ++k) {
        w0[k] = 0;
        const uint64_t j = j0 + k;
        if (j < nw1) {
            const uint64_t w1 = *bm_word(h, bmid, 1, j);
            if ((w1 >> lane) & 1) w0[k] = *bm_word(h, bmid, 0, (j << 6) | lane);
        }
        n += popc64(w0[k]);
    }
    uint32_t incl = n;                                    // inclusive prefix of n in the wave
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o) incl += y;
    }
    if (lane == 63) wave_total[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t t = wave_total[0] + wave_total[1] + wave_total[2] + wave_total[3];
        wg_base = t ? atomicAdd(count, (unsigned long long)t) : 0;
    }
    __syncthreads();
    uint64_t pos = wg_base + incl - n;
    for (uint32_t k = 0; k < wv; ++k) pos += wave_total[k];
#pragma unroll
    for (uint32_t k = 0; k < kEnumPerWave; ++k) {
        const uint64_t child = ((j0 + k) << 6) | lane;
        uint64_t w = w0[k];
        while (w) {
            R[pos++] = (uint32_t)((child << 6) | ctz64(w));
            w &= w - 1;
        }
    }
}

// --------------------------------------------------- iteration snapshot ----
// iter <- alloc (without padding) for every allocated block of `cls`, before
// a do-all whose method may create objects of its own class (Sec. 3.1).
// Direct form: one thread per block.  List form (big heaps): one thread per
// block of the list k_enum_blocks wrote.
__global__ void k_snapshot(DevHeap h, uint32_t cls, const uint32_t* R, const unsigned long long* nR) {
    const uint64_t valid = ~h.cls_pad[cls];
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!R) {
        if (i >= h.M) return;
        uint64_t w = *bm_word(h, bm_allocated(cls), 0, i >> 6);
        if ((w >> (i & 63)) & 1) h.iter[i] = h.alloc[i] & valid;
        return;
    }
    const uint64_t n = *nR;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t e = i; e < n; e += stride) {
        const uint64_t b = R[e];
        h.iter[b] = h.alloc[b] & valid;
    }
}

// ----------------------------------------------------------- do-all ----
// Per-lane view of the object in (block, slot = lane).
struct Obj {
    const DevHeap& h;
    uint32_t cls;
    uint64_t bid;
    uint32_t lane;
    bool live;          // slot enumerated by this do-all
    uint8_t* base;      // block data segment
    uint64_t seed;      // per-wave seed for allocator rotations
    template <class F>
    __device__ F& at(uint32_t off) const { return *reinterpret_cast<F*>(base + off + lane * sizeof(F)); }
    __device__ uint64_t self() const { return make_ref(cls, bid, lane); }
    // device-side new, wave-collective; `salt` varies the allocator's random
    // picks between calls of one method
    __device__ __forceinline__ uint64_t alloc(uint32_t c, bool want, uint64_t salt = 0) const {
        return wave_alloc(h, c, want, seed ^ salt);
    }
};

// Parallel do-all (Sec. 3.7), enumeration fused in: the L0 words of
// allocated[cls] are cut into units of 64 >> s_log2 block bits; a wave takes
// units grid-stride (the bitmap words of up to 64 of them in one round trip),
// walks the set bits of each in ascending order (the bitmap scan is the
// compaction) and runs the method on each block with lane = slot, so
// every field access of the wave is one contiguous SOA segment.  Objects the
// method creates are not visited: with M::kSnapshot the wave reads the
// iteration word written by k_snapshot (blocks initialized meanwhile have it
// zeroed), otherwise no object of the class can appear during the do-all and
// the allocation word itself is the snapshot.
// With a block list (big heaps, from k_enum_blocks) a unit is a run of list
// entries instead: lane l loads entry l of the run and that block's word, and
// the wave then walks the run; the run length grows with the list so that
// there are at most 16,384 units.
// kSnap: read the iteration words of k_snapshot (always so when the do-all
// covers a class and its subclasses, whose methods may create objects of any
// of them).  kRecord (methods that create and destroy no object of any class,
// RecordsSnapshot below): after the method ran on a block, its lane 0 stores
// the block's live slots as its iteration word, so the class's snapshot is
// taken in passing and the next do-all that needs one skips the k_snapshot
// pass.
template <class M>
struct RecordsSnapshot {
    template <class T> static constexpr bool test(decltype(T::kRecordSnapshot)*) { return T::kRecordSnapshot; }
    template <class T> static constexpr bool test(...) { return false; }
    static constexpr bool value = test<M>(nullptr);
};
template <class M, bool kSnap = M::kSnapshot, bool kRecord = false>
__global__ __launch_bounds__(kBlockThreads) void k_doall(DevHeap h, uint32_t cls, uint32_t s_log2,
                                                          uint64_t nunits, const uint32_t* R,
                                                          const unsigned long long* nR, typename M::Args a) {
    const uint32_t lane = lane_id();
    const uint64_t wave = global_wave();
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint64_t* l0 = bm_word(h, bm_allocated(cls), 0, 0);
    const uint64_t valid = ~h.cls_pad[cls];
    const uint32_t span = 64u >> s_log2;
    const uint64_t span_mask = span == 64 ? kOnes : ((1ull << span) - 1);
    const typename M::Prep prep = M::prepare(h, cls, a);
    if (R) {
        const uint64_t n = *nR;
        uint32_t rl = 0;                                  // run length 1 << rl
        while (rl < 6 && (n >> rl) > 16384) ++rl;
        const uint64_t runs = (n + (1ull << rl) - 1) >> rl;
        for (uint64_t u = wave; u < runs; u += nwaves) {
            const uint64_t e0 = u << rl;
            const uint32_t len = n - e0 < (1ull << rl) ? (uint32_t)(n - e0) : (1u << rl);
            uint64_t my_blk = 0, my_word = 0;
            if (lane < len) {
                my_blk = R[e0 + lane];
                // a listed block stays allocated to the class, and its
                // iteration word unchanged, until its own wave has visited it
                // (a method destroys only its own object), so the word is
                // read right away
                my_word = kSnap ? h.iter[my_blk] : h.alloc[my_blk];
            }
            for (uint32_t k = 0; k < len; ++k) {
                const uint64_t bid = (uint64_t)__shfl((unsigned long long)my_blk, (int)k, 64);
                const uint64_t live = (uint64_t)__shfl((unsigned long long)my_word, (int)k, 64) & valid;
                Obj o{h, cls, bid, lane, ((live >> lane) & 1) != 0, h.data + bid * h.block_bytes,
                      wave_seed(wave, bid)};
                M::run(o, prep, a);
                if (kRecord && lane == 0) h.iter[bid] = live;
            }
        }
        return;
    }
    // The wave's units are wave + k * nwaves.  Lane k reads the bitmap word
    // of the k-th (64 units per round trip), so a unit with no block of the
    // class costs nothing more and a small grid does not pay a dependent load
    // per empty unit; the wave then visits the units that hold blocks.
    for (uint64_t base = wave; base < nunits; base += 64 * nwaves) {
        const uint64_t uk = base + (uint64_t)lane * nwaves;
        uint64_t wk = 0;
        if (uk < nunits) {
            const uint64_t w = uk >> s_log2;
            const uint32_t first = (uint32_t)(uk & ((1u << s_log2) - 1)) * span;
            wk = (kSnap ? at_load(l0 + w * kBmStride) : l0[w * kBmStride]) & (span_mask << first);
        }
        // the first unit's allocation words travel with the bitmap words: the
        // class gains no block during this do-all and a block leaves only
        // through its own wave, so they are current, and the words of blocks
        // whose bit is clear are never used
        const uint32_t first0 = (uint32_t)(base & ((1u << s_log2) - 1)) * span;
        const uint64_t blk0 = ((base >> s_log2) << 6) + first0 + lane;
        uint64_t word0 = 0;
        if (!kSnap && lane < span && blk0 < h.M) word0 = h.alloc[blk0];
        for (uint64_t todo = ballot(wk != 0); todo; todo &= todo - 1) {
            const uint32_t k = ctz64(todo);
            const uint64_t u = base + (uint64_t)k * nwaves;
            const uint64_t w = u >> s_log2;
            const uint32_t first = (uint32_t)(u & ((1u << s_log2) - 1)) * span;   // first block bit of the unit
            const uint64_t my_blk = (w << 6) + first + lane;                       // lane l: block first + l
            const bool mine = lane < span && my_blk < h.M;
            uint64_t word = readlane64(wk, k);
            uint64_t my_word = 0;
            if (!kSnap) {
                if (k == 0) my_word = word0;
                else if (mine) my_word = h.alloc[my_blk];
            } else {
                // blocks may be (re)initialized meanwhile: the iteration words
                // of the bits the bitmap word showed (a block initialized
                // since has its word zeroed)
                if (mine && ((word >> (first + lane)) & 1)) my_word = at_load(&h.iter[my_blk]);
            }
            while (word) {
                const uint32_t b = ctz64(word);
                word &= word - 1;
                const uint64_t bid = (w << 6) | b;
                const uint64_t live = (uint64_t)__shfl((unsigned long long)my_word, (int)(b - first), 64) & valid;
                Obj o{h, cls, bid, lane, ((live >> lane) & 1) != 0, h.data + bid * h.block_bytes,
                      wave_seed(wave, bid)};
                M::run(o, prep, a);
                if (kRecord && lane == 0) h.iter[bid] = live;
            }
        }
    }
}

// ------------------------------------------------------ parallel_new ----
// The first `nb` set bits of block bitmap `bmid` in ascending order -> R[0..nb)
// (Sec. 3.7, the ordered compaction of Fig. "scan_enumeration"); *found =
// how many were written.  parallel_new uses it on the free bitmap, the n-body
// force phase on allocated[T].
// One workgroup; each thread scans a contiguous range of L0 words.
__global__ __launch_bounds__(1024) void k_enum(DevHeap h, uint32_t bmid, uint64_t nb, uint32_t* R,
                                                    unsigned long long* found) {
    __shared__ unsigned long long wsum[16];
    __shared__ unsigned long long total_s;
    const uint32_t t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const uint64_t W0 = (h.M + 63) >> 6;
    const uint64_t per = (W0 + 1023) / 1024;
    const uint64_t lo = (uint64_t)t * per, hi = lo + per < W0 ? lo + per : W0;
    const uint64_t* l0 = bm_word(h, bmid, 0, 0);
    unsigned long long cnt = 0;
    for (uint64_t i = lo; i < hi; ++i) cnt += popc64(l0[i * kBmStride]);
    // inclusive scan inside the wave
    unsigned long long inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        unsigned long long y = __shfl_up(inc, o, 64);
        if (lane >= (uint32_t)o) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    if (t == 0) {
        unsigned long long s = 0;
        for (int i = 0; i < 16; ++i) { unsigned long long v = wsum[i]; wsum[i] = s; s += v; }
        total_s = s;
    }
    __syncthreads();
    unsigned long long off = wsum[wv] + inc - cnt;
    for (uint64_t i = lo; i < hi && off < nb; ++i) {
        uint64_t w = l0[i * kBmStride];
        while (w && off < nb) {
            R[off++] = (uint32_t)((i << 6) | ctz64(w));
            w &= w - 1;
        }
    }
    if (t == 0) *found = total_s < nb ? total_s : nb;
}

// Fill block rank j (one wave per block) with objects j*N .. j*N+cnt-1.
template <class C>
__global__ __launch_bounds__(kBlockThreads) void k_new_fill(DevHeap h, uint32_t cls, uint64_t n,
                                                             const uint32_t* R, const unsigned long long* found,
                                                             typename C::Args a) {
    const uint32_t lane = lane_id();
    const uint64_t j = global_wave();
    const uint32_t N = h.cls_cap[cls];
    const uint64_t nb = (n + N - 1) / N;
    if (j >= nb) return;                                  // wave-uniform
    if (*found < nb) {
        if (j == 0 && lane == 0) set_status(h, SMMO_STATUS_OOM);
        return;
    }
    const uint64_t bid = R[j];
    const uint64_t rem = n - j * N;
    const uint32_t cnt = rem < N ? (uint32_t)rem : N;
    if (lane == 0) {
        const uint64_t live = cnt == 64 ? kOnes : ((1ull << cnt) - 1);
        at_store32(&h.type[bid], cls);
        at_store(&h.iter[bid], 0);
        at_store_ordered(&h.alloc[bid], h.cls_pad[cls] | live);
        bm_clear(h, bm_free(), bid);
        bm_set(h, bm_allocated(cls), bid);
        if (cnt < N) bm_set(h, bm_active(h, cls), bid);
    }
    if (lane < cnt) C::run(h, cls, bid, lane, j * N + lane, make_ref(cls, bid, lane), a);
}

// --------------------------------------------- device-side allocation ----
// nthreads threads each allocate `per` objects in sequence; object of thread
// t, call k gets constructor index t*per + k.
template <class C>
__global__ __launch_bounds__(kBlockThreads) void k_alloc(DevHeap h, uint32_t cls, uint64_t nthreads,
                                                          uint32_t per, typename C::Args a) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t wave = global_wave();
    if ((wave << 6) >= nthreads) return;                 // wave-uniform
    const bool act = tid < nthreads;
    for (uint32_t k = 0; k < per; ++k) {
        uint64_t ref = wave_alloc(h, cls, act, wave_seed(wave, k));
        if (act && ref) C::run(h, cls, ref_block(ref), ref_slot(ref), tid * per + k, ref, a);
    }
}

// ------------------------------------------------ device-side destroy ----
// Thread t destroys refs[t*per + k] for k = 0..per-1 in sequence; lanes of a
// wave whose handles share a block are combined (wave_destroy).
__global__ __launch_bounds__(kBlockThreads) void k_destroy(DevHeap h, const uint64_t* refs, uint64_t nthreads,
                                                            uint32_t per) {
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((global_wave() << 6) >= nthreads) return;         // wave-uniform
    const bool act = tid < nthreads;
    for (uint32_t k = 0; k < per; ++k) {
        const uint64_t r = act ? refs[tid * per + k] : 0;
        wave_destroy(h, r, act);
    }
}

// ------------------------------------------------------------ counting ----
// Live objects of `cls` -> *out (added).  Direct form: one thread per block;
// list form: one thread per listed block.
__global__ void k_live_count(DevHeap h, uint32_t cls, const uint32_t* R, const unsigned long long* nR,
                             unsigned long long* out) {
    uint32_t c = 0;
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (!R) {
        if (i < h.M) {
            uint64_t w = *bm_word(h, bm_allocated(cls), 0, i >> 6);
            if ((w >> (i & 63)) & 1) c = popc64(h.alloc[i] & ~h.cls_pad[cls]);
        }
    } else {
        const uint64_t n = *nR;
        const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
        for (uint64_t e = i; e < n; e += stride) c += popc64(h.alloc[R[e]] & ~h.cls_pad[cls]);
    }
    c = wave_add(c);
    if (lane_id() == 0 && c) atomicAdd(out, (unsigned long long)c);
}

// Per-class slot occupancy (the fragmentation measure): out[3c] += live
// objects, out[3c+1] += N_c per block, out[3c+2] += blocks, over every block
// whose free bit is clear (at rest such a block belongs to class type[b]).
__global__ void k_occupancy(DevHeap h, unsigned long long* out) {
    const uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t t = kNoType, used = 0;
    if (b < h.M && !((*bm_word(h, bm_free(), 0, b >> 6) >> (b & 63)) & 1)) {
        t = h.type[b];
        if (t < h.ncls) used = popc64(h.alloc[b] & ~h.cls_pad[t]);
    }
    for (uint32_t c = 0; c < h.ncls; ++c) {
        const uint32_t nb = (uint32_t)popc64(ballot(t == c));
        if (!nb) continue;                                  // wave-uniform
        const uint32_t u = wave_add(t == c ? used : 0u);
        if (lane_id() == 0) {
            atomicAdd(out + 3 * c, (unsigned long long)u);
            atomicAdd(out + 3 * c + 1, (unsigned long long)nb * h.cls_cap[c]);
            atomicAdd(out + 3 * c + 2, (unsigned long long)nb);
        }
    }
}

// ------------------------------------------------------- measurement ----
// Atomic-throughput reference: `rounds` agent-scope 64-bit ORs per thread on
// word (t / lanes_per_word) % nwords; the returned values are folded into one
// store per wave so that no OR can be dropped.
__global__ __launch_bounds__(kBlockThreads) void k_atomic_probe(unsigned long long* words, uint64_t nwords,
                                                                 uint32_t lanes_per_word, uint64_t nthreads,
                                                                 uint32_t rounds) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((global_wave() << 6) >= nthreads) return;          // wave-uniform
    uint64_t acc = 0;
    if (t < nthreads) {
        uint64_t* w = reinterpret_cast<uint64_t*>(words) + (t / lanes_per_word) % nwords;
        for (uint32_t r = 0; r < rounds; ++r) acc ^= at_or(w, 1ull << ((t + r) & 63));
    }
    acc = wave_or(acc);
    if (lane_id() == 0 && acc == 0x5bd1e995ull) words[0] = acc;   // practically never taken
}

// VALU issue-cost reference (not part of the method): eight independent
// chains of one instruction kind per lane, `iters` times, all operands in
// vector registers (the forms the force kernel issues); kind 0 FP32 add,
// 1 FP32 multiply-add into the chain (fmac), 2 hardware square root,
// 3 hardware reciprocal.  The chains' ends are folded into one store so that
// nothing is optimized away.
__global__ __launch_bounds__(256) void k_valu_probe(float* out, uint32_t kind, uint32_t iters, float c0) {
    float v[8];
    for (int k = 0; k < 8; ++k) v[k] = 1.0f + (float)(threadIdx.x + k) * 0x1p-12f;
    const float c = c0 + (float)(threadIdx.x % 3) * 0x1p-30f;      // per-lane, so it lives in a vector register
    const float d = 0x1p-20f * c;
    switch (kind) {
        case 0: for (uint32_t i = 0; i < iters; ++i) for (int k = 0; k < 8; ++k) v[k] = v[k] + c; break;
        case 1: for (uint32_t i = 0; i < iters; ++i) for (int k = 0; k < 8; ++k) v[k] = __builtin_fmaf(c, d, v[k]); break;
        case 2: for (uint32_t i = 0; i < iters; ++i) for (int k = 0; k < 8; ++k) v[k] = __builtin_amdgcn_sqrtf(v[k]); break;
        default: for (uint32_t i = 0; i < iters; ++i) for (int k = 0; k < 8; ++k) v[k] = __builtin_amdgcn_rcpf(v[k]); break;
    }
    out[(uint64_t)blockIdx.x * blockDim.x + threadIdx.x] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
}

// -------------------------------------------------------- constructors ----
struct CtorZero {
    struct Args { uint64_t unused; };
    __device__ static void run(const DevHeap& h, uint32_t cls, uint64_t bid, uint32_t slot, uint64_t,
                               uint64_t, const Args&) {
        const uint32_t nf = (uint32_t)h.hdr->nfields[cls];
        for (uint32_t f = 0; f < nf; ++f) {
            uint8_t* p = field_addr(h, cls, bid, slot, f);
            switch (h.hdr->field_bytes[cls][f]) {
                case 1: *p = 0; break;
                case 2: *reinterpret_cast<uint16_t*>(p) = 0; break;
                case 4: *reinterpret_cast<uint32_t*>(p) = 0; break;
                default: *reinterpret_cast<uint64_t*>(p) = 0; break;
            }
        }
    }
};

struct CtorNone {
    using Args = smmo_ctor_none;
    __device__ static void run(const DevHeap&, uint32_t, uint64_t, uint32_t, uint64_t i, uint64_t ref,
                               const Args& a) {
        if (a.ref_out) a.ref_out[i] = ref;
    }
};

struct CtorArrays {
    using Args = smmo_ctor_arrays;
    __device__ static void run(const DevHeap& h, uint32_t cls, uint64_t bid, uint32_t slot, uint64_t i,
                               uint64_t ref, const Args& a) {
        const uint32_t nf = (uint32_t)h.hdr->nfields[cls];
        for (uint32_t f = 0; f < nf; ++f) {
            uint8_t* p = field_addr(h, cls, bid, slot, f);
            const uint8_t* s = static_cast<const uint8_t*>(a.src[f]);
            switch (h.hdr->field_bytes[cls][f]) {
                case 1: *p = s ? s[i] : 0; break;
                case 2: *reinterpret_cast<uint16_t*>(p) = s ? reinterpret_cast<const uint16_t*>(s)[i] : 0; break;
                case 4: *reinterpret_cast<uint32_t*>(p) = s ? reinterpret_cast<const uint32_t*>(s)[i] : 0; break;
                default: *reinterpret_cast<uint64_t*>(p) = s ? reinterpret_cast<const uint64_t*>(s)[i] : 0; break;
            }
        }
        if (a.ref_out) a.ref_out[a.ref_index ? (uint64_t)a.ref_index[i] : i] = ref;
    }
};

}  // namespace smmo
