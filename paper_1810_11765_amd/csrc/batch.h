// Batched predator-prey instances: many independent heaps advanced by one
// persistent kernel.
//
// Every admitted instance owns a contiguous range of the kernel's workgroups
// (proportional to its grid size).  The four phases of a step (fish plan,
// fish move, shark plan, shark move) run back to back inside the kernel with
// a barrier among the instance's own workgroups between phases, so instances
// never wait for each other and the whole step needs one launch for all of
// them.  The iteration snapshot each move phase needs (Sec. 3.1) is taken
// inside the preceding plan phase, block by block.  All workgroups of the
// kernel are resident at once (the host sizes the grid from the occupancy),
// so the instance barriers always complete; their spins are bounded anyway.
#pragma once

#include "methods.h"

namespace smmo {

struct BatchDesc {          // written by the host when the instance is added
    DevHeap h;
    smmo_wator_args a;      // a.step = steps already done (device-updated)
};
struct BatchProg {          // device-updated progress
    uint32_t remaining;
    uint32_t done;
};
struct BatchSched {         // host-written schedule
    uint32_t wg_begin, wg_count;
    uint32_t unit_log2;     // a phase's unit of work: 1 << unit_log2 consecutive block bits
    uint32_t pad;
};

constexpr uint32_t kBarrierSpin = 1u << 24;
constexpr uint32_t kBatchUnitLog2Max = 3;                 // at most 8 blocks per unit of work in a phase

// Barrier among the workgroups of one instance, a two-level tree: each
// workgroup arrives at the counter of its group of kBarGroup workgroups (a
// release: its stores of the phase become visible at agent scope); the last
// arrival of a group acquires them and arrives at the instance's top counter;
// the last of those opens the barrier by storing the barrier's number in a
// word of its own, which every workgroup polls with relaxed loads and
// back-off, then acquires once.  A single counter that every workgroup both
// incremented and polled cost ~0.2 ms per barrier at ~400 workgroups (the
// polls and increments of one line queue behind each other at the memory
// side); here at most kBarGroup increments meet on a group line, and the
// polled word changes once per barrier.  On gfx950 an agent-scope acquire
// invalidates the XCD's L2, so only group leaders take one on arrival.  An
// instance of a single group (most instances of a large batch) polls its
// group counter directly: the hop through the opening word would add an
// acquire and a release (an L2 invalidation and write-back) to every barrier.
// Layout of an instance's region (uint32 words, zeroed before each launch):
// [0] top counter, [32] number of the last barrier opened, [64 + 32 g] the
// counter of group g (each on its own 128-B line).
constexpr uint32_t kBarGroup = 16;
__host__ __device__ inline uint32_t bar_words(uint32_t grid) { return 64 + 32 * ((grid + kBarGroup - 1) / kBarGroup); }

__device__ inline void instance_barrier(uint32_t* bar, uint32_t number, uint32_t rank, uint32_t nwg, uint32_t* status) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t g = rank / kBarGroup;
        const uint32_t gsize = nwg - g * kBarGroup < kBarGroup ? nwg - g * kBarGroup : kBarGroup;
        const uint32_t ngroups = (nwg + kBarGroup - 1) / kBarGroup;
        uint32_t* gcnt = &bar[64 + 32 * g];
        const uint32_t old = __hip_atomic_fetch_add(gcnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        // one group: the group counter itself opens the barrier at nwg * number
        const uint32_t* poll = gcnt;
        uint32_t target = number * gsize;
        if (ngroups > 1) {
            poll = &bar[32];
            target = number;
            if (old + 1 == number * gsize) {                    // last of its group
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                const uint32_t t = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                if (t + 1 == number * ngroups) {                // last group: open the barrier
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    __hip_atomic_store(&bar[32], number, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
        }
        uint32_t spins = 0;
        while (__hip_atomic_load(poll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kBarrierSpin) {
                __hip_atomic_fetch_or(status, SMMO_STATUS_RETRY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            if (ngroups == 1 || spins < 8) __builtin_amdgcn_s_sleep(1);    // back off after the first polls
            else __builtin_amdgcn_s_sleep(4);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// One phase of one instance, spread over the instance's waves; units of
// 1 << unit_log2 block bits of allocated[cls] (the host picks the size per
// instance: 8 when its waves are few for its heap, down to 1 when it has
// waves to spare, so that a lone instance's blocks are not visited one after
// the other by a few waves).  With `snap`, each visited block's iteration
// word is set from its allocation word after the method ran (the method of a
// plan phase neither creates nor destroys objects of the class).
template <class M>
__device__ inline void batch_phase(const DevHeap& h, uint32_t cls, const smmo_wator_args& a, uint32_t wave_rank,
                                   uint32_t nwaves, uint32_t unit_log2, bool snap) {
    const uint32_t lane = lane_id();
    const uint64_t* l0 = bm_word(h, bm_allocated(cls), 0, 0);
    const uint64_t valid = ~h.cls_pad[cls];
    const uint32_t span = 1u << unit_log2, per_word_log2 = 6 - unit_log2;
    const uint64_t unit_mask = (1ull << span) - 1;
    const uint64_t nunits = h.level_words[0] << per_word_log2;
    const typename M::Prep prep = M::prepare(h, cls, a);
    // as in the do-all: lane k reads the bitmap word of the wave's k-th unit
    // (64 per round trip, with the first unit's allocation words in a plan
    // phase), and the wave visits only the units that hold blocks
    for (uint64_t base = wave_rank; base < nunits; base += 64ull * nwaves) {
        const uint64_t uk = base + (uint64_t)lane * nwaves;
        uint64_t wk = 0;
        if (uk < nunits) {
            const uint64_t w = uk >> per_word_log2;
            const uint32_t first = (uint32_t)(uk & ((1u << per_word_log2) - 1)) << unit_log2;
            wk = at_load(l0 + w * kBmStride) & (unit_mask << first);
        }
        const uint32_t first0 = (uint32_t)(base & ((1u << per_word_log2) - 1)) << unit_log2;
        const uint64_t blk0 = ((base >> per_word_log2) << 6) + first0 + lane;
        uint64_t word0 = 0;
        if (!M::kSnapshot && lane < span && blk0 < h.M) word0 = at_load(&h.alloc[blk0]);   // no block of the class appears during a plan phase
        for (uint64_t todo = ballot(wk != 0); todo; todo &= todo - 1) {
            const uint32_t k = ctz64(todo);
            const uint64_t u = base + (uint64_t)k * nwaves;
            const uint64_t w = u >> per_word_log2;
            const uint32_t first = (uint32_t)(u & ((1u << per_word_log2) - 1)) << unit_log2;
            const uint64_t my_blk = (w << 6) + first + lane;
            const bool mine = lane < span && my_blk < h.M;
            uint64_t word = readlane64(wk, k);
            uint64_t my_word = 0;
            if (!M::kSnapshot) {
                if (k == 0) my_word = word0;
                else if (mine) my_word = at_load(&h.alloc[my_blk]);
            } else {
                if (mine && ((word >> (first + lane)) & 1)) my_word = at_load(&h.iter[my_blk]);
            }
            while (word) {
                const uint32_t b = ctz64(word);
                word &= word - 1;
                const uint64_t bid = (w << 6) | b;
                const uint64_t live = (uint64_t)__shfl((unsigned long long)my_word, (int)(b - first), 64) & valid;
                Obj o{h, cls, bid, lane, ((live >> lane) & 1) != 0, h.data + bid * h.block_bytes,
                      wave_seed(((uint64_t)a.step << 20) ^ wave_rank, bid)};
                M::run(o, prep, a);
                if (snap && lane == 0) h.iter[bid] = at_load(&h.alloc[bid]) & valid;
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_batch_wator(BatchDesc* desc, BatchProg* prog, const BatchSched* sched,
                                                      const int32_t* wg_inst, uint32_t* bars, uint32_t bar_stride,
                                                      uint32_t steps) {
    const int32_t i = wg_inst[blockIdx.x];
    if (i < 0) return;                                            // idle workgroup (uniform)
    BatchDesc& D = desc[i];
    const BatchSched S = sched[i];
    const uint32_t r = blockIdx.x - S.wg_begin;
    const uint32_t todo = steps < prog[i].remaining ? steps : prog[i].remaining;
    const uint32_t done0 = prog[i].done;
    const uint32_t wave_rank = r * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t nwaves = S.wg_count * (blockDim.x >> 6);
    uint32_t nbar = 0;
    uint32_t* bar = bars + (uint64_t)i * bar_stride;
    for (uint32_t s = 0; s < todo; ++s) {
        smmo_wator_args a = D.a;
        a.step = (int32_t)(done0 + s + 1);
        batch_phase<MFishPlan>(D.h, a.fish_cls, a, wave_rank, nwaves, S.unit_log2, true);
        instance_barrier(bar, ++nbar, r, S.wg_count, D.h.status);
        batch_phase<MFishMove>(D.h, a.fish_cls, a, wave_rank, nwaves, S.unit_log2, false);
        instance_barrier(bar, ++nbar, r, S.wg_count, D.h.status);
        batch_phase<MSharkPlan>(D.h, a.shark_cls, a, wave_rank, nwaves, S.unit_log2, true);
        instance_barrier(bar, ++nbar, r, S.wg_count, D.h.status);
        batch_phase<MSharkMove>(D.h, a.shark_cls, a, wave_rank, nwaves, S.unit_log2, false);
        instance_barrier(bar, ++nbar, r, S.wg_count, D.h.status);
    }
    if (r == 0 && threadIdx.x == 0) {
        prog[i].remaining -= todo;
        prog[i].done = done0 + todo;
    }
}

// Phased form: one phase of step s of every admitted instance per launch;
// the kernel boundaries separate the phases, so no instance barrier is
// needed, and each phase's kernel holds only its own method (fewer registers,
// more waves per SIMD than the persistent kernel, which holds all four).
template <class M, bool kShark, bool kSnap>
__global__ __launch_bounds__(256)
#ifdef SMMO_PHASED_WPE
__attribute__((amdgpu_waves_per_eu(SMMO_PHASED_WPE)))
#endif
void k_batch_phase(const BatchDesc* __restrict__ desc,
                                                      const BatchProg* __restrict__ prog,
                                                      const BatchSched* __restrict__ sched,
                                                      const int32_t* __restrict__ wg_inst, uint32_t s) {
    const int32_t i = wg_inst[blockIdx.x];
    if (i < 0) return;                                            // idle workgroup (uniform)
    const BatchProg P = prog[i];
    if (s >= P.remaining) return;                                 // the instance has finished
    const BatchDesc& D = desc[i];
    const BatchSched S = sched[i];
    const uint32_t r = blockIdx.x - S.wg_begin;
    const uint32_t wave_rank = r * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const uint32_t nwaves = S.wg_count * (blockDim.x >> 6);
    smmo_wator_args a = D.a;
    a.step = (int32_t)(P.done + s + 1);
    batch_phase<M>(D.h, kShark ? a.shark_cls : a.fish_cls, a, wave_rank, nwaves, S.unit_log2, kSnap);
}
// after a phased launch group of `steps` steps: every slot's progress
__global__ void k_batch_advance(BatchProg* prog, uint32_t n, uint32_t steps) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t todo = steps < prog[i].remaining ? steps : prog[i].remaining;
    prog[i].remaining -= todo;
    prog[i].done += todo;
}

}  // namespace smmo
