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
};

constexpr uint32_t kBarrierSpin = 1u << 24;

// Barrier among the workgroups of one instance.  Arrival is a release (this
// workgroup's stores of the phase become visible at agent scope); the wait
// polls the counter with relaxed loads and acquires once, after the last
// poll: on gfx950 an agent-scope acquire invalidates the XCD's L2, so an
// acquire on every poll would evict what the other workgroups there are
// working on, once per poll.
__device__ inline void instance_barrier(uint32_t* cnt, uint32_t target, uint32_t* status) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins > kBarrierSpin) {
                __hip_atomic_fetch_or(status, SMMO_STATUS_RETRY, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// One phase of one instance, spread over the instance's waves; units of 16
// block bits of allocated[cls].  With `snap`, each visited block's iteration
// word is set from its allocation word after the method ran (the method of a
// plan phase neither creates nor destroys objects of the class).
template <class M>
__device__ inline void batch_phase(const DevHeap& h, uint32_t cls, const smmo_wator_args& a, uint32_t wave_rank,
                                   uint32_t nwaves, bool snap) {
    const uint32_t lane = lane_id();
    const uint64_t* l0 = bm_word(h, bm_allocated(cls), 0, 0);
    const uint64_t valid = ~h.cls_pad[cls];
    const uint64_t nunits = h.level_words[0] * 4;
    const typename M::Prep prep = M::prepare(h, cls, a);
    for (uint64_t u = wave_rank; u < nunits; u += nwaves) {
        const uint64_t w = u >> 2;
        const uint32_t first = (uint32_t)(u & 3) * 16;
        const uint64_t my_blk = (w << 6) + first + lane;
        const bool mine = lane < 16 && my_blk < h.M;
        uint64_t my_word = 0, word;
        if (!M::kSnapshot) {       // no block of the class appears during a plan phase
            if (mine) my_word = at_load(&h.alloc[my_blk]);
            word = at_load(l0 + w) & (0xFFFFull << first);
        } else {
            word = at_load(l0 + w) & (0xFFFFull << first);
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

__global__ __launch_bounds__(256) void k_batch_wator(BatchDesc* desc, BatchProg* prog, const BatchSched* sched,
                                                      const int32_t* wg_inst, uint32_t* bar, uint32_t steps) {
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
    for (uint32_t s = 0; s < todo; ++s) {
        smmo_wator_args a = D.a;
        a.step = (int32_t)(done0 + s + 1);
        batch_phase<MFishPlan>(D.h, a.fish_cls, a, wave_rank, nwaves, true);
        instance_barrier(&bar[i], ++nbar * S.wg_count, D.h.status);
        batch_phase<MFishMove>(D.h, a.fish_cls, a, wave_rank, nwaves, false);
        instance_barrier(&bar[i], ++nbar * S.wg_count, D.h.status);
        batch_phase<MSharkPlan>(D.h, a.shark_cls, a, wave_rank, nwaves, true);
        instance_barrier(&bar[i], ++nbar * S.wg_count, D.h.status);
        batch_phase<MSharkMove>(D.h, a.shark_cls, a, wave_rank, nwaves, false);
        instance_barrier(&bar[i], ++nbar * S.wg_count, D.h.status);
    }
    if (r == 0 && threadIdx.x == 0) {
        prog[i].remaining -= todo;
        prog[i].done = done0 + todo;
    }
}

}  // namespace smmo
