// Methods run by parallel do-all, one struct per method id of smmo.h.
//
// Contract of a method (Sec. 2.1): it runs on every object of its class that
// is live when the do-all starts; it may read other objects, create objects
// of any class, destroy `this` or objects of other classes.  Each run() is
// called by all 64 lanes of a wave (lane = slot of one block), live or not,
// because allocation and destruction are wave-collective.  A method writes
// no field of an object it destroys in the same do-all, so a freed slot that
// another wave re-uses at once never receives a late store from its old owner.
#pragma once

#include "kernels.h"

namespace smmo {

// y += a*x on two float32 fields, through the generic do-all (SMMO_M_AXPY_GENERIC;
// SMMO_M_AXPY runs the streaming kernel below).
struct MAxpy {
    using Args = smmo_axpy_args;
    static constexpr bool kSnapshot = false;
    struct Prep { uint32_t ox, oy; };
    __device__ static Prep prepare(const DevHeap& h, uint32_t cls, const Args& a) {
        return {h.hdr->field_off[cls][a.fx], h.hdr->field_off[cls][a.fy]};
    }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        if (o.live) {
            float& y = o.at<float>(p.oy);
            const float ax = a.a * o.at<float>(p.ox);
            y = y + ax;
        }
    }
};

// Streaming form of the same do-all for the HBM-bound sweep.  The method only
// reads and writes its own object's fields and creates / destroys nothing, so
// four blocks can share a wave: lanes 16g..16g+15 take block g of the group,
// each lane four consecutive slots with 16-byte loads and stores (one 256-B
// SOA segment per 16 lanes).  A wave owns a unit of one L0 word of
// allocated[T]; it fetches the unit's 64 allocation words with one coalesced
// load and walks the word's set bits eight blocks at a time, so eight blocks'
// loads are in flight before the first store.  Field loads and stores are
// non-temporal: every byte is touched once, and streaming them past the
// caches measured about 5% more bandwidth on MI355X.  A dead slot keeps its
// bytes (the old value is stored back), which is safe because nothing else
// writes this class's slots during the do-all.
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ inline float4 load_stream(const float4* p) {
    const f32x4 v = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline void store_stream(float4* p, const float4& v) {
    const f32x4 r = {v.x, v.y, v.z, v.w};
    __builtin_nontemporal_store(r, reinterpret_cast<f32x4*>(p));
}

template <int kGroups>
__global__ __launch_bounds__(kBlockThreads) void k_doall_axpy(DevHeap h, uint32_t cls, uint64_t nwords,
                                                               smmo_axpy_args a) {
    const uint32_t lane = lane_id();
    const uint32_t g = lane >> 4, q = lane & 15;          // block of the group, lane within it
    const uint64_t wave = global_wave();
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
    const uint64_t* l0 = bm_word(h, bm_allocated(cls), 0, 0);
    const uint64_t valid = ~h.cls_pad[cls];
    const uint32_t N = h.cls_cap[cls];
    const uint32_t ox = h.hdr->field_off[cls][a.fx], oy = h.hdr->field_off[cls][a.fy];
    const bool in_cap = 4 * q < N;
    for (uint64_t w = wave; w < nwords; w += nwaves) {
        const uint64_t word = l0[w * kBmStride];
        if (!word) continue;
        // allocation word of block w*64 + lane
        const uint64_t my_alloc = ((word >> lane) & 1) ? h.alloc[(w << 6) | lane] : 0;
        const uint32_t nb = popc64(word);
        for (uint32_t base = 0; base < nb; base += 4 * kGroups) {
            float4 xv[kGroups], yv[kGroups];
            uint32_t live4[kGroups];
            float4* py[kGroups];
#pragma unroll
            for (int u = 0; u < kGroups; ++u) {
                const uint32_t k = base + 4 * u + g;           // k-th block of the word
                const bool have = k < nb && in_cap;
                const uint32_t b = have ? nth_set_bit(word, k) : 0;
                const uint64_t live = (uint64_t)__shfl((unsigned long long)my_alloc, (int)b, 64) & valid;
                live4[u] = have ? (uint32_t)((live >> (4 * q)) & 0xF) : 0;
                uint8_t* blk = h.data + ((w << 6) | b) * h.block_bytes;
                py[u] = reinterpret_cast<float4*>(blk + oy) + q;
                if (live4[u]) {
                    xv[u] = load_stream(reinterpret_cast<const float4*>(blk + ox) + q);
                    yv[u] = load_stream(py[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < kGroups; ++u) {
                if (!live4[u]) continue;
                float4 r = yv[u];
                const uint32_t m = live4[u];
                if (m & 1) r.x = yv[u].x + a.a * xv[u].x;
                if (m & 2) r.y = yv[u].y + a.a * xv[u].y;
                if (m & 4) r.z = yv[u].z + a.a * xv[u].z;
                if (m & 8) r.w = yv[u].w + a.a * xv[u].w;
                store_stream(py[u], r);
            }
        }
    }
}

// Every object destroys itself (the deallocation kernel of the allocation
// microbenchmarks, Sec. 6.4).
struct MDestroyAll {
    struct Args { uint64_t unused; };
    static constexpr bool kSnapshot = false;
    struct Prep {};
    __device__ static Prep prepare(const DevHeap&, uint32_t, const Args&) { return {}; }
    __device__ __forceinline__ static void run(const Obj& o, const Prep&, const Args&) {
        wave_destroy_self(o.h, o.cls, o.bid, o.live);
    }
};

// Allocation at scale with partial wave requests: the first a.lanes slots of
// every block each create one object of class a.cls (memory untouched), so
// each wave asks for at most a.lanes slots and several waves share an
// active block.
struct MSpawn {
    using Args = smmo_spawn_args;
    static constexpr bool kSnapshot = false;
    struct Prep {};
    __device__ static Prep prepare(const DevHeap&, uint32_t, const Args&) { return {}; }
    __device__ __forceinline__ static void run(const Obj& o, const Prep&, const Args& a) {
        (void)o.alloc(a.cls, o.live && o.lane < a.lanes);
    }
};

// Test method: count visits per id (field 0, int32).
struct MVisit {
    using Args = smmo_visit_args;
    static constexpr bool kSnapshot = false;
    struct Prep { uint32_t oid; };
    __device__ static Prep prepare(const DevHeap& h, uint32_t cls, const Args&) {
        return {h.hdr->field_off[cls][0]};
    }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        if (o.live) atomicAdd(&a.visits[o.at<int32_t>(p.oid)], 1u);
    }
};

// Alloc microbench churn on {int32 id, f32 x, f32 v}: a selected object
// destroys itself and allocates its replacement in the same method.
struct MChurn {
    using Args = smmo_churn_args;
    static constexpr bool kSnapshot = true;     // creates objects of its own class
    struct Prep { uint32_t oid, ox, ov; };
    __device__ static Prep prepare(const DevHeap& h, uint32_t cls, const Args&) {
        return {h.hdr->field_off[cls][0], h.hdr->field_off[cls][1], h.hdr->field_off[cls][2]};
    }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        bool die = false;
        int32_t nid = 0;
        if (o.live) {
            const int32_t id = o.at<int32_t>(p.oid);
            die = (splitmix64(a.seed ^ (uint64_t)(uint32_t)id ^ (uint64_t)a.round) & 1) != 0;
            nid = (int32_t)(((uint32_t)(a.round + 1) << 18) | ((uint32_t)id & 0x3FFFFu));
        }
        wave_destroy_self(o.h, o.cls, o.bid, die);
        const uint64_t r = o.alloc(o.cls, die);
        if (die && r) {
            const uint64_t b = ref_block(r);
            const uint32_t s = ref_slot(r);
            uint8_t* base = o.h.data + b * o.h.block_bytes;
            reinterpret_cast<int32_t*>(base + p.oid)[s] = nid;
            reinterpret_cast<float*>(base + p.ox)[s] =
                unit_float(ctr_draw(a.seed, a.round + 1, (uint64_t)(uint32_t)nid, 0));
            reinterpret_cast<float*>(base + p.ov)[s] =
                unit_float(ctr_draw(a.seed, a.round + 1, (uint64_t)(uint32_t)nid, 1));
        }
    }
};

// Two-class churn: replacements land in either class, so blocks are freed
// and re-initialized to the other class while other waves still hold picks
// from the active bitmaps (type-change rollback, Alg. 1; App. A.3).
struct MMix {
    using Args = smmo_mix_args;
    static constexpr bool kSnapshot = true;
    struct Prep { uint32_t oid, oa, ob; };
    __device__ static Prep prepare(const DevHeap& h, uint32_t cls, const Args& a) {
        return {h.hdr->field_off[cls][0], h.hdr->field_off[a.cls_a][0], h.hdr->field_off[a.cls_b][0]};
    }
    __device__ static void zero_rest(const DevHeap& h, uint64_t r) {
        const uint32_t c = ref_cls(r);
        const uint32_t nf = (uint32_t)h.hdr->nfields[c];
        for (uint32_t f = 1; f < nf; ++f) {
            uint8_t* q = field_addr(h, c, ref_block(r), ref_slot(r), f);
            for (uint32_t k = 0; k < h.hdr->field_bytes[c][f]; ++k) q[k] = 0;
        }
    }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        bool die = false, to_b = false;
        int32_t nid = 0;
        if (o.live) {
            const int32_t id = o.at<int32_t>(p.oid);
            const uint64_t hsh = splitmix64(a.seed ^ (uint64_t)(uint32_t)id ^ ((uint64_t)a.round << 32));
            die = hsh & 1;
            to_b = (hsh >> 1) & 1;
            nid = (int32_t)(((uint32_t)(a.round + 1) << 18) | ((uint32_t)id & 0x3FFFFu));
        }
        wave_destroy_self(o.h, o.cls, o.bid, die);
        const uint64_t ra = o.alloc(a.cls_a, die && !to_b);
        const uint64_t rb = o.alloc(a.cls_b, die && to_b, 0x9e37ull);
        const uint64_t r = to_b ? rb : ra;
        if (die && r) {
            field_of<int32_t>(o.h, r, 0) = nid;
            zero_rest(o.h, r);
        }
    }
};

// Allocation storm on a tiny heap: many waves allocate into and free the same
// few blocks at once, so blocks empty, get invalidated, freed and
// re-initialized to the other class while other waves hold stale picks.
// A wave frees its class-a objects before it asks for class-b ones: a wave
// that waited for b while holding a could pin every spare block as a class-a
// block (hold and wait), a true out-of-memory that no allocator can resolve.
struct MStress {
    using Args = smmo_stress_args;
    static constexpr bool kSnapshot = false;
    struct Prep { uint32_t unused; };
    __device__ static Prep prepare(const DevHeap&, uint32_t, const Args&) { return {0}; }
    __device__ __forceinline__ static void run(const Obj& o, const Prep&, const Args& a) {
        const uint32_t key = (uint32_t)(o.bid * 64 + o.lane);
        for (uint32_t k = 0; k < a.iters; ++k) {
            const bool act = o.live && o.lane < a.lanes;
            const bool to_b = splitmix64(a.seed ^ ((uint64_t)key << 20) ^ k) & 1;
            const uint64_t ra = o.alloc(a.cls_a, act && !to_b, k);
            if (act && !to_b && ra) field_of<int32_t>(o.h, ra, 0) = (int32_t)key;
            wave_destroy(o.h, ra, act && !to_b && ra != 0);
            const uint64_t rb = o.alloc(a.cls_b, act && to_b, (k << 8) ^ 0x51ull);
            if (act && to_b && rb) field_of<int32_t>(o.h, rb, 0) = (int32_t)key;
            wave_destroy(o.h, rb, act && to_b && rb != 0);
        }
    }
};

// ------------------------------------------------------ Life-like grid ----
// Cell {int32 x, int32 y, int8 alive}, Agent {int32 cell, int32 age}.
struct LifePrep { uint32_t cx, cy, ca, gc, ga; };
__device__ inline LifePrep life_prep(const DevHeap& h, const smmo_life_args& a) {
    return {h.hdr->field_off[a.cell_cls][0], h.hdr->field_off[a.cell_cls][1], h.hdr->field_off[a.cell_cls][2],
            h.hdr->field_off[a.agent_cls][0], h.hdr->field_off[a.agent_cls][1]};
}
__device__ inline uint8_t life_alive_byte(const DevHeap& h, const LifePrep& p, uint64_t ref) {
    return h.data[ref_block(ref) * h.block_bytes + p.ca + ref_slot(ref)];
}

// Cell::plan: next state from the 8 neighbours' current bit (B3/S23).
struct MLifePlan {
    using Args = smmo_life_args;
    static constexpr bool kSnapshot = false;
    using Prep = LifePrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t, const Args& a) { return life_prep(h, a); }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        if (!o.live) return;
        const int32_t x = o.at<int32_t>(p.cx), y = o.at<int32_t>(p.cy);
        const int32_t W = a.width, H = a.height;
        const int32_t xm = x == 0 ? W - 1 : x - 1, xp = x == W - 1 ? 0 : x + 1;
        const int32_t ym = y == 0 ? H - 1 : y - 1, yp = y == H - 1 ? 0 : y + 1;
        const int32_t xs[3] = {xm, x, xp}, ys[3] = {ym, y, yp};
        uint32_t cnt = 0;
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                if (i == 1 && j == 1) continue;
                cnt += life_alive_byte(o.h, p, a.cell_ref[(int64_t)ys[j] * W + xs[i]]) & 1;
            }
        uint8_t& al = o.at<uint8_t>(p.ca);
        const uint8_t cur = al & 1;
        const uint8_t nxt = cur ? (cnt == 2 || cnt == 3) : (cnt == 3);
        al = (uint8_t)(cur | (nxt << 1));
    }
};

// Agent::step: die when the cell's next state is dead, otherwise age.
struct MLifeAgent {
    using Args = smmo_life_args;
    static constexpr bool kSnapshot = false;
    using Prep = LifePrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t, const Args& a) { return life_prep(h, a); }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        bool die = false;
        if (o.live) {
            const int32_t c = o.at<int32_t>(p.gc);
            die = ((life_alive_byte(o.h, p, a.cell_ref[c]) >> 1) & 1) == 0;
            if (!die) o.at<int32_t>(p.ga) += 1;
        }
        wave_destroy_self(o.h, o.cls, o.bid, die);
    }
};

// Cell::commit: a dead cell that becomes alive creates its Agent; alive <- next.
// Bit 1 keeps the next state, so Agent::step may run before, after or during
// this phase and read the same value.
struct MLifeCommit {
    using Args = smmo_life_args;
    static constexpr bool kSnapshot = false;    // creates Agents, enumerates Cells
    using Prep = LifePrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t, const Args& a) { return life_prep(h, a); }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        bool born = false;
        int32_t c = 0;
        if (o.live) {
            uint8_t& al = o.at<uint8_t>(p.ca);
            const uint8_t v = al;
            born = !(v & 1) && (v & 2);
            al = (uint8_t)((v & 2) ? 3 : 0);     // current <- next; bit 1 (next) stays for the agent phase
            c = o.at<int32_t>(p.cy) * a.width + o.at<int32_t>(p.cx);
        }
        const uint64_t r = o.alloc(a.agent_cls, born);
        if (born && r) {
            uint8_t* base = o.h.data + ref_block(r) * o.h.block_bytes;
            reinterpret_cast<int32_t*>(base + p.gc)[ref_slot(r)] = c;
            reinterpret_cast<int32_t*>(base + p.ga)[ref_slot(r)] = 0;
        }
    }
};

// ------------------------------------------------------ predator-prey ----
// Fish {int32 pos, int32 age}, Shark {int32 pos, int32 age, int32 energy}.
struct WatorPrep { uint32_t fp, fa, sp, sa, se; };
__device__ inline WatorPrep wator_prep(const DevHeap& h, const smmo_wator_args& a) {
    return {h.hdr->field_off[a.fish_cls][0], h.hdr->field_off[a.fish_cls][1], h.hdr->field_off[a.shark_cls][0],
            h.hdr->field_off[a.shark_cls][1], h.hdr->field_off[a.shark_cls][2]};
}
// element k (0..3) of a 4-array without indexed (scratch) addressing
__device__ inline int32_t pick4(const int32_t v[4], uint32_t k) {
    return k == 0 ? v[0] : k == 1 ? v[1] : k == 2 ? v[2] : v[3];
}
// neighbours N, E, S, W of cell c on the torus
__device__ inline void wator_nbrs(int32_t c, int32_t W, int32_t H, int32_t nb[4]) {
    const int32_t x = c % W, y = c / W;
    nb[0] = (y == 0 ? H - 1 : y - 1) * W + x;
    nb[1] = y * W + (x == W - 1 ? 0 : x + 1);
    nb[2] = (y == H - 1 ? 0 : y + 1) * W + x;
    nb[3] = y * W + (x == 0 ? W - 1 : x - 1);
}

struct MFishPlan {
    using Args = smmo_wator_args;
    static constexpr bool kSnapshot = false;
    static constexpr bool kRecordSnapshot = true;     // creates and destroys nothing; the move phase needs one
    using Prep = WatorPrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t, const Args& a) { return wator_prep(h, a); }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        if (!o.live) return;
        const int32_t pos = o.at<int32_t>(p.fp);
        o.at<int32_t>(p.fa) += 1;
        int32_t nb[4];
        wator_nbrs(pos, a.width, a.height, nb);
        uint32_t m = 0;                          // candidate neighbours, in N, E, S, W order
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (a.occ[nb[k]] == 0) m |= 1u << k;
        int32_t t = -1;
        if (m) {
            const uint32_t n = (uint32_t)__popc(m);
            const uint32_t i = (uint32_t)((ctr_draw(a.seed, (uint64_t)a.step, (uint64_t)pos, 1) >> 32) % n);
            t = pick4(nb, nth_set_bit(m, i));
            atomicMin(&a.claim[t], pos);
        }
        a.want[pos] = t;
    }
};

struct MFishMove {
    using Args = smmo_wator_args;
    static constexpr bool kSnapshot = true;     // creates Fish
    using Prep = WatorPrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t, const Args& a) { return wator_prep(h, a); }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        bool win = false, breed = false;
        int32_t pos = 0, t = -1;
        if (o.live) {
            pos = o.at<int32_t>(p.fp);
            t = a.want[pos];
            win = t >= 0 && a.claim[t] == pos;
            breed = win && o.at<int32_t>(p.fa) >= a.fish_breed;
        }
        const uint64_t child = o.alloc(a.fish_cls, breed);
        if (win) {
            a.claim[t] = INT32_MAX;
            a.occ[t] = o.self();
            o.at<int32_t>(p.fp) = t;
            if (breed) {
                o.at<int32_t>(p.fa) = 0;
                if (child) {
                    uint8_t* base = o.h.data + ref_block(child) * o.h.block_bytes;
                    reinterpret_cast<int32_t*>(base + p.fp)[ref_slot(child)] = pos;
                    reinterpret_cast<int32_t*>(base + p.fa)[ref_slot(child)] = 0;
                }
                a.occ[pos] = child;
            } else {
                a.occ[pos] = 0;
            }
        }
    }
};

struct MSharkPlan {
    using Args = smmo_wator_args;
    static constexpr bool kSnapshot = false;
    static constexpr bool kRecordSnapshot = true;     // creates and destroys nothing; the move phase needs one
    using Prep = WatorPrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t, const Args& a) { return wator_prep(h, a); }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        if (!o.live) return;
        const int32_t pos = o.at<int32_t>(p.sp);
        o.at<int32_t>(p.sa) += 1;
        int32_t nb[4];
        wator_nbrs(pos, a.width, a.height, nb);
        uint32_t fm = 0, em = 0;                 // fish / empty neighbours, N, E, S, W order
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t r = a.occ[nb[k]];
            if (r == 0) em |= 1u << k;
            else if (ref_cls(r) == a.fish_cls) fm |= 1u << k;
        }
        const uint32_t m = fm ? fm : em;
        int32_t t = -1;
        if (m) {
            const uint32_t n = (uint32_t)__popc(m);
            const uint32_t i = (uint32_t)((ctr_draw(a.seed, (uint64_t)a.step, (uint64_t)pos, 2) >> 32) % n);
            t = pick4(nb, nth_set_bit(m, i));
            atomicMin(&a.claim[t], pos);
        }
        a.want[pos] = t;
    }
};

struct MSharkMove {
    using Args = smmo_wator_args;
    static constexpr bool kSnapshot = true;     // creates Sharks
    using Prep = WatorPrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t, const Args& a) { return wator_prep(h, a); }
    __device__ __forceinline__ static void run(const Obj& o, const Prep& p, const Args& a) {
        bool win = false, breed = false, starve = false;
        int32_t pos = 0, t = -1, age = 0, energy = 0;
        uint64_t prey = 0;
        if (o.live) {
            pos = o.at<int32_t>(p.sp);
            age = o.at<int32_t>(p.sa);
            energy = o.at<int32_t>(p.se);
            t = a.want[pos];
            win = t >= 0 && a.claim[t] == pos;
            if (win) prey = a.occ[t];            // a fish or nothing
        }
        wave_destroy(o.h, prey, prey != 0);
        if (prey) energy += a.eat_gain;
        breed = win && age >= a.shark_breed;
        const uint64_t child = o.alloc(a.shark_cls, breed);
        energy -= 1;
        starve = o.live && energy <= 0;
        if (win) {
            a.claim[t] = INT32_MAX;
            a.occ[t] = starve ? 0 : o.self();
            if (breed) {
                age = 0;
                if (child) {
                    uint8_t* base = o.h.data + ref_block(child) * o.h.block_bytes;
                    reinterpret_cast<int32_t*>(base + p.sp)[ref_slot(child)] = pos;
                    reinterpret_cast<int32_t*>(base + p.sa)[ref_slot(child)] = 0;
                    reinterpret_cast<int32_t*>(base + p.se)[ref_slot(child)] = a.shark_e0;
                }
                a.occ[pos] = child;
            } else {
                a.occ[pos] = 0;
            }
        } else if (starve) {
            a.occ[pos] = 0;
        }
        if (o.live && !starve) {
            o.at<int32_t>(p.sp) = win ? t : pos;
            o.at<int32_t>(p.sa) = age;
            o.at<int32_t>(p.se) = energy;
        }
        wave_destroy_self(o.h, o.cls, o.bid, starve);
    }
};

}  // namespace smmo
