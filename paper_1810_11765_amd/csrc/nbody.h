// N-body with merging (DynaSOAr Sec. 1 "n-body simulation with collisions",
// Table 1 "collision"; force as in the API example of Sec. 2.1) on
// Body {f32 x, f32 y, f32 vx, f32 vy, f32 m}.
//
// A body's key is block*64 + slot.  parallel_new fills the lowest free blocks
// in ascending order and bodies are never created afterwards, so ascending
// key order is ascending creation index: every order-dependent FP32 sum below
// runs over keys in ascending order, as the sequential definition does.
#pragma once

#include "kernels.h"

namespace smmo {

struct NbPrep { uint32_t ox, oy, ovx, ovy, om; };
__device__ inline NbPrep nb_prep(const DevHeap& h, uint32_t cls) {
    return {h.hdr->field_off[cls][0], h.hdr->field_off[cls][1], h.hdr->field_off[cls][2],
            h.hdr->field_off[cls][3], h.hdr->field_off[cls][4]};
}
__device__ inline float& nb_f(const DevHeap& h, uint32_t off, uint32_t key) {
    return *reinterpret_cast<float*>(h.data + (uint64_t)(key >> 6) * h.block_bytes + off + (key & 63) * 4);
}
// cell coordinates of a position in the hashed grid (cell edge 1/inv_cell)
__device__ inline int32_t nb_cell(float v, float inv_cell) {
    float c = floorf((v + 64.0f) * inv_cell);
    c = fminf(fmaxf(c, 0.0f), 1073741823.0f);
    return (int32_t)c;
}
__device__ inline uint32_t nb_hash(int32_t cx, int32_t cy, uint32_t bits) {
    uint32_t k = (uint32_t)cx * 0x9E3779B1u ^ (uint32_t)cy * 0x85EBCA77u;
    k ^= k >> 15;
    k *= 0x2C1B3C6Du;
    k ^= k >> 13;
    return k & ((1u << bits) - 1u);
}

// INSERT: push the body on its cell's list; its component label starts as itself.
struct MNbInsert {
    using Args = smmo_nbody_args;
    static constexpr bool kSnapshot = false;
    using Prep = NbPrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t cls, const Args&) { return nb_prep(h, cls); }
    __device__ static void run(const Obj& o, const Prep& p, const Args& a) {
        if (!o.live) return;
        const int32_t key = (int32_t)(o.bid * 64 + o.lane);
        const uint32_t s = nb_hash(nb_cell(o.at<float>(p.ox), a.inv_cell), nb_cell(o.at<float>(p.oy), a.inv_cell),
                                   a.hash_bits);
        a.next[key] = atomicExch(&a.head[s], key);
        a.lab[key] = key;
    }
};

// PAIRS: every pair closer than merge_dist, found once by its lower key.
struct MNbPairs {
    using Args = smmo_nbody_args;
    static constexpr bool kSnapshot = false;
    using Prep = NbPrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t cls, const Args&) { return nb_prep(h, cls); }
    __device__ static void run(const Obj& o, const Prep& p, const Args& a) {
        if (!o.live) return;
        const int32_t key = (int32_t)(o.bid * 64 + o.lane);
        const float xi = o.at<float>(p.ox), yi = o.at<float>(p.oy);
        const int32_t cx = nb_cell(xi, a.inv_cell), cy = nb_cell(yi, a.inv_cell);
        uint32_t seen[9];
        int nseen = 0;
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const uint32_t s = nb_hash(cx + dx, cy + dy, a.hash_bits);
                bool dup = false;
                for (int q = 0; q < nseen; ++q) dup |= seen[q] == s;   // two cells, one slot
                if (dup) continue;
                seen[nseen++] = s;
                for (int32_t k = a.head[s]; k >= 0; k = a.next[k]) {
                    if (k <= key) continue;
                    const float ddx = nb_f(o.h, p.ox, (uint32_t)k) - xi;
                    const float ddy = nb_f(o.h, p.oy, (uint32_t)k) - yi;
                    const float d = sqrtf(ddx * ddx + ddy * ddy);
                    if (d < a.merge_dist) {
                        const uint32_t q = atomicAdd(a.npairs, 1u);
                        if (q < a.pair_cap) {
                            a.pairs[2 * q] = key;
                            a.pairs[2 * q + 1] = k;
                        } else {
                            set_status(o.h, SMMO_STATUS_CORRUPT);
                        }
                    }
                }
            }
    }
};

// REAP: merged bodies destroy themselves; every body clears its grid slot so
// the table is empty again for the next step.
struct MNbReap {
    using Args = smmo_nbody_args;
    static constexpr bool kSnapshot = false;
    using Prep = NbPrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t cls, const Args&) { return nb_prep(h, cls); }
    __device__ static void run(const Obj& o, const Prep& p, const Args& a) {
        bool die = false;
        if (o.live) {
            const int32_t key = (int32_t)(o.bid * 64 + o.lane);
            a.head[nb_hash(nb_cell(o.at<float>(p.ox), a.inv_cell), nb_cell(o.at<float>(p.oy), a.inv_cell),
                           a.hash_bits)] = -1;
            die = a.merged[key] != 0;
            if (die) a.merged[key] = 0;
        }
        wave_destroy_self(o.h, o.cls, o.bid, die);
    }
};

// MOVE: x += v*dt.
struct MNbMove {
    using Args = smmo_nbody_args;
    static constexpr bool kSnapshot = false;
    using Prep = NbPrep;
    __device__ static Prep prepare(const DevHeap& h, uint32_t cls, const Args&) { return nb_prep(h, cls); }
    __device__ static void run(const Obj& o, const Prep& p, const Args& a) {
        if (!o.live) return;
        float& x = o.at<float>(p.ox);
        float& y = o.at<float>(p.oy);
        const float mx = o.at<float>(p.ovx) * a.dt, my = o.at<float>(p.ovy) * a.dt;
        x = x + mx;
        y = y + my;
    }
};

// ------------------------------------------------------------- RESOLVE ----
// One workgroup: connected components of the close-pair graph by min-label
// propagation, then the merge sums in ascending key order.
constexpr uint32_t kResolveNodes = 8192;    // max distinct bodies in close pairs (pair_cap <= 4096)

__device__ inline int32_t at_load_i32(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ __launch_bounds__(1024) void k_nbody_resolve(DevHeap h, uint32_t cls, smmo_nbody_args a) {
    __shared__ int32_t nodes[kResolveNodes];
    __shared__ float ms[kResolveNodes], px[kResolveNodes], py[kResolveNodes];
    __shared__ int changed;
    __shared__ uint32_t nnodes;
    const uint32_t t = threadIdx.x;
    const uint32_t total = *a.npairs;
    const uint32_t cap = a.pair_cap < kResolveNodes / 2 ? a.pair_cap : kResolveNodes / 2;
    const uint32_t n = total < cap ? total : cap;
    if (total > cap && t == 0) set_status(h, SMMO_STATUS_CORRUPT);
    if (n == 0) {
        if (t == 0) *a.npairs = 0;
        return;
    }
    const NbPrep p = nb_prep(h, cls);
    // min-label propagation over the pairs until nothing changes
    for (uint32_t it = 0; it <= n + 1; ++it) {
        if (t == 0) changed = 0;
        __syncthreads();
        for (uint32_t q = t; q < n; q += blockDim.x) {
            const int32_t i = a.pairs[2 * q], j = a.pairs[2 * q + 1];
            const int32_t li = at_load_i32(&a.lab[i]), lj = at_load_i32(&a.lab[j]);
            const int32_t m = li < lj ? li : lj;
            if (li != m) { atomicMin(&a.lab[i], m); changed = 1; }
            if (lj != m) { atomicMin(&a.lab[j], m); changed = 1; }
        }
        __syncthreads();
        if (!changed) break;
        __syncthreads();
    }
    // distinct bodies of all pairs, ascending (bitonic sort of the endpoints)
    uint32_t m2 = 1;
    while (m2 < 2 * n) m2 <<= 1;
    for (uint32_t q = t; q < m2; q += blockDim.x) nodes[q] = q < 2 * n ? a.pairs[q] : INT32_MAX;
    __syncthreads();
    for (uint32_t k = 2; k <= m2; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t q = t; q < m2; q += blockDim.x) {
                const uint32_t r = q ^ j;
                if (r > q) {
                    const bool up = (q & k) == 0;
                    const int32_t x = nodes[q], y = nodes[r];
                    if ((x > y) == up) { nodes[q] = y; nodes[r] = x; }
                }
            }
            __syncthreads();
        }
    if (t == 0) {
        uint32_t u = 0;
        for (uint32_t q = 0; q < 2 * n; ++q)
            if (q == 0 || nodes[q] != nodes[q - 1]) nodes[u++] = nodes[q];
        nnodes = u;
        // merge sums in ascending key: the first member of a component is its
        // lowest key, i.e. its root
        for (uint32_t q = 0; q < u; ++q) {
            const uint32_t k = (uint32_t)nodes[q];
            const int32_t root = at_load_i32(&a.lab[k]);
            uint32_t lo = 0, hi = u;                  // position of the root in nodes[]
            while (lo < hi) {
                uint32_t mid = (lo + hi) >> 1;
                if (nodes[mid] < root) lo = mid + 1; else hi = mid;
            }
            const float mk = nb_f(h, p.om, k);
            const float pxk = mk * nb_f(h, p.ovx, k), pyk = mk * nb_f(h, p.ovy, k);
            if (lo == q) {
                ms[q] = mk; px[q] = pxk; py[q] = pyk;
            } else {
                ms[lo] = ms[lo] + mk; px[lo] = px[lo] + pxk; py[lo] = py[lo] + pyk;
                a.merged[k] = 1;
            }
        }
    }
    __syncthreads();
    const uint32_t u = nnodes;
    for (uint32_t q = t; q < u; q += blockDim.x) {
        const uint32_t k = (uint32_t)nodes[q];
        if (at_load_i32(&a.lab[k]) == (int32_t)k) {  // survivor: keeps its position
            nb_f(h, p.om, k) = ms[q];
            nb_f(h, p.ovx, k) = px[q] / ms[q];
            nb_f(h, p.ovy, k) = py[q] / ms[q];
        }
    }
    if (t == 0) *a.npairs = 0;
}

// ---------------------------------------------------------------- FORCE ----
// The force term of body i from body j (Listing 1 of Sec. 2.1 restated):
// s = G m_j / (d2 * sqrt(d2)), d2 = dx*dx + dy*dy, then s*dx and s*dy are
// added to i's sums in ascending key order of j.  Every operation is one
// IEEE-754 rounding (correctly rounded sqrt and division), as in the oracle.
//
// Fast forms of the correctly rounded sqrt and division, for operands in
// ranges where the general sequences' scaling and special-case steps do
// nothing.  The force kernel takes them only where a per-lane range check
// shows they apply, and the results are the IEEE results bit for bit there
// (smmo_check_force_arith checks the square root on every float of the range
// and the division on random pairs of it).
//  * sqrt, for 2^-96 <= x < +inf: the hardware square root s (within one unit
//    in the last place), then the rounding test on its neighbours: x minus
//    the product of s with the neighbour below (above) tells on which side of
//    the midpoint between them the exact root lies.
//  * division a / b, for b and a / b normal, a >= 2^-100 and a / b < 2^96: the
//    hardware reciprocal, one Newton-Raphson step on it, the quotient, then
//    two corrections by the remainder computed with a fused multiply-add
//    (Markstein's method; the same steps as the general sequence with its
//    operand scaling and final fix-up left out).
__device__ __forceinline__ float sqrt_cr_fast(float x) {
    const float s = __builtin_amdgcn_sqrtf(x);
    const float below = __uint_as_float(__float_as_uint(s) - 1u);
    const float above = __uint_as_float(__float_as_uint(s) + 1u);
    const float r_below = __builtin_fmaf(-below, s, x);
    const float r_above = __builtin_fmaf(-above, s, x);
    float r = r_below <= 0.0f ? below : s;
    r = r_above > 0.0f ? above : r;
    return r;
}
__device__ __forceinline__ float div_cr_fast(float a, float b) {
    float r = __builtin_amdgcn_rcpf(b);
    const float e = __builtin_fmaf(-b, r, 1.0f);
    r = __builtin_fmaf(e, r, r);
    float q = a * r;
    float rem = __builtin_fmaf(-b, q, a);
    q = __builtin_fmaf(rem, r, q);
    rem = __builtin_fmaf(-b, q, a);
    return __builtin_fmaf(rem, r, q);
}
// Ranges of the fast path, as float bit patterns: d2 in [2^-40, 2^40), so that
// d2 * sqrt(d2) lies in [2^-60, 2^60); G m in [2^-50, 2^30) or exactly 0 (an
// empty tile entry), so that the quotient lies in [2^-110, 2^90).
constexpr uint32_t kD2Lo = 0x2B800000u, kD2Hi = 0x53800000u;
constexpr uint32_t kGmLo = 0x26800000u, kGmHi = 0x4E800000u;
// Position of an empty tile entry: far from every body of the unit-disk
// workload, so that with G m = 0 its term is exactly +0 (adding it leaves a
// sum unchanged: a sum that starts at +0 is never -0).
constexpr float kFarPos = 1024.0f;
// Coordinates below kBox in magnitude keep every d2 of two of them at most
// 2^39 (|dx| <= 2^19 after rounding), inside the fast range's upper end, so a
// tile whose entries and bodies are all inside needs only d2's lower end
// checked per entry: the minimum of four d2 against 2^-40.
constexpr float kBox = 262144.0f;

// offset of d2's bit pattern from the range's start: the value is in the
// range iff the (unsigned) offset is below kD2Hi - kD2Lo
__device__ __forceinline__ uint32_t d2_offset(float d2) { return __float_as_uint(d2) - kD2Lo; }

// device_do over all bodies for every body (Sec. 2.1), tiled through LDS.
// R = allocated blocks of the class in ascending order (k_enum).  A workgroup
// owns four i-blocks (one per wave, lane = slot); all its waves stream the
// j-blocks of R in ascending order, kTile blocks per LDS tile, so every body
// adds its terms in ascending key order.  The tile is consumed four entries
// at a time: if every lane's four d2 are in the fast range (and every G m of
// the tile is), the four terms come from the fast sqrt and division and are
// added in order; otherwise (the body itself, an empty slot near a body, or
// operands outside the range) the four entries go through the general
// operations with each term taken or skipped by a select.  When every
// coordinate of the workgroup's bodies and of the tile is inside kBox, the
// four d2 are checked through their minimum alone.
#ifndef SMMO_NB_TILE
#define SMMO_NB_TILE 32
#endif
constexpr uint32_t kTile = SMMO_NB_TILE;
#ifndef SMMO_NB_BOX_GROUP
#define SMMO_NB_BOX_GROUP 4
#endif
constexpr uint32_t kBoxGroup = SMMO_NB_BOX_GROUP;   // tile entries per check in a boxed tile (divides 64)

__global__ __launch_bounds__(256) void k_nbody_force(DevHeap h, uint32_t cls, const uint32_t* R,
                                                      const unsigned long long* rcount, smmo_nbody_args a) {
    __shared__ float4 tile[kTile * 64];
    const uint64_t r = *rcount;
    if ((uint64_t)blockIdx.x * 4 >= r) return;          // workgroup-uniform
    const NbPrep p = nb_prep(h, cls);
    const uint64_t valid = ~h.cls_pad[cls];
    const uint32_t wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const uint64_t irank = (uint64_t)blockIdx.x * 4 + wv;
    uint32_t ib = 0;
    uint64_t ilive = 0;
    if (irank < r) {
        ib = R[irank];
        ilive = h.alloc[ib] & valid;
    }
    const bool me = (ilive >> lane) & 1;
    const uint32_t ikey = ib * 64 + lane;
    const float xi = me ? nb_f(h, p.ox, ikey) : 0.0f;
    const float yi = me ? nb_f(h, p.oy, ikey) : 0.0f;
    float sx = 0.0f, sy = 0.0f;
    const bool wg_box = __syncthreads_and(fabsf(xi) < kBox && fabsf(yi) < kBox) != 0;   // false for NaN
    // general form of one entry: skipped entries (an empty slot, or body i
    // itself) may produce inf or NaN in s, never used (a select keeps the sums)
    auto exact = [&](const float4& v) {
        const uint32_t tag = (uint32_t)__float_as_int(v.w);
        const float dx = v.x - xi, dy = v.y - yi;
        const float d2 = dx * dx + dy * dy;
        const float s = v.z / (d2 * sqrtf(d2));
        const float nx = sx + s * dx, ny = sy + s * dy;
        const bool use = tag != 0 && tag - 1 != ikey;
        sx = use ? nx : sx;
        sy = use ? ny : sy;
    };
    for (uint64_t t0 = 0; t0 < r; t0 += kTile) {
        __syncthreads();
        bool slow = false, far = false;
        for (uint32_t e = threadIdx.x; e < kTile * 64; e += blockDim.x) {
            const uint64_t jr = t0 + (e >> 6);
            const uint32_t sl = e & 63;
            float4 v = make_float4(kFarPos, kFarPos, 0.0f, 0.0f);
            if (jr < r) {
                const uint32_t jb = R[jr];
                if (((h.alloc[jb] & valid) >> sl) & 1) {
                    const uint32_t jk = jb * 64 + sl;
                    v = make_float4(nb_f(h, p.ox, jk), nb_f(h, p.oy, jk), a.G * nb_f(h, p.om, jk),
                                    __int_as_float((int)(jk + 1)));
                    slow |= __float_as_uint(v.z) - kGmLo >= kGmHi - kGmLo;
                    far |= !(fabsf(v.x) < kBox && fabsf(v.y) < kBox);
                }
            }
            tile[e] = v;
        }
        const bool tile_slow = __syncthreads_or(slow) != 0;
        const bool tile_box = wg_box && __syncthreads_or(far) == 0;
        const uint32_t ne = (uint32_t)((r - t0 < kTile ? r - t0 : kTile) * 64);   // a multiple of 64
        if (tile_slow) {
            for (uint32_t e = 0; e < ne; ++e) exact(tile[e]);
            continue;
        }
        if (tile_box) {
            for (uint32_t e = 0; e < ne; e += kBoxGroup) {
                float4 v[kBoxGroup];
                float dx[kBoxGroup], dy[kBoxGroup], d2[kBoxGroup];
#pragma unroll
                for (uint32_t k = 0; k < kBoxGroup; ++k) {
                    v[k] = tile[e + k];
                    dx[k] = v[k].x - xi;
                    dy[k] = v[k].y - yi;
                    d2[k] = dx[k] * dx[k] + dy[k] * dy[k];
                }
                float m = d2[0];
#pragma unroll
                for (uint32_t k = 1; k < kBoxGroup; ++k) m = fminf(m, d2[k]);
                if (__all(m >= 0x1p-40f)) {
                    float sk[kBoxGroup];
#pragma unroll
                    for (uint32_t k = 0; k < kBoxGroup; ++k) sk[k] = div_cr_fast(v[k].z, d2[k] * sqrt_cr_fast(d2[k]));
#pragma unroll
                    for (uint32_t k = 0; k < kBoxGroup; ++k) {
                        sx = sx + sk[k] * dx[k];
                        sy = sy + sk[k] * dy[k];
                    }
                } else {
#pragma unroll
                    for (uint32_t k = 0; k < kBoxGroup; ++k) exact(v[k]);
                }
            }
            continue;
        }
        for (uint32_t e = 0; e < ne; e += 4) {
            const float4 v0 = tile[e], v1 = tile[e + 1], v2 = tile[e + 2], v3 = tile[e + 3];
            const float dx0 = v0.x - xi, dy0 = v0.y - yi, dx1 = v1.x - xi, dy1 = v1.y - yi;
            const float dx2 = v2.x - xi, dy2 = v2.y - yi, dx3 = v3.x - xi, dy3 = v3.y - yi;
            const float d20 = dx0 * dx0 + dy0 * dy0, d21 = dx1 * dx1 + dy1 * dy1;
            const float d22 = dx2 * dx2 + dy2 * dy2, d23 = dx3 * dx3 + dy3 * dy3;
            const uint32_t off = max(max(d2_offset(d20), d2_offset(d21)), max(d2_offset(d22), d2_offset(d23)));
            if (__all(off < kD2Hi - kD2Lo)) {
                const float s0 = div_cr_fast(v0.z, d20 * sqrt_cr_fast(d20));
                const float s1 = div_cr_fast(v1.z, d21 * sqrt_cr_fast(d21));
                const float s2 = div_cr_fast(v2.z, d22 * sqrt_cr_fast(d22));
                const float s3 = div_cr_fast(v3.z, d23 * sqrt_cr_fast(d23));
                sx = sx + s0 * dx0; sy = sy + s0 * dy0;
                sx = sx + s1 * dx1; sy = sy + s1 * dy1;
                sx = sx + s2 * dx2; sy = sy + s2 * dy2;
                sx = sx + s3 * dx3; sy = sy + s3 * dy3;
            } else {
                exact(v0); exact(v1); exact(v2); exact(v3);
            }
        }
    }
    if (me) {
        float& vx = nb_f(h, p.ovx, ikey);
        float& vy = nb_f(h, p.ovy, ikey);
        const float ax = sx * a.dt, ay = sy * a.dt;
        vx = vx + ax;
        vy = vy + ay;
    }
}

// Self-check of the fast arithmetic against the general correctly rounded
// operations: out[0] += square roots that differ, over every float bit
// pattern in [lo, hi) (one thread per pattern, grid-stride); out[1] +=
// quotients that differ over `pairs` pseudo-random (G m, d2 * sqrt(d2))
// operand pairs drawn from the fast ranges.
__global__ void k_check_force_arith(uint32_t lo, uint32_t hi, uint64_t pairs, uint64_t seed,
                                    unsigned long long* out) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint32_t bad_sqrt = 0, bad_div = 0;
    for (uint64_t b = lo + t; b < hi; b += stride) {
        const float x = __uint_as_float((uint32_t)b);
        bad_sqrt += __float_as_uint(sqrt_cr_fast(x)) != __float_as_uint(sqrtf(x));
    }
    for (uint64_t i = t; i < pairs; i += stride) {
        const uint64_t z = splitmix64(seed ^ i);
        const float gm = __uint_as_float(kGmLo + (uint32_t)(((z & 0xFFFFFFFFull) * (kGmHi - kGmLo)) >> 32));
        const float d2 = __uint_as_float(kD2Lo + (uint32_t)(((z >> 32) * (kD2Hi - kD2Lo)) >> 32));
        const float b = d2 * sqrtf(d2);
        bad_div += __float_as_uint(div_cr_fast(gm, b)) != __float_as_uint(gm / b);
    }
    bad_sqrt = wave_add(bad_sqrt);
    bad_div = wave_add(bad_div);
    if (lane_id() == 0) {
        if (bad_sqrt) atomicAdd(out, (unsigned long long)bad_sqrt);
        if (bad_div) atomicAdd(out + 1, (unsigned long long)bad_div);
    }
}

}  // namespace smmo
