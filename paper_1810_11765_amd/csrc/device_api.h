// Definitions of the device-side API declared in include/smmo_device.h, in
// terms of the allocator (alloc.h) and the do-all's object view (kernels.h).
#pragma once

#include "kernels.h"
#include "smmo_device.h"

__device__ __forceinline__ smmo_ref smmo_self(const smmo_obj& o) { return o.self(); }
__device__ __forceinline__ bool smmo_live(const smmo_obj& o) { return o.live; }
__device__ __forceinline__ uint32_t smmo_class(const smmo_obj& o) { return o.cls; }

__device__ __forceinline__ smmo_ref smmo_alloc(const smmo_obj& o, uint32_t cls, bool want) {
    return o.alloc(cls, want);
}

__device__ __forceinline__ void smmo_destroy(const smmo_obj& o, smmo_ref r, bool want) {
    smmo::wave_destroy(o.h, r, want);
}

__device__ __forceinline__ void smmo_destroy_self(const smmo_obj& o, bool want) {
    smmo::wave_destroy_self(o.h, o.cls, o.bid, want);
}

__device__ __forceinline__ void* smmo_field_ptr(const smmo_obj& o, smmo_ref r, uint32_t field) {
    return smmo::field_addr(o.h, smmo::ref_cls(r), smmo::ref_block(r), smmo::ref_slot(r), field);
}

__device__ __forceinline__ uint64_t smmo_splitmix64(uint64_t x) { return smmo::splitmix64(x); }
__device__ __forceinline__ uint64_t smmo_draw(uint64_t seed, uint64_t step, uint64_t id, uint64_t stream) {
    return smmo::ctr_draw(seed, step, id, stream);
}
__device__ __forceinline__ float smmo_unit_float(uint64_t h) { return smmo::unit_float(h); }
