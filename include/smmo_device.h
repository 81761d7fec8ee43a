/*
 * smmo_device.h — device-side API of the MI355X SMMO object heap, for the
 * methods and constructors compiled into libsmmo (HIP, gfx950).
 *
 * Method: Springer & Masuhara, "DynaSOAr: A Parallel Memory Allocator for
 * Object-oriented Programming on GPUs with Efficient Memory Access", ECOOP
 * 2019 (arXiv 1810.11765).  Sec. 2.1: inside a method run by parallel_do, a
 * thread may create objects with `new` (device-side allocation) and delete
 * them with `destroy`; a method reads and writes the fields of `this` and of
 * other objects through their pointers.  Here a pointer is an smmo_ref handle
 * (class, block, slot) and the calls below are what a method uses.
 *
 * A method (see the SMMO_M_* ids of smmo.h) is a struct with
 *     using Args = <POD argument blob>;            // <= SMMO_ARGS_MAX bytes
 *     static constexpr bool kSnapshot;             // true if it creates objects of its own class
 *     struct Prep; static Prep prepare(const smmo::DevHeap&, uint32_t cls, const Args&);
 *     static void run(const smmo_obj& self, const Prep&, const Args&);
 * The library's do-all calls run() for every slot of every block of the
 * class, with all 64 lanes of a wavefront (lane = slot), live or not: test
 * smmo_live(self) before touching `this`.
 *
 * Collective calls.  smmo_alloc, smmo_destroy and smmo_destroy_self are
 * wavefront-collective (workgroup-collective when the method asks for
 * workgroup-aggregated allocation): every lane of the wave calls them at the
 * same point, with `want` saying whether that lane takes part, so that the
 * wave's requests are coalesced into one atomic per block (Sec. 4.2).  Do not
 * call them from divergent code.
 *
 * Preconditions (not checked in release builds, Sec. 2.1): destroy only live
 * handles, each at most once; a method of class T destroys no object of T or
 * of T's subclasses other than `this`; a method writes no field of an object
 * it destroys in the same do-all.  Handles stay valid until destroyed.
 * Out of memory: smmo_alloc returns SMMO_NULL for the lanes it could not
 * serve and raises SMMO_STATUS_OOM in the heap's status word (smmo_status).
 */
#ifndef SMMO_DEVICE_H
#define SMMO_DEVICE_H

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "smmo.h"

namespace smmo {
struct DevHeap;   /* the heap as a kernel sees it (passed to prepare()) */
struct Obj;       /* one slot of the block a wave is visiting */
}
typedef smmo::Obj smmo_obj;
typedef uint64_t smmo_ref;   /* (class+1) << 56 | block << 6 | slot; 0 = null */
#define SMMO_NULL ((smmo_ref)0)

/* The object this lane visits: its handle, whether it is live in this
 * do-all, and its class id. */
__device__ smmo_ref smmo_self(const smmo_obj& self);
__device__ bool smmo_live(const smmo_obj& self);
__device__ uint32_t smmo_class(const smmo_obj& self);

/* Device-side new (Sec. 2.1, Alg. 1): lanes with want = true each receive a
 * fresh object of class `cls` (fields uninitialized) or SMMO_NULL on OOM;
 * other lanes receive SMMO_NULL.  Collective (see above). */
__device__ smmo_ref smmo_alloc(const smmo_obj& self, uint32_t cls, bool want);

/* Device-side destroy (Sec. 2.1, Alg. 2): lanes with want = true destroy the
 * object `r` (any class; r != SMMO_NULL); the lanes' handles are grouped by
 * block, one atomic AND per block.  Collective. */
__device__ void smmo_destroy(const smmo_obj& self, smmo_ref r, bool want);

/* destroy(this) for the lanes with want = true (their objects must be live).
 * Collective; cheaper than smmo_destroy (all lanes share one block). */
__device__ void smmo_destroy_self(const smmo_obj& self, bool want);

/* Address of field `field` of object `r` (Sec. 3.2 SOA layout: the field's
 * array in r's block, element r's slot).  Any lane, no collective. */
__device__ void* smmo_field_ptr(const smmo_obj& self, smmo_ref r, uint32_t field);
template <class F>
__device__ inline F& smmo_field(const smmo_obj& self, smmo_ref r, uint32_t field) {
    return *static_cast<F*>(smmo_field_ptr(self, r, field));
}

/* The counter-based generator the workloads draw from: SplitMix64 (Steele,
 * Lea & Flood, OOPSLA 2014), a draw keyed on (seed, step, id, stream), and
 * a float in [0, 1) from its top 24 bits. */
__device__ uint64_t smmo_splitmix64(uint64_t x);
__device__ uint64_t smmo_draw(uint64_t seed, uint64_t step, uint64_t id, uint64_t stream);
__device__ float smmo_unit_float(uint64_t h);

#endif
