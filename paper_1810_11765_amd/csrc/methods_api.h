// A method written against the public device API only (include/smmo_device.h):
// the allocation microbenchmark's churn round (the same rule as MChurn in
// methods.h), so that the tests exercise device-side new / destroy / field
// access exactly as a method author outside the library core would use them.
#pragma once

#include "smmo_device.h"

// {int32 id, float32 x, float32 v}: an object selected by
// splitmix64(seed ^ id ^ round) & 1 destroys itself and creates its
// replacement id' = ((round+1) << 18) | (id & 0x3FFFF), x' and v' drawn from
// (seed, round+1, id', 0 | 1).  The replacement is not visited by this do-all.
struct MChurnApi {
    using Args = smmo_churn_args;
    static constexpr bool kSnapshot = true;      // creates objects of its own class
    struct Prep {};
    __device__ static Prep prepare(const smmo::DevHeap&, uint32_t, const Args&) { return {}; }
    __device__ static void run(const smmo_obj& self, const Prep&, const Args& a) {
        bool die = false;
        int32_t nid = 0;
        if (smmo_live(self)) {
            const int32_t id = smmo_field<int32_t>(self, smmo_self(self), 0);
            die = (smmo_splitmix64(a.seed ^ (uint64_t)(uint32_t)id ^ (uint64_t)a.round) & 1) != 0;
            nid = (int32_t)(((uint32_t)(a.round + 1) << 18) | ((uint32_t)id & 0x3FFFFu));
        }
        smmo_destroy_self(self, die);
        const smmo_ref r = smmo_alloc(self, smmo_class(self), die);
        if (die && r != SMMO_NULL) {
            smmo_field<int32_t>(self, r, 0) = nid;
            smmo_field<float>(self, r, 1) = smmo_unit_float(smmo_draw(a.seed, a.round + 1, (uint64_t)(uint32_t)nid, 0));
            smmo_field<float>(self, r, 2) = smmo_unit_float(smmo_draw(a.seed, a.round + 1, (uint64_t)(uint32_t)nid, 1));
        }
    }
};
