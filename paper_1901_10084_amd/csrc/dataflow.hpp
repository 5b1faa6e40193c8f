// dataflow.hpp -- types and the dependency wait of the dataflow executor
// (one persistent launch per pass over the schedule, whose tile steps wait
// only for the earlier steps that touch the same blocks of x).
#pragma once

#include "common.hpp"

namespace ccp {

struct DTile {
    int32_t P, Q;
    int64_t ybase;
    int32_t jsbase;  // index of the tile's first step in the `needs` table
    uint32_t needC;  // touches of block (P,Q) before this tile, per sweep
};

__host__ __device__ __forceinline__ int block_id(int A, int B) { return B * (B + 1) / 2 + A; }

// Arguments of one dataflow launch.
struct DataflowArgs {
    const DTile *tiles;
    int ntiles;
    const uint32_t *needs;
    const uint32_t *K;
    uint32_t *cnt;       // completed touches per block (cumulative over epochs), stride kCntStride
    uint32_t *ctl;       // [0] ticket counter, [1] abort flag
    uint32_t epoch;      // sweeps already run on these counters
    uint64_t wait_ticks; // wall-clock limit of one wait
    unsigned long long *prof;  // optional: wall-clock ticks per phase, summed
};

// Thread 0 only.  True once each of the three counters has reached its
// need; false on time-out or abort.  The counters and the abort flag are
// read in the same round trip; an unused slot reads the abort flag with
// need 0, which it always meets (the flag is 0 or 1).
__device__ __forceinline__ bool wait_counts(const uint32_t *c0, uint32_t n0, const uint32_t *c1, uint32_t n1,
                                            const uint32_t *c2, uint32_t n2, uint32_t *abort_flag,
                                            uint64_t ticks) {
    const uint64_t start = wall_clock64();
    bool res;
    for (;;) {
        const uint32_t v0 = __hip_atomic_load(c0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t v1 = __hip_atomic_load(c1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t v2 = __hip_atomic_load(c2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t ab = __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (int32_t(v0 - n0) >= 0 && int32_t(v1 - n1) >= 0 && int32_t(v2 - n2) >= 0) {
            res = true;
            break;
        }
        if (ab) {
            res = false;
            break;
        }
        if (wall_clock64() - start > ticks) {
            __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            res = false;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    // No poll may stay in flight: a load pending at the step loop's head
    // makes the compiler drain every wave's stores before the next loads.
    __builtin_amdgcn_s_waitcnt(0);
    return res;
}

}  // namespace ccp
