// common.hpp -- shared types and helpers of the gfx950 solver library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "ccproj.h"

namespace ccp {

// One tile (P,Q) of the tiled schedule (Sec. III-C): every triplet i<j<k
// with i in index block P and k in index block Q.  `ybase` is the offset of
// the tile's segment in the schedule-ordered metric dual array.
struct Tile {
    int32_t P, Q;
    int64_t ybase;
};

// Dataflow executor: each block's touch counter sits alone in a 128-byte
// line, so polls of different counters go to different memory channels
// instead of queueing on a few shared lines.
constexpr int kCntStride = 32;

// The residual and warm-start inference kernels walk each tile in chunks of
// at most this many tile steps, one workgroup per chunk: whole tiles (1 to
// nb steps) leave most of the chip idle behind the longest ones.
constexpr int kChunkSteps = 4;

// What the warm-start kernels read of the graph and the schedule.
struct GraphView {
    const Tile *tiles;
    int64_t ntiles;
    int b;
    int64_t n;
    const double *w;
    const uint8_t *d;
    const float *deg;
    const float *mean_deg;
    const int32_t *chunks;  // (tile, first step) per chunk of kChunkSteps steps
    int64_t nchunks;
};

// Compacted dual lists (sweeps without a dense dual array): tile step c's
// cnt[c] entries (slot within the step, dual) start at off[c] in a pool; a
// sweep reads the _in pool and writes the _out pool.
template <typename T>
struct CompactArgs {
    const uint16_t *idx_in;
    const T *val_in;
    const int64_t *off_in;
    const uint32_t *cnt_in;
    uint16_t *idx_out;
    T *val_out;
    int64_t *off_out;
    uint32_t *cnt_out;
    unsigned long long *alloc;  // entries taken from the output pool
    int64_t cap;                // output pool capacity, entries
    uint32_t *overflow;         // raised when a step's list does not fit
};

// Packed column-major upper-triangular pair index, i < j.
__host__ __device__ __forceinline__ int64_t pidx(int64_t i, int64_t j) {
    return j * (j - 1) / 2 + i;
}

// Colex triplet index, i < j < k.
__host__ __device__ __forceinline__ int64_t tidx(int64_t i, int64_t j, int64_t k) {
    return k * (k - 1) * (k - 2) / 6 + j * (j - 1) / 2 + i;
}

// Middle-index offset of lane (il, kl) at sub-step t: il + jl + kl = t (mod b).
// Three indices in one block with equal sum mod b can share at most one
// index unless they are equal, which makes every sub-step conflict-free.
__host__ __device__ __forceinline__ int mid_offset(int t, int il, int kl, int b) {
    return (t - il - kl + 2 * b) % b;
}

// Order of the middle blocks J inside tile (P,Q): from Q down to P in the
// rounds of the first double loop of Fig. 2 (P + Q < nb), from P up to Q in
// those of the second.  Step m = 0..Q-P of the tile visits tile_J(m).  (The
// paper leaves this order open; this one lets a tile release the block that
// the next tile of its column waits for as early as possible.)
__host__ __device__ __forceinline__ bool tile_desc(int P, int Q, int nb) { return P + Q < nb; }
__host__ __device__ __forceinline__ int tile_J(int P, int Q, int m, bool desc) {
    return desc ? Q - m : P + m;
}

// Thread-local error reporting for the C ABI.
void set_error(const std::string &msg);
int fail(int code, const std::string &msg);

}  // namespace ccp

#define CCP_HIP_CHECK(expr)                                                       \
    do {                                                                          \
        hipError_t e_ = (expr);                                                   \
        if (e_ != hipSuccess)                                                     \
            return ::ccp::fail(CC_EHIP, std::string(#expr) + ": " +               \
                                            hipGetErrorString(e_));               \
    } while (0)

#define CCP_LAUNCH_CHECK(what)                                                    \
    do {                                                                          \
        hipError_t e_ = hipGetLastError();                                        \
        if (e_ != hipSuccess)                                                     \
            return ::ccp::fail(CC_EHIP, std::string("launch of ") + (what) +      \
                                            ": " + hipGetErrorString(e_));        \
    } while (0)
