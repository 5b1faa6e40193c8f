// dataflow.hip -- the sweep as one persistent launch whose tiles wait only
// for the tile steps they depend on, instead of for whole rounds.
//
// The result of a sweep depends only on the order in which each variable is
// updated.  The schedule of Sec. III fixes that order: a block of x (the
// pairs with one index in block A and the other in block B) is touched by a
// sequence of tile steps (tile, middle block J), in schedule order.  Here
// every block X carries a counter of completed touches; a tile step waits
// until the counters of the blocks it touches reach the number of touches
// that precede it in schedule order, so every block sees exactly the
// schedule's sequence of updates and the result equals the round-by-round
// executor's bit for bit.  Tiles are handed out by a ticket counter in
// schedule order, so the oldest unfinished tile never waits on an unfinished
// one and the launch always makes progress.  Every wait is bounded by a
// wall-clock limit; a timed-out wait raises an abort flag that every other
// wait also checks, so the grid always drains.
//
// Memory ordering across the chip's per-XCD L2 caches: the shared x blocks
// are read and written only with agent-scope atomic loads and stores, which
// every CU observes coherently.  A tile step stores its blocks, every wave
// waits until its stores are complete, and then one thread bumps the
// counters; a waiting tile polls the counters (agent-scope loads) before it
// loads the blocks.  No L2 write-back is needed: the dual stream, which is
// private to its tile, stays out of the release.
//
// Sparse dual access (Sec. III-D keeps only the nonzero duals, in visit
// order, per processor).  Here the dense schedule-ordered dual array stays
// the storage every other kernel reads, and a bit mask with one bit per dual
// slot marks the slots that may hold a nonzero dual.  The sparse sweep loads
// only marked duals (an unmarked one is 0), stores a dual only where its
// value changed, and rewrites the mask from the new duals; its results equal
// the dense sweep's bit for bit.  Mask layout: tile step c (schedule order)
// holds 3 b^2 words of b bits, word [c][o][lane] with bit t for sub-step t.
//
// Compacted dual lists (the memory form of Sec. III-D, for b = 8 and 16):
// no dense dual array at all.  Tile step c keeps a list of (slot, dual)
// pairs for its nonzero duals in a pool; a sweep expands a step's list into
// an LDS copy of the step's duals, runs the sub-steps on it, and writes the
// step's new nonzeros to the other pool through a bump allocator.  A list
// that does not fit raises a flag; the host then restores x and repeats the
// sweep with a larger pool.  Results equal the dense sweep's bit for bit.
#include <vector>

#include "common.hpp"
#include "dataflow.hpp"
#include "project.hpp"

namespace ccp {

template <int B> struct MaskWord;
template <> struct MaskWord<8> { using type = uint8_t; };
template <> struct MaskWord<16> { using type = uint16_t; };
template <> struct MaskWord<32> { using type = uint32_t; };
// b = 24: 24 bits of a 32-bit word, the top 8 always clear.
template <> struct MaskWord<24> { using type = uint32_t; };
template <int B> constexpr bool kSparseB = (B == 8 || B == 16 || B == 24 || B == 32);

// Bit pattern of a dual: the mask marks every slot whose bits are not those
// of +0.0 (a -0.0 counts as nonzero), so an unmarked slot reads back exactly.
__device__ __forceinline__ uint64_t dual_bits(double v) { return __builtin_bit_cast(uint64_t, v); }
__device__ __forceinline__ uint64_t dual_bits(float v) { return __builtin_bit_cast(uint32_t, v); }
// 1 if a dual's bits are not +0.0's, else 0 (no compare: a min of its words)
__device__ __forceinline__ uint32_t nonzero01(double v) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    return __builtin_elementwise_min(uint32_t(u) | uint32_t(u >> 32), 1u);
}
__device__ __forceinline__ uint32_t nonzero01(float v) {
    return __builtin_elementwise_min(__builtin_bit_cast(uint32_t, v), 1u);
}

// Masked dual accesses go through a buffer resource over the tile's dual
// segment: an offset at or beyond its size (kOffNone) reads 0 and writes
// nothing, without a memory access, so a masked lane needs no branch (and
// the prefetch ring keeps exact memory-counter waits).  Cache policy 2 is
// the non-temporal hint of the dense accesses.
constexpr uint32_t kOffNone = 0x80000000u;
constexpr int kBufNT = 2;
constexpr int kBufFlags = 0x00020000;  // gfx9 raw buffer, 32-bit data format
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(off), 0, kBufNT));
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(off), 0, kBufNT));
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, int(off), 0, kBufNT);
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(off), 0, kBufNT);
}
// Dense accesses: a wave-uniform byte offset (scalar register) plus the
// lane's own, so no vector address arithmetic is needed per access.
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(voff), int(soff), kBufNT));
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(voff), int(soff), kBufNT));
}
__device__ __forceinline__ void buf_store(double v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, int(voff), int(soff), kBufNT);
}
__device__ __forceinline__ void buf_store(float v, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(voff), int(soff), kBufNT);
}




// ---------------------------------------------------------------------------
// Host: dependency tables.  For tile step (tile, m) with middle block J the
// blocks touched besides (P,Q) are A = (P,J) unless J = Q and B = (J,Q)
// unless J = P; needs[2 s], needs[2 s + 1] count the touches of A and B that
// precede the step in one sweep.  K[X] = touches of block X per sweep.
// ---------------------------------------------------------------------------
void build_dataflow_tables(int64_t n, int b, std::vector<DTile> &tiles,
                           std::vector<uint32_t> &needs, std::vector<uint32_t> &K) {
    const int nb = int((n + b - 1) / b);
    const int64_t bb = int64_t(b) * b;
    K.assign(size_t(nb) * (nb + 1) / 2, 0u);
    tiles.clear();
    needs.clear();
    int64_t ybase = 0;
    for (int r = 0; r < 2 * nb - 1; ++r) {
        const int s = (r < nb) ? (nb - 1 - r) : r;
        for (int P = 0; 2 * P <= s; ++P) {
            const int Q = s - P;
            if (Q >= nb) continue;
            DTile t;
            t.P = P;
            t.Q = Q;
            t.ybase = ybase;
            t.jsbase = int32_t(needs.size() / 2);
            t.needC = K[block_id(P, Q)];
            const bool desc = tile_desc(P, Q, nb);
            for (int m = 0; m <= Q - P; ++m) {
                const int J = tile_J(P, Q, m, desc);
                uint32_t na = 0, nbn = 0;
                if (J != Q) na = K[block_id(P, J)]++;
                if (J != P) nbn = K[block_id(J, Q)]++;
                needs.push_back(na);
                needs.push_back(nbn);
            }
            K[block_id(P, Q)] += uint32_t(Q - P + 1);
            tiles.push_back(t);
            ybase += int64_t(Q - P + 1) * b * 3 * bb;
        }
    }
}

// ---------------------------------------------------------------------------
// Device.
// ---------------------------------------------------------------------------


template <typename T, int B, int D, bool SP, bool CP>
__global__ void __launch_bounds__(B * B)
k_sweep_dataflow(DataflowArgs a, int64_t n, T *__restrict__ x, const T *__restrict__ g,
                 T *__restrict__ y, typename MaskWord<B>::type *__restrict__ mask, CompactArgs<T> cp) {
    using MW = typename MaskWord<B>::type;
    static_assert(!CP || (!SP && B <= 16), "compacted lists: b = 8 or 16, 16-bit slot indices");
    static_assert(!SP || kSparseB<B>, "sparse dual access: one mask word of b bits per lane");
    // the first and last groups of D sub-steps are peeled: refills of the
    // other groups stay inside the step
    static_assert(B % D == 0 && B >= 2 * D, "ring depth must divide b, twice at least");
    constexpr int b = B;
    constexpr int bb = B * B;
    const int tid = threadIdx.x;
    // sub-step lane (il, kl); its dual slot is il*b + kl
    const int il = tid / b, kl = tid % b;
    // stage/publish element (sr, sc) of a block: the row index runs fastest
    // across threads, so the accesses are contiguous in the packed upper
    // triangle
    const int sr = tid % b, sc = tid / b;
    const int nn = int(n);
    const int nb = (nn + b - 1) / b;

    // LDS: x and g of blocks A = (P,J), B = (J,Q) and C = (P,Q) in separate
    // arrays, each row-major [row*b + col].  With 4-byte elements every
    // sub-step access is free of bank conflicts; only the transposing
    // stage/publish accesses conflict, once per tile step.
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *const lds = reinterpret_cast<T *>(smem_raw);
    T *const Ax0 = lds, *const Ag0 = lds + bb, *const Bx0 = lds + 2 * bb, *const Bg0 = lds + 3 * bb;
    T *const Cx = lds + 4 * bb, *const Cg = lds + 5 * bb;
    // compacted lists: the current step's 3 b^3 duals, [t][o][lane]
    T *const ly = lds + 6 * bb;
    __shared__ int s_tix, s_ok;

    // Control structure: every `if (tid == 0)` region is closed by a
    // barrier, and every value broadcast through LDS is made wave-uniform
    // (readfirstlane) before it steers a branch.  Branches around barriers
    // must be uniform; otherwise the compiler may merge thread-0 regions
    // across a loop back-edge and split a wave's lanes between barriers.
    //
    // Per tile step: sub-steps, publish the step's blocks, then one thread-0
    // region that releases them and waits for the next step's blocks.  The
    // dual ring is refilled for the next step only after that release, so
    // the release's drain of the memory counter (each wave waits for every
    // outstanding access) covers the published stores rather than a full
    // ring of prefetched duals.
    //
    // optional breakdown (thread 0): [0] waiting for blocks, [1] loading
    // blocks into LDS, [2] sub-steps, [3] publishing, [4] tile steps
    // kept in LDS: per-thread 64-bit counters would hold registers for the
    // whole kernel
    __shared__ uint64_t s_pt[6];  // [0..4] as above, [5] the last mark
    auto mark = [&](int e) {      // thread 0 only
        const uint64_t t1 = wall_clock64();
        s_pt[e] += t1 - s_pt[5];
        s_pt[5] = t1;
    };
    if (tid == 0)
        for (int e = 0; e < 6; ++e) s_pt[e] = 0;
    if constexpr (CP)
        for (int e = tid; e < 3 * B * B * B; e += B * B) ly[e] = T(0);
    if (tid == 0) s_tix = int(atomicAdd(&a.ctl[0], 1u));
    __syncthreads();
    for (;;) {
        const int tix = __builtin_amdgcn_readfirstlane(s_tix);
        if (tix >= a.ntiles) break;
        const DTile tl = a.tiles[tix];
        const int P = tl.P, Q = tl.Q;
        const bool desc = tile_desc(P, Q, nb);
        const int i = P * b + il, k = Q * b + kl;
        const int idC = block_id(P, Q);

        // element (sr, sc) of block (R, S): pair (R*b+sr, S*b+sc) when it is one
        // (zeros elsewhere); the loads are unconditional
        // split in a load and a store half, so that other loads can be
        // issued between them; padding is masked at the store
        auto blk_ok = [&](int R, int S) {
            const int ii = R * b + sr, jj = S * b + sc;
            return ii < jj && jj < nn;
        };
        // x of a block is read and written with agent-scope atomic accesses
        // (coherent across the chip's L2 caches); g never changes.
        auto blk_load = [&](int R, int S, T &vx, T &vg) {
            const int64_t p = blk_ok(R, S) ? pidx(R * b + sr, S * b + sc) : 0;
            vx = __hip_atomic_load(&x[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            vg = g[p];
        };
        auto blk_store = [&](int R, int S, T vx, T vg, T *X, T *G) {
            const bool ok = blk_ok(R, S);
            X[sr * b + sc] = ok ? vx : T(0);
            G[sr * b + sc] = ok ? vg : T(0);
        };
        auto stage = [&](int R, int S, T *X, T *G) {
            T vx, vg;
            blk_load(R, S, vx, vg);
            blk_store(R, S, vx, vg, X, G);
        };
        auto publish = [&](int R, int S, const T *X) {
            const int ii = R * b + sr, jj = S * b + sc;
            if (ii < jj && jj < nn)
                __hip_atomic_store(&x[pidx(ii, jj)], X[sr * b + sc], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        };
        // blocks (P,J) and (J,Q) of step m, -1 where the step uses (P,Q)
        auto step_ids = [&](int m, int &idA, int &idB) {
            const int J = tile_J(P, Q, m, desc);
            idA = (J != Q) ? block_id(P, J) : -1;
            idB = (J != P) ? block_id(J, Q) : -1;
        };
        // thread 0: wait until step m's blocks have all earlier touches
        // thread 0: wait for step m's blocks (and, with withC, for (P,Q))
        auto wait_step = [&](int m, bool withC) {
            int idA, idB;
            step_ids(m, idA, idB);
            const uint32_t *nd = a.needs + 2 * int64_t(tl.jsbase + m);
            uint32_t *const none = &a.ctl[1];
            return wait_counts(idA >= 0 ? &a.cnt[int64_t(idA) * kCntStride] : none,
                               idA >= 0 ? a.epoch * a.K[idA] + nd[0] : 0u,
                               idB >= 0 ? &a.cnt[int64_t(idB) * kCntStride] : none,
                               idB >= 0 ? a.epoch * a.K[idB] + nd[1] : 0u,
                               withC ? &a.cnt[int64_t(idC) * kCntStride] : none,
                               withC ? a.epoch * a.K[idC] + tl.needC : 0u, &a.ctl[1], a.wait_ticks);
        };

        // Dual addresses: a wave-uniform part per sub-step plus a fixed lane
        // offset, so that they need no vector address arithmetic.  Each dual
        // is read and written once per sweep: non-temporal accesses.
        T *const ytile = y + tl.ybase;
        const int64_t ystep = int64_t(3) * bb;
        const unsigned lane = unsigned(tid);
        T yq[D][3];
        // Sparse access: mw holds the mask words of the current step, mwn
        // those of the next step (loaded one step ahead), nm the new words.
        // Two formulations of the mask arithmetic, chosen per tile size by
        // measurement (b = 32: 8% faster with the lean one; b = 16: 2-4%
        // slower with it): lean keeps the words complemented, pushes an
        // offset out of range by shifting the complemented bit into bit 31,
        // and forms a new bit as min(bits, 1); the other selects the offset
        // and compares the bits with zero.
        constexpr bool lean = (B == 32);
        uint32_t mw[3] = {0u, 0u, 0u}, mwn[3] = {0u, 0u, 0u}, nm[3] = {0u, 0u, 0u};
        auto mask_row = [&](int m) { return mask + (int64_t(tl.jsbase) + m) * 3 * bb; };
        auto load_mask = [&](int m) {
            const MW *r = mask_row(m);
            const uint32_t flip = lean ? ~0u : 0u;
            mwn[0] = uint32_t(r[lane]) ^ flip;
            mwn[1] = uint32_t(r[lane + bb]) ^ flip;
            mwn[2] = uint32_t(r[lane + 2 * bb]) ^ flip;
        };
        // The tile's dual segment as a buffer (its size stays below
        // kOffNone, at most nb 3 b^3 elements).
        // (inputs made wave-uniform: a descriptor in vector registers would
        // cost a loop over the distinct values at every access)
        const uint64_t ya = reinterpret_cast<uint64_t>(ytile);
        const uint64_t yau = (uint64_t(__builtin_amdgcn_readfirstlane(uint32_t(ya >> 32))) << 32) |
                             uint32_t(__builtin_amdgcn_readfirstlane(uint32_t(ya)));
        const __amdgpu_buffer_rsrc_t yr = __builtin_amdgcn_make_buffer_rsrc(
            reinterpret_cast<void *>(yau), 0,
            __builtin_amdgcn_readfirstlane(int(int64_t(Q - P + 1) * b * ystep * int64_t(sizeof(T)))), kBufFlags);
        // byte offset of dual (u, o) of this lane, out of range (bit 31 set,
        // above any tile's size) where mask bit t is clear
        auto boff = [&](int u, int t, int o) {
            if constexpr (lean) {
                const uint32_t off = uint32_t(int64_t(u) * ystep * int64_t(sizeof(T))) +
                                     uint32_t((o * bb + int(lane)) * int(sizeof(T)));
                return off | ((mw[o] << (31 - t)) & kOffNone);
            } else {
                const uint32_t off = uint32_t((int64_t(u) * ystep + o * bb + int(lane)) * int64_t(sizeof(T)));
                return ((mw[o] >> t) & 1u) ? off : kOffNone;
            }
        };
        // Dense accesses.  FP64: through the buffer, at the byte offset of
        // sub-step u's duals (wave-uniform, scalar) plus this lane's offset
        // of dual o; without it the compiler forms 64-bit vector addresses
        // (n = 500: 0.885 against 0.915 ms).  FP32: a wave-uniform base
        // pointer plus a 32-bit lane offset, which the compiler already
        // keeps scalar (the buffer form measured 2-9% slower there).
        constexpr bool kBufDense = sizeof(T) == 8;
        auto soff = [&](int u) {
            return uint32_t(__builtin_amdgcn_readfirstlane(int(int64_t(u) * ystep * int64_t(sizeof(T)))));
        };
        auto voff = [&](int o) { return uint32_t((o * bb + int(lane)) * int(sizeof(T))); };
        // dual o of sub-step t of step m (flat sub-step u = m b + t), at p
        // in the pointer form
        auto ld = [&](const T *p, int u, int t, int o) {
            if constexpr (SP)
                return buf_load(yr, boff(u, t, o), T(0));
            else if constexpr (kBufDense)
                return buf_load(yr, voff(o), soff(u), T(0));
            else
                return __builtin_nontemporal_load(p);
        };
        // Ring slot d <- the duals of sub-step t of the step (flat sub-step
        // u).  Sparse access issues every load (unmarked lanes read 0 out of
        // range): a load under a branch would leave the compiler unable to
        // count the loads in flight, and it would then wait for all of them.
        auto ring_load = [&](int d, const T *src, int u, int t) {
            yq[d][0] = ld(&src[lane], u, t, 0);
            yq[d][1] = ld(&src[lane + bb], u, t, 1);
            yq[d][2] = ld(&src[lane + 2 * bb], u, t, 2);
        };
        // ring: the first D sub-steps of step m (all inside the step, D | b)
        auto fill_ring = [&](int m) {
#pragma unroll
            for (int d = 0; d < D; ++d) ring_load(d, ytile + int64_t(m * b + d) * ystep, m * b + d, d);
        };

        if constexpr (SP) load_mask(0);
        // Block (P,Q) and the first step's blocks: wait, then hold (P,Q).
        if (tid == 0) {
            if (a.prof) s_pt[5] = wall_clock64();
            const bool ok = wait_step(0, true);
            if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_ok = ok;
            if (a.prof) mark(0);
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(s_ok)) break;
        stage(P, Q, Cx, Cg);

        bool aborted = false;
        for (int m = 0; m <= Q - P; ++m) {
            const int J = tile_J(P, Q, m, desc);
            int idA, idB;
            step_ids(m, idA, idB);
            // A or B is the resident C block where the middle block is Q or P
            T *const Ax = (J == Q) ? Cx : Ax0, *const Ag = (J == Q) ? Cg : Ag0;
            T *const Bx = (J == P) ? Cx : Bx0, *const Bg = (J == P) ? Cg : Bg0;

            // Stage the step's blocks (their waits are done).  The step's
            // dual ring is issued between the block loads and their use:
            // loads complete in order, so the ring's HBM latency then
            // overlaps the staging rather than delaying it.
            // Loads and stores are unconditional: where A or B is the
            // resident C block, the staging buffer it would use is idle this
            // step and takes a copy nobody reads.  (A load under a branch is
            // sunk behind the ring's loads, and its wait then drains them.)
            T vax, vag, vbx, vbg;
            blk_load(P, J, vax, vag);
            blk_load(J, Q, vbx, vbg);
            if constexpr (SP) {
#pragma unroll
                for (int o = 0; o < 3; ++o) {
                    mw[o] = mwn[o];
                    nm[o] = 0u;
                }
                if (m < Q - P) load_mask(m + 1);
            }
            if constexpr (!CP) fill_ring(m);
            blk_store(P, J, vax, vag, Ax0, Ag0);
            blk_store(J, Q, vbx, vbg, Bx0, Bg0);
            if constexpr (CP) {
                // the step's duals: the array is all zeros between steps
                // (zeroed once per workgroup, and each step's write-out
                // clears the slots it wrote), so only the list's entries
                // are stored
                const int64_t c = int64_t(tl.jsbase) + m;
                const uint32_t cnt = cp.cnt_in[c];
                const int64_t off = cp.off_in[c];
                for (uint32_t e = uint32_t(tid); e < cnt; e += uint32_t(bb)) {
                    const uint32_t sl = cp.idx_in[off + e];
                    if (sl < uint32_t(3 * b * bb)) ly[sl] = cp.val_in[off + e];
                }
            }
            lds_barrier();
            const T gC = Cg[tid];
            if (tid == 0 && a.prof) mark(1);

            // q of sub-step t (1 / sum of the three g), with the g of A and B
            auto gq = [&](int t, T &ga, T &gb) {
                const int jl = mid_offset(t, il, kl, b);
                ga = Ag[il * b + jl];
                gb = Bg[jl * b + kl];
                const T s = (ga + gC) + gb;
                return recip<T>(s > T(0) ? s : T(1));
            };
            T gan, gbn;
            T qn = gq(0, gan, gbn);
            // compacted lists: bit 3t + o set where this lane's dual (t, o)
            // ends the step nonzero (each is final once its sub-step ran)
            uint64_t nzm = 0;
            // D sub-steps, one per ring slot.  The first group is peeled off
            // the loop so that the loop is entered with the ring in the
            // state it has at every later iteration; the compiler's memory
            // waits at the loop head are then exact (a wait of 6D-3 accesses
            // per slot) rather than those of a freshly filled ring.  The last
            // group is peeled too: it refills nothing (the ring for the next
            // step is loaded after the release).
            auto group = [&](const int t0, const bool refill) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int t = t0 + d;
                    const int u = m * b + t;
                    const int sl = 3 * t * bb + int(lane);
                    T y0, y1, y2;
                    if constexpr (CP) {
                        y0 = ly[sl];
                        y1 = ly[sl + bb];
                        y2 = ly[sl + 2 * bb];
                    } else {
                        y0 = yq[d][0];
                        y1 = yq[d][1];
                        y2 = yq[d][2];
                    }
                    // The x reads go out first: they head the sub-step's
                    // dependent chain, and the reciprocal of q (x-independent)
                    // then runs in their latency instead of ahead of them.
                    const int jl = mid_offset(t, il, kl, b);
                    T xa = Ax[il * b + jl], xb = Bx[jl * b + kl], xc = Cx[tid];
                    __builtin_amdgcn_sched_barrier(0);
                    const T q = qn, ga = gan, gb = gbn;
                    if (t + 1 < b) qn = gq(t + 1, gan, gbn);
                    const int j = J * b + jl;
                    {
                        // Every lane runs the step; a lane whose (i,j,k) is
                        // padding takes q = 0 and floor -inf, which leaves its
                        // dual and the three distances exactly as read (the
                        // max returns its first operand's value whenever the
                        // floor is 0 and that operand is not below it).  Only
                        // triplet lanes write the distances back: where the
                        // middle block is P or Q, the A or B block is the
                        // resident (P,Q) block, and a padding lane's entry can
                        // be a triplet lane's entry of the same sub-step.
                        const bool ok = (i < j) & (j < k) & (k < nn);
                        const T qm = ok ? q : T(0);
                        const T floor_ = ok ? T(0) : T(-__builtin_huge_val());
                        project_lo(xa, xc, xb, ga, gC, gb, qm, floor_, y0);
                        project_lo(xc, xa, xb, gC, ga, gb, qm, floor_, y1);
                        project_lo(xb, xa, xc, gb, ga, gC, qm, floor_, y2);
                        if (ok) {
                            Ax[il * b + jl] = xa;
                            Bx[jl * b + kl] = xb;
                            Cx[tid] = xc;
                        }
                    }
                    if constexpr (CP) {
                        ly[sl] = y0;
                        ly[sl + bb] = y1;
                        ly[sl + 2 * bb] = y2;
                        nzm |= uint64_t(nonzero01(y0) | (nonzero01(y1) << 1) | (nonzero01(y2) << 2)) << (3 * t);
                    } else if constexpr (SP) {
                        // store only changed duals; mark the nonzero ones
                        const uint64_t b0 = dual_bits(y0), b1 = dual_bits(y1), b2 = dual_bits(y2);
                        const uint32_t ou = uint32_t(int64_t(u) * ystep * int64_t(sizeof(T)));
                        constexpr uint32_t os = uint32_t(bb * sizeof(T));
                        const uint32_t l = uint32_t(lane * sizeof(T));
                        // (under a branch: a wave with nothing to store skips
                        // the instruction, which would otherwise queue ahead
                        // of the ring's loads)
                        if (b0 != dual_bits(yq[d][0])) buf_store(y0, yr, ou + l);
                        if (b1 != dual_bits(yq[d][1])) buf_store(y1, yr, ou + os + l);
                        if (b2 != dual_bits(yq[d][2])) buf_store(y2, yr, ou + 2 * os + l);
                        if constexpr (lean) {
                            nm[0] |= nonzero01(y0) << t;
                            nm[1] |= nonzero01(y1) << t;
                            nm[2] |= nonzero01(y2) << t;
                        } else {
                            nm[0] |= uint32_t(b0 != 0) << t;
                            nm[1] |= uint32_t(b1 != 0) << t;
                            nm[2] |= uint32_t(b2 != 0) << t;
                        }
                    } else if constexpr (kBufDense) {
                        const uint32_t so = soff(u);
                        buf_store(y0, yr, voff(0), so);
                        buf_store(y1, yr, voff(1), so);
                        buf_store(y2, yr, voff(2), so);
                    } else {
                        T *const dst = ytile + int64_t(__builtin_amdgcn_readfirstlane(u)) * ystep;
                        __builtin_nontemporal_store(y0, &dst[lane]);
                        __builtin_nontemporal_store(y1, &dst[lane + bb]);
                        __builtin_nontemporal_store(y2, &dst[lane + 2 * bb]);
                    }
                    if (refill && !CP) {
                        // Refill slot d after its duals are consumed, so the
                        // old and new values never live at once (no register
                        // copies of loads in flight).
                        ring_load(d, ytile + int64_t(__builtin_amdgcn_readfirstlane(u + D)) * ystep, u + D, t + D);
                    }
                    lds_barrier();
                }
            };
            group(0, true);
#pragma nounroll
            for (int t0 = D; t0 < b - D; t0 += D) group(t0, true);
            group(b - D, false);
            if constexpr (CP) {
                // Write the step's nonzero duals to the output pool: a block
                // prefix over the threads' counts (slots k b^2 + tid), one
                // allocation per step, then each thread's entries in order.
                __shared__ uint32_t s_wave[B * B / 64];
                __shared__ unsigned long long s_base;
                __shared__ int s_fit;
                const uint32_t nz = uint32_t(__builtin_popcountll(nzm));
                uint32_t incl = nz;
#pragma unroll
                for (int sh = 1; sh < 64; sh <<= 1) {
                    const uint32_t v = __shfl_up(incl, sh, 64);
                    if ((tid & 63) >= sh) incl += v;
                }
                if ((tid & 63) == 63) s_wave[tid >> 6] = incl;
                lds_barrier();
                uint32_t before = 0, total = 0;
#pragma unroll
                for (int w = 0; w < bb / 64; ++w) {
                    const uint32_t v = s_wave[w];
                    if (w < (tid >> 6)) before += v;
                    total += v;
                }
                const int64_t c = int64_t(tl.jsbase) + m;
                if (tid == 0) {
                    const unsigned long long base = atomicAdd(cp.alloc, (unsigned long long)total);
                    const int fit = (base + total <= (unsigned long long)cp.cap) ? 1 : 0;
                    if (!fit) atomicOr(cp.overflow, 1u);
                    cp.off_out[c] = int64_t(base);
                    cp.cnt_out[c] = fit ? total : 0u;
                    s_base = base;
                    s_fit = fit;
                }
                lds_barrier();
                const bool fit = __builtin_amdgcn_readfirstlane(s_fit) != 0;
                int64_t pos = int64_t(s_base) + before + (incl - nz);
                while (nzm) {
                    const int k = __builtin_ctzll(nzm);
                    nzm &= nzm - 1;
                    const int e = k * bb + tid;
                    if (fit) {
                        cp.idx_out[pos] = uint16_t(e);
                        cp.val_out[pos] = ly[e];
                        ++pos;
                    }
                    ly[e] = T(0);  // leave the array all zeros for the next step
                }
            }
            if constexpr (SP) {
                MW *r = mask_row(m);
                const uint32_t flip = lean ? ~0u : 0u;
                if (MW(nm[0]) != MW(mw[0] ^ flip)) r[lane] = MW(nm[0]);
                if (MW(nm[1]) != MW(mw[1] ^ flip)) r[lane + bb] = MW(nm[1]);
                if (MW(nm[2]) != MW(mw[2] ^ flip)) r[lane + 2 * bb] = MW(nm[2]);
            }
            if (tid == 0 && a.prof) mark(2);

            // Publish this step's (P,J) and (J,Q) blocks (and (P,Q) after the
            // last step); release them; wait for the next step's blocks.
            const bool last = (m == Q - P);
            if (idA >= 0) publish(P, J, Ax0);
            if (idB >= 0) publish(J, Q, Bx0);
            if (last) publish(P, Q, Cx);
            // Release: every wave waits until its agent-scope stores are
            // complete (performed where every CU's agent-scope loads read),
            // then thread 0 raises the counters.  The readers poll the
            // counters and then load the blocks with agent-scope loads.  An
            // agent-scope release fence would add a write-back of every dirty
            // line in this XCD's L2, the dual stream's included, on every
            // tile step; that cost a quarter of the sweep time.
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0) {
                if (idA >= 0) __hip_atomic_fetch_add(&a.cnt[int64_t(idA) * kCntStride], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (idB >= 0) __hip_atomic_fetch_add(&a.cnt[int64_t(idB) * kCntStride], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                bool ok = true;
                if (last) {
                    __hip_atomic_fetch_add(&a.cnt[int64_t(idC) * kCntStride], uint32_t(Q - P + 1), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    s_tix = int(atomicAdd(&a.ctl[0], 1u));
                }
                if (a.prof) {
                    mark(3);
                    s_pt[4] += 1;
                }
                if (!last) {
                    ok = wait_step(m + 1, false);
                    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    if (a.prof) mark(0);
                }
                s_ok = ok;
            }
            __syncthreads();
            if (!__builtin_amdgcn_readfirstlane(s_ok)) {
                aborted = true;
                break;
            }
        }
        if (aborted) break;
    }
    if (tid == 0 && a.prof)
        for (int e = 0; e < 5; ++e) atomicAdd(&a.prof[e], (unsigned long long)s_pt[e]);
}

// A'y on the dataflow schedule: every tile step adds each triplet's three
// duals into the FP64 accumulators of its pairs (i,j): y0 - y1 - y2,
// (i,k): y1 - y0 - y2, (j,k): y2 - y0 - y1, with the same waits and the same
// order of additions per pair as the sweep, so the sums equal those of the
// round-by-round kernel bit for bit.  ax must hold zeros (or a partial sum)
// on entry.
template <typename T, int B, int D>
__global__ void __launch_bounds__(B * B)
k_aty_dataflow(DataflowArgs a, int64_t n, const T *__restrict__ y, double *__restrict__ ax) {
    static_assert(B % D == 0 && B >= 2 * D, "ring depth must divide b, twice at least");
    constexpr int b = B;
    constexpr int bb = B * B;
    const int tid = threadIdx.x;
    const int il = tid / b, kl = tid % b;
    const int sr = tid % b, sc = tid / b;
    const int nn = int(n);
    const int nb = (nn + b - 1) / b;
    __shared__ double Abuf[bb], Bbuf[bb], Cs[bb];
    __shared__ int s_tix, s_ok;

    if (tid == 0) s_tix = int(atomicAdd(&a.ctl[0], 1u));
    __syncthreads();
    for (;;) {
        const int tix = __builtin_amdgcn_readfirstlane(s_tix);
        if (tix >= a.ntiles) break;
        const DTile tl = a.tiles[tix];
        const int P = tl.P, Q = tl.Q;
        const bool desc = tile_desc(P, Q, nb);
        const int i = P * b + il, k = Q * b + kl;
        const int idC = block_id(P, Q);

        auto blk_ok = [&](int R, int S) {
            const int ii = R * b + sr, jj = S * b + sc;
            return ii < jj && jj < nn;
        };
        // ax is read and written with agent-scope atomic accesses, released
        // as in the sweep: stores complete in every wave, then the counters.
        auto blk_load = [&](int R, int S) {
            return __hip_atomic_load(&ax[blk_ok(R, S) ? pidx(R * b + sr, S * b + sc) : 0], __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_AGENT);
        };
        auto blk_store = [&](int R, int S, double v, double *X) { X[sr * b + sc] = blk_ok(R, S) ? v : 0.0; };
        auto stage = [&](int R, int S, double *X) { blk_store(R, S, blk_load(R, S), X); };
        auto publish = [&](int R, int S, const double *X) {
            if (blk_ok(R, S))
                __hip_atomic_store(&ax[pidx(R * b + sr, S * b + sc)], X[sr * b + sc], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        };
        auto step_ids = [&](int m, int &idA, int &idB) {
            const int J = tile_J(P, Q, m, desc);
            idA = (J != Q) ? block_id(P, J) : -1;
            idB = (J != P) ? block_id(J, Q) : -1;
        };
        // thread 0: wait for step m's blocks (and, with withC, for (P,Q))
        auto wait_step = [&](int m, bool withC) {
            int idA, idB;
            step_ids(m, idA, idB);
            const uint32_t *nd = a.needs + 2 * int64_t(tl.jsbase + m);
            uint32_t *const none = &a.ctl[1];
            return wait_counts(idA >= 0 ? &a.cnt[int64_t(idA) * kCntStride] : none,
                               idA >= 0 ? a.epoch * a.K[idA] + nd[0] : 0u,
                               idB >= 0 ? &a.cnt[int64_t(idB) * kCntStride] : none,
                               idB >= 0 ? a.epoch * a.K[idB] + nd[1] : 0u,
                               withC ? &a.cnt[int64_t(idC) * kCntStride] : none,
                               withC ? a.epoch * a.K[idC] + tl.needC : 0u, &a.ctl[1], a.wait_ticks);
        };

        const T *const ytile = y + tl.ybase;
        const int64_t ystep = int64_t(3) * bb;
        const unsigned lane = unsigned(tid);
        T yq[D][3];
        auto fill_ring = [&](int m) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const T *src = ytile + int64_t(m * b + d) * ystep;
                yq[d][0] = __builtin_nontemporal_load(&src[lane]);
                yq[d][1] = __builtin_nontemporal_load(&src[lane + bb]);
                yq[d][2] = __builtin_nontemporal_load(&src[lane + 2 * bb]);
            }
        };

        if (tid == 0) {
            const bool ok = wait_step(0, true);
            if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_ok = ok;
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(s_ok)) break;
        stage(P, Q, Cs);

        bool aborted = false;
        for (int m = 0; m <= Q - P; ++m) {
            const int J = tile_J(P, Q, m, desc);
            int idA, idB;
            step_ids(m, idA, idB);
            double *const Ab = (J == Q) ? Cs : Abuf;
            double *const Bb = (J == P) ? Cs : Bbuf;
            // unconditional, as in the sweep (Abuf / Bbuf are idle where A
            // or B is the resident block)
            const double va = blk_load(P, J), vb = blk_load(J, Q);
            fill_ring(m);
            blk_store(P, J, va, Abuf);
            blk_store(J, Q, vb, Bbuf);
            lds_barrier();
            auto group = [&](const int t0, const bool refill) {
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    const int t = t0 + d;
                    const int u = m * b + t;
                    const double y0 = double(yq[d][0]), y1 = double(yq[d][1]), y2 = double(yq[d][2]);
                    const int jl = mid_offset(t, il, kl, b);
                    const int j = J * b + jl;
                    if (i < j && j < k && k < nn) {
                        Ab[il * b + jl] += (y0 - y1) - y2;  // pair (i,j)
                        Cs[tid] += (y1 - y0) - y2;          // pair (i,k)
                        Bb[jl * b + kl] += (y2 - y0) - y1;  // pair (j,k)
                    }
                    if (refill) {
                        const T *src = ytile + int64_t(u + D) * ystep;
                        yq[d][0] = __builtin_nontemporal_load(&src[lane]);
                        yq[d][1] = __builtin_nontemporal_load(&src[lane + bb]);
                        yq[d][2] = __builtin_nontemporal_load(&src[lane + 2 * bb]);
                    }
                    lds_barrier();
                }
            };
            group(0, true);
#pragma nounroll
            for (int t0 = D; t0 < b - D; t0 += D) group(t0, true);
            group(b - D, false);

            const bool last = (m == Q - P);
            if (idA >= 0) publish(P, J, Abuf);
            if (idB >= 0) publish(J, Q, Bbuf);
            if (last) publish(P, Q, Cs);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0) {
                if (idA >= 0) __hip_atomic_fetch_add(&a.cnt[int64_t(idA) * kCntStride], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (idB >= 0) __hip_atomic_fetch_add(&a.cnt[int64_t(idB) * kCntStride], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                bool ok = true;
                if (last) {
                    __hip_atomic_fetch_add(&a.cnt[int64_t(idC) * kCntStride], uint32_t(Q - P + 1), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    s_tix = int(atomicAdd(&a.ctl[0], 1u));
                } else {
                    ok = wait_step(m + 1, false);
                    if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                }
                s_ok = ok;
            }
            __syncthreads();
            if (!__builtin_amdgcn_readfirstlane(s_ok)) {
                aborted = true;
                break;
            }
        }
        if (aborted) break;
    }
}

__global__ void k_dataflow_reset(uint32_t *ctl) {
    if (threadIdx.x == 0) {
        ctl[0] = 0u;
    }
}

int launch_dataflow_reset(uint32_t *ctl, hipStream_t s) {
    hipLaunchKernelGGL(k_dataflow_reset, dim3(1), dim3(64), 0, s, ctl);
    CCP_LAUNCH_CHECK("k_dataflow_reset");
    return CC_OK;
}

__global__ void k_fill_u32(int64_t count, uint32_t *a) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += int64_t(gridDim.x) * blockDim.x)
        a[e] = 0u;
}

// The mask of a dual array: bit t of word [c][o][lane] is set where slot
// (t, o, lane) of tile step c holds a dual whose bits are not +0.0.
template <typename T, int B>
__global__ void __launch_bounds__(B * B)
k_mask_build(int64_t nsteps, const T *__restrict__ y, typename MaskWord<B>::type *__restrict__ mask) {
    using MW = typename MaskWord<B>::type;
    constexpr int bb = B * B;
    const int lane = threadIdx.x;
    for (int64_t c = blockIdx.x; c < nsteps; c += gridDim.x) {
        const T *yc = y + c * 3 * B * bb;
        uint32_t w0 = 0u, w1 = 0u, w2 = 0u;
#pragma unroll 4
        for (int t = 0; t < B; ++t) {
            const T *r = yc + int64_t(t) * 3 * bb;
            w0 |= uint32_t(dual_bits(__builtin_nontemporal_load(&r[lane])) != 0) << t;
            w1 |= uint32_t(dual_bits(__builtin_nontemporal_load(&r[lane + bb])) != 0) << t;
            w2 |= uint32_t(dual_bits(__builtin_nontemporal_load(&r[lane + 2 * bb])) != 0) << t;
        }
        MW *m = mask + c * 3 * bb;
        m[lane] = MW(w0);
        m[lane + bb] = MW(w1);
        m[lane + 2 * bb] = MW(w2);
    }
}

template <typename T, int B>
static int launch_mask_build_t(int64_t nsteps, const T *y, void *mask, hipStream_t s) {
    if (nsteps <= 0) return CC_OK;
    const int64_t grid = nsteps < (int64_t(1) << 20) ? nsteps : (int64_t(1) << 20);
    hipLaunchKernelGGL((k_mask_build<T, B>), dim3(unsigned(grid)), dim3(B * B), 0, s, nsteps, y,
                       static_cast<typename MaskWord<B>::type *>(mask));
    CCP_LAUNCH_CHECK("k_mask_build");
    return CC_OK;
}

template <typename T>
int launch_mask_build(int b, int64_t nsteps, const T *y, void *mask, hipStream_t s) {
    switch (b) {
        case 8: return launch_mask_build_t<T, 8>(nsteps, y, mask, s);
        case 16: return launch_mask_build_t<T, 16>(nsteps, y, mask, s);
        case 24: return launch_mask_build_t<T, 24>(nsteps, y, mask, s);
        case 32: return launch_mask_build_t<T, 32>(nsteps, y, mask, s);
        default: return fail(CC_EINVAL, "sparse dual access supports b = 8, 16, 24, 32");
    }
}

template <typename T>
size_t dataflow_lds_bytes(int b) {
    return size_t(6) * b * b * sizeof(T);
}

// Ring depth of the sparse sweep: the mask state does not fit beside the
// dense sweep's ring without spilling at b = 24 (576 threads, at most 168
// VGPRs a lane; a ring of 8 sub-steps) nor at b = 32 in FP64 (1024
// threads, at most 128; a ring of 4), so those keep 4 and 2.
template <typename T, int B, int D> constexpr int sparse_ring() {
    return B == 24 ? 4 : (B == 32 ? (sizeof(T) == 8 ? 2 : 4) : D);
}
// Ring depth of the dense sweep at b = 32.
template <typename T> constexpr int kDenseRing32 = sizeof(T) == 4 ? 8 : 4;

template <typename T, int B, int D>
static int launch_df_t(const DataflowArgs &a, int grid, int64_t n, T *x, const T *g, T *y,
                       void *mask, const CompactArgs<T> *cp, hipStream_t s) {
    using MW = typename MaskWord<B>::type;
    const size_t lds = dataflow_lds_bytes<T>(B);
    hipLaunchKernelGGL(k_dataflow_reset, dim3(1), dim3(64), 0, s, a.ctl);
    CCP_LAUNCH_CHECK("k_dataflow_reset");
    if (cp) {
        if constexpr (B <= 16) {
            const size_t lds_cp = lds + size_t(3) * B * B * B * sizeof(T);
            const hipError_t e = hipFuncSetAttribute((const void *)k_sweep_dataflow<T, B, D, false, true>,
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_cp));
            if (e != hipSuccess) return fail(CC_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
            hipLaunchKernelGGL((k_sweep_dataflow<T, B, D, false, true>), dim3(grid), dim3(B * B), lds_cp, s, a, n,
                               x, g, y, static_cast<MW *>(nullptr), *cp);
        } else {
            return fail(CC_EINVAL, "compacted dual lists need b = 8 or 16");
        }
    } else if (mask) {
        if constexpr (kSparseB<B>) {
            hipLaunchKernelGGL((k_sweep_dataflow<T, B, sparse_ring<T, B, D>(), true, false>), dim3(grid), dim3(B * B),
                               lds, s, a, n, x, g, y, static_cast<MW *>(mask), CompactArgs<T>{});
        } else {
            return fail(CC_EINVAL, "sparse dual access needs b = 8, 16, 24 or 32");
        }
    } else {
        hipLaunchKernelGGL((k_sweep_dataflow<T, B, D, false, false>), dim3(grid), dim3(B * B), lds, s, a, n, x, g,
                           y, static_cast<MW *>(nullptr), CompactArgs<T>{});
    }
    CCP_LAUNCH_CHECK("k_sweep_dataflow");
    return CC_OK;
}

// mask == nullptr and cp == nullptr: the dense sweep; mask: the sparse one
// with this mask; cp: the compacted-list one (y unused).
template <typename T>
int launch_sweep_dataflow(const DataflowArgs &a, int grid, int b, int64_t n, T *x, const T *g,
                          T *y, void *mask, const CompactArgs<T> *cp, hipStream_t s) {
    switch (b) {
        case 8: return launch_df_t<T, 8, 4>(a, grid, n, x, g, y, mask, cp, s);
        case 16: return launch_df_t<T, 16, 8>(a, grid, n, x, g, y, mask, cp, s);
        case 24: return launch_df_t<T, 24, 8>(a, grid, n, x, g, y, mask, cp, s);
        // b = 32: a ring of 8 sub-steps in FP32 (127 registers a lane, no
        // spill; n = 4000 48.9 against 49.9 ms with 4), 4 in FP64 (8 spills)
        case 32: return launch_df_t<T, 32, kDenseRing32<T>>(a, grid, n, x, g, y, mask, cp, s);
        default: return fail(CC_EINVAL, "the dataflow executor supports b = 8, 16, 24, 32");
    }
}

// Dense schedule-ordered duals from compacted lists (y zero-filled first):
// one block per step, threads over its entries.
template <typename T, int B>
__global__ void __launch_bounds__(256)
k_compact_to_slots(int64_t nsteps, const uint16_t *__restrict__ idx, const T *__restrict__ val,
                   const int64_t *__restrict__ off, const uint32_t *__restrict__ cnt, T *__restrict__ y) {
    constexpr int64_t per = int64_t(3) * B * B * B;
    for (int64_t c = blockIdx.x; c < nsteps; c += gridDim.x) {
        const uint32_t k = cnt[c];
        const int64_t o = off[c];
        for (uint32_t e = threadIdx.x; e < k; e += blockDim.x) {
            const uint32_t sl = idx[o + e];
            if (sl < uint32_t(per)) y[c * per + sl] = val[o + e];
        }
    }
}

// The entries of compacted lists as (colex row index 3 tidx(i,j,k) + o,
// dual), at their pool positions.  step_tile[c] is step c's tile.
template <typename T, int B>
__global__ void __launch_bounds__(256)
k_compact_export(int64_t nsteps, int nb, const DTile *__restrict__ tiles, const int32_t *__restrict__ step_tile,
                 const uint16_t *__restrict__ idx, const T *__restrict__ val, const int64_t *__restrict__ off,
                 const uint32_t *__restrict__ cnt, int64_t *__restrict__ lex, T *__restrict__ out) {
    constexpr int bb = B * B;
    for (int64_t c = blockIdx.x; c < nsteps; c += gridDim.x) {
        const DTile tl = tiles[step_tile[c]];
        const int m = int(c - tl.jsbase);
        const int J = tile_J(tl.P, tl.Q, m, tile_desc(tl.P, tl.Q, nb));
        const uint32_t k = cnt[c];
        const int64_t o = off[c];
        for (uint32_t e = threadIdx.x; e < k; e += blockDim.x) {
            const int sl = idx[o + e];
            const int t = sl / (3 * bb), rem = sl % (3 * bb), or_ = rem / bb, lane = rem % bb;
            const int il = lane / B, kl = lane % B, jl = mid_offset(t, il, kl, B);
            const int64_t i = int64_t(tl.P) * B + il, j = int64_t(J) * B + jl, kk = int64_t(tl.Q) * B + kl;
            lex[o + e] = 3 * tidx(i, j, kk) + or_;
            out[o + e] = val[o + e];
        }
    }
}

template <typename T>
int launch_compact_to_slots(int b, int64_t nsteps, const uint16_t *idx, const T *val, const int64_t *off,
                            const uint32_t *cnt, T *y, hipStream_t s) {
    const int64_t grid = nsteps < (int64_t(1) << 20) ? nsteps : (int64_t(1) << 20);
    if (grid <= 0) return CC_OK;
    switch (b) {
        case 8: hipLaunchKernelGGL((k_compact_to_slots<T, 8>), dim3(unsigned(grid)), dim3(256), 0, s, nsteps, idx, val, off, cnt, y); break;
        case 16: hipLaunchKernelGGL((k_compact_to_slots<T, 16>), dim3(unsigned(grid)), dim3(256), 0, s, nsteps, idx, val, off, cnt, y); break;
        default: return fail(CC_EINVAL, "compacted dual lists need b = 8 or 16");
    }
    CCP_LAUNCH_CHECK("k_compact_to_slots");
    return CC_OK;
}

template <typename T>
int launch_compact_export(int b, int64_t nsteps, int nb, const DTile *tiles, const int32_t *step_tile,
                          const uint16_t *idx, const T *val, const int64_t *off, const uint32_t *cnt,
                          int64_t *lex, T *out, hipStream_t s) {
    const int64_t grid = nsteps < (int64_t(1) << 20) ? nsteps : (int64_t(1) << 20);
    if (grid <= 0) return CC_OK;
    switch (b) {
        case 8: hipLaunchKernelGGL((k_compact_export<T, 8>), dim3(unsigned(grid)), dim3(256), 0, s, nsteps, nb, tiles, step_tile, idx, val, off, cnt, lex, out); break;
        case 16: hipLaunchKernelGGL((k_compact_export<T, 16>), dim3(unsigned(grid)), dim3(256), 0, s, nsteps, nb, tiles, step_tile, idx, val, off, cnt, lex, out); break;
        default: return fail(CC_EINVAL, "compacted dual lists need b = 8 or 16");
    }
    CCP_LAUNCH_CHECK("k_compact_export");
    return CC_OK;
}

template <typename T>
int dataflow_occupancy(int b, int *blocks_per_cu) {
    hipError_t e = hipSuccess;
    const int lds = int(dataflow_lds_bytes<T>(b));
    switch (b) {
        case 8:
            e = hipFuncSetAttribute((const void *)k_sweep_dataflow<T, 8, 4, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e == hipSuccess) e = hipFuncSetAttribute((const void *)k_sweep_dataflow<T, 8, sparse_ring<T, 8, 4>(), true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_sweep_dataflow<T, 8, 4, false, false>, 64, lds);
            break;
        case 16:
            e = hipFuncSetAttribute((const void *)k_sweep_dataflow<T, 16, 8, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e == hipSuccess) e = hipFuncSetAttribute((const void *)k_sweep_dataflow<T, 16, sparse_ring<T, 16, 8>(), true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_sweep_dataflow<T, 16, 8, false, false>, 256, lds);
            break;
        case 24:
            e = hipFuncSetAttribute((const void *)k_sweep_dataflow<T, 24, 8, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e == hipSuccess) e = hipFuncSetAttribute((const void *)k_sweep_dataflow<T, 24, sparse_ring<T, 24, 8>(), true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_sweep_dataflow<T, 24, 8, false, false>, 576, lds);
            break;
        case 32:
            e = hipFuncSetAttribute((const void *)k_sweep_dataflow<T, 32, kDenseRing32<T>, false, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e == hipSuccess) e = hipFuncSetAttribute((const void *)k_sweep_dataflow<T, 32, sparse_ring<T, 32, kDenseRing32<T>>(), true, false>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_sweep_dataflow<T, 32, kDenseRing32<T>, false, false>, 1024, lds);
            break;
        default:
            *blocks_per_cu = 0;
            return CC_OK;
    }
    if (e != hipSuccess) return fail(CC_EHIP, std::string("dataflow occupancy: ") + hipGetErrorString(e));
    return CC_OK;
}

template <typename T, int B, int D>
static int launch_aty_df_t(const DataflowArgs &a, int grid, int64_t n, const T *y, double *ax,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_dataflow_reset, dim3(1), dim3(64), 0, s, a.ctl);
    CCP_LAUNCH_CHECK("k_dataflow_reset");
    hipLaunchKernelGGL((k_aty_dataflow<T, B, D>), dim3(grid), dim3(B * B), 0, s, a, n, y, ax);
    CCP_LAUNCH_CHECK("k_aty_dataflow");
    return CC_OK;
}

template <typename T>
int launch_aty_dataflow(const DataflowArgs &a, int grid, int b, int64_t n, const T *y, double *ax,
                        hipStream_t s) {
    switch (b) {
        case 8: return launch_aty_df_t<T, 8, 4>(a, grid, n, y, ax, s);
        case 16: return launch_aty_df_t<T, 16, 8>(a, grid, n, y, ax, s);
        case 24: return launch_aty_df_t<T, 24, 8>(a, grid, n, y, ax, s);
        case 32: return launch_aty_df_t<T, 32, 4>(a, grid, n, y, ax, s);
        default: return fail(CC_EINVAL, "the dataflow executor supports b = 8, 16, 24, 32");
    }
}

template <typename T>
int aty_dataflow_occupancy(int b, int *blocks_per_cu) {
    hipError_t e = hipSuccess;
    switch (b) {
        case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_aty_dataflow<T, 8, 4>, 64, 0); break;
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_aty_dataflow<T, 16, 8>, 256, 0); break;
        case 24: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_aty_dataflow<T, 24, 8>, 576, 0); break;
        case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_aty_dataflow<T, 32, 4>, 1024, 0); break;
        default: *blocks_per_cu = 0; return CC_OK;
    }
    if (e != hipSuccess) return fail(CC_EHIP, std::string("A'y occupancy: ") + hipGetErrorString(e));
    return CC_OK;
}

int launch_fill_u32(int64_t count, uint32_t *a, hipStream_t s) {
    if (count <= 0) return CC_OK;
    int64_t grid = (count + 255) / 256;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_fill_u32, dim3(unsigned(grid)), dim3(256), 0, s, count, a);
    CCP_LAUNCH_CHECK("k_fill_u32");
    return CC_OK;
}

template int launch_sweep_dataflow<double>(const DataflowArgs &, int, int, int64_t, double *,
                                           const double *, double *, void *, const CompactArgs<double> *,
                                           hipStream_t);
template int launch_sweep_dataflow<float>(const DataflowArgs &, int, int, int64_t, float *,
                                          const float *, float *, void *, const CompactArgs<float> *,
                                          hipStream_t);
template int launch_compact_to_slots<double>(int, int64_t, const uint16_t *, const double *, const int64_t *,
                                             const uint32_t *, double *, hipStream_t);
template int launch_compact_to_slots<float>(int, int64_t, const uint16_t *, const float *, const int64_t *,
                                            const uint32_t *, float *, hipStream_t);
template int launch_compact_export<double>(int, int64_t, int, const DTile *, const int32_t *, const uint16_t *,
                                           const double *, const int64_t *, const uint32_t *, int64_t *,
                                           double *, hipStream_t);
template int launch_compact_export<float>(int, int64_t, int, const DTile *, const int32_t *, const uint16_t *,
                                          const float *, const int64_t *, const uint32_t *, int64_t *, float *,
                                          hipStream_t);
template int launch_mask_build<double>(int, int64_t, const double *, void *, hipStream_t);
template int launch_mask_build<float>(int, int64_t, const float *, void *, hipStream_t);
template int launch_aty_dataflow<double>(const DataflowArgs &, int, int, int64_t, const double *, double *, hipStream_t);
template int launch_aty_dataflow<float>(const DataflowArgs &, int, int, int64_t, const float *, double *, hipStream_t);
template int aty_dataflow_occupancy<double>(int, int *);
template int aty_dataflow_occupancy<float>(int, int *);
template int dataflow_occupancy<double>(int, int *);
template int dataflow_occupancy<float>(int, int *);

}  // namespace ccp
