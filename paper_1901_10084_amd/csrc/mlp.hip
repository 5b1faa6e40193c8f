// mlp.hip -- the learned warm start: a 4-32-32-1 network that predicts a
// nonnegative dual for every metric row from local features, trained on
// converged duals.  A warm start is valid because Algorithm 1 is dual
// coordinate ascent: it converges from any y >= 0 started at x = x(y).
//
// Network: ReLU after every layer, mean squared error of the output, with the
// output ReLU's gradient passed through where the target is positive (a row
// whose target is 0 is fitted by any output <= 0).  Parameters are one
// flat fp32 vector: W1[32][4], b1[32], W2[32][32], b2[32], W3[32], b3.
// Products take bf16 operands (phi, W1, h1, W2, h2, W3; in the backward pass
// delta2 before it meets W2 and h1) and accumulate in fp32.
//
// Layout on a 64-lane wave: lane l works on sample s = l % 16 of a group of
// 16 samples and on the units U_g = {4g..4g+3, 16+4g..16+4g+3}, g = l / 16.
// The 32x32 layer and its transpose run on v_mfma_f32_16x16x32_bf16 with the
// K index permuted so that a lane's 8 K slots are exactly its units U_g:
// the B operand is then the lane's own h1 (forward) or delta2 (backward) and
// the D rows it receives are again units U_g, so every layer stays in
// registers.  The weight gradient dW2 = sum over samples of delta2 h1^T is an
// MFMA with K = 32 samples, fed through a small LDS transpose.
#include <type_traits>

#include "common.hpp"
#include "dataflow.hpp"
#include "project.hpp"

namespace ccp {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(2))) float f32x2;

constexpr int kNParam = 1249;
constexpr int oW1 = 0, oB1 = 128, oW2 = 160, oB2 = 1184, oW3 = 1216, oB3 = 1248;

__host__ __device__ __forceinline__ int unit_of(int g, int q) {
    return q < 4 ? 4 * g + q : 16 + 4 * g + (q - 4);
}

// Round to the nearest bfloat16 (ties to even): the hardware conversion,
// two values per instruction.
__device__ __forceinline__ bf16x2 tobf2(float a, float b) {
    const f32x2 v = {a, b};
    return __builtin_convertvector(v, bf16x2);
}
__device__ __forceinline__ float bf16r(float v) { return float(tobf2(v, 0.0f)[0]); }
__device__ __forceinline__ __bf16 tobf(float v) { return tobf2(v, 0.0f)[0]; }

struct LaneNet {
    float w1[8][4];
    float b1[8];
    bf16x8 a2[2];   // a2[t][q]  = W2[16t + i][U_g[q]]   (forward)
    bf16x8 a2t[2];  // a2t[t][q] = W2[U_g[q]][16t + i]   (backward, transposed)
    float b2[8];
    float w3[8];
    float b3;
};

__device__ __forceinline__ void load_net(LaneNet &N, const float *__restrict__ P) {
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int u = unit_of(g, q);
#pragma unroll
        for (int k = 0; k < 4; ++k) N.w1[q][k] = bf16r(P[oW1 + u * 4 + k]);
        N.b1[q] = P[oB1 + u];
        N.b2[q] = P[oB2 + u];
        N.w3[q] = bf16r(P[oW3 + u]);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            N.a2[t][q] = tobf(P[oW2 + (16 * t + i) * 32 + u]);
            N.a2t[t][q] = tobf(P[oW2 + u * 32 + 16 * t + i]);
        }
    }
    N.b3 = P[oB3];
}

struct Fwd {
    float z1[8], h1[8], z2[8], h2[8];
    float z3, y;
};

// Forward pass of the lane's sample (phi already bf16-rounded).
__device__ __forceinline__ void forward(const LaneNet &N, const float phi[4], Fwd &F) {
    bf16x8 bh;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        float z = N.b1[q];
#pragma unroll
        for (int k = 0; k < 4; ++k) z = fmaf(N.w1[q][k], phi[k], z);
        F.z1[q] = z;
    }
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
        const bf16x2 h = tobf2(fmaxf(F.z1[q], 0.0f), fmaxf(F.z1[q + 1], 0.0f));
        bh[q] = h[0];
        bh[q + 1] = h[1];
        F.h1[q] = float(h[0]);
        F.h1[q + 1] = float(h[1]);
    }
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    const f32x4 d0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a2[0], bh, zero, 0, 0, 0);
    const f32x4 d1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a2[1], bh, zero, 0, 0, 0);
    float part = 0.0f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        F.z2[r] = d0[r] + N.b2[r];
        F.z2[4 + r] = d1[r] + N.b2[4 + r];
    }
#pragma unroll
    for (int q = 0; q < 8; q += 2) {
        const bf16x2 h = tobf2(fmaxf(F.z2[q], 0.0f), fmaxf(F.z2[q + 1], 0.0f));
        F.h2[q] = float(h[0]);
        F.h2[q + 1] = float(h[1]);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) part = fmaf(N.w3[q], F.h2[q], part);
    part += __shfl_xor(part, 16, 64);
    part += __shfl_xor(part, 32, 64);
    F.z3 = part + N.b3;
    F.y = fmaxf(F.z3, 0.0f);
}

// ---------------------------------------------------------------------------
// Metric-row features (the reading of "3 edge weights + endpoint degrees"):
// for the row with long side (a,b) and apex c,
// (s_ab w_ab, s_ac w_ac, s_bc w_bc, (deg_a + deg_b) / (2 mean deg)),
// s = +1 for a positive pair, -1 for a negative one.  Rounded to bf16.
// ---------------------------------------------------------------------------

// Decodes schedule slot s of tile tl; false for padding.
__device__ __forceinline__ bool decode_slot(const Tile &tl, int64_t s, int b, int64_t n, int64_t &i,
                                            int64_t &j, int64_t &k, int &o) {
    const int64_t bb = int64_t(b) * b;
    const int64_t off = s - tl.ybase;
    const int64_t u = off / (3 * bb), rem = off - u * 3 * bb;
    o = int(rem / bb);
    const int lane = int(rem - int64_t(o) * bb);
    const int il = lane / b, kl = lane - (lane / b) * b;
    const int m = int(u / b), t = int(u - int64_t(m) * b);
    const int nb = int((n + b - 1) / b);
    const int J = tile_J(tl.P, tl.Q, m, tile_desc(tl.P, tl.Q, nb));
    i = int64_t(tl.P) * b + il;
    k = int64_t(tl.Q) * b + kl;
    j = int64_t(J) * b + mid_offset(t, il, kl, b);
    return m <= tl.Q - tl.P && i < j && j < k && k < n;
}

__device__ __forceinline__ void row_features(const GraphView &G, int64_t i, int64_t j, int64_t k,
                                             int o, float phi[4]) {
    const int64_t pij = pidx(i, j), pik = pidx(i, k), pjk = pidx(j, k);
    const int64_t L = o == 0 ? pij : (o == 1 ? pik : pjk);
    const int64_t S1 = o == 2 ? pij : (o == 1 ? pij : pik);
    const int64_t S2 = o == 0 ? pjk : (o == 1 ? pjk : pik);
    const int64_t a = o == 2 ? j : i;
    const int64_t bn = o == 0 ? j : k;
    auto sw = [&](int64_t p) { return float(G.d[p] == 0 ? G.w[p] : -G.w[p]); };
    const float md = G.mean_deg[0];
    phi[0] = bf16r(sw(L));
    phi[1] = bf16r(sw(S1));
    phi[2] = bf16r(sw(S2));
    phi[3] = bf16r(md > 0.0f ? (G.deg[a] + G.deg[bn]) / (2.0f * md) : 0.0f);
}

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // splitmix64 finaliser
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Sample sources for training.
struct ExplicitSource {
    const float *phi;
    const float *target;
    int64_t count;
    __device__ void get(int64_t idx, float phi[4], float &t, float &wgt) const {
        const bool ok = idx < count;
        const int64_t e = ok ? idx : 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) phi[k] = bf16r(this->phi[4 * e + k]);
        t = this->target[e];
        wgt = ok ? 1.0f : 0.0f;
    }
};

template <typename T>
struct GraphSource {
    GraphView G;
    const T *ystar;   // converged duals, schedule order
    int64_t slots;
    uint64_t seed;
    int64_t count;    // samples in the batch
    __device__ void get(int64_t idx, float phi[4], float &t, float &wgt) const {
        const int64_t s = int64_t(mix64(seed ^ (uint64_t(idx) * 0xD1B54A32D192ED03ull)) %
                                  uint64_t(slots));
        int64_t lo = 0, hi = G.ntiles - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (G.tiles[mid].ybase <= s) lo = mid; else hi = mid - 1;
        }
        int64_t i, j, k;
        int o;
        const bool ok = idx < count && decode_slot(G.tiles[lo], s, G.b, G.n, i, j, k, o);
        if (ok) {
            row_features(G, i, j, k, o, phi);
        } else {
            phi[0] = phi[1] = phi[2] = phi[3] = 0.0f;
        }
        // target: the dual times n - 2 (see k_mlp_infer)
        t = ok ? float(ystar[s]) * float(G.n - 2) : 0.0f;
        wgt = ok ? 1.0f : 0.0f;
    }
};

// ---------------------------------------------------------------------------
// Training: one wave per workgroup; chunks of 32 samples; per-workgroup
// partial gradients (kNParam values + the loss) in a fixed order.
// ---------------------------------------------------------------------------
template <typename Src>
__global__ void __launch_bounds__(64)
k_mlp_grad(Src src, int64_t count, float inv_norm, const float *__restrict__ P,
           float *__restrict__ partial) {
    __shared__ __bf16 D2s[32][32];
    __shared__ __bf16 H1s[32][32];
    const int lane = threadIdx.x, j = lane & 15, g = lane >> 4;
    LaneNet N;
    load_net(N, P);
    float gW1[8][4], gb1[8], gb2[8], gW3[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        gb1[q] = gb2[q] = gW3[q] = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) gW1[q][k] = 0.0f;
    }
    float gb3 = 0.0f, loss = 0.0f;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[a][c] = f32x4{0.f, 0.f, 0.f, 0.f};

    const int64_t nchunks = (count + 31) / 32;
    for (int64_t c = blockIdx.x; c < nchunks; c += gridDim.x) {
#pragma unroll
        for (int G = 0; G < 2; ++G) {
            float phi[4], t, wgt;
            src.get(32 * c + 16 * G + j, phi, t, wgt);
            Fwd F;
            forward(N, phi, F);
            // squared error of the ReLU output; where the target is
            // positive the output ReLU passes the gradient, so a row pushed
            // below zero can still learn a positive dual
            const float r = (t > 0.0f) ? F.z3 - t : F.y;
            if (g == 0) loss = fmaf(wgt * r, r, loss);
            const float d3 = (t > 0.0f || F.z3 > 0.0f) ? wgt * 2.0f * r * inv_norm : 0.0f;
            if (g == 0) gb3 += d3;
            bf16x8 bd2;
            float d2b[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                gW3[q] = fmaf(d3, F.h2[q], gW3[q]);
                const float d2 = (F.z2[q] > 0.0f) ? d3 * N.w3[q] : 0.0f;
                gb2[q] += d2;
                d2b[q] = bf16r(d2);
                bd2[q] = tobf(d2b[q]);
            }
            const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
            const f32x4 e0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a2t[0], bd2, zero, 0, 0, 0);
            const f32x4 e1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a2t[1], bd2, zero, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float dh1 = q < 4 ? e0[q] : e1[q - 4];
                const float d1 = F.z1[q] > 0.0f ? dh1 : 0.0f;
                gb1[q] += d1;
#pragma unroll
                for (int k = 0; k < 4; ++k) gW1[q][k] = fmaf(d1, phi[k], gW1[q][k]);
                D2s[16 * G + j][unit_of(g, q)] = tobf(d2b[q]);
                H1s[16 * G + j][unit_of(g, q)] = tobf(F.h1[q]);
            }
        }
        __syncthreads();
        // dW2 += sum over the 32 samples of delta2 h1^T (K = samples)
#pragma unroll
        for (int Mt = 0; Mt < 2; ++Mt) {
            bf16x8 A;
#pragma unroll
            for (int q = 0; q < 8; ++q) A[q] = D2s[8 * g + q][16 * Mt + j];
#pragma unroll
            for (int Nt = 0; Nt < 2; ++Nt) {
                bf16x8 Bv;
#pragma unroll
                for (int q = 0; q < 8; ++q) Bv[q] = H1s[8 * g + q][16 * Nt + j];
                acc[Mt][Nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bv, acc[Mt][Nt], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // Reduce the per-sample accumulators over the 16 lanes of a unit group.
    auto red16 = [](float v) {
#pragma unroll
        for (int m = 1; m < 16; m <<= 1) v += __shfl_xor(v, m, 64);
        return v;
    };
    float *out = partial + int64_t(blockIdx.x) * (kNParam + 1);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int u = unit_of(g, q);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float v = red16(gW1[q][k]);
            if (j == 0) out[oW1 + u * 4 + k] = v;
        }
        const float vb1 = red16(gb1[q]), vb2 = red16(gb2[q]), vw3 = red16(gW3[q]);
        if (j == 0) {
            out[oB1 + u] = vb1;
            out[oB2 + u] = vb2;
            out[oW3 + u] = vw3;
        }
    }
    // acc[Mt][Nt][r] = dW2[16 Mt + 4 g + r][16 Nt + j]
#pragma unroll
    for (int Mt = 0; Mt < 2; ++Mt)
#pragma unroll
        for (int Nt = 0; Nt < 2; ++Nt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[oW2 + (16 * Mt + 4 * g + r) * 32 + 16 * Nt + j] = acc[Mt][Nt][r];
    float v3 = red16(gb3), vl = red16(loss);
    v3 += __shfl_xor(v3, 16, 64);
    v3 += __shfl_xor(v3, 32, 64);
    vl += __shfl_xor(vl, 16, 64);
    vl += __shfl_xor(vl, 32, 64);
    if (lane == 0) {
        out[oB3] = v3;
        out[kNParam] = vl;
    }
}

// Sum of the per-workgroup partial gradients and losses.  Workgroup g takes
// entries 64g..64g+63 (lane = entry, so every load is 64 consecutive
// floats); wave w of its 16 sums the partials p = w, w + 16, ..., and the 16
// wave sums are added in wave order.  The order is fixed, so the result is
// deterministic.  (One thread per entry looping over every partial, as
// before, left 20 waves on the chip and took 60 us at 1024 partials.)
constexpr int kReduceWaves = 16;
__global__ void __launch_bounds__(64 * kReduceWaves)
k_mlp_reduce(const float *__restrict__ partial, int nparts, float *__restrict__ grad,
             float *__restrict__ loss_out, float loss_scale) {
    __shared__ float wsum[kReduceWaves][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    float s = 0.0f;
    if (e <= kNParam) {
#pragma unroll 8
        for (int p = w; p < nparts; p += kReduceWaves) s += partial[int64_t(p) * (kNParam + 1) + e];
    }
    wsum[w][lane] = s;
    __syncthreads();
    if (w == 0 && e <= kNParam) {
        float t = 0.0f;
        for (int k = 0; k < kReduceWaves; ++k) t += wsum[k][lane];
        if (e < kNParam) grad[e] = t;
        else loss_out[0] = t * loss_scale;
    }
}

__global__ void k_adam(float *__restrict__ P, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ grad, float lr, float b1c, float b2c) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kNParam) return;
    const float gr = grad[e];
    const float mm = 0.9f * m[e] + 0.1f * gr;
    const float vv = 0.999f * v[e] + 0.001f * gr * gr;
    m[e] = mm;
    v[e] = vv;
    P[e] -= lr * (mm / b1c) / (sqrtf(vv / b2c) + 1e-8f);
}

// Forward on explicit features (16 samples per wave).
__global__ void __launch_bounds__(256)
k_mlp_forward(const float *__restrict__ P, const float *__restrict__ phi, int64_t count,
              float *__restrict__ y) {
    LaneNet N;
    load_net(N, P);
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = (int64_t(gridDim.x) * blockDim.x) >> 6;
    for (int64_t grp = wave; grp * 16 < count; grp += nwaves) {
        const int64_t s = grp * 16 + j;
        const int64_t e = s < count ? s : 0;
        float f[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) f[k] = bf16r(phi[4 * e + k]);
        Fwd F;
        forward(N, f, F);
        if (g == 0 && s < count) y[s] = F.y;
    }
}

// Warm-start inference straight into the schedule-ordered dual array: one
// workgroup per tile, every slot of the tile (padding gets 0).  The network
// predicts the dual times n - 2, the number of triplets through a pair: a
// pair's share of the total pull A'y is spread over n - 2 rows, so this is
// the scale on which one network serves instances of every size.
template <typename T>
__global__ void __launch_bounds__(256)
k_mlp_infer(GraphView G, const float *__restrict__ P, T *__restrict__ y) {
    LaneNet N;
    load_net(N, P);
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const Tile tl = G.tiles[blockIdx.x];
    const int64_t bb = int64_t(G.b) * G.b;
    const int64_t nslots = int64_t(tl.Q - tl.P + 1) * G.b * 3 * bb;
    for (int64_t grp = wave; grp * 16 < nslots; grp += nw) {
        const int64_t s = tl.ybase + grp * 16 + j;
        const bool in = grp * 16 + j < nslots;
        int64_t i, jj, k;
        int o;
        const bool ok = in && decode_slot(tl, s, G.b, G.n, i, jj, k, o);
        float phi[4] = {0.f, 0.f, 0.f, 0.f};
        if (ok) row_features(G, i, jj, k, o, phi);
        Fwd F;
        forward(N, phi, F);
        if (g == 0 && in) y[s] = ok ? T(F.y / float(G.n - 2)) : T(0);
    }
}

// Inference-only form of the network: all three layers on
// v_mfma_f32_16x16x32_bf16, biases entering as the accumulator input.
// A 64-slot group runs as four passes; in pass q the samples are those of
// lane group q, and lane l of that group holds sample l itself.  Each lane
// puts its own sample's 4 features in its lane group's K slots (B operand),
// computes them once and keeps its own sample's output.
//   layer 1: A = W1 in the K slots of lane group q only (zero elsewhere),
//            with K padded from 4 to 32, so pass q's product reads only
//            group q's features.  Lane l receives units U_g of sample
//            l % 16 of pass q: layer 2's B operand.
//   layer 2: as in forward().
//   layer 3: A = W3 (permuted like K) on the output rows of lane group q
//            only, the four passes chained through the accumulator from b3:
//            row group g collects pass g's output, so lane l ends with the
//            output of its own sample, with no selects.  (The other passes
//            add exact zeros to a row group: the same sums as one product.)
struct InferNet {
    bf16x8 a1[4][2];  // a1[q][t][c] = W1[16t + i][c] if g == q and c < 4, else 0
    bf16x8 a2[2];     // as LaneNet::a2
    bf16x8 a3[4];     // a3[q][c] = W3[U_g[c]] if i / 4 == q, else 0
    f32x4 c1[2];      // c1[t][r] = b1[16t + 4g + r]
    f32x4 c2[2];      // c2[t][r] = b2[16t + 4g + r]
    float b3;
};

__device__ __forceinline__ void load_infer_net(InferNet &N, const float *__restrict__ P) {
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float w1 = c < 4 ? P[oW1 + (16 * t + i) * 4 + c] : 0.0f;
#pragma unroll
            for (int q = 0; q < 4; ++q) N.a1[q][t][c] = tobf(g == q ? w1 : 0.0f);
            N.a2[t][c] = tobf(P[oW2 + (16 * t + i) * 32 + unit_of(g, c)]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            N.c1[t][r] = P[oB1 + 16 * t + 4 * g + r];
            N.c2[t][r] = P[oB2 + 16 * t + 4 * g + r];
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float w3 = P[oW3 + unit_of(g, c)];
#pragma unroll
        for (int q = 0; q < 4; ++q) N.a3[q][c] = tobf(i / 4 == q ? w3 : 0.0f);
    }
    N.b3 = P[oB3];
}

// ReLU of a rounded bf16 pair: as 16-bit integers, negative values (and -0)
// are exactly those below 0, so one packed integer max clears them.
// Rounding commutes with ReLU (a negative value rounds to a value <= 0).
__device__ __forceinline__ bf16x2 relu2(const bf16x2 h) {
    typedef __attribute__((ext_vector_type(2))) short s16x2;
    const s16x2 zero = {0, 0};
    return __builtin_bit_cast(bf16x2, __builtin_elementwise_max(__builtin_bit_cast(s16x2, h), zero));
}

// ReLU of two 4-row accumulators, rounded to bf16, in the K order U_g.
__device__ __forceinline__ bf16x8 relu_bf16(const f32x4 lo, const f32x4 hi) {
    bf16x8 h;
#pragma unroll
    for (int r = 0; r < 4; r += 2) {
        const bf16x2 u = relu2(tobf2(lo[r], lo[r + 1]));
        const bf16x2 v = relu2(tobf2(hi[r], hi[r + 1]));
        h[r] = u[0];
        h[r + 1] = u[1];
        h[4 + r] = v[0];
        h[5 + r] = v[1];
    }
    return h;
}

// The four passes of a 64-row group, layer by layer: every lane carries its
// own sample's features in feat, and lane l receives its own sample's
// output.  The passes are independent until layer 3, so running them layer
// by layer puts one pass's VALU work in another's MFMA latency.
__device__ __forceinline__ float infer_group(const InferNet &N, const bf16x8 feat) {
    f32x4 z[4][2];
    bf16x8 h[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        z[q][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a1[q][0], feat, N.c1[0], 0, 0, 0);
        z[q][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a1[q][1], feat, N.c1[1], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q] = relu_bf16(z[q][0], z[q][1]);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        z[q][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a2[0], h[q], N.c2[0], 0, 0, 0);
        z[q][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a2[1], h[q], N.c2[1], 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) h[q] = relu_bf16(z[q][0], z[q][1]);
    f32x4 z3 = {N.b3, N.b3, N.b3, N.b3};
#pragma unroll
    for (int q = 0; q < 4; ++q) z3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a3[q], h[q], z3, 0, 0, 0);
    return z3[0] > 0.0f ? z3[0] : 0.0f;
}

// The same network in fewer registers, for the fused kernel at b = 24 and
// 32 (576 and 1024 lanes a workgroup leave 168 and 128 registers a lane):
// one copy of W1 and W3 in every lane group, the features of pass q kept
// only in lane group q's K slots and the output taken from pass q in lane
// group q, two passes at a time.  The products and sums are those of
// infer_group (the same nonzero products in the same K slots; the other
// passes' rows add exact zeros there), so the outputs are the same bits.
struct InferNetSmall {
    bf16x8 a1[2];  // a1[t][c] = W1[16t + i][c] for c < 4, else 0
    bf16x8 a2[2];
    bf16x8 a3;     // a3[c] = W3[U_g[c]] on every row
    f32x4 c1[2];
    f32x4 c2[2];
    float b3;
};

__device__ __forceinline__ void load_infer_net(InferNetSmall &N, const float *__restrict__ P) {
    const int lane = threadIdx.x & 63, i = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            N.a1[t][c] = tobf(c < 4 ? P[oW1 + (16 * t + i) * 4 + c] : 0.0f);
            N.a2[t][c] = tobf(P[oW2 + (16 * t + i) * 32 + unit_of(g, c)]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            N.c1[t][r] = P[oB1 + 16 * t + 4 * g + r];
            N.c2[t][r] = P[oB2 + 16 * t + 4 * g + r];
        }
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) N.a3[c] = tobf(P[oW3 + unit_of(g, c)]);
    N.b3 = P[oB3];
}

__device__ __forceinline__ float infer_group(const InferNetSmall &N, const bf16x8 feat) {
    const int g = (threadIdx.x & 63) >> 4;
    const bf16x8 zero8 = {};
    const f32x4 c3 = {N.b3, N.b3, N.b3, N.b3};
    float out = 0.0f;
#pragma unroll
    for (int q0 = 0; q0 < 4; q0 += 2) {
        f32x4 z[2][2];
        bf16x8 h[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const bf16x8 x = g == q0 + q ? feat : zero8;
            z[q][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a1[0], x, N.c1[0], 0, 0, 0);
            z[q][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a1[1], x, N.c1[1], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) h[q] = relu_bf16(z[q][0], z[q][1]);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            z[q][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a2[0], h[q], N.c2[0], 0, 0, 0);
            z[q][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a2[1], h[q], N.c2[1], 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) h[q] = relu_bf16(z[q][0], z[q][1]);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const f32x4 z3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(N.a3, h[q], c3, 0, 0, 0);
            if (g == q0 + q) out = z3[0];
        }
    }
    return out > 0.0f ? out : 0.0f;
}

// The inference for b = 8, 16, 32, walking the tile's segment in its own
// order instead of decoding every slot.  A workgroup takes one chunk of a
// tile's steps.  Per tile step the signed weights of blocks (P,J), (J,Q),
// (P,Q) and the degrees of the three vertex blocks sit in LDS, and a wave
// takes 64 consecutive slots (one sub-step t, one orientation o, lanes
// L0..L0+63), lane l computing the features and the output of slot L0 + l,
// so the store is contiguous.  Features are those of k_mlp_infer bit for
// bit; outputs differ only in fp32 summation order.
// Signed weight of pair (r, c) rounded to bf16, 0 where (r, c) is no pair.
__device__ __forceinline__ float signed_weight(const GraphView &G, int r, int c) {
    if (!(r < c && c < int(G.n))) return 0.0f;
    const int64_t p = pidx(r, c);
    return bf16r(float(G.d[p] == 0 ? G.w[p] : -G.w[p]));
}
__device__ __forceinline__ float vertex_degree(const GraphView &G, int v) { return v < int(G.n) ? G.deg[v] : 0.0f; }
// degree feature of a pair whose endpoints have degrees da, db
__device__ __forceinline__ float degree_feature(float da, float db, float md) {
    return bf16r(md > 0.0f ? (da + db) / (2.0f * md) : 0.0f);
}

// Features of slot (sub-step t, orientation o, lane L) of a tile step with
// blocks P, J, Q, from the step's tables (signed weights and degree
// features of blocks A = (P,J), B = (J,Q), C = (P,Q), [row * b + col]);
// ok = the slot is a triplet (else the features are zero).
template <int B>
__device__ __forceinline__ bf16x8 step_features(const float *swA, const float *swB, const float *swC,
                                                const float *fA, const float *fB, const float *fC, int t,
                                                int o, int L, int P, int J, int Q, int nn, bool &ok) {
    constexpr int b = B;
    const int il = L / b, kl = L % b;
    const int jl = mid_offset(t, il, kl, b);
    const int i = P * b + il, j = J * b + jl, k = Q * b + kl;
    ok = i < j && j < k && k < nn;
    const int eA = il * b + jl, eC = il * b + kl, eB = jl * b + kl;
    const float wij = swA[eA], wik = swC[eC], wjk = swB[eB];
    // long side ij, ik or jk
    const float p0 = o == 0 ? wij : (o == 1 ? wik : wjk);
    const float p1 = o == 0 ? wik : wij;
    const float p2 = o == 0 ? wjk : (o == 1 ? wjk : wik);
    const float p3 = o == 0 ? fA[eA] : (o == 1 ? fC[eC] : fB[eB]);
    const bf16x2 f01 = tobf2(ok ? p0 : 0.0f, ok ? p1 : 0.0f);
    const bf16x2 f23 = tobf2(ok ? p2 : 0.0f, ok ? p3 : 0.0f);
    bf16x8 feat = {};
    feat[0] = f01[0];
    feat[1] = f01[1];
    feat[2] = f23[0];
    feat[3] = f23[1];
    return feat;
}

// The inference for b = 8, 16, 32, walking the tile's segment in its own
// order instead of decoding every slot.  A workgroup takes one chunk of a
// tile's steps.  Per tile step the signed weights of blocks (P,J), (J,Q),
// (P,Q) and the degrees of the three vertex blocks sit in LDS, and a wave
// takes 64 consecutive slots (one sub-step t, one orientation o, lanes
// L0..L0+63), lane l computing the features and the output of slot L0 + l,
// so the store is contiguous.  Features are those of k_mlp_infer bit for
// bit; outputs differ only in fp32 summation order.
template <typename T, int B>
__global__ void __launch_bounds__(256)
k_mlp_infer_tiled(GraphView G, const float *__restrict__ P, T *__restrict__ y) {
    constexpr int b = B, bb = B * B;
    InferNet N;
    load_infer_net(N, P);
    const int lane = threadIdx.x & 63;
    // wave-uniform, so that a group's sub-step, orientation and first slot
    // sit in scalar registers and its feature selects are scalar
    const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6)), nw = blockDim.x >> 6;
    const int m0 = G.chunks[2 * int64_t(blockIdx.x) + 1];
    const Tile tl = G.tiles[G.chunks[2 * int64_t(blockIdx.x)]];
    const int Pb = tl.P, Qb = tl.Q;
    const int nn = int(G.n), nb = (nn + b - 1) / b;
    const bool desc = tile_desc(Pb, Qb, nb);
    const int m1 = min(m0 + kChunkSteps, Qb - Pb + 1);  // this chunk's steps: [m0, m1)
    __shared__ float swA[bb], swB[bb], swC[bb], fA[bb], fB[bb], fC[bb], dP[b], dJ[b], dQ[b];
    const float md = G.mean_deg[0];
    const float inv_scale = 1.0f / float(G.n - 2);
    for (int e = threadIdx.x; e < b; e += blockDim.x) {
        dP[e] = vertex_degree(G, Pb * b + e);
        dQ[e] = vertex_degree(G, Qb * b + e);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < bb; e += blockDim.x) {
        swC[e] = signed_weight(G, Pb * b + e / b, Qb * b + e % b);
        fC[e] = degree_feature(dP[e / b], dQ[e % b], md);
    }
    T *const ytile = y + tl.ybase;
    constexpr int gps = 3 * bb / 64;  // 64-slot groups per sub-step
    for (int m = m0; m < m1; ++m) {
        const int J = tile_J(Pb, Qb, m, desc);
        __syncthreads();  // the last step's readers are done
        for (int e = threadIdx.x; e < b; e += blockDim.x) dJ[e] = vertex_degree(G, J * b + e);
        __syncthreads();
        for (int e = threadIdx.x; e < bb; e += blockDim.x) {
            swA[e] = signed_weight(G, Pb * b + e / b, J * b + e % b);
            swB[e] = signed_weight(G, J * b + e / b, Qb * b + e % b);
            fA[e] = degree_feature(dP[e / b], dJ[e % b], md);
            fB[e] = degree_feature(dJ[e / b], dQ[e % b], md);
        }
        __syncthreads();
        for (int grp = wave; grp < b * gps; grp += nw) {
            const int t = grp / gps, rem = grp - t * gps;
            const int o = rem / (bb / 64), L0 = (rem - o * (bb / 64)) * 64;
            bool ok;
            const bf16x8 feat = step_features<B>(swA, swB, swC, fA, fB, fC, t, o, L0 + lane, Pb, J, Qb, nn, ok);
            const float out = infer_group(N, feat);
            ytile[(int64_t(m) * b + t) * 3 * bb + o * bb + L0 + lane] = T(ok ? out * inv_scale : 0.0f);
        }
    }
}

// Warm-start inference fused with A'y on the dataflow executor (b = 8, 16,
// 24, 32): one workgroup of b^2 lanes per tile, as in the sweep.  Per tile
// step and sub-step t, lane (il, kl) computes the network's predictions of
// its triplet's three rows (one 64-row group per orientation per wave: the
// wave's lanes are 64 consecutive slots, as in k_mlp_infer_tiled), writes
// them to y, and adds them into the FP64 accumulators of the triplet's
// pairs in LDS, in the order of k_aty_dataflow: the predictions equal
// k_mlp_infer_tiled's bit for bit (same features, same network code) and
// the sums equal A'y of those duals bit for bit, without reading y back.
// ax must hold zeros on entry.
template <typename T, int B>
__global__ void __launch_bounds__(B * B)
k_infer_aty_dataflow(DataflowArgs a, GraphView G, const float *__restrict__ P, T *__restrict__ y,
                     double *__restrict__ ax) {
    constexpr int b = B, bb = B * B;
    typename std::conditional<(B >= 24), InferNetSmall, InferNet>::type N;
    load_infer_net(N, P);
    const int tid = threadIdx.x;
    const int il = tid / b, kl = tid % b;
    const int sr = tid % b, sc = tid / b;
    const int nn = int(G.n), nb = (nn + b - 1) / b;
    __shared__ double Abuf[bb], Bbuf[bb], Cs[bb];
    __shared__ float swA[bb], swB[bb], swC[bb], fA[bb], fB[bb], fC[bb], dP[b], dJ[b], dQ[b];
    __shared__ int s_tix, s_ok;
    const float md = G.mean_deg[0];
    const float inv_scale = 1.0f / float(G.n - 2);

    if (tid == 0) s_tix = int(atomicAdd(&a.ctl[0], 1u));
    __syncthreads();
    for (;;) {
        const int tix = __builtin_amdgcn_readfirstlane(s_tix);
        if (tix >= a.ntiles) break;
        const DTile tl = a.tiles[tix];
        const int Pb = tl.P, Qb = tl.Q;
        const bool desc = tile_desc(Pb, Qb, nb);
        const int i = Pb * b + il, k = Qb * b + kl;
        const int idC = block_id(Pb, Qb);

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
        auto publish = [&](int R, int S, const double *X) {
            if (blk_ok(R, S))
                __hip_atomic_store(&ax[pidx(R * b + sr, S * b + sc)], X[sr * b + sc], __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        };
        auto step_ids = [&](int m, int &idA, int &idB) {
            const int J = tile_J(Pb, Qb, m, desc);
            idA = (J != Qb) ? block_id(Pb, J) : -1;
            idB = (J != Pb) ? block_id(J, Qb) : -1;
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

        if (tid < b) {
            dP[tid] = vertex_degree(G, Pb * b + tid);
            dQ[tid] = vertex_degree(G, Qb * b + tid);
        }
        if (tid == 0) {
            const bool ok = wait_step(0, true);
            if (ok) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_ok = ok;
        }
        __syncthreads();
        if (!__builtin_amdgcn_readfirstlane(s_ok)) break;
        blk_store(Pb, Qb, blk_load(Pb, Qb), Cs);
        swC[tid] = signed_weight(G, Pb * b + tid / b, Qb * b + tid % b);
        fC[tid] = degree_feature(dP[tid / b], dQ[tid % b], md);

        bool aborted = false;
        for (int m = 0; m <= Qb - Pb; ++m) {
            const int J = tile_J(Pb, Qb, m, desc);
            int idA, idB;
            step_ids(m, idA, idB);
            double *const Ab = (J == Qb) ? Cs : Abuf;
            double *const Bb = (J == Pb) ? Cs : Bbuf;
            // unconditional, as in the sweep (Abuf / Bbuf are idle where A
            // or B is the resident block)
            const double va = blk_load(Pb, J), vb = blk_load(J, Qb);
            if (tid < b) dJ[tid] = vertex_degree(G, J * b + tid);
            blk_store(Pb, J, va, Abuf);
            blk_store(J, Qb, vb, Bbuf);
            __syncthreads();  // dJ
            swA[tid] = signed_weight(G, Pb * b + tid / b, J * b + tid % b);
            swB[tid] = signed_weight(G, J * b + tid / b, Qb * b + tid % b);
            fA[tid] = degree_feature(dP[tid / b], dJ[tid % b], md);
            fB[tid] = degree_feature(dJ[tid / b], dQ[tid % b], md);
            __syncthreads();
            T *const ystep = y + tl.ybase + int64_t(m) * b * 3 * bb;
#pragma unroll 1
            for (int t = 0; t < b; ++t) {
                // one copy of the network code per sub-step (the orientation
                // loop is not unrolled: three copies would not fit the
                // registers at b = 32)
                double y0 = 0.0, y1 = 0.0, y2 = 0.0;
#pragma unroll 1
                for (int o = 0; o < 3; ++o) {
                    bool ok;
                    const bf16x8 feat = step_features<B>(swA, swB, swC, fA, fB, fC, t, o, tid, Pb, J, Qb, nn, ok);
                    const float out = infer_group(N, feat);
                    const T v = T(ok ? out * inv_scale : 0.0f);
                    __builtin_nontemporal_store(v, &ystep[(t * 3 + o) * bb + tid]);
                    if (o == 0) y0 = double(v);
                    else if (o == 1) y1 = double(v);
                    else y2 = double(v);
                }
                const int jl = mid_offset(t, il, kl, b);
                const int j = J * b + jl;
                if (i < j && j < k && k < nn) {
                    Ab[il * b + jl] += (y0 - y1) - y2;  // pair (i,j)
                    Cs[tid] += (y1 - y0) - y2;          // pair (i,k)
                    Bb[jl * b + kl] += (y2 - y0) - y1;  // pair (j,k)
                }
                lds_barrier();
            }

            const bool last = (m == Qb - Pb);
            if (idA >= 0) publish(Pb, J, Abuf);
            if (idB >= 0) publish(J, Qb, Bbuf);
            if (last) publish(Pb, Qb, Cs);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            if (tid == 0) {
                if (idA >= 0) __hip_atomic_fetch_add(&a.cnt[int64_t(idA) * kCntStride], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (idB >= 0) __hip_atomic_fetch_add(&a.cnt[int64_t(idB) * kCntStride], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                bool ok = true;
                if (last) {
                    __hip_atomic_fetch_add(&a.cnt[int64_t(idC) * kCntStride], uint32_t(Qb - Pb + 1), __ATOMIC_RELAXED,
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

// Features of given slots (for checks against the reference).
__global__ void k_mlp_slot_features(GraphView G, const int64_t *__restrict__ slots, int64_t count,
                                    float *__restrict__ phi) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t s = slots[e];
        int64_t lo = 0, hi = G.ntiles - 1;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (G.tiles[mid].ybase <= s) lo = mid; else hi = mid - 1;
        }
        int64_t i, j, k;
        int o;
        float f[4] = {0.f, 0.f, 0.f, 0.f};
        if (decode_slot(G.tiles[lo], s, G.b, G.n, i, j, k, o)) row_features(G, i, j, k, o, f);
        for (int q = 0; q < 4; ++q) phi[4 * e + q] = f[q];
    }
}

// The sampled warm-start gate.  Workgroup s takes the pair pairs[s] = (a, c),
// a < c, given by its packed index.  It sums, over every third vertex v, the
// predictions of the three rows of the triplet {a, c, v}: +1 for the row
// whose long side is (a, c), -1 for the other two.  That sum is the pair's
// metric part of A'y at the predicted duals.  Each prediction is the value
// the full inference writes for that row: the features of row_features, the
// same network code, the same scaling and rounding to T.  Only the FP64
// summation order differs from the full A'y.  An index outside [0, N_p)
// gives NaN.
template <typename T>
__global__ void __launch_bounds__(256)
k_gate_sample_aty(GraphView G, const float *__restrict__ P, const int64_t *__restrict__ pairs,
                  double *__restrict__ aty) {
    InferNet N;
    load_infer_net(N, P);
    __shared__ double red[256];
    const int64_t p = pairs[blockIdx.x];
    if (p < 0 || p >= G.n * (G.n - 1) / 2) {  // no pair: NaN (the whole workgroup leaves)
        if (threadIdx.x == 0) aty[blockIdx.x] = __builtin_nan("");
        return;
    }
    int64_t c = int64_t(0.5 * (1.0 + sqrt(1.0 + 8.0 * double(p))));
    while (c * (c - 1) / 2 > p) --c;
    while ((c + 1) * c / 2 <= p) ++c;
    const int64_t a = p - c * (c - 1) / 2;
    const int64_t n = G.n;
    const float inv_scale = 1.0f / float(n - 2);
    double acc = 0.0;
    // the same trip count in every lane: the network's MFMAs need the whole wave
    for (int64_t v0 = 0; v0 < n; v0 += blockDim.x) {
        const int64_t v = v0 + threadIdx.x;
        const bool ok = v < n && v != a && v != c;
        // the triplet in order, and the side (a, c) takes in it: ij, ik or jk
        const int64_t i = v < a ? v : a;
        const int64_t j = v < a ? a : (v < c ? v : c);
        const int64_t k = v < c ? c : v;
        const int side = v < a ? 2 : (v < c ? 1 : 0);
        double s = 0.0;
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            float phi[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (ok) row_features(G, i, j, k, o, phi);
            bf16x8 feat = {};
#pragma unroll
            for (int e = 0; e < 4; ++e) feat[e] = tobf(phi[e]);
            const float out = infer_group(N, feat);
            const double yv = double(T(ok ? out * inv_scale : 0.0f));
            s += o == side ? yv : -yv;
        }
        acc += s;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) aty[blockIdx.x] = red[0];
}

__global__ void k_mean_deg(const float *__restrict__ deg, int64_t n, float *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t v = threadIdx.x; v < n; v += blockDim.x) s += deg[v];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = float(red[0] / double(n));
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
int mlp_num_params() { return kNParam; }
// One-wave workgroups, 32 samples a chunk, at most 1024 of them: 4096
// (4 waves a SIMD) was slower at batches of 64K and 1M samples, the partials
// to reduce growing with them.
int mlp_grad_blocks(int64_t count) {
    int64_t c = (count + 31) / 32;
    return int(c < 1 ? 1 : (c > 1024 ? 1024 : c));
}
size_t mlp_workspace_bytes(int64_t count) {
    return size_t(mlp_grad_blocks(count)) * (kNParam + 1) * sizeof(float) +
           size_t(kNParam + 1) * sizeof(float) + 64;
}

static int finish_step(float *partial, int nparts, float *P, float *m, float *v, int step, float lr,
                       float *grad_out, float *ws_grad, float *loss_dev, float loss_scale,
                       hipStream_t s) {
    float *grad = grad_out ? grad_out : ws_grad;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kNParam + 1 + 63) / 64), dim3(64 * kReduceWaves), 0, s, partial,
                       nparts, grad, loss_dev, loss_scale);
    CCP_LAUNCH_CHECK("k_mlp_reduce");
    if (lr > 0.0f && m && v) {
        const float b1c = 1.0f - powf(0.9f, float(step));
        const float b2c = 1.0f - powf(0.999f, float(step));
        hipLaunchKernelGGL(k_adam, dim3((kNParam + 255) / 256), dim3(256), 0, s, P, m, v, grad,
                           lr, b1c, b2c);
        CCP_LAUNCH_CHECK("k_adam");
    }
    return CC_OK;
}

int launch_mlp_train_explicit(const float *phi, const float *target, int64_t count, float *P,
                              float *m, float *v, int step, float lr, float *grad_out,
                              void *workspace, float *loss_dev, hipStream_t s) {
    const int nb = mlp_grad_blocks(count);
    float *partial = static_cast<float *>(workspace);
    float *ws_grad = partial + size_t(nb) * (kNParam + 1);
    ExplicitSource src{phi, target, count};
    hipLaunchKernelGGL(k_mlp_grad<ExplicitSource>, dim3(nb), dim3(64), 0, s, src, count,
                       1.0f / float(count), (const float *)P, partial);
    CCP_LAUNCH_CHECK("k_mlp_grad");
    return finish_step(partial, nb, P, m, v, step, lr, grad_out, ws_grad, loss_dev,
                       1.0f / float(count), s);
}

template <typename T>
int launch_mlp_train_graph(const GraphView &G, const T *ystar, int64_t slots, uint64_t seed,
                           int64_t batch, float *P, float *m, float *v, int step, float lr,
                           void *workspace, float *loss_dev, hipStream_t s) {
    const int nb = mlp_grad_blocks(batch);
    float *partial = static_cast<float *>(workspace);
    float *ws_grad = partial + size_t(nb) * (kNParam + 1);
    GraphSource<T> src{G, ystar, slots, seed, batch};
    hipLaunchKernelGGL(k_mlp_grad<GraphSource<T>>, dim3(nb), dim3(64), 0, s, src, batch,
                       1.0f / float(batch), (const float *)P, partial);
    CCP_LAUNCH_CHECK("k_mlp_grad");
    return finish_step(partial, nb, P, m, v, step, lr, nullptr, ws_grad, loss_dev,
                       1.0f / float(batch), s);
}

int launch_mlp_forward(const float *P, const float *phi, int64_t count, float *y, hipStream_t s) {
    if (count <= 0) return CC_OK;
    int64_t waves = (count + 15) / 16;
    int64_t blocks = (waves + 3) / 4;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_mlp_forward, dim3(unsigned(blocks)), dim3(256), 0, s, P, phi, count, y);
    CCP_LAUNCH_CHECK("k_mlp_forward");
    return CC_OK;
}

template <typename T>
int launch_mlp_infer(const GraphView &G, const float *P, T *y, hipStream_t s) {
    switch (G.b) {
        case 8: hipLaunchKernelGGL((k_mlp_infer_tiled<T, 8>), dim3(unsigned(G.nchunks)), dim3(256), 0, s, G, P, y); break;
        case 16: hipLaunchKernelGGL((k_mlp_infer_tiled<T, 16>), dim3(unsigned(G.nchunks)), dim3(256), 0, s, G, P, y); break;
        case 32: hipLaunchKernelGGL((k_mlp_infer_tiled<T, 32>), dim3(unsigned(G.nchunks)), dim3(256), 0, s, G, P, y); break;
        default: hipLaunchKernelGGL(k_mlp_infer<T>, dim3(unsigned(G.ntiles)), dim3(256), 0, s, G, P, y); break;
    }
    CCP_LAUNCH_CHECK("k_mlp_infer");
    return CC_OK;
}

int launch_mlp_slot_features(const GraphView &G, const int64_t *slots, int64_t count, float *phi,
                             hipStream_t s) {
    if (count <= 0) return CC_OK;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_mlp_slot_features, dim3(unsigned(blocks)), dim3(256), 0, s, G, slots, count,
                       phi);
    CCP_LAUNCH_CHECK("k_mlp_slot_features");
    return CC_OK;
}

template <typename T>
int launch_gate_sample_aty(const GraphView &G, const float *P, const int64_t *pairs, int64_t count,
                           double *aty, hipStream_t s) {
    if (count <= 0) return CC_OK;
    if (count > int64_t(INT32_MAX)) return fail(CC_EINVAL, "too many sampled pairs");
    hipLaunchKernelGGL(k_gate_sample_aty<T>, dim3(unsigned(count)), dim3(256), 0, s, G, P, pairs, aty);
    CCP_LAUNCH_CHECK("k_gate_sample_aty");
    return CC_OK;
}
template int launch_gate_sample_aty<double>(const GraphView &, const float *, const int64_t *, int64_t,
                                            double *, hipStream_t);
template int launch_gate_sample_aty<float>(const GraphView &, const float *, const int64_t *, int64_t,
                                           double *, hipStream_t);

int launch_mean_deg(const float *deg, int64_t n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_mean_deg, dim3(1), dim3(256), 0, s, deg, n, out);
    CCP_LAUNCH_CHECK("k_mean_deg");
    return CC_OK;
}

template int launch_mlp_train_graph<double>(const GraphView &, const double *, int64_t, uint64_t,
                                            int64_t, float *, float *, float *, int, float, void *,
                                            float *, hipStream_t);
template int launch_mlp_train_graph<float>(const GraphView &, const float *, int64_t, uint64_t,
                                           int64_t, float *, float *, float *, int, float, void *,
                                           float *, hipStream_t);
template <typename T>
int launch_infer_aty_dataflow(const DataflowArgs &a, int grid, const GraphView &G, const float *P, T *y,
                              double *ax, hipStream_t s) {
    switch (G.b) {
        case 8: hipLaunchKernelGGL((k_infer_aty_dataflow<T, 8>), dim3(grid), dim3(64), 0, s, a, G, P, y, ax); break;
        case 16: hipLaunchKernelGGL((k_infer_aty_dataflow<T, 16>), dim3(grid), dim3(256), 0, s, a, G, P, y, ax); break;
        case 24: hipLaunchKernelGGL((k_infer_aty_dataflow<T, 24>), dim3(grid), dim3(576), 0, s, a, G, P, y, ax); break;
        case 32: hipLaunchKernelGGL((k_infer_aty_dataflow<T, 32>), dim3(grid), dim3(1024), 0, s, a, G, P, y, ax); break;
        default: return fail(CC_EINVAL, "the fused inference runs for b = 8, 16, 24, 32");
    }
    CCP_LAUNCH_CHECK("k_infer_aty_dataflow");
    return CC_OK;
}

template <typename T>
int infer_aty_occupancy(int b, int *blocks_per_cu) {
    hipError_t e = hipSuccess;
    switch (b) {
        case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_infer_aty_dataflow<T, 8>, 64, 0); break;
        case 16: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_infer_aty_dataflow<T, 16>, 256, 0); break;
        case 24: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_infer_aty_dataflow<T, 24>, 576, 0); break;
        case 32: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_infer_aty_dataflow<T, 32>, 1024, 0); break;
        default: *blocks_per_cu = 0; return CC_OK;
    }
    if (e != hipSuccess) return fail(CC_EHIP, std::string("fused inference occupancy: ") + hipGetErrorString(e));
    return CC_OK;
}

template int launch_infer_aty_dataflow<double>(const DataflowArgs &, int, const GraphView &, const float *, double *,
                                               double *, hipStream_t);
template int launch_infer_aty_dataflow<float>(const DataflowArgs &, int, const GraphView &, const float *, float *,
                                              double *, hipStream_t);
template int infer_aty_occupancy<double>(int, int *);
template int infer_aty_occupancy<float>(int, int *);
template int launch_mlp_infer<double>(const GraphView &, const float *, double *, hipStream_t);
template int launch_mlp_infer<float>(const GraphView &, const float *, float *, hipStream_t);

}  // namespace ccp
