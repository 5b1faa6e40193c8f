// resid.hip -- FP64 convergence measures, A'y, and dual layout conversion.
//
// Convergence (Sec. IV-D stops once the rows hold to a tolerance and the
// primal and dual objectives have met):
//   max violation over every metric row and every pair row;
//   primal QP value c'v + (eps/2) v'Wv and the LP cost sum w |x - d|;
//   complementary slackness y (b - a'v) over every row;
//   the dual objective D(y) = -b'y - (1/(2 eps)) (c + A'y)' W^{-1} (c + A'y)
//   of (qp), and the distance of v from v(y) = -(1/eps) W^{-1} (c + A'y),
//   the point Algorithm 1 keeps v at (its initial v and every update keep
//   c + eps W v + A'y = 0).
// All sums and maxima are taken in FP64 and are deterministic: per-workgroup
// partials in a fixed order, then one fixed-order final reduction.
//
// A'y is accumulated with the same round structure as the sweep (tiles of a
// round own disjoint pairs), so it needs no atomics and has a fixed order.
#include "common.hpp"

namespace ccp {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}

// Block reduction of NV values; op[v] = 0 for sum, 1 for max.  Result in
// thread 0.  Requires blockDim.x a multiple of 64 (or <= 64) and
// scratch[NV * 16].
template <int NV>
__device__ void block_reduce(double (&v)[NV], const int (&op)[NV], double *scratch) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int e = 0; e < NV; ++e) v[e] = op[e] ? wave_max(v[e]) : wave_sum(v[e]);
    __syncthreads();
    if (lane == 0)
        for (int e = 0; e < NV; ++e) scratch[e * 16 + wave] = v[e];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int e = 0; e < NV; ++e) {
            double a = scratch[e * 16];
            for (int w = 1; w < nw; ++w)
                a = op[e] ? fmax(a, scratch[e * 16 + w]) : a + scratch[e * 16 + w];
            v[e] = a;
        }
    }
}

__device__ __forceinline__ bool finite(double v) { return v - v == 0.0; }

// ---------------------------------------------------------------------------
// Metric rows: violation and complementary slackness, one workgroup per
// chunk of at most kChunkSteps tile steps (all chunks in one launch;
// read-only, so no ordering between them).
// partial[chunk*4 + 0..3] = {max violation, sum y*slack, max |y*slack|,
// non-finite flag}.
// ---------------------------------------------------------------------------
template <typename T, int B>
__global__ void __launch_bounds__(B ? B * B : 1024)
k_metric_resid(const Tile *__restrict__ tiles, const int32_t *__restrict__ chunks, int b_rt, int64_t n,
               const T *__restrict__ x, const T *__restrict__ y, double *__restrict__ partial) {
    const int b = B ? B : b_rt;
    const int bb = b * b;
    const int tid = threadIdx.x;
    const int il = tid / b, kl = tid - (tid / b) * b;
    const Tile tl = tiles[chunks[2 * int64_t(blockIdx.x)]];
    const int m0 = chunks[2 * int64_t(blockIdx.x) + 1];
    const int P = tl.P, Q = tl.Q;
    const int m1 = min(m0 + kChunkSteps, Q - P + 1);  // this chunk's tile steps: [m0, m1)
    __shared__ double As[1024], Bs[1024], Cs[1024];
    __shared__ double red[4 * 16];
    const int64_t i = int64_t(P) * b + il, k = int64_t(Q) * b + kl;
    {
        const bool ok = i < k && k < n;
        Cs[tid] = ok ? double(x[pidx(i, k)]) : 0.0;
    }
    double vmax = 0.0, cs_sum = 0.0, cs_max = 0.0, bad = 0.0;
    const bool desc = tile_desc(P, Q, int((n + b - 1) / b));
    for (int m = m0; m < m1; ++m) {
        const int J = tile_J(P, Q, m, desc);
        if (J != Q) {
            const int64_t ii = int64_t(P) * b + il, jj = int64_t(J) * b + kl;
            As[tid] = (ii < jj && jj < n) ? double(x[pidx(ii, jj)]) : 0.0;
        }
        if (J != P) {
            const int64_t jj = int64_t(J) * b + il, kk = int64_t(Q) * b + kl;
            Bs[tid] = (jj < kk && kk < n) ? double(x[pidx(jj, kk)]) : 0.0;
        }
        __syncthreads();
        const double *Ab = (J == Q) ? Cs : As;
        const double *Bb = (J == P) ? Cs : Bs;
        for (int t = 0; t < b; ++t) {
            const int jl = mid_offset(t, il, kl, b);
            const int64_t j = int64_t(J) * b + jl;
            if (i < j && j < k && k < n) {
                const double xa = Ab[il * b + jl], xb = Bb[jl * b + kl], xc = Cs[tid];
                const double s0 = (xc + xb) - xa;  // slack of x_ij <= x_ik + x_jk
                const double s1 = (xa + xb) - xc;  // slack of x_ik <= x_ij + x_jk
                const double s2 = (xa + xc) - xb;  // slack of x_jk <= x_ij + x_ik
                vmax = fmax(vmax, fmax(-s0, fmax(-s1, -s2)));
                if (!finite(s0 + s1 + s2)) bad = 1.0;
                if (y) {
                    const int64_t u = int64_t(m) * b + t;
                    const T *src = y + tl.ybase + u * 3 * bb + tid;
                    const double c0 = double(src[0]) * s0, c1 = double(src[bb]) * s1,
                                 c2 = double(src[2 * bb]) * s2;
                    cs_sum += (c0 + c1) + c2;
                    cs_max = fmax(cs_max, fmax(fabs(c0), fmax(fabs(c1), fabs(c2))));
                }
            }
        }
        __syncthreads();
    }
    double v[4] = {vmax, cs_sum, cs_max, bad};
    const int op[4] = {1, 0, 1, 1};
    block_reduce<4>(v, op, red);
    if (tid == 0)
        for (int e = 0; e < 4; ++e) partial[int64_t(blockIdx.x) * 4 + e] = v[e];
}

// Metric rows, violations only (no duals read): the maximum of
// k_metric_resid, bit for bit, in fewer operations.  A read-only pass needs
// no conflict-free order, so each lane walks its middle offsets jl in order
// over the range where (i, j, k) is a triplet (i < j < k < n); a step whose
// middle block lies strictly inside the tile and whose blocks are whole
// (every lane valid for every jl) runs without any test.  The three
// negated slacks are those of k_metric_resid (a - b = -(b - a) exactly).
// The finiteness check is taken on the x values as they are staged: every
// pair lies in some triplet, and a slack of finite values overflows only
// for |x| above DBL_MAX / 2.  partial[chunk*4 + 0..3] = {max violation, 0,
// 0, non-finite flag}, the layout of k_metric_resid.
template <typename T, int B>
__global__ void __launch_bounds__(B ? B * B : 1024)
k_metric_viol(const Tile *__restrict__ tiles, const int32_t *__restrict__ chunks, int b_rt, int64_t n,
              const T *__restrict__ x, double *__restrict__ partial) {
    const int b = B ? B : b_rt;
    const int tid = threadIdx.x;
    const int il = tid / b, kl = tid - (tid / b) * b;
    const Tile tl = tiles[chunks[2 * int64_t(blockIdx.x)]];
    const int m0 = chunks[2 * int64_t(blockIdx.x) + 1];
    const int P = tl.P, Q = tl.Q;
    const int m1 = min(m0 + kChunkSteps, Q - P + 1);  // this chunk's tile steps: [m0, m1)
    __shared__ double As[1024], Bs[1024], Cs[1024];
    __shared__ double red[4 * 16];
    const int64_t i = int64_t(P) * b + il, k = int64_t(Q) * b + kl;
    const bool lane_ok = i < k && k < n;
    double bad = 0.0;
    const double xc = lane_ok ? double(x[pidx(i, k)]) : 0.0;
    if (!finite(xc)) bad = 1.0;
    Cs[tid] = xc;
    double vmax = 0.0;
    const int nb = int((n + b - 1) / b);
    const bool desc = tile_desc(P, Q, nb);
    const bool q_whole = int64_t(Q + 1) * b <= n;
    for (int m = m0; m < m1; ++m) {
        const int J = tile_J(P, Q, m, desc);
        if (J != Q) {
            const int64_t ii = int64_t(P) * b + il, jj = int64_t(J) * b + kl;
            const double v = (ii < jj && jj < n) ? double(x[pidx(ii, jj)]) : 0.0;
            if (!finite(v)) bad = 1.0;
            As[tid] = v;
        }
        if (J != P) {
            const int64_t jj = int64_t(J) * b + il, kk = int64_t(Q) * b + kl;
            const double v = (jj < kk && kk < n) ? double(x[pidx(jj, kk)]) : 0.0;
            if (!finite(v)) bad = 1.0;
            Bs[tid] = v;
        }
        __syncthreads();
        const double *Ab = (J == Q) ? Cs : As;
        const double *Bb = (J == P) ? Cs : Bs;
        if (P < J && J < Q && q_whole) {
            // every (i, j, k) of the step is a triplet
            const double *arow = Ab + il * b;
#pragma unroll
            for (int jl = 0; jl < (B ? B : 32); ++jl) {
                if (!B && jl >= b) break;
                const double xa = arow[jl], xb = Bb[jl * b + kl];
                vmax = fmax(vmax, fmax(xa - (xc + xb), fmax(xc - (xa + xb), xb - (xa + xc))));
            }
        } else if (lane_ok) {
            // i < j: jl > il in the tile's own first block; j < k: jl < kl
            // in its last; j < n
            const int lo = (J == P) ? il + 1 : 0;
            int hi = (J == Q) ? kl : b;
            const int64_t room = n - int64_t(J) * b;
            if (room < hi) hi = int(room);
            for (int jl = lo; jl < hi; ++jl) {
                const double xa = Ab[il * b + jl], xb = Bb[jl * b + kl];
                vmax = fmax(vmax, fmax(xa - (xc + xb), fmax(xc - (xa + xb), xb - (xa + xc))));
            }
        }
        __syncthreads();
    }
    double v[4] = {vmax, 0.0, 0.0, bad};
    const int op[4] = {1, 0, 1, 1};
    block_reduce<4>(v, op, red);
    if (tid == 0)
        for (int e = 0; e < 4; ++e) partial[int64_t(blockIdx.x) * 4 + e] = v[e];
}

// ---------------------------------------------------------------------------
// Pair rows and the objective sums.  partial[block*10 + e]:
//  0 max pair violation   1 sum w f          2 sum w (x^2 + f^2)
//  3 sum w |x - d|        4 max |y * slack|  5 sum y * slack
//  6 sum (c+A'y)^2 / w    7 b'y              8 max |v - v(y)|
//  9 non-finite flag
// ax (metric part of A'y on x) may be null: then 6-8 stay 0.
// ---------------------------------------------------------------------------
constexpr int kPairBlocks = 1024;

// d: uint8 0/1 for correlation clustering, double for l1 metric nearness
template <typename T, typename DT>
__global__ void __launch_bounds__(256)
k_pair_resid(int64_t np, const T *__restrict__ x, const T *__restrict__ f,
             const T *__restrict__ yp, const double *__restrict__ w,
             const DT *__restrict__ d, const double *__restrict__ ax, double gamma,
             double *__restrict__ partial) {
    __shared__ double red[10 * 16];
    double vp = 0, swf = 0, swq = 0, lp = 0, csm = 0, css = 0, qd = 0, by = 0, st = 0, bad = 0;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < np;
         p += int64_t(gridDim.x) * blockDim.x) {
        const double xv = double(x[p]), fv = double(f[p]), wv = w[p], dv = double(d[p]);
        const double s1 = dv - (xv - fv);     // slack of  x - f <= d
        const double s2 = -dv - (-xv - fv);   // slack of -x - f <= -d
        vp = fmax(vp, fmax(-s1, -s2));
        swf += wv * fv;
        swq += wv * (xv * xv + fv * fv);
        lp += wv * fabs(xv - dv);
        if (!finite(xv) || !finite(fv)) bad = 1.0;
        if (yp) {
            const double y1 = double(yp[2 * p]), y2 = double(yp[2 * p + 1]);
            const double c1 = y1 * s1, c2 = y2 * s2;
            csm = fmax(csm, fmax(fabs(c1), fabs(c2)));
            css += c1 + c2;
            if (ax) {
                const double gx = ax[p] + (y1 - y2);     // c_x = 0
                const double gf = wv + (-y1 - y2);       // c_f = w
                qd += (gx * gx + gf * gf) / wv;
                by += dv * y1 - dv * y2;
                st = fmax(st, fmax(fabs(xv + gamma * gx / wv), fabs(fv + gamma * gf / wv)));
            }
        }
    }
    double v[10] = {vp, swf, swq, lp, csm, css, qd, by, st, bad};
    const int op[10] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 1};
    block_reduce<10>(v, op, red);
    if (threadIdx.x == 0)
        for (int e = 0; e < 10; ++e) partial[int64_t(blockIdx.x) * 10 + e] = v[e];
}

// Pair terms of the l2 metric nearness problem, in the slots of k_pair_resid
// (so k_final_reduce serves both): 2 sum w (x - d)^2, 6 sum (A'y)^2 / w,
// 7 d'A'y, 8 max |x - (d - A'y / w)|, 9 non-finite flag; the others 0.
// ax (the metric A'y) may be null: then 6-8 stay 0.
template <typename T>
__global__ void __launch_bounds__(256)
k_nearness_pair_resid(int64_t np, const T *__restrict__ x, const double *__restrict__ dv,
                      const double *__restrict__ w, const double *__restrict__ ax,
                      double *__restrict__ partial) {
    __shared__ double red[10 * 16];
    double sq = 0, qd = 0, dy = 0, st = 0, bad = 0;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < np;
         p += int64_t(gridDim.x) * blockDim.x) {
        const double xv = double(x[p]), dp = dv[p], wv = w[p];
        const double e = xv - dp;
        sq += wv * (e * e);
        if (!finite(xv)) bad = 1.0;
        if (ax) {
            const double a = ax[p];
            qd += (a * a) / wv;
            dy += dp * a;
            st = fmax(st, fabs(xv - (dp - a / wv)));
        }
    }
    double v[10] = {0, 0, sq, 0, 0, 0, qd, dy, st, bad};
    const int op[10] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 1};
    block_reduce<10>(v, op, red);
    if (threadIdx.x == 0)
        for (int e = 0; e < 10; ++e) partial[int64_t(blockIdx.x) * 10 + e] = v[e];
}

// Weight of the positive and of the negative pairs, in k_pair_resid's
// partial slots 1 (sum of w over d = 0) and 2 (sum of w over d = 1), the
// others 0, so that k_final_reduce returns them as out[5] and out[6].
__global__ void __launch_bounds__(256)
k_weight_classes(int64_t np, const double *__restrict__ w, const uint8_t *__restrict__ d,
                 double *__restrict__ partial) {
    __shared__ double red[10 * 16];
    double w0 = 0.0, w1 = 0.0;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < np;
         p += int64_t(gridDim.x) * blockDim.x) {
        if (d[p]) w1 += w[p];
        else w0 += w[p];
    }
    double v[10] = {0, w0, w1, 0, 0, 0, 0, 0, 0, 0};
    const int op[10] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 1};
    block_reduce<10>(v, op, red);
    if (threadIdx.x == 0)
        for (int e = 0; e < 10; ++e) partial[int64_t(blockIdx.x) * 10 + e] = v[e];
}

// Fixed-order final reduction: out[0..3] from the metric partials, out[4..13]
// from the pair partials.  One workgroup of 1024 lanes: at n = 4000, b = 32
// there are 86,336 metric partials, which 256 lanes took 94 us to walk.
__global__ void __launch_bounds__(1024)
k_final_reduce(const double *__restrict__ mpart, int64_t nm, const double *__restrict__ ppart,
               int64_t npb, double *__restrict__ out) {
    __shared__ double red[14 * 16];
    double v[14];
    for (int e = 0; e < 14; ++e) v[e] = 0.0;
    const int opm[4] = {1, 0, 1, 1};
    const int opp[10] = {1, 0, 0, 0, 1, 0, 0, 0, 1, 1};
    for (int64_t r = threadIdx.x; r < nm; r += blockDim.x)
        for (int e = 0; e < 4; ++e)
            v[e] = opm[e] ? fmax(v[e], mpart[r * 4 + e]) : v[e] + mpart[r * 4 + e];
    for (int64_t r = threadIdx.x; r < npb; r += blockDim.x)
        for (int e = 0; e < 10; ++e)
            v[4 + e] = opp[e] ? fmax(v[4 + e], ppart[r * 10 + e]) : v[4 + e] + ppart[r * 10 + e];
    int op[14];
    for (int e = 0; e < 4; ++e) op[e] = opm[e];
    for (int e = 0; e < 10; ++e) op[4 + e] = opp[e];
    block_reduce<14>(v, op, red);
    if (threadIdx.x == 0)
        for (int e = 0; e < 14; ++e) out[e] = v[e];
}

// ---------------------------------------------------------------------------
// A'y on the x block, metric rows only, one round per launch.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void lds_barrier_r() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T, int B>
__global__ void __launch_bounds__(B ? B * B : 1024)
k_aty_round(const Tile *__restrict__ tiles, int b_rt, int64_t n, const T *__restrict__ y,
            double *__restrict__ ax) {
    const int b = B ? B : b_rt;
    const int bb = b * b;
    const int tid = threadIdx.x;
    const int il = tid / b, kl = tid - (tid / b) * b;
    const Tile tl = tiles[blockIdx.x];
    const int P = tl.P, Q = tl.Q;
    __shared__ double As[1024], Bs[1024], Cs[1024];
    const int64_t i = int64_t(P) * b + il, k = int64_t(Q) * b + kl;
    const bool c_ok = i < k && k < n;
    Cs[tid] = c_ok ? ax[pidx(i, k)] : 0.0;
    const bool desc = tile_desc(P, Q, int((n + b - 1) / b));
    for (int m = 0; m <= Q - P; ++m) {
        const int J = tile_J(P, Q, m, desc);
        int64_t pa = -1, pb = -1;
        if (J != Q) {
            const int64_t ii = int64_t(P) * b + il, jj = int64_t(J) * b + kl;
            if (ii < jj && jj < n) pa = pidx(ii, jj);
            As[tid] = pa >= 0 ? ax[pa] : 0.0;
        }
        if (J != P) {
            const int64_t jj = int64_t(J) * b + il, kk = int64_t(Q) * b + kl;
            if (jj < kk && kk < n) pb = pidx(jj, kk);
            Bs[tid] = pb >= 0 ? ax[pb] : 0.0;
        }
        lds_barrier_r();
        double *Ab = (J == Q) ? Cs : As;
        double *Bb = (J == P) ? Cs : Bs;
        for (int t = 0; t < b; ++t) {
            const int jl = mid_offset(t, il, kl, b);
            const int64_t j = int64_t(J) * b + jl;
            if (i < j && j < k && k < n) {
                const int64_t u = int64_t(m) * b + t;
                const T *src = y + tl.ybase + u * 3 * bb + tid;
                const double y0 = double(src[0]), y1 = double(src[bb]), y2 = double(src[2 * bb]);
                Ab[il * b + jl] += (y0 - y1) - y2;  // pair (i,j)
                Cs[tid] += (y1 - y0) - y2;          // pair (i,k)
                Bb[jl * b + kl] += (y2 - y0) - y1;  // pair (j,k)
            }
            lds_barrier_r();
        }
        if (pa >= 0) ax[pa] = As[tid];
        if (pb >= 0) ax[pb] = Bs[tid];
        lds_barrier_r();
    }
    if (c_ok) ax[pidx(i, k)] = Cs[tid];
}

// x = -gamma W^{-1} (c + A'y): adds the pair rows' part of A'y.
template <typename T>
__global__ void k_x_from_aty(int64_t np, const double *__restrict__ ax, const T *__restrict__ yp,
                             const double *__restrict__ w, double gamma, T *__restrict__ x,
                             T *__restrict__ f) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < np;
         p += int64_t(gridDim.x) * blockDim.x) {
        const double y1 = double(yp[2 * p]), y2 = double(yp[2 * p + 1]);
        const double gx = ax[p] + (y1 - y2);
        const double gf = w[p] + (-y1 - y2);
        x[p] = T(-gamma * gx / w[p]);
        f[p] = T(-gamma * gf / w[p]);
    }
}

// The sampled warm-start gate: weights, labels and g of the drawn pairs, in
// draw order, so that the pair kernels run on the sample as on all pairs.
// An index outside [0, np) gets NaN weights.
template <typename T>
__global__ void k_gate_gather(int64_t np, int64_t count, const int64_t *__restrict__ pairs,
                              const double *__restrict__ w, const uint8_t *__restrict__ d,
                              const T *__restrict__ g, double *__restrict__ ws,
                              uint8_t *__restrict__ ds, T *__restrict__ gs) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t p = pairs[e];
        const bool ok = p >= 0 && p < np;
        ws[e] = ok ? w[p] : __builtin_nan("");
        ds[e] = ok ? d[p] : 0;
        gs[e] = ok ? g[p] : T(__builtin_nan(""));
    }
}

// Each drawn pair's term of D_warm - D_cold.  With the pair rows at their
// values after one pair pass, the dual objective of k_pair_resid,
// D = -b'y - (gamma/2) sum (c + A'y)^2 / w, is a sum of one term per pair:
// -d (y1 - y2) - (gamma/2) ((A'y_metric + y1 - y2)^2 + (w - y1 - y2)^2) / w.
// ypw: the pair duals of the predicted start, whose metric part of A'y is
// aty; ypc: those of the cold start, whose metric part is 0.
template <typename T>
__global__ void k_gate_delta(int64_t count, const double *__restrict__ aty,
                             const T *__restrict__ ypw, const T *__restrict__ ypc,
                             const double *__restrict__ ws, const uint8_t *__restrict__ ds,
                             double gamma, double *__restrict__ delta) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += int64_t(gridDim.x) * blockDim.x) {
        const double wv = ws[e], dv = double(ds[e]);
        double term[2];
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const T *yp = s == 0 ? ypw : ypc;
            const double y1 = double(yp[2 * e]), y2 = double(yp[2 * e + 1]);
            const double gx = (s == 0 ? aty[e] : 0.0) + (y1 - y2);
            const double gf = wv + (-y1 - y2);
            term[s] = -(dv * y1 - dv * y2) - 0.5 * gamma * ((gx * gx + gf * gf) / wv);
        }
        delta[e] = term[0] - term[1];
    }
}

// ---------------------------------------------------------------------------
// Layout conversion: schedule order -> colex order.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(1024)
k_to_lex(const Tile *__restrict__ tiles, int b, int64_t n, const T *__restrict__ y,
         T *__restrict__ ylex) {
    const int bb = b * b;
    const int tid = threadIdx.x;
    const int il = tid / b, kl = tid - (tid / b) * b;
    const Tile tl = tiles[blockIdx.x];
    const int64_t i = int64_t(tl.P) * b + il, k = int64_t(tl.Q) * b + kl;
    const bool desc = tile_desc(tl.P, tl.Q, int((n + b - 1) / b));
    for (int m = 0; m <= tl.Q - tl.P; ++m)
        for (int t = 0; t < b; ++t) {
            const int J = tile_J(tl.P, tl.Q, m, desc);
            const int64_t j = int64_t(J) * b + mid_offset(t, il, kl, b);
            if (i < j && j < k && k < n) {
                const int64_t u = int64_t(m) * b + t;
                const T *src = y + tl.ybase + u * 3 * bb + tid;
                T *dst = ylex + 3 * tidx(i, j, k);
                dst[0] = src[0];
                dst[1] = src[bb];
                dst[2] = src[2 * bb];
            }
        }
}

__global__ void k_slots_to_lex(const Tile *__restrict__ tiles, int64_t ntiles, int b, int64_t n,
                               const int64_t *__restrict__ slots, int64_t count,
                               int64_t *__restrict__ out) {
    const int64_t bb = int64_t(b) * b;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int64_t s = slots[e];
        int64_t lo = 0, hi = ntiles - 1;
        while (lo < hi) {  // last tile with ybase <= s
            const int64_t mid = (lo + hi + 1) / 2;
            if (tiles[mid].ybase <= s) lo = mid; else hi = mid - 1;
        }
        const Tile tl = tiles[lo];
        const int64_t off = s - tl.ybase;
        const int64_t u = off / (3 * bb), rem = off - u * 3 * bb;
        const int o = int(rem / bb), lane = int(rem - (rem / bb) * bb);
        const int il = lane / b, kl = lane % b;
        const int mm = int(u / b), t = int(u % b);
        const bool desc = tile_desc(tl.P, tl.Q, int((n + b - 1) / b));
        const int J = tile_J(tl.P, tl.Q, mm, desc);
        const int64_t i = int64_t(tl.P) * b + il, k = int64_t(tl.Q) * b + kl;
        const int64_t j = int64_t(J) * b + mid_offset(t, il, kl, b);
        const bool ok = s >= 0 && mm <= tl.Q - tl.P && i < j && j < k && k < n;
        out[e] = ok ? 3 * tidx(i, j, k) + o : -1;
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
static inline unsigned grid_of(int64_t count, int block) {
    int64_t g = (count + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return unsigned(g);
}

template <typename T>
int launch_metric_resid(const Tile *tiles, const int32_t *chunks, int64_t nchunks, int b, int64_t n,
                        const T *x, const T *y, double *partial, hipStream_t s) {
    const dim3 grid = dim3(unsigned(nchunks));
    if (!y) {
        switch (b) {
            case 8: hipLaunchKernelGGL((k_metric_viol<T, 8>), grid, dim3(64), 0, s, tiles, chunks, b, n, x, partial); break;
            case 16: hipLaunchKernelGGL((k_metric_viol<T, 16>), grid, dim3(256), 0, s, tiles, chunks, b, n, x, partial); break;
            case 32: hipLaunchKernelGGL((k_metric_viol<T, 32>), grid, dim3(1024), 0, s, tiles, chunks, b, n, x, partial); break;
            default: hipLaunchKernelGGL((k_metric_viol<T, 0>), grid, dim3(b * b), 0, s, tiles, chunks, b, n, x, partial); break;
        }
        CCP_LAUNCH_CHECK("k_metric_viol");
        return CC_OK;
    }
    switch (b) {
        case 8: hipLaunchKernelGGL((k_metric_resid<T, 8>), grid, dim3(64), 0, s, tiles, chunks, b, n, x, y, partial); break;
        case 16: hipLaunchKernelGGL((k_metric_resid<T, 16>), grid, dim3(256), 0, s, tiles, chunks, b, n, x, y, partial); break;
        case 32: hipLaunchKernelGGL((k_metric_resid<T, 32>), grid, dim3(1024), 0, s, tiles, chunks, b, n, x, y, partial); break;
        default: hipLaunchKernelGGL((k_metric_resid<T, 0>), grid, dim3(b * b), 0, s, tiles, chunks, b, n, x, y, partial); break;
    }
    CCP_LAUNCH_CHECK("k_metric_resid");
    return CC_OK;
}

template <typename T>
int launch_nearness_pair_resid(int64_t np, const T *x, const double *dv, const double *w,
                               const double *ax, double *partial, hipStream_t s) {
    hipLaunchKernelGGL(k_nearness_pair_resid<T>, dim3(kPairBlocks), dim3(256), 0, s, np, x, dv, w,
                       ax, partial);
    CCP_LAUNCH_CHECK("k_nearness_pair_resid");
    return CC_OK;
}

template <typename T, typename DT>
int launch_pair_resid(int64_t np, const T *x, const T *f, const T *yp, const double *w,
                      const DT *d, const double *ax, double gamma, double *partial,
                      hipStream_t s) {
    hipLaunchKernelGGL((k_pair_resid<T, DT>), dim3(kPairBlocks), dim3(256), 0, s, np, x, f, yp, w, d,
                       ax, gamma, partial);
    CCP_LAUNCH_CHECK("k_pair_resid");
    return CC_OK;
}

int launch_final_reduce(const double *mpart, int64_t nm, const double *ppart, double *out,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_final_reduce, dim3(1), dim3(1024), 0, s, mpart, nm, ppart,
                       int64_t(kPairBlocks), out);
    CCP_LAUNCH_CHECK("k_final_reduce");
    return CC_OK;
}

int launch_weight_classes(int64_t np, const double *w, const uint8_t *d, double *partial, hipStream_t s) {
    hipLaunchKernelGGL(k_weight_classes, dim3(kPairBlocks), dim3(256), 0, s, np, w, d, partial);
    CCP_LAUNCH_CHECK("k_weight_classes");
    return CC_OK;
}

int pair_partial_blocks() { return kPairBlocks; }

template <typename T>
int launch_aty_round(const Tile *tiles, int ntiles, int b, int64_t n, const T *y, double *ax,
                     hipStream_t s) {
    if (ntiles <= 0) return CC_OK;
    switch (b) {
        case 8: hipLaunchKernelGGL((k_aty_round<T, 8>), dim3(ntiles), dim3(64), 0, s, tiles, b, n, y, ax); break;
        case 16: hipLaunchKernelGGL((k_aty_round<T, 16>), dim3(ntiles), dim3(256), 0, s, tiles, b, n, y, ax); break;
        case 32: hipLaunchKernelGGL((k_aty_round<T, 32>), dim3(ntiles), dim3(1024), 0, s, tiles, b, n, y, ax); break;
        default: hipLaunchKernelGGL((k_aty_round<T, 0>), dim3(ntiles), dim3(b * b), 0, s, tiles, b, n, y, ax); break;
    }
    CCP_LAUNCH_CHECK("k_aty_round");
    return CC_OK;
}

template <typename T>
int launch_x_from_aty(int64_t np, const double *ax, const T *yp, const double *w, double gamma,
                      T *x, T *f, hipStream_t s) {
    hipLaunchKernelGGL(k_x_from_aty<T>, dim3(grid_of(np, 256)), dim3(256), 0, s, np, ax, yp, w,
                       gamma, x, f);
    CCP_LAUNCH_CHECK("k_x_from_aty");
    return CC_OK;
}

template <typename T>
int launch_to_lex(const Tile *tiles, int64_t ntiles, int b, int64_t n, const T *y, T *ylex,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_to_lex<T>, dim3(ntiles), dim3(b * b), 0, s, tiles, b, n, y, ylex);
    CCP_LAUNCH_CHECK("k_to_lex");
    return CC_OK;
}

int launch_slots_to_lex(const Tile *tiles, int64_t ntiles, int b, int64_t n,
                        const int64_t *slots, int64_t count, int64_t *out, hipStream_t s) {
    if (count <= 0) return CC_OK;
    hipLaunchKernelGGL(k_slots_to_lex, dim3(grid_of(count, 256)), dim3(256), 0, s, tiles,
                       ntiles, b, n, slots, count, out);
    CCP_LAUNCH_CHECK("k_slots_to_lex");
    return CC_OK;
}

template <typename T>
int launch_gate_pairs(int64_t np, int64_t count, const int64_t *pairs, const double *w, const uint8_t *d,
                      const T *g, double *ws, uint8_t *ds, T *gs, hipStream_t s) {
    if (count <= 0) return CC_OK;
    hipLaunchKernelGGL(k_gate_gather<T>, dim3(grid_of(count, 256)), dim3(256), 0, s, np, count, pairs,
                       w, d, g, ws, ds, gs);
    CCP_LAUNCH_CHECK("k_gate_gather");
    return CC_OK;
}

template <typename T>
int launch_gate_delta(int64_t count, const double *aty, const T *ypw, const T *ypc, const double *ws,
                      const uint8_t *ds, double gamma, double *delta, hipStream_t s) {
    if (count <= 0) return CC_OK;
    hipLaunchKernelGGL(k_gate_delta<T>, dim3(grid_of(count, 256)), dim3(256), 0, s, count, aty, ypw,
                       ypc, ws, ds, gamma, delta);
    CCP_LAUNCH_CHECK("k_gate_delta");
    return CC_OK;
}

template int launch_gate_pairs<double>(int64_t, int64_t, const int64_t *, const double *, const uint8_t *,
                                       const double *, double *, uint8_t *, double *, hipStream_t);
template int launch_gate_pairs<float>(int64_t, int64_t, const int64_t *, const double *, const uint8_t *,
                                      const float *, double *, uint8_t *, float *, hipStream_t);
template int launch_gate_delta<double>(int64_t, const double *, const double *, const double *,
                                       const double *, const uint8_t *, double, double *, hipStream_t);
template int launch_gate_delta<float>(int64_t, const double *, const float *, const float *,
                                      const double *, const uint8_t *, double, double *, hipStream_t);
template int launch_nearness_pair_resid<double>(int64_t, const double *, const double *,
                                                const double *, const double *, double *,
                                                hipStream_t);
template int launch_nearness_pair_resid<float>(int64_t, const float *, const double *,
                                               const double *, const double *, double *,
                                               hipStream_t);
template int launch_metric_resid<double>(const Tile *, const int32_t *, int64_t, int, int64_t,
                                         const double *, const double *, double *, hipStream_t);
template int launch_metric_resid<float>(const Tile *, const int32_t *, int64_t, int, int64_t,
                                        const float *, const float *, double *, hipStream_t);
template int launch_pair_resid<double, uint8_t>(int64_t, const double *, const double *, const double *,
                                                const double *, const uint8_t *, const double *, double,
                                                double *, hipStream_t);
template int launch_pair_resid<float, uint8_t>(int64_t, const float *, const float *, const float *,
                                               const double *, const uint8_t *, const double *, double,
                                               double *, hipStream_t);
template int launch_pair_resid<double, double>(int64_t, const double *, const double *, const double *,
                                               const double *, const double *, const double *, double,
                                               double *, hipStream_t);
template int launch_pair_resid<float, double>(int64_t, const float *, const float *, const float *,
                                              const double *, const double *, const double *, double,
                                              double *, hipStream_t);
template int launch_aty_round<double>(const Tile *, int, int, int64_t, const double *, double *,
                                      hipStream_t);
template int launch_aty_round<float>(const Tile *, int, int, int64_t, const float *, double *,
                                     hipStream_t);
template int launch_x_from_aty<double>(int64_t, const double *, const double *, const double *,
                                       double, double *, double *, hipStream_t);
template int launch_x_from_aty<float>(int64_t, const double *, const float *, const double *,
                                      double, float *, float *, hipStream_t);
template int launch_to_lex<double>(const Tile *, int64_t, int, int64_t, const double *, double *,
                                   hipStream_t);
template int launch_to_lex<float>(const Tile *, int64_t, int, int64_t, const float *, float *,
                                  hipStream_t);

}  // namespace ccp
