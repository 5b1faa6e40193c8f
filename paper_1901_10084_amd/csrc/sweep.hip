// sweep.hip -- the projection sweep on gfx950: metric rounds and pair pass.
//
// Method: Algorithm 1 of the paper (Dykstra's = Hildreth's method for the
// regularised LP (qp)), one dual per constraint.  For a row a'v <= beta the
// correction step followed by the projection step of Algorithm 1 collapse
// into one update of v, because the correction moves v along the same
// direction gamma W^{-1} a that the projection then moves back along:
//     theta = max(y + (a'v - beta) / (gamma a'W^{-1}a), 0),
//     v    -= (theta - y) * gamma W^{-1} a,      y = theta.
// With g_p = gamma / w_p this reads, for a metric row with long side L and
// short sides S1, S2 (a = e_L - e_S1 - e_S2, beta = 0; Sec. II-B shows the
// W = I case, where the three entries move by delta/3):
//     q = 1 / (g_L + g_S1 + g_S2),  theta = max(fma(a'x, q, y), 0),
//     x_L -= (theta - y) g_L,  x_S1 += (theta - y) g_S1,  x_S2 += ... g_S2.
//
// Schedule (Sec. III-B, III-C): tile (P,Q) = all triplets with smallest
// index in block P and largest in block Q; a round = every tile on one block
// anti-diagonal P+Q, run concurrently (one workgroup per tile, no locks: two
// tiles of a round never share a pair).  Inside a tile the middle block J
// runs from Q down to P in the rounds of Fig. 2's first double loop
// (P + Q < nb) and from P up to Q in those of the second (tile_J); inside
// a (tile, J) cube, sub-step t gives lane (il, kl) the
// middle offset jl with il + jl + kl = t (mod b), so the b*b lanes of a
// sub-step touch pairwise distinct pairs and run in parallel; sub-steps are
// separated by workgroup barriers.
//
// Data movement per tile: the x/g blocks (P,J), (J,Q) and (P,Q) live in LDS
// (b*b pairs each; the (P,Q) block stays for the whole tile, the other two
// are double-buffered and the next J's pair is fetched during the current
// J); the duals stream through a register ring D sub-steps deep.  Each
// sub-step reads and writes three contiguous vectors of b*b duals.
#include "common.hpp"
#include "project.hpp"

namespace ccp {

// Metric rounds: one workgroup of b*b threads per tile of the round.
// B: compile-time tile size (0 = runtime b), D: dual prefetch depth (D | b).
//
// Every thread issues its dual loads and stores unconditionally, at an
// address inside its tile's segment (lanes without a triplet touch their
// own padding slot and write back what they read), so the hardware's
// in-order load counter lets each sub-step wait only for the load it needs
// and the prefetch ring stays in flight.  1/(g_ij + g_ik + g_jk) does not
// depend on x, so it is computed one sub-step ahead.
template <typename T, int B, int D>
__global__ void __launch_bounds__(B ? B * B : 1024)
k_sweep_round(const Tile *__restrict__ tiles, int b_rt, int64_t n, T *__restrict__ x,
              const T *__restrict__ g, T *__restrict__ y) {
    const int b = B ? B : b_rt;
    const int bb = b * b;
    const int tid = threadIdx.x;
    const int il = tid / b, kl = tid - (tid / b) * b;
    const Tile tl = tiles[blockIdx.x];
    const int P = tl.P, Q = tl.Q;
    const int nn = int(n);

    extern __shared__ __align__(16) unsigned char smem_raw[];
    XG<T> *lds = reinterpret_cast<XG<T> *>(smem_raw);
    XG<T> *const Cs = lds + 4 * bb;

    const int i = P * b + il;
    const int k = Q * b + kl;

    // (P,Q) block: pair (i,k) of this lane.
    const bool c_ok = (i < k) && (k < nn);
    const int64_t pc = c_ok ? pidx(i, k) : 0;
    {
        const T cx = x[pc], cg = g[pc];
        Cs[tid] = XG<T>{c_ok ? cx : T(0), c_ok ? cg : T(0)};
    }

    // Element (il, kl) of the (P,J) and (J,Q) blocks, fetched and written
    // back by this thread (pair 0 stands in for missing pairs).
    auto a_pair = [&](int J, int64_t &p) {
        const int ii = P * b + il, jj = J * b + kl;
        const bool ok = ii < jj && jj < nn;
        p = ok ? pidx(ii, jj) : 0;
        return ok;
    };
    auto b_pair = [&](int J, int64_t &p) {
        const int jj = J * b + il, kk = Q * b + kl;
        const bool ok = jj < kk && kk < nn;
        p = ok ? pidx(jj, kk) : 0;
        return ok;
    };

    // Linear sub-step u = m * b + t (m-th middle block of the tile, see
    // tile_J); the duals of step u live at y[ybase + u*3*bb + o*bb + tid].
    const int U = (Q - P + 1) * b;
    const bool desc = tile_desc(P, Q, (nn + b - 1) / b);
    T *const ylane = y + tl.ybase + tid;
    const int64_t ystep = int64_t(3) * bb;

    T yq[D][3];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const T *src = ylane + int64_t(d < U ? d : U - 1) * ystep;
        yq[d][0] = src[0];
        yq[d][1] = src[bb];
        yq[d][2] = src[2 * bb];
    }

    // Prologue: stage the first middle block's (P,J) / (J,Q) block into
    // buffer 0.  J = P: A is block (P,P), B aliases C.  J = Q: A aliases C,
    // B is block (Q,Q).
    if (P != Q) {
        int64_t p;
        const bool ok = desc ? b_pair(Q, p) : a_pair(P, p);
        const T vx = x[p], vg = g[p];
        lds[(desc ? 2 : 0) * bb + tid] = XG<T>{ok ? vx : T(0), ok ? vg : T(0)};
    }
    lds_barrier();

    for (int m = 0; m <= Q - P; ++m) {
        const int J = tile_J(P, Q, m, desc);
        const int cur = m & 1;
        XG<T> *const As = (J == Q) ? Cs : lds + cur * bb;
        XG<T> *const Bs = (J == P) ? Cs : lds + (2 + cur) * bb;

        // Next middle block: fetched now, staged into LDS after this one.
        const bool more = m < Q - P;
        const int Jn = more ? tile_J(P, Q, m + 1, desc) : J;
        int64_t pa, pb;
        const bool na_ok = more && Jn != Q && a_pair(Jn, pa);
        const bool nb_ok = more && Jn != P && b_pair(Jn, pb);
        if (!na_ok) pa = 0;
        if (!nb_ok) pb = 0;
        const T nax = x[pa], nag = g[pa], nbx = x[pb], nbg = g[pb];

        auto qof = [&](int t) {
            const int jl = mid_offset(t, il, kl, b);
            const T s = (As[il * b + jl].g + Cs[tid].g) + Bs[jl * b + kl].g;
            return recip<T>(s > T(0) ? s : T(1));
        };
        T qn = qof(0);

        for (int t0 = 0; t0 < b; t0 += D) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int t = t0 + d;
                const int u = m * b + t;
                T y0 = yq[d][0], y1 = yq[d][1], y2 = yq[d][2];
                // prefetch step u + D into the freed ring slot
                {
                    const int un = u + D < U ? u + D : U - 1;
                    const T *src = ylane + int64_t(un) * ystep;
                    yq[d][0] = src[0];
                    yq[d][1] = src[bb];
                    yq[d][2] = src[2 * bb];
                }
                const T q = qn;
                if (t + 1 < b) qn = qof(t + 1);
                const int jl = mid_offset(t, il, kl, b);
                const int j = J * b + jl;
                const bool ok = i < j && j < k && k < nn;
                if (ok) {
                    XG<T> ea = As[il * b + jl];  // pair (i,j)
                    XG<T> eb = Bs[jl * b + kl];  // pair (j,k)
                    XG<T> ec = Cs[tid];          // pair (i,k)
                    T xa = ea.x, xb = eb.x, xc = ec.x;
                    project(xa, xc, xb, ea.g, ec.g, eb.g, q, y0);  // x_ij <= x_ik + x_jk
                    project(xc, xa, xb, ec.g, ea.g, eb.g, q, y1);  // x_ik <= x_ij + x_jk
                    project(xb, xa, xc, eb.g, ea.g, ec.g, q, y2);  // x_jk <= x_ij + x_ik
                    As[il * b + jl].x = xa;
                    Bs[jl * b + kl].x = xb;
                    Cs[tid].x = xc;
                }
                T *dst = ylane + int64_t(u) * ystep;
                dst[0] = y0;
                dst[bb] = y1;
                dst[2 * bb] = y2;
                lds_barrier();
            }
        }

        // Write back this step's (P,J) and (J,Q) blocks; stage the next.
        {
            int64_t p;
            if (As != Cs && a_pair(J, p)) x[p] = As[tid].x;
            if (Bs != Cs && b_pair(J, p)) x[p] = Bs[tid].x;
            if (more) {
                const int nxt = cur ^ 1;
                if (Jn != Q) lds[nxt * bb + tid] = XG<T>{na_ok ? nax : T(0), na_ok ? nag : T(0)};
                if (Jn != P) lds[(2 + nxt) * bb + tid] = XG<T>{nb_ok ? nbx : T(0), nb_ok ? nbg : T(0)};
            }
        }
        lds_barrier();
    }

    if (c_ok) x[pc] = Cs[tid].x;
}

// Pair pass: rows x - f <= d and -x - f <= -d of every pair, in that order.
// d: uint8 0/1 for correlation clustering, double for l1 metric nearness
template <typename T, typename DT>
__global__ void __launch_bounds__(256)
k_pair_pass(int64_t np, T *__restrict__ x, T *__restrict__ f, T *__restrict__ yp,
            const T *__restrict__ g, const DT *__restrict__ d) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < np;
         p += int64_t(gridDim.x) * blockDim.x) {
        T xv = x[p], fv = f[p];
        const T gv = g[p], dv = T(d[p]);
        const T q = recip<T>(gv + gv);
        T y1 = yp[2 * p], y2 = yp[2 * p + 1];
        // x - f <= d
        T delta = (xv - fv) - dv;
        T th = fma(delta, q, y1);
        th = th > T(0) ? th : T(0);
        T dl = th - y1;
        xv = fma(-dl, gv, xv);
        fv = fma(dl, gv, fv);
        y1 = th;
        // -x - f <= -d
        delta = (-xv - fv) + dv;
        th = fma(delta, q, y2);
        th = th > T(0) ? th : T(0);
        dl = th - y2;
        xv = fma(dl, gv, xv);
        fv = fma(dl, gv, fv);
        y2 = th;
        x[p] = xv;
        f[p] = fv;
        yp[2 * p] = y1;
        yp[2 * p + 1] = y2;
    }
}

// g = gamma / w; flags a weight that is not finite and positive.
template <typename T>
__global__ void k_prepare(int64_t np, const double *__restrict__ w, double gamma,
                          T *__restrict__ g, int *__restrict__ bad) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < np;
         p += int64_t(gridDim.x) * blockDim.x) {
        const double wp = w[p];
        if (!(wp > 0.0) || !(wp <= 1.7976931348623157e308)) atomicOr(bad, 1);
        g[p] = T(gamma / wp);
    }
}

// Starting point: x = 0, f = -gamma, y_pair = 0 (the duals are zero-filled
// separately).
template <typename T>
__global__ void k_init_cold(int64_t np, T *__restrict__ x, T *__restrict__ f,
                            T *__restrict__ yp, double gamma) {
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < np;
         p += int64_t(gridDim.x) * blockDim.x) {
        x[p] = T(0);
        f[p] = T(-gamma);
        yp[2 * p] = T(0);
        yp[2 * p + 1] = T(0);
    }
}

template <typename T>
__global__ void k_fill_zero(int64_t count, T *__restrict__ a) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += int64_t(gridDim.x) * blockDim.x)
        a[e] = T(0);
}

template <typename S, typename D>
__global__ void k_convert(int64_t count, const S *__restrict__ src, D *__restrict__ dst) {
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count;
         e += int64_t(gridDim.x) * blockDim.x)
        dst[e] = D(src[e]);
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t count, int block) {
    int64_t g = (count + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return unsigned(g);
}

template <typename T>
size_t sweep_lds_bytes(int b) {
    return size_t(5) * b * b * sizeof(XG<T>);
}

template <typename T, int B, int D>
static int launch_round_t(const Tile *tiles, int ntiles, int b, int64_t n, T *x, const T *g,
                          T *y, hipStream_t s) {
    const size_t lds = sweep_lds_bytes<T>(b);
    hipLaunchKernelGGL((k_sweep_round<T, B, D>), dim3(ntiles), dim3(b * b), lds, s, tiles, b,
                       n, x, g, y);
    CCP_LAUNCH_CHECK("k_sweep_round");
    return CC_OK;
}

template <typename T>
int launch_sweep_round(const Tile *tiles, int ntiles, int b, int64_t n, T *x, const T *g,
                       T *y, hipStream_t s) {
    if (ntiles <= 0) return CC_OK;
    switch (b) {
        case 8: return launch_round_t<T, 8, 4>(tiles, ntiles, b, n, x, g, y, s);
        case 16: return launch_round_t<T, 16, 8>(tiles, ntiles, b, n, x, g, y, s);
        case 32: return launch_round_t<T, 32, 4>(tiles, ntiles, b, n, x, g, y, s);
        default: return launch_round_t<T, 0, 1>(tiles, ntiles, b, n, x, g, y, s);
    }
}

template <typename T>
int set_sweep_lds_limits(int b) {
    const int lds = int(sweep_lds_bytes<T>(b));
    hipError_t e = hipSuccess;
    switch (b) {
        case 8: e = hipFuncSetAttribute((const void *)k_sweep_round<T, 8, 4>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
        case 16: e = hipFuncSetAttribute((const void *)k_sweep_round<T, 16, 8>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
        case 32: e = hipFuncSetAttribute((const void *)k_sweep_round<T, 32, 4>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
        default: e = hipFuncSetAttribute((const void *)k_sweep_round<T, 0, 1>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, lds); break;
    }
    if (e != hipSuccess) return fail(CC_EHIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    return CC_OK;
}

template <typename T, typename DT>
int launch_pair_pass(int64_t np, T *x, T *f, T *yp, const T *g, const DT *d,
                     hipStream_t s) {
    hipLaunchKernelGGL((k_pair_pass<T, DT>), dim3(grid_for(np, 256)), dim3(256), 0, s, np, x, f, yp,
                       g, d);
    CCP_LAUNCH_CHECK("k_pair_pass");
    return CC_OK;
}

template <typename T>
int launch_prepare(int64_t np, const double *w, double gamma, T *g, int *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_prepare<T>, dim3(grid_for(np, 256)), dim3(256), 0, s, np, w, gamma, g,
                       bad);
    CCP_LAUNCH_CHECK("k_prepare");
    return CC_OK;
}

template <typename T>
int launch_init_cold(int64_t np, int64_t slots, T *x, T *f, T *y, T *yp, double gamma,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_init_cold<T>, dim3(grid_for(np, 256)), dim3(256), 0, s, np, x, f, yp,
                       gamma);
    CCP_LAUNCH_CHECK("k_init_cold");
    if (y) {
        hipLaunchKernelGGL(k_fill_zero<T>, dim3(grid_for(slots, 256)), dim3(256), 0, s, slots,
                           y);
        CCP_LAUNCH_CHECK("k_fill_zero");
    }
    return CC_OK;
}

// l2 metric nearness: Algorithm 1 starts at x = d (the dissimilarities, in
// the context's precision) with every dual 0.
template <typename T>
int launch_nearness_init(int64_t np, int64_t slots, const double *dv, T *x, T *y, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<double, T>), dim3(grid_for(np, 256)), dim3(256), 0, s, np, dv, x);
    CCP_LAUNCH_CHECK("k_convert");
    hipLaunchKernelGGL(k_fill_zero<T>, dim3(grid_for(slots, 256)), dim3(256), 0, s, slots, y);
    CCP_LAUNCH_CHECK("k_fill_zero");
    return CC_OK;
}

template <typename S, typename D>
int launch_convert(int64_t count, const S *src, D *dst, hipStream_t s) {
    if (count <= 0) return CC_OK;
    hipLaunchKernelGGL((k_convert<S, D>), dim3(grid_for(count, 256)), dim3(256), 0, s, count,
                       src, dst);
    CCP_LAUNCH_CHECK("k_convert");
    return CC_OK;
}

template int launch_sweep_round<double>(const Tile *, int, int, int64_t, double *,
                                        const double *, double *, hipStream_t);
template int launch_sweep_round<float>(const Tile *, int, int, int64_t, float *, const float *,
                                       float *, hipStream_t);
template int set_sweep_lds_limits<double>(int);
template int set_sweep_lds_limits<float>(int);
template int launch_pair_pass<double, uint8_t>(int64_t, double *, double *, double *, const double *,
                                               const uint8_t *, hipStream_t);
template int launch_pair_pass<float, uint8_t>(int64_t, float *, float *, float *, const float *,
                                              const uint8_t *, hipStream_t);
template int launch_pair_pass<double, double>(int64_t, double *, double *, double *, const double *,
                                              const double *, hipStream_t);
template int launch_pair_pass<float, double>(int64_t, float *, float *, float *, const float *,
                                             const double *, hipStream_t);
template int launch_prepare<double>(int64_t, const double *, double, double *, int *,
                                    hipStream_t);
template int launch_prepare<float>(int64_t, const double *, double, float *, int *,
                                   hipStream_t);
template int launch_init_cold<double>(int64_t, int64_t, double *, double *, double *, double *,
                                      double, hipStream_t);
template int launch_init_cold<float>(int64_t, int64_t, float *, float *, float *, float *,
                                     double, hipStream_t);
template int launch_nearness_init<double>(int64_t, int64_t, const double *, double *, double *,
                                          hipStream_t);
template int launch_nearness_init<float>(int64_t, int64_t, const double *, float *, float *,
                                         hipStream_t);
template int launch_convert<float, double>(int64_t, const float *, double *, hipStream_t);
template int launch_convert<double, float>(int64_t, const double *, float *, hipStream_t);

}  // namespace ccp
