// colour.hip -- the metric rows in the order of the sum-mod-n colouring.
//
// Triplets that share a pair conflict (the colouring view of the related-
// work section); colour t holds every triplet i<j<k with i + j + k = t
// (mod n).  A pair fixes the third index of its colour, so no two triplets
// of a colour share a pair and all of them can be projected at once.  A
// sweep visits the colours t = 0..n-1 in turn, one launch each (the launch
// boundary orders the colours), then the pair pass.  Against the tiled
// schedule this trades locality for parallelism: a colour holds about
// n^2/6 independent triplets, but their distances are gathered from
// anywhere in x.
//
// Duals are kept in colex triplet order y[3 tidx(i,j,k) + o], the layout of
// cc_duals_to_lex, so a triplet's three duals are one contiguous access.
#include <math.h>

#include "common.hpp"
#include "project.hpp"

namespace ccp {

// One thread per pair (i,j) in packed order; the pair's triplet in colour t
// is (i, j, k) with k = (t - i - j) mod n, visited from its two smallest
// indices (k > j).  Per triplet: the three orientations in the schedule's
// order, with the sweep kernels' merged update.
template <typename T>
__global__ void __launch_bounds__(256)
k_sweep_colour(int64_t n, int64_t t, T *__restrict__ x, const T *__restrict__ g,
               T *__restrict__ y) {
    const int64_t np = n * (n - 1) / 2;
    for (int64_t p = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; p < np;
         p += int64_t(gridDim.x) * blockDim.x) {
        // p = j (j - 1) / 2 + i with 0 <= i < j
        int64_t j = int64_t((1.0 + sqrt(1.0 + 8.0 * double(p))) * 0.5);
        while (j * (j - 1) / 2 > p) --j;
        while ((j + 1) * j / 2 <= p) ++j;
        const int64_t i = p - j * (j - 1) / 2;
        int64_t k = (t - i - j) % n;
        if (k < 0) k += n;
        if (k <= j) continue;
        const int64_t pij = p, pik = pidx(i, k), pjk = pidx(j, k);
        T xij = x[pij], xik = x[pik], xjk = x[pjk];
        const T gij = g[pij], gik = g[pik], gjk = g[pjk];
        const T s = (gij + gik) + gjk;
        const T q = recip<T>(s > T(0) ? s : T(1));
        T *yt = y + 3 * tidx(i, j, k);
        T y0 = yt[0], y1 = yt[1], y2 = yt[2];
        project(xij, xik, xjk, gij, gik, gjk, q, y0);
        project(xik, xij, xjk, gik, gij, gjk, q, y1);
        project(xjk, xij, xik, gjk, gij, gik, q, y2);
        x[pij] = xij;
        x[pik] = xik;
        x[pjk] = xjk;
        yt[0] = y0;
        yt[1] = y1;
        yt[2] = y2;
    }
}

template <typename T>
int launch_sweep_colour(int64_t n, T *x, const T *g, T *y, hipStream_t s) {
    const int64_t np = n * (n - 1) / 2;
    int64_t grid = (np + 255) / 256;
    if (grid > 65536) grid = 65536;
    for (int64_t t = 0; t < n; ++t) {
        hipLaunchKernelGGL(k_sweep_colour<T>, dim3(unsigned(grid)), dim3(256), 0, s, n, t, x, g, y);
        CCP_LAUNCH_CHECK("k_sweep_colour");
    }
    return CC_OK;
}

template int launch_sweep_colour<double>(int64_t, double *, const double *, double *, hipStream_t);
template int launch_sweep_colour<float>(int64_t, float *, const float *, float *, hipStream_t);

}  // namespace ccp
