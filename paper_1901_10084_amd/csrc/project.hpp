// project.hpp -- device pieces shared by the sweep executors.
#pragma once

#include "common.hpp"

namespace ccp {

template <typename T>
struct XG {
    T x;  // distance variable x_p
    T g;  // gamma / w_p
};

__device__ __forceinline__ void lds_barrier() {
    // Orders LDS only: global loads in flight (the dual prefetch) stay in
    // flight across the barrier.
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// 1/s.  FP64: hardware reciprocal refined by two Newton steps (about one
// ulp; the oracle's correctly rounded quotient differs by at most that).
template <typename T>
__device__ __forceinline__ T recip(T s) {
    double r = __builtin_amdgcn_rcp(s);
    double e = fma(-s, r, 1.0);
    r = fma(r, e, r);
    e = fma(-s, r, 1.0);
    return fma(r, e, r);
}
template <>
__device__ __forceinline__ float recip<float>(float s) {
    return __builtin_amdgcn_rcpf(s);
}

// One row of Algorithm 1 (correction + projection + dual update, merged).
template <typename T>
__device__ __forceinline__ void project(T &xL, T &xS1, T &xS2, T gL, T gS1, T gS2, T q,
                                        T &y) {
    T delta = (xL - xS1) - xS2;
    T th = fma(delta, q, y);
    th = th > T(0) ? th : T(0);
    T dlt = th - y;
    xL = fma(-dlt, gL, xL);
    xS1 = fma(dlt, gS1, xS1);
    xS2 = fma(dlt, gS2, xS2);
    y = th;
}

// The same step with a per-row floor: lo = 0 gives the step above (up to the
// sign of a zero theta); a padding lane passes q = 0 and lo = -inf, so
// th = y exactly and nothing moves.  Lets every lane run the step without a
// branch.
template <typename T>
__device__ __forceinline__ void project_lo(T &xL, T &xS1, T &xS2, T gL, T gS1, T gS2, T q,
                                           T lo, T &y) {
    T delta = (xL - xS1) - xS2;
    T th = fmax(fma(delta, q, y), lo);
    T dlt = th - y;
    xL = fma(-dlt, gL, xL);
    xS1 = fma(dlt, gS1, xS1);
    xS2 = fma(dlt, gS2, xS2);
    y = th;
}

}  // namespace ccp
