// Double-double helpers for building Abel nodes to full FP64 accuracy.
// Every function compiles with FP contraction off: the error-free
// transformations depend on separately rounded products and sums.
#pragma once

#include <hip/hip_runtime.h>

namespace lc {

// 1 - a b for double-double a, b (a b in [0, 2]), rounded to FP64.
__device__ __forceinline__ double node_dd(double2 a, double2 b) {
#pragma clang fp contract(off)
    const double p = a.x * b.x;
    double e = fma(a.x, b.x, -p);
    e = fma(a.x, b.y, fma(a.y, b.x, e));
    const double s = 1.0 - p;
    const double bb = s - 1.0;
    const double err = (1.0 - (s - bb)) + (-p - bb);
    return s + (err - e);
}

// a b for double-double a, b, rounded to FP64 (the complement 1 - x of the
// node node_dd(a, b)).
__device__ __forceinline__ double omx_dd(double2 a, double2 b) {
#pragma clang fp contract(off)
    const double p = a.x * b.x;
    double e = fma(a.x, b.x, -p);
    e = fma(a.x, b.y, fma(a.y, b.x, e));
    return p + e;
}

__device__ __forceinline__ double2 dd_quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    return make_double2(s, b - (s - a));
}

__device__ __forceinline__ double2 dd_two_sum(double a, double b) {
#pragma clang fp contract(off)
    const double s = a + b;
    const double bb = s - a;
    return make_double2(s, (a - (s - bb)) + (b - bb));
}

__device__ __forceinline__ double2 dd_add(double2 a, double2 b) {
#pragma clang fp contract(off)
    const double2 s = dd_two_sum(a.x, b.x);
    return dd_quick_two_sum(s.x, s.y + (a.y + b.y));
}

__device__ __forceinline__ double2 dd_mul(double2 a, double2 b) {
#pragma clang fp contract(off)
    const double p = a.x * b.x;
    double e = fma(a.x, b.x, -p);
    e += a.x * b.y + a.y * b.x;
    return dd_quick_two_sum(p, e);
}

}  // namespace lc
