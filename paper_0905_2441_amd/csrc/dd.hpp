// Double-double (unevaluated sum hi + lo) arithmetic for the resampling CDF.
//
// Error-free transformations: TwoSum (Knuth, TAOCP vol. 2, 4.2.2) and
// FastTwoSum (Dekker 1971). The library is compiled with floating-point
// contraction off, so every + and - below rounds exactly once, which these
// transformations require.
#pragma once
#include <hip/hip_runtime.h>

namespace smc {

struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    const double err = (a - (s - bb)) + (b - bb);
    return dd{s, err};
}

// requires |a| >= |b| (or a == 0)
__device__ __forceinline__ dd fast_two_sum(double a, double b) {
    const double s = a + b;
    return dd{s, b - (s - a)};
}

__device__ __forceinline__ dd dd_add(dd x, double y) {
    dd s = two_sum(x.hi, y);
    s.lo += x.lo;
    return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_add(dd x, dd y) {
    dd s = two_sum(x.hi, y.hi);
    s.lo += x.lo + y.lo;
    return fast_two_sum(s.hi, s.lo);
}

__device__ __forceinline__ dd dd_zero() { return dd{0.0, 0.0}; }

}  // namespace smc
