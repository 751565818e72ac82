// Wavefront (64-lane) and workgroup reductions and scans.
//
// Every reduction here combines values in one fixed order that depends only on
// lane and block indices, so a result is bit-reproducible across launches.
#pragma once
#include <hip/hip_runtime.h>

#include "dd.hpp"

namespace smc {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ dd wave_sum(dd v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        dd o{__shfl_xor(v.hi, off, kWave), __shfl_xor(v.lo, off, kWave)};
        v = dd_add(v, o);
    }
    return v;
}

// Running log-sum-exp state: the set {x} is represented by (m, s) with
// sum exp(x) = s * exp(m). Combining is associative up to rounding.
struct LseAcc {
    double m, s;
};

__device__ __forceinline__ LseAcc lse_empty() { return LseAcc{-INFINITY, 0.0}; }

__device__ __forceinline__ LseAcc lse_push(LseAcc a, double x) {
    if (x == -INFINITY) return a;
    if (x > a.m) {
        const double s = (a.m == -INFINITY) ? 0.0 : a.s * exp(a.m - x);
        return LseAcc{x, s + 1.0};
    }
    return LseAcc{a.m, a.s + exp(x - a.m)};
}

__device__ __forceinline__ LseAcc lse_merge(LseAcc a, LseAcc b) {
    if (b.m == -INFINITY) return a;
    if (a.m == -INFINITY) return b;
    if (a.m >= b.m) return LseAcc{a.m, a.s + b.s * exp(b.m - a.m)};
    return LseAcc{b.m, b.s + a.s * exp(a.m - b.m)};
}

__device__ __forceinline__ LseAcc wave_lse(LseAcc v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        LseAcc o{__shfl_xor(v.m, off, kWave), __shfl_xor(v.s, off, kWave)};
        // combine in lane order so that lanes agree bit for bit
        v = (lane_id() & off) ? lse_merge(o, v) : lse_merge(v, o);
    }
    return v;
}

__device__ __forceinline__ double lse_value(LseAcc a) {
    return (a.m == -INFINITY) ? -INFINITY : a.m + log(a.s);
}

}  // namespace smc
