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

}  // namespace smc
