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

// Orders the wave's LDS accesses before the call against those after it (for
// data one lane writes and other lanes of the same wave read).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

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

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
    return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
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
