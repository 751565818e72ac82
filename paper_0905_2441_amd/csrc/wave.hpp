// Wavefront (64-lane) and workgroup reductions and scans.
//
// Every reduction here combines values in one fixed order that depends only on
// lane and block indices, so a result is bit-reproducible across launches.
#pragma once
#include <hip/hip_runtime.h>

#include <climits>

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

// The largest and smallest of the wave's 64 values of v, in every lane, by
// DPP row shifts and row broadcasts (no LDS round trips). Floats are compared
// through integer keys that keep their order (a NaN comes out largest or
// smallest, by its sign bit).
__device__ __forceinline__ int float_order_key(float v) {
    const int b = __builtin_bit_cast(int, v);
    return b >= 0 ? b : b ^ 0x7fffffff;
}
__device__ __forceinline__ float float_of_order_key(int k) {
    return __builtin_bit_cast(float, k >= 0 ? k : k ^ 0x7fffffff);
}
template <bool MAX, int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_extreme_step(int v) {
    // a lane whose DPP source is outside its row, or whose row is masked off,
    // reads the operation's identity (so the DPP move folds into the min/max)
    constexpr int kId = MAX ? INT_MIN : INT_MAX;
    const int o = __builtin_amdgcn_update_dpp(kId, v, CTRL, ROW_MASK, 0xf, false);
    return MAX ? (v > o ? v : o) : (v < o ? v : o);
}
template <bool MAX>
__device__ __forceinline__ int wave_extreme_key(int v) {
    v = dpp_extreme_step<MAX, 0x111, 0xf>(v);   // row_shr:1
    v = dpp_extreme_step<MAX, 0x112, 0xf>(v);   // row_shr:2
    v = dpp_extreme_step<MAX, 0x114, 0xf>(v);   // row_shr:4
    v = dpp_extreme_step<MAX, 0x118, 0xf>(v);   // row_shr:8
    v = dpp_extreme_step<MAX, 0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_extreme_step<MAX, 0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ float wave_max_dpp(float v) {
    return float_of_order_key(wave_extreme_key<true>(float_order_key(v)));
}
__device__ __forceinline__ float wave_min_dpp(float v) {
    return float_of_order_key(wave_extreme_key<false>(float_order_key(v)));
}

// The sum of the wave's 64 values of v, in every lane: an inclusive scan within
// each row of 16 lanes by DPP row shifts (a source outside the row reads 0),
// then the row totals carried up by row broadcasts, so lane 63 ends with the
// total. The order of the additions is fixed.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_add_step(float v) {
    const int o = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROW_MASK, 0xf,
                                              true);
    return v + __builtin_bit_cast(float, o);
}
__device__ __forceinline__ float wave_sum_dpp(float v) {
    v = dpp_add_step<0x111, 0xf>(v);   // row_shr:1
    v = dpp_add_step<0x112, 0xf>(v);   // row_shr:2
    v = dpp_add_step<0x114, 0xf>(v);   // row_shr:4
    v = dpp_add_step<0x118, 0xf>(v);   // row_shr:8
    v = dpp_add_step<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
    v = dpp_add_step<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
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
