// Workgroup reductions and scans shared by the weight and resampling kernels
// (one workgroup = kRedBlock threads). Every combine runs in a fixed lane and
// wave order, so results are bit-reproducible.
#pragma once
#include "internal.hpp"
#include "wave.hpp"

namespace smc {

struct Lse3 {
    double m, s1, s2;          // sum exp(x - m), sum exp(2 (x - m))
};

__device__ __forceinline__ Lse3 lse3_empty() { return Lse3{-INFINITY, 0.0, 0.0}; }

// Add x to a running (m, s1, s2). One exp whichever of x and m is larger:
// e = exp(-|x - m|) rescales the old sums when x is the new maximum and is the
// new term otherwise (selects instead of branches, so divergent lanes do not
// issue both exps). Bitwise the same as branching on x > m.
__device__ __forceinline__ Lse3 lse3_push(Lse3 a, double x) {
    if (x == -INFINITY) return a;
    const double d = x - a.m;                   // +inf while the sums are empty
    const double e = exp(-fabs(d));
    const bool up = d > 0.0;
    return Lse3{up ? x : a.m, up ? a.s1 * e + 1.0 : a.s1 + e,
                up ? a.s2 * (e * e) + 1.0 : a.s2 + e * e};
}

// Wave (64 lanes) log-sum-exp, the same value in every lane: the wave maximum
// first, then each lane's sums rescaled to it with one exp and added by a
// fixed butterfly.
__device__ __forceinline__ Lse3 wave_lse3(Lse3 v) {
    const double m = wave_max(v.m);
    const double r = (v.m == -INFINITY) ? 0.0 : exp(v.m - m);
    return Lse3{m, wave_sum(v.s1 * r), wave_sum(v.s2 * (r * r))};
}

__device__ __forceinline__ Lse3 lse3_merge(Lse3 a, Lse3 b) {
    if (b.m == -INFINITY) return a;
    if (a.m == -INFINITY) return b;
    if (a.m >= b.m) {
        const double r = exp(b.m - a.m);
        return Lse3{a.m, a.s1 + b.s1 * r, a.s2 + b.s2 * (r * r)};
    }
    const double r = exp(a.m - b.m);
    return Lse3{b.m, b.s1 + a.s1 * r, b.s2 + a.s2 * (r * r)};
}

// Block (kRedBlock threads) log-sum-exp; the result is valid in thread 0.
// The block maximum is formed first, then every thread rescales its sums to it
// with one exp and the rescaled sums are added in fixed order: one exp per
// thread instead of one per butterfly stage.
__device__ __forceinline__ Lse3 block_lse3(Lse3 v) {
    __shared__ double sm[kRedBlock / kWave], s1[kRedBlock / kWave], s2[kRedBlock / kWave];
    const double mw = wave_max(v.m);
    if (lane_id() == 0) sm[wave_id()] = mw;
    __syncthreads();
    double M = sm[0];
#pragma unroll
    for (int w = 1; w < kRedBlock / kWave; ++w) M = fmax(M, sm[w]);
    const double r = (v.m == -INFINITY) ? 0.0 : exp(v.m - M);
    const double a = wave_sum(v.s1 * r);
    const double b = wave_sum(v.s2 * (r * r));
    if (lane_id() == 0) {
        s1[wave_id()] = a;
        s2[wave_id()] = b;
    }
    __syncthreads();
    Lse3 out{M, 0.0, 0.0};
    if (threadIdx.x == 0) {
        for (int w = 0; w < kRedBlock / kWave; ++w) {
            out.s1 += s1[w];
            out.s2 += s2[w];
        }
    }
    __syncthreads();
    return out;
}

// Block (kRedBlock threads) maximum, valid in every thread.
__device__ __forceinline__ double block_max(double v) {
    __shared__ double sh[kRedBlock / kWave];
    v = wave_max(v);
    if (lane_id() == 0) sh[wave_id()] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < kRedBlock / kWave; ++w) r = fmax(r, sh[w]);
    __syncthreads();
    return r;
}

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double sh[kRedBlock / kWave];
    v = wave_sum(v);
    if (lane_id() == 0) sh[wave_id()] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedBlock / kWave; ++w) r += sh[w];
    __syncthreads();
    return r;
}

// Block (kRedBlock threads) sums of n values per thread, each added as
// block_sum adds one (wave butterfly, then the waves in order); the results
// are valid in thread 0.
template <int n>
__device__ __forceinline__ void block_sum_n(double (&v)[n]) {
    __shared__ double sh[n][kRedBlock / kWave];
#pragma unroll
    for (int i = 0; i < n; ++i) {
        v[i] = wave_sum(v[i]);
        if (lane_id() == 0) sh[i][wave_id()] = v[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < n; ++i) {
            double r = 0.0;
            for (int w = 0; w < kRedBlock / kWave; ++w) r += sh[i][w];
            v[i] = r;
        }
    }
    __syncthreads();
}

// Exclusive scan of one dd value per thread over the block (thread order);
// also returns the block total in `total` (valid in every thread).
__device__ __forceinline__ dd block_dd_exclusive_scan(dd v, dd& total) {
    __shared__ double wh[kRedBlock / kWave], wl[kRedBlock / kWave];
    const int lane = lane_id();
    dd inc = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const dd up{__shfl_up(inc.hi, o, kWave), __shfl_up(inc.lo, o, kWave)};
        if (lane >= o) inc = dd_add(up, inc);
    }
    if (lane == kWave - 1) {
        wh[wave_id()] = inc.hi;
        wl[wave_id()] = inc.lo;
    }
    dd excl{__shfl_up(inc.hi, 1, kWave), __shfl_up(inc.lo, 1, kWave)};
    if (lane == 0) excl = dd_zero();
    __syncthreads();
    dd off = dd_zero();
    for (int w = 0; w < wave_id(); ++w) off = dd_add(off, dd{wh[w], wl[w]});
    dd tot = dd_zero();
    for (int w = 0; w < kRedBlock / kWave; ++w) tot = dd_add(tot, dd{wh[w], wl[w]});
    total = tot;
    __syncthreads();
    return dd_add(off, excl);
}

}  // namespace smc
