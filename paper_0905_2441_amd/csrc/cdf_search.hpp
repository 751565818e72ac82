// Search of the correctly rounded CDF kept as within-chunk prefixes
// (cdf_hi/cdf_lo, each rounded once from a double-double scan of its chunk)
// plus per-chunk double-double totals: the pieces of systematic, stratified and
// multinomial resampling shared by the standalone search-and-gather pass and
// the particle filter's fused propagation.
#pragma once
#include "internal.hpp"
#include "dd.hpp"
#include "philox.hpp"
#include "reduce.hpp"

namespace smc {

// Chunk offsets into LDS offh/offl [kMaxChunks]: the exclusive double-double
// scan of the chunk totals [2 * nchunks] (hi, lo), formed by every thread of a
// kRedBlock-thread block (cooperative; ends with a barrier).
__device__ __forceinline__ void block_cdf_offsets(const double* chunk_tot, int nchunks,
                                                  double* offh, double* offl) {
    constexpr int per = kMaxChunks / kRedBlock;
    const int c0 = threadIdx.x * per;
    dd loc[per];
    dd run = dd_zero();
#pragma unroll
    for (int q = 0; q < per; ++q) {
        loc[q] = run;
        if (c0 + q < nchunks) run = dd_add(run, dd{chunk_tot[2 * (c0 + q)], chunk_tot[2 * (c0 + q) + 1]});
    }
    dd total;
    const dd lead = block_dd_exclusive_scan(run, total);
#pragma unroll
    for (int q = 0; q < per; ++q) {
        const dd o = dd_add(lead, loc[q]);
        offh[c0 + q] = o.hi;
        offl[c0 + q] = o.lo;
    }
    __syncthreads();
}

// idx = min{j : U < C_j}, or the first j with C_j = C_{N-1} when U is not below
// it; cdf(j) returns C_j (non-decreasing in j).
template <class Cdf>
__device__ __forceinline__ int cdf_search_fn(double U, int N, Cdf cdf) {
    const double clast = cdf(N - 1);
    int lo = 0, hi = N - 1;
    if (U < clast) {
        while (lo < hi) {
            const int mid = lo + ((hi - lo) >> 1);
            if (U < cdf(mid)) hi = mid;
            else lo = mid + 1;
        }
    } else {
        while (lo < hi) {
            const int mid = lo + ((hi - lo) >> 1);
            if (cdf(mid) >= clast) hi = mid;
            else lo = mid + 1;
        }
    }
    return lo;
}

// The same idx for the points of a whole wave whose valid lanes hold
// non-decreasing points in lane order (systematic and stratified resampling,
// one point per particle, particles consecutive along the lanes). Every lane
// of the wave must call it (invalid lanes get an unspecified result).
// idx(U) is non-decreasing in U, so the ancestors a and b of the wave's first
// and last points bound every lane's. Those two come from one 32-ary search
// each, run together by the two half-waves (each level probes 32 positions at
// once and shrinks the range 32-fold: four levels at N = 2^20, five at 2^24,
// where a lane's own binary search takes 20 and 24 dependent probes); each
// lane then searches only the window [a, b]. The result equals
// cdf_search_fn's for every valid lane.
template <class Cdf>
__device__ __forceinline__ int cdf_search_sorted_wave_fn(double U, bool valid, int N, Cdf cdf) {
    const int lane = threadIdx.x & 63;
    const double clast = cdf(N - 1);
    // pred(u, C_j) is monotone in j and true at N - 1; the answer is the first
    // j where it holds
    auto pred = [&](double u, double c) -> bool { return u < clast ? (u < c) : (c >= clast); };
    // the wave's first and last valid points (lane order = point order)
    const unsigned long long vm = __ballot(valid);
    if (vm == 0ull) return 0;
    const int first = __ffsll(static_cast<long long>(vm)) - 1;
    const int last = 63 - __clzll(static_cast<long long>(vm));
    const double u_first = __shfl(U, first, 64);
    const double u_last = __shfl(U, last, 64);
    const int half = lane >> 5;
    const int hl = lane & 31;
    const double us = half ? u_last : u_first;
    int lo = 0, hi = N - 1;                 // the answer lies in [lo, hi]
    while (__any(hi > lo)) {
        const int len = hi - lo + 1;
        const int step = (len + 31) >> 5;
        int q = lo + (hl + 1) * step - 1;
        q = q < hi ? q : hi;
        const unsigned long long m = __ballot(pred(us, cdf(q)));
        const unsigned mh = static_cast<unsigned>(half ? (m >> 32) : (m & 0xffffffffull));
        const int f = __ffs(mh) - 1;        // the probe at hi is always true
        const int nlo = lo + f * step;
        const int nhi = lo + (f + 1) * step - 1;
        lo = nlo;
        hi = nhi < hi ? nhi : hi;
    }
    int l = __shfl(lo, 0, 64);
    int h = __shfl(lo, 32, 64);
    if (valid) {
        while (l < h) {
            const int mid = l + ((h - l) >> 1);
            if (pred(U, cdf(mid))) h = mid;
            else l = mid + 1;
        }
    }
    return l;
}

// The searches over a CDF kept as within-chunk prefixes (cdf_hi, cdf_lo) plus
// chunk offsets (offh, offl: LDS or global), C_j = offset + prefix rounded once.
__device__ __forceinline__ int cdf_search(double U, int N, int chunk, const double* cdf_hi,
                                          const double* cdf_lo, const double* offh,
                                          const double* offl) {
    return cdf_search_fn(U, N, [&](int j) -> double {
        const int b = j / chunk;
        return dd_add(dd{offh[b], offl[b]}, dd{cdf_hi[j], cdf_lo[j]}).hi;
    });
}

__device__ __forceinline__ int cdf_search_sorted_wave(double U, bool valid, int N, int chunk,
                                                      const double* cdf_hi,
                                                      const double* cdf_lo,
                                                      const double* offh,
                                                      const double* offl) {
    return cdf_search_sorted_wave_fn(U, valid, N, [&](int j) -> double {
        const int b = j / chunk;
        return dd_add(dd{offh[b], offl[b]}, dd{cdf_hi[j], cdf_lo[j]}).hi;
    });
}

}  // namespace smc
