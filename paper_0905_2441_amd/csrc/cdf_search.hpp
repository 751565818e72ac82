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
// it, where C_j = chunk offset + within-chunk prefix, rounded once.
__device__ __forceinline__ int cdf_search(double U, int N, int chunk, const double* cdf_hi,
                                          const double* cdf_lo, const double* offh,
                                          const double* offl) {
    auto cdf = [&](int j) -> double {
        const int b = j / chunk;
        return dd_add(dd{offh[b], offl[b]}, dd{cdf_hi[j], cdf_lo[j]}).hi;
    };
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

}  // namespace smc
