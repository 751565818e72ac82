// Ascending in-place sort of FP32 data in device memory (smc_sort_data).
//
// The likelihood of independent data does not depend on their order (a sum
// over data in the Gaussian mixture model), so the data of a 1-D mixture can
// be held in ascending order; the FP32 pivot form of the likelihood then sees
// narrow windows of 64 data (partial_fp32).
//
// A bitonic network in the form where every comparator puts the smaller key at
// the lower index: the first step of each merge stage of size k compares
// positions mirrored about the middle of their k-block (two ascending halves
// then form a bitonic sequence), and the later steps compare i with i + j for
// j = k/4, ..., 1. Because no comparator ever moves a key to a higher index
// than the larger one it holds, positions at or past n can stand for +infinity
// without storage: a comparator whose upper position is at or past n does
// nothing. Stages up to a tile of 4096 keys, and the steps of larger stages
// whose distance is below a tile, run in LDS; the other steps are one launch
// each over all pairs.
//
// Values are compared through integer keys that keep their order, so NaNs
// have a place: -NaN < -inf < ... < -0 < +0 < ... < +inf < +NaN.
#include <limits.h>

#include "internal.hpp"
#include "wave.hpp"

namespace smc {
namespace {

constexpr int kSortThreads = 1024;
constexpr int kSortTile = 4 * kSortThreads;     // keys per workgroup in LDS

// full != 0: sorts each tile of kSortTile data. full == 0: the steps with
// distance below a tile of a merge stage larger than a tile (the same steps
// for every such stage).
__global__ void __launch_bounds__(kSortThreads)
k_sort_tile(float* __restrict__ y, int64_t n, int full) {
    __shared__ int key[kSortTile];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
    for (int e = threadIdx.x; e < kSortTile; e += kSortThreads) {
        const int64_t i = base + e;
        key[e] = i < n ? float_order_key(y[i]) : INT_MAX;     // past n: +infinity
    }
    __syncthreads();
    auto exchange = [&](int i, int l) {
        const int a = key[i], b = key[l];
        if (a > b) {
            key[i] = b;
            key[l] = a;
        }
    };
    auto steps_below = [&](int j0) {
        for (int j = j0; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < kSortTile / 2; t += kSortThreads) {
                const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
                exchange(i, i + j);
            }
            __syncthreads();
        }
    };
    if (full != 0) {
        for (int k = 2; k <= kSortTile; k <<= 1) {
            const int h = k >> 1;
            for (int t = threadIdx.x; t < kSortTile / 2; t += kSortThreads) {
                const int blk = (t / h) * k, o = t % h;
                exchange(blk + o, blk + k - 1 - o);
            }
            __syncthreads();
            steps_below(k >> 2);
        }
    } else {
        steps_below(kSortTile / 2);
    }
    for (int e = threadIdx.x; e < kSortTile; e += kSortThreads) {
        const int64_t i = base + e;
        if (i < n) y[i] = float_of_order_key(key[e]);
    }
}

// One step of a merge stage of size k (> kSortTile) over all pairs: mirrored
// positions of each k-block (mirror != 0) or i against i + j.
__global__ void __launch_bounds__(256)
k_sort_step(float* __restrict__ y, int64_t n, int64_t k, int64_t j, int mirror) {
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    int64_t i, l;
    if (mirror != 0) {
        const int64_t h = k >> 1, blk = (t / h) * k, o = t % h;
        i = blk + o;
        l = blk + k - 1 - o;
    } else {
        i = ((t & ~(j - 1)) << 1) | (t & (j - 1));
        l = i + j;
    }
    if (l >= n) return;                  // the upper position stands for +infinity
    const float a = y[i], b = y[l];
    if (float_order_key(a) > float_order_key(b)) {
        y[i] = b;
        y[l] = a;
    }
}

}  // namespace

hipError_t launch_sort_data(float* y, int64_t n, hipStream_t s) {
    if (n < 2) return hipSuccess;
    int64_t np = kSortTile;              // padded length: a power of two >= n
    while (np < n) np <<= 1;
    const unsigned tiles = static_cast<unsigned>((n + kSortTile - 1) / kSortTile);
    hipLaunchKernelGGL(k_sort_tile, dim3(tiles), dim3(kSortThreads), 0, s, y, n, 1);
    hipError_t e = hipGetLastError();
    const unsigned step_blocks = static_cast<unsigned>((np / 2 + 255) / 256);
    for (int64_t k = 2 * kSortTile; e == hipSuccess && k <= np; k <<= 1) {
        hipLaunchKernelGGL(k_sort_step, dim3(step_blocks), dim3(256), 0, s, y, n, k,
                           static_cast<int64_t>(0), 1);
        for (int64_t j = k >> 2; j >= kSortTile; j >>= 1)
            hipLaunchKernelGGL(k_sort_step, dim3(step_blocks), dim3(256), 0, s, y, n, k, j, 0);
        hipLaunchKernelGGL(k_sort_tile, dim3(tiles), dim3(kSortThreads), 0, s, y, n, 0);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace smc
