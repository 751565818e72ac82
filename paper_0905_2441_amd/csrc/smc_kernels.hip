// Weight, resampling and exchange kernels (FP64) for gfx950.
//
// Reweight and ESS are HBM-bound streaming passes; their grid-wide reductions
// use the "last block finishes" pattern: every block writes a partial, fences,
// takes a ticket, and the block that takes the last ticket combines all
// partials in block order (so results are bit-reproducible) and resets the
// ticket. Device-scope fences make the partials visible across the eight XCDs,
// whose L2 caches are not coherent with each other.
//
// Systematic resampling builds the correctly rounded empirical CDF of the
// weights with a double-double scan in three phases (block totals; per-block
// scan with the block's offset; search and gather). Every phase can be
// predicated on a device-side ESS test, so a tempering step never returns to
// the host.
#include "internal.hpp"
#include "philox.hpp"
#include "wave.hpp"

namespace smc {
namespace {

__device__ __forceinline__ bool take_last_ticket(unsigned* ticket) {
    __shared__ bool last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = (atomicAdd(ticket, 1u) == gridDim.x - 1);
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// Block (kRedBlock threads) reductions; the result is valid in thread 0.
__device__ LseAcc block_lse(LseAcc v) {
    __shared__ LsePair sh[kRedBlock / kWave];
    v = wave_lse(v);
    if (lane_id() == 0) sh[wave_id()] = LsePair{v.m, v.s};
    __syncthreads();
    LseAcc r = lse_empty();
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedBlock / kWave; ++w) r = lse_merge(r, LseAcc{sh[w].m, sh[w].s});
    __syncthreads();
    return r;
}

__device__ double block_sum(double v) {
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

__device__ dd block_dd_sum(dd v) {
    __shared__ double shh[kRedBlock / kWave], shl[kRedBlock / kWave];
    v = wave_sum(v);
    if (lane_id() == 0) {
        shh[wave_id()] = v.hi;
        shl[wave_id()] = v.lo;
    }
    __syncthreads();
    dd r = dd_zero();
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedBlock / kWave; ++w) r = dd_add(r, dd{shh[w], shl[w]});
    __syncthreads();
    return r;
}

// ---------------------------------------------------------------- reweight

__global__ void __launch_bounds__(kRedBlock)
k_reweight_a(double* __restrict__ logw, const double* __restrict__ l, int N, StepSrc src,
             Scratch sc, double* logZ) {
    double dbeta = src.dbeta_host;
    if (src.beta_dev) {
        const int t = step_index(src);
        dbeta = src.beta_dev[t] - src.beta_dev[t - 1];
    }
    LseAcc old_acc = lse_empty(), new_acc = lse_empty();
    bool bad = false;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        const double lo = logw[p];
        const double ln = lo + dbeta * l[p];
        logw[p] = ln;
        bad = bad || (ln != ln) || (ln == INFINITY);
        old_acc = lse_push(old_acc, lo);
        new_acc = lse_push(new_acc, ln);
    }
    if (bad) atomicOr(sc.status, kStatusNaN);
    const LseAcc bo = block_lse(old_acc);
    const LseAcc bn = block_lse(new_acc);
    if (threadIdx.x == 0) {
        sc.part_old[blockIdx.x] = LsePair{bo.m, bo.s};
        sc.part_new[blockIdx.x] = LsePair{bn.m, bn.s};
    }
    if (!take_last_ticket(&sc.tickets[0])) return;
    LseAcc o = lse_empty(), nw = lse_empty();
    for (int b = threadIdx.x; b < static_cast<int>(gridDim.x); b += blockDim.x) {
        const LsePair po = sc.part_old[b], pn = sc.part_new[b];
        o = lse_merge(o, LseAcc{po.m, po.s});
        nw = lse_merge(nw, LseAcc{pn.m, pn.s});
    }
    o = block_lse(o);
    nw = block_lse(nw);
    if (threadIdx.x == 0) {
        StepState* st = sc.state;
        st->M = nw.m;
        st->S = nw.s;
        st->lse_old = lse_value(o);
        st->lse_new = lse_value(nw);
        if (nw.m == -INFINITY) atomicOr(sc.status, kStatusAllZeroWeight);
        if (logZ) *logZ += st->lse_new - st->lse_old;
        sc.tickets[0] = 0u;
    }
}

__global__ void __launch_bounds__(kRedBlock)
k_reweight_b(const double* __restrict__ logw, int N, double* __restrict__ W, Scratch sc,
             double* ess_out, double ess_frac, double* resample_count) {
    const double M = sc.state->M;
    const double S = sc.state->S;
    double sq = 0.0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        const double w = exp(logw[p] - M) / S;
        W[p] = w;
        sq += w * w;
    }
    const double bs = block_sum(sq);
    if (threadIdx.x == 0) sc.part_sq[blockIdx.x] = bs;
    if (!take_last_ticket(&sc.tickets[1])) return;
    double acc = 0.0;
    for (int b = threadIdx.x; b < static_cast<int>(gridDim.x); b += blockDim.x) acc += sc.part_sq[b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) {
        const double e = 1.0 / acc;
        sc.state->ess = e;
        const int fire = (ess_frac > 0.0) && (e < ess_frac * static_cast<double>(N));
        sc.state->resampled = fire;
        if (ess_out) *ess_out = e;
        if (resample_count && fire) *resample_count += 1.0;
        sc.tickets[1] = 0u;
    }
}

__global__ void __launch_bounds__(kRedBlock)
k_ess(const double* __restrict__ W, int N, Scratch sc, double* ess_out) {
    double sq = 0.0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        const double w = W[p];
        sq += w * w;
    }
    const double bs = block_sum(sq);
    if (threadIdx.x == 0) sc.part_sq[blockIdx.x] = bs;
    if (!take_last_ticket(&sc.tickets[2])) return;
    double acc = 0.0;
    for (int b = threadIdx.x; b < static_cast<int>(gridDim.x); b += blockDim.x) acc += sc.part_sq[b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) {
        *ess_out = 1.0 / acc;
        sc.tickets[2] = 0u;
    }
}

// ---------------------------------------------------------------- resampling

struct ResamplePred {
    const double* ess;           // fire iff *ess < thresh (nullable)
    double thresh;
    const StepState* state;      // fire iff state->resampled (nullable)
};

__device__ __forceinline__ bool should_fire(const ResamplePred& pr) {
    if (pr.state) return pr.state->resampled != 0;
    if (pr.ess) return *pr.ess < pr.thresh;
    return true;
}

// Phase 1: double-double total of each chunk of kScanChunk weights.
__global__ void __launch_bounds__(kRedBlock)
k_cdf_totals(const double* __restrict__ W, int N, Scratch sc, ResamplePred pred) {
    if (!should_fire(pred)) return;
    const int base = blockIdx.x * kScanChunk + threadIdx.x * kScanPerThread;
    dd acc = dd_zero();
#pragma unroll
    for (int e = 0; e < kScanPerThread; ++e)
        if (base + e < N) acc = dd_add(acc, W[base + e]);
    acc = block_dd_sum(acc);
    if (threadIdx.x == 0) {
        sc.dd_part[2 * blockIdx.x] = acc.hi;
        sc.dd_part[2 * blockIdx.x + 1] = acc.lo;
    }
}

// Phase 2: per-chunk inclusive scan plus the sum of all earlier chunks; each
// prefix is rounded once from double-double to double.
__global__ void __launch_bounds__(kRedBlock)
k_cdf_scan(const double* __restrict__ W, int N, Scratch sc, ResamplePred pred) {
    if (!should_fire(pred)) return;
    __shared__ double wh[kRedBlock / kWave], wl[kRedBlock / kWave];
    __shared__ double oh, ol;
    // offset = sum of the totals of chunks 0..b-1, in chunk order per thread
    dd off = dd_zero();
    for (int b = threadIdx.x; b < static_cast<int>(blockIdx.x); b += blockDim.x)
        off = dd_add(off, dd{sc.dd_part[2 * b], sc.dd_part[2 * b + 1]});
    off = block_dd_sum(off);
    if (threadIdx.x == 0) {
        oh = off.hi;
        ol = off.lo;
    }
    // this thread's inclusive prefixes
    const int base = blockIdx.x * kScanChunk + threadIdx.x * kScanPerThread;
    dd pre[kScanPerThread];
    dd run = dd_zero();
#pragma unroll
    for (int e = 0; e < kScanPerThread; ++e) {
        if (base + e < N) run = dd_add(run, W[base + e]);
        pre[e] = run;
    }
    // inclusive scan of thread totals within the wave (earlier + later)
    dd inc = run;
    const int lane = lane_id();
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
    dd wave_off{oh, ol};
    for (int w = 0; w < wave_id(); ++w) wave_off = dd_add(wave_off, dd{wh[w], wl[w]});
    const dd lead = dd_add(wave_off, excl);
#pragma unroll
    for (int e = 0; e < kScanPerThread; ++e)
        if (base + e < N) sc.cdf[base + e] = dd_add(lead, pre[e]).hi;
}

// Phase 3: U_i = (i + u)/N, idx_i = min{j : U_i < C_j} (or the first j with
// C_j = C_{N-1} when U_i >= C_{N-1}), then gather.
__global__ void __launch_bounds__(kRedBlock)
k_search_gather(int N, Scratch sc, ResamplePred pred, uint64_t seed, StepSrc src,
                const double* u_override, int32_t* idx_out, const double* __restrict__ theta_in,
                double* __restrict__ theta_out, int kd, const double* __restrict__ l_in,
                double* __restrict__ l_out, double* logw, double* W_reset,
                int copy_when_skipped) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    if (!should_fire(pred)) {
        if (!copy_when_skipped) return;
        if (idx_out) idx_out[i] = i;
        if (theta_in && theta_out)
            for (int c = 0; c < kd; ++c)
                theta_out[static_cast<size_t>(c) * N + i] = theta_in[static_cast<size_t>(c) * N + i];
        if (l_in && l_out) l_out[i] = l_in[i];
        return;
    }
    const double* C = sc.cdf;
    double u;
    if (u_override) {
        u = *u_override;
    } else {
        const uint32_t step = static_cast<uint32_t>(step_index(src));
        u = u01_left_closed(draw(seed, 0, 0, step, kResamp, 0).w0);
    }
    const double U = (static_cast<double>(i) + u) / static_cast<double>(N);
    const double clast = C[N - 1];
    int lo = 0, hi = N - 1;
    if (U < clast) {
        while (lo < hi) {
            const int mid = lo + ((hi - lo) >> 1);
            if (U < C[mid]) hi = mid;
            else lo = mid + 1;
        }
    } else {
        while (lo < hi) {
            const int mid = lo + ((hi - lo) >> 1);
            if (C[mid] >= clast) hi = mid;
            else lo = mid + 1;
        }
    }
    const int j = lo;
    if (idx_out) idx_out[i] = j;
    if (theta_in && theta_out)
        for (int c = 0; c < kd; ++c)
            theta_out[static_cast<size_t>(c) * N + i] = theta_in[static_cast<size_t>(c) * N + j];
    if (l_in && l_out) l_out[i] = l_in[j];
    if (logw) logw[i] = 0.0;
    if (W_reset) W_reset[i] = 1.0 / static_cast<double>(N);
}

// ---------------------------------------------------------------- exchange

__global__ void __launch_bounds__(kRedBlock)
k_exchange(double* __restrict__ theta, double* __restrict__ l, const double* __restrict__ beta,
           int M, int kd, int parity_mode, int parity_host, int wrap, uint64_t seed,
           StepSrc src, unsigned* n_swap) {
    const uint32_t it = static_cast<uint32_t>(step_index(src));
    int parity;
    if (parity_mode == 0) parity = static_cast<int>(it & 1u);
    else if (parity_mode == 1) parity = static_cast<int>(draw(seed, 0, 0, it, kParity, 0).w0 >> 31);
    else parity = parity_host & 1;
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const int regular = (M - parity) / 2;        // pairs (parity + 2q, parity + 2q + 1)
    int a, b;
    if (q < regular) {
        a = parity + 2 * q;
        b = a + 1;
    } else if (q == regular && wrap && parity == 1 && M >= 2 && (M % 2) == 0) {
        a = M - 1;
        b = 0;
    } else {
        return;
    }
    const double la = (beta[a] - beta[b]) * (l[b] - l[a]);
    const double u = u01_open(draw(seed, static_cast<uint32_t>(a), 0, it, kExch, 0).w0);
    if (la >= 0.0 || log(u) < la) {
        const double t = l[a];
        l[a] = l[b];
        l[b] = t;
        for (int c = 0; c < kd; ++c) {
            double* r = theta + static_cast<size_t>(c) * M;
            const double x = r[a];
            r[a] = r[b];
            r[b] = x;
        }
        if (n_swap) atomicAdd(n_swap, 1u);
    }
}

// After a step whose moves were all skipped: adopt the resampled population.
__global__ void __launch_bounds__(kRedBlock)
k_copy_back(double* __restrict__ theta, double* __restrict__ l, int N, int kd, Scratch sc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N || sc.state->resampled == 0) return;
    for (int c = 0; c < kd; ++c)
        theta[static_cast<size_t>(c) * N + i] = sc.theta_tmp[static_cast<size_t>(c) * N + i];
    l[i] = sc.l_tmp[i];
}

__global__ void k_counter_inc(int* c) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *c += 1;
}

__global__ void k_rng_words(uint64_t seed, int64_t count, uint32_t block, uint32_t step,
                            uint32_t purpose, uint32_t move, uint32_t* out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const Words4 w = draw(seed, static_cast<uint32_t>(i), block, step, purpose, move);
    out[4 * i + 0] = w.w0;
    out[4 * i + 1] = w.w1;
    out[4 * i + 2] = w.w2;
    out[4 * i + 3] = w.w3;
}

__global__ void k_rng_normals(uint64_t seed, int64_t count, int per_index, uint32_t step,
                              uint32_t purpose, uint32_t move, double* out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    for (int b = 0; 4 * b < per_index; ++b) {
        const Words4 w = draw(seed, static_cast<uint32_t>(i), b, step, purpose, move);
        double z[4];
        box_muller(w.w0, w.w1, z[0], z[1]);
        box_muller(w.w2, w.w3, z[2], z[3]);
        for (int q = 0; q < 4 && 4 * b + q < per_index; ++q) out[(4 * b + q) * count + i] = z[q];
    }
}

int red_grid(int64_t N) {
    int64_t g = (N + kRedBlock - 1) / kRedBlock;
    if (g > kMaxRedBlocks) g = kMaxRedBlocks;
    if (g < 1) g = 1;
    return static_cast<int>(g);
}

}  // namespace

hipError_t launch_reweight(const Scratch& sc, double* logw, const double* l, int64_t N,
                           StepSrc src, double* W, double* logZ, double* ess,
                           double ess_threshold_frac, hipStream_t s) {
    const int g = red_grid(N);
    hipLaunchKernelGGL(k_reweight_a, dim3(g), dim3(kRedBlock), 0, s, logw, l,
                       static_cast<int>(N), src, sc, logZ);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || W == nullptr) return e;
    hipLaunchKernelGGL(k_reweight_b, dim3(g), dim3(kRedBlock), 0, s, logw,
                       static_cast<int>(N), W, sc, ess, ess_threshold_frac,
                       static_cast<double*>(nullptr));
    return hipGetLastError();
}

hipError_t launch_reweight_step(const Scratch& sc, double* logw, const double* l, int64_t N,
                                StepSrc src, double* W, double* stats, double ess_frac,
                                hipStream_t s) {
    const int g = red_grid(N);
    hipLaunchKernelGGL(k_reweight_a, dim3(g), dim3(kRedBlock), 0, s, logw, l,
                       static_cast<int>(N), src, sc, stats);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reweight_b, dim3(g), dim3(kRedBlock), 0, s, logw,
                       static_cast<int>(N), W, sc, stats + 1, ess_frac, stats + 2);
    return hipGetLastError();
}

hipError_t launch_ess(const Scratch& sc, const double* W, int64_t N, double* ess,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_ess, dim3(red_grid(N)), dim3(kRedBlock), 0, s, W,
                       static_cast<int>(N), sc, ess);
    return hipGetLastError();
}

static hipError_t launch_resample_impl(const Scratch& sc, const double* W, int64_t N,
                                       uint64_t seed, StepSrc src, const double* u_override,
                                       ResamplePred pred, int32_t* idx, const double* theta_in,
                                       double* theta_out, int32_t kd, const double* l_in,
                                       double* l_out, double* logw, double* W_reset,
                                       int copy_when_skipped, hipStream_t s) {
    const int chunks = static_cast<int>((N + kScanChunk - 1) / kScanChunk);
    hipLaunchKernelGGL(k_cdf_totals, dim3(chunks), dim3(kRedBlock), 0, s, W,
                       static_cast<int>(N), sc, pred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cdf_scan, dim3(chunks), dim3(kRedBlock), 0, s, W,
                       static_cast<int>(N), sc, pred);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int g = static_cast<int>((N + kRedBlock - 1) / kRedBlock);
    hipLaunchKernelGGL(k_search_gather, dim3(g), dim3(kRedBlock), 0, s, static_cast<int>(N),
                       sc, pred, seed, src, u_override, idx, theta_in, theta_out, kd, l_in,
                       l_out, logw, W_reset, copy_when_skipped);
    return hipGetLastError();
}

hipError_t launch_resample(const Scratch& sc, const double* W, int64_t N, uint64_t seed,
                           StepSrc src, const double* u_override, const double* ess,
                           double ess_threshold, const StepState* pred_state,
                           int32_t* idx, const double* theta_in, double* theta_out,
                           int32_t kd, const double* l_in, double* l_out, double* logw,
                           hipStream_t s) {
    ResamplePred pred{ess, ess_threshold, pred_state};
    const int copy = pred_state ? 0 : 1;
    double* W_reset = pred_state ? const_cast<double*>(W) : nullptr;
    return launch_resample_impl(sc, W, N, seed, src, u_override, pred, idx, theta_in,
                                theta_out, kd, l_in, l_out, logw, W_reset, copy, s);
}

hipError_t launch_exchange(double* theta, double* l, const double* beta, int64_t M,
                           int32_t kd, int parity_mode, int parity_host, int wrap,
                           uint64_t seed, StepSrc src, unsigned* n_swap, hipStream_t s) {
    const int64_t pairs = M / 2 + 1;
    const int g = static_cast<int>((pairs + kRedBlock - 1) / kRedBlock);
    hipLaunchKernelGGL(k_exchange, dim3(g), dim3(kRedBlock), 0, s, theta, l, beta,
                       static_cast<int>(M), kd, parity_mode, parity_host, wrap, seed, src,
                       n_swap);
    return hipGetLastError();
}

hipError_t launch_copy_back(const Scratch& sc, double* theta, double* l, int64_t N, int kd,
                            hipStream_t s) {
    const int g = static_cast<int>((N + kRedBlock - 1) / kRedBlock);
    hipLaunchKernelGGL(k_copy_back, dim3(g), dim3(kRedBlock), 0, s, theta, l,
                       static_cast<int>(N), kd, sc);
    return hipGetLastError();
}

hipError_t launch_counter_inc(int* counter, hipStream_t s) {
    hipLaunchKernelGGL(k_counter_inc, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

hipError_t launch_rng_words(uint64_t seed, int64_t count, uint32_t block, uint32_t step,
                            uint32_t purpose, uint32_t move, uint32_t* out, hipStream_t s) {
    const int g = static_cast<int>((count + 255) / 256);
    hipLaunchKernelGGL(k_rng_words, dim3(g), dim3(256), 0, s, seed, count, block, step,
                       purpose, move, out);
    return hipGetLastError();
}

hipError_t launch_rng_normals(uint64_t seed, int64_t count, int32_t per_index, uint32_t step,
                              uint32_t purpose, uint32_t move, double* out, hipStream_t s) {
    const int g = static_cast<int>((count + 255) / 256);
    hipLaunchKernelGGL(k_rng_normals, dim3(g), dim3(256), 0, s, seed, count, per_index, step,
                       purpose, move, out);
    return hipGetLastError();
}

}  // namespace smc
