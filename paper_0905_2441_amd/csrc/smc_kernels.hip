// Weight, resampling and exchange kernels (FP64) for gfx950.
//
// Grid-wide reductions never communicate between workgroups inside a kernel:
// a streaming kernel writes one partial per workgroup and a one-workgroup
// kernel combines them in block order. On MI355X a device-scope fence inside a
// kernel writes back and invalidates the L2 of the issuing XCD, so per-block
// "last block finishes" tickets cost far more than the kernel boundary they
// would save. Combining in a fixed order keeps every result bit-reproducible.
//
// Reweight (SMC Sampler subsection: incremental weight L^dbeta) is one pass
// over (logw, l) that keeps three running sums per thread: the log-sum-exp of
// the old log-weights, and of the new ones together with the sum of their
// squares, so the normalising constant, the log-evidence increment and the ESS
// 1/sum W^2 = S1^2/S2 all come out of the same pass.
//
// Systematic resampling (Sequential Monte Carlo subsection: the empirical CDF
// of the weights, sampled N times) builds the CDF with a double-double scan:
// each chunk's workgroup stores within-chunk inclusive prefixes and the chunk
// total; the search kernel forms the chunk offsets once per workgroup in LDS
// and rounds offset + prefix once, so every C_j is the correctly rounded
// prefix sum (up to double-double error, about 2^-104 relative). Both kernels
// can be predicated on the device-side ESS test.
#include "internal.hpp"
#include "philox.hpp"
#include "exchange.hpp"
#include "reduce.hpp"
#include "cdf_search.hpp"

namespace smc {
namespace {

constexpr int kMaxMomK = 4;    // state components of a particle filter's step moments

// ---------------------------------------------------------------- reweight

__global__ void __launch_bounds__(kRedBlock)
k_reweight_partial(double* __restrict__ logw, const double* __restrict__ l, int N, StepSrc src,
                   Scratch sc) {
    double dbeta = src.dbeta_host;
    if (src.beta_dev) {
        const int t = step_index(src);
        dbeta = src.beta_dev[t] - src.beta_dev[t - 1];
    }
    Lse3 o = lse3_empty(), nw = lse3_empty();
    bool bad = false;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        const double lo = logw[p];
        const double ln = lo + dbeta * l[p];
        logw[p] = ln;
        bad = bad || (ln != ln) || (ln == INFINITY);
        o = lse3_push(o, lo);
        nw = lse3_push(nw, ln);
    }
    if (bad) atomicOr(sc.status, kStatusNaN);
    o = block_lse3(o);
    nw = block_lse3(nw);
    if (threadIdx.x == 0) sc.rw_part[blockIdx.x] = RwPartial{o.m, o.s1, nw.m, nw.s1, nw.s2, 0.0};
}

__global__ void __launch_bounds__(kRedBlock)
k_reweight_final(int parts, int N, StepSrc src, int* t_advance, Scratch sc, double* logZ,
                 double* ess_out, double ess_frac, double* resample_count) {
    Lse3 o = lse3_empty(), nw = lse3_empty();
    for (int b = threadIdx.x; b < parts; b += blockDim.x) {
        const RwPartial q = sc.rw_part[b];
        o = lse3_merge(o, Lse3{q.mo, q.so, 0.0});
        nw = lse3_merge(nw, Lse3{q.mn, q.s1, q.s2});
    }
    o = block_lse3(o);
    nw = block_lse3(nw);
    if (threadIdx.x != 0) return;
    StepState* st = sc.state;
    st->M = nw.m;
    st->S = nw.s1;
    st->S2 = nw.s2;
    st->lse_old = (o.m == -INFINITY) ? -INFINITY : o.m + log(o.s1);
    st->lse_new = (nw.m == -INFINITY) ? -INFINITY : nw.m + log(nw.s1);
    const double e = (nw.s1 * nw.s1) / nw.s2;
    st->ess = e;
    const int fire = (ess_frac > 0.0) && (e < ess_frac * static_cast<double>(N));
    st->resampled = fire;
    if (nw.m == -INFINITY || !(e == e)) atomicOr(sc.status, kStatusAllZeroWeight);
    if (logZ) *logZ += st->lse_new - st->lse_old;
    if (ess_out) *ess_out = e;
    if (resample_count && fire) *resample_count += 1.0;
    if (t_advance) {
        const int t = step_index(src);
        st->t = t;
        *t_advance = t + 1;
    }
}

__global__ void __launch_bounds__(kRedBlock)
k_weights(const double* __restrict__ logw, int N, Scratch sc, double* __restrict__ W) {
    const double M = sc.state->M, S = sc.state->S;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x)
        W[p] = exp(logw[p] - M) / S;
}

__global__ void __launch_bounds__(kRedBlock)
k_sq_partial(const double* __restrict__ W, int N, Scratch sc) {
    double sq = 0.0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        const double w = W[p];
        sq += w * w;
    }
    const double bs = block_sum(sq);
    if (threadIdx.x == 0) sc.sq_part[blockIdx.x] = bs;
}

__global__ void __launch_bounds__(kRedBlock)
k_sq_final(int parts, Scratch sc, double* ess_out) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < parts; b += blockDim.x) acc += sc.sq_part[b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) *ess_out = 1.0 / acc;
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

__device__ __forceinline__ double weight_at(const WeightSrc& w, int j) {
    if (w.W) return w.W[j];
    return exp(w.logw[j] - w.state->M) / w.state->S;
}

// Within-chunk inclusive prefixes (double-double) of chunk b and its total.
// Chunk b covers [b*chunk, min(N, (b+1)*chunk)), processed kScanChunk at a time.
template <class WeightAt>
__device__ __forceinline__ void scan_chunk(int b, int N, int chunk, const Scratch& sc,
                                           WeightAt weight) {
    const int begin = b * chunk;
    const int end = min(N, begin + chunk);
    dd carry = dd_zero();
    for (int piece = begin; piece < end; piece += kScanChunk) {
        const int base = piece + threadIdx.x * kScanPerThread;
        dd pre[kScanPerThread];
        dd run = dd_zero();
#pragma unroll
        for (int e = 0; e < kScanPerThread; ++e) {
            if (base + e < end) run = dd_add(run, weight(base + e));
            pre[e] = run;
        }
        dd total;
        const dd excl = block_dd_exclusive_scan(run, total);
        const dd lead = dd_add(carry, excl);
#pragma unroll
        for (int e = 0; e < kScanPerThread; ++e) {
            if (base + e < end) {
                const dd c = dd_add(lead, pre[e]);
                sc.cdf_hi[base + e] = c.hi;
                sc.cdf_lo[base + e] = c.lo;
            }
        }
        carry = dd_add(carry, total);
    }
    if (threadIdx.x == 0) {
        sc.dd_part[2 * b] = carry.hi;
        sc.dd_part[2 * b + 1] = carry.lo;
    }
}

// Phase 1 of standalone resampling: the chunk scans.
__global__ void __launch_bounds__(kRedBlock)
k_cdf_local(WeightSrc w, int N, int chunk, Scratch sc, ResamplePred pred) {
    if (!should_fire(pred)) return;
    scan_chunk(blockIdx.x, N, chunk, sc, [&](int j) { return weight_at(w, j); });
}

// Middle of a fused tempering step: every workgroup combines the reweight
// partials in block order (so all reach the same M, S1, S2 and decision);
// workgroup 0 publishes the step state, the statistics and the next step index;
// when the ESS test fires, workgroup b scans CDF chunk b of the weights
// exp(logw - M) / S1. With `mom` (a particle filter's per-workgroup sums of
// w x and w x^2 over k state components, w = exp(logw - block max), stride
// mom_stride per workgroup), workgroup 0 also writes the step's weighted means
// and standard deviations to moments[(t-1) * 2k ...]. With `chained`, the
// partials are the per-tile ones of the new weights made by the previous move
// of a chain of steps (many more than the reweight pass makes): their maximum
// is formed first so that the loads and exps of different partials do not
// wait on each other, and the old weights' log-sum-exp is taken from the step
// state (the previous step's new one, or log N after its resampling).
__global__ void __launch_bounds__(kRedBlock)
k_step_mid(int parts, int N, int chunk, StepSrc src, int* t_advance, Scratch sc,
           double* stats, double ess_frac, const double* __restrict__ logw,
           const double* __restrict__ mom, int mom_k, int mom_stride,
           double* __restrict__ moments, const RwPartial* __restrict__ part, int chained) {
    __shared__ double sh_M, sh_S;
    __shared__ int sh_fire, sh_t;
    // what thread 0 of workgroup 0 updates at the end (step counter, the
    // previous step's state, the running statistics) is read here, so that
    // these loads overlap the partials' instead of following the combine
    int t_pre = 0, rs_pre = 0;
    double lse_pre = 0.0, z_pre = 0.0, nres_pre = 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        t_pre = step_index(src);
        rs_pre = sc.state->resampled;
        lse_pre = sc.state->lse_new;
        z_pre = stats[0];
        nres_pre = stats[2];
    }
    Lse3 o = lse3_empty(), nw = lse3_empty();
    if (chained) {
        // kU partials per thread per round, their loads issued together
        constexpr int kU = 8;
        double m = -INFINITY;
        for (int b0 = threadIdx.x; b0 < parts; b0 += kU * kRedBlock) {
            double v[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int b = b0 + u * kRedBlock;
                v[u] = b < parts ? part[b].mn : -INFINITY;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) m = fmax(m, v[u]);
        }
        m = block_max(m);
        double a = 0.0, c = 0.0;
        for (int b0 = threadIdx.x; b0 < parts; b0 += kU * kRedBlock) {
            double vm[kU], v1[kU], v2[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int b = b0 + u * kRedBlock;
                vm[u] = b < parts ? part[b].mn : -INFINITY;
                v1[u] = b < parts ? part[b].s1 : 0.0;
                v2[u] = b < parts ? part[b].s2 : 0.0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const double r = vm[u] == -INFINITY ? 0.0 : exp(vm[u] - m);
                a += v1[u] * r;
                c += v2[u] * (r * r);
            }
        }
        nw = Lse3{m, block_sum(a), block_sum(c)};
    } else {
        for (int b = threadIdx.x; b < parts; b += blockDim.x) {
            const RwPartial q = part[b];
            o = lse3_merge(o, Lse3{q.mo, q.so, 0.0});
            nw = lse3_merge(nw, Lse3{q.mn, q.s1, q.s2});
        }
        o = block_lse3(o);
        nw = block_lse3(nw);
    }
    if (threadIdx.x == 0) {
        const double e = (nw.s1 * nw.s1) / nw.s2;
        const int fire = (ess_frac > 0.0) && (e < ess_frac * static_cast<double>(N));
        sh_M = nw.m;
        sh_S = nw.s1;
        sh_fire = fire;
        if (blockIdx.x == 0) {
            StepState* st = sc.state;
            const int t = t_pre;
            sh_t = t;
            const double lse_old =
                chained ? (rs_pre ? log(static_cast<double>(N)) : lse_pre)
                        : ((o.m == -INFINITY) ? -INFINITY : o.m + log(o.s1));
            const double lse_new = (nw.m == -INFINITY) ? -INFINITY : nw.m + log(nw.s1);
            st->M = nw.m;
            st->S = nw.s1;
            st->S2 = nw.s2;
            st->lse_old = lse_old;
            st->lse_new = lse_new;
            st->ess = e;
            st->resampled = fire;
            st->t = t;
            if (nw.m == -INFINITY || !(e == e)) atomicOr(sc.status, kStatusAllZeroWeight);
            stats[0] = z_pre + (lse_new - lse_old);
            stats[1] = e;
            if (fire) stats[2] = nres_pre + 1.0;
            *t_advance = t + 1;
        }
    }
    __syncthreads();
    const double M = sh_M, S = sh_S;
    if (mom != nullptr && blockIdx.x == 0) {
        // each workgroup's sums rescaled from its own maximum to M, added in
        // order; all 2 mom_k sums in one pass and one block reduction
        double* out = moments + static_cast<size_t>(sh_t - 1) * 2 * mom_k;
        double acc[2 * kMaxMomK];
#pragma unroll
        for (int c = 0; c < 2 * kMaxMomK; ++c) acc[c] = 0.0;
        for (int q = threadIdx.x; q < parts; q += blockDim.x) {
            const double mb = part[q].mn;
            const double r = (mb == -INFINITY) ? 0.0 : exp(mb - M);
            const double* mq = mom + static_cast<size_t>(q) * mom_stride;
#pragma unroll
            for (int c = 0; c < kMaxMomK; ++c) {
                if (c < mom_k) {
                    acc[c] += mq[c] * r;
                    acc[kMaxMomK + c] += mq[mom_k + c] * r;
                }
            }
        }
        block_sum_n<2 * kMaxMomK>(acc);
        if (threadIdx.x == 0) {
            for (int c = 0; c < mom_k; ++c) {
                const double mean = acc[c] / S;
                const double var = acc[kMaxMomK + c] / S - mean * mean;
                out[c] = mean;
                out[mom_k + c] = sqrt(var > 0.0 ? var : 0.0);
            }
        }
    }
    if (!sh_fire) return;
    scan_chunk(blockIdx.x, N, chunk, sc, [&](int j) { return exp(logw[j] - M) / S; });
}

// Publish the normalised weights of a step that made no move.
__global__ void __launch_bounds__(kRedBlock)
k_publish_w(double* __restrict__ W, const double* __restrict__ logw, int N, Scratch sc) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const StepState* st = sc.state;
    W[i] = st->resampled ? 1.0 / static_cast<double>(N) : exp(logw[i] - st->M) / st->S;
}

// Phase 2: chunk offsets (exclusive scan of the chunk totals, once per block in
// LDS), then the scheme's point U_i, idx_i = min{j : U_i < C_j} (or the first j with
// C_j = C_{N-1} when U_i >= C_{N-1}), then gather.
__global__ void __launch_bounds__(kRedBlock)
k_search_gather(int N, int chunk, int nchunks, Scratch sc, ResamplePred pred, int scheme,
                uint64_t seed, StepSrc src, const double* u_override, int32_t* idx_out,
                const double* __restrict__ theta_in, double* __restrict__ theta_out, int kd,
                const double* __restrict__ l_in, double* __restrict__ l_out, double* logw,
                int copy_when_skipped) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (!should_fire(pred)) {
        if (!copy_when_skipped || i >= N) return;
        if (idx_out) idx_out[i] = i;
        if (theta_in && theta_out)
            for (int c = 0; c < kd; ++c)
                theta_out[static_cast<size_t>(c) * N + i] = theta_in[static_cast<size_t>(c) * N + i];
        if (l_in && l_out) l_out[i] = l_in[i];
        return;
    }
    __shared__ double offh[kMaxChunks], offl[kMaxChunks];
    block_cdf_offsets(sc.dd_part, nchunks, offh, offl);
    if (i >= N) return;
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    double u = 0.0;
    if (scheme == 0)
        u = u_override ? *u_override : u01_left_closed(draw(seed, 0, 0, step, kResamp, 0).w0);
    const double U = resample_point(scheme, seed, step, i, N, u);
    const int j = cdf_search(U, N, chunk, sc.cdf_hi, sc.cdf_lo, offh, offl);
    if (idx_out) idx_out[i] = j;
    if (theta_in && theta_out)
        for (int c = 0; c < kd; ++c)
            theta_out[static_cast<size_t>(c) * N + i] = theta_in[static_cast<size_t>(c) * N + j];
    if (l_in && l_out) l_out[i] = l_in[j];
    if (logw) logw[i] = 0.0;
}

// ---------------------------------------------------------------- exchange

__global__ void __launch_bounds__(kRedBlock)
k_exchange(double* __restrict__ theta, double* __restrict__ l, const double* __restrict__ beta,
           int M, int kd, int parity_mode, int parity_host, int wrap, uint64_t seed,
           StepSrc src, int* t_advance, unsigned* n_swap) {
    const uint32_t it = static_cast<uint32_t>(step_index(src));
    // the iteration index is read from a snapshot, so the caller's counter can
    // be advanced here without racing the other blocks' reads
    if (t_advance != nullptr && blockIdx.x == 0 && threadIdx.x == 0)
        *t_advance = static_cast<int>(it) + 1;
    const int parity = pt_parity(parity_mode, parity_host, seed, it);
    int a, b;
    if (!pt_slot(M, parity, wrap, blockIdx.x * blockDim.x + threadIdx.x, a, b) || b < 0) return;
    if (pt_swap(theta, l, beta, M, kd, a, b, seed, it) && n_swap) atomicAdd(n_swap, 1u);
}

__global__ void k_pt_record(const double* __restrict__ theta, int M, int kd, int chain,
                            const int32_t* it_dev, double* __restrict__ out, int64_t max_iters) {
    const int64_t it = *it_dev;
    const int c = threadIdx.x;
    if (it < 1 || it > max_iters || c >= kd) return;
    out[(it - 1) * kd + c] = theta[static_cast<size_t>(c) * M + chain];
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

// Elements per CDF chunk: a multiple of kScanChunk, so that at most kMaxChunks chunks cover N.
int cdf_chunk(int64_t N) {
    int64_t per = (N + kMaxChunks - 1) / kMaxChunks;
    per = ((per + kScanChunk - 1) / kScanChunk) * kScanChunk;
    if (per < kScanChunk) per = kScanChunk;
    return static_cast<int>(per);
}

}  // namespace

hipError_t launch_reweight(const Scratch& sc, double* logw, const double* l, int64_t N,
                           StepSrc src, int* t_advance, double* logZ, double* ess,
                           double ess_frac, double* resample_count, hipStream_t s) {
    const int g = red_grid(N);
    hipLaunchKernelGGL(k_reweight_partial, dim3(g), dim3(kRedBlock), 0, s, logw, l,
                       static_cast<int>(N), src, sc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reweight_final, dim3(1), dim3(kRedBlock), 0, s, g, static_cast<int>(N),
                       src, t_advance, sc, logZ, ess, ess_frac, resample_count);
    return hipGetLastError();
}

hipError_t launch_reweight_partial(const Scratch& sc, double* logw, const double* l, int64_t N,
                                   StepSrc src, hipStream_t s) {
    hipLaunchKernelGGL(k_reweight_partial, dim3(red_grid(N)), dim3(kRedBlock), 0, s, logw, l,
                       static_cast<int>(N), src, sc);
    return hipGetLastError();
}

hipError_t launch_weights(const Scratch& sc, const double* logw, int64_t N, double* W,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_weights, dim3(red_grid(N)), dim3(kRedBlock), 0, s, logw,
                       static_cast<int>(N), sc, W);
    return hipGetLastError();
}

hipError_t launch_ess(const Scratch& sc, const double* W, int64_t N, double* ess,
                      hipStream_t s) {
    const int g = red_grid(N);
    hipLaunchKernelGGL(k_sq_partial, dim3(g), dim3(kRedBlock), 0, s, W, static_cast<int>(N), sc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sq_final, dim3(1), dim3(kRedBlock), 0, s, g, sc, ess);
    return hipGetLastError();
}

hipError_t launch_resample(const Scratch& sc, WeightSrc w, int64_t N, int scheme, uint64_t seed,
                           StepSrc src, const double* u_override, const double* pred_ess,
                           double ess_threshold, const StepState* pred_state,
                           int32_t* idx, const double* theta_in, double* theta_out,
                           int32_t kd, const double* l_in, double* l_out, double* logw,
                           int copy_when_skipped, hipStream_t s) {
    ResamplePred pred{pred_ess, ess_threshold, pred_state};
    const int chunk = cdf_chunk(N);
    const int nchunks = static_cast<int>((N + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_cdf_local, dim3(nchunks), dim3(kRedBlock), 0, s, w,
                       static_cast<int>(N), chunk, sc, pred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int g = static_cast<int>((N + kRedBlock - 1) / kRedBlock);
    hipLaunchKernelGGL(k_search_gather, dim3(g), dim3(kRedBlock), 0, s, static_cast<int>(N),
                       chunk, nchunks, sc, pred, scheme, seed, src, u_override, idx, theta_in,
                       theta_out, kd, l_in, l_out, logw, copy_when_skipped);
    return hipGetLastError();
}

hipError_t launch_exchange(double* theta, double* l, const double* beta, int64_t M,
                           int32_t kd, int parity_mode, int parity_host, int wrap,
                           uint64_t seed, StepSrc src, int* t_advance, unsigned* n_swap,
                           hipStream_t s) {
    const int64_t pairs = M / 2 + 1;
    const int g = static_cast<int>((pairs + kRedBlock - 1) / kRedBlock);
    hipLaunchKernelGGL(k_exchange, dim3(g), dim3(kRedBlock), 0, s, theta, l, beta,
                       static_cast<int>(M), kd, parity_mode, parity_host, wrap, seed, src,
                       t_advance, n_swap);
    return hipGetLastError();
}

hipError_t launch_step_mid(const Scratch& sc, int64_t N, StepSrc src, int* t_advance,
                           double* stats, double ess_frac, const double* logw, hipStream_t s,
                           const double* mom, int mom_k, int mom_stride, double* moments,
                           const RwPartial* part, int nparts) {
    if (mom != nullptr && (mom_k < 1 || mom_k > kMaxMomK)) return hipErrorInvalidValue;
    const int parts = part ? nparts : red_grid(N);
    const int chunk = cdf_chunk(N);
    const int nchunks = static_cast<int>((N + chunk - 1) / chunk);
    hipLaunchKernelGGL(k_step_mid, dim3(nchunks), dim3(kRedBlock), 0, s, parts, static_cast<int>(N),
                       chunk, src, t_advance, sc, stats, ess_frac, logw, mom, mom_k, mom_stride,
                       moments, part ? part : static_cast<const RwPartial*>(sc.rw_part),
                       part ? 1 : 0);
    return hipGetLastError();
}

void cdf_layout(int64_t N, int* chunk, int* nchunks) {
    *chunk = cdf_chunk(N);
    *nchunks = static_cast<int>((N + *chunk - 1) / *chunk);
}

hipError_t launch_search_gather(const Scratch& sc, int64_t N, int scheme, uint64_t seed,
                                StepSrc src, const StepState* pred_state, const double* theta_in,
                                double* theta_out, int32_t kd, const double* l_in, double* l_out,
                                double* logw, int copy_when_skipped, hipStream_t s) {
    ResamplePred pred{nullptr, 0.0, pred_state};
    int chunk, nchunks;
    cdf_layout(N, &chunk, &nchunks);
    const int g = static_cast<int>((N + kRedBlock - 1) / kRedBlock);
    hipLaunchKernelGGL(k_search_gather, dim3(g), dim3(kRedBlock), 0, s, static_cast<int>(N), chunk,
                       nchunks, sc, pred, scheme, seed, src, static_cast<const double*>(nullptr),
                       static_cast<int32_t*>(nullptr), theta_in, theta_out, kd, l_in, l_out, logw,
                       copy_when_skipped);
    return hipGetLastError();
}

hipError_t launch_publish_w(const Scratch& sc, double* W, const double* logw, int64_t N,
                            hipStream_t s) {
    const int g = static_cast<int>((N + kRedBlock - 1) / kRedBlock);
    hipLaunchKernelGGL(k_publish_w, dim3(g), dim3(kRedBlock), 0, s, W, logw, static_cast<int>(N), sc);
    return hipGetLastError();
}

hipError_t launch_pt_record(const double* theta, int64_t M, int32_t kd, int64_t chain,
                            const int32_t* it_dev, double* out, int64_t max_iters, hipStream_t s) {
    hipLaunchKernelGGL(k_pt_record, dim3(1), dim3(64), 0, s, theta, static_cast<int>(M), kd,
                       static_cast<int>(chain), it_dev, out, max_iters);
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
