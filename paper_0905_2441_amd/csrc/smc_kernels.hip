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

// Inclusive prefixes (double-double) of the piece [piece, piece + kRedBlock*PER)
// clipped to `end`, offset by `carry`, stored rounded in two halves to
// out_hi/out_lo; returns carry plus the piece's total. Each thread scans PER
// consecutive elements, but the weights are read and the prefixes written
// striped across the block (element e*256 + t by thread t: every wave access
// is 512 contiguous bytes) through LDS, whose rows are padded by one double per
// PER elements so that the per-thread runs do not fall on the same banks.
template <int PER, class WeightAt>
__device__ __forceinline__ dd scan_piece(int piece, int end, dd carry, double* out_hi,
                                         double* out_lo, WeightAt weight) {
    constexpr int kPiece = kRedBlock * PER;
    constexpr int kPadded = kPiece + kPiece / PER;
    __shared__ double sh_hi[kPadded], sh_lo[kPadded];
    auto at = [](int j) { return j + j / PER; };
    const int t = threadIdx.x;
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int j = e * kRedBlock + t;
        sh_hi[at(j)] = piece + j < end ? weight(piece + j) : 0.0;
    }
    __syncthreads();
    const int base = t * PER;
    dd pre[PER];
    dd run = dd_zero();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        if (piece + base + e < end) run = dd_add(run, sh_hi[at(base + e)]);
        pre[e] = run;
    }
    dd total;
    const dd excl = block_dd_exclusive_scan(run, total);     // ends with a barrier
    const dd lead = dd_add(carry, excl);
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const dd c = dd_add(lead, pre[e]);
        sh_hi[at(base + e)] = c.hi;
        sh_lo[at(base + e)] = c.lo;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < PER; ++e) {
        const int j = e * kRedBlock + t;
        if (piece + j < end) {
            out_hi[piece + j] = sh_hi[at(j)];
            out_lo[piece + j] = sh_lo[at(j)];
        }
    }
    __syncthreads();
    return dd_add(carry, total);
}

// Within-chunk inclusive prefixes of chunk b of the fused step's layout (up to
// kMaxChunks chunks of kScanChunk-element pieces) and the chunk's total.
template <class WeightAt>
__device__ __forceinline__ void scan_chunk(int b, int N, int chunk, const Scratch& sc,
                                           WeightAt weight) {
    const int begin = b * chunk;
    const int end = min(N, begin + chunk);
    dd carry = dd_zero();
    for (int piece = begin; piece < end; piece += kScanChunk)
        carry = scan_piece<kScanPerThread>(piece, end, carry, sc.cdf_hi, sc.cdf_lo, weight);
    if (threadIdx.x == 0) {
        sc.dd_part[2 * b] = carry.hi;
        sc.dd_part[2 * b + 1] = carry.lo;
    }
}

// Standalone resampling (smc_resample*) in three passes over chunks of
// kResChunk elements: (1) each chunk's within-chunk prefixes and total; (2) one
// workgroup scans the chunk totals into chunk offsets; (3) search and gather,
// reading C_j = offset + prefix (rounded once) with the offsets in memory, so
// no workgroup rescans the totals.
constexpr int kResPer = 4;
constexpr int kResChunk = kRedBlock * kResPer;

__global__ void __launch_bounds__(kRedBlock)
k_cdf_chunks(WeightSrc w, int N, Scratch sc, ResamplePred pred) {
    if (!should_fire(pred)) return;
    const int piece = blockIdx.x * kResChunk;
    const int end = min(N, piece + kResChunk);
    const dd tot = scan_piece<kResPer>(piece, end, dd_zero(), sc.cdf_hi, sc.cdf_lo,
                                       [&](int j) { return weight_at(w, j); });
    if (threadIdx.x == 0) {
        sc.res_tot[2 * blockIdx.x] = tot.hi;
        sc.res_tot[2 * blockIdx.x + 1] = tot.lo;
    }
}

// Exclusive double-double scan of the nchunks chunk totals into res_off
// (one workgroup; kScanPerThread consecutive totals per thread per round).
__global__ void __launch_bounds__(kRedBlock)
k_cdf_offsets(int nchunks, Scratch sc, ResamplePred pred) {
    if (!should_fire(pred)) return;
    dd carry = dd_zero();
    for (int piece = 0; piece < nchunks; piece += kScanChunk) {
        const int base = piece + threadIdx.x * kScanPerThread;
        dd loc[kScanPerThread];
        dd run = dd_zero();
#pragma unroll
        for (int e = 0; e < kScanPerThread; ++e) {
            loc[e] = run;
            if (base + e < nchunks)
                run = dd_add(run, dd{sc.res_tot[2 * (base + e)], sc.res_tot[2 * (base + e) + 1]});
        }
        dd total;
        const dd lead = dd_add(carry, block_dd_exclusive_scan(run, total));
#pragma unroll
        for (int e = 0; e < kScanPerThread; ++e) {
            if (base + e < nchunks) {
                const dd o = dd_add(lead, loc[e]);
                sc.res_off[2 * (base + e)] = o.hi;
                sc.res_off[2 * (base + e) + 1] = o.lo;
            }
        }
        carry = dd_add(carry, total);
    }
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
// of a chain of steps (many more than the reweight pass makes): they are read
// in one pass, with the loads of a thread's partials issued together, and the
// old weights' log-sum-exp is taken from the step state (the previous step's
// new one, or log N after its resampling).
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
        // one pass over the partials: kU of them per thread per round, all
        // their loads issued together; each thread sums its partials about
        // its own largest mn (rescaling its running sums when that grows), and
        // the block log-sum-exp rescales the threads' sums to the block's
        constexpr int kU = 8;
        double m = -INFINITY, a = 0.0, c = 0.0;
        for (int b0 = threadIdx.x; b0 < parts; b0 += kU * kRedBlock) {
            double vm[kU], v1[kU], v2[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int b = b0 + u * kRedBlock;
                vm[u] = b < parts ? part[b].mn : -INFINITY;
                v1[u] = b < parts ? part[b].s1 : 0.0;
                v2[u] = b < parts ? part[b].s2 : 0.0;
            }
            double mr = m;
#pragma unroll
            for (int u = 0; u < kU; ++u) mr = fmax(mr, vm[u]);
            const double rr = m == -INFINITY ? 0.0 : exp(m - mr);
            a *= rr;
            c *= rr * rr;
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const double r = vm[u] == -INFINITY ? 0.0 : exp(vm[u] - mr);
                a += v1[u] * r;
                c += v2[u] * (r * r);
            }
            m = mr;
        }
        nw = block_lse3(Lse3{m, a, c});
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
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    double u = 0.0;
    if (scheme == 0)
        u = u_override ? *u_override : u01_left_closed(draw(seed, 0, 0, step, kResamp, 0).w0);
    // lanes past N take point N - 1, so a wave's points stay sorted for the
    // sorted schemes' wave-cooperative search
    const int ic = i < N ? i : N - 1;
    const double U = resample_point(scheme, seed, step, ic, N, u);
    const int j = scheme == SMC_RESAMPLE_MULTINOMIAL
                      ? cdf_search(U, N, chunk, sc.cdf_hi, sc.cdf_lo, offh, offl)
                      : cdf_search_sorted_wave(U, true, N, chunk, sc.cdf_hi, sc.cdf_lo, offh, offl);
    if (i >= N) return;
    if (idx_out) idx_out[i] = j;
    if (theta_in && theta_out)
        for (int c = 0; c < kd; ++c)
            theta_out[static_cast<size_t>(c) * N + i] = theta_in[static_cast<size_t>(c) * N + j];
    if (l_in && l_out) l_out[i] = l_in[j];
    if (logw) logw[i] = 0.0;
}

// Phase 3 of standalone resampling: each particle's point U_i, its ancestor
// idx_i, the gather. Lanes past N take point N - 1.
//
// Sorted points (systematic, stratified): a workgroup takes kRedBlock * PER
// consecutive points. The ancestors a and b of its first and last point bound
// all of its ancestors (idx is non-decreasing in U); wave 0 finds both with
// one 32-ary search per half-wave. The window [a, b] of C_j is then loaded
// into LDS in pieces of kMergePiece values with independent coalesced loads,
// and every thread finds its PER consecutive points' ancestors there (a binary
// search for the first, then a galloping search forward from the previous
// answer): the only dependent global loads are the few levels of the 32-ary
// search. The indices go through LDS so that the gather and every store are
// striped over the block. Large populations take 8 points per thread (fewer
// 32-ary searches), smaller ones 2 (more workgroups in flight).
// Multinomial points are unsorted: one binary search per point.
constexpr int kMergePiece = 2048;
constexpr int64_t kMergeWideN = int64_t{1} << 22;   // PER = 8 from here on

__device__ __forceinline__ void resample_gather_point(int i, int j, int N, int32_t* idx_out,
                                                      const double* __restrict__ theta_in,
                                                      double* __restrict__ theta_out, int kd,
                                                      const double* __restrict__ l_in,
                                                      double* __restrict__ l_out, double* logw) {
    if (idx_out) idx_out[i] = j;
    if (theta_in && theta_out)
        for (int c = 0; c < kd; ++c)
            theta_out[static_cast<size_t>(c) * N + i] = theta_in[static_cast<size_t>(c) * N + j];
    if (l_in && l_out) l_out[i] = l_in[j];
    if (logw) logw[i] = 0.0;
}

__device__ __forceinline__ bool resample_copy_if_skipped(const ResamplePred& pred,
                                                         int copy_when_skipped, int i, int N,
                                                         int32_t* idx_out,
                                                         const double* theta_in,
                                                         double* theta_out, int kd,
                                                         const double* l_in, double* l_out) {
    if (should_fire(pred)) return false;
    if (copy_when_skipped && i < N) {
        if (idx_out) idx_out[i] = i;
        if (theta_in && theta_out)
            for (int c = 0; c < kd; ++c)
                theta_out[static_cast<size_t>(c) * N + i] = theta_in[static_cast<size_t>(c) * N + i];
        if (l_in && l_out) l_out[i] = l_in[i];
    }
    return true;
}

template <int PER>
__global__ void __launch_bounds__(kRedBlock)
k_resample_merge(int N, Scratch sc, ResamplePred pred, int scheme, uint64_t seed, StepSrc src,
                 const double* u_override, int32_t* idx_out,
                 const double* __restrict__ theta_in, double* __restrict__ theta_out, int kd,
                 const double* __restrict__ l_in, double* __restrict__ l_out, double* logw,
                 int copy_when_skipped) {
    constexpr int kMergePer = PER;
    constexpr int kMergeTile = kRedBlock * PER;
    __shared__ double cwin[kMergePiece];
    __shared__ int idx_sh[kMergeTile];
    __shared__ int ab[2];
    const int t = threadIdx.x;
    const int i0 = blockIdx.x * kMergeTile;
    if (!should_fire(pred)) {
        for (int e = 0; e < kMergePer; ++e)
            resample_copy_if_skipped(pred, copy_when_skipped, i0 + e * kRedBlock + t, N, idx_out,
                                     theta_in, theta_out, kd, l_in, l_out);
        return;
    }
    const double* __restrict__ hi = sc.cdf_hi;
    const double* __restrict__ lo = sc.cdf_lo;
    const double* __restrict__ off = sc.res_off;
    auto cdf = [&](int j) -> double {
        const int b = j / kResChunk;
        return dd_add(dd{off[2 * b], off[2 * b + 1]}, dd{hi[j], lo[j]}).hi;
    };
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    double u = 0.0;
    if (scheme == 0)
        u = u_override ? *u_override : u01_left_closed(draw(seed, 0, 0, step, kResamp, 0).w0);
    const double clast = cdf(N - 1);
    auto pred_c = [&](double uu, double c) -> bool {
        return uu < clast ? (uu < c) : (c >= clast);
    };
    const int i_last = min(N, i0 + kMergeTile) - 1;
    if (wave_id() == 0) {
        // lanes 0-31 search the ancestor of the tile's first point, 32-63 of its last
        const int lane = lane_id();
        const int half = lane >> 5, hl = lane & 31;
        const double us = resample_point(scheme, seed, step, half ? i_last : i0, N, u);
        int lo_ = 0, hi_ = N - 1;
        while (__any(hi_ > lo_)) {
            const int len = hi_ - lo_ + 1;
            const int stp = (len + 31) >> 5;
            int q = lo_ + (hl + 1) * stp - 1;
            q = q < hi_ ? q : hi_;
            const unsigned long long m = __ballot(pred_c(us, cdf(q)));
            const unsigned mh = static_cast<unsigned>(half ? (m >> 32) : (m & 0xffffffffull));
            const int f = __ffs(mh) - 1;
            const int nhi = lo_ + (f + 1) * stp - 1;
            lo_ = lo_ + f * stp;
            hi_ = nhi < hi_ ? nhi : hi_;
        }
        if (lane == 0) ab[0] = lo_;
        if (lane == 32) ab[1] = lo_;
    }
    // this thread's points, consecutive (sorted) within the thread
    double U[kMergePer];
    int found[kMergePer];
#pragma unroll
    for (int e = 0; e < kMergePer; ++e) {
        const int i = min(i0 + t * kMergePer + e, N - 1);
        U[e] = resample_point(scheme, seed, step, i, N, u);
        found[e] = -1;
    }
    __syncthreads();
    const int a = ab[0], b = ab[1];
    for (int p0 = a; p0 <= b; p0 += kMergePiece) {
        const int len = min(kMergePiece, b - p0 + 1);
        for (int r = t; r < len; r += kRedBlock) cwin[r] = cdf(p0 + r);
        __syncthreads();
        const double c_end = cwin[len - 1];
        int from = 0;             // no answer of this thread in this piece lies below it
#pragma unroll
        for (int e = 0; e < kMergePer; ++e) {
            if (found[e] < 0 && pred_c(U[e], c_end)) {
                // first position in [from, len) where pred holds: gallop, then bisect
                int l = from, h = len - 1;
                if (!pred_c(U[e], cwin[l])) {
                    int k = 1;
                    while (l + k < h && !pred_c(U[e], cwin[l + k])) k <<= 1;
                    h = l + k < h ? l + k : h;
                    l = l + (k >> 1) + 1;
                    while (l < h) {
                        const int mid = (l + h) >> 1;
                        if (pred_c(U[e], cwin[mid])) h = mid;
                        else l = mid + 1;
                    }
                }
                found[e] = p0 + l;
                from = l;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int e = 0; e < kMergePer; ++e) idx_sh[t * kMergePer + e] = found[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kMergePer; ++e) {
        const int r = e * kRedBlock + t;
        const int i = i0 + r;
        if (i < N)
            resample_gather_point(i, idx_sh[r], N, idx_out, theta_in, theta_out, kd, l_in, l_out,
                                  logw);
    }
}

__global__ void __launch_bounds__(kRedBlock)
k_resample_gather(int N, Scratch sc, ResamplePred pred, int scheme, uint64_t seed, StepSrc src,
                  const double* u_override, int32_t* idx_out,
                  const double* __restrict__ theta_in, double* __restrict__ theta_out, int kd,
                  const double* __restrict__ l_in, double* __restrict__ l_out, double* logw,
                  int copy_when_skipped) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (resample_copy_if_skipped(pred, copy_when_skipped, i, N, idx_out, theta_in, theta_out, kd,
                                 l_in, l_out))
        return;
    if (i >= N) return;
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    double u = 0.0;
    if (scheme == 0)
        u = u_override ? *u_override : u01_left_closed(draw(seed, 0, 0, step, kResamp, 0).w0);
    const double U = resample_point(scheme, seed, step, i, N, u);
    const double* __restrict__ hi = sc.cdf_hi;
    const double* __restrict__ lo = sc.cdf_lo;
    const double* __restrict__ off = sc.res_off;
    const int j = cdf_search_fn(U, N, [&](int jj) -> double {
        const int b = jj / kResChunk;
        return dd_add(dd{off[2 * b], off[2 * b + 1]}, dd{hi[jj], lo[jj]}).hi;
    });
    resample_gather_point(i, j, N, idx_out, theta_in, theta_out, kd, l_in, l_out, logw);
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
    const int nchunks = static_cast<int>((N + kResChunk - 1) / kResChunk);
    hipLaunchKernelGGL(k_cdf_chunks, dim3(nchunks), dim3(kRedBlock), 0, s, w,
                       static_cast<int>(N), sc, pred);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_cdf_offsets, dim3(1), dim3(kRedBlock), 0, s, nchunks, sc, pred);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (scheme == SMC_RESAMPLE_MULTINOMIAL) {
        const int g = static_cast<int>((N + kRedBlock - 1) / kRedBlock);
        hipLaunchKernelGGL(k_resample_gather, dim3(g), dim3(kRedBlock), 0, s, static_cast<int>(N),
                           sc, pred, scheme, seed, src, u_override, idx, theta_in, theta_out, kd,
                           l_in, l_out, logw, copy_when_skipped);
    } else {
        if (N >= kMergeWideN) {
            const int g = static_cast<int>((N + kRedBlock * 8 - 1) / (kRedBlock * 8));
            hipLaunchKernelGGL(k_resample_merge<8>, dim3(g), dim3(kRedBlock), 0, s,
                               static_cast<int>(N), sc, pred, scheme, seed, src, u_override, idx,
                               theta_in, theta_out, kd, l_in, l_out, logw, copy_when_skipped);
        } else {
            const int g = static_cast<int>((N + kRedBlock * 2 - 1) / (kRedBlock * 2));
            hipLaunchKernelGGL(k_resample_merge<2>, dim3(g), dim3(kRedBlock), 0, s,
                               static_cast<int>(N), sc, pred, scheme, seed, src, u_override, idx,
                               theta_in, theta_out, kd, l_in, l_out, logw, copy_when_skipped);
        }
    }
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
