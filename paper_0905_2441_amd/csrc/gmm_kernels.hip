// Mixture log-likelihood, random-walk MH move and prior draws for gfx950.
//
// Decomposition (one workgroup = 64 particles x S data slices):
//   * lane l of every wave owns particle blockIdx.x*64 + l and keeps that
//     particle's k*d means in registers (as FP32 scaled offsets, or FP64);
//   * wave w of the workgroup owns a data slice of about n/S observations
//     (slice_bounds); its bounds are made wave-uniform, so in the plain forms
//     every observation is fetched by a scalar load into SGPRs and broadcast
//     to all 64 lanes, and in the pivot form (1-D data) the wave stages its
//     observations, 64 at a time, in its own LDS row and reads them back as
//     broadcasts; no barrier inside the data loop;
//   * the S per-slice partial sums of a particle meet in LDS and wave 0 adds
//     them in slice order (bit-reproducible for a given S).
// The paper evaluated one likelihood per thread over data in shared memory
// and remarked that long data can be split over several threads (Comparison
// subsection); here both are combined: lanes over particles, waves over data.
//
// FP32 forms, in base-2 units, a_i = log2 w_i - s^2 (y - mu_i)^2 with
// s = sqrt(log2(e)/(2 sigma2)) (partial_fp32):
//   * pivot (1-D data): per window of 64 data (or pair of windows, while the
//     pair's range is narrow enough) about its midpoint c, each
//     particle's component p with the largest a_p(c) is its pivot; the
//     others enter through t_i = a_i - a_p, which is linear in y (one FMA),
//     as 2^(t_i) (hardware v_exp_f32), and the pivot's own a_p summed over
//     the window comes from two data sums shared by the wave's particles;
//   * plain: t_i = s*y - s*mu_i (one FMA), a_i = log2 w_i - t_i^2 (one FMA),
//     and the datum's mixture sum e = sum_i 2^(a_i), taken directly for
//     waves near the data or relative to m = max_i a_i otherwise.
// Instead of one log per datum, the per-datum factors are multiplied into a
// running FP32 product whose exponent is extracted exactly after each block
// of data (frexp), and the m's and the pivot terms are summed apart and
// promoted into an FP64 accumulator. Neither is a Kahan sum: the product
// loses no exponent range (the integer exponents are exact), the block sums
// round at most 16 FP32 terms, and the relative error of the particle's
// log-likelihood stays below 1e-6 for n up to 10^5.
//
// FP64 form ("plain"): the same decomposition in FP64 with natural logs, the
// device library's exp/log for every term and a plain FP64 sum over data.
#include <algorithm>
#include <vector>

#include "exchange.hpp"
#include "gmm_common.hpp"
#include "reduce.hpp"

namespace smc {
namespace {

// Form counts of the FP32 single-move kernel (k_rwmh) since the last reset, on
// this device (partial_fp32: observation x 64-particle tile pairs in the plain
// shifted form, pairs in the pivot form, and the pivot form's other components
// summed over its pairs), each spread over kFormSlots counters (a diagnostic
// of which forms the moves took; summed by smc_fp32_form_counts).
__device__ unsigned long long g_fp32_form_ctr[kFormCounts * kFormSlots];

template <int K, int D, int PREC>
__global__ void __launch_bounds__(1024)
k_loglik(const float* __restrict__ y, int n, const double* __restrict__ theta, int N,
         GmmDev g, double* __restrict__ out, int* status) {
    constexpr int KD = K * D;
    // LDS sized by the launch (loglik_dyn_lds_bytes): red [S][64] doubles, then
    // for the FP32 1-D form the waves' staging rows [S][kPivotRow] floats
    extern __shared__ __align__(16) double lds[];
    const int S = wave_uniform(blockDim.x / kWave);
    double (*red)[kWave] = reinterpret_cast<double (*)[kWave]>(lds);
    const int lane = lane_id();
    const int w = wave_uniform(threadIdx.x / kWave);
    float* row = (PREC == SMC_PREC_FP32 && D == 1)
                     ? reinterpret_cast<float*>(lds + S * kWave) + w * kPivotRow
                     : nullptr;
    const int p = blockIdx.x * kWave + lane;
    const int pc = p < N ? p : N - 1;
    int j0, j1;
    slice_bounds(n, w, S, j0, j1);
    double pr[KD];
#pragma unroll
    for (int c = 0; c < KD; ++c) pr[c] = theta[static_cast<size_t>(c) * N + pc];
    red[w][lane] = slice_partial<K, D, PREC>(y, j0, j1, pr, g, true, PivotStage{row});
    __syncthreads();
    if (w == 0 && p < N) {
        double acc = red[0][lane];
        for (int s = 1; s < S; ++s) acc += red[s][lane];
        const double l = finish_loglik<PREC>(acc, n, g);
        out[p] = l;
        if (l != l) atomicOr(status, kStatusNaN);
    }
}

// The next tempering step's reweight of one 64-particle tile, made by wave 0 of
// the tile's move after its last decision (the pass a separate reweight kernel
// would make): lw_next[p] = (0 after resampling, else this step's log-weight
// lw_now) + (beta[t+1] - beta[t]) l_new, and the tile's log-sum-exp partial of
// those weights. Every lane of the wave takes part.
__device__ __forceinline__ void chain_reweight(const MoveStep& ms, int p, int N, int tile,
                                               uint32_t step, double lw_now, double l_new,
                                               int* status) {
    const int t1 = static_cast<int>(step) + 1 > ms.t_max ? ms.t_max : static_cast<int>(step) + 1;
    const double dbeta = ms.beta_dev[t1] - ms.beta_dev[t1 - 1];
    Lse3 nw = lse3_empty();
    if (p < N) {
        const double ln = (ms.state->resampled != 0 ? 0.0 : lw_now) + dbeta * l_new;
        ms.lw_next[p] = ln;
        if (ln != ln || ln == INFINITY) atomicOr(status, kStatusNaN);
        if (ln != -INFINITY) nw = Lse3{ln, 1.0, 1.0};
    }
    nw = wave_lse3(nw);
    if (lane_id() == 0) ms.next_part[tile] = RwPartial{0.0, 0.0, nw.m, nw.s1, nw.s2, 0.0};
}

// CHAIN: the move also makes the next tempering step's reweight (ms.lw_next set,
// one workgroup per tile); a separate instantiation keeps the plain move's code
// free of it.
template <int K, int D, int PREC, bool CHAIN>
__global__ void __launch_bounds__(1024)
k_rwmh(const float* __restrict__ y, int n, double* theta, double* l, int N,
       const double* __restrict__ beta_vec, StepSrc src, double sd, uint64_t seed,
       uint32_t move, GmmDev g, unsigned long long* n_acc, int* status, MoveStep ms, int G,
       double* __restrict__ part, int* __restrict__ anc_out) {
    constexpr int KD = K * D;
    constexpr bool kRows = PREC == SMC_PREC_FP32 && D == 1;
    // the current state held in LDS for the decision (small k*d)
    constexpr bool kHold = KD <= 16;
    __shared__ double red[kMaxSlices][kWave];
    __shared__ int anc[kWave];
    __shared__ double prs[KD][kWave];
    __shared__ double hold[kHold ? KD : 1][kWave];
    __shared__ double hold_l[kWave];
    // LDS sized by the launch (rwmh_dyn_lds_bytes): for the FP32 1-D form the
    // waves' staging rows [S][kPivotRow] floats, then offh, offl [nch] (nch =
    // ms.nchunks when the move can resample, else 0)
    extern __shared__ __align__(16) double lds[];
    const int S = wave_uniform(blockDim.x / kWave);
    const int nch = ms.cdf_hi != nullptr ? ms.nchunks : 0;
    double* offh = lds + (kRows ? S * (kPivotRow / 2) : 0);
    double* offl = offh + nch;
    const int lane = lane_id();
    const int w = wave_uniform(threadIdx.x / kWave);
    float* row = kRows ? reinterpret_cast<float*>(lds) + w * kPivotRow : nullptr;
    const int tile = static_cast<int>(blockIdx.x) / G;
    const int grp = static_cast<int>(blockIdx.x) - tile * G;
    const int p = tile * kWave + lane;
    const int pc = p < N ? p : N - 1;
    const int nsl = S * G;
    const int sl = grp * S + w;
    int j0, j1;
    slice_bounds(n, sl, nsl, j0, j1);
    // the lane's first datum of the slice for the pivot form, loaded ahead
    // of the ancestor search and the proposals (their barriers and Box-Muller
    // work hide its latency)
    const bool y_pre = kRows && j1 - j0 >= kPivotMinData;
    const float y_first = y_pre && j0 + lane < j1 ? y[j0 + lane] : 0.0f;
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    if (ms.t_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0)
        *ms.t_out = static_cast<int>(step);
    const bool fused = (ms.cdf_hi != nullptr) && (ms.state != nullptr) && (ms.state->resampled != 0);
    if (fused) fused_ancestors(ms, N, step, pc, anc, offh, offl);
    const MoveSource srcs = move_source(ms, theta, l);
    const int a = fused ? anc[lane] : pc;

    double pr[KD];
    block_proposals<KD>(seed, static_cast<uint32_t>(pc), step, move, srcs.th, N, a, sd, w, S, prs,
                        pr, kHold && G == 1 ? hold : nullptr, srcs.l, hold_l);
    red[w][lane] = slice_partial<K, D, PREC>(y, j0, j1, pr, g, near_data(srcs.l[a], n, g),
                                             PivotStage{row, y_first, y_pre}, g_fp32_form_ctr);
    __syncthreads();
    if (w != 0) return;

    if (G > 1) {
        // this group's share; k_rwmh_accept adds the groups and decides
        if (p < N) {
            double tot = red[0][lane];
            for (int s = 1; s < S; ++s) tot += red[s][lane];
            part[static_cast<size_t>(grp) * N + p] = tot;
            if (grp == 0 && fused) anc_out[p] = a;
        }
        return;
    }
    // this step's log-weight, loaded while the decision is made (with a chain of
    // steps logw and lw_next may be one array: read before it is overwritten)
    const double lw_now = (CHAIN && p < N) ? ms.logw[p] : 0.0;
    bool acc = false;
    double l_new = 0.0;
    if (p < N) {
        double tot = red[0][lane];
        for (int s = 1; s < S; ++s) tot += red[s][lane];
        const double l_prop = finish_loglik<PREC>(tot, n, g);
        if constexpr (kHold) {
            acc = rwmh_accept_state<KD>(
                p, N, [&](int c) { return pr[c]; }, [&](int c) { return hold[c][lane]; },
                hold_l[lane], l_prop, srcs.write_always, theta, l, beta_vec, src, step, seed,
                move, g, status, ms, CHAIN ? &l_new : nullptr);
        } else {
            acc = rwmh_accept<KD>(p, a, N, [&](int c) { return pr[c]; }, l_prop, srcs, theta, l,
                                  beta_vec, src, step, seed, move, g, status, ms,
                                  CHAIN ? &l_new : nullptr);
        }
    }
    const unsigned long long mask = __ballot(acc);
    if (lane == 0 && n_acc != nullptr && mask != 0ull)
        atomicAdd(n_acc, static_cast<unsigned long long>(__popcll(mask)));
    if constexpr (CHAIN) chain_reweight(ms, p, N, tile, step, lw_now, l_new, status);
}

// Several consecutive moves of one tempering step in one launch (one
// workgroup per 64-particle tile): the tile's state lives in LDS between moves,
// wave 0 decides each move and updates it, and the output population, W and
// logw are written once at the end. The moves of a particle use only its own
// state, so this equals n_moves separate launches bit for bit. CHAIN: as in
// k_rwmh, the next step's reweight after the last move.
template <int K, int D, int PREC, bool CHAIN>
__global__ void __launch_bounds__(1024)
k_rwmh_multi(const float* __restrict__ y, int n, double* theta, double* l, int N, StepSrc src,
             double sd, uint64_t seed, uint32_t move0, int n_moves, GmmDev g,
             unsigned long long* n_acc, int* status, MoveStep ms) {
    constexpr int KD = K * D;
    constexpr bool kRows = PREC == SMC_PREC_FP32 && D == 1;
    __shared__ double red[kMaxSlices][kWave];
    __shared__ int anc[kWave];
    __shared__ double prs[KD][kWave];
    __shared__ double cur[KD][kWave];
    __shared__ double lcur[kWave];
    // LDS sized by the launch (rwmh_dyn_lds_bytes), as in k_rwmh
    extern __shared__ __align__(16) double lds[];
    const int S = wave_uniform(blockDim.x / kWave);
    const int nch = ms.cdf_hi != nullptr ? ms.nchunks : 0;
    double* offh = lds + (kRows ? S * (kPivotRow / 2) : 0);
    double* offl = offh + nch;
    const int lane = lane_id();
    const int w = wave_uniform(threadIdx.x / kWave);
    float* row = kRows ? reinterpret_cast<float*>(lds) + w * kPivotRow : nullptr;
    const int p = static_cast<int>(blockIdx.x) * kWave + lane;
    const int pc = p < N ? p : N - 1;
    int j0, j1;
    slice_bounds(n, w, S, j0, j1);
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    const bool fused = (ms.cdf_hi != nullptr) && (ms.state != nullptr) && (ms.state->resampled != 0);
    if (fused) fused_ancestors(ms, N, step, pc, anc, offh, offl);
    const MoveSource srcs = move_source(ms, theta, l);
    if (w == 0) {
        const int a = fused ? anc[lane] : pc;
#pragma unroll
        for (int c = 0; c < KD; ++c) cur[c][lane] = srcs.th[static_cast<size_t>(c) * N + a];
        lcur[lane] = srcs.l[a];
    }
    __syncthreads();
    unsigned long long accepted = 0;
    for (int m = 0; m < n_moves; ++m) {
        const uint32_t mv = move0 + static_cast<uint32_t>(m);
        double pr[KD];
        block_proposals<KD>(seed, static_cast<uint32_t>(pc), step, mv, &cur[0][0], kWave, lane, sd,
                            w, S, prs, pr);
        red[w][lane] = slice_partial<K, D, PREC>(y, j0, j1, pr, g, near_data(lcur[lane], n, g),
                                                 PivotStage{row});
        __syncthreads();
        if (w == 0) {
            double tot = red[0][lane];
            for (int q = 1; q < S; ++q) tot += red[q][lane];
            const double l_prop = finish_loglik<PREC>(tot, n, g);
            const bool acc = rwmh_decide<KD>(
                pc, [&](int c) { return pr[c]; }, [&](int c) { return cur[c][lane]; }, lcur[lane],
                l_prop, nullptr, src, step, seed, mv, g);
            if (acc) {
#pragma unroll
                for (int c = 0; c < KD; ++c) cur[c][lane] = pr[c];
                lcur[lane] = l_prop;
            }
            if (p < N && l_prop != l_prop) atomicOr(status, kStatusNaN);
            accepted += static_cast<unsigned long long>(__popcll(__ballot(acc && p < N)));
        }
        __syncthreads();
    }
    if (w != 0) return;
    // with a chain of steps logw and lw_next may be one array: read it first
    const double lw_now = (CHAIN && p < N) ? ms.logw[p] : 0.0;
    if (p < N) {
#pragma unroll
        for (int c = 0; c < KD; ++c) theta[static_cast<size_t>(c) * N + p] = cur[c][lane];
        l[p] = lcur[lane];
        move_duties(p, N, ms);
    }
    if (lane == 0 && n_acc != nullptr && accepted != 0ull) atomicAdd(n_acc, accepted);
    if constexpr (CHAIN)
        chain_reweight(ms, p, N, static_cast<int>(blockIdx.x), step, lw_now, lcur[lane], status);
}

// Data (floats) the one-launch population-MCMC kernel stages in LDS.
constexpr int kPtLocalData = 2048;

// Several population-MCMC iterations in one launch of one workgroup, for
// populations small enough that every chain's state fits in LDS. The
// workgroup's waves are `tiles` 64-chain tiles x S data slices. An iteration
// has three phases separated by barriers:
//   1. every wave forms its tile's proposals (state + sd * the normals held in
//      LDS) and sums its data slice;
//   2. the first wave of each tile adds the slices and decides each chain's
//      move at its own beta, while the tile's other waves draw the next
//      iteration's random numbers (normals, log u of the acceptance and
//      exchange tests, the partition parity) into LDS;
//   3. the workgroup takes the iteration's exchanges on the LDS states.
// The chains' states, their betas and (when n d <= kPtLocalData) the data
// stay in LDS for the whole launch.
// The random numbers are drawn from the same streams and with the same
// arithmetic as in separate iterations, so the results (bit for bit, for the
// same slicing) equal those of n_iters pt_iteration calls. The iteration
// index is read once from the caller's counter, which ends advanced by n_iters.
template <int K, int D, int PREC, int MAXC>
__global__ void __launch_bounds__(1024)
k_pt_local(const float* __restrict__ y, int n, double* theta, double* l, int M,
           const double* __restrict__ beta, int* it_dev, int n_iters, double sd, uint64_t seed,
           int parity_mode, int wrap, int S, GmmDev g, unsigned long long* n_acc,
           unsigned* n_swap, int* status) {
    constexpr int KD = K * D;
    constexpr int NP = (KD + 1) / 2;            // Box-Muller pairs per chain
    constexpr int NITEM = NP + 2;               // + the acceptance and exchange uniforms
    __shared__ double red[kMaxSlices][kWave];
    __shared__ double cur[KD][MAXC];
    __shared__ double zs[KD][MAXC];             // the coming iteration's normals
    __shared__ double lcur[MAXC];
    __shared__ double lua[2][MAXC];             // log u of the acceptance tests
    __shared__ double lux[2][MAXC];             // log u of the exchange led by each chain
    __shared__ double lbeta[MAXC];
    __shared__ float ys[kPtLocalData];          // the data, when they fit
    __shared__ int par[2];
    const int lane = lane_id();
    const int w = wave_uniform(threadIdx.x / kWave);
    const int tile = w / S;
    const int sl = w - tile * S;
    const int col = tile * kWave + lane;          // chain held by this lane
    const int cc = col < M ? col : M - 1;
    int j0, j1;
    slice_bounds(n, sl, S, j0, j1);
    // random items of chain col for iteration it, items first, first + stride, ...
    auto draw_items = [&](uint32_t it, int buf, int first, int stride) {
        for (int i = first; i < NITEM; i += stride) {
            if (i < NP) {
                const Words4 wd = draw(seed, static_cast<uint32_t>(cc), static_cast<uint32_t>(i / 2),
                                       it, kProp, 0);
                double z0, z1;
                if (i & 1) box_muller(wd.w2, wd.w3, z0, z1);
                else box_muller(wd.w0, wd.w1, z0, z1);
                zs[2 * i][col] = z0;
                if (2 * i + 1 < KD) zs[2 * i + 1][col] = z1;
            } else if (i == NP) {
                lua[buf][col] = rwmh_log_u(cc, it, seed, 0);
            } else {
                lux[buf][col] = pt_log_u(cc, seed, it);
                if (col == 0) par[buf] = pt_parity(parity_mode, 0, seed, it);
            }
        }
    };
    const int it0 = *it_dev;
    if (sl == 0) {
#pragma unroll
        for (int c = 0; c < KD; ++c) cur[c][col] = theta[static_cast<size_t>(c) * M + cc];
        lcur[col] = l[cc];
        lbeta[col] = beta[cc];
    }
    const bool stage = static_cast<int64_t>(n) * D <= kPtLocalData;
    if (stage)
        for (int i = threadIdx.x; i < n * D; i += blockDim.x) ys[i] = y[i];
    const float* yl = stage ? ys : y;
    draw_items(static_cast<uint32_t>(it0), 0, sl, S);
    __syncthreads();
    unsigned long long accepted = 0;
    unsigned swaps = 0;
    for (int m = 0; m < n_iters; ++m) {
        const uint32_t it = static_cast<uint32_t>(it0 + m);
        const int buf = m & 1;
        double pr[KD];
#pragma unroll
        for (int c = 0; c < KD; ++c) pr[c] = cur[c][col] + sd * zs[c][col];
        // the same per-datum forms as the one-launch-per-iteration path, so the
        // two agree bit for bit
        red[w][lane] = slice_partial<K, D, PREC>(yl, j0, j1, pr, g, near_data(lcur[col], n, g),
                                                 PivotStage{pivot_row<PREC, D, kMaxSlices>()});
        __syncthreads();
        if (sl == 0) {
            double tot = red[w][lane];
            for (int q = 1; q < S; ++q) tot += red[w + q][lane];
            const double l_prop = finish_loglik<PREC>(tot, n, g);
            const double la = rwmh_log_alpha<KD>(
                col, [&](int c) { return pr[c]; }, [&](int c) { return cur[c][col]; }, lcur[col],
                l_prop, lbeta, StepSrc{}, it, g);
            const bool acc = (la >= 0.0) || (lua[buf][col] < la);
            if (acc) {
#pragma unroll
                for (int c = 0; c < KD; ++c) cur[c][col] = pr[c];
                lcur[col] = l_prop;
            }
            if (col < M && l_prop != l_prop) atomicOr(status, kStatusNaN);
            accepted += static_cast<unsigned long long>(__popcll(__ballot(acc && col < M)));
        }
        if (m + 1 < n_iters) {
            if (S == 1) draw_items(it + 1u, buf ^ 1, 0, 1);
            else if (sl > 0) draw_items(it + 1u, buf ^ 1, sl - 1, S - 1);
        }
        __syncthreads();
        const int parity = par[buf];
        for (int q = threadIdx.x;; q += blockDim.x) {
            int a, b;
            if (!pt_slot(M, parity, wrap, q, a, b)) break;
            if (b < 0) continue;
            if (pt_swap_given(&cur[0][0], lcur, lbeta, MAXC, KD, a, b, lux[buf][a])) ++swaps;
        }
        __syncthreads();
    }
    if (sl == 0 && col < M) {
#pragma unroll
        for (int c = 0; c < KD; ++c) theta[static_cast<size_t>(c) * M + col] = cur[c][col];
        l[col] = lcur[col];
    }
    if (sl == 0 && lane == 0 && n_acc != nullptr && accepted != 0ull) atomicAdd(n_acc, accepted);
    if (n_swap != nullptr && swaps != 0u) atomicAdd(n_swap, swaps);
    __syncthreads();
    if (threadIdx.x == 0) *it_dev = it0 + n_iters;
}

// One population-MCMC iteration per launch for populations spread over many
// workgroups, with the exchange deferred: a launch reads the population after
// the previous iteration's moves (th_in, l_in), first takes that iteration's
// exchange for each of its chains (both chains of a pair reach the same
// decision from the same inputs; each keeps its own side), then makes this
// iteration's move and writes the population to the other buffer (th_out,
// l_out). The iteration index comes from *it_in; workgroup 0 stores it + 1 in
// *it_out (a different counter, so no workgroup reads a changed value). With
// pending = 0 (the first iteration of a sequence) no exchange precedes the
// move. Arithmetic and random streams are those of the move and exchange
// kernels, so the results equal theirs bit for bit.
template <int K, int D, int PREC>
__global__ void __launch_bounds__(1024)
k_pt_deferred(const float* __restrict__ y, int n, const double* __restrict__ th_in,
              const double* __restrict__ l_in, double* __restrict__ th_out,
              double* __restrict__ l_out, int M, const double* __restrict__ beta,
              const int* it_in, int* it_out, int pending, int parity_mode, int wrap, double sd,
              uint64_t seed, GmmDev g, unsigned long long* n_acc, unsigned* n_swap, int* status) {
    constexpr int KD = K * D;
    __shared__ double red[kMaxSlices][kWave];
    __shared__ double cur[KD][kWave];
    __shared__ double prs[KD][kWave];
    __shared__ double lcur[kWave];
    // LDS sized by the launch: for the FP32 1-D form the waves' staging rows
    // [S][kPivotRow] floats
    extern __shared__ __align__(16) double lds[];
    const int S = wave_uniform(blockDim.x / kWave);
    const int lane = lane_id();
    const int w = wave_uniform(threadIdx.x / kWave);
    float* row = (PREC == SMC_PREC_FP32 && D == 1)
                     ? reinterpret_cast<float*>(lds) + w * kPivotRow
                     : nullptr;
    const int p = static_cast<int>(blockIdx.x) * kWave + lane;
    const int pc = p < M ? p : M - 1;
    int j0, j1;
    slice_bounds(n, w, S, j0, j1);
    const uint32_t it = static_cast<uint32_t>(*it_in);
    if (blockIdx.x == 0 && threadIdx.x == 0) *it_out = static_cast<int>(it) + 1;
    if (w == 0) {
        int src = pc;
        if (pending) {
            const uint32_t prev = it - 1u;
            const int parity = pt_parity(parity_mode, 0, seed, prev);
            int a, b;
            if (pt_pair_of(M, parity, wrap, pc, a, b)) {
                const double la = (beta[a] - beta[b]) * (l_in[b] - l_in[a]);
                if (la >= 0.0 || pt_log_u(a, seed, prev) < la) {
                    src = pc == a ? b : a;
                    if (p < M && p == a && n_swap != nullptr) atomicAdd(n_swap, 1u);
                }
            }
        }
#pragma unroll
        for (int c = 0; c < KD; ++c) cur[c][lane] = th_in[static_cast<size_t>(c) * M + src];
        lcur[lane] = l_in[src];
    }
    __syncthreads();
    double pr[KD];
    block_proposals<KD>(seed, static_cast<uint32_t>(pc), it, 0, &cur[0][0], kWave, lane, sd, w, S,
                        prs, pr);
    red[w][lane] = slice_partial<K, D, PREC>(y, j0, j1, pr, g, near_data(lcur[lane], n, g),
                                             PivotStage{row});
    __syncthreads();
    if (w != 0) return;
    double tot = red[0][lane];
    for (int q = 1; q < S; ++q) tot += red[q][lane];
    const double l_prop = finish_loglik<PREC>(tot, n, g);
    const bool acc = rwmh_decide<KD>(
        pc, [&](int c) { return pr[c]; }, [&](int c) { return cur[c][lane]; }, lcur[lane], l_prop,
        beta, StepSrc{}, it, seed, 0, g);
    if (p < M) {
#pragma unroll
        for (int c = 0; c < KD; ++c) th_out[static_cast<size_t>(c) * M + p] = acc ? pr[c] : cur[c][lane];
        l_out[p] = acc ? l_prop : lcur[lane];
        if (l_prop != l_prop) atomicOr(status, kStatusNaN);
    }
    const unsigned long long mask = __ballot(acc && p < M);
    if (lane == 0 && n_acc != nullptr && mask != 0ull)
        atomicAdd(n_acc, static_cast<unsigned long long>(__popcll(mask)));
}

// The last deferred exchange of a sequence, out of place: each chain reads its
// pair from (th_in, l_in) and writes its own side to (th_out, l_out); the
// iteration is *it_src - 1 and *it_dst receives *it_src.
__global__ void __launch_bounds__(256)
k_pt_deferred_exchange(const double* __restrict__ th_in, const double* __restrict__ l_in,
                       double* __restrict__ th_out, double* __restrict__ l_out, int M, int kd,
                       const double* __restrict__ beta, const int* it_src, int* it_dst,
                       int parity_mode, int wrap, uint64_t seed, unsigned* n_swap) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const int itp1 = *it_src;
    if (blockIdx.x == 0 && threadIdx.x == 0) *it_dst = itp1;
    if (c >= M) return;
    const uint32_t prev = static_cast<uint32_t>(itp1) - 1u;
    const int parity = pt_parity(parity_mode, 0, seed, prev);
    int src = c;
    int a, b;
    if (pt_pair_of(M, parity, wrap, c, a, b)) {
        const double la = (beta[a] - beta[b]) * (l_in[b] - l_in[a]);
        if (la >= 0.0 || pt_log_u(a, seed, prev) < la) {
            src = c == a ? b : a;
            if (c == a && n_swap != nullptr) atomicAdd(n_swap, 1u);
        }
    }
    for (int q = 0; q < kd; ++q) th_out[static_cast<size_t>(q) * M + c] = th_in[static_cast<size_t>(q) * M + src];
    l_out[c] = l_in[src];
}

// Second half of a move whose tile data were split over G workgroups, for
// particle p: add the G partial sums in group order, re-form the same proposal
// (same counter, same arithmetic) and take the MH decision.
template <int KD, int PREC>
__device__ __forceinline__ bool complete_split_move(int p, int n, double* theta, double* l, int N,
                                                    const double* beta_vec, const StepSrc& src,
                                                    uint32_t step, double sd, uint64_t seed,
                                                    uint32_t move, const GmmDev& g, int* status,
                                                    const MoveStep& ms, int G,
                                                    const double* part, const int* anc_in) {
    const bool fused = (ms.cdf_hi != nullptr) && (ms.state != nullptr) && (ms.state->resampled != 0);
    const MoveSource srcs = move_source(ms, theta, l);
    const int a = fused ? anc_in[p] : p;
    double pr[KD];
    {
        double z[KD];
        normals<KD>(seed, static_cast<uint32_t>(p), step, kProp, move, z);
#pragma unroll
        for (int c = 0; c < KD; ++c) pr[c] = srcs.th[static_cast<size_t>(c) * N + a] + sd * z[c];
    }
    double tot = part[p];
    for (int q = 1; q < G; ++q) tot += part[static_cast<size_t>(q) * N + p];
    const double l_prop = finish_loglik<PREC>(tot, n, g);
    return rwmh_accept<KD>(p, a, N, [&](int c) { return pr[c]; }, l_prop, srcs, theta, l,
                           beta_vec, src, step, seed, move, g, status, ms);
}

__device__ __forceinline__ void count_accepts(bool acc, unsigned long long* n_acc) {
    const unsigned long long mask = __ballot(acc);
    if ((threadIdx.x & (kWave - 1)) == 0 && n_acc != nullptr && mask != 0ull)
        atomicAdd(n_acc, static_cast<unsigned long long>(__popcll(mask)));
}

// One thread per particle completes a split move.
template <int KD, int PREC>
__global__ void __launch_bounds__(256)
k_rwmh_accept(int n, double* theta, double* l, int N, const double* __restrict__ beta_vec,
              StepSrc src, double sd, uint64_t seed, uint32_t move, GmmDev g,
              unsigned long long* n_acc, int* status, MoveStep ms, int G,
              const double* __restrict__ part, const int* __restrict__ anc_in) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    bool acc = false;
    if (p < N)
        acc = complete_split_move<KD, PREC>(p, n, theta, l, N, beta_vec, src, step, sd, seed, move,
                                            g, status, ms, G, part, anc_in);
    count_accepts(acc, n_acc);
}

// Population-MCMC iteration after a split move: two threads per slot of the
// iteration's partition, adjacent lanes of one wave, one for each chain of the
// slot's pair (the odd lane idles when the slot holds a single chain). Each
// lane completes its chain's move in registers (the proposal regenerated from
// the same counter, the groups' partial sums added in group order); both lanes
// then take the pair's exchange decision on the moved states, the partner's
// fetched by a lane shuffle, and each writes its chain once. The same result as
// all moves followed by all exchanges: the moves are independent per chain and
// the pairs are disjoint. The iteration index comes from the step state
// recorded by the move; the caller's counter is advanced.
template <int KD, int PREC>
__global__ void __launch_bounds__(256)
k_pt_accept_exchange(int n, double* theta, double* l, int M, const double* __restrict__ beta,
                     StepSrc src, double sd, uint64_t seed, GmmDev g, int G,
                     const double* __restrict__ part, int parity_mode, int wrap, int* t_advance,
                     unsigned long long* n_acc, unsigned* n_swap, int* status) {
    const uint32_t it = static_cast<uint32_t>(step_index(src));
    if (t_advance != nullptr && blockIdx.x == 0 && threadIdx.x == 0)
        *t_advance = static_cast<int>(it) + 1;
    const int parity = pt_parity(parity_mode, 0, seed, it);
    const int gt = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
    const bool odd = (gt & 1) != 0;
    int a = -1, b = -1;
    const bool slot = pt_slot(M, parity, wrap, gt >> 1, a, b);
    const int c = odd ? b : a;
    const bool active = slot && c >= 0;
    double th[KD];
#pragma unroll
    for (int k = 0; k < KD; ++k) th[k] = 0.0;
    double lc = 0.0;
    bool acc = false;
    if (active) {
        double pr[KD];
        {
            double z[KD];
            normals<KD>(seed, static_cast<uint32_t>(c), it, kProp, 0, z);
#pragma unroll
            for (int k = 0; k < KD; ++k) {
                th[k] = theta[static_cast<size_t>(k) * M + c];
                pr[k] = th[k] + sd * z[k];
            }
        }
        double tot = part[c];
        for (int q = 1; q < G; ++q) tot += part[static_cast<size_t>(q) * M + c];
        const double l_prop = finish_loglik<PREC>(tot, n, g);
        const double l_cur = l[c];
        acc = rwmh_decide<KD>(
            c, [&](int k) { return pr[k]; }, [&](int k) { return th[k]; }, l_cur, l_prop, beta,
            src, it, seed, 0u, g);
        if (l_prop != l_prop) atomicOr(status, kStatusNaN);
        lc = acc ? l_prop : l_cur;
        if (acc) {
#pragma unroll
            for (int k = 0; k < KD; ++k) th[k] = pr[k];
        }
    }
    // the partner lane's moved state (every lane takes part in the shuffles)
    const double lp = __shfl_xor(lc, 1);
    double tp[KD];
#pragma unroll
    for (int k = 0; k < KD; ++k) tp[k] = __shfl_xor(th[k], 1);
    bool swap = false;
    if (active && b >= 0) {
        const double l_a = odd ? lp : lc;
        const double l_b = odd ? lc : lp;
        const double la = (beta[a] - beta[b]) * (l_b - l_a);
        swap = la >= 0.0 || pt_log_u(a, seed, it) < la;
    }
    if (active) {
#pragma unroll
        for (int k = 0; k < KD; ++k) theta[static_cast<size_t>(k) * M + c] = swap ? tp[k] : th[k];
        l[c] = swap ? lp : lc;
    }
    count_accepts(acc, n_acc);
    const unsigned long long sw = __ballot(swap && !odd);
    if ((threadIdx.x & (kWave - 1)) == 0 && n_swap != nullptr && sw != 0ull)
        atomicAdd(n_swap, static_cast<unsigned>(__popcll(sw)));
}

template <int KD>
__global__ void k_prior(int N, uint64_t seed, GmmDev g, double* __restrict__ theta) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    if (g.prior == SMC_PRIOR_GAUSS) {
        double z[KD];
        normals<KD>(seed, static_cast<uint32_t>(p), 0, kPrior, 0, z);
#pragma unroll
        for (int c = 0; c < KD; ++c) theta[static_cast<size_t>(c) * N + p] = g.pa + g.pb * z[c];
    } else {
        const double width = g.pb - g.pa;
#pragma unroll
        for (int b = 0; b < (KD + 3) / 4; ++b) {
            const Words4 w = draw(seed, static_cast<uint32_t>(p), b, 0, kPrior, 0);
            const uint32_t ws[4] = {w.w0, w.w1, w.w2, w.w3};
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (4 * b + q < KD)
                    theta[static_cast<size_t>(4 * b + q) * N + p] = g.pa + width * u01_open(ws[q]);
        }
    }
}

}  // namespace

// (K, D) pairs compiled into the library.
#define SMC_KD_CASES(X) \
    X(1, 1) X(2, 1) X(3, 1) X(4, 1) X(5, 1) X(6, 1) X(7, 1) X(8, 1) X(1, 8) X(2, 8) X(4, 8) X(8, 8)

namespace {

// Largest dynamic LDS a k_rwmh or k_rwmh_multi launch asks for (their static
// part is at most 8 KB + 64 KB + 768 B).
constexpr size_t kMaxRwmhLds = 24 * 1024;

// LDS bytes of the pivot form's staging rows of `slices` waves (FP32, d = 1).
size_t rows_lds_bytes(int slices, bool rows) {
    return rows ? sizeof(float) * slices * kPivotRow : 0;
}

// Dynamic LDS bytes of one k_rwmh / k_rwmh_multi workgroup (the layout at the
// top of k_rwmh).
size_t rwmh_dyn_lds_bytes(int slices, int nchunks, bool rows) {
    return rows_lds_bytes(slices, rows) + sizeof(double) * 2 * static_cast<size_t>(nchunks);
}

}  // namespace

bool supported_kd(int k, int d, int prec) {
    if (prec == SMC_PREC_BF16X3) return dd_supported(k, d);
    if (prec != SMC_PREC_FP32 && prec != SMC_PREC_FP64) return false;
#define SMC_CASE(K, D) \
    if (k == K && d == D) return true;
    SMC_KD_CASES(SMC_CASE)
#undef SMC_CASE
    return false;
}

hipError_t launch_loglik(const GmmDev& g, const float* y, int64_t n, const double* theta,
                         int64_t N, int prec, double* out, int slices, int* status,
                         hipStream_t s) {
    if (slices < 1 || slices > kMaxSlices) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>((N + kWave - 1) / kWave));
    const dim3 block(static_cast<unsigned>(kWave * slices));
    // LDS of k_loglik: red [slices][64] doubles, then the staging rows
    const size_t red_bytes = sizeof(double) * kWave * slices;
#define SMC_CASE(K, D)                                                                        \
    if (g.k == K && g.d == D) {                                                               \
        if (prec == SMC_PREC_FP32)                                                            \
            hipLaunchKernelGGL((k_loglik<K, D, SMC_PREC_FP32>), grid, block,                  \
                               red_bytes + rows_lds_bytes(slices, D == 1), s, y,              \
                               static_cast<int>(n), theta, static_cast<int>(N), g, out,       \
                               status);                                                       \
        else                                                                                  \
            hipLaunchKernelGGL((k_loglik<K, D, SMC_PREC_FP64>), grid, block, red_bytes, s, y, \
                               static_cast<int>(n), theta, static_cast<int>(N), g, out,       \
                               status);                                                       \
        return hipGetLastError();                                                             \
    }
    SMC_KD_CASES(SMC_CASE)
#undef SMC_CASE
    return hipErrorInvalidValue;
}

namespace {

bool valid_split(const Split& sp, int64_t N) {
    return sp.groups >= 1 && sp.groups <= kMaxGroups && sp.slices >= 1 &&
           sp.slices <= kMaxSlices && (sp.groups == 1 || N <= kSplitCap);
}

// The likelihood half of a move (with the decision when groups == 1).
template <int K, int D, int P>
hipError_t launch_move_partials(const float* y, int64_t n, double* theta, double* l, int64_t N,
                                const double* beta_vec, const StepSrc& src, double sd,
                                uint64_t seed, uint32_t move, const GmmDev& g,
                                unsigned long long* n_accept, const Split& sp, const Scratch& sc,
                                const MoveStep& ms, hipStream_t s) {
    const int64_t tiles = (N + kWave - 1) / kWave;
    const dim3 grid(static_cast<unsigned>(tiles * sp.groups));
    const dim3 block(static_cast<unsigned>(kWave * sp.slices));
    const int nch = ms.cdf_hi != nullptr ? ms.nchunks : 0;
    if (nch < 0 || nch > kMaxChunks) return hipErrorInvalidValue;
    const size_t lds = rwmh_dyn_lds_bytes(sp.slices, nch, P == SMC_PREC_FP32 && D == 1);
    if (lds > kMaxRwmhLds) return hipErrorInvalidValue;
    if (ms.lw_next != nullptr)
        hipLaunchKernelGGL((k_rwmh<K, D, P, true>), grid, block, lds, s, y, static_cast<int>(n),
                           theta, l, static_cast<int>(N), beta_vec, src, sd, seed, move, g,
                           n_accept, sc.status, ms, sp.groups, sc.mv_part, sc.mv_anc);
    else
        hipLaunchKernelGGL((k_rwmh<K, D, P, false>), grid, block, lds, s, y, static_cast<int>(n),
                           theta, l, static_cast<int>(N), beta_vec, src, sd, seed, move, g,
                           n_accept, sc.status, ms, sp.groups, sc.mv_part, sc.mv_anc);
    return hipSuccess;
}

}  // namespace

hipError_t launch_rwmh(const GmmDev& g, const float* y, int64_t n, double* theta, double* l,
                       int64_t N, const double* beta_vec, StepSrc src, double sd,
                       uint64_t seed, uint32_t move, int prec,
                       unsigned long long* n_accept, Split sp, const Scratch& sc, MoveStep ms,
                       hipStream_t s) {
    if (!valid_split(sp, N)) return hipErrorInvalidValue;
    const dim3 agrid(static_cast<unsigned>((N + 255) / 256));
#define SMC_MOVE(K, D, P)                                                                      \
    do {                                                                                       \
        const hipError_t e0 = launch_move_partials<K, D, P>(y, n, theta, l, N, beta_vec, src,  \
                                                            sd, seed, move, g, n_accept, sp,   \
                                                            sc, ms, s);                        \
        if (e0 != hipSuccess) return e0;                                                       \
        if (sp.groups > 1)                                                                     \
            hipLaunchKernelGGL((k_rwmh_accept<K * D, P>), agrid, dim3(256), 0, s,              \
                               static_cast<int>(n), theta, l, static_cast<int>(N), beta_vec,   \
                               src, sd, seed, move, g, n_accept, sc.status, ms, sp.groups,     \
                               static_cast<const double*>(sc.mv_part),                         \
                               static_cast<const int*>(sc.mv_anc));                            \
    } while (0)
#define SMC_CASE(K, D)                                                                         \
    if (g.k == K && g.d == D) {                                                                \
        if (prec == SMC_PREC_FP32) SMC_MOVE(K, D, SMC_PREC_FP32);                              \
        else SMC_MOVE(K, D, SMC_PREC_FP64);                                                    \
        return hipGetLastError();                                                              \
    }
    SMC_KD_CASES(SMC_CASE)
#undef SMC_CASE
#undef SMC_MOVE
    return hipErrorInvalidValue;
}

bool rwmh_moves_chainable(const GmmDev& g, int n_moves, const Split& sp) {
    if (sp.groups != 1 || n_moves < 1) return false;
    if (n_moves == 1) return true;
    bool multi = false;
#define SMC_CASE(K, D)                                                                         \
    if (g.k == K && g.d == D && K * D <= 16) multi = true;
    SMC_KD_CASES(SMC_CASE)
#undef SMC_CASE
    return multi;
}

hipError_t launch_rwmh_moves(const GmmDev& g, const float* y, int64_t n, double* theta,
                             double* l, int64_t N, StepSrc src, double sd, uint64_t seed,
                             int n_moves, int prec, unsigned long long* n_accept, Split sp,
                             const Scratch& sc, MoveStep ms, hipStream_t s) {
    if (!valid_split(sp, N) || n_moves < 1) return hipErrorInvalidValue;
    // the next step's reweight is made by the last move of a single launch
    if (ms.lw_next != nullptr && !rwmh_moves_chainable(g, n_moves, sp)) return hipErrorInvalidValue;
    const bool one_launch = n_moves > 1 && rwmh_moves_chainable(g, n_moves, sp);
    if (!one_launch) {
        for (int m = 0; m < n_moves; ++m) {
            const hipError_t e = launch_rwmh(g, y, n, theta, l, N, nullptr, src, sd, seed,
                                             static_cast<uint32_t>(m), prec, n_accept, sp, sc,
                                             m == 0 ? ms : MoveStep{}, s);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    const dim3 grid(static_cast<unsigned>((N + kWave - 1) / kWave));
    const dim3 block(static_cast<unsigned>(kWave * sp.slices));
    const int nch = ms.cdf_hi != nullptr ? ms.nchunks : 0;
    if (nch < 0 || nch > kMaxChunks) return hipErrorInvalidValue;
#define SMC_MULTI(K, D, P)                                                                     \
    do {                                                                                       \
        const size_t lds = rwmh_dyn_lds_bytes(sp.slices, nch, P == SMC_PREC_FP32 && D == 1);   \
        if (lds > kMaxRwmhLds) return hipErrorInvalidValue;                                    \
        if (ms.lw_next != nullptr)                                                             \
            hipLaunchKernelGGL((k_rwmh_multi<K, D, P, true>), grid, block, lds, s, y,          \
                               static_cast<int>(n), theta, l, static_cast<int>(N), src, sd,    \
                               seed, 0u, n_moves, g, n_accept, sc.status, ms);                 \
        else                                                                                   \
            hipLaunchKernelGGL((k_rwmh_multi<K, D, P, false>), grid, block, lds, s, y,         \
                               static_cast<int>(n), theta, l, static_cast<int>(N), src, sd,    \
                               seed, 0u, n_moves, g, n_accept, sc.status, ms);                 \
    } while (0)
#define SMC_CASE(K, D)                                                                         \
    if constexpr (K * D <= 16) {                                                               \
        if (g.k == K && g.d == D) {                                                            \
            if (prec == SMC_PREC_FP32) SMC_MULTI(K, D, SMC_PREC_FP32);                         \
            else SMC_MULTI(K, D, SMC_PREC_FP64);                                               \
            return hipGetLastError();                                                          \
        }                                                                                      \
    }
    SMC_KD_CASES(SMC_CASE)
#undef SMC_CASE
#undef SMC_MULTI
    return hipErrorInvalidValue;
}

// Chains per workgroup of the one-launch form: at most 4096 state doubles
// (two 32 KB arrays in LDS at k*d = 4), in whole 64-chain tiles, at most 16 tiles.
constexpr int kPtLocalCap = 4096;

constexpr int pt_local_cap(int kd) {
    return kd > 16 ? 0 : ((kPtLocalCap / kd) / kWave * kWave < 1024 ? (kPtLocalCap / kd) / kWave * kWave : 1024);
}

int pt_local_chains(int kd) { return kd < 1 ? 0 : pt_local_cap(kd); }

// One workgroup runs on one compute unit, so the single-launch form pays off
// only while an iteration's likelihood work (64-lane tiles x n data x k*d) is
// small enough that the launches it saves cost more than the parallelism it
// gives up against the one-launch-per-iteration (deferred exchange) form:
// measured on the paper's population-MCMC runs (n = 100, k = 4), up to 128
// chains at n = 100.
constexpr int64_t kPtLocalWork = int64_t{1} << 16;

bool pt_local_pays(int kd, int64_t n, int64_t M) {
    const int64_t tiles = (M + kWave - 1) / kWave;
    return tiles * kWave * n * kd <= kPtLocalWork;
}

int pt_local_slices(int64_t n, int64_t M) {
    const int tiles = static_cast<int>((M + kWave - 1) / kWave);
    int S = 8 / tiles;                       // about eight waves in all
    const int64_t by_data = n / 12;          // at least a dozen data per slice
    if (by_data < S) S = static_cast<int>(by_data);
    return S < 1 ? 1 : S;
}

hipError_t launch_pt_local(const GmmDev& g, const float* y, int64_t n, double* theta, double* l,
                           int64_t M, const double* beta, int* it_dev, int n_iters, double sd,
                           uint64_t seed, int prec, int parity_mode, int wrap, int slices,
                           unsigned long long* n_accept, unsigned* n_swap, int* status,
                           hipStream_t s) {
    const int kd = g.k * g.d;
    const int tiles = static_cast<int>((M + kWave - 1) / kWave);
    if (M < 2 || M > pt_local_chains(kd) || tiles > kMaxSlices) return hipErrorInvalidValue;
    int S = slices < 1 ? 1 : slices;
    if (S * tiles > kMaxSlices) S = kMaxSlices / tiles;
    if (S > n) S = static_cast<int>(n);
    if (S < 1) S = 1;
    const dim3 block(static_cast<unsigned>(kWave * tiles * S));
#define SMC_LOCAL(K, D, P, C)                                                                  \
    hipLaunchKernelGGL((k_pt_local<K, D, P, C>), dim3(1), block, 0, s, y, static_cast<int>(n), \
                       theta, l, static_cast<int>(M), beta, it_dev, n_iters, sd, seed,         \
                       parity_mode, wrap, S, g, n_accept, n_swap, status)
#define SMC_CASE(K, D)                                                                         \
    if constexpr (K * D <= 16) {                                                               \
        if (g.k == K && g.d == D) {                                                            \
            constexpr int C = pt_local_cap(K * D);                                              \
            if (prec == SMC_PREC_FP32) SMC_LOCAL(K, D, SMC_PREC_FP32, C);                      \
            else SMC_LOCAL(K, D, SMC_PREC_FP64, C);                                            \
            return hipGetLastError();                                                          \
        }                                                                                      \
    }
    SMC_KD_CASES(SMC_CASE)
#undef SMC_CASE
#undef SMC_LOCAL
    return hipErrorInvalidValue;
}

hipError_t launch_pt_iteration(const GmmDev& g, const float* y, int64_t n, double* theta,
                               double* l, int64_t M, const double* beta, StepSrc src,
                               StepSrc later, double sd, uint64_t seed, int prec,
                               unsigned long long* n_accept, Split sp, const Scratch& sc,
                               MoveStep ms, int parity_mode, int wrap, int* t_advance,
                               unsigned* n_swap, hipStream_t s) {
    if (!valid_split(sp, M)) return hipErrorInvalidValue;
    if (sp.groups == 1) {
        hipError_t e = launch_rwmh(g, y, n, theta, l, M, beta, src, sd, seed, 0, prec, n_accept,
                                   sp, sc, ms, s);
        if (e != hipSuccess) return e;
        return launch_exchange(theta, l, beta, M, g.k * g.d, parity_mode, 0, wrap, seed, later,
                               t_advance, n_swap, s);
    }
    // slots: at most M/2 pairs plus two singles, two threads each
    const dim3 xgrid(static_cast<unsigned>((2 * (M / 2 + 2) + 255) / 256));
#define SMC_PT(K, D, P)                                                                        \
    do {                                                                                       \
        const hipError_t e0 = launch_move_partials<K, D, P>(y, n, theta, l, M, beta, src, sd,  \
                                                            seed, 0, g, n_accept, sp, sc, ms,  \
                                                            s);                                \
        if (e0 != hipSuccess) return e0;                                                       \
        hipLaunchKernelGGL((k_pt_accept_exchange<K * D, P>), xgrid, dim3(256), 0, s,           \
                           static_cast<int>(n), theta, l, static_cast<int>(M), beta, later,    \
                           sd, seed, g, sp.groups, static_cast<const double*>(sc.mv_part),     \
                           parity_mode, wrap, t_advance, n_accept, n_swap, sc.status);         \
    } while (0)
#define SMC_CASE(K, D)                                                                         \
    if (g.k == K && g.d == D) {                                                                \
        if (prec == SMC_PREC_FP32) SMC_PT(K, D, SMC_PREC_FP32);                                \
        else SMC_PT(K, D, SMC_PREC_FP64);                                                      \
        return hipGetLastError();                                                              \
    }
    SMC_KD_CASES(SMC_CASE)
#undef SMC_CASE
#undef SMC_PT
    return hipErrorInvalidValue;
}

hipError_t launch_pt_deferred(const GmmDev& g, const float* y, int64_t n, double* theta,
                              double* l, int64_t M, const double* beta, int* it_dev,
                              int n_iters, double sd, uint64_t seed, int prec, int parity_mode,
                              int wrap, int slices, unsigned long long* n_accept,
                              unsigned* n_swap, const Scratch& sc, int* counter2,
                              hipStream_t s) {
    const int kd = g.k * g.d;
    if (M < 2 || n_iters < 1 || slices < 1 || slices > kMaxSlices || sc.cap < M) return hipErrorInvalidValue;
    const int64_t tiles = (M + kWave - 1) / kWave;
    // buffers X0 = (theta, l) and X1 = scratch, counters C0 = it_dev and C1
    double* th[2] = {theta, sc.theta_tmp};
    double* lb[2] = {l, sc.l_tmp};
    int* ctr[2] = {it_dev, counter2};
    const dim3 grid(static_cast<unsigned>(tiles)), block(static_cast<unsigned>(kWave * slices));
    for (int i = 0; i < n_iters; ++i) {
        const int a = i & 1, b = a ^ 1;
#define SMC_DEF(K, D, P)                                                                       \
    hipLaunchKernelGGL((k_pt_deferred<K, D, P>), grid, block,                                  \
                       rows_lds_bytes(slices, P == SMC_PREC_FP32 && D == 1), s, y,             \
                       static_cast<int>(n), th[a], lb[a], th[b], lb[b], static_cast<int>(M),   \
                       beta, ctr[a], ctr[b], i > 0 ? 1 : 0, parity_mode, wrap, sd, seed, g,    \
                       n_accept, n_swap, sc.status)
#define SMC_CASE(K, D)                                                                                 if (g.k == K && g.d == D) {                                                                        if (prec == SMC_PREC_FP32) SMC_DEF(K, D, SMC_PREC_FP32);                                       else SMC_DEF(K, D, SMC_PREC_FP64);                                                         } else
        SMC_KD_CASES(SMC_CASE) { return hipErrorInvalidValue; }
#undef SMC_CASE
#undef SMC_DEF
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // the last exchange: in place on X0 (pairs) when the population ended there,
    // else from X1 into X0 (chains)
    if ((n_iters & 1) == 0) {
        StepSrc src{};
        src.t_dev = counter2;                  // holds the last iteration's index
        return launch_exchange(theta, l, beta, M, kd, parity_mode, 0, wrap, seed, src, it_dev,
                               n_swap, s);
    }
    hipLaunchKernelGGL(k_pt_deferred_exchange, dim3(static_cast<unsigned>((M + 255) / 256)),
                       dim3(256), 0, s, sc.theta_tmp, sc.l_tmp, theta, l, static_cast<int>(M), kd,
                       beta, static_cast<const int*>(counter2), it_dev, parity_mode, wrap, seed,
                       n_swap);
    return hipGetLastError();
}

hipError_t launch_prior(const GmmDev& g, int64_t N, uint64_t seed, double* theta,
                        hipStream_t s) {
    const int kd = g.k * g.d;
    const dim3 block(256);
    const dim3 grid(static_cast<unsigned>((N + 255) / 256));
#define SMC_KD(KD)                                                                            \
    if (kd == KD) {                                                                           \
        hipLaunchKernelGGL((k_prior<KD>), grid, block, 0, s, static_cast<int>(N), seed, g,    \
                           theta);                                                            \
        return hipGetLastError();                                                             \
    }
    SMC_KD(1) SMC_KD(2) SMC_KD(3) SMC_KD(4) SMC_KD(5) SMC_KD(6) SMC_KD(7) SMC_KD(8)
    SMC_KD(16) SMC_KD(32) SMC_KD(64)
#undef SMC_KD
    return hipErrorInvalidValue;
}

hipError_t fp32_form_counts(unsigned long long* out, bool reset) {
    constexpr int kAll = kFormCounts * kFormSlots;
    static_assert(sizeof(g_fp32_form_ctr) == kAll * sizeof(unsigned long long), "");
    std::vector<unsigned long long> v(kAll);
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpyFromSymbol(v.data(), HIP_SYMBOL(g_fp32_form_ctr), kAll * sizeof(v[0]), 0,
                                hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    for (int c = 0; c < kFormCounts; ++c) {
        unsigned long long sum = 0;
        for (int i = 0; i < kFormSlots; ++i) sum += v[c * kFormSlots + i];
        out[c] = sum;
    }
    if (reset) {
        std::fill(v.begin(), v.end(), 0ull);
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_fp32_form_ctr), v.data(), kAll * sizeof(v[0]), 0,
                              hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    return e;
}

}  // namespace smc
