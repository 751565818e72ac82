// Many independent SMC runs with uneven sizes in one step (serving-style batch).
//
// Each run r owns a contiguous block of particles [p_off, p_off + N_r) in the
// concatenated state arrays (its theta block is the usual [kd][N_r] layout at
// theta + kd*p_off) and a contiguous block of observations [y_off, y_off + n_r).
// All runs share the model constants and the tempering schedule and advance in
// lockstep; each has its own Philox key (seed), so a run's random numbers are
// exactly those it would draw alone.
//
// A batched tempering step is three launches whatever the number of runs:
//   k_b_reweight  one workgroup per run: the run's reweight, log-sum-exp, ESS,
//                 log-evidence increment and resampling decision (no partials:
//                 a run fits one workgroup's pass);
//   k_b_resample  one workgroup per run that resamples: double-double CDF scan
//                 of the run's weights, then search and gather of all N_r
//                 offspring (runs that keep their weights exit at once);
//   k_b_move      persistent: a grid sized to the GPU pulls work units from an
//                 atomic counter. A unit is 8 / S consecutive 64-particle tiles
//                 of one run, each moved by S of the workgroup's 8 waves
//                 (proposal + mixture likelihood over the run's n_r
//                 observations, the S waves splitting the data + accept). S is
//                 per run (launch table or built-in rule), so short-data runs
//                 fill the workgroup with several tiles instead of leaving waves
//                 idle. Units are listed longest data first (LPT), so runs whose
//                 work differs by 10^3 balance.
// and a one-thread kernel that advances the step counter and rewinds the work
// counter for the next replay.
#include "gmm_common.hpp"
#include "reduce.hpp"

namespace smc {
namespace {

constexpr int kBatchBlock = kBatchWaves * kWave;

__global__ void __launch_bounds__(kRedBlock)
k_b_reweight(const BatchRun* __restrict__ runs, double* __restrict__ logw,
             const double* __restrict__ l, StepSrc src, StepState* __restrict__ st,
             double* __restrict__ stats, double ess_frac, int* status) {
    const BatchRun rd = runs[blockIdx.x];
    const int t = step_index(src);
    const double dbeta = src.beta_dev[t] - src.beta_dev[t - 1];
    double* lw = logw + rd.p_off;
    const double* lr = l + rd.p_off;
    Lse3 o = lse3_empty(), nw = lse3_empty();
    bool bad = false;
    for (int p = threadIdx.x; p < rd.N; p += blockDim.x) {
        const double lo = lw[p];
        const double ln = lo + dbeta * lr[p];
        lw[p] = ln;
        bad = bad || (ln != ln) || (ln == INFINITY);
        o = lse3_push(o, lo);
        nw = lse3_push(nw, ln);
    }
    if (bad) atomicOr(status, kStatusNaN);
    o = block_lse3(o);
    nw = block_lse3(nw);
    if (threadIdx.x != 0) return;
    StepState s{};
    s.M = nw.m;
    s.S = nw.s1;
    s.S2 = nw.s2;
    s.lse_old = (o.m == -INFINITY) ? -INFINITY : o.m + log(o.s1);
    s.lse_new = (nw.m == -INFINITY) ? -INFINITY : nw.m + log(nw.s1);
    s.ess = (nw.s1 * nw.s1) / nw.s2;
    s.resampled = (ess_frac > 0.0) && (s.ess < ess_frac * static_cast<double>(rd.N));
    s.t = t;
    if (nw.m == -INFINITY || !(s.ess == s.ess)) atomicOr(status, kStatusAllZeroWeight);
    st[blockIdx.x] = s;
    double* sr = stats + 4 * static_cast<size_t>(blockIdx.x);
    sr[0] += s.lse_new - s.lse_old;
    sr[1] = s.ess;
    if (s.resampled) sr[2] += 1.0;
}

__global__ void __launch_bounds__(kRedBlock)
k_b_resample(const BatchRun* __restrict__ runs, const StepState* __restrict__ st,
             double* __restrict__ logw, const double* __restrict__ theta,
             const double* __restrict__ l, double* __restrict__ cdf,
             double* __restrict__ theta_tmp, double* __restrict__ l_tmp, int kd, StepSrc src,
             int scheme) {
    const BatchRun rd = runs[blockIdx.x];
    const StepState s = st[blockIdx.x];
    if (!s.resampled) return;
    const int N = rd.N;
    double* lw = logw + rd.p_off;
    double* C = cdf + rd.p_off;
    // correctly rounded prefix sums of W_j = exp(logw_j - M) / S, one pass in pieces
    dd carry = dd_zero();
    for (int piece = 0; piece < N; piece += kScanChunk) {
        const int base = piece + threadIdx.x * kScanPerThread;
        dd pre[kScanPerThread];
        dd run = dd_zero();
#pragma unroll
        for (int e = 0; e < kScanPerThread; ++e) {
            if (base + e < N) run = dd_add(run, exp(lw[base + e] - s.M) / s.S);
            pre[e] = run;
        }
        dd total;
        const dd excl = block_dd_exclusive_scan(run, total);
        const dd lead = dd_add(carry, excl);
#pragma unroll
        for (int e = 0; e < kScanPerThread; ++e)
            if (base + e < N) C[base + e] = dd_add(lead, pre[e]).hi;
        carry = dd_add(carry, total);
    }
    __threadfence_block();
    __syncthreads();
    const uint32_t step = static_cast<uint32_t>(s.t);
    const double u = scheme == 0 ? u01_left_closed(draw(rd.seed, 0, 0, step, kResamp, 0).w0) : 0.0;
    const double clast = C[N - 1];
    const double* th = theta + static_cast<size_t>(kd) * rd.p_off;
    double* tt = theta_tmp + static_cast<size_t>(kd) * rd.p_off;
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
        const double U = resample_point(scheme, rd.seed, step, i, N, u);
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
        for (int c = 0; c < kd; ++c)
            tt[static_cast<size_t>(c) * N + i] = th[static_cast<size_t>(c) * N + lo];
        l_tmp[rd.p_off + i] = l[rd.p_off + lo];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) lw[i] = 0.0;
}

template <int K, int PREC>
__global__ void __launch_bounds__(kBatchBlock, 4)
k_b_move(const BatchRun* __restrict__ runs, const BatchUnit* __restrict__ units, int n_units,
         unsigned* work, const float* __restrict__ y, double* theta, double* l,
         const double* __restrict__ logw, double* __restrict__ W,
         const double* __restrict__ theta_tmp, const double* __restrict__ l_tmp,
         const StepState* __restrict__ st, StepSrc src, double sd, uint32_t move, int first,
         GmmDev g, unsigned long long* n_acc, int* status) {
    constexpr int KD = K;
    __shared__ double red[kBatchWaves][kWave];
    __shared__ double prs[kBatchWaves][KD][kWave];
    __shared__ int unit_sh;
    const int lane = lane_id();
    const int w = wave_uniform(threadIdx.x / kWave);
    for (;;) {
        if (threadIdx.x == 0) unit_sh = static_cast<int>(atomicAdd(work, 1u));
        __syncthreads();
        const int u = unit_sh;
        __syncthreads();
        if (u >= n_units) break;
        const BatchUnit un = units[u];
        const BatchRun rd = runs[un.run];
        const int S = wave_uniform(un.slices);
        const int grp = w / S;                       // this wave's tile within the unit
        const int sl = w - grp * S;                  // and its data slice
        const bool active = grp < un.ntiles;
        const int N = rd.N;
        const int n = rd.n;
        const int p = (un.tile0 + (active ? grp : 0)) * kWave + lane;
        const int pc = p < N ? p : N - 1;
        const StepState* sr = st + un.run;
        const uint32_t step = static_cast<uint32_t>(sr->t);
        const bool use_alt = first && sr->resampled;
        double* th_run = theta + static_cast<size_t>(KD) * rd.p_off;
        double* l_run = l + rd.p_off;
        const double* th_src = use_alt ? theta_tmp + static_cast<size_t>(KD) * rd.p_off : th_run;
        const double l_src = use_alt ? l_tmp[rd.p_off + pc] : l_run[pc];
        // the tile's Box-Muller pairs shared out over its S waves (an idle
        // wave of a short last unit draws none but meets the barrier)
        double pr[KD];
        block_proposals<KD>(rd.seed, static_cast<uint32_t>(pc), step, move, th_src, N, pc, sd,
                            active ? sl : (KD + 1) / 2, S, prs[grp], pr);
        double part = 0.0;
        if (active) {
            int j0, j1;
            slice_bounds(n, sl, S, j0, j1);
            part = slice_partial<K, 1, PREC>(y + rd.y_off, j0, j1, pr, g, near_data(l_src, n, g),
                                             PivotStage{pivot_row<PREC, 1, kBatchWaves>()});
        }
        red[w][lane] = part;
        __syncthreads();
        if (active && sl == 0) {
            bool acc = false;
            if (p < N) {
                double tot = red[w][lane];
                for (int q = 1; q < S; ++q) tot += red[w + q][lane];
                const double l_prop = finish_loglik<PREC>(tot, n, g);
                MoveStep ms{};
                if (first) {
                    ms.theta_alt = theta_tmp + static_cast<size_t>(KD) * rd.p_off;
                    ms.l_alt = l_tmp + rd.p_off;
                    ms.state = sr;
                    ms.W_out = W + rd.p_off;
                    ms.logw = const_cast<double*>(logw) + rd.p_off;
                }
                const MoveSource srcs = move_source(ms, th_run, l_run);
                acc = rwmh_accept<KD>(p, p, N, [&](int c) { return pr[c]; }, l_prop, srcs, th_run,
                                      l_run, nullptr, src, step, rd.seed, move, g, status, ms);
            }
            const unsigned long long mask = __ballot(acc);
            if (lane == 0 && n_acc != nullptr && mask != 0ull)
                atomicAdd(n_acc, static_cast<unsigned long long>(__popcll(mask)));
        }
        __syncthreads();
    }
}

__global__ void k_b_end(int* t_dev, unsigned* work) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *t_dev += 1;
        *work = 0u;
    }
}

__global__ void k_b_rewind(unsigned* work) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *work = 0u;
}

}  // namespace

int batch_move_grid() {
    int dev = 0, cus = 256, per_cu = 1;
    if (hipGetDevice(&dev) == hipSuccess)
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void*>(&k_b_move<4, SMC_PREC_FP32>), kBatchBlock, 0) !=
            hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    return cus * per_cu;
}

hipError_t launch_batch_step(const BatchDev& b, const GmmDev& g, const float* y, double* theta,
                             double* l, double* logw, double* W, const double* beta, int T,
                             int* t_dev, double sd, int n_moves, double ess_frac, int prec,
                             double* stats, unsigned long long* n_acc, int* status, int scheme,
                             hipStream_t s) {
    StepSrc src{};
    src.t_dev = t_dev;
    src.beta_dev = beta;
    src.t_max = T;
    hipLaunchKernelGGL(k_b_reweight, dim3(b.R), dim3(kRedBlock), 0, s, b.runs, logw, l, src, b.state,
                       stats, ess_frac, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_b_resample, dim3(b.R), dim3(kRedBlock), 0, s, b.runs, b.state, logw,
                       theta, l, b.cdf, b.theta_tmp, b.l_tmp, g.k * g.d, src, scheme);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int pi = prec == SMC_PREC_FP32 ? 1 : 0;
    const BatchUnit* units = b.units[pi];
    const int n_units = b.n_units[pi];
    const int grid = n_units < b.move_grid ? n_units : b.move_grid;
    for (int m = 0; m < n_moves; ++m) {
        if (m > 0) {
            hipLaunchKernelGGL(k_b_rewind, dim3(1), dim3(64), 0, s, b.work);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
#define SMC_BK(KK)                                                                              \
        if (g.k == KK) {                                                                        \
            if (prec == SMC_PREC_FP32)                                                          \
                hipLaunchKernelGGL((k_b_move<KK, SMC_PREC_FP32>), dim3(grid), dim3(kBatchBlock), 0, s, \
                                   b.runs, units, n_units, b.work, y, theta, l, logw, W,    \
                                   b.theta_tmp, b.l_tmp, b.state, src, sd, static_cast<uint32_t>(m), \
                                   m == 0 ? 1 : 0, g, n_acc, status);                           \
            else                                                                                \
                hipLaunchKernelGGL((k_b_move<KK, SMC_PREC_FP64>), dim3(grid), dim3(kBatchBlock), 0, s, \
                                   b.runs, units, n_units, b.work, y, theta, l, logw, W,    \
                                   b.theta_tmp, b.l_tmp, b.state, src, sd, static_cast<uint32_t>(m), \
                                   m == 0 ? 1 : 0, g, n_acc, status);                           \
        }
        SMC_BK(1) SMC_BK(2) SMC_BK(3) SMC_BK(4) SMC_BK(5) SMC_BK(6) SMC_BK(7) SMC_BK(8)
#undef SMC_BK
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_b_end, dim3(1), dim3(64), 0, s, t_dev, b.work);
    return hipGetLastError();
}

}  // namespace smc
