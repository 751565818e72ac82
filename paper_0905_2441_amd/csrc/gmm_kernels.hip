// Mixture log-likelihood, random-walk MH move and prior draws for gfx950.
//
// Decomposition (one workgroup = 64 particles x S data slices):
//   * lane l of every wave owns particle blockIdx.x*64 + l and keeps that
//     particle's k*d means in registers (as FP32 scaled offsets, or FP64);
//   * wave w of the workgroup owns the data slice [w*n/S, (w+1)*n/S); its index
//     is made wave-uniform, so every observation is fetched by a scalar load
//     into SGPRs and broadcast to all 64 lanes with no LDS traffic, no VGPR
//     copies and no barriers inside the data loop;
//   * the S per-slice partial sums of a particle meet in LDS and wave 0 adds
//     them in slice order (bit-reproducible for a given S).
// The paper evaluated one likelihood per thread over data in shared memory
// and remarked that long data can be split over several threads (Comparison
// subsection); here both are combined: lanes over particles, waves over data.
//
// FP32 form, per datum y and component i, in base-2 units:
//   t_i = s*y - s*mu_i            (s = sqrt(log2(e)/(2 sigma2)); one FMA)
//   a_i = log2 w_i - t_i^2        (one FMA)
//   m = max_i a_i;  e = sum_i 2^(a_i - m)   (hardware v_exp_f32)
// and log2 of the datum's mixture density (up to the constant) is m + log2 e.
// Instead of one log per datum, the e's are multiplied into a running FP32
// product whose exponent is extracted exactly every 8 data (frexp), and the
// m's are summed in blocks of 8 in FP32 and promoted into an FP64
// accumulator. Both are compensated schemes: the relative error of the
// particle's log-likelihood stays below 1e-6 for n up to 10^5.
//
// FP64 form ("plain"): the same decomposition in FP64 with natural logs, the
// device library's exp/log for every term and a plain FP64 sum over data.
#include "gmm_common.hpp"

namespace smc {
namespace {

template <int K, int D, int PREC>
__global__ void __launch_bounds__(1024)
k_loglik(const float* __restrict__ y, int n, const double* __restrict__ theta, int N,
         GmmDev g, double* __restrict__ out, int* status) {
    constexpr int KD = K * D;
    __shared__ double red[kMaxSlices][kWave];
    const int S = wave_uniform(blockDim.x / kWave);
    const int lane = lane_id();
    const int w = wave_uniform(threadIdx.x / kWave);
    const int p = blockIdx.x * kWave + lane;
    const int pc = p < N ? p : N - 1;
    const int j0 = wave_uniform(static_cast<int>((static_cast<int64_t>(n) * w) / S));
    const int j1 = wave_uniform(static_cast<int>((static_cast<int64_t>(n) * (w + 1)) / S));
    double pr[KD];
#pragma unroll
    for (int c = 0; c < KD; ++c) pr[c] = theta[static_cast<size_t>(c) * N + pc];
    red[w][lane] = slice_partial<K, D, PREC>(y, j0, j1, pr, g);
    __syncthreads();
    if (w == 0 && p < N) {
        double acc = red[0][lane];
        for (int s = 1; s < S; ++s) acc += red[s][lane];
        const double l = finish_loglik<PREC>(acc, n, g);
        out[p] = l;
        if (l != l) atomicOr(status, kStatusNaN);
    }
}

template <int K, int D, int PREC>
__global__ void __launch_bounds__(1024)
k_rwmh(const float* __restrict__ y, int n, double* theta, double* l, int N,
       const double* __restrict__ beta_vec, StepSrc src, double sd, uint64_t seed,
       uint32_t move, GmmDev g, unsigned long long* n_acc, int* status, MoveStep ms, int G,
       double* __restrict__ part, int* __restrict__ anc_out) {
    constexpr int KD = K * D;
    __shared__ double red[kMaxSlices][kWave];
    __shared__ int anc[kWave];
    __shared__ double offh[kMaxChunks], offl[kMaxChunks];
    __shared__ double prs[KD][kWave];
    const int S = wave_uniform(blockDim.x / kWave);
    const int lane = lane_id();
    const int w = wave_uniform(threadIdx.x / kWave);
    const int tile = static_cast<int>(blockIdx.x) / G;
    const int grp = static_cast<int>(blockIdx.x) - tile * G;
    const int p = tile * kWave + lane;
    const int pc = p < N ? p : N - 1;
    const int64_t nsl = static_cast<int64_t>(S) * G;
    const int sl = grp * S + w;
    const int j0 = wave_uniform(static_cast<int>((static_cast<int64_t>(n) * sl) / nsl));
    const int j1 = wave_uniform(static_cast<int>((static_cast<int64_t>(n) * (sl + 1)) / nsl));
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    if (ms.t_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0)
        *ms.t_out = static_cast<int>(step);
    const bool fused = (ms.cdf_hi != nullptr) && (ms.state != nullptr) && (ms.state->resampled != 0);
    if (fused) fused_ancestors(ms, N, step, pc, anc, offh, offl);
    const MoveSource srcs = move_source(ms, theta, l);
    const int a = fused ? anc[lane] : pc;

    double pr[KD];
    block_proposals<KD>(seed, static_cast<uint32_t>(pc), step, move, srcs.th, N, a, sd, w, S, prs,
                        pr);
    red[w][lane] = slice_partial<K, D, PREC>(y, j0, j1, pr, g);
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
    bool acc = false;
    if (p < N) {
        double tot = red[0][lane];
        for (int s = 1; s < S; ++s) tot += red[s][lane];
        const double l_prop = finish_loglik<PREC>(tot, n, g);
        acc = rwmh_accept<KD>(p, a, N, [&](int c) { return pr[c]; }, l_prop, srcs, theta, l,
                              beta_vec, src, step, seed, move, g, status, ms);
    }
    const unsigned long long mask = __ballot(acc);
    if (lane == 0 && n_acc != nullptr && mask != 0ull)
        atomicAdd(n_acc, static_cast<unsigned long long>(__popcll(mask)));
}

// Second half of a move whose tile data were split over G workgroups: one
// thread per particle adds the G partial sums in group order, re-forms the same
// proposal (same counter, same arithmetic) and takes the MH decision.
template <int KD, int PREC>
__global__ void __launch_bounds__(256)
k_rwmh_accept(int n, double* theta, double* l, int N, const double* __restrict__ beta_vec,
              StepSrc src, double sd, uint64_t seed, uint32_t move, GmmDev g,
              unsigned long long* n_acc, int* status, MoveStep ms, int G,
              const double* __restrict__ part, const int* __restrict__ anc_in) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    bool acc = false;
    if (p < N) {
        const bool fused =
            (ms.cdf_hi != nullptr) && (ms.state != nullptr) && (ms.state->resampled != 0);
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
        acc = rwmh_accept<KD>(p, a, N, [&](int c) { return pr[c]; }, l_prop, srcs, theta, l,
                              beta_vec, src, step, seed, move, g, status, ms);
    }
    const unsigned long long mask = __ballot(acc);
    if ((threadIdx.x & (kWave - 1)) == 0 && n_acc != nullptr && mask != 0ull)
        atomicAdd(n_acc, static_cast<unsigned long long>(__popcll(mask)));
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
    const dim3 grid(static_cast<unsigned>((N + kWave - 1) / kWave));
    const dim3 block(static_cast<unsigned>(kWave * slices));
#define SMC_CASE(K, D)                                                                        \
    if (g.k == K && g.d == D) {                                                               \
        if (prec == SMC_PREC_FP32)                                                            \
            hipLaunchKernelGGL((k_loglik<K, D, SMC_PREC_FP32>), grid, block, 0, s, y,         \
                               static_cast<int>(n), theta, static_cast<int>(N), g, out,       \
                               status);                                                       \
        else                                                                                  \
            hipLaunchKernelGGL((k_loglik<K, D, SMC_PREC_FP64>), grid, block, 0, s, y,         \
                               static_cast<int>(n), theta, static_cast<int>(N), g, out,       \
                               status);                                                       \
        return hipGetLastError();                                                             \
    }
    SMC_KD_CASES(SMC_CASE)
#undef SMC_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_rwmh(const GmmDev& g, const float* y, int64_t n, double* theta, double* l,
                       int64_t N, const double* beta_vec, StepSrc src, double sd,
                       uint64_t seed, uint32_t move, int prec,
                       unsigned long long* n_accept, Split sp, const Scratch& sc, MoveStep ms,
                       hipStream_t s) {
    const int G = sp.groups;
    if (G < 1 || G > kMaxGroups || sp.slices < 1 || sp.slices > kMaxSlices ||
        (G > 1 && N > kSplitCap))
        return hipErrorInvalidValue;
    const int64_t tiles = (N + kWave - 1) / kWave;
    const dim3 grid(static_cast<unsigned>(tiles * G));
    const dim3 block(static_cast<unsigned>(kWave * sp.slices));
    const dim3 agrid(static_cast<unsigned>((N + 255) / 256));
    const int n32 = static_cast<int>(n), N32 = static_cast<int>(N);
#define SMC_MOVE(K, D, P)                                                                     \
    do {                                                                                      \
        hipLaunchKernelGGL((k_rwmh<K, D, P>), grid, block, 0, s, y, n32, theta, l, N32,       \
                           beta_vec, src, sd, seed, move, g, n_accept, sc.status, ms, G,      \
                           sc.mv_part, sc.mv_anc);                                            \
        if (G > 1)                                                                            \
            hipLaunchKernelGGL((k_rwmh_accept<K * D, P>), agrid, dim3(256), 0, s, n32, theta, \
                               l, N32, beta_vec, src, sd, seed, move, g, n_accept, sc.status, \
                               ms, G, static_cast<const double*>(sc.mv_part),                 \
                               static_cast<const int*>(sc.mv_anc));                           \
    } while (0)
#define SMC_CASE(K, D)                                                                        \
    if (g.k == K && g.d == D) {                                                               \
        if (prec == SMC_PREC_FP32) SMC_MOVE(K, D, SMC_PREC_FP32);                             \
        else SMC_MOVE(K, D, SMC_PREC_FP64);                                                   \
        return hipGetLastError();                                                             \
    }
    SMC_KD_CASES(SMC_CASE)
#undef SMC_CASE
#undef SMC_MOVE
    return hipErrorInvalidValue;
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

}  // namespace smc
