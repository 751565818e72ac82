// Device helpers shared by the mixture likelihood kernels (VALU and MFMA forms).
#pragma once
#include "internal.hpp"
#include "philox.hpp"
#include "wave.hpp"

namespace smc {

constexpr double kLn2 = 0.6931471805599453;

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int PREC>
__device__ __forceinline__ double finish_loglik(double acc, int n, const GmmDev& g) {
    const double body = (PREC == SMC_PREC_FP32) ? kLn2 * acc : acc;
    return static_cast<double>(n) * g.cst + body;
}

// Metropolis-Hastings decision for particle p of a random-walk move and the
// write-back: log alpha = beta (l' - l) + log p0(theta') - log p0(theta); accept
// iff log alpha >= 0 or log u < log alpha, u from stream (p, 0, step, ACC, move).
// pr_at(c) returns coordinate c of the proposal. The prior terms are
// accumulated coordinate by coordinate in index order, the current state is
// re-read rather than held, and with the step duties of `ms` the current state
// comes from the gathered population when the ESS test fired and the step's
// normalised weight is published.
template <int KD, class PropAt>
__device__ __forceinline__ bool rwmh_accept(int p, int N, PropAt pr_at, double l_prop,
                                            double* theta, double* l, const double* beta_vec,
                                            const StepSrc& src, uint32_t step, uint64_t seed,
                                            uint32_t move, const GmmDev& g, int* status,
                                            const MoveStep& ms) {
    const bool use_alt = (ms.state != nullptr) && (ms.state->resampled != 0);
    const double* th_src = use_alt ? ms.theta_alt : theta;
    const double* l_src = use_alt ? ms.l_alt : l;
    const double l_cur = l_src[p];
    double lp_cur, lp_prop;
    if (g.prior == SMC_PRIOR_GAUSS) {
        const double den = 2.0 * g.pb * g.pb;
        lp_cur = 0.0;
        lp_prop = 0.0;
#pragma unroll
        for (int c = 0; c < KD; ++c) {
            const double zc = th_src[static_cast<size_t>(c) * N + p] - g.pa;
            const double zp = pr_at(c) - g.pa;
            lp_cur += g.lp_const - (zc * zc) / den;
            lp_prop += g.lp_const - (zp * zp) / den;
        }
    } else {
        bool in_cur = true, in_prop = true;
#pragma unroll
        for (int c = 0; c < KD; ++c) {
            const double xc = th_src[static_cast<size_t>(c) * N + p];
            const double xp = pr_at(c);
            in_cur = in_cur && (xc >= g.pa) && (xc <= g.pb);
            in_prop = in_prop && (xp >= g.pa) && (xp <= g.pb);
        }
        const double inside = -static_cast<double>(KD) * log(g.pb - g.pa);
        lp_cur = in_cur ? inside : -INFINITY;
        lp_prop = in_prop ? inside : -INFINITY;
    }
    const double beta = beta_vec ? beta_vec[p]
                                 : (src.beta_dev ? src.beta_dev[step] : src.beta_host);
    const double la = beta * (l_prop - l_cur) + (lp_prop - lp_cur);
    const double u = u01_open(draw(seed, static_cast<uint32_t>(p), 0, step, kAcc, move).w0);
    const bool acc = (la >= 0.0) || (log(u) < la);
    if (acc) {
#pragma unroll
        for (int c = 0; c < KD; ++c) theta[static_cast<size_t>(c) * N + p] = pr_at(c);
        l[p] = l_prop;
    } else if (use_alt) {
#pragma unroll
        for (int c = 0; c < KD; ++c)
            theta[static_cast<size_t>(c) * N + p] = th_src[static_cast<size_t>(c) * N + p];
        l[p] = l_cur;
    }
    if (l_prop != l_prop) atomicOr(status, kStatusNaN);
    if (ms.W_out) {
        ms.W_out[p] = use_alt ? 1.0 / static_cast<double>(N)
                              : exp(ms.logw[p] - ms.state->M) / ms.state->S;
    }
    return acc;
}

}  // namespace smc
