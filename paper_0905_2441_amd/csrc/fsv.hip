// Bootstrap particle filter for the factor stochastic-volatility model
// (Factor Stochastic Volatility subsection) on gfx950.
//
// One thread per particle (grid-stride, at most kMaxRedBlocks workgroups so the
// step's combine kernel reads one partial per workgroup):
//   x_t = Phi x_{t-1} + L z          L = chol(U), z the Philox normals of (p, 0, t, PROP, 0)
//   Sigma = B diag(exp(x_t)) B^T + diag(psi)       (M x M, FP64, registers)
//   log g = -(M/2) ln 2 pi - ln prod_i L_ii - |L^{-1} y_t|^2 / 2    (Cholesky, forward solve)
//   logw += log g, with the running log-sum-exp of the old and new log-weights
//   and the new-weight sums of x and x^2 per thread, combined per workgroup.
// The arithmetic per particle is ~300 FP64 operations and 56 bytes of HBM
// traffic (read x, logw; write x_t, logw), so a step is launch-latency bound
// up to N of a few million; the paper's observation that this filter gains
// less than the mixture sampler (resampling nearly every step, matrix work per
// particle) shows here as a smaller share of the time in arithmetic.
#include "fsv.hpp"
#include "philox.hpp"
#include "reduce.hpp"
#include "cdf_search.hpp"

namespace smc {
namespace {

template <int KF>
struct Moments {
    double m, s;               // running max and sum of exp(lw - m)
    double sx[KF], sxx[KF];    // sums of exp(lw - m) x and exp(lw - m) x^2
};

template <int KF>
__device__ __forceinline__ void moments_push(Moments<KF>& a, double lw, const double (&x)[KF]) {
    if (lw == -INFINITY) return;
    const double d = lw - a.m;
    const double e = exp(-fabs(d));
    const bool up = d > 0.0;
    a.m = up ? lw : a.m;
    a.s = up ? a.s * e + 1.0 : a.s + e;
#pragma unroll
    for (int c = 0; c < KF; ++c) {
        const double w = up ? 1.0 : e;
        const double r = up ? e : 1.0;
        a.sx[c] = a.sx[c] * r + w * x[c];
        a.sxx[c] = a.sxx[c] * r + w * x[c] * x[c];
    }
}

template <int MO, int KF>
__global__ void __launch_bounds__(kRedBlock)
k_fsv_weight(FsvDev f, const double* __restrict__ y, int T, const double* __restrict__ x,
             double* __restrict__ x_out, double* __restrict__ logw, int N, StepSrc src,
             uint64_t seed, Scratch sc, double* __restrict__ mom, FsvAnc anc) {
    __shared__ double offh[kMaxChunks], offl[kMaxChunks];
    const uint32_t t = static_cast<uint32_t>(step_index(src));
    // the previous step's resampling (one value for the whole grid), searched
    // exactly as the standalone search-and-gather pass does
    const bool rs = anc.state != nullptr && anc.state->resampled != 0;
    uint32_t rs_step = 0;
    double rs_u = 0.0;
    if (rs) {
        block_cdf_offsets(anc.chunk_tot, anc.nchunks, offh, offl);
        rs_step = static_cast<uint32_t>(anc.state->t);
        if (anc.scheme == 0) rs_u = u01_left_closed(draw(seed, 0, 0, rs_step, kResamp, 0).w0);
    }
    const double* yt = y + static_cast<size_t>(t - 1) * MO;
    double yv[MO];
#pragma unroll
    for (int a = 0; a < MO; ++a) yv[a] = yt[a];
    Lse3 o = lse3_empty(), nw = lse3_empty();
    Moments<KF> mo;
    mo.m = -INFINITY;
    mo.s = 0.0;
#pragma unroll
    for (int c = 0; c < KF; ++c) mo.sx[c] = mo.sxx[c] = 0.0;
    bool bad = false;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < N; p += gridDim.x * blockDim.x) {
        const int a = rs ? cdf_search(resample_point(anc.scheme, seed, rs_step, p, N, rs_u), N,
                                      anc.chunk, anc.cdf_hi, anc.cdf_lo, offh, offl)
                         : p;
        double z[KF];
        normals<KF>(seed, static_cast<uint32_t>(p), t, kProp, 0, z);
        double xn[KF], h[KF];
#pragma unroll
        for (int c = 0; c < KF; ++c) {
            double v = f.phi[c] * x[static_cast<size_t>(c) * N + a];
#pragma unroll
            for (int j = 0; j <= c; ++j) v = fma(f.L[c * SMC_FSV_KMAX + j], z[j], v);
            xn[c] = v;
            h[c] = exp(v);
            x_out[static_cast<size_t>(c) * N + p] = v;
        }
        // Cholesky of Sigma = B diag(h) B^T + diag(psi), lower triangle, row by row
        double Lc[MO][MO];
        double prod = 1.0;
#pragma unroll
        for (int i = 0; i < MO; ++i) {
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                double sij = (i == j) ? f.psi[i] : 0.0;
#pragma unroll
                for (int c = 0; c < KF; ++c)
                    sij = fma(f.B[i * SMC_FSV_KMAX + c] * h[c], f.B[j * SMC_FSV_KMAX + c], sij);
#pragma unroll
                for (int q = 0; q < j; ++q) sij = fma(-Lc[i][q], Lc[j][q], sij);
                if (i == j) {
                    Lc[i][i] = sqrt(sij);
                    prod *= Lc[i][i];
                } else {
                    Lc[i][j] = sij / Lc[j][j];
                }
            }
        }
        // forward solve L v = y and the quadratic form |v|^2
        double v[MO];
        double quad = 0.0;
#pragma unroll
        for (int i = 0; i < MO; ++i) {
            double r = yv[i];
#pragma unroll
            for (int q = 0; q < i; ++q) r = fma(-Lc[i][q], v[q], r);
            v[i] = r / Lc[i][i];
            quad = fma(v[i], v[i], quad);
        }
        const double lg = f.cst - log(prod) - 0.5 * quad;
        const double lo = rs ? 0.0 : logw[p];
        const double ln = lo + lg;
        logw[p] = ln;
        bad = bad || (ln != ln) || (ln == INFINITY);
        o = lse3_push(o, lo);
        nw = lse3_push(nw, ln);
        moments_push<KF>(mo, ln, xn);
    }
    if (bad) atomicOr(sc.status, kStatusNaN);
    o = block_lse3(o);
    nw = block_lse3(nw);
    // moment sums rescaled to the block maximum of the new log-weights (nw.m,
    // the same in every thread), then added in fixed order
    const double r = (mo.m == -INFINITY) ? 0.0 : exp(mo.m - nw.m);
    double acc[2 * KF];
#pragma unroll
    for (int c = 0; c < KF; ++c) {
        acc[c] = block_sum(mo.sx[c] * r);
        acc[KF + c] = block_sum(mo.sxx[c] * r);
    }
    if (threadIdx.x == 0) {
        sc.rw_part[blockIdx.x] = RwPartial{o.m, o.s1, nw.m, nw.s1, nw.s2, 0.0};
#pragma unroll
        for (int q = 0; q < 2 * KF; ++q) mom[static_cast<size_t>(blockIdx.x) * 2 * SMC_FSV_KMAX + q] = acc[q];
    }
}

__global__ void k_fsv_init(int k, int N, double* __restrict__ x, double* __restrict__ logw) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    for (int c = 0; c < k; ++c) x[static_cast<size_t>(c) * N + p] = 0.0;
    logw[p] = 0.0;
}

}  // namespace

#define SMC_FSV_CASES(X) X(5, 3) X(2, 2) X(1, 1)

bool fsv_supported(int m, int k) {
#define SMC_CASE(MO, KF) \
    if (m == MO && k == KF) return true;
    SMC_FSV_CASES(SMC_CASE)
#undef SMC_CASE
    return false;
}

int fsv_parts(int64_t N) {
    int64_t g = (N + kRedBlock - 1) / kRedBlock;
    if (g > kMaxRedBlocks) g = kMaxRedBlocks;
    return static_cast<int>(g < 1 ? 1 : g);
}

hipError_t launch_fsv_init(int k, int64_t N, double* x, double* logw, hipStream_t s) {
    hipLaunchKernelGGL(k_fsv_init, dim3(static_cast<unsigned>((N + 255) / 256)), dim3(256), 0, s,
                       k, static_cast<int>(N), x, logw);
    return hipGetLastError();
}

hipError_t launch_fsv_weight(const FsvDev& f, const double* y, int T, const double* x,
                             double* x_out, double* logw, int64_t N, StepSrc src, uint64_t seed,
                             const Scratch& sc, double* mom, hipStream_t s, const FsvAnc& anc) {
    const dim3 grid(static_cast<unsigned>(fsv_parts(N)));
#define SMC_CASE(MO, KF)                                                                      \
    if (f.m == MO && f.k == KF) {                                                             \
        hipLaunchKernelGGL((k_fsv_weight<MO, KF>), grid, dim3(kRedBlock), 0, s, f, y, T, x,   \
                           x_out, logw, static_cast<int>(N), src, seed, sc, mom, anc);        \
        return hipGetLastError();                                                             \
    }
    SMC_FSV_CASES(SMC_CASE)
#undef SMC_CASE
    return hipErrorInvalidValue;
}

}  // namespace smc
