// Device helpers shared by the mixture likelihood kernels (VALU and MFMA forms).
#pragma once
#include <type_traits>

#include "cdf_search.hpp"
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

// Sum over data j in [j0, j1) of log2 sum_i 2^{a_ij}, a_ij = log2 w_i - s^2 ||y_j - mu_i||^2
// (FP32 per-datum arithmetic, FP64 result). Per-datum factors are multiplied
// into a running FP32 product that is renormalised (frexp) after each block of
// data, its exponents summed as integers. Three forms:
//  - pivot (1-D data with a staging row, slices of at least kPivotMinData
//    data): the slice goes window by window, 64 data at a time. In a window
//    with midpoint c and half-width h, each particle takes as its pivot p the
//    component with the largest exponent at c. The difference of two
//    exponents is linear in y, so
//      log2 sum_i 2^{a_ij} = a_pj + log2(1 + sum_{i != p} 2^{t_ij}),
//      t_ij = dX_i + dB_i (y_j - c),  dX_i = a_i(c) - a_p(c) <= 0,
//      dB_i = 2 s^2 (mu_i - mu_p),
//    and sum_j a_pj over the window follows in FP64 from two sums over the
//    window's data (of y_j - c and of its square) that every particle shares.
//    Per datum and particle that is at most K-1 FMAs, K-1 exp2, K-2 adds and
//    one FMA into the product: each particle orders its other components by
//    the largest t_ij the window can hold, and the wave takes only as many as
//    its neediest particle has that can reach 2^kPivotSkip (near the data
//    mostly the one or two nearest neighbours of the pivot; the terms left out
//    are below the factor's FP32 resolution). Every factor is at least 1, so
//    the product cannot
//    underflow; a window is taken when, for every particle of the wave, every
//    dX_i + |dB_i| h (the largest t_ij the window can hold) is at most
//    pivot_over_max<K>(), which keeps a block of 8 factors below 2^128. A window
//    that some particle fails (components far apart across a wide window, a
//    datum or parameter not finite) goes through the plain forms below. On
//    data in ascending order the windows are narrow and nearly all are
//    taken; on unordered data nearly none are;
//  - direct (weights of total mass <= 1): e_j = sum_i 2^{a_ij}. Every factor
//    is then <= 1, so the partial products only fall, and a block of 8 whose
//    product ends at or above 2^-100 had no factor or partial product in the
//    FP32 subnormal range: it is as accurate as the shifted form;
//  - shifted: each datum's sum is taken relative to its largest term
//    m_j = max_i a_ij (blocks of 16), and the m_j are added apart.
// The plain forms: a wave starts in the direct form when every lane's `near`
// hint holds (the caller's guess that the particle sits near the data, from
// its current log-likelihood) and, at the first block where any of its lanes
// ends below 2^-100 (a particle far from these data, or a NaN), drops that
// block and takes the shifted form for the rest of its slice; otherwise it
// takes the shifted form throughout. All forms are within the FP32 error
// bound; which one a particle's data went through depends on the wave it
// shares (fixed for a given launch shape, population and data order). j0 and
// j1 must be the same in every lane of the wave, and every lane of the wave
// must take part (the forms use cross-lane operations, scalar loads and the
// wave's LDS row). With form_ctr set (kFormCounts arrays of kFormSlots
// counters), a wave adds to slot `slot` of each array (one atomic per nonzero
// count, slots spread so that waves rarely share one): [0] the number of data
// it took in the plain shifted form, counted up to the last full block of 8
// of each range the plain forms took (a whole slice, or a refused window; the
// fewer than 8 data after such a range's last full block always take the
// shifted form and are not counted); [1] the number of data it took in the
// pivot form; [2] the sum over those data of the number of other components
// the pivot form evaluated for them.
constexpr int kFormSlots = 1024;
constexpr int kFormCounts = 3;
// Data per window of the pivot form (one per lane), and the floats of a wave's
// staging row (two windows).
constexpr int kPivotWin = kWave;
constexpr int kPivotRow = 2 * kPivotWin;
// Shortest slice that takes the pivot form. Short slices come from short data
// (the paper's runs have 100 observations), whose windows of 64 span most of
// the data's range: the pivot form refuses nearly all of them, and trying cost
// 5-8% there.
constexpr int kPivotMinData = 128;
// Largest t_ij a window of the pivot form may hold with K components: a
// factor is then below 1 + (K-1) 2^T, and a block of 8 factors times a
// mantissa below 1 stays below the FP32 overflow at 2^128:
// (1 + 3 * 2^14)^8 < 2^125 for K <= 4, (1 + 7 * 2^13)^8 < 2^127 for K <= 8.
template <int K>
constexpr float pivot_over_max() {
    static_assert(K <= 8, "pivot_over_max assumes at most 8 components");
    return K <= 4 ? 14.0f : 13.0f;
}
static_assert(SMC_KMAX <= 8, "pivot_over_max assumes at most 8 components");
// A component other than the pivot whose t_ij stays below this in a window
// for every particle of the wave is left out there: its term is below 2^-25,
// under half the relative resolution of the product update p (1 + e) it would
// join (at most 7 such terms, so a datum's log2 factor is short by less than
// 3.1e-7, of the order of that update's own rounding).
constexpr float kPivotSkip = -25.0f;

// Calls f(std::integral_constant<int, m>) for a wave-uniform m in [0, M].
template <int M, class F>
__device__ __forceinline__ void with_count(int m, F&& f) {
    if constexpr (M == 0) {
        f(std::integral_constant<int, 0>{});
    } else {
        if (m == M) f(std::integral_constant<int, M>{});
        else with_count<M - 1>(m, f);
    }
}

// A wave's staging for the pivot form: its LDS row of kPivotRow floats
// (nullptr: plain forms only) and, when `pre` is set, each lane's datum
// y[j0 + lane] of its slice already loaded where j0 + lane < j1 (a caller may
// issue that load early, ahead of other work).
struct PivotStage {
    float* row = nullptr;
    float y0 = 0.0f;
    bool pre = false;
};

// The data slice [j0, j1) of slice sl out of nsl over n data (the same in
// every lane). Slices of at least 64 data start on multiples of 8, the FP32
// forms' blocks, so that only a slice ending at n can end in a partial block.
__device__ __forceinline__ void slice_bounds(int n, int sl, int nsl, int& j0, int& j1) {
    const int a = static_cast<int>((static_cast<int64_t>(n) * sl) / nsl);
    const int b = static_cast<int>((static_cast<int64_t>(n) * (sl + 1)) / nsl);
    const bool blocks = static_cast<int64_t>(n) >= static_cast<int64_t>(64) * nsl;
    j0 = wave_uniform(blocks ? a & ~7 : a);
    j1 = wave_uniform(blocks && sl + 1 < nsl ? b & ~7 : b);
}

// Data counts of one wave's slice by form (the form counters of partial_fp32).
struct FormCount {
    int shifted = 0;           // in the plain shifted form (up to full blocks of 8)
    int pivot = 0;             // in the pivot form
    int terms = 0;             // other components evaluated, summed over pivot data
};

// The pivot form over the 1-D slice [j0, j1) (see partial_fp32): adds the
// slice's terms to prod, expo and msum and its data counts to fc. nms[i] =
// -s mu_i in FP32; plain(ja, jb) runs the plain forms over [ja, jb) and
// returns the count of data they took in the shifted form.
template <int K, class Plain>
__device__ __forceinline__ void pivot_slice(const float* __restrict__ y, int j0, int j1,
                                            const double (&mu)[K], const GmmDev& g,
                                            const float (&nms)[K], const PivotStage& st,
                                            float& prod, int& expo, double& msum, FormCount& fc,
                                            Plain&& plain) {
    constexpr double kLog2eD = 1.4426950408889634;
    constexpr int KO = K > 1 ? K - 1 : 1;
    const int lane = lane_id();
    const float s = g.s32;
    const double s2 = g.inv2s2 * kLog2eD;
    float* row = st.row;
    float beta[K];
#pragma unroll
    for (int i = 0; i < K; ++i) beta[i] = static_cast<float>(2.0 * s2 * mu[i]);
    // each lane's datum of the current window and of the next one, loaded a
    // window ahead of their use
    float ycur = st.pre ? st.y0 : (j0 + lane < j1 ? y[j0 + lane] : 0.0f);
    float ynext = j0 + kPivotWin + lane < j1 ? y[j0 + kPivotWin + lane] : 0.0f;
    // the pivot of each lane for a window with midpoint c and half-width h:
    // the others' offsets dX, slopes dB and largest offsets ub, and the pivot's
    // mean and log-weight; ok when no lane's ub passes pivot_over_max<K>() (and h is
    // finite)
    float dX[KO], dB[KO], ub[KO];
    double mp = 0.0, lwp = 0.0;
    auto choose = [&](float c, float h) {
        float a[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const float t = __builtin_fmaf(c, s, nms[i]);
            a[i] = __builtin_fmaf(-t, t, g.lw2[i]);
        }
        int piv = 0;
        float best = a[0];
#pragma unroll
        for (int i = 1; i < K; ++i) {
            const bool up = a[i] > best;
            best = up ? a[i] : best;
            piv = up ? i : piv;
        }
        float bp = beta[0];
        mp = mu[0];
        lwp = g.lw[0];
#pragma unroll
        for (int i = 1; i < K; ++i) {
            const bool at = piv == i;
            bp = at ? beta[i] : bp;
            mp = at ? mu[i] : mp;
            lwp = at ? g.lw[i] : lwp;
        }
        bool ok = h <= 3.0e38f;               // false for a datum not finite
#pragma unroll
        for (int o = 0; o + 1 < K; ++o) {
            const bool up = o >= piv;
            dX[o] = (up ? a[o + 1] : a[o]) - best;
            dB[o] = (up ? beta[o + 1] : beta[o]) - bp;
            ub[o] = __builtin_fmaf(fabsf(dB[o]), h, dX[o]);
            ok &= ub[o] <= pivot_over_max<K>();
        }
        return __all(ok);
    };
    // while it works, two windows at a time share one choice of pivots
    bool pairs = true;
    for (int wb = j0; wb < j1;) {
        const int left = j1 - wb;
        const int nw0 = wave_uniform(left < kPivotWin ? left : kPivotWin);
        const int nw1 = wave_uniform(left > kPivotWin ? (left - kPivotWin < kPivotWin
                                                             ? left - kPivotWin : kPivotWin) : 0);
        const float v0 = ycur, v1 = ynext;
        const bool in0 = lane < nw0, in1 = lane < nw1;
        int nw = 0;
        float c = 0.0f, S1 = 0.0f, S2 = 0.0f;
        if (pairs && nw1 > 0) {
            // the pair's range and its data sums about its midpoint (all lanes)
            const int k0 = float_order_key(v0);
            const int k1 = in1 ? float_order_key(v1) : INT_MAX;
            const int k1x = in1 ? float_order_key(v1) : INT_MIN;
            const float lo = float_of_order_key(wave_extreme_key<false>(k0 < k1 ? k0 : k1));
            const float hi = float_of_order_key(wave_extreme_key<true>(k0 > k1x ? k0 : k1x));
            c = 0.5f * lo + 0.5f * hi;
            const float h = 0.5f * hi - 0.5f * lo;
            if (choose(c, h)) {
                const float d0 = v0 - c;
                const float d1 = in1 ? v1 - c : 0.0f;
                S1 = wave_sum_dpp(d0 + d1);
                S2 = wave_sum_dpp(__builtin_fmaf(d1, d1, d0 * d0));
                wave_sync();                  // the previous window's reads come first
                row[lane] = d0;
                row[kPivotWin + lane] = d1;
                // the next two windows' data, in flight while these are consumed
                // (issued after these are used, so that no wait covers them)
                const int jn = wb + 2 * kPivotWin + lane;
                ycur = jn < j1 ? y[jn] : 0.0f;
                ynext = jn + kPivotWin < j1 ? y[jn + kPivotWin] : 0.0f;
                wave_sync();                  // the windows are written before they are read
                nw = nw0 + nw1;
            } else {
                pairs = false;
            }
        }
        if (nw == 0) {
            // one window: its range and data sums about its midpoint
            const float lo = wave_min_dpp(in0 ? v0 : INFINITY);
            const float hi = wave_max_dpp(in0 ? v0 : -INFINITY);
            c = 0.5f * lo + 0.5f * hi;
            const float h = 0.5f * hi - 0.5f * lo;
            const bool take = choose(c, h);
            const float d0 = in0 ? v0 - c : 0.0f;
            if (take) {
                S1 = wave_sum_dpp(d0);
                S2 = wave_sum_dpp(d0 * d0);
                wave_sync();
                row[lane] = d0;
            }
            // the window after next, in flight
            const int jn = wb + 2 * kPivotWin + lane;
            ycur = v1;
            ynext = jn < j1 ? y[jn] : 0.0f;
            if (!take) {
                fc.shifted += plain(wb, wb + nw0);
                wb += nw0;
                continue;
            }
            wave_sync();
            nw = nw0;
        }
        fc.pivot += nw;
        if constexpr (K > 1) {
            // each lane's others in decreasing order of ub (odd-even
            // transposition network); the wave takes as many of them as its
            // neediest lane has with ub >= kPivotSkip
#pragma unroll
            for (int r = 0; r < KO; ++r) {
#pragma unroll
                for (int o = r & 1; o + 1 < KO; o += 2) {
                    const bool sw = ub[o + 1] > ub[o];
                    const float u0 = ub[o], x0 = dX[o], b0 = dB[o];
                    ub[o] = sw ? ub[o + 1] : u0;
                    dX[o] = sw ? dX[o + 1] : x0;
                    dB[o] = sw ? dB[o + 1] : b0;
                    ub[o + 1] = sw ? u0 : ub[o + 1];
                    dX[o + 1] = sw ? x0 : dX[o + 1];
                    dB[o + 1] = sw ? b0 : dB[o + 1];
                }
            }
            int need = 0;
#pragma unroll
            for (int o = 0; o < KO; ++o) need += ub[o] >= kPivotSkip ? 1 : 0;
            int m = 0;
#pragma unroll
            for (int q = 1; q < K; ++q) m = __any(need >= q) ? q : m;
            m = wave_uniform(m);
            fc.terms += m * nw;
            with_count<KO>(m, [&](auto mc) {
                constexpr int M = decltype(mc)::value;
                if constexpr (M > 0) {
                    auto factor = [&](float p, float d) {
                        float e = __builtin_amdgcn_exp2f(__builtin_fmaf(d, dB[0], dX[0]));
#pragma unroll
                        for (int o = 1; o < M; ++o)
                            e += __builtin_amdgcn_exp2f(__builtin_fmaf(d, dB[o], dX[o]));
                        return __builtin_fmaf(p, e, p);
                    };
                    int u = 0;
                    for (; u + 8 <= nw; u += 8) {
                        float p = prod;
#pragma unroll
                        for (int q = 0; q < 8; q += 4) {
                            const float4 d4 = *reinterpret_cast<const float4*>(row + u + q);
                            p = factor(p, d4.x);
                            p = factor(p, d4.y);
                            p = factor(p, d4.z);
                            p = factor(p, d4.w);
                        }
                        expo += __builtin_amdgcn_frexp_expf(p);
                        prod = __builtin_amdgcn_frexp_mantf(p);
                    }
                    if (u < nw) {
                        float p = prod;
                        for (; u < nw; ++u) p = factor(p, row[u]);
                        expo += __builtin_amdgcn_frexp_expf(p);
                        prod = __builtin_amdgcn_frexp_mantf(p);
                    }
                }
            });
        }
        // the pivots' own terms over the window(s), in FP64
        const double d = static_cast<double>(c) - mp;
        const double sq = static_cast<double>(S2) +
                          d * (2.0 * static_cast<double>(S1) + static_cast<double>(nw) * d);
        msum += static_cast<double>(nw) * lwp * kLog2eD - s2 * sq;
        wb += nw;
    }
}

template <int K, int D>
__device__ __forceinline__ double partial_fp32(const float* __restrict__ y, int j0, int j1,
                                               const double (&mu)[K * D], const GmmDev& g,
                                               bool near, const PivotStage& st,
                                               unsigned long long* form_ctr = nullptr) {
    constexpr int UF = 8;            // direct-form block
    constexpr int US = 16;           // shifted-form block
    constexpr float kFloor = 0x1p-100f;
    const float s = g.s32;
    double msum = 0.0;
    float prod = 1.0f;
    int expo = 0;
    float nms[K * D];                // -s mu in FP32
#pragma unroll
    for (int c = 0; c < K * D; ++c) nms[c] = static_cast<float>(-(static_cast<double>(s) * mu[c]));
    auto exponents = [&](const float* yj, float (&a)[K]) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            if constexpr (D == 1) {
                const float t = __builtin_fmaf(yj[0], s, nms[i]);
                a[i] = __builtin_fmaf(-t, t, g.lw2[i]);
            } else {
                float q = 0.0f;
#pragma unroll
                for (int c = 0; c < D; ++c) {
                    const float t = __builtin_fmaf(yj[c], s, nms[i * D + c]);
                    q = __builtin_fmaf(t, t, q);
                }
                a[i] = g.lw2[i] - q;
            }
        }
    };
    auto shifted = [&](const float* yj, float& m_out, float& e_out) {
        float a[K];
        exponents(yj, a);
        float m = a[0];
#pragma unroll
        for (int i = 1; i < K; ++i) m = fmaxf(m, a[i]);
        float e = __builtin_amdgcn_exp2f(a[0] - m);
#pragma unroll
        for (int i = 1; i < K; ++i) e += __builtin_amdgcn_exp2f(a[i] - m);
        m_out = m;
        e_out = e;
    };
    auto direct = [&](const float* yj) {
        float a[K];
        exponents(yj, a);
        float e = __builtin_amdgcn_exp2f(a[0]);
#pragma unroll
        for (int i = 1; i < K; ++i) e += __builtin_amdgcn_exp2f(a[i]);
        return e;
    };
    // the plain forms over [ja, jb); the direct form, once left, is not taken
    // again in this slice. Returns the data taken in the shifted form up to
    // the range's last full block of 8.
    bool take_direct = g.unit_mass != 0 && __all(near);
    auto plain = [&](int ja, int jb) {
        int j = ja;
        if (take_direct) {
            for (; j + UF <= jb; j += UF) {
                const float* yb = y + (size_t)wave_uniform(j) * D;    // wave-uniform: scalar loads
                float p = prod;
#pragma unroll
                for (int u = 0; u < UF; ++u) p *= direct(yb + u * D);
                if (!__all(p >= kFloor)) {
                    take_direct = false;
                    break;
                }
                expo += __builtin_amdgcn_frexp_expf(p);
                prod = __builtin_amdgcn_frexp_mantf(p);
            }
        }
        const int counted = ((jb - ja) & ~(UF - 1)) - (j - ja);
        for (; j + US <= jb; j += US) {
            float mblk = 0.0f;
#pragma unroll 8
            for (int u = 0; u < US; ++u) {
                float m, e;
                shifted(y + (size_t)(j + u) * D, m, e);
                prod *= e;
                mblk += m;
            }
            msum += static_cast<double>(mblk);
            expo += __builtin_amdgcn_frexp_expf(prod);
            prod = __builtin_amdgcn_frexp_mantf(prod);
        }
#pragma unroll 4
        for (; j < jb; ++j) {
            float m, e;
            shifted(y + (size_t)j * D, m, e);
            prod *= e;
            msum += static_cast<double>(m);
        }
        return counted;
    };
    FormCount fc;
    if constexpr (D == 1) {
        if (st.row != nullptr && j1 - j0 >= kPivotMinData)
            pivot_slice<K>(y, j0, j1, mu, g, nms, st, prod, expo, msum, fc, plain);
        else
            fc.shifted = plain(j0, j1);
    } else {
        fc.shifted = plain(j0, j1);
    }
    if (form_ctr != nullptr && lane_id() == 0) {
        const int slot = (static_cast<int>(blockIdx.x) * (static_cast<int>(blockDim.x) >> 6) +
                          wave_id()) & (kFormSlots - 1);
        const int cnt[kFormCounts] = {fc.shifted, fc.pivot, fc.terms};
#pragma unroll
        for (int c = 0; c < kFormCounts; ++c)
            if (cnt[c] > 0)
                atomicAdd(form_ctr + c * kFormSlots + slot, static_cast<unsigned long long>(cnt[c]));
    }
    // the product's mantissa in [0.5, 1): its hardware log2 is within 2^-23 of
    // the exact value, far below the bound per slice
    expo += __builtin_amdgcn_frexp_expf(prod);
    prod = __builtin_amdgcn_frexp_mantf(prod);
    return msum + static_cast<double>(expo) + static_cast<double>(__builtin_amdgcn_logf(prod));
}

// Sum over data j in [j0, j1) of ln sum_i w_i exp(-||y_j - mu_i||^2 / (2 sigma2)), FP64.
template <int K, int D>
__device__ __forceinline__ double partial_fp64(const float* __restrict__ y, int j0, int j1,
                                               const double (&mu)[K * D], const GmmDev& g) {
    double acc = 0.0;
    for (int j = j0; j < j1; ++j) {
        const float* yj = y + (size_t)j * D;
        double a[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            double q = 0.0;
#pragma unroll
            for (int c = 0; c < D; ++c) {
                const double t = static_cast<double>(yj[c]) - mu[i * D + c];
                q += t * t;
            }
            a[i] = g.lw[i] - q * g.inv2s2;
        }
        double m = a[0];
#pragma unroll
        for (int i = 1; i < K; ++i) m = fmax(m, a[i]);
        double e = 0.0;
#pragma unroll
        for (int i = 0; i < K; ++i) e += exp(a[i] - m);
        acc += m + log(e);
    }
    return acc;
}

// Whether a particle with log-likelihood l over n data sits near the data in
// the sense the FP32 direct form needs: its per-datum mixture sums average at
// least 2^-6 (blocks of 8 then stay far above 2^-100). False for NaN and -inf.
__device__ __forceinline__ bool near_data(double l, int n, const GmmDev& g) {
    return l >= static_cast<double>(n) * (g.cst - 6.0 * kLn2);
}

// The slice partial of one lane for parameters pr[0..K*D-1] (FP64 values);
// `near` is the hint of partial_fp32 and `st` the wave's staging for the
// pivot form; both unused in FP64.
template <int K, int D, int PREC>
__device__ __forceinline__ double slice_partial(const float* __restrict__ y, int j0, int j1,
                                                const double (&pr)[K * D], const GmmDev& g,
                                                bool near = true, const PivotStage& st = {},
                                                unsigned long long* form_ctr = nullptr) {
    if constexpr (PREC == SMC_PREC_FP32) {
        return partial_fp32<K, D>(y, j0, j1, pr, g, near, st, form_ctr);
    } else {
        return partial_fp64<K, D>(y, j0, j1, pr, g);
    }
}

// This wave's staging row for the pivot form in a kernel of at most W waves
// per workgroup (a static LDS array of that kernel), or nullptr where the form
// does not apply (FP64, d > 1).
template <int PREC, int D, int W>
__device__ __forceinline__ float* pivot_row() {
    if constexpr (PREC == SMC_PREC_FP32 && D == 1) {
        __shared__ __align__(16) float win[W][kPivotRow];
        return win[wave_id()];
    } else {
        return nullptr;
    }
}

// Random-walk proposals th_src[:, a] + sd * z for the 64 particles of a
// workgroup. The ceil(KD/2) Box-Muller pairs of each particle are shared out
// over the block's nw waves (pair q: Philox block q/2, words 0-1 for even q and
// 2-3 for odd q, normals 2q and 2q+1) and exchanged through LDS, so no wave
// repeats another's draws. Cooperative: every thread of the block calls it (it
// contains one barrier); prs holds KD rows of 64 doubles. With hold set, the
// current state is kept in LDS for the decision as well: hold[c] (KD rows of 64
// doubles) gets th_src[c, a] and hold_l the current log-likelihood l_src[a]
// (read by the block's last wave), so the decision after the likelihood does
// not wait on global loads.
template <int KD>
__device__ __forceinline__ void block_proposals(uint64_t seed, uint32_t index, uint32_t step,
                                                uint32_t move, const double* th_src, int N,
                                                int a, double sd, int w, int nw,
                                                double (*prs)[kWave], double (&pr)[KD],
                                                double (*hold)[kWave] = nullptr,
                                                const double* l_src = nullptr,
                                                double* hold_l = nullptr) {
    const int lane = lane_id();
    if (hold != nullptr && w == nw - 1) hold_l[lane] = l_src[a];
    for (int q = w; q < (KD + 1) / 2; q += nw) {
        const int c = 2 * q;
        const double t0 = th_src[static_cast<size_t>(c) * N + a];
        const double t1 = c + 1 < KD ? th_src[static_cast<size_t>(c + 1) * N + a] : 0.0;
        const Words4 wd = draw(seed, index, static_cast<uint32_t>(q / 2), step, kProp, move);
        double z0, z1;
        if (q & 1) box_muller(wd.w2, wd.w3, z0, z1);
        else box_muller(wd.w0, wd.w1, z0, z1);
        prs[c][lane] = t0 + sd * z0;
        if (c + 1 < KD) prs[c + 1][lane] = t1 + sd * z1;
        if (hold != nullptr) {
            hold[c][lane] = t0;
            if (c + 1 < KD) hold[c + 1][lane] = t1;
        }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < KD; ++c) pr[c] = prs[c][lane];
}

// Source of a move's current state for the arrays (theta, l) it writes.
struct MoveSource {
    const double* th;
    const double* l;
    bool write_always;         // out of place: rejected particles are copied too
};

__device__ __forceinline__ MoveSource move_source(const MoveStep& ms, double* theta, double* l) {
    const bool rs = (ms.state != nullptr) && (ms.state->resampled != 0);
    if (rs && ms.theta_alt != nullptr) return MoveSource{ms.theta_alt, ms.l_alt, true};
    const double* th = ms.theta_src ? ms.theta_src : theta;
    const double* ll = ms.l_src ? ms.l_src : l;
    return MoveSource{th, ll, th != theta};
}

// Ancestors of the 64 particles of this workgroup after systematic resampling
// (cooperative: every thread of the block must call it). Wave 0 forms the chunk
// offsets in LDS (exclusive double-double scan of the chunk totals; offh and
// offl hold ms.nchunks entries each), then each of its lanes takes the
// scheme's point U_i for particle i and finds idx = min{j : U < C_j} (or the
// first j with C_j = C_{N-1}), C_j = offset + within-chunk prefix rounded once.
__device__ __forceinline__ void fused_ancestors(const MoveStep& ms, int N, uint32_t step, int pc,
                                                int* anc, double* offh, double* offl) {
    const int lane = lane_id();
    if (wave_id() == 0) {
        // two passes over the lane's chunk totals (sum, then running offsets)
        // keep the register footprint of this prologue small
        const int per = wave_uniform((ms.nchunks + kWave - 1) / kWave);
        dd run = dd_zero();
        for (int q = 0; q < per; ++q) {
            const int c = lane * per + q;
            if (c < ms.nchunks) run = dd_add(run, dd{ms.chunk_tot[2 * c], ms.chunk_tot[2 * c + 1]});
        }
        dd inc = run;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const dd up{__shfl_up(inc.hi, o, kWave), __shfl_up(inc.lo, o, kWave)};
            if (lane >= o) inc = dd_add(up, inc);
        }
        dd excl{__shfl_up(inc.hi, 1, kWave), __shfl_up(inc.lo, 1, kWave)};
        if (lane == 0) excl = dd_zero();
        for (int q = 0; q < per; ++q) {
            const int c = lane * per + q;
            if (c < ms.nchunks) {
                offh[c] = excl.hi;
                offl[c] = excl.lo;
                excl = dd_add(excl, dd{ms.chunk_tot[2 * c], ms.chunk_tot[2 * c + 1]});
            }
        }
    }
    __syncthreads();
    if (wave_id() == 0) {
        const double u = ms.scheme == 0 ? u01_left_closed(draw(ms.seed, 0, 0, step, kResamp, 0).w0)
                                        : 0.0;
        // pc is clamped to N - 1 past the end, so the tile's points are sorted
        // for the systematic and stratified schemes
        const double U = resample_point(ms.scheme, ms.seed, step, pc, N, u);
        anc[lane] = ms.scheme == SMC_RESAMPLE_MULTINOMIAL
                        ? cdf_search(U, N, ms.chunk, ms.cdf_hi, ms.cdf_lo, offh, offl)
                        : cdf_search_sorted_wave(U, true, N, ms.chunk, ms.cdf_hi, ms.cdf_lo, offh,
                                                 offl);
    }
    __syncthreads();
}

// Metropolis-Hastings log acceptance ratio for particle p of a random-walk
// move: log alpha = beta (l' - l) + log p0(theta') - log p0(theta).
// cur_at(c) / pr_at(c) return coordinate c of the current state / proposal;
// the prior terms are accumulated coordinate by coordinate in index order.
template <int KD, class PropAt, class CurAt>
__device__ __forceinline__ double rwmh_log_alpha(int p, PropAt pr_at, CurAt cur_at, double l_cur,
                                                 double l_prop, const double* beta_vec,
                                                 const StepSrc& src, uint32_t step,
                                                 const GmmDev& g) {
    double lp_cur, lp_prop;
    if (g.prior == SMC_PRIOR_GAUSS) {
        const double den = 2.0 * g.pb * g.pb;
        lp_cur = 0.0;
        lp_prop = 0.0;
#pragma unroll
        for (int c = 0; c < KD; ++c) {
            const double zc = cur_at(c) - g.pa;
            const double zp = pr_at(c) - g.pa;
            lp_cur += g.lp_const - (zc * zc) / den;
            lp_prop += g.lp_const - (zp * zp) / den;
        }
    } else {
        bool in_cur = true, in_prop = true;
#pragma unroll
        for (int c = 0; c < KD; ++c) {
            const double xc = cur_at(c);
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
    return beta * (l_prop - l_cur) + (lp_prop - lp_cur);
}

// log u of the acceptance test of particle p, u from stream (p, 0, step, ACC, move).
__device__ __forceinline__ double rwmh_log_u(int p, uint32_t step, uint64_t seed, uint32_t move) {
    return log(u01_open(draw(seed, static_cast<uint32_t>(p), 0, step, kAcc, move).w0));
}

// Metropolis-Hastings decision: accept iff log alpha >= 0 or log u < log alpha.
template <int KD, class PropAt, class CurAt>
__device__ __forceinline__ bool rwmh_decide(int p, PropAt pr_at, CurAt cur_at, double l_cur,
                                            double l_prop, const double* beta_vec,
                                            const StepSrc& src, uint32_t step, uint64_t seed,
                                            uint32_t move, const GmmDev& g) {
    const double la = rwmh_log_alpha<KD>(p, pr_at, cur_at, l_cur, l_prop, beta_vec, src, step, g);
    return (la >= 0.0) || (rwmh_log_u(p, step, seed, move) < la);
}

// The step duties of a move's first launch: publish W (1/N after resampling)
// and reset logw after resampling (in place, or into logw_out).
__device__ __forceinline__ void move_duties(int p, int N, const MoveStep& ms) {
    const bool rs = (ms.state != nullptr) && (ms.state->resampled != 0);
    if (ms.W_out) {
        ms.W_out[p] = rs ? 1.0 / static_cast<double>(N)
                         : exp(ms.logw[p] - ms.state->M) / ms.state->S;
    }
    if (ms.logw_out) ms.logw_out[p] = rs ? 0.0 : ms.logw[p];
    else if (rs && ms.reset_logw) ms.logw[p] = 0.0;
}

// Decision and write-back of particle p of a random-walk move, its current
// state given by cur_at(c) and l_cur; pr_at(c) returns coordinate c of the
// proposal. Rejected particles are copied when the move is out of place
// (write_always). l_new (optional) receives the particle's log-likelihood after
// the move.
template <int KD, class PropAt, class CurAt>
__device__ __forceinline__ bool rwmh_accept_state(int p, int N, PropAt pr_at, CurAt cur_at,
                                                  double l_cur, double l_prop, bool write_always,
                                                  double* theta, double* l,
                                                  const double* beta_vec, const StepSrc& src,
                                                  uint32_t step, uint64_t seed, uint32_t move,
                                                  const GmmDev& g, int* status,
                                                  const MoveStep& ms, double* l_new = nullptr) {
    const bool acc = rwmh_decide<KD>(p, pr_at, cur_at, l_cur, l_prop, beta_vec, src, step, seed,
                                     move, g);
    if (acc) {
#pragma unroll
        for (int c = 0; c < KD; ++c) theta[static_cast<size_t>(c) * N + p] = pr_at(c);
        l[p] = l_prop;
    } else if (write_always) {
#pragma unroll
        for (int c = 0; c < KD; ++c) theta[static_cast<size_t>(c) * N + p] = cur_at(c);
        l[p] = l_cur;
    }
    if (l_prop != l_prop) atomicOr(status, kStatusNaN);
    move_duties(p, N, ms);
    if (l_new) *l_new = acc ? l_prop : l_cur;
    return acc;
}

// rwmh_accept_state with the current state read from column a of (th_src,
// l_src) (a = p, or p's ancestor after a fused resampling).
template <int KD, class PropAt>
__device__ __forceinline__ bool rwmh_accept(int p, int a, int N, PropAt pr_at, double l_prop,
                                            const MoveSource& srcs, double* theta, double* l,
                                            const double* beta_vec, const StepSrc& src,
                                            uint32_t step, uint64_t seed, uint32_t move,
                                            const GmmDev& g, int* status, const MoveStep& ms,
                                            double* l_new = nullptr) {
    const double* th_src = srcs.th;
    return rwmh_accept_state<KD>(
        p, N, pr_at, [&](int c) { return th_src[static_cast<size_t>(c) * N + a]; }, srcs.l[a],
        l_prop, srcs.write_always, theta, l, beta_vec, src, step, seed, move, g, status, ms,
        l_new);
}

}  // namespace smc
