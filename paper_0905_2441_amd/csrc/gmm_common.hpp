// Device helpers shared by the mixture likelihood kernels (VALU and MFMA forms).
#pragma once
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
// (FP32 arithmetic, FP64 result). The per-datum sums are multiplied into a
// running product that is renormalised (frexp) after each block of data, its
// exponents summed as integers. Three forms:
//  - direct (weights of total mass <= 1): e_j = sum_i 2^{a_ij}. Every factor
//    is then <= 1, so the partial products only fall, and a block of 8 whose
//    product ends at or above 2^-100 had no factor or partial product in the
//    FP32 subnormal range: it is as accurate as the shifted form;
//  - expanded direct (1-D data, for the windows of 64 data whose every datum
//    keeps s^2 (y - c)^2 <= kExpQmax, c the midrange of the slice's first 64
//    data): the same e_j, computed from the split a_ij = x_ij - q_j
//    (expanded_direct below), one FMA and one exp2 per component instead of
//    two FMAs and an exp2; the direct form takes over from the first window
//    that does not keep it;
//  - shifted: each datum's sum is taken relative to its largest term
//    m_j = max_i a_ij (blocks of 16), and the m_j are added apart.
// A wave starts in a direct form when every lane's `near` hint holds (the
// caller's guess that the particle sits near the data, from its current
// log-likelihood) and, at the first block where any of its lanes ends below
// 2^-100 (a particle far from these data, or a NaN), drops that block and
// runs the rest of its slice in the shifted form; otherwise it runs the
// shifted form throughout. All forms are within the FP32 error bound; which
// one a particle's data went through depends on the wave it shares (fixed for
// a given launch shape and population). j0 and j1 must be the same in every
// lane of the wave, and every lane of the wave must take part (the data are
// read by scalar loads, or staged by the wave's lanes in LDS). With
// shifted_ctr set, a wave that left (or never took) the direct forms adds the
// number of data it then took in the shifted form, up to its slice's last
// full block of 8, to the counter slot shifted_ctr[slot] (one atomic per such
// wave, slots spread so that waves rarely share one; the fewer than 8 data
// after the last full block always take the shifted form and are not
// counted).
constexpr int kFormSlots = 1024;
// Data staged per window of the expanded forms (one per lane).
constexpr int kExpWin = kWave;
// Shortest slice that takes the expanded forms (below it their per-wave
// set-up, the centre and the FP64 B and C, costs more than they save).
constexpr int kExpMinData = 128;
// Largest s^2 (y - c)^2 for which a datum takes the expanded forms: their
// terms 2^{x_ij} then stay below 2^120 and the data factors above 2^-120, and
// |x_ij| < 128 bounds x_ij's rounding error by 2^-18.
constexpr double kExpQmax = 120.0;

// The expanded forms (1-D data). With c a data centre, y' = y - c (FP32) and
// m_i = mu_i - c,
//   a_ij = log2 w_i - s2 (y'_j - m_i)^2 = x_ij - q_j,
//   x_ij = C_i + B_i y'_j,  B_i = 2 s2 m_i,  C_i = log2 w_i - s2 m_i^2,
//   q_j = s2 y'_j^2,
// and q_j does not depend on the particle: one FMA per component gives x_ij,
// and each datum's log2 sum_i 2^{a_ij} follows from the x_ij and q_j.
// B_i and C_i are formed in FP64 and rounded once, C_i with B_i's rounding
// error at y' = m_i folded in, so that x_ij is exact up to its own rounding at
// the component's centre. The wave stages its data 64 at a time, one datum per
// lane (q in FP64), in its own row of LDS (`row`, 2 * kExpWin floats), and
// reads them back as broadcasts; each lane fetches its datum of the next
// window while the current one is consumed. A window holding a datum with
// q_j > kExpQmax (or not finite) ends a form at its start: this bounds the
// magnitude of x_ij and so its rounding error (and, in the direct form, keeps
// 2^{x_ij} finite and g_j normal).
// A wave's staging for the expanded forms: its LDS row of 2 * kExpWin floats
// (nullptr: plain forms only) and, when `pre` is set, each lane's datum
// y[j0 + lane] of its slice already loaded (a caller may issue that load early,
// ahead of other work).
struct ExpStage {
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

template <int K>
struct Expanded {
    double s2;                 // s^2 = log2(e) / (2 sigma2)
    float c;
    float B[K], C[K];
};

// c = the midrange of the data in [j0, jlim) (at most 64 of them) and the
// lane's B_i, C_i. False when those data are not all finite.
// v: the lane's datum y[j0 + lane] (unused past jlim).
template <int K>
__device__ __forceinline__ bool expanded_setup(float v, int j0, int jlim,
                                               const double (&mu)[K], const GmmDev& g,
                                               Expanded<K>& f) {
    constexpr double kLog2eD = 1.4426950408889634;
    const int jj = j0 + lane_id();
    const float lo = wave_min_dpp(jj < jlim ? v : INFINITY);
    const float hi = wave_max_dpp(jj < jlim ? v : -INFINITY);
    f.s2 = g.inv2s2 * kLog2eD;
    f.c = 0.5f * lo + 0.5f * hi;          // the same in every lane
    if (!(fabsf(f.c) <= 3.0e38f)) return false;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const double m = mu[i] - static_cast<double>(f.c);
        const double b = 2.0 * f.s2 * m;
        f.B[i] = static_cast<float>(b);
        f.C[i] = static_cast<float>(g.lw[i] * kLog2eD - f.s2 * m * m +
                                    (b - static_cast<double>(f.B[i])) * m);
    }
    return true;
}

// The expanded direct form over the blocks of 8 data from j to jend:
// e_j = g_j sum_i 2^{x_ij} with g_j = 2^{-q_j} (= 2^-round(q) times the
// hardware exp2 of the small remainder), staged as (y'_j, g_j) pairs. Updates
// prod and expo over the blocks it took and moves j past them; returns true
// when it stopped for the range (the caller goes on in the scalar-load direct
// form from j), false when it took every block or a block failed the 2^-100
// check (the caller goes on in the shifted forms). ycur: the lane's datum
// y[j + lane] (unused past jend).
template <int K>
__device__ __forceinline__ bool expanded_direct(const float* __restrict__ y, int jend,
                                                const Expanded<K>& f, float* row, float& prod,
                                                int& expo, int& j, float ycur) {
    constexpr float kFloor = 0x1p-100f;
    const int lane = lane_id();
    for (int wb = j; wb < jend; wb += kExpWin) {
        const int jj = wb + lane;
        bool ok = true;
        wave_sync();                          // the previous window's reads come first
        if (jj < jend) {
            const float yp = ycur - f.c;
            const double q = f.s2 * static_cast<double>(yp) * static_cast<double>(yp);
            ok = q <= kExpQmax;
            const double qi = rint(q);
            row[2 * lane] = yp;
            row[2 * lane + 1] = __builtin_amdgcn_ldexpf(
                __builtin_amdgcn_exp2f(static_cast<float>(qi - q)), -static_cast<int>(qi));
        }
        // the next window's datum, in flight while this window is consumed
        ycur = jj + kExpWin < jend ? y[jj + kExpWin] : 0.0f;
        if (!__all(ok)) return true;
        wave_sync();                          // the window is written before it is read
        const int we = wb + kExpWin < jend ? wb + kExpWin : jend;
        for (; j < we; j += 8) {
            float p = prod;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float yp = row[2 * (j - wb + u)];
                const float gj = row[2 * (j - wb + u) + 1];
                float e = __builtin_amdgcn_exp2f(__builtin_fmaf(yp, f.B[0], f.C[0]));
#pragma unroll
                for (int i = 1; i < K; ++i)
                    e += __builtin_amdgcn_exp2f(__builtin_fmaf(yp, f.B[i], f.C[i]));
                p *= e * gj;
            }
            if (!__all(p >= kFloor)) return false;
            expo += __builtin_amdgcn_frexp_expf(p);
            prod = __builtin_amdgcn_frexp_mantf(p);
        }
    }
    return false;
}

// The expanded shifted form over the blocks of 16 data from j to jend:
// log2 e_j = (M_j - q_j) + log2 sum_i 2^{x_ij - M_j} with M_j = max_i x_ij,
// staged as (y'_j, q_j) pairs (q_j rounded to FP32). The M_j - q_j are summed
// in FP32 per block and added to msum in FP64, as in the shifted form.
// Updates prod, expo and msum and moves j past the blocks it took; stops at
// the first window out of range.
template <int K>
__device__ __forceinline__ void expanded_shifted(const float* __restrict__ y, int jend,
                                                 const Expanded<K>& f, float* row, float& prod,
                                                 int& expo, double& msum, int& j) {
    constexpr int US = 16;
    const int lane = lane_id();
    float ycur = j + lane < jend ? y[j + lane] : 0.0f;
    for (int wb = j; wb < jend; wb += kExpWin) {
        const int jj = wb + lane;
        bool ok = true;
        wave_sync();                          // the previous window's reads come first
        if (jj < jend) {
            const float yp = ycur - f.c;
            const double q = f.s2 * static_cast<double>(yp) * static_cast<double>(yp);
            ok = q <= kExpQmax;
            row[2 * lane] = yp;
            row[2 * lane + 1] = static_cast<float>(q);
        }
        ycur = jj + kExpWin < jend ? y[jj + kExpWin] : 0.0f;
        if (!__all(ok)) return;
        wave_sync();                          // the window is written before it is read
        const int we = wb + kExpWin < jend ? wb + kExpWin : jend;
        for (; j < we; j += US) {
            float mblk = 0.0f;
#pragma unroll 8
            for (int u = 0; u < US; ++u) {
                const float yp = row[2 * (j - wb + u)];
                const float qj = row[2 * (j - wb + u) + 1];
                float x[K];
#pragma unroll
                for (int i = 0; i < K; ++i) x[i] = __builtin_fmaf(yp, f.B[i], f.C[i]);
                float m = x[0];
#pragma unroll
                for (int i = 1; i < K; ++i) m = fmaxf(m, x[i]);
                float e = __builtin_amdgcn_exp2f(x[0] - m);
#pragma unroll
                for (int i = 1; i < K; ++i) e += __builtin_amdgcn_exp2f(x[i] - m);
                prod *= e;
                mblk += m - qj;
            }
            msum += static_cast<double>(mblk);
            expo += __builtin_amdgcn_frexp_expf(prod);
            prod = __builtin_amdgcn_frexp_mantf(prod);
        }
    }
}

template <int K, int D>
__device__ __forceinline__ double partial_fp32(const float* __restrict__ y, int j0, int j1,
                                               const double (&mu)[K * D], const GmmDev& g,
                                               bool near, const ExpStage& st,
                                               unsigned long long* shifted_ctr = nullptr) {
    constexpr int UF = 8;            // direct-form block
    constexpr int US = 16;           // shifted-form block
    constexpr float kFloor = 0x1p-100f;
    const float s = g.s32;
    double msum = 0.0;
    float prod = 1.0f;
    int expo = 0;
    int j = j0;
    // -s mu in FP32 for the plain forms, formed where they run (not held
    // through the expanded forms)
    float nms[K * D];
    auto form_nms = [&]() {
#pragma unroll
        for (int c = 0; c < K * D; ++c)
            nms[c] = static_cast<float>(-(static_cast<double>(s) * mu[c]));
    };
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
    // the expanded forms' setup (1-D data, a staging row given): the centre of
    // the slice's first 64 data
    float* row = st.row;
    Expanded<K> xf;
    bool xok = false;
    float y0 = 0.0f;
    if constexpr (D == 1) {
        if (row != nullptr && j1 - j0 >= kExpMinData) {
            // j1 - j0 >= 64: every lane's datum y[j0 + lane] is in the slice
            y0 = st.pre ? st.y0 : y[j0 + lane_id()];
            xok = expanded_setup<K>(y0, j0, j0 + kExpWin, mu, g, xf);
        }
    }
    if (g.unit_mass != 0 && __all(near)) {
        bool plain = true;                    // whether the scalar-load direct form runs from j
        if constexpr (D == 1) {
            if (xok) plain = expanded_direct<K>(y, j0 + ((j1 - j0) & ~(UF - 1)), xf, row, prod,
                                                expo, j, y0);
        }
        if (plain) {
            form_nms();
            for (; j + UF <= j1; j += UF) {
                const float* yb = y + (size_t)wave_uniform(j) * D;    // wave-uniform: scalar loads
                float p = prod;
#pragma unroll
                for (int u = 0; u < UF; ++u) p *= direct(yb + u * D);
                if (!__all(p >= kFloor)) break;
                expo += __builtin_amdgcn_frexp_expf(p);
                prod = __builtin_amdgcn_frexp_mantf(p);
            }
        }
    }
    if (shifted_ctr != nullptr) {
        const int counted = ((j1 - j0) & ~(UF - 1)) - (j - j0);
        if (counted > 0 && lane_id() == 0) {
            const int slot = (static_cast<int>(blockIdx.x) * (static_cast<int>(blockDim.x) >> 6) +
                              wave_id()) & (kFormSlots - 1);
            atomicAdd(shifted_ctr + slot, static_cast<unsigned long long>(counted));
        }
    }
    if constexpr (D == 1) {
        if (xok && j + US <= j1)
            expanded_shifted<K>(y, j + ((j1 - j) & ~(US - 1)), xf, row, prod, expo, msum, j);
    }
    if (j < j1) form_nms();
    for (; j + US <= j1; j += US) {
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
    for (; j < j1; ++j) {
        float m, e;
        shifted(y + (size_t)j * D, m, e);
        prod *= e;
        msum += static_cast<double>(m);
    }
    return msum + static_cast<double>(expo) + log2(static_cast<double>(prod));
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
// expanded forms; both unused in FP64.
template <int K, int D, int PREC>
__device__ __forceinline__ double slice_partial(const float* __restrict__ y, int j0, int j1,
                                                const double (&pr)[K * D], const GmmDev& g,
                                                bool near = true, const ExpStage& st = {},
                                                unsigned long long* shifted_ctr = nullptr) {
    if constexpr (PREC == SMC_PREC_FP32) {
        return partial_fp32<K, D>(y, j0, j1, pr, g, near, st, shifted_ctr);
    } else {
        return partial_fp64<K, D>(y, j0, j1, pr, g);
    }
}

// This wave's staging row for the expanded forms in a kernel of at most W
// waves per workgroup (a static LDS array of that kernel), or nullptr where the
// forms do not apply (FP64, d > 1).
template <int PREC, int D, int W>
__device__ __forceinline__ float* expanded_row() {
    if constexpr (PREC == SMC_PREC_FP32 && D == 1) {
        __shared__ float win[W][2 * kExpWin];
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
// contains one barrier); prs holds KD rows of 64 doubles.
template <int KD>
__device__ __forceinline__ void block_proposals(uint64_t seed, uint32_t index, uint32_t step,
                                                uint32_t move, const double* th_src, int N,
                                                int a, double sd, int w, int nw,
                                                double (*prs)[kWave], double (&pr)[KD]) {
    const int lane = lane_id();
    for (int q = w; q < (KD + 1) / 2; q += nw) {
        const Words4 wd = draw(seed, index, static_cast<uint32_t>(q / 2), step, kProp, move);
        double z0, z1;
        if (q & 1) box_muller(wd.w2, wd.w3, z0, z1);
        else box_muller(wd.w0, wd.w1, z0, z1);
        const int c = 2 * q;
        prs[c][lane] = th_src[static_cast<size_t>(c) * N + a] + sd * z0;
        if (c + 1 < KD) prs[c + 1][lane] = th_src[static_cast<size_t>(c + 1) * N + a] + sd * z1;
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

// Decision and write-back of particle p of a random-walk move. The current
// state is column a of (th_src, l_src) (a = p, or p's ancestor after a fused
// resampling) and is re-read rather than held; pr_at(c) returns coordinate c of
// the proposal. Rejected particles are copied when the move is out of place.
// l_new (optional) receives the particle's log-likelihood after the move.
template <int KD, class PropAt>
__device__ __forceinline__ bool rwmh_accept(int p, int a, int N, PropAt pr_at, double l_prop,
                                            const MoveSource& srcs, double* theta, double* l,
                                            const double* beta_vec, const StepSrc& src,
                                            uint32_t step, uint64_t seed, uint32_t move,
                                            const GmmDev& g, int* status, const MoveStep& ms,
                                            double* l_new = nullptr) {
    const double* th_src = srcs.th;
    const double l_cur = srcs.l[a];
    const bool acc = rwmh_decide<KD>(
        p, pr_at, [&](int c) { return th_src[static_cast<size_t>(c) * N + a]; }, l_cur, l_prop,
        beta_vec, src, step, seed, move, g);
    if (acc) {
#pragma unroll
        for (int c = 0; c < KD; ++c) theta[static_cast<size_t>(c) * N + p] = pr_at(c);
        l[p] = l_prop;
    } else if (srcs.write_always) {
#pragma unroll
        for (int c = 0; c < KD; ++c)
            theta[static_cast<size_t>(c) * N + p] = th_src[static_cast<size_t>(c) * N + a];
        l[p] = l_cur;
    }
    if (l_prop != l_prop) atomicOr(status, kStatusNaN);
    move_duties(p, N, ms);
    if (l_new) *l_new = acc ? l_prop : l_cur;
    return acc;
}

}  // namespace smc
