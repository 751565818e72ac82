// d-dimensional mixture log-likelihood on the matrix cores (gfx950 MFMA).
//
// For d-variate components with covariance sigma2*I the per-component term is
// a quadratic form; in base-2 units
//   a_{j,i} = log2 w_i - s2 ||y_j - mu_i||^2,        s2 = log2(e) / (2 sigma2)
//           = (2 s2 y_j) . mu_i  - s2 ||y_j||^2  + (log2 w_i - s2 ||mu_i||^2),
// which is one contraction over K = 64 between a data row and a component
// column. BF16 keeps 8 significant bits, so every FP32/FP64 value is split into
// three BF16 parts (hi + mid + lo, exact for FP32 data and 24-bit accurate for
// the FP64 means) and the cross term keeps the six products down to 2^-16 of
// the leading one (hi*hi, hi*mid, mid*hi, hi*lo, lo*hi, mid*mid); the two norm
// terms enter the same contraction as three BF16 parts against ones. Products
// of BF16 values are exact in the FP32 accumulator, so the result carries only
// FP32 accumulation error and the 2^-24 truncation of the dropped products.
// The quadratic forms are evaluated at the represented means (hi+mid+lo), so
// the norm and cross terms are consistent and no systematic bias is introduced.
//
// K layout (eight slots of eight coordinates; slots 0-3 feed the first
// 16x16x32 MFMA and slots 4-7 the second):
//   slot  A (data row j)                         B (particle p, component i)
//   0     u_hi                                   mu_hi
//   1     u_hi                                   mu_mid
//   2     u_mid                                  mu_hi
//   3     u_hi                                   mu_lo
//   4     u_lo                                   mu_hi
//   5     u_mid                                  mu_mid
//   6     [Y_hi, Y_mid, Y_lo, 1, 1, 1, 0, 0]     [1, 1, 1, C_hi, C_mid, C_lo, 0, 0]
//   7     0                                      0
// with u = 2 s2 y (FP32), Y = -s2 ||y||^2, C_i = log2 w_i - s2 ||mu_i||^2.
// In the 16x16x32 operand layout lane l holds row (l mod 16) of A and column
// (l mod 16) of B for K elements 8*(l/16)..+7, so every lane handles exactly one
// slot per MFMA, and the output lane holds four data rows 4*(l/16)..+3 of its
// column. One MFMA pair per mixture component puts all k component values of a
// (datum, particle) pair in the same lane: the epilogue (hardware exp2, sum,
// product accumulation; with the per-datum max shift only for waves holding a
// particle far from the data) needs no cross-lane traffic.
//
// Workgroup = 4 waves x 16 particles; the data rows of a slice are staged in LDS
// (16 KB stages, double-buffered, 16-byte slots XOR-swizzled by row to spread
// the banks) and shared by the 4 waves. Slices of the data go to different
// workgroups; their partial sums are combined in slice order by a second kernel.
#include "gmm_common.hpp"

namespace smc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRowElems = 64;              // BF16 per staged data row
constexpr int kRowBytes = 2 * kRowElems;
constexpr int kTileRows = 16;
constexpr int kStageTiles = 8;
constexpr int kStageRows = kStageTiles * kTileRows;
constexpr int kStageBytes = kStageRows * kRowBytes;   // 16 KB
constexpr int kDdBlock = 256;                          // 4 waves, 64 particles
constexpr int kDdDim = 8;                              // coordinates per slot
constexpr double kLog2e = 1.4426950408889634;

__device__ __forceinline__ void split3(float x, __bf16& h, __bf16& m, __bf16& l) {
    h = static_cast<__bf16>(x);
    const float r1 = x - static_cast<float>(h);
    m = static_cast<__bf16>(r1);
    const float r2 = r1 - static_cast<float>(m);
    l = static_cast<__bf16>(r2);
}

// FP64 value -> three BF16 parts and the value they represent (exact sum).
__device__ __forceinline__ double split3d(double x, __bf16& h, __bf16& m, __bf16& l) {
    h = static_cast<__bf16>(static_cast<float>(x));
    const double r1 = x - static_cast<double>(static_cast<float>(h));
    m = static_cast<__bf16>(static_cast<float>(r1));
    const double r2 = r1 - static_cast<double>(static_cast<float>(m));
    l = static_cast<__bf16>(static_cast<float>(r2));
    return (static_cast<double>(static_cast<float>(h)) + static_cast<double>(static_cast<float>(m))) +
           static_cast<double>(static_cast<float>(l));
}

// One thread per (padded) data row: the 64-element A row of the K layout.
__global__ void __launch_bounds__(256)
k_dd_prep(const float* __restrict__ y, int n, int n_pad, double s2, __bf16* __restrict__ A) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_pad) return;
    bf16x8 slot[8];
    const __bf16 zero = static_cast<__bf16>(0.0f);
    const __bf16 one = static_cast<__bf16>(1.0f);
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int c = 0; c < 8; ++c) slot[s][c] = zero;
    if (j < n) {
        double yn = 0.0;
#pragma unroll
        for (int c = 0; c < kDdDim; ++c) {
            const float yc = y[static_cast<size_t>(j) * kDdDim + c];
            yn += static_cast<double>(yc) * static_cast<double>(yc);
            const float u = static_cast<float>(2.0 * s2 * static_cast<double>(yc));
            __bf16 h, m, l;
            split3(u, h, m, l);
            slot[0][c] = h;
            slot[1][c] = h;
            slot[2][c] = m;
            slot[3][c] = h;
            slot[4][c] = l;
            slot[5][c] = m;
        }
        __bf16 h, m, l;
        split3(static_cast<float>(-s2 * yn), h, m, l);
        slot[6][0] = h;
        slot[6][1] = m;
        slot[6][2] = l;
        slot[6][3] = one;
        slot[6][4] = one;
        slot[6][5] = one;
    }
    bf16x8* dst = reinterpret_cast<bf16x8*>(A + static_cast<size_t>(j) * kRowElems);
#pragma unroll
    for (int s = 0; s < 8; ++s) dst[s] = slot[s];
}

// One thread per (particle, component): the 64-element B column of the K
// layout, from the current means or (PROP) from the random-walk proposal of the
// move, which is also stored for the accept kernel.
template <bool PROP>
__global__ void __launch_bounds__(256)
k_dd_build(const double* __restrict__ theta, int N, int K, GmmDev g, double s2, MoveStep ms,
           double sd, uint64_t seed, StepSrc src, uint32_t move, __bf16* __restrict__ B,
           double* __restrict__ theta_prop) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N * K) return;
    const int p = q / K;
    const int i = q - p * K;
    const double* th = theta;
    if constexpr (PROP) {
        const bool rs = ms.state != nullptr && ms.state->resampled != 0;
        th = (rs && ms.theta_alt) ? ms.theta_alt : (ms.theta_src ? ms.theta_src : theta);
    }
    double mu[kDdDim];
#pragma unroll
    for (int c = 0; c < kDdDim; ++c) mu[c] = th[static_cast<size_t>(i * kDdDim + c) * N + p];
    if constexpr (PROP) {
        const uint32_t step = static_cast<uint32_t>(step_index(src));
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const Words4 wd = draw(seed, static_cast<uint32_t>(p), 2 * i + b, step, kProp, move);
            double z0, z1, z2, z3;
            box_muller(wd.w0, wd.w1, z0, z1);
            box_muller(wd.w2, wd.w3, z2, z3);
            mu[4 * b + 0] = mu[4 * b + 0] + sd * z0;
            mu[4 * b + 1] = mu[4 * b + 1] + sd * z1;
            mu[4 * b + 2] = mu[4 * b + 2] + sd * z2;
            mu[4 * b + 3] = mu[4 * b + 3] + sd * z3;
        }
#pragma unroll
        for (int c = 0; c < kDdDim; ++c) theta_prop[static_cast<size_t>(i * kDdDim + c) * N + p] = mu[c];
    }
    const __bf16 zero = static_cast<__bf16>(0.0f);
    const __bf16 one = static_cast<__bf16>(1.0f);
    bf16x8 sh, sm, sl, s6, s7;
    double nrm = 0.0;
#pragma unroll
    for (int c = 0; c < kDdDim; ++c) {
        __bf16 h, m, l;
        const double rep = split3d(mu[c], h, m, l);
        nrm += rep * rep;
        sh[c] = h;
        sm[c] = m;
        sl[c] = l;
        s7[c] = zero;
    }
    __bf16 ch, cm, cl;
    split3(static_cast<float>(g.lw[i] * kLog2e - s2 * nrm), ch, cm, cl);
    s6[0] = one; s6[1] = one; s6[2] = one;
    s6[3] = ch; s6[4] = cm; s6[5] = cl;
    s6[6] = zero; s6[7] = zero;
    bf16x8* dst = reinterpret_cast<bf16x8*>(B + static_cast<size_t>(q) * kRowElems);
    dst[0] = sh;   // slot 0: mu_hi
    dst[1] = sm;   // slot 1: mu_mid
    dst[2] = sh;   // slot 2: mu_hi
    dst[3] = sl;   // slot 3: mu_lo
    dst[4] = sh;   // slot 4: mu_hi
    dst[5] = sm;   // slot 5: mu_mid
    dst[6] = s6;   // slot 6: ones against the data norm, the component constant
    dst[7] = s7;   // slot 7: padding
}

template <int K>
__global__ void __launch_bounds__(kDdBlock)
k_dd_partial(const __bf16* __restrict__ A, int n, int n_pad, const __bf16* __restrict__ B, int N,
             int S, int unit_mass, double* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) unsigned char lds[2][kStageBytes];
    const int lane = lane_id();
    const int w = wave_id();
    const int grp = lane >> 4;            // K group of this lane: slots grp and 4 + grp
    const int col = lane & 15;            // particle column within the wave's tile
    const int p = blockIdx.x * 64 + w * 16 + col;
    const int pc = p < N ? p : N - 1;
    const int slice = blockIdx.y;
    const int ntiles = n_pad / kTileRows;
    const int t0 = static_cast<int>((static_cast<int64_t>(ntiles) * slice) / S);
    const int t1 = static_cast<int>((static_cast<int64_t>(ntiles) * (slice + 1)) / S);

    // B operands of this lane: slot grp (first MFMA) and 4 + grp (second)
    bf16x8 b1[K], b2[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const bf16x8* colp = reinterpret_cast<const bf16x8*>(B + (static_cast<size_t>(pc) * K + i) * kRowElems);
        b1[i] = colp[grp];
        b2[i] = colp[4 + grp];
    }

    double msum = 0.0;
    float prod = 1.0f;
    int expo = 0;
    // direct form (no per-datum max shift) while every lane's tile product
    // stays >= 2^-100; the wave keeps the shifted form from the first tile
    // where one does not (the same rule as the VALU form's partial_fp32)
    bool direct = unit_mass != 0;
    constexpr float kFloor = 0x1p-100f;
    const int nst = (t1 - t0 + kStageTiles - 1) / kStageTiles;
    uint4 regs[4];
    auto load_stage = [&](int st) {
        const int row0 = (t0 + st * kStageTiles) * kTileRows;
        const int rows_avail = min(kStageRows, t1 * kTileRows - row0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int q = threadIdx.x * 4 + k;
            const int row = q >> 3, sl = q & 7;
            regs[k] = (row < rows_avail)
                          ? *reinterpret_cast<const uint4*>(A + static_cast<size_t>(row0 + row) * kRowElems + sl * 8)
                          : make_uint4(0u, 0u, 0u, 0u);
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int q = threadIdx.x * 4 + k;
            const int row = q >> 3, sl = q & 7;
            *reinterpret_cast<uint4*>(&lds[buf][row * kRowBytes + ((sl ^ (row & 7)) << 4)]) = regs[k];
        }
    };
    if (nst > 0) {
        load_stage(0);
        store_stage(0);
    }
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int buf = st & 1;
        const bool more = st + 1 < nst;
        if (more) load_stage(st + 1);
        const int tile0 = t0 + st * kStageTiles;
        const int tiles_here = min(kStageTiles, t1 - tile0);
        for (int tt = 0; tt < tiles_here; ++tt) {
            const int row = tt * kTileRows + col;
            const bf16x8 a1 = *reinterpret_cast<const bf16x8*>(
                &lds[buf][row * kRowBytes + ((grp ^ (row & 7)) << 4)]);
            const bf16x8 a2 = *reinterpret_cast<const bf16x8*>(
                &lds[buf][row * kRowBytes + (((4 + grp) ^ (row & 7)) << 4)]);
            f32x4 acc[K];
#pragma unroll
            for (int i = 0; i < K; ++i) {
                const f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, b1[i], z, 0, 0, 0);
                acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b2[i], acc[i], 0, 0, 0);
            }
            const int grow = (tile0 + tt) * kTileRows + grp * 4;
            bool done = false;
            if (direct) {
                float pd = prod;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (grow + r < n) {
                        float e = __builtin_amdgcn_exp2f(acc[0][r]);
#pragma unroll
                        for (int i = 1; i < K; ++i) e += __builtin_amdgcn_exp2f(acc[i][r]);
                        pd *= e;
                    }
                }
                if (__all(pd >= kFloor)) {
                    prod = pd;
                    done = true;
                } else {
                    direct = false;
                }
            }
            if (!done) {
                float mblk = 0.0f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (grow + r < n) {
                        float m = acc[0][r];
#pragma unroll
                        for (int i = 1; i < K; ++i) m = fmaxf(m, acc[i][r]);
                        float e = __builtin_amdgcn_exp2f(acc[0][r] - m);
#pragma unroll
                        for (int i = 1; i < K; ++i) e += __builtin_amdgcn_exp2f(acc[i][r] - m);
                        prod *= e;
                        mblk += m;
                    }
                }
                msum += static_cast<double>(mblk);
            }
            expo += __builtin_amdgcn_frexp_expf(prod);
            prod = __builtin_amdgcn_frexp_mantf(prod);
        }
        if (more) store_stage(buf ^ 1);
        __syncthreads();
    }
    double v = msum + static_cast<double>(expo) + log2(static_cast<double>(prod));
    v += __shfl_xor(v, 16, kWave);
    v += __shfl_xor(v, 32, kWave);
    if (grp == 0 && p < N) part[static_cast<size_t>(slice) * N + p] = v;
}

__global__ void __launch_bounds__(256)
k_dd_finish(const double* __restrict__ part, int S, int N, int n, GmmDev g,
            double* __restrict__ out, int* status) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    double acc = part[p];
    for (int s = 1; s < S; ++s) acc += part[static_cast<size_t>(s) * N + p];
    const double l = finish_loglik<SMC_PREC_FP32>(acc, n, g);
    out[p] = l;
    if (l != l) atomicOr(status, kStatusNaN);
}

template <int K>
__global__ void __launch_bounds__(256)
k_dd_accept(const double* __restrict__ part, int S, int N, int n,
            const double* __restrict__ theta_prop, double* theta, double* l,
            const double* __restrict__ beta_vec, StepSrc src, uint64_t seed, uint32_t move,
            GmmDev g, unsigned long long* n_acc, int* status, MoveStep ms) {
    constexpr int KD = K * kDdDim;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t step = static_cast<uint32_t>(step_index(src));
    if (ms.t_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0)
        *ms.t_out = static_cast<int>(step);
    bool acc = false;
    if (p < N) {
        double tot = part[p];
        for (int s = 1; s < S; ++s) tot += part[static_cast<size_t>(s) * N + p];
        const double l_prop = finish_loglik<SMC_PREC_FP32>(tot, n, g);
        const MoveSource srcs = move_source(ms, theta, l);
        acc = rwmh_accept<KD>(
            p, p, N, [&](int c) { return theta_prop[static_cast<size_t>(c) * N + p]; }, l_prop,
            srcs, theta, l, beta_vec, src, step, seed, move, g, status, ms);
    }
    const unsigned long long mask = __ballot(acc);
    if (lane_id() == 0 && n_acc != nullptr && mask != 0ull)
        atomicAdd(n_acc, static_cast<unsigned long long>(__popcll(mask)));
}

double s2_of(const GmmDev& g) { return g.inv2s2 * kLog2e; }

}  // namespace

int64_t dd_padded_rows(int64_t n) { return ((n + kTileRows - 1) / kTileRows) * kTileRows; }

int dd_clamp_slices(int64_t n, int64_t S) {
    const int64_t tiles = dd_padded_rows(n) / kTileRows;
    if (S > 16) S = 16;
    if (S > tiles) S = tiles;
    if (S < 1) S = 1;
    return static_cast<int>(S);
}

int dd_slices(int64_t n, int64_t N) {
    const int64_t groups = (N + 63) / 64;
    return dd_clamp_slices(n, (2048 + groups - 1) / groups);
}

bool dd_supported(int k, int d) { return d == kDdDim && (k == 1 || k == 2 || k == 4 || k == 8); }

hipError_t launch_dd_prep(const GmmDev& g, const float* y, int64_t n, __bf16* A, hipStream_t s) {
    const int64_t np = dd_padded_rows(n);
    hipLaunchKernelGGL(k_dd_prep, dim3(static_cast<unsigned>((np + 255) / 256)), dim3(256), 0, s, y,
                       static_cast<int>(n), static_cast<int>(np), s2_of(g), A);
    return hipGetLastError();
}

hipError_t launch_dd_loglik(const GmmDev& g, const __bf16* A, int64_t n, const double* theta,
                            int64_t N, __bf16* B, double* part, int S, double* out, int* status,
                            hipStream_t s) {
    const int64_t np = dd_padded_rows(n);
    const unsigned gb = static_cast<unsigned>((N * g.k + 255) / 256);
    hipLaunchKernelGGL((k_dd_build<false>), dim3(gb), dim3(256), 0, s, theta, static_cast<int>(N),
                       g.k, g, s2_of(g), MoveStep{}, 0.0, 0ull, StepSrc{}, 0u, B,
                       static_cast<double*>(nullptr));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(static_cast<unsigned>((N + 63) / 64), static_cast<unsigned>(S));
#define SMC_DD(KK)                                                                              \
    if (g.k == KK)                                                                              \
        hipLaunchKernelGGL((k_dd_partial<KK>), grid, dim3(kDdBlock), 0, s, A, static_cast<int>(n), \
                           static_cast<int>(np), B, static_cast<int>(N), S, g.unit_mass, part);
    SMC_DD(1) SMC_DD(2) SMC_DD(4) SMC_DD(8)
#undef SMC_DD
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dd_finish, dim3(static_cast<unsigned>((N + 255) / 256)), dim3(256), 0, s,
                       part, S, static_cast<int>(N), static_cast<int>(n), g, out, status);
    return hipGetLastError();
}

hipError_t launch_dd_rwmh(const GmmDev& g, const __bf16* A, int64_t n, double* theta, double* l,
                          int64_t N, const double* beta_vec, StepSrc src, double sd,
                          uint64_t seed, uint32_t move, unsigned long long* n_accept,
                          __bf16* B, double* theta_prop, double* part, int S, int* status,
                          MoveStep ms, hipStream_t s) {
    const int64_t np = dd_padded_rows(n);
    const unsigned gb = static_cast<unsigned>((N * g.k + 255) / 256);
    hipLaunchKernelGGL((k_dd_build<true>), dim3(gb), dim3(256), 0, s, theta, static_cast<int>(N),
                       g.k, g, s2_of(g), ms, sd, seed, src, move, B, theta_prop);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const dim3 grid(static_cast<unsigned>((N + 63) / 64), static_cast<unsigned>(S));
    const dim3 g1(static_cast<unsigned>((N + 255) / 256));
#define SMC_DD(KK)                                                                              \
    if (g.k == KK) {                                                                            \
        hipLaunchKernelGGL((k_dd_partial<KK>), grid, dim3(kDdBlock), 0, s, A, static_cast<int>(n), \
                           static_cast<int>(np), B, static_cast<int>(N), S, g.unit_mass, part);              \
        e = hipGetLastError();                                                                  \
        if (e != hipSuccess) return e;                                                          \
        hipLaunchKernelGGL((k_dd_accept<KK>), g1, dim3(256), 0, s, part, S, static_cast<int>(N), \
                           static_cast<int>(n), theta_prop, theta, l, beta_vec, src, seed, move, \
                           g, n_accept, status, ms);                                            \
        return hipGetLastError();                                                               \
    }
    SMC_DD(1) SMC_DD(2) SMC_DD(4) SMC_DD(8)
#undef SMC_DD
    return hipErrorInvalidValue;
}

}  // namespace smc
