// Philox4x32-10 counter-based generator for gfx950, with exact uniform maps
// and Box-Muller normals.
//
// Generator: Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as
// 1, 2, 3" (SC'11). Ten rounds of a 4-word bijection keyed by two words; each
// round multiplies words 0 and 2 by fixed odd constants, keeps both halves of
// the 64-bit products, mixes the high halves into the other two words with the
// round key, and the key advances by two Weyl increments between rounds.
//
// The paper's own generators (MRG32k3a and xorshift with skip-ahead, Parallel
// Random Number Generation subsection) keep per-thread state; a counter-based
// generator needs none: every draw is a pure function of (seed, counter), so
// the CPU and GPU produce the same words for the same draw.
//
// Counter layout used by every kernel:
//   c0 = index (particle, chain or pair), c1 = block of four words,
//   c2 = step (tempering step or PT iteration), c3 = purpose << 24 | move;
//   key = (seed low word, seed high word).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

enum Purpose : uint32_t { kPrior = 1, kProp = 2, kAcc = 3, kResamp = 4, kExch = 5, kParity = 6 };

struct Words4 {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                                uint32_t c3, uint32_t k0, uint32_t k1) {
    constexpr uint32_t kMulA = 0xD2511F53u;   // multiplies word 0
    constexpr uint32_t kMulB = 0xCD9E8D57u;   // multiplies word 2
    constexpr uint32_t kBumpA = 0x9E3779B9u;  // golden-ratio Weyl step
    constexpr uint32_t kBumpB = 0xBB67AE85u;  // sqrt(3) - 1 Weyl step
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += kBumpA;
            k1 += kBumpB;
        }
        const uint32_t hiA = __umulhi(kMulA, c0);
        const uint32_t loA = kMulA * c0;
        const uint32_t hiB = __umulhi(kMulB, c2);
        const uint32_t loB = kMulB * c2;
        const uint32_t n0 = hiB ^ c1 ^ k0;
        const uint32_t n2 = hiA ^ c3 ^ k1;
        c0 = n0;
        c1 = loB;
        c2 = n2;
        c3 = loA;
    }
    return Words4{c0, c1, c2, c3};
}

__device__ __forceinline__ Words4 draw(uint64_t seed, uint32_t index, uint32_t block,
                                       uint32_t step, uint32_t purpose, uint32_t move) {
    return philox4x32_10(index, block, step, (purpose << 24) | (move & 0xFFFFFFu),
                         static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
}

// (w + 1/2) 2^-32: strictly inside (0, 1), exact in FP64.
__device__ __forceinline__ double u01_open(uint32_t w) {
    return (static_cast<double>(w) + 0.5) * 0x1p-32;
}

// w 2^-32: in [0, 1), exact in FP64.
__device__ __forceinline__ double u01_left_closed(uint32_t w) {
    return static_cast<double>(w) * 0x1p-32;
}

// (wa 2^21 + (wb >> 11)) 2^-53: a 53-bit uniform in [0, 1), exact in FP64.
__device__ __forceinline__ double u01_53(uint32_t wa, uint32_t wb) {
    const uint64_t v = (static_cast<uint64_t>(wa) << 21) | static_cast<uint64_t>(wb >> 11);
    return static_cast<double>(v) * 0x1p-53;
}

// Point U_i of a resampling scheme (codes as the C ABI's smc_resampling):
// 0 systematic (i + u)/N with the step's single offset u_sys, 1 stratified
// (i + u_i)/N, 2 multinomial u_i, where u_i is the 53-bit uniform of stream
// (i, 0, step, RESAMP, scheme). Each point is one rounding of its formula.
__device__ __forceinline__ double resample_point(int scheme, uint64_t seed, uint32_t step, int i,
                                                 int N, double u_sys) {
    if (scheme == 0) return (static_cast<double>(i) + u_sys) / static_cast<double>(N);
    const Words4 w = draw(seed, static_cast<uint32_t>(i), 0, step, kResamp,
                          static_cast<uint32_t>(scheme));
    const double u = u01_53(w.w0, w.w1);
    return scheme == 1 ? (static_cast<double>(i) + u) / static_cast<double>(N) : u;
}

// sin and cos of an angle a in [0, 2 pi]. Reduction to x = a - k pi/2 with k
// the nearest integer to a * 2/pi and pi/2 split in two doubles P1 + P2: for
// k >= 1, a >= pi/4 and k*P1 are both multiples of 2^-53, so a - k*P1 (one FMA)
// is exact and only the tiny k*P2 term rounds. On |x| <= pi/4 the Taylor series
// of sin (through x^17) and cos (through x^18) are truncated below 1e-18
// relative and evaluated in Horner form with FMAs; the coefficients are 1/n!
// rounded to double. Against a correctly rounded libm over 4.4e7 Box-Muller
// angles the error stays within 2 ulp (absolute 2.3e-16). The general device
// sincos must also reduce huge arguments and costs several times more.
__device__ __forceinline__ void sincos_0_2pi(double a, double* s, double* c) {
    constexpr double kP1 = 1.5707963267948966;
    constexpr double kP2 = 6.123233995736766e-17;
    constexpr double kTwoOverPi = 0.6366197723675814;
    const double k = rint(a * kTwoOverPi);
    double x = fma(-k, kP1, a);
    x = fma(-k, kP2, x);
    const double x2 = x * x;
    double ps = 2.8114572543455206e-15;             // 1/17!
    ps = fma(ps, x2, -7.647163731819816e-13);       // 1/15!
    ps = fma(ps, x2, 1.6059043836821613e-10);       // 1/13!
    ps = fma(ps, x2, -2.505210838544172e-08);       // 1/11!
    ps = fma(ps, x2, 2.7557319223985893e-06);       // 1/9!
    ps = fma(ps, x2, -0.0001984126984126984);       // 1/7!
    ps = fma(ps, x2, 0.008333333333333333);         // 1/5!
    ps = fma(ps, x2, -0.16666666666666666);         // 1/3!
    const double sx = fma(x * x2, ps, x);
    double pc = -1.5619206968586225e-16;            // 1/18!
    pc = fma(pc, x2, 4.779477332387385e-14);        // 1/16!
    pc = fma(pc, x2, -1.1470745597729725e-11);      // 1/14!
    pc = fma(pc, x2, 2.08767569878681e-09);         // 1/12!
    pc = fma(pc, x2, -2.755731922398589e-07);       // 1/10!
    pc = fma(pc, x2, 2.48015873015873e-05);         // 1/8!
    pc = fma(pc, x2, -0.001388888888888889);        // 1/6!
    pc = fma(pc, x2, 0.041666666666666664);         // 1/4!
    const double cx = fma(x2 * x2, pc, fma(-0.5, x2, 1.0));
    const int q = static_cast<int>(k) & 3;
    *s = (q == 0) ? sx : (q == 1) ? cx : (q == 2) ? -sx : -cx;
    *c = (q == 0) ? cx : (q == 1) ? -sx : (q == 2) ? -cx : sx;
}

// Box & Muller (1958): two independent standard normals from two uniforms.
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, double& z0, double& z1) {
    constexpr double kTwoPi = 6.283185307179586;
    const double r = sqrt(-2.0 * log(u01_open(wa)));
    const double ang = kTwoPi * u01_open(wb);
    double s, c;
    sincos_0_2pi(ang, &s, &c);
    z0 = r * c;
    z1 = r * s;
}

// Standard normal number c of the stream (index, step, purpose, move):
// block c/4, words (0,1) -> c%4 in {0,1}, words (2,3) -> c%4 in {2,3}.
template <int COUNT>
__device__ __forceinline__ void normals(uint64_t seed, uint32_t index, uint32_t step,
                                        uint32_t purpose, uint32_t move, double* z) {
#pragma unroll
    for (int b = 0; b < (COUNT + 3) / 4; ++b) {
        const Words4 w = draw(seed, index, b, step, purpose, move);
        double a0, a1, a2, a3;
        box_muller(w.w0, w.w1, a0, a1);
        box_muller(w.w2, w.w3, a2, a3);
        if (4 * b + 0 < COUNT) z[4 * b + 0] = a0;
        if (4 * b + 1 < COUNT) z[4 * b + 1] = a1;
        if (4 * b + 2 < COUNT) z[4 * b + 2] = a2;
        if (4 * b + 3 < COUNT) z[4 * b + 3] = a3;
    }
}

}  // namespace smc
