// Exchange moves of population MCMC (Population-based MCMC subsection):
// adjacent chains (a, b) of the current partition swap states with
// probability min(1, exp((beta_a - beta_b) (l_b - l_a))); the prior cancels.
#pragma once
#include "internal.hpp"
#include "philox.hpp"

namespace smc {

// Partition parity of iteration `it`: it & 1 (alternating), one Philox bit of
// stream (0, 0, it, PARITY, 0) (random), or a host value.
__device__ __forceinline__ int pt_parity(int parity_mode, int parity_host, uint64_t seed,
                                         uint32_t it) {
    if (parity_mode == 0) return static_cast<int>(it & 1u);
    if (parity_mode == 1) return static_cast<int>(draw(seed, 0, 0, it, kParity, 0).w0 >> 31);
    return parity_host & 1;
}

// Slot q of the partition: the pairs (parity + 2q, parity + 2q + 1), then the
// wrap pair (M-1, 0) when `wrap`, parity is 1 and M is even, else the chains
// left without a partner (0 when parity is 1, M-1 when M - parity is odd) as
// singles (b = -1). Returns false past the last slot.
__device__ __forceinline__ bool pt_slot(int M, int parity, int wrap, int q, int& a, int& b) {
    const int regular = (M - parity) / 2;
    if (q < regular) {
        a = parity + 2 * q;
        b = a + 1;
        return true;
    }
    q -= regular;
    const bool lead = parity == 1;
    const bool tail = ((M - parity) & 1) == 1;
    if (wrap && lead && tail) {
        a = M - 1;
        b = 0;
        return q == 0;
    }
    b = -1;
    if (lead) {
        if (q == 0) {
            a = 0;
            return true;
        }
        --q;
    }
    if (tail && q == 0) {
        a = M - 1;
        return true;
    }
    return false;
}

// The pair of the partition that chain c belongs to (the pairs of pt_slot):
// returns false when c is left single.
__device__ __forceinline__ bool pt_pair_of(int M, int parity, int wrap, int c, int& a, int& b) {
    if (wrap && parity == 1 && (M & 1) == 0 && (c == 0 || c == M - 1)) {
        a = M - 1;
        b = 0;
        return true;
    }
    const int d = c - parity;
    if (d < 0) return false;
    if ((d & 1) == 0) {
        if (c + 1 >= M) return false;
        a = c;
        b = c + 1;
        return true;
    }
    a = c - 1;
    b = c;
    return true;
}

// log u of the exchange test of the pair led by chain a: stream (a, 0, it, EXCH, 0).
__device__ __forceinline__ double pt_log_u(int a, uint64_t seed, uint32_t it) {
    return log(u01_open(draw(seed, static_cast<uint32_t>(a), 0, it, kExch, 0).w0));
}

// Swap columns a and b of theta [kd][M] (row stride M) and of l.
__device__ __forceinline__ void pt_swap_columns(double* theta, double* l, int M, int kd, int a,
                                                int b) {
    const double t = l[a];
    l[a] = l[b];
    l[b] = t;
    for (int c = 0; c < kd; ++c) {
        double* r = theta + static_cast<size_t>(c) * M;
        const double x = r[a];
        r[a] = r[b];
        r[b] = x;
    }
}

// The exchange decision of pair (a, b) given log u; on acceptance the two
// states are swapped in place. Returns whether they were.
__device__ __forceinline__ bool pt_swap_given(double* theta, double* l, const double* beta, int M,
                                              int kd, int a, int b, double log_u) {
    const double la = (beta[a] - beta[b]) * (l[b] - l[a]);
    if (!(la >= 0.0 || log_u < la)) return false;
    pt_swap_columns(theta, l, M, kd, a, b);
    return true;
}

// The exchange decision of pair (a, b) with the uniform of its own stream.
__device__ __forceinline__ bool pt_swap(double* theta, double* l, const double* beta, int M,
                                        int kd, int a, int b, uint64_t seed, uint32_t it) {
    return pt_swap_given(theta, l, beta, M, kd, a, b, pt_log_u(a, seed, it));
}

}  // namespace smc
