// Factor stochastic-volatility particle filter: device model and launchers.
#pragma once
#include "../../include/smc_fsv.h"
#include "internal.hpp"

namespace smc {

// Model constants as the kernels consume them (built on the host per call).
struct FsvDev {
    int m, k;
    double B[SMC_FSV_MMAX * SMC_FSV_KMAX];
    double psi[SMC_FSV_MMAX];
    double phi[SMC_FSV_KMAX];
    double L[SMC_FSV_KMAX * SMC_FSV_KMAX];      // lower Cholesky factor of U, row-major
    double cst;                                 // -(m/2) ln(2 pi)
};

// The previous step's resampling, taken by the next step's propagation in a
// chain of filter steps: with state set and state->resampled, particle p
// propagates from x[:, a] with a its ancestor (the scheme's point of step
// state->t searched in the CDF of that step) and starts from log-weight 0.
struct FsvAnc {
    const StepState* state;    // nullable: propagate x[:, p] with its log-weight
    const double* cdf_hi;
    const double* cdf_lo;
    const double* chunk_tot;   // [2 * nchunks] (hi, lo)
    int chunk, nchunks;
    int scheme;
};

bool fsv_supported(int m, int k);
// Number of per-block partials the weight pass writes (as the step's combine expects).
int fsv_parts(int64_t N);
hipError_t launch_fsv_init(int k, int64_t N, double* x, double* logw, hipStream_t s);
// Propagate + weight + reweight partials (sc.rw_part) + moment partials (mom).
hipError_t launch_fsv_weight(const FsvDev& f, const double* y, int T, const double* x,
                             double* x_out, double* logw, int64_t N, StepSrc src, uint64_t seed,
                             const Scratch& sc, double* mom, hipStream_t s,
                             const FsvAnc& anc = FsvAnc{});

}  // namespace smc
