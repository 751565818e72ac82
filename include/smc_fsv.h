/* Bootstrap particle filter for the factor stochastic-volatility model
 * (Factor Stochastic Volatility subsection), on the same context as smc.h.
 *
 *   x_t ~ N(Phi x_{t-1}, U),  x_0 = 0          (K latent log-variances)
 *   y_t | x_t ~ N(0, B diag(exp(x_t)) B^T + Psi)   (M observations)
 *
 * One filter step t: every particle is propagated by the transition (noise:
 * the Philox normals of stream (p, 0, t, PROP, 0)), weighted by the
 * observation density (FP64 Cholesky of the M x M covariance), the
 * log-likelihood increment log sum_p W_p^{(t-1)} g(y_t | x_p) is accumulated,
 * the weighted mean and standard deviation of x_t are recorded, and the
 * population is resampled from the empirical CDF (the context's scheme, see
 * smc_set_resampling) when ESS < ess_frac * N. All pointers are caller-owned
 * device pointers; calls are asynchronous on `stream` and graph-replayable
 * (t lives in device memory). Errors as in smc.h. */
#ifndef SMC_FSV_H
#define SMC_FSV_H

#include "smc.h"

#ifdef __cplusplus
extern "C" {
#endif

#define SMC_FSV_MMAX 8
#define SMC_FSV_KMAX 4

/* Model parameters. B is m x k row-major (zero above the diagonal in the
 * paper, not required here); U must be symmetric positive definite. Compiled
 * (m, k): (5, 3), (2, 2), (1, 1); others return SMC_ERR_UNSUPPORTED. */
typedef struct {
    int32_t m, k;
    double B[SMC_FSV_MMAX * SMC_FSV_KMAX];
    double psi[SMC_FSV_MMAX];
    double phi[SMC_FSV_KMAX];
    double U[SMC_FSV_KMAX * SMC_FSV_KMAX];      /* k x k row-major */
} smc_fsv;

/* x [k][N] = 0, logw [N] = 0 (the filter's start). */
int fsv_init(smc_ctx ctx, int32_t k, int64_t N, double* x, double* logw, void* stream);

/* One filter step t = *t_dev (clamped to 1..T), then *t_dev = t + 1.
 * y: [T][m] FP64 observations. x: [k][N] in/out (the population after the
 * step's resampling, if any); x_tmp: [k][N] scratch (the propagated population);
 * logw: [N] in/out (0 after resampling). stats: device FP64 [4] = {log-likelihood
 * (accumulated), last ESS, resample count, unused}. moments: device FP64
 * [T][2k]: row t-1 = weighted means then standard deviations of x_t before
 * resampling. Kernels: propagate + weight + partial sums; combine + decision +
 * CDF chunks; moments; search + gather (a copy when not resampling). */
int fsv_step(smc_ctx ctx, const smc_fsv* model, const double* y, int32_t T, int64_t N,
             double* x, double* x_tmp, double* logw, int32_t* t_dev, uint64_t seed,
             double ess_frac, double* stats, double* moments, void* stream);

/* n_steps consecutive fsv_step calls (n_steps >= 1): the same arguments, random
 * streams and results bit for bit (x, logw, stats and moments), except that
 * x_tmp ends with unspecified contents. Within the call each step's
 * propagation takes the previous step's resampling itself (the ancestor
 * search of that step's CDF, reading the other buffer), so only the last step
 * runs the search-and-gather pass: two kernels per step instead of three.
 * Uses the context scratch (reserve N and k first when capturing). Errors as
 * fsv_step, and n_steps < 1 is an invalid argument; nothing is enqueued on an
 * argument error. */
int fsv_steps(smc_ctx ctx, const smc_fsv* model, const double* y, int32_t T, int64_t N,
              double* x, double* x_tmp, double* logw, int32_t* t_dev, int32_t n_steps,
              uint64_t seed, double ess_frac, double* stats, double* moments, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SMC_FSV_H */
