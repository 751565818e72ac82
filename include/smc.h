/*
 * smc.h -- C ABI of libsmcgpu: the data-parallel hot path of tempered
 * Gaussian-mixture SMC samplers and population MCMC on one AMD Instinct
 * MI355X (gfx950).
 *
 * What is computed (Lee, Yau, Giles, Doucet & Holmes, "On the utility of
 * graphics cards to perform massively parallel simulation of advanced Monte
 * Carlo methods"):
 *   - the per-particle mixture log-likelihood over all observations
 *     (Mixture Modelling section);
 *   - the random-walk Metropolis-Hastings move targeting a tempered posterior
 *     p0 * L^beta (Population-Based MCMC and SMC Sampler subsections);
 *   - the incremental reweight, log-sum-exp normalisation and effective sample
 *     size, and systematic resampling by prefix sum and search (Sequential Monte
 *     Carlo and SMC Samplers subsections; importance weights as in the
 *     Importance Sampling equations);
 *   - the exchange move between adjacent tempered chains on disjoint pairs
 *     (Population-Based MCMC: exchange ratio alpha_ij and partitions I_1..I_R).
 *
 * Conventions (every entry point):
 *   - Array arguments are DEVICE pointers on the context's GPU, owned by the
 *     caller; the library never frees or keeps them beyond the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream). Calls
 *     enqueue work asynchronously on it unless marked [sync].
 *   - Return value: SMC_OK (0) or a negative SMC_ERR_* code. On an argument
 *     error nothing is enqueued. No C++ exception crosses the ABI.
 *     smc_last_error() returns a thread-local description of the last failure.
 *   - Numeric degeneracy found on the device (NaN log-likelihood, all weights
 *     zero) cannot be returned by an asynchronous call: kernels raise a device
 *     status flag that smc_check() reports as SMC_ERR_NUMERIC.
 *   - Particle parameters theta are FP64, structure-of-arrays [k*d][N]: element
 *     (i*d + c)*N + p is coordinate c of mean i of particle p.
 *   - Observations y are FP32, row-major [n][d].
 *   - Random numbers come from Philox4x32-10 (Salmon et al., SC'11) with
 *     counter (index, block, step, purpose<<24 | move) and key = seed; the same
 *     words are produced on the CPU for the same counter.
 *   - A context must not be used from two host threads at the same time; calls
 *     on one context that overlap on different streams share its scratch and
 *     race.
 */
#ifndef SMC_H
#define SMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SMC_KMAX 8            /* most mixture components supported */
#define SMC_DMAX 8            /* most dimensions supported */
#define SMC_KDMAX 64          /* SMC_KMAX * SMC_DMAX */

enum {
    SMC_OK = 0,
    SMC_ERR_INVALID_ARG = -1, /* bad pointer, size or parameter */
    SMC_ERR_UNSUPPORTED = -2, /* (k, d, precision) combination not compiled */
    SMC_ERR_HIP = -3,         /* a HIP runtime call failed */
    SMC_ERR_NUMERIC = -4,     /* device status flag: NaN or all-zero weights */
    SMC_ERR_NOMEM = -5,       /* device allocation failed */
    SMC_ERR_CAPTURE = -6      /* scratch would have to grow during stream capture */
};

typedef enum {
    SMC_PREC_FP64 = 0,        /* plain FP64 arithmetic with device-library exp/log */
    SMC_PREC_FP32 = 1,        /* FP32 terms + hardware exp2, per-datum sums multiplied into a
                                 renormalised FP32 product (exponents kept as integers),
                                 FP64 total */
    SMC_PREC_BF16X3 = 2       /* d-dim: split-BF16 MFMA cross term, FP32 accumulation */
} smc_prec;

typedef enum { SMC_PRIOR_GAUSS = 0, SMC_PRIOR_BOX = 1 } smc_prior_kind;

/* Resampling schemes (Sequential Monte Carlo subsection: the new population is
 * drawn from the empirical CDF of the weights). All use idx_i = min{j : U_i < C_j}
 * on the correctly rounded CDF; they differ in the points U_i:
 *   SYSTEMATIC   (i + u)/N, one u = w0 2^-32 per step from stream (0, 0, step, RESAMP, 0);
 *   STRATIFIED   (i + u_i)/N, MULTINOMIAL  u_i (N independent draws),
 *   with u_i = (w0 2^21 + (w1 >> 11)) 2^-53 from stream (i, 0, step, RESAMP, scheme). */
typedef enum {
    SMC_RESAMPLE_SYSTEMATIC = 0,
    SMC_RESAMPLE_STRATIFIED = 1,
    SMC_RESAMPLE_MULTINOMIAL = 2
} smc_resampling;

/* The mixture model: k components in d dimensions with known covariance
 * sigma2 * I and known natural-log weights log_w[0..k-1] (summing to one in
 * probability); the unknowns are the k means. Prior on every coordinate of
 * every mean: N(prior_a, prior_b^2) (SMC_PRIOR_GAUSS) or uniform on
 * [prior_a, prior_b] (SMC_PRIOR_BOX, the paper's hypercube prior). */
typedef struct {
    int32_t k, d;
    double sigma2;
    double log_w[SMC_KMAX];
    int32_t prior;
    double prior_a, prior_b;
} smc_gmm;

typedef struct smc_ctx_s* smc_ctx;

/* [sync] Create a context on HIP device `device` (it becomes current while
 * the context allocates its scratch). */
int smc_create(smc_ctx* out, int device);

/* [sync] Destroy a context and free its scratch. NULL is accepted. */
int smc_destroy(smc_ctx ctx);

/* [sync] Size the context scratch for up to N particles of up to kd = k*d
 * parameters each and, when n > 0, for the MFMA form over up to n observations,
 * so that later calls (in particular inside hipGraph stream capture) never
 * allocate. Scratch that a larger reservation (or a call needing more room)
 * supersedes is kept until smc_destroy, so graphs captured before the growth
 * stay valid; a graph must be destroyed before its context. */
int smc_reserve(smc_ctx ctx, int64_t N, int32_t kd, int64_t n);

/* [sync] Synchronise `stream`, then read and clear the device status flag:
 * SMC_OK, or SMC_ERR_NUMERIC if a kernel saw a NaN log-likelihood or weights
 * that were all zero since the last check. */
int smc_check(smc_ctx ctx, void* stream);

const char* smc_last_error(void);

/* Override the number of data slices (contiguous ranges of the observations
 * whose partial sums for the same 64 particles are formed by separate waves)
 * used by the likelihood kernels; 0 restores the built-in choice. Range 0..128.
 * Up to 16 slices run as the waves of one workgroup; a move with more slices
 * and N <= 32768 spreads them over up to 8 workgroups per 64 particles and
 * completes in a second, per-particle kernel. Other kernels use min(slices, 16).
 * Results depend on the slicing only through the order of FP64 additions and,
 * in FP32, through which of the equivalent per-datum forms (see smc_loglik) a
 * wave's slice takes and, in the pivot form, through its windows. */
int smc_set_slices(smc_ctx ctx, int32_t slices);

/* Which launches a rule of the launch table shapes. */
enum {
    SMC_RULE_CALL = 0,    /* the likelihood and move kernels of every per-call entry point */
    SMC_RULE_BATCH = 1    /* the persistent move of smc_step_batched, per run */
};

/* One entry of a context's launch table (the output of the autotuner in the
 * Python package). kind SMC_RULE_CALL: calls whose model, precision and sizes
 * fall in the rule's ranges use `slices` data slices per 64-particle tile
 * (same meaning and range as smc_set_slices; the MFMA form uses
 * min(slices, 16)). kind SMC_RULE_BATCH: in a batch created while the rule is
 * in force, every run whose (n, N) fall in its ranges has each 64-particle tile
 * moved by `slices` waves (1, 2, 4 or 8) of the persistent move's 8-wave
 * workgroups, which therefore take 8 / slices tiles of the run at once.
 * k, d = 0 and prec = -1 match anything; ranges are inclusive. */
typedef struct {
    int32_t k, d, prec;
    int32_t kind;
    int32_t slices;
    int64_t n_lo, n_hi;
    int64_t N_lo, N_hi;
} smc_launch_rule;

/* Replace the context's launch table with a copy of `rules[0..count-1]`
 * (count = 0 clears it). The first matching rule of the call's kind wins; an
 * explicit smc_set_slices override takes precedence over the table for
 * per-call launches, and launches that match no rule use the built-in choice.
 * Invalid rules (unknown kind, slices outside 1..128 or, for a batch rule, not
 * 1, 2, 4 or 8, empty ranges) reject the whole table and leave the old one in
 * place. */
int smc_set_launch_table(smc_ctx ctx, const smc_launch_rule* rules, int32_t count);

/* Per-particle log-likelihood (Mixture Modelling section):
 *   loglik[p] = sum_j log sum_i w_i N_d(y_j; mu_{p,i}, sigma2 I).
 * y: [n][d] FP32; theta: [k*d][N] FP64; loglik: [N] FP64 out.
 * prec FP64: plain form (device-library exp and log per datum, plain sum);
 * FP32: FP32 arithmetic in base 2 with hardware exp2, no per-datum log: each
 * datum's mixture sum is multiplied into a running FP32 product that is
 * renormalised by frexp after every block of 8 or 16 data, its exponents added
 * as integers, and one hardware log2 of the product's mantissa per slice finishes (relative
 * error below 1e-6). The per-datum sum is taken directly for waves whose
 * particles sit near the data (weights of total mass <= 1) and relative to its
 * largest term otherwise (those maxima added in 16-term FP32 blocks promoted to
 * FP64). For d = 1 a third form, the pivot form, runs first: a wave's slice
 * goes in windows of 64 data, two at a time sharing one choice of pivots while
 * the test below holds over both; in a window with midpoint c each particle's
 * component p with the largest exponent at c is its pivot, each other
 * component's exponent difference to it is linear in y (one FMA and one exp2
 * per datum and component), every per-datum factor is at least 1, and the
 * pivot's own exponents summed over the window come in FP64 from two data sums
 * the wave forms once for all its particles. A window is taken when none of
 * the wave's particles can see a base-2 exponent difference above 14 in it
 * (13 for k > 4; the bound keeps a block of 8 factors below FP32 overflow;
 * narrow windows, which data in ascending order give, see smc_sort_data);
 * other windows, and windows holding a datum or parameter that is not finite,
 * go through the plain forms. All forms are within the bound (the form
 * depends on the wave and the data order, fixed for a given launch shape,
 * population and data array); BF16X3: d = 8, k in
 * {1,2,4,8}: the quadratic forms as one K = 64 BF16 MFMA contraction of
 * three-way (hi/mid/lo) split operands with FP32 accumulation, then the same
 * FP32 epilogue (relative error below 1e-6). */
int smc_loglik(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n,
               const double* theta, int64_t N, smc_prec prec, double* loglik,
               void* stream);

/* Draw theta_0 from the prior: [k*d][N] out. Gaussian coordinates use the
 * Box-Muller normals of stream (p, block, step 0, PRIOR, move 0); the box prior
 * maps the same words to (a, b) by a + (b - a) (w + 1/2) 2^-32. */
int smc_prior_init(smc_ctx ctx, const smc_gmm* model, int64_t N, uint64_t seed,
                   double* theta, void* stream);

/* One random-walk Metropolis-Hastings move of every particle, in place
 * (Population-Based MCMC subsection: the stage-one move of each chain is an
 * N(0, I) random walk; SMC Sampler subsection: the same move keeps each
 * tempered target invariant; Mixture Modelling section: the prior p0).
 * Proposal theta' = theta + step_sd * xi, xi ~ N(0, I_{kd}) jointly (normal c
 * of stream (p, c/4, step, PROP, move)). Accept iff log alpha >= 0 or
 * log u < log alpha, with log alpha = b_p (l' - l) + log p0(theta') - log p0(theta),
 * b_p = beta_vec[p] if beta_vec is non-NULL (one beta per chain) else beta,
 * u = (w0 + 1/2) 2^-32 from stream (p, 0, step, ACC, move).
 * theta, loglik: in/out (loglik must hold l(theta) on entry).
 * n_accept: nullable device u64 counter, incremented by the accepted count. */
int smc_rwmh_move(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n,
                  double* theta, double* loglik, int64_t N, const double* beta_vec,
                  double beta, double step_sd, uint64_t seed, uint64_t step,
                  uint32_t move, smc_prec prec, unsigned long long* n_accept,
                  void* stream);

/* Incremental reweight of a tempering step (SMC Sampler subsection: with a
 * pi_t-invariant move the incremental weight is pi_t/pi_{t-1} = L^dbeta):
 *   logw[p] += dbeta * loglik[p]            (in/out, FP64)
 *   W[p] = exp(logw[p] - m) / sum_q exp(logw[q] - m)   (out, nullable)
 *   *logZ += lse(logw_new) - lse(logw_old)  (device scalar in/out, nullable)
 *   *ess = 1 / sum W^2                      (device scalar out, nullable)
 * All three come out of one pass over (logw, loglik) plus a one-workgroup
 * combine in a fixed order (bit-reproducible). */
int smc_reweight(smc_ctx ctx, double* logw, const double* loglik, int64_t N, double dbeta,
                 double* W, double* logZ, double* ess, void* stream);

/* Effective sample size 1 / sum_p W[p]^2 of normalised weights W [N]
 * (Sequential Monte Carlo subsection: the ESS criterion that decides when to
 * resample). ess: device scalar out. One pass plus a fixed-order combine. */
int smc_ess(smc_ctx ctx, const double* W, int64_t N, double* ess, void* stream);

/* Systematic resampling (Sequential Monte Carlo subsection: build the
 * empirical CDF of the normalised weights and sample N times from it).
 * C_j is the correctly rounded prefix sum W_0 + ... + W_j (double-double scan,
 * rounded once); U_i = (i + u)/N with u = w0 2^-32 from stream
 * (0, 0, step, RESAMP, 0), or *u_override if non-NULL (device scalar in [0,1));
 * idx[i] = min{j : U_i < C_j}, or the first j with C_j = C_{N-1} if none.
 * If `ess` is non-NULL the step runs only when *ess < ess_threshold; when
 * skipped idx is the identity and theta_out/l_out are copies of the inputs.
 * idx: [N] int32 out (nullable). theta_in/theta_out: [kd][N] (nullable pair;
 * must not alias). l_in/l_out: [N] (nullable pair). logw: [N], set to 0 when
 * resampling happened (nullable). Bit-exact for N <= 2^20. */
int smc_resample_systematic(smc_ctx ctx, const double* W, int64_t N, uint64_t seed,
                            uint64_t step, const double* u_override, const double* ess,
                            double ess_threshold, int32_t* idx, const double* theta_in,
                            double* theta_out, int32_t kd, const double* l_in,
                            double* l_out, double* logw, void* stream);

/* Resampling under any scheme of smc_resampling, with the same arguments and
 * behaviour as smc_resample_systematic (no offset override). Multinomial
 * indices are in draw order (not sorted). Bit-exact for N <= 2^20. */
int smc_resample(smc_ctx ctx, smc_resampling scheme, const double* W, int64_t N, uint64_t seed,
                 uint64_t step, const double* ess, double ess_threshold, int32_t* idx,
                 const double* theta_in, double* theta_out, int32_t kd, const double* l_in,
                 double* l_out, double* logw, void* stream);

/* smc_resample for callers that cannot allocate device memory (code under
 * hipGraph stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments (no context), kernels and results, but the
 * scratch (correctly rounded CDF halves and chunk totals) lives in a fixed
 * 16 MiB device array of the library, one per GPU, held until the process
 * ends; the call itself allocates nothing (the array's device address is
 * looked up once per GPU, on the first call with that GPU current). N is
 * limited to 2^20 (larger N: SMC_ERR_INVALID_ARG, nothing enqueued). Every
 * call on one GPU shares that GPU's array: calls that overlap on one GPU (on
 * different streams, or from several threads) race; calls in one stream order
 * do not. Errors are reported by smc_last_error(). */
int smc_resample_noalloc(smc_resampling scheme, const double* W, int64_t N, uint64_t seed,
                         uint64_t step, const double* ess, double ess_threshold, int32_t* idx,
                         const double* theta_in, double* theta_out, int32_t kd,
                         const double* l_in, double* l_out, double* logw, void* stream);

/* The scheme used by later smc_step and smc_step_batched calls on this
 * context (default SYSTEMATIC); a captured graph keeps the scheme it was
 * captured with. */
int smc_set_resampling(smc_ctx ctx, smc_resampling scheme);

/* Exchange moves between adjacent chains (Population-Based MCMC subsection).
 * Pairs (a, a+1) with a = parity, parity+2, ... < M-1; with `wrap` and
 * parity 1 (M even) also (M-1, 0). log alpha = (beta[a] - beta[b]) (l_b - l_a);
 * swap the states and log-likelihoods iff log alpha >= 0 or log u < log alpha,
 * u = (w0 + 1/2) 2^-32 from stream (a, 0, iter, EXCH, 0).
 * theta: [kd][M] in/out; loglik, beta: [M]; n_swap: nullable device u32 counter. */
int pt_exchange(smc_ctx ctx, double* theta, double* loglik, const double* beta, int64_t M,
                int32_t kd, int32_t parity, int32_t wrap, uint64_t seed, uint64_t iter,
                unsigned int* n_swap, void* stream);

/* One whole tempering step of the SMC sampler with every per-step value read on
 * the device, so the same enqueued work can be captured once in a hipGraph and
 * replayed (SMC Samplers subsection; resampling as in the Sequential Monte
 * Carlo subsection):
 *   t = *t_dev clamped to 1..T; dbeta = beta[t] - beta[t-1];
 *   logw += dbeta * loglik_in; *logZ += lse(logw_new) - lse(logw_old);
 *   ESS = 1 / sum W^2; if ESS < ess_frac * N: resampling under the context's
 *   scheme (smc_set_resampling; systematic by default) with the points of
 *   step t, logw = 0;
 *   n_moves RW-MH moves at beta[t] (move m uses stream move m);
 *   *t_dev = t + 1.
 * The step reads the population (theta_in [k*d][N], loglik_in [N]) and writes
 * the next one (theta_out, loglik_out): the ancestor search and gather are
 * fused into the first move, so the two populations must not alias. Callers
 * alternate two buffers between steps. logw [N] and W [N] are updated in place
 * (W = the step's normalised weights, 1/N after resampling).
 * beta: [T+1] device FP64. stats: device FP64 [4] = {logZ (accumulated), last
 * ESS, resample count, unused}. n_accept: nullable device u64 counter.
 * Kernels: reweight partials; combine + decision + CDF chunk scans (when
 * resampling); the moves. */
int smc_step(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n, int64_t N,
             const double* theta_in, const double* loglik_in, double* theta_out,
             double* loglik_out, double* logw, double* W, const double* beta, int32_t T,
             int32_t* t_dev, double step_sd, int32_t n_moves, uint64_t seed, double ess_frac,
             smc_prec prec, double* stats, unsigned long long* n_accept, void* stream);

/* n_steps consecutive smc_step calls, the populations alternating: step i reads
 * (theta_a, loglik_a) for even i and (theta_b, loglik_b) for odd i and writes
 * the other pair, so the population ends in the a pair for even n_steps and
 * the b pair for odd. Same arguments and results as those calls, except that
 * with VALU precision, tiles of one workgroup each and all of a step's moves in
 * one launch (one move, or up to k*d = 16 several), the moves of every step but
 * the last also make the next step's reweight (and its log-sum-exp partials
 * per 64 particles), so that step runs without its own reweight pass: the
 * weights, ESS and evidence then come from partial sums grouped differently and
 * may differ from smc_step's in the last bits. W and logw are written by the
 * last step only (their values in between are not observable in the calls'
 * results either). Uses the context scratch (reserve N first when capturing). */
int smc_steps(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n, int64_t N,
              double* theta_a, double* loglik_a, double* theta_b, double* loglik_b,
              double* logw, double* W, const double* beta, int32_t T, int32_t* t_dev,
              int32_t n_steps, double step_sd, int32_t n_moves, uint64_t seed, double ess_frac,
              smc_prec prec, double* stats, unsigned long long* n_accept, void* stream);

/* One population-MCMC iteration with the iteration index read on the device
 * (graph-replayable): it = *it_dev; one RW-MH move per chain at its own
 * beta[i] with step = it; exchanges on partition parity (it & 1 when
 * parity_mode = 0; a Philox bit from stream (0, 0, it, PARITY, 0) when 1), with
 * the wrap pair if `wrap`; then *it_dev = it + 1. The move records `it` in the
 * context's step state and the exchange kernel advances *it_dev from there, so
 * the iteration is the move kernel(s) plus one exchange kernel. */
int pt_iteration(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n, int64_t M,
                 double* theta, double* loglik, const double* beta, int32_t* it_dev,
                 double step_sd, uint64_t seed, int32_t parity_mode, int32_t wrap,
                 smc_prec prec, unsigned long long* n_accept, unsigned int* n_swap,
                 void* stream);

/* n_iters consecutive pt_iteration calls: the same arguments, the same random
 * streams and the same results (bit for bit, for the same data slicing).
 * Small populations run all n_iters iterations in one launch of a single
 * workgroup that keeps the chains' states in LDS and takes each iteration's
 * exchanges there; this needs FP32 or FP64, M at most 1024 chains at
 * k*d <= 4 (576 at 7, 512 at 8, 256 at 16) and, by default, a small iteration
 * (64-chain tiles x n x k*d <= 2^16; see pt_set_single_workgroup). Larger
 * populations whose 64-chain tiles each fit one workgroup (the launch shape
 * of pt_iteration) take one launch per iteration: each launch first takes the
 * previous iteration's exchange, then this iteration's moves, alternating the
 * population between (theta, loglik) and context scratch (reserve M chains of
 * k*d first when capturing), and one closing launch takes the last exchange;
 * the rest enqueue n_iters pt_iteration calls. The single launch takes
 * smc_set_slices' value (at most 16 waves in all) or its own choice. *it_dev
 * advances by n_iters; n_iters < 1 is an argument error. */
int pt_iterations(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n, int64_t M,
                  double* theta, double* loglik, const double* beta, int32_t* it_dev,
                  int32_t n_iters, double step_sd, uint64_t seed, int32_t parity_mode,
                  int32_t wrap, smc_prec prec, unsigned long long* n_accept,
                  unsigned int* n_swap, void* stream);

/* Which fused forms pt_iterations may use: mode 0 (default) the
 * single-workgroup form when the population fits and the iteration is small,
 * else the deferred-exchange form when it applies; 1 the single-workgroup
 * form whenever the population fits; -1 neither (n_iters pt_iteration calls). */
int pt_set_single_workgroup(smc_ctx ctx, int32_t mode);

/* Record one chain's state after an iteration (graph-replayable; enqueue it
 * after pt_iteration): with it = *it_dev (the number of finished iterations),
 * out[(it - 1) * kd + c] = theta[c * M + chain] for c < kd, when
 * 1 <= it <= max_iters (otherwise nothing is written). out: device FP64
 * [max_iters][kd]. Used for the mode-traversal time of the beta = 1 chain
 * (Population-Based MCMC subsection). */
int pt_record(smc_ctx ctx, const double* theta, int64_t M, int32_t kd, int64_t chain,
              const int32_t* it_dev, double* out, int64_t max_iters, void* stream);

/* Many independent SMC runs advanced together (serving-style batch).
 * Run r owns particles [p_off, p_off + N) of the concatenated state arrays (its
 * theta block is [k*d][N] at theta + k*d*p_off) and observations
 * [y_off, y_off + n) of the concatenated data; all runs share the model, the
 * schedule beta[0..T] and the proposal sd, and each draws from its own Philox
 * key `seed`, exactly as it would alone. */
typedef struct {
    int64_t p_off, y_off;
    int32_t N, n;
    uint64_t seed;
} smc_run_desc;
typedef struct smc_batch_s* smc_batch;

/* [sync] Upload R run descriptors (host array) and size the batch scratch for
 * runs of kd = k*d parameters (d must be 1). The move's work list holds units
 * of 8 / S consecutive 64-particle tiles of one run, each tile moved by S
 * waves, ordered by decreasing n (longest first); S per run comes from the
 * context's SMC_RULE_BATCH launch rules in force now (one list per precision),
 * else the largest power of two <= min(8, n / 32) (at least 1). */
int smc_batch_create(smc_ctx ctx, const smc_run_desc* runs, int32_t R, int32_t kd,
                     smc_batch* out);
int smc_batch_destroy(smc_batch b);

/* One tempering step of every run of the batch, graph-replayable like smc_step
 * (t = *t_dev, advanced at the end):
 *   one workgroup per run: reweight, log-sum-exp, ESS and the resampling
 *   decision (ESS < ess_frac * N_r); one workgroup per resampling run:
 *   systematic resampling and gather; then n_moves (>= 1) RW-MH moves as one
 *   persistent launch over the work list (workgroups pull units from a device
 *   counter). run_stats: device FP64 [R][4] = {log Z (accumulated), last ESS,
 *   resample count, unused}. prec: FP32 or FP64. A run's results depend on its
 *   S only through the order of its FP64 slice sums and, in FP32, through which
 *   of the per-datum forms a wave takes and its data centre (see smc_loglik). */
int smc_step_batched(smc_ctx ctx, smc_batch b, const smc_gmm* model, const float* y,
                     double* theta, double* loglik, double* logw, double* W, const double* beta,
                     int32_t T, int32_t* t_dev, double step_sd, int32_t n_moves, double ess_frac,
                     smc_prec prec, double* run_stats, unsigned long long* n_accept,
                     void* stream);

/* Graph helpers: capture `reps` calls of smc_step (or pt_iteration) enqueued by
 * the caller between smc_graph_begin and smc_graph_end on `stream` into one
 * executable hipGraph, then launch it. */
typedef struct smc_graph_s* smc_graph;
int smc_graph_begin(smc_ctx ctx, void* stream);
int smc_graph_end(smc_ctx ctx, void* stream, smc_graph* out);
int smc_graph_launch(smc_graph g, void* stream);
int smc_graph_destroy(smc_graph g);

/* [sync] Diagnostic of the FP32 likelihood's per-datum forms (see
 * smc_loglik), summed over every context on the context's device since the
 * last reset, for the FP32 moves launched one move at a time (smc_rwmh_move,
 * and the moves of smc_step / smc_steps unless a step's several moves run in
 * one launch), counted in (observation, 64-particle tile) pairs. out[3]:
 *   out[0]: pairs evaluated in the plain shifted form: the data of a wave's
 *           slice (d > 1, or slices shorter than 128) or of a window the pivot
 *           form refused (d = 1) from where the wave left, or never took, the
 *           plain direct form; not counted: the fewer than 8 observations
 *           after the last full block of 8 of each such range, which always
 *           take the shifted form;
 *   out[1]: pairs evaluated in the pivot form;
 *   out[2]: the number of components other than the pivot that the pivot
 *           form evaluated, summed over those pairs (out[2] / out[1] is the
 *           mean, at most k - 1).
 * With reset != 0 the counts are cleared after the read. */
int smc_fp32_form_counts(smc_ctx ctx, uint64_t* out, int32_t reset);

/* Sort n FP32 values of the device array y in place into ascending order
 * (Mixture Modelling section: the data are independent draws, so the
 * likelihood, a sum over data, does not depend on their order; the 1-D FP32
 * likelihood's pivot form wants them ascending). The order is that of the
 * values' bit patterns read as sign-magnitude integers: -NaN < -inf < ... <
 * -0 < +0 < ... < +inf < +NaN. Device-side bitonic network, enqueued on
 * stream; no allocation. n in [0, 2^30] (0 and 1: nothing to do); y may be
 * NULL only when n is 0. The samplers of the Python binding sort their own
 * copy of 1-D data once when they are created. */
int smc_sort_data(float* y, int64_t n, void* stream);

/* Diagnostics used by the CPU/GPU bit-identity tests: Philox words and
 * Box-Muller normals for indices 0..count-1 of one stream.
 * rng_words out: [count][4] u32 for counter (i, block, step, purpose<<24|move).
 * rng_normals out: [per_index][count] FP64, normal c of index i at c*count + i. */
int smc_rng_words(uint64_t seed, int64_t count, uint32_t block, uint32_t step,
                  uint32_t purpose, uint32_t move, uint32_t* out, void* stream);
int smc_rng_normals(uint64_t seed, int64_t count, int32_t per_index, uint32_t step,
                    uint32_t purpose, uint32_t move, double* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* SMC_H */
