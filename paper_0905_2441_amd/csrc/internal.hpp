// Internal declarations shared by the HIP translation units of libsmcgpu.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smc.h"

namespace smc {

constexpr int kMaxSlices = 16;          // waves per workgroup in the likelihood kernels
constexpr int kMaxGroups = 8;           // workgroups sharing one 64-particle tile's data
constexpr int kSplitCap = 32768;        // largest N whose move may use several groups
constexpr int kRedBlock = 256;          // threads per block in the weight/resample kernels
constexpr int kMaxRedBlocks = 1024;     // grid cap of the grid-stride weight kernels
constexpr int kScanPerThread = 8;       // W elements per thread in the CDF scan
constexpr int kScanChunk = kRedBlock * kScanPerThread;

// Status bits raised by kernels and reported by smc_check.
enum StatusBits : int { kStatusNaN = 1, kStatusAllZeroWeight = 2 };

// Model constants in the form the kernels consume (built on the host once per call).
struct GmmDev {
    int k, d;
    float s32;                 // sqrt(log2(e) / (2 sigma2)), rounded to FP32
    float lw2[SMC_KMAX];       // log2 w_i, FP32
    double lw[SMC_KMAX];       // ln w_i, FP64
    double inv2s2;             // 1 / (2 sigma2)
    double cst;                // per-datum constant -(d/2) ln(2 pi sigma2)
    int prior;                 // SMC_PRIOR_GAUSS or SMC_PRIOR_BOX
    double pa, pb;
    double lp_const;           // Gaussian prior: -(1/2) ln(2 pi pb^2) per coordinate
    int unit_mass;             // sum_i w_i <= 1 (+1e-6): the FP32 form may skip the max shift
};

// Per-step values one kernel computes and later kernels of the same step read.
struct StepState {
    double M;                  // max log-weight after the reweight
    double S;                  // sum exp(logw - M)
    double S2;                 // sum exp(2 (logw - M))
    double lse_old, lse_new;
    double ess;
    int resampled;             // 1 when the ESS test fired this step
    int t;                     // step index of the current device-driven step
};

// Per-block partial of the reweight pass: running log-sum-exp of the old
// log-weights (mo, so) and of the new ones with the sum of squares (mn, s1, s2).
struct alignas(16) RwPartial {
    double mo, so, mn, s1, s2, pad;
};

constexpr int kMaxChunks = 1024;        // CDF chunks (one per scan block)

// Device scratch owned by a context.
struct Scratch {
    RwPartial* rw_part;        // [kMaxRedBlocks]
    double* sq_part;           // [kMaxRedBlocks]
    double* dd_part;           // [2 * kMaxChunks] chunk totals (hi, lo)
    int* status;               // [1]
    StepState* state;          // [1]
    double* cdf_hi;            // [cap] within-chunk inclusive prefix, high part
    double* cdf_lo;            // [cap] low part
    double* res_tot;           // standalone resampling: chunk totals [2 * res_chunks(cap)]
    double* res_off;           // standalone resampling: chunk offsets [2 * res_chunks(cap)]
    double* theta_tmp;         // [kd * cap]
    double* l_tmp;             // [cap]
    int64_t cap;
    __bf16* mm_rows;           // MFMA path: data rows in the K layout [mm_rows_cap][64]
    __bf16* mm_cols;           // MFMA path: particle-component columns [mm_n_cap * 8][64]
    double* mm_prop;           // MFMA path: proposals [64][mm_n_cap]
    double* mm_part;           // MFMA path: per-slice partial sums [16][mm_n_cap]
    int64_t mm_rows_cap, mm_n_cap;
    double* mv_part;           // split move: partial sums [kMaxGroups][kSplitCap]
    int* mv_anc;               // split move: ancestors of the fused resampling [kSplitCap]
};

// How kernels obtain the step / iteration index and the inverse temperature:
// from host scalars, or (graph replay) from a device counter and beta array.
struct StepSrc {
    const int* t_dev;          // nullable: device step counter
    const double* beta_dev;    // nullable: device beta[0..t_max]
    int t_max;                 // with beta_dev: steps index beta[1..t_max]; t is clamped
    int t_host;
    double beta_host;
    double dbeta_host;
};

// Step index of the current call: the device counter (clamped to 1..t_max when a
// beta array is indexed with it) or the host value.
__device__ __forceinline__ int step_index(const StepSrc& src) {
    if (!src.t_dev) return src.t_host;
    int t = *src.t_dev;
    if (src.beta_dev) t = t < 1 ? 1 : (t > src.t_max ? src.t_max : t);
    return t;
}

// Where a random-walk move reads each particle's current state and the extra
// duties of the first move of a fused tempering step.
//   * The move writes the arrays it is given (theta, l). Its current state is
//     read from theta_src/l_src (default: the written arrays, i.e. in place).
//   * When the step's ESS test fired (state->resampled):
//       - with theta_alt set, the current state is the population gathered by a
//         separate search-and-gather pass;
//       - with cdf_hi set, the move finds each particle's ancestor itself
//         (systematic offsets, binary search of the correctly rounded CDF kept
//         as within-chunk prefixes plus chunk totals) and reads the ancestor
//         from theta_src/l_src, which must then differ from the written arrays.
//   * W_out: publish the step's normalised weights (1/N after resampling);
//     reset_logw: set logw to 0 after resampling.
struct MoveStep {
    const double* theta_src;
    const double* l_src;
    const double* theta_alt;
    const double* l_alt;
    const StepState* state;    // nullable: no step duties
    double* W_out;
    double* logw;
    int reset_logw;
    const double* cdf_hi;
    const double* cdf_lo;
    const double* chunk_tot;   // [2 * nchunks] (hi, lo)
    int chunk, nchunks;
    uint64_t seed;
    int scheme;                // resampling points (smc_resampling)
    int* t_out;                // nullable: the move records its step index here
    // a chain of tempering steps (smc_steps): the move also writes the step's
    // final log-weights to logw_out (0 after resampling, else logw) and, with
    // lw_next set, the next step's reweighted ones, lw_next[p] = that value +
    // (beta[t1] - beta[t1 - 1]) l[p] with t1 = min(t + 1, t_max), and per
    // 64-particle tile the log-sum-exp partials of the new weights (next_part:
    // mn, s1, s2; the old weights' log-sum-exp is known from the step state)
    double* logw_out;
    double* lw_next;
    RwPartial* next_part;
    const double* beta_dev;
    int t_max;
};

// Launch shape of a VALU move for one 64-particle tile: `groups` workgroups of
// `slices` waves split the observations into groups * slices contiguous slices.
// With groups > 1 each workgroup writes its partial sums to scratch and a
// per-particle kernel completes the move.
struct Split {
    int slices;
    int groups;
};

// How the CDF kernels obtain the normalised weights: read W, or form
// exp(logw - M) / S from the step state.
struct WeightSrc {
    const double* W;           // nullable
    const double* logw;
    const StepState* state;
};

// Batched runs (one step for many independent SMC runs).
struct BatchRun {
    int64_t p_off, y_off;      // first particle / observation of the run
    int N, n;
    uint64_t seed;
};
constexpr int kBatchWaves = 8;          // waves per workgroup of the persistent batched move
// Work unit of the persistent batched move: ntiles consecutive 64-particle
// tiles of run `run` from tile0 on, each moved by `slices` waves (slices *
// ntiles <= kBatchWaves).
struct BatchUnit {
    int run, tile0, ntiles, slices;
};
struct BatchDev {
    int R;
    BatchRun* runs;            // [R]
    BatchUnit* units[2];       // work lists of the FP64 [0] and FP32 [1] moves, longest data first
    int n_units[2];
    unsigned* work;            // work-queue counter, zero between launches
    StepState* state;          // [R]
    double* cdf;               // [N_total]
    double* theta_tmp;         // [kd * N_total]
    double* l_tmp;             // [N_total]
    int move_grid;             // persistent grid size
};
int batch_move_grid();
hipError_t launch_batch_step(const BatchDev& b, const GmmDev& g, const float* y, double* theta,
                             double* l, double* logw, double* W, const double* beta, int T,
                             int* t_dev, double sd, int n_moves, double ess_frac, int prec,
                             double* stats, unsigned long long* n_acc, int* status, int scheme,
                             hipStream_t s);

// Read (and with reset, clear) the device's count of observations x tiles that
// FP32 single moves evaluated in the shifted form (synchronous).
hipError_t fp32_form_counts(unsigned long long* out, bool reset);   // out[kFormCounts]

// The text smc_last_error() returns on this thread (set by every failing call).
void set_last_error(const char* msg);

hipError_t launch_loglik(const GmmDev& g, const float* y, int64_t n, const double* theta,
                         int64_t N, int prec, double* out, int slices, int* status,
                         hipStream_t s);
hipError_t launch_rwmh(const GmmDev& g, const float* y, int64_t n, double* theta, double* l,
                       int64_t N, const double* beta_vec, StepSrc src, double sd,
                       uint64_t seed, uint32_t move, int prec,
                       unsigned long long* n_accept, Split sp, const Scratch& sc, MoveStep ms,
                       hipStream_t s);
// The n_moves moves of one tempering step (move numbers 0..n_moves-1; ms holds
// the first move's duties): one launch with the tiles' states in LDS when a
// tile fits one workgroup and k*d <= 16, else one launch per move.
// Whether launch_rwmh_moves runs all n_moves in one launch of one workgroup per
// tile (a single move, or the LDS-resident multi-move kernel at k*d <= 16), the
// form whose last move can also make the next step's reweight (MoveStep.lw_next).
bool rwmh_moves_chainable(const GmmDev& g, int n_moves, const Split& sp);
hipError_t launch_rwmh_moves(const GmmDev& g, const float* y, int64_t n, double* theta,
                             double* l, int64_t N, StepSrc src, double sd, uint64_t seed,
                             int n_moves, int prec, unsigned long long* n_accept, Split sp,
                             const Scratch& sc, MoveStep ms, hipStream_t s);
// Largest population the one-workgroup population-MCMC form holds (0: none).
int pt_local_chains(int kd);
bool pt_local_pays(int kd, int64_t n, int64_t M);
// n_iters population-MCMC iterations with one launch each (the exchange of an
// iteration deferred into the next launch) plus one closing exchange; the
// population alternates between (theta, l) and the scratch theta_tmp/l_tmp
// (sc.cap >= M, kd rows), and the iteration index between *it_dev and
// *counter2. Tiles of 64 chains in one workgroup of `slices` waves.
hipError_t launch_pt_deferred(const GmmDev& g, const float* y, int64_t n, double* theta,
                              double* l, int64_t M, const double* beta, int* it_dev,
                              int n_iters, double sd, uint64_t seed, int prec, int parity_mode,
                              int wrap, int slices, unsigned long long* n_accept,
                              unsigned* n_swap, const Scratch& sc, int* counter2,
                              hipStream_t s);
int pt_local_slices(int64_t n, int64_t M);
// n_iters population-MCMC iterations in one single-workgroup launch (chains in
// LDS; M <= pt_local_chains(k*d)); `slices` data slices per 64-chain tile.
hipError_t launch_pt_local(const GmmDev& g, const float* y, int64_t n, double* theta, double* l,
                           int64_t M, const double* beta, int* it_dev, int n_iters, double sd,
                           uint64_t seed, int prec, int parity_mode, int wrap, int slices,
                           unsigned long long* n_accept, unsigned* n_swap, int* status,
                           hipStream_t s);
// One population-MCMC iteration: the move (reading the iteration from src and
// recording it through ms.t_out), then the exchanges (reading it from later and
// advancing *t_advance); with groups > 1 the decisions of both run in one kernel.
hipError_t launch_pt_iteration(const GmmDev& g, const float* y, int64_t n, double* theta,
                               double* l, int64_t M, const double* beta, StepSrc src,
                               StepSrc later, double sd, uint64_t seed, int prec,
                               unsigned long long* n_accept, Split sp, const Scratch& sc,
                               MoveStep ms, int parity_mode, int wrap, int* t_advance,
                               unsigned* n_swap, hipStream_t s);
hipError_t launch_prior(const GmmDev& g, int64_t N, uint64_t seed, double* theta,
                        hipStream_t s);
bool supported_kd(int k, int d, int prec);

// MFMA (split-BF16) form of the d-dimensional likelihood and move.
int64_t dd_padded_rows(int64_t n);
int dd_slices(int64_t n, int64_t N);
int dd_clamp_slices(int64_t n, int64_t S);   // to 1..min(16, 16-row data tiles)
bool dd_supported(int k, int d);
hipError_t launch_dd_prep(const GmmDev& g, const float* y, int64_t n, __bf16* A, hipStream_t s);
hipError_t launch_dd_loglik(const GmmDev& g, const __bf16* A, int64_t n, const double* theta,
                            int64_t N, __bf16* B, double* part, int S, double* out, int* status,
                            hipStream_t s);
hipError_t launch_dd_rwmh(const GmmDev& g, const __bf16* A, int64_t n, double* theta, double* l,
                          int64_t N, const double* beta_vec, StepSrc src, double sd,
                          uint64_t seed, uint32_t move, unsigned long long* n_accept,
                          __bf16* B, double* theta_prop, double* part, int S, int* status,
                          MoveStep ms, hipStream_t s);

// Reweight pass and its one-block finalisation. With t_dev set (fused step)
// the finaliser also records t in the step state and advances the counter.
hipError_t launch_reweight(const Scratch& sc, double* logw, const double* l, int64_t N,
                           StepSrc src, int* t_advance, double* logZ, double* ess,
                           double ess_frac, double* resample_count, hipStream_t s);
hipError_t launch_weights(const Scratch& sc, const double* logw, int64_t N, double* W,
                          hipStream_t s);
hipError_t launch_ess(const Scratch& sc, const double* W, int64_t N, double* ess,
                      hipStream_t s);
// Resampling (scheme: smc_resampling): CDF of the weights, then search and
// gather. pred_ess / pred_state make both kernels no-ops unless the ESS test fired.
// Chunks of the standalone resampling CDF for N particles (1024 per chunk).
inline int64_t res_chunks(int64_t N) { return (N + kRedBlock * 4 - 1) / (kRedBlock * 4); }

hipError_t launch_resample(const Scratch& sc, WeightSrc w, int64_t N, int scheme, uint64_t seed,
                           StepSrc src, const double* u_override, const double* pred_ess,
                           double ess_threshold, const StepState* pred_state,
                           int32_t* idx, const double* theta_in, double* theta_out,
                           int32_t kd, const double* l_in, double* l_out, double* logw,
                           int copy_when_skipped, hipStream_t s);
hipError_t launch_exchange(double* theta, double* l, const double* beta, int64_t M,
                           int32_t kd, int parity_mode, int parity_host, int wrap,
                           uint64_t seed, StepSrc src, int* t_advance, unsigned* n_swap,
                           hipStream_t s);
// Fused tempering step pieces: reweight partials -> step_mid (combine, decide,
// CDF chunks) -> moves (ancestor search fused into the first move).
// With `mom` (a particle filter's moment partials), also the step's weighted
// moments into moments[(t-1) * 2 mom_k ...] (means, then standard deviations).
// With `part` (nparts per-tile partials of the new weights made by the previous
// step's move in a chain of steps), the combine reads those instead of the
// reweight pass's, and the old weights' log-sum-exp is the previous step's
// (log N after a resampling) from the step state.
hipError_t launch_step_mid(const Scratch& sc, int64_t N, StepSrc src, int* t_advance,
                           double* stats, double ess_frac, const double* logw, hipStream_t s,
                           const double* mom = nullptr, int mom_k = 0, int mom_stride = 0,
                           double* moments = nullptr, const RwPartial* part = nullptr,
                           int nparts = 0);
void cdf_layout(int64_t N, int* chunk, int* nchunks);
hipError_t launch_search_gather(const Scratch& sc, int64_t N, int scheme, uint64_t seed,
                                StepSrc src, const StepState* pred_state, const double* theta_in,
                                double* theta_out, int32_t kd, const double* l_in, double* l_out,
                                double* logw, int copy_when_skipped, hipStream_t s);
hipError_t launch_publish_w(const Scratch& sc, double* W, const double* logw, int64_t N,
                            hipStream_t s);
hipError_t launch_reweight_partial(const Scratch& sc, double* logw, const double* l, int64_t N,
                                   StepSrc src, hipStream_t s);
hipError_t launch_pt_record(const double* theta, int64_t M, int32_t kd, int64_t chain,
                            const int32_t* it_dev, double* out, int64_t max_iters, hipStream_t s);
hipError_t launch_sort_data(float* y, int64_t n, hipStream_t s);
hipError_t launch_rng_words(uint64_t seed, int64_t count, uint32_t block, uint32_t step,
                            uint32_t purpose, uint32_t move, uint32_t* out, hipStream_t s);
hipError_t launch_rng_normals(uint64_t seed, int64_t count, int32_t per_index, uint32_t step,
                              uint32_t purpose, uint32_t move, double* out, hipStream_t s);

}  // namespace smc
