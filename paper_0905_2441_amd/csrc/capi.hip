// C ABI of libsmcgpu: argument checking, context scratch, launch choices,
// tempering-step orchestration and hipGraph capture helpers.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "fsv.hpp"
#include "internal.hpp"
#include "wave.hpp"

using namespace smc;

struct smc_ctx_s {
    int device = 0;
    int slices_override = 0;
    int pt_single = 0;                        // pt_set_single_workgroup mode
    int scheme = SMC_RESAMPLE_SYSTEMATIC;
    std::vector<smc_launch_rule> table;
    Scratch sc{};
    void* fixed = nullptr;       // partials, chunk totals, status, state
    void* grow = nullptr;        // cdf, dd partials, l_tmp, theta_tmp
    int64_t grow_kd = 0;
    void* mm = nullptr;          // MFMA form: data rows, columns, proposals, partials
    double* fsv_mom = nullptr;   // particle filter: per-block moment sums (in `fixed`)
    // Scratch superseded by a larger allocation. Graphs captured earlier hold
    // its addresses as kernel arguments, so it stays allocated (and those
    // graphs valid) until the context is destroyed.
    std::vector<void*> retired;
};

struct smc_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(SMC_ERR_HIP, m);
}

#define SMC_CHECK_HIP(call, what)                 \
    do {                                          \
        hipError_t e_ = (call);                   \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

bool capturing(hipStream_t s) {
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
    return st != hipStreamCaptureStatusNone;
}

size_t align_up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

int check_model(const smc_gmm* m, GmmDev* out) {
    if (!m) return fail(SMC_ERR_INVALID_ARG, "model is NULL");
    if (m->k < 1 || m->k > SMC_KMAX) return fail(SMC_ERR_INVALID_ARG, "k must be in 1..8");
    if (m->d < 1 || m->d > SMC_DMAX) return fail(SMC_ERR_INVALID_ARG, "d must be in 1..8");
    if (!(m->sigma2 > 0.0) || !isfinite(m->sigma2))
        return fail(SMC_ERR_INVALID_ARG, "sigma2 must be positive and finite");
    bool any_finite = false;
    for (int i = 0; i < m->k; ++i) {
        if (m->log_w[i] != m->log_w[i] || m->log_w[i] == INFINITY)
            return fail(SMC_ERR_INVALID_ARG, "log_w must not be NaN or +inf");
        any_finite = any_finite || isfinite(m->log_w[i]);
    }
    if (!any_finite) return fail(SMC_ERR_INVALID_ARG, "every mixture weight is zero");
    if (m->prior == SMC_PRIOR_GAUSS) {
        if (!(m->prior_b > 0.0) || !isfinite(m->prior_a) || !isfinite(m->prior_b))
            return fail(SMC_ERR_INVALID_ARG, "Gaussian prior needs finite mean and sd > 0");
    } else if (m->prior == SMC_PRIOR_BOX) {
        if (!(m->prior_b > m->prior_a) || !isfinite(m->prior_a) || !isfinite(m->prior_b))
            return fail(SMC_ERR_INVALID_ARG, "box prior needs finite a < b");
    } else {
        return fail(SMC_ERR_INVALID_ARG, "unknown prior kind");
    }
    GmmDev g{};
    g.k = m->k;
    g.d = m->d;
    const double log2e = 1.4426950408889634;
    g.s32 = static_cast<float>(sqrt(log2e / (2.0 * m->sigma2)));
    double mass = 0.0;
    for (int i = 0; i < SMC_KMAX; ++i) {
        const double lw = (i < m->k) ? m->log_w[i] : -INFINITY;
        g.lw[i] = lw;
        g.lw2[i] = static_cast<float>(lw * log2e);
        mass += exp(lw);
    }
    g.unit_mass = mass <= 1.0 + 1e-6 ? 1 : 0;
    g.inv2s2 = 1.0 / (2.0 * m->sigma2);
    g.cst = -0.5 * static_cast<double>(m->d) * log(2.0 * M_PI * m->sigma2);
    g.prior = m->prior;
    g.pa = m->prior_a;
    g.pb = m->prior_b;
    g.lp_const = (m->prior == SMC_PRIOR_GAUSS) ? -0.5 * log(2.0 * M_PI * m->prior_b * m->prior_b)
                                               : 0.0;
    *out = g;
    return SMC_OK;
}

int check_prec(const GmmDev& g, int prec) {
    if (prec != SMC_PREC_FP64 && prec != SMC_PREC_FP32 && prec != SMC_PREC_BF16X3)
        return fail(SMC_ERR_INVALID_ARG, "unknown precision");
    if (!supported_kd(g.k, g.d, prec))
        return fail(SMC_ERR_UNSUPPORTED, "(k, d, precision) combination is not compiled");
    return SMC_OK;
}

int check_sizes(int64_t n, int64_t N) {
    if (n < 1 || n > (int64_t{1} << 30)) return fail(SMC_ERR_INVALID_ARG, "n must be in 1..2^30");
    if (N < 1 || N > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "N must be in 1..2^31-1");
    return SMC_OK;
}

// Slices per tile from the first launch rule of `kind` that matches (0 when none).
int64_t table_slices(const smc_ctx_s* ctx, int k, int d, int prec, int64_t n, int64_t N,
                     int kind = SMC_RULE_CALL) {
    for (const smc_launch_rule& r : ctx->table) {
        if (r.kind == kind && (r.k == 0 || r.k == k) && (r.d == 0 || r.d == d) &&
            (r.prec < 0 || r.prec == prec) && n >= r.n_lo && n <= r.n_hi && N >= r.N_lo &&
            N <= r.N_hi)
            return r.slices;
    }
    return 0;
}

int64_t table_slices(const smc_ctx_s* ctx, const GmmDev& g, int prec, int64_t n, int64_t N) {
    return table_slices(ctx, g.k, g.d, prec, n, N);
}

// Waves per 64-particle tile of a batched run: its SMC_RULE_BATCH rule, else
// the largest power of two <= min(kBatchWaves, n / 32), at least 1.
int batch_slices(const smc_ctx_s* ctx, int k, int prec, int64_t n, int64_t N) {
    const int64_t t = table_slices(ctx, k, 1, prec, n, N, SMC_RULE_BATCH);
    if (t > 0) return static_cast<int>(t);
    int S = 1;
    while (2 * S <= kBatchWaves && 2 * S <= n / 32) S *= 2;
    return S;
}

// Data slices per 64-particle tile: the explicit override, else the launch
// table, else the built-in choice: enough waves to fill 256 CUs several times
// over (about 8192), at least 32 observations per slice, and a grid within 2^32
// threads. More than kMaxSlices slices (small N, long data) are spread over up
// to kMaxGroups workgroups per tile so that every CU receives work; only moves
// with N <= kSplitCap do that, everything else stays within one workgroup.
Split choose_split(const smc_ctx_s* ctx, const GmmDev& g, int prec, int64_t n, int64_t N,
                   bool allow_groups) {
    const int64_t tiles = (N + kWave - 1) / kWave;
    int64_t T = ctx->slices_override;
    if (T <= 0) T = table_slices(ctx, g, prec, n, N);
    if (T <= 0) {
        T = (8192 + tiles - 1) / tiles;
        if (T > kMaxSlices * kMaxGroups) T = kMaxSlices * kMaxGroups;
        while (T > 1 && n / T < 32) --T;
    }
    if (T > n) T = n;
    if (T < 1) T = 1;
    if (!allow_groups || N > kSplitCap) T = T < kMaxSlices ? T : kMaxSlices;
    const int64_t G = (T + kMaxSlices - 1) / kMaxSlices;
    int64_t S = (T + G - 1) / G;
    while (S > 1 && tiles * kWave * S * G >= (int64_t{1} << 32)) --S;
    return Split{static_cast<int>(S), static_cast<int>(G)};
}

int choose_slices(const smc_ctx_s* ctx, const GmmDev& g, int prec, int64_t n, int64_t N) {
    return choose_split(ctx, g, prec, n, N, false).slices;
}

// Slices of the MFMA form: the override or table entry clamped to its limits,
// else its own built-in choice.
int choose_dd_slices(const smc_ctx_s* ctx, const GmmDev& g, int64_t n, int64_t N) {
    int64_t T = ctx->slices_override;
    if (T <= 0) T = table_slices(ctx, g, SMC_PREC_BF16X3, n, N);
    return T > 0 ? dd_clamp_slices(n, T) : dd_slices(n, N);
}

int ensure_scratch(smc_ctx ctx, int64_t N, int64_t kd, hipStream_t s) {
    if (ctx->sc.cap >= N && ctx->grow_kd >= kd) return SMC_OK;
    if (capturing(s))
        return fail(SMC_ERR_CAPTURE, "scratch must grow; call smc_reserve before capture");
    const int64_t cap = ctx->sc.cap >= N ? ctx->sc.cap : N;
    const int64_t kdc = ctx->grow_kd >= kd ? ctx->grow_kd : (kd < 8 ? 8 : kd);
    const size_t b_cdf = align_up(sizeof(double) * cap);
    const size_t b_l = align_up(sizeof(double) * cap);
    const size_t b_th = align_up(sizeof(double) * cap * kdc);
    const size_t b_res = align_up(sizeof(double) * 2 * res_chunks(cap));
    SMC_CHECK_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    SMC_CHECK_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize before scratch growth");
    if (ctx->grow) {
        ctx->retired.push_back(ctx->grow);
        ctx->grow = nullptr;
    }
    void* p = nullptr;
    if (hipMalloc(&p, 2 * b_cdf + b_l + b_th + 2 * b_res) != hipSuccess) {
        ctx->sc.cap = 0;
        ctx->grow_kd = 0;
        return fail(SMC_ERR_NOMEM, "device allocation of context scratch failed");
    }
    char* c = static_cast<char*>(p);
    ctx->grow = p;
    ctx->sc.cdf_hi = reinterpret_cast<double*>(c);
    ctx->sc.cdf_lo = reinterpret_cast<double*>(c + b_cdf);
    ctx->sc.l_tmp = reinterpret_cast<double*>(c + 2 * b_cdf);
    ctx->sc.theta_tmp = reinterpret_cast<double*>(c + 2 * b_cdf + b_l);
    ctx->sc.res_tot = reinterpret_cast<double*>(c + 2 * b_cdf + b_l + b_th);
    ctx->sc.res_off = reinterpret_cast<double*>(c + 2 * b_cdf + b_l + b_th + b_res);
    ctx->sc.cap = cap;
    ctx->grow_kd = kdc;
    return SMC_OK;
}

// Scratch of the MFMA form: data rows [n_pad][64] bf16, particle-component
// columns [N*8][64] bf16, proposals [64][N] and slice partials [16][N] FP64.
int ensure_mm_scratch(smc_ctx ctx, int64_t n, int64_t N, hipStream_t s) {
    const int64_t rows = dd_padded_rows(n);
    if (ctx->sc.mm_rows_cap >= rows && ctx->sc.mm_n_cap >= N) return SMC_OK;
    if (capturing(s))
        return fail(SMC_ERR_CAPTURE, "scratch must grow; call smc_reserve before capture");
    const int64_t rc = ctx->sc.mm_rows_cap >= rows ? ctx->sc.mm_rows_cap : rows;
    const int64_t nc = ctx->sc.mm_n_cap >= N ? ctx->sc.mm_n_cap : N;
    const size_t b_rows = align_up(static_cast<size_t>(rc) * 128);
    const size_t b_cols = align_up(static_cast<size_t>(nc) * SMC_KMAX * 128);
    const size_t b_prop = align_up(sizeof(double) * nc * SMC_KDMAX);
    const size_t b_part = align_up(sizeof(double) * nc * kMaxSlices);
    SMC_CHECK_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    SMC_CHECK_HIP(hipDeviceSynchronize(), "hipDeviceSynchronize before scratch growth");
    if (ctx->mm) {
        ctx->retired.push_back(ctx->mm);
        ctx->mm = nullptr;
    }
    void* p = nullptr;
    if (hipMalloc(&p, b_rows + b_cols + b_prop + b_part) != hipSuccess) {
        ctx->sc.mm_rows_cap = 0;
        ctx->sc.mm_n_cap = 0;
        return fail(SMC_ERR_NOMEM, "device allocation of MFMA scratch failed");
    }
    char* c = static_cast<char*>(p);
    ctx->mm = p;
    ctx->sc.mm_rows = reinterpret_cast<__bf16*>(c);
    ctx->sc.mm_cols = reinterpret_cast<__bf16*>(c + b_rows);
    ctx->sc.mm_prop = reinterpret_cast<double*>(c + b_rows + b_cols);
    ctx->sc.mm_part = reinterpret_cast<double*>(c + b_rows + b_cols + b_prop);
    ctx->sc.mm_rows_cap = rc;
    ctx->sc.mm_n_cap = nc;
    return SMC_OK;
}

int enter(smc_ctx ctx) {
    if (!ctx) return fail(SMC_ERR_INVALID_ARG, "context is NULL");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return SMC_OK;
}

StepSrc host_src(int t, double beta, double dbeta) {
    StepSrc s{};
    s.t_dev = nullptr;
    s.beta_dev = nullptr;
    s.t_host = t;
    s.beta_host = beta;
    s.dbeta_host = dbeta;
    return s;
}

}  // namespace

namespace smc {
void set_last_error(const char* msg) { g_last_error = msg; }
}  // namespace smc

extern "C" {

const char* smc_last_error(void) { return g_last_error.c_str(); }

int smc_create(smc_ctx* out, int device) {
    if (!out) return fail(SMC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    int count = 0;
    SMC_CHECK_HIP(hipGetDeviceCount(&count), "hipGetDeviceCount");
    if (device < 0 || device >= count) return fail(SMC_ERR_INVALID_ARG, "no such device");
    SMC_CHECK_HIP(hipSetDevice(device), "hipSetDevice");
    smc_ctx ctx = new (std::nothrow) smc_ctx_s();
    if (!ctx) return fail(SMC_ERR_NOMEM, "host allocation failed");
    ctx->device = device;
    const size_t b_part = align_up(sizeof(RwPartial) * kMaxRedBlocks);
    const size_t b_sq = align_up(sizeof(double) * kMaxRedBlocks);
    const size_t b_dd = align_up(sizeof(double) * 2 * kMaxChunks);
    const size_t b_st = align_up(sizeof(int));
    const size_t b_state = align_up(sizeof(StepState));
    const size_t b_mv = align_up(sizeof(double) * kMaxGroups * kSplitCap);
    const size_t b_anc = align_up(sizeof(int) * kSplitCap);
    const size_t b_fsv = align_up(sizeof(double) * kMaxRedBlocks * 2 * SMC_FSV_KMAX);
    const size_t total = b_part + b_sq + b_dd + b_st + b_state + b_mv + b_anc + b_fsv;
    void* p = nullptr;
    if (hipMalloc(&p, total) != hipSuccess) {
        delete ctx;
        return fail(SMC_ERR_NOMEM, "device allocation of context scratch failed");
    }
    if (hipMemset(p, 0, total) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(p);
        delete ctx;
        return fail(SMC_ERR_HIP, "clearing context scratch failed");
    }
    char* c = static_cast<char*>(p);
    ctx->fixed = p;
    ctx->sc.rw_part = reinterpret_cast<RwPartial*>(c);
    ctx->sc.sq_part = reinterpret_cast<double*>(c + b_part);
    ctx->sc.dd_part = reinterpret_cast<double*>(c + b_part + b_sq);
    ctx->sc.status = reinterpret_cast<int*>(c + b_part + b_sq + b_dd);
    ctx->sc.state = reinterpret_cast<StepState*>(c + b_part + b_sq + b_dd + b_st);
    ctx->sc.mv_part = reinterpret_cast<double*>(c + b_part + b_sq + b_dd + b_st + b_state);
    ctx->sc.mv_anc = reinterpret_cast<int*>(c + b_part + b_sq + b_dd + b_st + b_state + b_mv);
    ctx->fsv_mom =
        reinterpret_cast<double*>(c + b_part + b_sq + b_dd + b_st + b_state + b_mv + b_anc);
    *out = ctx;
    return SMC_OK;
}

int smc_destroy(smc_ctx ctx) {
    if (!ctx) return SMC_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->grow) (void)hipFree(ctx->grow);
    if (ctx->mm) (void)hipFree(ctx->mm);
    for (void* p : ctx->retired) (void)hipFree(p);
    if (ctx->fixed) (void)hipFree(ctx->fixed);
    delete ctx;
    return SMC_OK;
}

int smc_reserve(smc_ctx ctx, int64_t N, int32_t kd, int64_t n) {
    int r = enter(ctx);
    if (r) return r;
    if (N < 1 || N > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "N must be in 1..2^31-1");
    if (kd < 1 || kd > SMC_KDMAX) return fail(SMC_ERR_INVALID_ARG, "kd in 1..64");
    if (n < 0 || n > (int64_t{1} << 30)) return fail(SMC_ERR_INVALID_ARG, "n in 0..2^30");
    if ((r = ensure_scratch(ctx, N, kd, nullptr))) return r;
    if (n > 0) return ensure_mm_scratch(ctx, n, N, nullptr);
    return SMC_OK;
}

int smc_check(smc_ctx ctx, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    SMC_CHECK_HIP(hipStreamSynchronize(as_stream(stream)), "hipStreamSynchronize");
    int flag = 0;
    SMC_CHECK_HIP(hipMemcpy(&flag, ctx->sc.status, sizeof(int), hipMemcpyDeviceToHost),
                  "hipMemcpy status");
    if (flag) {
        const int zero = 0;
        SMC_CHECK_HIP(hipMemcpy(ctx->sc.status, &zero, sizeof(int), hipMemcpyHostToDevice),
                      "hipMemcpy status");
        std::string m = "device status:";
        if (flag & kStatusNaN) m += " NaN or +inf in log-likelihoods or log-weights;";
        if (flag & kStatusAllZeroWeight) m += " every weight is zero;";
        return fail(SMC_ERR_NUMERIC, m);
    }
    return SMC_OK;
}

int smc_set_slices(smc_ctx ctx, int32_t slices) {
    if (!ctx) return fail(SMC_ERR_INVALID_ARG, "context is NULL");
    if (slices < 0 || slices > kMaxSlices * kMaxGroups)
        return fail(SMC_ERR_INVALID_ARG, "slices in 0..128");
    ctx->slices_override = slices;
    return SMC_OK;
}

int pt_set_single_workgroup(smc_ctx ctx, int32_t mode) {
    if (!ctx) return fail(SMC_ERR_INVALID_ARG, "context is NULL");
    if (mode < -1 || mode > 1) return fail(SMC_ERR_INVALID_ARG, "mode in -1..1");
    ctx->pt_single = mode;
    return SMC_OK;
}

int smc_set_launch_table(smc_ctx ctx, const smc_launch_rule* rules, int32_t count) {
    if (!ctx) return fail(SMC_ERR_INVALID_ARG, "context is NULL");
    if (count < 0 || (count > 0 && !rules)) return fail(SMC_ERR_INVALID_ARG, "bad rule array");
    for (int32_t i = 0; i < count; ++i) {
        const smc_launch_rule& r = rules[i];
        if (r.kind != SMC_RULE_CALL && r.kind != SMC_RULE_BATCH)
            return fail(SMC_ERR_INVALID_ARG, "rule kind is SMC_RULE_CALL or SMC_RULE_BATCH");
        if (r.slices < 1 || r.slices > kMaxSlices * kMaxGroups)
            return fail(SMC_ERR_INVALID_ARG, "rule slices in 1..128");
        if (r.kind == SMC_RULE_BATCH && (r.slices > kBatchWaves || (r.slices & (r.slices - 1))))
            return fail(SMC_ERR_INVALID_ARG, "batch rule slices must be 1, 2, 4 or 8");
        if (r.n_lo > r.n_hi || r.N_lo > r.N_hi || r.k < 0 || r.d < 0 || r.prec < -1)
            return fail(SMC_ERR_INVALID_ARG, "rule ranges are empty or fields negative");
    }
    ctx->table.assign(rules, rules + count);
    return SMC_OK;
}

int smc_loglik(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n,
               const double* theta, int64_t N, smc_prec prec, double* loglik, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    GmmDev g;
    if ((r = check_model(model, &g))) return r;
    if ((r = check_prec(g, prec))) return r;
    if ((r = check_sizes(n, N))) return r;
    if (!y || !theta || !loglik) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    const hipStream_t s = as_stream(stream);
    if (prec == SMC_PREC_BF16X3) {
        if ((r = ensure_mm_scratch(ctx, n, N, s))) return r;
        hipError_t e = launch_dd_prep(g, y, n, ctx->sc.mm_rows, s);
        if (e == hipSuccess)
            e = launch_dd_loglik(g, ctx->sc.mm_rows, n, theta, N, ctx->sc.mm_cols, ctx->sc.mm_part,
                                 choose_dd_slices(ctx, g, n, N), loglik, ctx->sc.status, s);
        if (e != hipSuccess) return hip_fail(e, "MFMA loglik launch");
        return SMC_OK;
    }
    const hipError_t e = launch_loglik(g, y, n, theta, N, prec, loglik,
                                       choose_slices(ctx, g, prec, n, N), ctx->sc.status, s);
    if (e != hipSuccess) return hip_fail(e, "loglik launch");
    return SMC_OK;
}

int smc_prior_init(smc_ctx ctx, const smc_gmm* model, int64_t N, uint64_t seed,
                   double* theta, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    GmmDev g;
    if ((r = check_model(model, &g))) return r;
    if (N < 1 || N > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "N must be in 1..2^31-1");
    if (!theta) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    const hipError_t e = launch_prior(g, N, seed, theta, as_stream(stream));
    if (e == hipErrorInvalidValue) return fail(SMC_ERR_UNSUPPORTED, "k*d not compiled for prior");
    if (e != hipSuccess) return hip_fail(e, "prior launch");
    return SMC_OK;
}

int smc_rwmh_move(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n,
                  double* theta, double* loglik, int64_t N, const double* beta_vec,
                  double beta, double step_sd, uint64_t seed, uint64_t step, uint32_t move,
                  smc_prec prec, unsigned long long* n_accept, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    GmmDev g;
    if ((r = check_model(model, &g))) return r;
    if ((r = check_prec(g, prec))) return r;
    if ((r = check_sizes(n, N))) return r;
    if (!y || !theta || !loglik) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (!(step_sd >= 0.0) || !isfinite(step_sd))
        return fail(SMC_ERR_INVALID_ARG, "step_sd must be finite and >= 0");
    if (!beta_vec && (!(beta >= 0.0) || !isfinite(beta)))
        return fail(SMC_ERR_INVALID_ARG, "beta must be finite and >= 0");
    if (step > 0xFFFFFFFFull) return fail(SMC_ERR_INVALID_ARG, "step must fit in 32 bits");
    if (move > 0xFFFFFFu) return fail(SMC_ERR_INVALID_ARG, "move must fit in 24 bits");
    if (prec == SMC_PREC_BF16X3) {
        const hipStream_t s = as_stream(stream);
        if ((r = ensure_mm_scratch(ctx, n, N, s))) return r;
        hipError_t e = launch_dd_prep(g, y, n, ctx->sc.mm_rows, s);
        if (e == hipSuccess)
            e = launch_dd_rwmh(g, ctx->sc.mm_rows, n, theta, loglik, N, beta_vec,
                               host_src(static_cast<int>(step), beta, 0.0), step_sd, seed, move,
                               n_accept, ctx->sc.mm_cols, ctx->sc.mm_prop, ctx->sc.mm_part,
                               choose_dd_slices(ctx, g, n, N), ctx->sc.status, MoveStep{}, s);
        if (e != hipSuccess) return hip_fail(e, "MFMA rwmh launch");
        return SMC_OK;
    }
    const hipError_t e = launch_rwmh(g, y, n, theta, loglik, N, beta_vec,
                                     host_src(static_cast<int>(step), beta, 0.0), step_sd, seed,
                                     move, prec, n_accept, choose_split(ctx, g, prec, n, N, true),
                                     ctx->sc, MoveStep{}, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "rwmh launch");
    return SMC_OK;
}

int smc_reweight(smc_ctx ctx, double* logw, const double* loglik, int64_t N, double dbeta,
                 double* W, double* logZ, double* ess, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (N < 1 || N > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "N must be in 1..2^31-1");
    if (!logw || !loglik) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (!isfinite(dbeta)) return fail(SMC_ERR_INVALID_ARG, "dbeta must be finite");
    const hipStream_t s = as_stream(stream);
    hipError_t e = launch_reweight(ctx->sc, logw, loglik, N, host_src(0, 0.0, dbeta), nullptr,
                                   logZ, ess, 0.0, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "reweight launch");
    if (W) {
        e = launch_weights(ctx->sc, logw, N, W, s);
        if (e != hipSuccess) return hip_fail(e, "weights launch");
    }
    return SMC_OK;
}

int smc_ess(smc_ctx ctx, const double* W, int64_t N, double* ess, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (N < 1 || N > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "N must be in 1..2^31-1");
    if (!W || !ess) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    const hipError_t e = launch_ess(ctx->sc, W, N, ess, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "ess launch");
    return SMC_OK;
}

int smc_resample_systematic(smc_ctx ctx, const double* W, int64_t N, uint64_t seed,
                            uint64_t step, const double* u_override, const double* ess,
                            double ess_threshold, int32_t* idx, const double* theta_in,
                            double* theta_out, int32_t kd, const double* l_in, double* l_out,
                            double* logw, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (N < 1 || N > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "N must be in 1..2^31-1");
    if (!W) return fail(SMC_ERR_INVALID_ARG, "W is NULL");
    if ((theta_in == nullptr) != (theta_out == nullptr))
        return fail(SMC_ERR_INVALID_ARG, "theta_in and theta_out go together");
    if (theta_in && (kd < 1 || kd > SMC_KDMAX)) return fail(SMC_ERR_INVALID_ARG, "kd in 1..64");
    if (theta_in && theta_in == theta_out) return fail(SMC_ERR_INVALID_ARG, "theta_out aliases theta_in");
    if ((l_in == nullptr) != (l_out == nullptr))
        return fail(SMC_ERR_INVALID_ARG, "l_in and l_out go together");
    if (l_in && l_in == l_out) return fail(SMC_ERR_INVALID_ARG, "l_out aliases l_in");
    if (step > 0xFFFFFFFFull) return fail(SMC_ERR_INVALID_ARG, "step must fit in 32 bits");
    if ((r = ensure_scratch(ctx, N, 1, as_stream(stream)))) return r;
    WeightSrc ws{W, nullptr, nullptr};
    const hipError_t e = launch_resample(ctx->sc, ws, N, SMC_RESAMPLE_SYSTEMATIC, seed,
                                         host_src(static_cast<int>(step), 0, 0), u_override, ess,
                                         ess_threshold, nullptr, idx, theta_in, theta_out,
                                         theta_in ? kd : 0, l_in, l_out, logw, 1,
                                         as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "resample launch");
    return SMC_OK;
}

int smc_resample(smc_ctx ctx, smc_resampling scheme, const double* W, int64_t N, uint64_t seed,
                 uint64_t step, const double* ess, double ess_threshold, int32_t* idx,
                 const double* theta_in, double* theta_out, int32_t kd, const double* l_in,
                 double* l_out, double* logw, void* stream) {
    if (scheme != SMC_RESAMPLE_SYSTEMATIC && scheme != SMC_RESAMPLE_STRATIFIED &&
        scheme != SMC_RESAMPLE_MULTINOMIAL)
        return fail(SMC_ERR_INVALID_ARG, "unknown resampling scheme");
    int r = enter(ctx);
    if (r) return r;
    if (N < 1 || N > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "N must be in 1..2^31-1");
    if (!W) return fail(SMC_ERR_INVALID_ARG, "W is NULL");
    if ((theta_in == nullptr) != (theta_out == nullptr))
        return fail(SMC_ERR_INVALID_ARG, "theta_in and theta_out go together");
    if (theta_in && (kd < 1 || kd > SMC_KDMAX)) return fail(SMC_ERR_INVALID_ARG, "kd in 1..64");
    if (theta_in && theta_in == theta_out) return fail(SMC_ERR_INVALID_ARG, "theta_out aliases theta_in");
    if ((l_in == nullptr) != (l_out == nullptr))
        return fail(SMC_ERR_INVALID_ARG, "l_in and l_out go together");
    if (l_in && l_in == l_out) return fail(SMC_ERR_INVALID_ARG, "l_out aliases l_in");
    if (step > 0xFFFFFFFFull) return fail(SMC_ERR_INVALID_ARG, "step must fit in 32 bits");
    if ((r = ensure_scratch(ctx, N, 1, as_stream(stream)))) return r;
    WeightSrc ws{W, nullptr, nullptr};
    const hipError_t e = launch_resample(ctx->sc, ws, N, scheme, seed,
                                         host_src(static_cast<int>(step), 0, 0), nullptr, ess,
                                         ess_threshold, nullptr, idx, theta_in, theta_out,
                                         theta_in ? kd : 0, l_in, l_out, logw, 1,
                                         as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "resample launch");
    return SMC_OK;
}

int smc_set_resampling(smc_ctx ctx, smc_resampling scheme) {
    if (!ctx) return fail(SMC_ERR_INVALID_ARG, "context is NULL");
    if (scheme != SMC_RESAMPLE_SYSTEMATIC && scheme != SMC_RESAMPLE_STRATIFIED &&
        scheme != SMC_RESAMPLE_MULTINOMIAL)
        return fail(SMC_ERR_INVALID_ARG, "unknown resampling scheme");
    ctx->scheme = scheme;
    return SMC_OK;
}

int pt_exchange(smc_ctx ctx, double* theta, double* loglik, const double* beta, int64_t M,
                int32_t kd, int32_t parity, int32_t wrap, uint64_t seed, uint64_t iter,
                unsigned int* n_swap, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (M < 2 || M > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "M must be in 2..2^31-1");
    if (!theta || !loglik || !beta) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (kd < 1 || kd > SMC_KDMAX) return fail(SMC_ERR_INVALID_ARG, "kd in 1..64");
    if (parity != 0 && parity != 1) return fail(SMC_ERR_INVALID_ARG, "parity is 0 or 1");
    if (iter > 0xFFFFFFFFull) return fail(SMC_ERR_INVALID_ARG, "iter must fit in 32 bits");
    const hipError_t e = launch_exchange(theta, loglik, beta, M, kd, 2, parity, wrap ? 1 : 0,
                                         seed, host_src(static_cast<int>(iter), 0, 0), nullptr,
                                         n_swap, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "exchange launch");
    return SMC_OK;
}

int smc_step(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n, int64_t N,
             const double* theta_in, const double* loglik_in, double* theta_out,
             double* loglik_out, double* logw, double* W, const double* beta, int32_t T,
             int32_t* t_dev, double step_sd, int32_t n_moves, uint64_t seed, double ess_frac,
             smc_prec prec, double* stats, unsigned long long* n_accept, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    GmmDev g;
    if ((r = check_model(model, &g))) return r;
    if ((r = check_prec(g, prec))) return r;
    if ((r = check_sizes(n, N))) return r;
    if (!y || !theta_in || !loglik_in || !theta_out || !loglik_out || !logw || !W || !beta ||
        !t_dev || !stats)
        return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (theta_in == theta_out || loglik_in == loglik_out)
        return fail(SMC_ERR_INVALID_ARG, "the step reads one population and writes another");
    if (n_moves < 0) return fail(SMC_ERR_INVALID_ARG, "n_moves must be >= 0");
    if (T < 1) return fail(SMC_ERR_INVALID_ARG, "T must be >= 1");
    if (!(step_sd >= 0.0) || !isfinite(step_sd))
        return fail(SMC_ERR_INVALID_ARG, "step_sd must be finite and >= 0");
    if (!(ess_frac >= 0.0) || ess_frac > 1.0) return fail(SMC_ERR_INVALID_ARG, "ess_frac in [0,1]");
    const hipStream_t s = as_stream(stream);
    const int kd = g.k * g.d;
    const bool mfma = (prec == SMC_PREC_BF16X3);
    if ((r = ensure_scratch(ctx, N, kd, s))) return r;
    if (mfma && (r = ensure_mm_scratch(ctx, n, N, s))) return r;
    // the reweight pass reads t from the caller's counter; step_mid records t in
    // the step state and advances the counter; later kernels read t from the state
    StepSrc src{};
    src.t_dev = t_dev;
    src.beta_dev = beta;
    src.t_max = T;
    StepSrc later = src;
    later.t_dev = &ctx->sc.state->t;
    hipError_t e = launch_reweight_partial(ctx->sc, logw, loglik_in, N, src, s);
    if (e != hipSuccess) return hip_fail(e, "reweight launch");
    e = launch_step_mid(ctx->sc, N, src, t_dev, stats, ess_frac, logw, s);
    if (e != hipSuccess) return hip_fail(e, "step launch");
    if (n_moves == 0) {
        // adopt the resampled (or unchanged) population and publish W
        e = launch_search_gather(ctx->sc, N, ctx->scheme, seed, later, ctx->sc.state, theta_in,
                                 theta_out, kd, loglik_in, loglik_out, logw, 1, s);
        if (e == hipSuccess) e = launch_publish_w(ctx->sc, W, logw, N, s);
        if (e != hipSuccess) return hip_fail(e, "gather launch");
        return SMC_OK;
    }
    int chunk, nchunks;
    cdf_layout(N, &chunk, &nchunks);
    if (mfma) {
        e = launch_search_gather(ctx->sc, N, ctx->scheme, seed, later, ctx->sc.state, theta_in,
                                 ctx->sc.theta_tmp, kd, loglik_in, ctx->sc.l_tmp, logw, 0, s);
        if (e == hipSuccess) e = launch_dd_prep(g, y, n, ctx->sc.mm_rows, s);
        if (e != hipSuccess) return hip_fail(e, "gather launch");
    }
    const Split sp = choose_split(ctx, g, prec, n, N, true);
    MoveStep first{};
    first.theta_src = theta_in;
    first.l_src = loglik_in;
    first.state = ctx->sc.state;
    first.W_out = W;
    first.logw = logw;
    if (mfma) {
        first.theta_alt = ctx->sc.theta_tmp;
        first.l_alt = ctx->sc.l_tmp;
    } else {
        first.reset_logw = 1;
        first.cdf_hi = ctx->sc.cdf_hi;
        first.cdf_lo = ctx->sc.cdf_lo;
        first.chunk_tot = ctx->sc.dd_part;
        first.chunk = chunk;
        first.nchunks = nchunks;
        first.seed = seed;
        first.scheme = ctx->scheme;
    }
    if (!mfma) {
        e = launch_rwmh_moves(g, y, n, theta_out, loglik_out, N, later, step_sd, seed, n_moves,
                              prec, n_accept, sp, ctx->sc, first, s);
        if (e != hipSuccess) return hip_fail(e, "rwmh launch");
        return SMC_OK;
    }
    for (int m = 0; m < n_moves; ++m) {
        e = launch_dd_rwmh(g, ctx->sc.mm_rows, n, theta_out, loglik_out, N, nullptr, later, step_sd,
                           seed, static_cast<uint32_t>(m), n_accept, ctx->sc.mm_cols,
                           ctx->sc.mm_prop, ctx->sc.mm_part, choose_dd_slices(ctx, g, n, N),
                           ctx->sc.status, m == 0 ? first : MoveStep{}, s);
        if (e != hipSuccess) return hip_fail(e, "rwmh launch");
    }
    return SMC_OK;
}

int smc_steps(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n, int64_t N,
              double* theta_a, double* loglik_a, double* theta_b, double* loglik_b,
              double* logw, double* W, const double* beta, int32_t T, int32_t* t_dev,
              int32_t n_steps, double step_sd, int32_t n_moves, uint64_t seed, double ess_frac,
              smc_prec prec, double* stats, unsigned long long* n_accept, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (n_steps < 1) return fail(SMC_ERR_INVALID_ARG, "n_steps must be >= 1");
    if (!theta_a || !loglik_a || !theta_b || !loglik_b) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    GmmDev g;
    if ((r = check_model(model, &g))) return r;
    if ((r = check_prec(g, prec))) return r;
    if ((r = check_sizes(n, N))) return r;
    const int64_t tiles = (N + kWave - 1) / kWave;
    constexpr int64_t kFusedTiles = static_cast<int64_t>(sizeof(double)) * kMaxGroups * kSplitCap /
                                    static_cast<int64_t>(sizeof(RwPartial));
    const Split sp = choose_split(ctx, g, prec, n, N, true);
    const bool fuse = prec != SMC_PREC_BF16X3 && rwmh_moves_chainable(g, n_moves, sp) &&
                      n_steps >= 2 && tiles <= kFusedTiles;
    if (!fuse) {
        for (int32_t i = 0; i < n_steps; ++i) {
            const bool odd = (i & 1) != 0;
            r = smc_step(ctx, model, y, n, N, odd ? theta_b : theta_a, odd ? loglik_b : loglik_a,
                         odd ? theta_a : theta_b, odd ? loglik_a : loglik_b, logw, W, beta, T,
                         t_dev, step_sd, n_moves, seed, ess_frac, prec, stats, n_accept, stream);
            if (r) return r;
        }
        return SMC_OK;
    }
    // the argument checks of smc_step
    if (!y || !logw || !W || !beta || !t_dev || !stats) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (theta_a == theta_b || loglik_a == loglik_b)
        return fail(SMC_ERR_INVALID_ARG, "the steps alternate between two populations");
    if (T < 1) return fail(SMC_ERR_INVALID_ARG, "T must be >= 1");
    if (!(step_sd >= 0.0) || !isfinite(step_sd))
        return fail(SMC_ERR_INVALID_ARG, "step_sd must be finite and >= 0");
    if (!(ess_frac >= 0.0) || ess_frac > 1.0) return fail(SMC_ERR_INVALID_ARG, "ess_frac in [0,1]");
    const hipStream_t s = as_stream(stream);
    if ((r = ensure_scratch(ctx, N, g.k * g.d, s))) return r;
    StepSrc src{};
    src.t_dev = t_dev;
    src.beta_dev = beta;
    src.t_max = T;
    StepSrc later = src;
    later.t_dev = &ctx->sc.state->t;
    int chunk, nchunks;
    cdf_layout(N, &chunk, &nchunks);
    double* lw_next = ctx->sc.l_tmp;
    RwPartial* next_part = reinterpret_cast<RwPartial*>(ctx->sc.mv_part);
    for (int32_t i = 0; i < n_steps; ++i) {
        const bool odd = (i & 1) != 0;
        hipError_t e;
        if (i == 0) {
            e = launch_reweight_partial(ctx->sc, logw, loglik_a, N, src, s);
            if (e == hipSuccess) e = launch_step_mid(ctx->sc, N, src, t_dev, stats, ess_frac, logw, s);
        } else {
            // the previous move made this step's reweight and its partials
            e = launch_step_mid(ctx->sc, N, src, t_dev, stats, ess_frac, lw_next, s, nullptr, 0,
                                0, nullptr, next_part, static_cast<int>(tiles));
        }
        if (e != hipSuccess) return hip_fail(e, "step launch");
        // W and the caller's logw are read by no later kernel of the chain and
        // rewritten by every step's move: only the last step publishes them
        const bool last = i + 1 == n_steps;
        MoveStep ms{};
        ms.theta_src = odd ? theta_b : theta_a;
        ms.l_src = odd ? loglik_b : loglik_a;
        ms.state = ctx->sc.state;
        ms.W_out = last ? W : nullptr;
        ms.logw = i == 0 ? logw : lw_next;
        ms.logw_out = last ? logw : nullptr;
        ms.cdf_hi = ctx->sc.cdf_hi;
        ms.cdf_lo = ctx->sc.cdf_lo;
        ms.chunk_tot = ctx->sc.dd_part;
        ms.chunk = chunk;
        ms.nchunks = nchunks;
        ms.seed = seed;
        ms.scheme = ctx->scheme;
        if (!last) {
            ms.lw_next = lw_next;
            ms.next_part = next_part;
            ms.beta_dev = beta;
            ms.t_max = T;
        }
        e = launch_rwmh_moves(g, y, n, odd ? theta_a : theta_b, odd ? loglik_a : loglik_b, N, later,
                              step_sd, seed, n_moves, prec, n_accept, sp, ctx->sc, ms, s);
        if (e != hipSuccess) return hip_fail(e, "rwmh launch");
    }
    return SMC_OK;
}

int pt_iteration(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n, int64_t M,
                 double* theta, double* loglik, const double* beta, int32_t* it_dev,
                 double step_sd, uint64_t seed, int32_t parity_mode, int32_t wrap, smc_prec prec,
                 unsigned long long* n_accept, unsigned int* n_swap, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    GmmDev g;
    if ((r = check_model(model, &g))) return r;
    if ((r = check_prec(g, prec))) return r;
    if ((r = check_sizes(n, M))) return r;
    if (M < 2) return fail(SMC_ERR_INVALID_ARG, "M must be >= 2");
    if (!y || !theta || !loglik || !beta || !it_dev) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (parity_mode != 0 && parity_mode != 1) return fail(SMC_ERR_INVALID_ARG, "parity_mode 0 or 1");
    if (!(step_sd >= 0.0) || !isfinite(step_sd))
        return fail(SMC_ERR_INVALID_ARG, "step_sd must be finite and >= 0");
    const hipStream_t s = as_stream(stream);
    // the move reads the iteration from the caller's counter and records it in
    // the step state; the exchange reads that record and advances the counter
    StepSrc src{};
    src.t_dev = it_dev;
    StepSrc later{};
    later.t_dev = &ctx->sc.state->t;
    MoveStep ms{};
    ms.t_out = &ctx->sc.state->t;
    hipError_t e;
    if (prec == SMC_PREC_BF16X3) {
        if ((r = ensure_mm_scratch(ctx, n, M, s))) return r;
        e = launch_dd_prep(g, y, n, ctx->sc.mm_rows, s);
        if (e == hipSuccess)
            e = launch_dd_rwmh(g, ctx->sc.mm_rows, n, theta, loglik, M, beta, src, step_sd, seed, 0,
                               n_accept, ctx->sc.mm_cols, ctx->sc.mm_prop, ctx->sc.mm_part,
                               choose_dd_slices(ctx, g, n, M), ctx->sc.status, ms, s);
        if (e != hipSuccess) return hip_fail(e, "rwmh launch");
        e = launch_exchange(theta, loglik, beta, M, g.k * g.d, parity_mode, 0, wrap ? 1 : 0,
                            seed, later, it_dev, n_swap, s);
        if (e != hipSuccess) return hip_fail(e, "exchange launch");
        return SMC_OK;
    }
    e = launch_pt_iteration(g, y, n, theta, loglik, M, beta, src, later, step_sd, seed, prec,
                            n_accept, choose_split(ctx, g, prec, n, M, true), ctx->sc, ms,
                            parity_mode, wrap ? 1 : 0, it_dev, n_swap, s);
    if (e != hipSuccess) return hip_fail(e, "population MCMC launch");
    return SMC_OK;
}

int pt_iterations(smc_ctx ctx, const smc_gmm* model, const float* y, int64_t n, int64_t M,
                  double* theta, double* loglik, const double* beta, int32_t* it_dev,
                  int32_t n_iters, double step_sd, uint64_t seed, int32_t parity_mode,
                  int32_t wrap, smc_prec prec, unsigned long long* n_accept,
                  unsigned int* n_swap, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (n_iters < 1) return fail(SMC_ERR_INVALID_ARG, "n_iters must be >= 1");
    GmmDev g;
    if ((r = check_model(model, &g))) return r;
    if ((r = check_prec(g, prec))) return r;
    if ((r = check_sizes(n, M))) return r;
    const int kd = g.k * g.d;
    const bool local = prec != SMC_PREC_BF16X3 && M >= 2 && M <= pt_local_chains(kd) &&
                       (ctx->pt_single > 0 || (ctx->pt_single == 0 && pt_local_pays(kd, n, M)));
    if (!local && prec != SMC_PREC_BF16X3 && ctx->pt_single >= 0) {
        const Split sp = choose_split(ctx, g, prec, n, M, true);
        if (sp.groups == 1) {
            // one launch per iteration, each taking the previous iteration's exchange
            if (!y || !theta || !loglik || !beta || !it_dev)
                return fail(SMC_ERR_INVALID_ARG, "NULL array");
            if (parity_mode != 0 && parity_mode != 1)
                return fail(SMC_ERR_INVALID_ARG, "parity_mode 0 or 1");
            if (!(step_sd >= 0.0) || !isfinite(step_sd))
                return fail(SMC_ERR_INVALID_ARG, "step_sd must be finite and >= 0");
            const hipStream_t s = as_stream(stream);
            if ((r = ensure_scratch(ctx, M, kd, s))) return r;
            const hipError_t e = launch_pt_deferred(g, y, n, theta, loglik, M, beta, it_dev,
                                                    n_iters, step_sd, seed, prec, parity_mode,
                                                    wrap ? 1 : 0, sp.slices, n_accept, n_swap,
                                                    ctx->sc, &ctx->sc.state->t, s);
            if (e != hipSuccess) return hip_fail(e, "population MCMC launch");
            return SMC_OK;
        }
    }
    if (!local) {
        for (int32_t i = 0; i < n_iters; ++i) {
            r = pt_iteration(ctx, model, y, n, M, theta, loglik, beta, it_dev, step_sd, seed,
                             parity_mode, wrap, prec, n_accept, n_swap, stream);
            if (r) return r;
        }
        return SMC_OK;
    }
    if (!y || !theta || !loglik || !beta || !it_dev) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (parity_mode != 0 && parity_mode != 1) return fail(SMC_ERR_INVALID_ARG, "parity_mode 0 or 1");
    if (!(step_sd >= 0.0) || !isfinite(step_sd))
        return fail(SMC_ERR_INVALID_ARG, "step_sd must be finite and >= 0");
    const hipError_t e = launch_pt_local(g, y, n, theta, loglik, M, beta, it_dev, n_iters,
                                         step_sd, seed, prec, parity_mode, wrap ? 1 : 0,
                                         ctx->slices_override > 0 ? ctx->slices_override
                                                                  : pt_local_slices(n, M),
                                         n_accept, n_swap,
                                         ctx->sc.status, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "population MCMC launch");
    return SMC_OK;
}

int pt_record(smc_ctx ctx, const double* theta, int64_t M, int32_t kd, int64_t chain,
              const int32_t* it_dev, double* out, int64_t max_iters, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (!theta || !it_dev || !out) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (M < 1 || M > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "M must be in 1..2^31-1");
    if (kd < 1 || kd > SMC_KDMAX) return fail(SMC_ERR_INVALID_ARG, "kd in 1..64");
    if (chain < 0 || chain >= M) return fail(SMC_ERR_INVALID_ARG, "chain must be in 0..M-1");
    if (max_iters < 1) return fail(SMC_ERR_INVALID_ARG, "max_iters must be >= 1");
    const hipError_t e = launch_pt_record(theta, M, kd, chain, it_dev, out, max_iters,
                                          as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "record launch");
    return SMC_OK;
}

int fsv_init(smc_ctx ctx, int32_t k, int64_t N, double* x, double* logw, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (k < 1 || k > SMC_FSV_KMAX) return fail(SMC_ERR_INVALID_ARG, "k in 1..4");
    if (N < 1 || N > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "N must be in 1..2^31-1");
    if (!x || !logw) return fail(SMC_ERR_INVALID_ARG, "NULL array");
    const hipError_t e = launch_fsv_init(k, N, x, logw, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "init launch");
    return SMC_OK;
}

namespace {

// Lower Cholesky factor of the k x k matrix U (row-major); false if U is not
// positive definite.
bool host_cholesky(const double* U, int k, double* L) {
    for (int i = 0; i < SMC_FSV_KMAX * SMC_FSV_KMAX; ++i) L[i] = 0.0;
    for (int i = 0; i < k; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = U[i * SMC_FSV_KMAX + j];
            for (int q = 0; q < j; ++q) s -= L[i * SMC_FSV_KMAX + q] * L[j * SMC_FSV_KMAX + q];
            if (i == j) {
                if (!(s > 0.0)) return false;
                L[i * SMC_FSV_KMAX + i] = sqrt(s);
            } else {
                L[i * SMC_FSV_KMAX + j] = s / L[j * SMC_FSV_KMAX + j];
            }
        }
    }
    return true;
}

}  // namespace

namespace {

// Argument checks of the filter calls and the device model they build.
int fsv_prepare(const smc_fsv* model, const double* y, int32_t T, int64_t N, const double* x,
                const double* x_tmp, const double* logw, const int32_t* t_dev,
                const double* stats, const double* moments, double ess_frac, FsvDev* out) {
    if (!model) return fail(SMC_ERR_INVALID_ARG, "model is NULL");
    if (!fsv_supported(model->m, model->k))
        return fail(SMC_ERR_UNSUPPORTED, "(m, k) of the factor model is not compiled");
    if (T < 1) return fail(SMC_ERR_INVALID_ARG, "T must be >= 1");
    if (N < 1 || N > INT32_MAX) return fail(SMC_ERR_INVALID_ARG, "N must be in 1..2^31-1");
    if (!y || !x || !x_tmp || !logw || !t_dev || !stats || !moments)
        return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (x == x_tmp) return fail(SMC_ERR_INVALID_ARG, "x_tmp must not alias x");
    if (!(ess_frac >= 0.0) || ess_frac > 1.0) return fail(SMC_ERR_INVALID_ARG, "ess_frac in [0,1]");
    FsvDev f{};
    f.m = model->m;
    f.k = model->k;
    for (int i = 0; i < f.m; ++i) {
        if (!(model->psi[i] > 0.0) || !isfinite(model->psi[i]))
            return fail(SMC_ERR_INVALID_ARG, "psi must be finite and > 0");
        f.psi[i] = model->psi[i];
        for (int c = 0; c < f.k; ++c) {
            if (!isfinite(model->B[i * SMC_FSV_KMAX + c]))
                return fail(SMC_ERR_INVALID_ARG, "B must be finite");
            f.B[i * SMC_FSV_KMAX + c] = model->B[i * SMC_FSV_KMAX + c];
        }
    }
    for (int c = 0; c < f.k; ++c) {
        if (!isfinite(model->phi[c])) return fail(SMC_ERR_INVALID_ARG, "phi must be finite");
        f.phi[c] = model->phi[c];
    }
    if (!host_cholesky(model->U, f.k, f.L))
        return fail(SMC_ERR_INVALID_ARG, "U is not symmetric positive definite");
    f.cst = -0.5 * f.m * log(2.0 * M_PI);
    *out = f;
    return SMC_OK;
}

// Propagate + weight (from x_in, optionally taking the previous step's
// resampling) into x_out, then the step's combine and decision.
hipError_t fsv_weight_mid(smc_ctx ctx, const FsvDev& f, const double* y, int32_t T, int64_t N,
                          const double* x_in, double* x_out, double* logw, int32_t* t_dev,
                          uint64_t seed, double ess_frac, double* stats, double* moments,
                          const FsvAnc& anc, hipStream_t s) {
    StepSrc src{};
    src.t_dev = t_dev;
    src.t_max = T;
    hipError_t e = launch_fsv_weight(f, y, T, x_in, x_out, logw, N, src, seed, ctx->sc,
                                     ctx->fsv_mom, s, anc);
    if (e == hipSuccess)
        e = launch_step_mid(ctx->sc, N, src, t_dev, stats, ess_frac, logw, s, ctx->fsv_mom, f.k,
                            2 * SMC_FSV_KMAX, moments);
    return e;
}

// The step's resampling (or copy) of x_tmp into x, logw reset after resampling.
hipError_t fsv_gather(smc_ctx ctx, int k, int64_t N, const double* x_tmp, double* x, double* logw,
                      uint64_t seed, hipStream_t s) {
    StepSrc later{};
    later.t_dev = &ctx->sc.state->t;
    return launch_search_gather(ctx->sc, N, ctx->scheme, seed, later, ctx->sc.state, x_tmp, x, k,
                                nullptr, nullptr, logw, 1, s);
}

}  // namespace

int fsv_step(smc_ctx ctx, const smc_fsv* model, const double* y, int32_t T, int64_t N,
             double* x, double* x_tmp, double* logw, int32_t* t_dev, uint64_t seed,
             double ess_frac, double* stats, double* moments, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    FsvDev f;
    if ((r = fsv_prepare(model, y, T, N, x, x_tmp, logw, t_dev, stats, moments, ess_frac, &f)))
        return r;
    const hipStream_t s = as_stream(stream);
    if ((r = ensure_scratch(ctx, N, f.k, s))) return r;
    hipError_t e = fsv_weight_mid(ctx, f, y, T, N, x, x_tmp, logw, t_dev, seed, ess_frac, stats,
                                  moments, FsvAnc{}, s);
    if (e == hipSuccess) e = fsv_gather(ctx, f.k, N, x_tmp, x, logw, seed, s);
    if (e != hipSuccess) return hip_fail(e, "particle filter launch");
    return SMC_OK;
}

int fsv_steps(smc_ctx ctx, const smc_fsv* model, const double* y, int32_t T, int64_t N,
              double* x, double* x_tmp, double* logw, int32_t* t_dev, int32_t n_steps,
              uint64_t seed, double ess_frac, double* stats, double* moments, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (n_steps < 1) return fail(SMC_ERR_INVALID_ARG, "n_steps must be >= 1");
    FsvDev f;
    if ((r = fsv_prepare(model, y, T, N, x, x_tmp, logw, t_dev, stats, moments, ess_frac, &f)))
        return r;
    const hipStream_t s = as_stream(stream);
    if ((r = ensure_scratch(ctx, N, f.k, s))) return r;
    int chunk, nchunks;
    cdf_layout(N, &chunk, &nchunks);
    FsvAnc prev{};
    prev.state = ctx->sc.state;
    prev.cdf_hi = ctx->sc.cdf_hi;
    prev.cdf_lo = ctx->sc.cdf_lo;
    prev.chunk_tot = ctx->sc.dd_part;
    prev.chunk = chunk;
    prev.nchunks = nchunks;
    prev.scheme = ctx->scheme;
    hipError_t e = hipSuccess;
    // the chain below has an odd length, so that its last step writes x_tmp; an
    // even count takes its first step on its own
    int32_t m = n_steps;
    if ((n_steps & 1) == 0) {
        e = fsv_weight_mid(ctx, f, y, T, N, x, x_tmp, logw, t_dev, seed, ess_frac, stats, moments,
                           FsvAnc{}, s);
        if (e == hipSuccess) e = fsv_gather(ctx, f.k, N, x_tmp, x, logw, seed, s);
        m = n_steps - 1;
    }
    // step j propagates from the previous step's states (x for j = 0, where the
    // resampling was already applied; otherwise the other buffer, taking that
    // step's resampling itself) into x_tmp for even j and x for odd j
    for (int32_t j = 0; j < m && e == hipSuccess; ++j) {
        const bool odd = (j & 1) != 0;
        e = fsv_weight_mid(ctx, f, y, T, N, odd ? x_tmp : x, odd ? x : x_tmp, logw, t_dev, seed,
                           ess_frac, stats, moments, j == 0 ? FsvAnc{} : prev, s);
    }
    if (e == hipSuccess) e = fsv_gather(ctx, f.k, N, x_tmp, x, logw, seed, s);
    if (e != hipSuccess) return hip_fail(e, "particle filter launch");
    return SMC_OK;
}

int smc_graph_begin(smc_ctx ctx, void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (!stream) return fail(SMC_ERR_INVALID_ARG, "the null stream cannot be captured");
    SMC_CHECK_HIP(hipStreamBeginCapture(as_stream(stream), hipStreamCaptureModeThreadLocal),
                  "hipStreamBeginCapture");
    return SMC_OK;
}

int smc_graph_end(smc_ctx ctx, void* stream, smc_graph* out) {
    int r = enter(ctx);
    if (r) return r;
    if (!out) return fail(SMC_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    hipGraph_t graph = nullptr;
    SMC_CHECK_HIP(hipStreamEndCapture(as_stream(stream), &graph), "hipStreamEndCapture");
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(e, "hipGraphInstantiate");
    }
    smc_graph g = new (std::nothrow) smc_graph_s();
    if (!g) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return fail(SMC_ERR_NOMEM, "host allocation failed");
    }
    g->graph = graph;
    g->exec = exec;
    *out = g;
    return SMC_OK;
}

int smc_graph_launch(smc_graph g, void* stream) {
    if (!g) return fail(SMC_ERR_INVALID_ARG, "graph is NULL");
    SMC_CHECK_HIP(hipGraphLaunch(g->exec, as_stream(stream)), "hipGraphLaunch");
    return SMC_OK;
}

int smc_graph_destroy(smc_graph g) {
    if (!g) return SMC_OK;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return SMC_OK;
}

int smc_fp32_form_counts(smc_ctx ctx, uint64_t* out, int32_t reset) {
    int r = enter(ctx);
    if (r) return r;
    if (!out) return fail(SMC_ERR_INVALID_ARG, "out is NULL");
    unsigned long long v[3] = {0, 0, 0};
    SMC_CHECK_HIP(fp32_form_counts(v, reset != 0), "reading the form counters");
    for (int c = 0; c < 3; ++c) out[c] = static_cast<uint64_t>(v[c]);
    return SMC_OK;
}

int smc_sort_data(float* y, int64_t n, void* stream) {
    if (n < 0 || n > (int64_t{1} << 30) || (n > 0 && !y))
        return fail(SMC_ERR_INVALID_ARG, "n must be in [0, 2^30] and y set when n > 0");
    const hipError_t e = launch_sort_data(y, n, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "sort launch");
    return SMC_OK;
}

int smc_rng_words(uint64_t seed, int64_t count, uint32_t block, uint32_t step, uint32_t purpose,
                  uint32_t move, uint32_t* out, void* stream) {
    if (count < 1 || count > INT32_MAX || !out) return fail(SMC_ERR_INVALID_ARG, "bad count or out");
    if (purpose > 255 || move > 0xFFFFFFu) return fail(SMC_ERR_INVALID_ARG, "purpose/move range");
    const hipError_t e = launch_rng_words(seed, count, block, step, purpose, move, out,
                                          as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "rng launch");
    return SMC_OK;
}

int smc_rng_normals(uint64_t seed, int64_t count, int32_t per_index, uint32_t step,
                    uint32_t purpose, uint32_t move, double* out, void* stream) {
    if (count < 1 || count > INT32_MAX || !out || per_index < 1 || per_index > SMC_KDMAX)
        return fail(SMC_ERR_INVALID_ARG, "bad count, per_index or out");
    if (purpose > 255 || move > 0xFFFFFFu) return fail(SMC_ERR_INVALID_ARG, "purpose/move range");
    const hipError_t e = launch_rng_normals(seed, count, per_index, step, purpose, move, out,
                                            as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "rng launch");
    return SMC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- batched runs

struct smc_batch_s {
    int device = 0;
    BatchDev dev{};
    void* mem = nullptr;
    int64_t n_total = 0, N_total = 0;
    int kd = 0;
};

extern "C" {

int smc_batch_create(smc_ctx ctx, const smc_run_desc* runs, int32_t R, int32_t kd,
                     smc_batch* out) {
    int r = enter(ctx);
    if (r) return r;
    if (!out || !runs) return fail(SMC_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    if (R < 1) return fail(SMC_ERR_INVALID_ARG, "R must be >= 1");
    if (kd < 1 || kd > SMC_KMAX) return fail(SMC_ERR_INVALID_ARG, "batched runs need d = 1, k <= 8");
    int64_t N_total = 0, n_total = 0, n_tiles = 0;
    for (int i = 0; i < R; ++i) {
        const smc_run_desc& d = runs[i];
        if (d.N < 1 || d.n < 1 || d.p_off < 0 || d.y_off < 0)
            return fail(SMC_ERR_INVALID_ARG, "run needs N >= 1, n >= 1, offsets >= 0");
        if (d.p_off + d.N > N_total) N_total = d.p_off + d.N;
        if (d.y_off + d.n > n_total) n_total = d.y_off + d.n;
        n_tiles += (d.N + 63) / 64;
    }
    if (N_total > INT32_MAX || n_tiles > INT32_MAX)
        return fail(SMC_ERR_INVALID_ARG, "batch too large");
    // work lists (FP64, FP32): runs by decreasing data length (ties: larger N
    // first), each run's tiles in units of kBatchWaves / S tiles
    std::vector<int> order(R);
    for (int i = 0; i < R; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (runs[a].n != runs[b].n) return runs[a].n > runs[b].n;
        return runs[a].N > runs[b].N;
    });
    std::vector<BatchUnit> units[2];
    for (int pi = 0; pi < 2; ++pi) {
        const int prec = pi == 1 ? SMC_PREC_FP32 : SMC_PREC_FP64;
        for (int i : order) {
            const int S = batch_slices(ctx, kd, prec, runs[i].n, runs[i].N);
            const int per = kBatchWaves / S;
            const int tiles = (runs[i].N + 63) / 64;
            for (int t = 0; t < tiles; t += per)
                units[pi].push_back(BatchUnit{i, t, std::min(per, tiles - t), S});
        }
    }
    std::vector<BatchRun> rd(R);
    for (int i = 0; i < R; ++i)
        rd[i] = BatchRun{runs[i].p_off, runs[i].y_off, runs[i].N, runs[i].n, runs[i].seed};
    const size_t b_runs = align_up(sizeof(BatchRun) * R);
    const size_t b_u0 = align_up(sizeof(BatchUnit) * units[0].size());
    const size_t b_items = b_u0 + align_up(sizeof(BatchUnit) * units[1].size());
    const size_t b_work = align_up(sizeof(unsigned));
    const size_t b_state = align_up(sizeof(StepState) * R);
    const size_t b_cdf = align_up(sizeof(double) * N_total);
    const size_t b_th = align_up(sizeof(double) * N_total * kd);
    const size_t b_l = align_up(sizeof(double) * N_total);
    const size_t total = b_runs + b_items + b_work + b_state + b_cdf + b_th + b_l;
    void* p = nullptr;
    if (hipMalloc(&p, total) != hipSuccess) return fail(SMC_ERR_NOMEM, "batch allocation failed");
    smc_batch b = new (std::nothrow) smc_batch_s();
    if (!b) {
        (void)hipFree(p);
        return fail(SMC_ERR_NOMEM, "host allocation failed");
    }
    char* c = static_cast<char*>(p);
    b->device = ctx->device;
    b->mem = p;
    b->kd = kd;
    b->N_total = N_total;
    b->n_total = n_total;
    BatchDev& d = b->dev;
    d.R = R;
    d.runs = reinterpret_cast<BatchRun*>(c);
    d.units[0] = reinterpret_cast<BatchUnit*>(c + b_runs);
    d.units[1] = reinterpret_cast<BatchUnit*>(c + b_runs + b_u0);
    d.n_units[0] = static_cast<int>(units[0].size());
    d.n_units[1] = static_cast<int>(units[1].size());
    d.work = reinterpret_cast<unsigned*>(c + b_runs + b_items);
    d.state = reinterpret_cast<StepState*>(c + b_runs + b_items + b_work);
    d.cdf = reinterpret_cast<double*>(c + b_runs + b_items + b_work + b_state);
    d.theta_tmp = reinterpret_cast<double*>(c + b_runs + b_items + b_work + b_state + b_cdf);
    d.l_tmp = reinterpret_cast<double*>(c + b_runs + b_items + b_work + b_state + b_cdf + b_th);
    d.move_grid = batch_move_grid();
    hipError_t e = hipMemset(p, 0, total);
    if (e == hipSuccess) e = hipMemcpy(d.runs, rd.data(), sizeof(BatchRun) * R, hipMemcpyHostToDevice);
    for (int pi = 0; pi < 2 && e == hipSuccess; ++pi)
        e = hipMemcpy(d.units[pi], units[pi].data(), sizeof(BatchUnit) * units[pi].size(),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(p);
        delete b;
        return hip_fail(e, "batch upload");
    }
    *out = b;
    return SMC_OK;
}

int smc_batch_destroy(smc_batch b) {
    if (!b) return SMC_OK;
    (void)hipSetDevice(b->device);
    (void)hipDeviceSynchronize();
    if (b->mem) (void)hipFree(b->mem);
    delete b;
    return SMC_OK;
}

int smc_step_batched(smc_ctx ctx, smc_batch b, const smc_gmm* model, const float* y,
                     double* theta, double* loglik, double* logw, double* W, const double* beta,
                     int32_t T, int32_t* t_dev, double step_sd, int32_t n_moves, double ess_frac,
                     smc_prec prec, double* run_stats, unsigned long long* n_accept,
                     void* stream) {
    int r = enter(ctx);
    if (r) return r;
    if (!b) return fail(SMC_ERR_INVALID_ARG, "batch is NULL");
    GmmDev g;
    if ((r = check_model(model, &g))) return r;
    if (g.d != 1 || g.k * g.d != b->kd)
        return fail(SMC_ERR_INVALID_ARG, "model does not match the batch (d = 1, k*d = kd)");
    if (prec != SMC_PREC_FP32 && prec != SMC_PREC_FP64)
        return fail(SMC_ERR_UNSUPPORTED, "batched runs use FP32 or FP64");
    if (!y || !theta || !loglik || !logw || !W || !beta || !t_dev || !run_stats)
        return fail(SMC_ERR_INVALID_ARG, "NULL array");
    if (T < 1) return fail(SMC_ERR_INVALID_ARG, "T must be >= 1");
    if (n_moves < 1) return fail(SMC_ERR_INVALID_ARG, "batched steps need n_moves >= 1");
    if (!(step_sd >= 0.0) || !isfinite(step_sd))
        return fail(SMC_ERR_INVALID_ARG, "step_sd must be finite and >= 0");
    if (!(ess_frac >= 0.0) || ess_frac > 1.0) return fail(SMC_ERR_INVALID_ARG, "ess_frac in [0,1]");
    const hipError_t e = launch_batch_step(b->dev, g, y, theta, loglik, logw, W, beta, T, t_dev,
                                           step_sd, n_moves, ess_frac, prec, run_stats, n_accept,
                                           ctx->sc.status, ctx->scheme, as_stream(stream));
    if (e != hipSuccess) return hip_fail(e, "batched step launch");
    return SMC_OK;
}

}  // extern "C"
