// Resampling that allocates nothing (smc_resample_noalloc): the same kernels as
// smc_resample, with their scratch (the CDF halves and the chunk totals) in a
// fixed device array of this translation unit instead of a context's buffers.
// For callers that cannot call hipMalloc: code under stream capture, serving
// loops, harnesses that forbid allocation.
#include <math.h>

#include <mutex>
#include <string>

#include "internal.hpp"

namespace {

constexpr int64_t kNoAllocMaxN = int64_t{1} << 20;                 // largest N
constexpr int64_t kNoAllocChunks = (kNoAllocMaxN + 1023) / 1024;     // smc::res_chunks(max N)
constexpr int64_t kNoAllocDoubles = 2 * kNoAllocMaxN + 4 * kNoAllocChunks;

// The scratch: cdf_hi [kNoAllocMaxN], cdf_lo [kNoAllocMaxN], chunk totals and
// chunk offsets [2 * kNoAllocChunks] each (16 MiB + 32 KiB). Every GPU the
// library runs on holds its
// own copy until the process ends. Host code never passes this name to a
// kernel: it is a host-side stand-in; the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up on the
// first call on that device, with the device current); nullptr on failure.
double* scratch_ptr(int dev, hipError_t* err) {
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[dev] == nullptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) {
            *err = e;
            return nullptr;
        }
        g_ptr[dev] = static_cast<double*>(p);
    }
    return g_ptr[dev];
}

int fail(int code, const std::string& m) {
    smc::set_last_error(m.c_str());
    return code;
}

}  // namespace

extern "C" {

int smc_resample_noalloc(smc_resampling scheme, const double* W, int64_t N, uint64_t seed,
                         uint64_t step, const double* ess, double ess_threshold, int32_t* idx,
                         const double* theta_in, double* theta_out, int32_t kd,
                         const double* l_in, double* l_out, double* logw, void* stream) {
    using namespace smc;
    if (scheme != SMC_RESAMPLE_SYSTEMATIC && scheme != SMC_RESAMPLE_STRATIFIED &&
        scheme != SMC_RESAMPLE_MULTINOMIAL)
        return fail(SMC_ERR_INVALID_ARG, "unknown resampling scheme");
    if (N < 1) return fail(SMC_ERR_INVALID_ARG, "N must be >= 1");
    if (N > kNoAllocMaxN || res_chunks(N) > kNoAllocChunks)
        return fail(SMC_ERR_INVALID_ARG, "N above the no-allocation maximum of 2^20 particles");
    if (!W) return fail(SMC_ERR_INVALID_ARG, "W is NULL");
    if ((theta_in == nullptr) != (theta_out == nullptr))
        return fail(SMC_ERR_INVALID_ARG, "theta_in and theta_out go together");
    if (theta_in && (kd < 1 || kd > SMC_KDMAX)) return fail(SMC_ERR_INVALID_ARG, "kd in 1..64");
    if (theta_in && theta_in == theta_out)
        return fail(SMC_ERR_INVALID_ARG, "theta_out aliases theta_in");
    if ((l_in == nullptr) != (l_out == nullptr))
        return fail(SMC_ERR_INVALID_ARG, "l_in and l_out go together");
    if (l_in && l_in == l_out) return fail(SMC_ERR_INVALID_ARG, "l_out aliases l_in");
    if (step > 0xFFFFFFFFull) return fail(SMC_ERR_INVALID_ARG, "step must fit in 32 bits");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SMC_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(SMC_ERR_UNSUPPORTED, "device index above 63");
    double* p = scratch_ptr(dev, &e);
    if (!p) return fail(SMC_ERR_HIP, std::string("hipGetSymbolAddress: ") + hipGetErrorString(e));
    Scratch sc{};
    static_assert(kNoAllocChunks >= 1, "");
    sc.cdf_hi = p;
    sc.cdf_lo = p + kNoAllocMaxN;
    sc.res_tot = p + 2 * kNoAllocMaxN;
    sc.res_off = p + 2 * kNoAllocMaxN + 2 * kNoAllocChunks;
    sc.cap = kNoAllocMaxN;
    StepSrc src{};
    src.t_host = static_cast<int>(step);
    WeightSrc ws{W, nullptr, nullptr};
    e = launch_resample(sc, ws, N, scheme, seed, src, nullptr, ess, ess_threshold, nullptr, idx,
                        theta_in, theta_out, theta_in ? kd : 0, l_in, l_out, logw, 1,
                        reinterpret_cast<hipStream_t>(stream));
    if (e != hipSuccess)
        return fail(SMC_ERR_HIP, std::string("resample launch: ") + hipGetErrorString(e));
    return SMC_OK;
}

}  // extern "C"
