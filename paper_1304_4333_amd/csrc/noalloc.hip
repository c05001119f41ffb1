// noalloc.hip -- sps_loglik_noalloc: the log-likelihood of sps_loglik for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// The scratch of sps_loglik (the observation-split partial sums and the
// multinomial sufficient statistics) lives in one file-scope device array
// per GPU instead of the context's grow-only buffers.  Its device address is
// resolved once per device, with that device current, when the first
// context on it is created (sps_create); host code uses only that address.
#include <mutex>

#include "sps_internal.h"

namespace sps {

// 2^21 doubles (16 MiB) for the split partials plus 1024 for the sufficient
// statistics (d <= 7 x 128 = 896 at the largest supported shape).
constexpr int64_t kScratchPart = int64_t(1) << 21;
constexpr int64_t kScratchSuff = 1024;
static __device__ __align__(256) double scratch[kScratchPart + kScratchSuff];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

int noalloc_setup(sps_ctx* c, int device) {
    if (device < 0 || device >= kMaxDevices) return fail(c, SPS_ERR_ARG, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return SPS_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(c, e != hipSuccess ? e : hipErrorUnknown, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[device] = (double*)p;
    return SPS_OK;
}

}  // namespace sps

using namespace sps;

extern "C" int sps_loglik_noalloc(sps_ctx* c, const double* theta, int64_t P, int64_t t0, int64_t t1,
                                  int prec, double* ll) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (c->has_data && c->d > kScratchSuff)
        return fail(c, SPS_ERR_ARG, "sps_loglik_noalloc: d = %d exceeds the scratch maximum of %lld", c->d,
                    (long long)kScratchSuff);
    double* base = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch_ptr[c->device];
    }
    if (!base) return fail(c, SPS_ERR_HIP, "sps_loglik_noalloc: scratch of device %d not resolved", c->device);
    const LoglikScratch ext{base, kScratchPart, base + kScratchPart};
    return loglik_launch_scratch(c, theta, P, t0, t1, prec, ll, ext);
}
