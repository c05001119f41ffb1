// sps_ctx.hip -- context lifetime, errors, scratch, and the data/prior set-up
// of libsps: the kernel copies of X in every precision are built once here.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>

#include "sps_internal.h"

namespace sps {

int fail(sps_ctx* c, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return code;
}

int hip_fail(sps_ctx* c, hipError_t e, const char* what) {
    int code = (e == hipErrorOutOfMemory) ? SPS_ERR_NOMEM : SPS_ERR_HIP;
    return fail(c, code, "%s: %s", what, hipGetErrorString(e));
}

int ensure(sps_ctx* c, Buf& b, size_t bytes, const char* what) {
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return SPS_OK;
    if (b.p) {
        // The old buffer may still be read by queued work on the stream.
        SPS_HIP(c, hipStreamSynchronize(c->stream));
        SPS_HIP(c, hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 8;  // headroom against repeated small growth
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        b.p = nullptr;
        return hip_fail(c, e, what);
    }
    b.bytes = want;
    return SPS_OK;
}

int ensure_host(sps_ctx* c, Buf& b, size_t bytes) {
    if (b.bytes >= bytes) return SPS_OK;
    if (b.p) {
        SPS_HIP(c, hipStreamSynchronize(c->stream));
        SPS_HIP(c, hipHostFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipHostMalloc(&b.p, bytes, hipHostMallocDefault);
    if (e != hipSuccess) {
        b.p = nullptr;
        return hip_fail(c, e, "hipHostMalloc(staging)");
    }
    b.bytes = bytes;
    return SPS_OK;
}

// ------------------------------------------------------------------ read-back
// One wave copies n8 words into host memory; after a system-scope fence
// (the wave's stores are complete and visible) lane 0 writes the sequence
// number.
__global__ __launch_bounds__(64) void publish_kernel(const unsigned long long* __restrict__ src, int64_t n8,
                                                     unsigned long long* dst, unsigned long long* flag,
                                                     unsigned long long seq) {
    for (int64_t i = threadIdx.x; i < n8; i += 64) dst[i] = src[i];
    __threadfence_system();
    if (threadIdx.x == 0) __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Pinned memory: kPublishSlots slots of [sequence word, padding to 64 bytes,
// kPublishBytes of data].
constexpr size_t kPubHeader = 64;
constexpr size_t kPubSlot = kPubHeader + kPublishBytes;

int publish_async(sps_ctx* c, const void* dsrc, size_t bytes, PubTicket* t) {
    if (bytes > kPublishBytes) return fail(c, SPS_ERR_ARG, "read-back of %zu bytes above the slot size", bytes);
    if (!c->pub) {
        hipError_t e = hipHostMalloc(&c->pub, kPubSlot * kPublishSlots, hipHostMallocCoherent);
        if (e != hipSuccess) {
            c->pub = nullptr;
            return hip_fail(c, e, "hipHostMalloc(read-back)");
        }
        c->pub_bytes = kPubSlot * kPublishSlots;
        for (int i = 0; i < kPublishSlots; ++i) *(volatile unsigned long long*)((char*)c->pub + i * kPubSlot) = 0;
        c->pub_seq = 0;
    }
    const uint64_t seq = ++c->pub_seq;
    const int slot = (int)(seq % kPublishSlots);
    char* base = (char*)c->pub + slot * kPubSlot;
    publish_kernel<<<1, 64, 0, c->stream>>>((const unsigned long long*)dsrc, (int64_t)((bytes + 7) / 8),
                                            (unsigned long long*)(base + kPubHeader), (unsigned long long*)base,
                                            seq);
    SPS_CHECK(launched(c, "publish_kernel"));
    *t = PubTicket{slot, seq, dsrc, bytes};
    return SPS_OK;
}

int publish_wait(sps_ctx* c, const PubTicket& t, const void** host) {
    char* base = (char*)c->pub + t.slot * kPubSlot;
    volatile unsigned long long* flag = (volatile unsigned long long*)base;
    for (uint64_t n = 1; *flag != t.seq; ++n) {
        if ((n & 1023) == 0) {
            const hipError_t e = hipStreamQuery(c->stream);
            if (e == hipSuccess) {
                // The stream has run the publishing kernel, whose system-scope stores
                // are visible once it completes.  (The device source cannot be read
                // again instead: launches queued after the publish may have changed it.)
                SPS_HIP(c, hipStreamSynchronize(c->stream));
                if (*flag == t.seq) break;
                return fail(c, SPS_ERR_HIP, "read-back: the published bytes did not arrive");
            }
            if (e != hipErrorNotReady) return hip_fail(c, e, "read-back");
        }
#if defined(__x86_64__)
        __builtin_ia32_pause();
#endif
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    *host = base + kPubHeader;
    return SPS_OK;
}

int readback(sps_ctx* c, const void* dsrc, size_t bytes, const void** host) {
    if (bytes > kPublishBytes) {
        SPS_CHECK(ensure_host(c, c->hostbuf, bytes));
        SPS_HIP(c, hipMemcpyAsync(c->hostbuf.p, dsrc, bytes, hipMemcpyDeviceToHost, c->stream));
        SPS_HIP(c, hipStreamSynchronize(c->stream));
        *host = c->hostbuf.p;
        return SPS_OK;
    }
    PubTicket t;
    SPS_CHECK(publish_async(c, dsrc, bytes, &t));
    return publish_wait(c, t, host);
}

// Round-to-nearest-even FP32 -> BF16 bits (inputs are finite).
__device__ __forceinline__ uint16_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ double bf16_value(uint16_t h) {
    return (double)__uint_as_float(((uint32_t)h) << 16);
}

// Checks y in [0, C) and X finite; flags[0] |= 1 bad y, |= 2 non-finite X.
__global__ void check_data_kernel(const double* __restrict__ X, const int32_t* __restrict__ y,
                                  int64_t T, int32_t k, int32_t C, unsigned* flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = T * k;
    unsigned f = 0;
    for (int64_t e = i; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        if (!isfinite(X[e])) f |= 2u;
    }
    for (int64_t t = i; t < T; t += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = y[t];
        if (v < 0 || v >= C) f |= 1u;
    }
    if (f) atomicOr(flags, f);
}

// Row-major padded copies: Xd, Xf (Tp x kp), Xh, Xl (Tp x kb) and y8.
__global__ void build_rows_kernel(const double* __restrict__ X, const int32_t* __restrict__ y,
                                  int64_t T, int32_t k, int32_t C, int64_t Tp, int32_t kp,
                                  int32_t kb, double* __restrict__ Xd, float* __restrict__ Xf,
                                  uint16_t* __restrict__ Xh, uint16_t* __restrict__ Xl,
                                  int8_t* __restrict__ y8) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t t = i / kb;
    int32_t col = (int32_t)(i % kb);
    if (t >= Tp) return;
    double v = 0.0;
    if (t < T && col < k) {
        double sgn = (C == 2) ? (1.0 - 2.0 * (double)y[t]) : 1.0;
        v = sgn * X[t * k + col];
    }
    if (col < kp) {
        Xd[t * kp + col] = v;
        Xf[t * kp + col] = (float)v;
    }
    uint16_t hi = bf16_bits((float)v);
    uint16_t lo = bf16_bits((float)(v - bf16_value(hi)));
    Xh[t * kb + col] = hi;
    Xl[t * kb + col] = lo;
    if (col == 0) y8[t] = (t < T) ? (int8_t)y[t] : (int8_t)0;
}

// Transposed copies (kp x Tp) for the adjoint contraction.
__global__ void build_cols_kernel(const double* __restrict__ Xd, int64_t Tp, int32_t kp, int32_t kt,
                                  double* __restrict__ XTd, float* __restrict__ XTf,
                                  uint16_t* __restrict__ XTh, uint16_t* __restrict__ XTl) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t t = i % Tp;
    int32_t col = (int32_t)(i / Tp);
    if (col >= kt) return;
    double v = col < kp ? Xd[t * kp + col] : 0.0;
    XTd[(int64_t)col * Tp + t] = v;
    XTf[(int64_t)col * Tp + t] = (float)v;
    uint16_t hi = bf16_bits((float)v);
    XTh[(int64_t)col * Tp + t] = hi;
    XTl[(int64_t)col * Tp + t] = bf16_bits((float)(v - bf16_value(hi)));
}

// Column means of the caller's X (unsigned), one block per column, fixed order.
__global__ void column_mean_kernel(const double* __restrict__ X, int64_t T, int32_t k,
                                   double* __restrict__ xbar) {
    __shared__ double red[256];
    int32_t col = blockIdx.x;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < T; t += blockDim.x) s += X[t * k + col];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) xbar[col] = red[0] / (double)T;
}

static void free_data(sps_ctx* c) {
    void* ps[] = {c->Xd, c->Xf, c->Xh, c->Xl, c->XTd, c->XTf, c->XTh, c->XTl, c->y8, c->xbar};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    c->Xd = nullptr; c->Xf = nullptr; c->Xh = nullptr; c->Xl = nullptr;
    c->XTd = nullptr; c->XTf = nullptr; c->XTh = nullptr; c->XTl = nullptr;
    c->y8 = nullptr; c->xbar = nullptr;
    c->has_data = false;
    c->suff_valid = false;
    c->has_sigma = false;
}

static void free_prior(sps_ctx* c) {
    double* ps[] = {c->prior_mean, c->prior_isd, c->prior_L, c->prior_Li, c->prior_LiT};
    for (double* p : ps)
        if (p) (void)hipFree(p);
    c->prior_mean = nullptr;
    c->prior_isd = nullptr;
    c->prior_L = nullptr;
    c->prior_Li = nullptr;
    c->prior_LiT = nullptr;
    c->prior_full = false;
    c->prior_cov_host.clear();
    c->has_prior = false;
}

int timing_begin(sps_ctx* c, int which, int* slot) {
    *slot = -1;
    if (!c->timing) return SPS_OK;
    hipEvent_t ev[2];
    for (int i = 0; i < 2; ++i) {
        if (!c->evpool.empty()) {
            ev[i] = c->evpool.back();
            c->evpool.pop_back();
        } else {
            SPS_HIP(c, hipEventCreate(&ev[i]));
        }
    }
    SPS_HIP(c, hipEventRecord(ev[0], c->stream));
    c->pending.push_back(sps_ctx::Timed{which, ev[0], ev[1]});
    *slot = (int)c->pending.size() - 1;
    return SPS_OK;
}

int timing_end(sps_ctx* c, int slot) {
    if (slot < 0) return SPS_OK;
    SPS_HIP(c, hipEventRecord(c->pending[slot].b, c->stream));
    return SPS_OK;
}

// Fold finished event pairs into the totals and recycle the events.
static int timing_collect(sps_ctx* c) {
    if (c->pending.empty()) return SPS_OK;
    SPS_HIP(c, hipStreamSynchronize(c->stream));
    for (auto& t : c->pending) {
        float ms = 0.f;
        SPS_HIP(c, hipEventElapsedTime(&ms, t.a, t.b));
        c->kt_ms[t.which] += ms;
        c->kt_n[t.which] += 1;
        c->evpool.push_back(t.a);
        c->evpool.push_back(t.b);
    }
    c->pending.clear();
    return SPS_OK;
}

void timing_release(sps_ctx* c) {
    (void)hipStreamSynchronize(c->stream);
    for (auto& t : c->pending) {
        (void)hipEventDestroy(t.a);
        (void)hipEventDestroy(t.b);
    }
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    c->pending.clear();
    c->evpool.clear();
}

}  // namespace sps

using namespace sps;

extern "C" int sps_timing_enable(sps_ctx* c, int enable) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    SPS_CHECK(timing_collect(c));
    c->timing = enable != 0;
    for (int i = 0; i < 3; ++i) {
        c->kt_ms[i] = 0.0;
        c->kt_n[i] = 0;
    }
    return SPS_OK;
}

extern "C" int sps_timing_read(sps_ctx* c, int which, int64_t* launches, double* total_ms) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (which < 0 || which > 2) return fail(c, SPS_ERR_ARG, "sps_timing_read: unknown kernel class %d", which);
    SPS_CHECK(timing_collect(c));
    if (launches) *launches = c->kt_n[which];
    if (total_ms) *total_ms = c->kt_ms[which];
    return SPS_OK;
}

extern "C" int sps_create(sps_ctx** out, int device, void* hip_stream) {
    if (!out) return SPS_ERR_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return SPS_ERR_HIP;
    if (device < 0 || device >= ndev) return SPS_ERR_ARG;
    sps_ctx* c = new (std::nothrow) sps_ctx();
    if (!c) return SPS_ERR_NOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return SPS_ERR_HIP;
    }
    // the no-allocation scratch of this device (its address, once per device)
    const int st = noalloc_setup(c, device);
    if (st != SPS_OK) {
        delete c;
        return st;
    }
    *out = c;
    return SPS_OK;
}

extern "C" void sps_destroy(sps_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_data(c);
    free_prior(c);
    Buf* bufs[] = {&c->part_ll, &c->part_g, &c->theta2, &c->ll2, &c->grad2, &c->cov, &c->chol,
                   &c->mean, &c->pstat, &c->z, &c->u, &c->u53, &c->corr_lw, &c->corr_red,
                   &c->small, &c->mstat, &c->W, &c->gstat, &c->suff, &c->pw};
    for (Buf* b : bufs)
        if (b->p) (void)hipFree(b->p);
    if (c->hostbuf.p) (void)hipHostFree(c->hostbuf.p);
    if (c->pub) (void)hipHostFree(c->pub);
    timing_release(c);
    delete c;
}

extern "C" const char* sps_last_error(const sps_ctx* c) { return c ? c->err.c_str() : "null context"; }

extern "C" int sps_set_stream(sps_ctx* c, void* hip_stream) {
    if (!c) return SPS_ERR_ARG;
    c->stream = (hipStream_t)hip_stream;
    return SPS_OK;
}

extern "C" int sps_set_data(sps_ctx* c, const double* X, const int32_t* y, int64_t T, int32_t k,
                            int32_t C) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!X || !y) return fail(c, SPS_ERR_ARG, "sps_set_data: null X or y");
    if (T < 1 || T >= (int64_t(1) << 31)) return fail(c, SPS_ERR_ARG, "sps_set_data: T=%lld out of range", (long long)T);
    if (k < 1 || k > 128) return fail(c, SPS_ERR_ARG, "sps_set_data: k=%d outside [1, 128]", k);
    if (C < 2 || C > 8) return fail(c, SPS_ERR_ARG, "sps_set_data: C=%d outside [2, 8]", C);
    SPS_HIP(c, hipSetDevice(c->device));
    SPS_HIP(c, hipStreamSynchronize(c->stream));
    free_data(c);
    free_prior(c);

    SPS_CHECK(ensure(c, c->small, 4096, "small"));
    SPS_CHECK(ensure_host(c, c->hostbuf, 4096));
    unsigned* flags = (unsigned*)c->small.p;
    SPS_HIP(c, hipMemsetAsync(flags, 0, sizeof(unsigned), c->stream));
    check_data_kernel<<<256, 256, 0, c->stream>>>(X, y, T, k, C, flags);
    SPS_CHECK(launched(c, "check_data_kernel"));
    SPS_HIP(c, hipMemcpyAsync(c->hostbuf.p, flags, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream));
    SPS_HIP(c, hipStreamSynchronize(c->stream));
    unsigned f = *(unsigned*)c->hostbuf.p;
    if (f & 1u) return fail(c, SPS_ERR_ARG, "sps_set_data: an outcome lies outside [0, %d)", C);
    if (f & 2u) return fail(c, SPS_ERR_NONFINITE, "sps_set_data: X holds NaN or inf");

    // Row strides are powers of two times the MFMA contraction length, so each
    // likelihood kernel instantiation sees a fixed number of k-steps:
    //   FP64/FP32 rows: kp = max(16, 4 * 2^ceil(log2(ceil(k / 4))))  (16..128)
    //   BF16 rows     : kb = 32 * 2^ceil(log2(ceil(k / 32)))          (32..128)
    //   transposed    : kt = max(kp, kb) rows of Tp
    auto np2 = [](int v) { int r = 1; while (r < v) r <<= 1; return r; };
    int64_t Tp = ((T + kObsStep - 1) / kObsStep) * kObsStep + kObsStep;
    int32_t kp = std::max(16, 4 * np2((k + 3) / 4));
    int32_t kb = 32 * np2((k + 31) / 32);
    int32_t kt = std::max(kp, kb);
    auto alloc = [&](void** p, size_t bytes, const char* what) -> int {
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            *p = nullptr;
            free_data(c);
            return hip_fail(c, e, what);
        }
        return SPS_OK;
    };
    SPS_CHECK(alloc((void**)&c->Xd, sizeof(double) * Tp * kp, "Xd"));
    SPS_CHECK(alloc((void**)&c->Xf, sizeof(float) * Tp * kp, "Xf"));
    SPS_CHECK(alloc((void**)&c->Xh, sizeof(uint16_t) * Tp * kb, "Xh"));
    SPS_CHECK(alloc((void**)&c->Xl, sizeof(uint16_t) * Tp * kb, "Xl"));
    SPS_CHECK(alloc((void**)&c->XTd, sizeof(double) * Tp * kt, "XTd"));
    SPS_CHECK(alloc((void**)&c->XTf, sizeof(float) * Tp * kt, "XTf"));
    SPS_CHECK(alloc((void**)&c->XTh, sizeof(uint16_t) * Tp * kt, "XTh"));
    SPS_CHECK(alloc((void**)&c->XTl, sizeof(uint16_t) * Tp * kt, "XTl"));
    SPS_CHECK(alloc((void**)&c->y8, (size_t)Tp, "y8"));
    SPS_CHECK(alloc((void**)&c->xbar, sizeof(double) * k, "xbar"));

    int64_t nrow = Tp * kb;
    build_rows_kernel<<<(unsigned)((nrow + 255) / 256), 256, 0, c->stream>>>(
        X, y, T, k, C, Tp, kp, kb, c->Xd, c->Xf, c->Xh, c->Xl, c->y8);
    SPS_CHECK(launched(c, "build_rows_kernel"));
    int64_t ncol = Tp * kt;
    build_cols_kernel<<<(unsigned)((ncol + 255) / 256), 256, 0, c->stream>>>(
        c->Xd, Tp, kp, kt, c->XTd, c->XTf, c->XTh, c->XTl);
    SPS_CHECK(launched(c, "build_cols_kernel"));
    column_mean_kernel<<<k, 256, 0, c->stream>>>(X, T, k, c->xbar);
    SPS_CHECK(launched(c, "column_mean_kernel"));
    SPS_HIP(c, hipStreamSynchronize(c->stream));

    c->T = T;
    c->k = k;
    c->C = C;
    c->d = k * (C - 1);
    c->Tp = Tp;
    c->kp = kp;
    c->kb = kb;
    c->kt = kt;
    c->has_data = true;
    return SPS_OK;
}

extern "C" int sps_set_prior(sps_ctx* c, const double* mean, const double* sd) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!c->has_data) return fail(c, SPS_ERR_STATE, "sps_set_prior: call sps_set_data first");
    if (!mean || !sd) return fail(c, SPS_ERR_ARG, "sps_set_prior: null mean or sd");
    int d = c->d;
    double* isd = (double*)malloc(sizeof(double) * d);
    if (!isd) return fail(c, SPS_ERR_NOMEM, "sps_set_prior: host allocation");
    for (int i = 0; i < d; ++i) {
        if (!(sd[i] > 0.0) || !std::isfinite(sd[i]) || !std::isfinite(mean[i])) {
            free(isd);
            return fail(c, SPS_ERR_ARG, "sps_set_prior: sd[%d] must be positive and finite", i);
        }
        isd[i] = 1.0 / sd[i];
    }
    SPS_HIP(c, hipSetDevice(c->device));
    SPS_HIP(c, hipStreamSynchronize(c->stream));
    free_prior(c);
    hipError_t e1 = hipMalloc((void**)&c->prior_mean, sizeof(double) * d);
    hipError_t e2 = hipMalloc((void**)&c->prior_isd, sizeof(double) * d);
    if (e1 != hipSuccess || e2 != hipSuccess) {
        free(isd);
        free_prior(c);
        return fail(c, SPS_ERR_NOMEM, "sps_set_prior: device allocation");
    }
    hipError_t e3 = hipMemcpy(c->prior_mean, mean, sizeof(double) * d, hipMemcpyHostToDevice);
    hipError_t e4 = hipMemcpy(c->prior_isd, isd, sizeof(double) * d, hipMemcpyHostToDevice);
    free(isd);
    if (e3 != hipSuccess) return hip_fail(c, e3, "sps_set_prior: copy");
    if (e4 != hipSuccess) return hip_fail(c, e4, "sps_set_prior: copy");
    c->prior_cov_host.assign((size_t)d * d, 0.0);
    for (int i = 0; i < d; ++i) c->prior_cov_host[(size_t)i * d + i] = sd[i] * sd[i];
    c->has_prior = true;
    return SPS_OK;
}

// ---- full prior covariance ------------------------------------------------

// Lower Cholesky factor of the symmetric n x n matrix A (row-major, lower
// triangle read).  False when A is not numerically positive definite.
static bool host_cholesky(const double* A, int n, double* L) {
    for (int i = 0; i < n * n; ++i) L[i] = 0.0;
    for (int j = 0; j < n; ++j) {
        double s = A[j * n + j];
        for (int q = 0; q < j; ++q) s -= L[j * n + q] * L[j * n + q];
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        const double ljj = std::sqrt(s);
        L[j * n + j] = ljj;
        for (int i = j + 1; i < n; ++i) {
            double t = A[i * n + j];
            for (int q = 0; q < j; ++q) t -= L[i * n + q] * L[j * n + q];
            L[i * n + j] = t / ljj;
        }
    }
    return true;
}

// Inverse of a lower-triangular n x n matrix (column by column forward substitution).
static void host_trinv(const double* L, int n, double* Li) {
    for (int i = 0; i < n * n; ++i) Li[i] = 0.0;
    for (int col = 0; col < n; ++col)
        for (int i = col; i < n; ++i) {
            double s = (i == col) ? 1.0 : 0.0;
            for (int q = col; q < i; ++q) s -= L[i * n + q] * Li[q * n + col];
            Li[i * n + col] = s / L[i * n + i];
        }
}

// Install N(mean, cov) on the free parameters (mean null: zero).
static int set_prior_full(sps_ctx* c, const double* mean, const std::vector<double>& cov, const char* who) {
    const int d = c->d;
    const size_t dd = (size_t)d * d;
    std::vector<double> L(dd), Li(dd), LiT(dd), mu(d, 0.0);
    if (mean)
        for (int i = 0; i < d; ++i) {
            if (!std::isfinite(mean[i])) return fail(c, SPS_ERR_ARG, "%s: mean[%d] is not finite", who, i);
            mu[i] = mean[i];
        }
    if (!host_cholesky(cov.data(), d, L.data()))
        return fail(c, SPS_ERR_NOT_PD, "%s: the prior covariance is not positive definite", who);
    host_trinv(L.data(), d, Li.data());
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j) LiT[(size_t)j * d + i] = Li[(size_t)i * d + j];
    SPS_HIP(c, hipSetDevice(c->device));
    SPS_HIP(c, hipStreamSynchronize(c->stream));
    free_prior(c);
    double** dst[] = {&c->prior_mean, &c->prior_L, &c->prior_Li, &c->prior_LiT};
    const double* src[] = {mu.data(), L.data(), Li.data(), LiT.data()};
    const size_t n[] = {(size_t)d, dd, dd, dd};
    for (int q = 0; q < 4; ++q) {
        if (hipMalloc((void**)dst[q], sizeof(double) * n[q]) != hipSuccess) {
            free_prior(c);
            return fail(c, SPS_ERR_NOMEM, "%s: device allocation", who);
        }
        hipError_t e = hipMemcpy(*dst[q], src[q], sizeof(double) * n[q], hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_prior(c);
            return hip_fail(c, e, who);
        }
    }
    c->prior_cov_host = cov;
    c->prior_full = true;
    c->has_prior = true;
    return SPS_OK;
}

extern "C" int sps_set_prior_cov(sps_ctx* c, const double* mean, const double* cov) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!c->has_data) return fail(c, SPS_ERR_STATE, "sps_set_prior_cov: call sps_set_data first");
    if (!cov) return fail(c, SPS_ERR_ARG, "sps_set_prior_cov: null covariance");
    const int d = c->d;
    std::vector<double> S(cov, cov + (size_t)d * d);
    for (int i = 0; i < d; ++i)
        for (int j = 0; j < i; ++j) {
            const double a = S[(size_t)i * d + j], b = S[(size_t)j * d + i];
            if (!std::isfinite(a) || !std::isfinite(b) ||
                std::fabs(a - b) > 1e-12 * std::max(1.0, std::max(std::fabs(a), std::fabs(b))))
                return fail(c, SPS_ERR_ARG, "sps_set_prior_cov: covariance not symmetric at (%d, %d)", i, j);
        }
    return set_prior_full(c, mean, S, "sps_set_prior_cov");
}

// X'X over all observations, one workgroup per entry (a <= b), fixed order.
// The sign folding of binary rows cancels in the products.
__global__ __launch_bounds__(256) void xtx_kernel(const double* __restrict__ XT, int64_t Tp, int64_t T,
                                                   int32_t k, double* __restrict__ out) {
    __shared__ double red[256];
    int32_t e = blockIdx.x, a = 0;
    while (e >= k - a) {  // blockIdx -> (a, b), b >= a
        e -= k - a;
        ++a;
    }
    const int32_t b = a + e;
    const double* xa = XT + (int64_t)a * Tp;
    const double* xb = XT + (int64_t)b * Tp;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < T; t += 256) s += xa[t] * xb[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[(int64_t)a * k + b] = red[0];
        out[(int64_t)b * k + a] = red[0];
    }
}

extern "C" int sps_set_prior_g(sps_ctx* c, double g, const double* mean) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!c->has_data) return fail(c, SPS_ERR_STATE, "sps_set_prior_g: call sps_set_data first");
    if (!(g > 0.0) || !std::isfinite(g)) return fail(c, SPS_ERR_ARG, "sps_set_prior_g: g must be positive");
    const int k = c->k, d = c->d, m = c->C - 1;
    SPS_HIP(c, hipSetDevice(c->device));
    SPS_CHECK(ensure(c, c->small, std::max<size_t>(4096, sizeof(double) * (size_t)k * k), "small"));
    const unsigned nblk = (unsigned)((int64_t)k * (k + 1) / 2);
    xtx_kernel<<<nblk, 256, 0, c->stream>>>(c->XTd, c->Tp, c->T, k, (double*)c->small.p);
    SPS_CHECK(launched(c, "xtx_kernel"));
    std::vector<double> XtX((size_t)k * k), Ls((size_t)k * k), Lsi((size_t)k * k);
    SPS_HIP(c, hipMemcpyAsync(XtX.data(), c->small.p, sizeof(double) * k * k, hipMemcpyDeviceToHost, c->stream));
    SPS_HIP(c, hipStreamSynchronize(c->stream));
    if (!host_cholesky(XtX.data(), k, Ls.data()))
        return fail(c, SPS_ERR_NOT_PD, "sps_set_prior_g: X'X is singular");
    // Sigma = g T (X'X)^-1 = g T Ls^-T Ls^-1
    host_trinv(Ls.data(), k, Lsi.data());
    std::vector<double> Sig((size_t)k * k);
    for (int i = 0; i < k; ++i)
        for (int j = 0; j < k; ++j) {
            double s = 0.0;
            for (int q = std::max(i, j); q < k; ++q) s += Lsi[(size_t)q * k + i] * Lsi[(size_t)q * k + j];
            Sig[(size_t)i * k + j] = g * (double)c->T * s;
        }
    // normalised on outcome 0: block (ci, cj) = (1 + [ci == cj]) Sigma
    std::vector<double> S((size_t)d * d);
    for (int ci = 0; ci < m; ++ci)
        for (int cj = 0; cj < m; ++cj)
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b)
                    S[((size_t)ci * k + a) * d + (size_t)cj * k + b] = (ci == cj ? 2.0 : 1.0) * Sig[(size_t)a * k + b];
    return set_prior_full(c, mean, S, "sps_set_prior_g");
}

extern "C" int sps_get_prior_cov(sps_ctx* c, double* cov) {
    if (!c) return SPS_ERR_ARG;
    c->err.clear();
    if (!c->has_prior) return fail(c, SPS_ERR_STATE, "sps_get_prior_cov: no prior set");
    if (!cov) return fail(c, SPS_ERR_ARG, "sps_get_prior_cov: null output");
    std::copy(c->prior_cov_host.begin(), c->prior_cov_host.end(), cov);
    return SPS_OK;
}
