// Random-access calibration: the device's rate of 4-byte gathers and
// read-modify-writes at distinct random word addresses of one buffer, of a
// plain copy, and of random read-modify-writes that stay inside one eighth
// of the buffer per XCD, on the caller's stream.  A measurement aid for
// reading the sweep kernels' times (their residual accesses are 4-byte and,
// for rows an earlier class owns, random inside the XCD's window of the row
// layout); nothing in the method calls it.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "thetis_internal.h"

namespace {

// bijection on [0, 2^k): odd multiplications and xor-shifts, each invertible
// on k-bit words, so the addresses of one pass are distinct
__device__ __forceinline__ uint32_t scramble(uint32_t x, uint32_t mask, int k) {
    x = (x * 0x9E3779B1u) & mask;
    x ^= x >> ((k + 1) / 2);
    x = (x * 0x85EBCA77u) & mask;
    x ^= x >> ((k + 2) / 3);
    x = (x * 0xC2B2AE3Du) & mask;
    x ^= x >> ((k + 1) / 2);
    return x;
}

__global__ __launch_bounds__(256) void k_cal_gather(const float *__restrict__ buf, uint32_t mask, int k,
                                                    float *__restrict__ sink) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i > mask) return;
    const float v = buf[scramble(i, mask, k)];
    if (v == -1.0f) sink[0] = v;          // never true: the buffer holds zeros and ones
}

__global__ __launch_bounds__(256) void k_cal_rmw(float *__restrict__ buf, uint32_t mask, int k) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i > mask) return;
    const uint32_t j = scramble(i, mask, k);
    buf[j] = buf[j] + 1.0f;
}

// workgroup b runs on XCD b % 8 and touches only window b % 8 (an eighth of
// the buffer), each word of it once per pass
__global__ __launch_bounds__(256) void k_cal_rmw_xcd(float *__restrict__ buf, uint32_t wmask, int wk) {
    const uint32_t x = blockIdx.x & 7u, i = (blockIdx.x >> 3) * 256u + threadIdx.x;
    if (i > wmask) return;
    const uint32_t j = x * (wmask + 1) + scramble(i, wmask, wk);
    buf[j] = buf[j] + 1.0f;
}

__global__ __launch_bounds__(256) void k_cal_copy(const float *__restrict__ a, float *__restrict__ b, uint32_t mask) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i <= mask) b[i] = a[i];
}

}  // namespace

using thetis::exception_status;
using thetis::fail;

extern "C" thetis_status thetis_calibrate_random(int32_t words_log2, int32_t iters, void *stream,
                                                 double *ms_host) {
    try {
        thetis::clear_error();
        if (words_log2 < 13 || words_log2 > 28) return fail(THETIS_EINVAL, "words_log2 must be in [13, 28]");
        if (iters < 1) return fail(THETIS_EINVAL, "iters must be positive");
        if (!ms_host) return fail(THETIS_EINVAL, "ms_host is NULL");
        const uint32_t words = 1u << words_log2, mask = words - 1;
        const hipStream_t st = (hipStream_t)stream;
        float *buf = nullptr, *dst = nullptr;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        thetis_status rc = THETIS_OK;
        auto check = [&](hipError_t e, const char *what) {
            if (e != hipSuccess && rc == THETIS_OK) rc = fail(THETIS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
            return rc == THETIS_OK;
        };
        if (check(hipMalloc(&buf, sizeof(float) * words), "hipMalloc") &&
            check(hipMalloc(&dst, sizeof(float) * words), "hipMalloc") &&
            check(hipMemsetAsync(buf, 0, sizeof(float) * words, st), "hipMemsetAsync") &&
            check(hipEventCreate(&e0), "hipEventCreate") && check(hipEventCreate(&e1), "hipEventCreate")) {
            const dim3 grid(words / 256u), block(256);
            for (int kind = 0; kind < 4 && rc == THETIS_OK; ++kind) {
                auto launch = [&]() {
                    if (kind == 0) hipLaunchKernelGGL(k_cal_gather, grid, block, 0, st, buf, mask, words_log2, dst);
                    else if (kind == 1) hipLaunchKernelGGL(k_cal_rmw, grid, block, 0, st, buf, mask, words_log2);
                    else if (kind == 2) hipLaunchKernelGGL(k_cal_copy, grid, block, 0, st, buf, dst, mask);
                    else hipLaunchKernelGGL(k_cal_rmw_xcd, grid, block, 0, st, buf, (words >> 3) - 1, words_log2 - 3);
                };
                launch();                                          // warm-up
                if (!check(hipEventRecord(e0, st), "hipEventRecord")) break;
                for (int it = 0; it < iters; ++it) launch();
                if (!check(hipGetLastError(), "kernel launch") || !check(hipEventRecord(e1, st), "hipEventRecord") ||
                    !check(hipEventSynchronize(e1), "hipEventSynchronize"))
                    break;
                float ms = 0.f;
                if (!check(hipEventElapsedTime(&ms, e0, e1), "hipEventElapsedTime")) break;
                ms_host[kind] = (double)ms / iters;
            }
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (buf) { (void)hipStreamSynchronize(st); (void)hipFree(buf); }
        if (dst) (void)hipFree(dst);
        return rc;
    } catch (...) {
        return exception_status();
    }
}
