// LDS read bandwidth of gfx950, measured: the denominator of the fused step's
// LDS roofline.  Every lane reads 16-byte words (ds_read_b128) from a 64 KiB
// LDS buffer, the 64 lanes of a wavefront one contiguous, aligned kilobyte per
// instruction, so no two lanes of an instruction share a bank cycle.  The
// reads are folded with xor into one word per thread, which is stored, so
// none of them can be dropped; the host recomputes the stored words.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "navsim_host.hpp"
#include "navsim_probe.h"

namespace navsim {
namespace {

constexpr int kWords = 4096;       // 16-byte words in the buffer (64 KiB)
constexpr int kUnroll = 16;        // reads per outer iteration, 256 words apart
constexpr int kSpan = 256;         // words between two reads of one lane

__host__ __device__ inline uint4 probe_word(uint32_t i) {
    return make_uint4(i * 2654435761u, i ^ 0x9E3779B9u, i + 7u, ~i);
}

template <int T>
__global__ __launch_bounds__(T) void lds_read_kernel(uint32_t *out, int iters) {
    __shared__ uint4 buf[kWords];
    const int tid = threadIdx.x;
    for (int i = tid; i < kWords; i += T) buf[i] = probe_word((uint32_t)i);
    __syncthreads();
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    for (int it = 0; it < iters; ++it) {
        // the wavefront's 64 lanes read 64 consecutive words (1 KiB, aligned)
        const uint4 *q = buf + ((tid + it * 64) & (kSpan - 1));
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            const uint4 v = q[k * kSpan];
            acc.x ^= v.x;
            acc.y ^= v.y;
            acc.z ^= v.z;
            acc.w ^= v.w;
        }
    }
    out[(size_t)blockIdx.x * T + tid] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

navsim_status hip_fail(const char *what, hipError_t e) {
    return fail(NAVSIM_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace
}  // namespace navsim

using namespace navsim;

extern "C" navsim_status navsim_probe_lds_read(int hip_device, int32_t threads, int32_t blocks,
                                               int32_t iters, int32_t launches, uint32_t *out_host,
                                               double *ms_per_launch, double *bytes_per_launch) {
    if (!(threads == 256 || threads == 512 || threads == 1024) || blocks < 1 ||
        blocks > (1 << 20) || iters < 1 || iters > (1 << 20) || launches < 1 || launches > 1000 ||
        !ms_per_launch || !bytes_per_launch) {
        return fail(NAVSIM_E_INVALID_ARG,
                    "navsim_probe_lds_read: threads must be 256, 512 or 1024, 1 <= blocks, iters "
                    "<= 2^20, 1 <= launches <= 1000, output pointers non-null");
    }
    DeviceGuard guard(hip_device);
    if (guard.err != hipSuccess) return hip_fail("hipSetDevice", guard.err);
    hipError_t e = hipSuccess;
    const size_t n = (size_t)blocks * (size_t)threads;
    uint32_t *d_out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    navsim_status rc = NAVSIM_OK;
    auto launch = [&]() {
        if (threads == 256)
            lds_read_kernel<256><<<blocks, 256>>>(d_out, iters);
        else if (threads == 512)
            lds_read_kernel<512><<<blocks, 512>>>(d_out, iters);
        else
            lds_read_kernel<1024><<<blocks, 1024>>>(d_out, iters);
        return hipGetLastError();
    };
    float ms = 0.0f;
    if ((e = hipMalloc(&d_out, n * sizeof(uint32_t))) != hipSuccess) return fail(NAVSIM_E_OOM, "hipMalloc: %s", hipGetErrorString(e));
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) {
        rc = hip_fail("hipEventCreate", e);
        goto done;
    }
    if ((e = launch()) != hipSuccess) {  // warm-up
        rc = hip_fail("lds_read_kernel", e);
        goto done;
    }
    if ((e = hipEventRecord(a, nullptr)) != hipSuccess) {
        rc = hip_fail("hipEventRecord", e);
        goto done;
    }
    for (int l = 0; l < launches; ++l)
        if ((e = launch()) != hipSuccess) {
            rc = hip_fail("lds_read_kernel", e);
            goto done;
        }
    if ((e = hipEventRecord(b, nullptr)) != hipSuccess || (e = hipEventSynchronize(b)) != hipSuccess ||
        (e = hipEventElapsedTime(&ms, a, b)) != hipSuccess) {
        rc = hip_fail("timing", e);
        goto done;
    }
    *ms_per_launch = (double)ms / launches;
    *bytes_per_launch = (double)n * (double)iters * kUnroll * 16.0;
    if (out_host && (e = hipMemcpy(out_host, d_out, n * sizeof(uint32_t), hipMemcpyDeviceToHost)) !=
                        hipSuccess)
        rc = hip_fail("hipMemcpy", e);
done:
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    (void)hipFree(d_out);
    return rc;
}
