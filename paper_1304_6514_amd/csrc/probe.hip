// The dependent-issue latency of the vector FMA (include/nv_probe.h): one
// wave, a chain of dependent FMAs per lane, timed with HIP events around the
// launch and with the shader clock counter inside the kernel.
#include "nv_probe.h"
#include "nv_internal.h"

#include <hip/hip_runtime.h>

namespace nv {
namespace {

// out[0]: clock ticks over the chain (lane 0), out[1..2]: the chain's result,
// stored so that the chain cannot be removed.
template <class R>
__global__ __launch_bounds__(64) void fma_chain_kernel(long long ops, R a, R b, R x0,
                                                       long long *ticks, R *out) {
    R x = x0 + R(threadIdx.x) * b;
    const long long t0 = clock64();
    for (long long i = 0; i < ops; i += 64) {
#pragma unroll
        for (int k = 0; k < 64; ++k) {
            if constexpr (sizeof(R) == 8)
                x = __builtin_fma(x, a, b);
            else
                x = __builtin_fmaf(x, a, b);
        }
    }
    const long long t1 = clock64();
    if (threadIdx.x == 0) ticks[0] = t1 - t0;
    out[threadIdx.x] = x;
}

}  // namespace
}  // namespace nv

extern "C" NV_API nv_status nv_probe_fma_latency(int precision, long long ops, void *stream,
                                                 double *ns_per_op, double *cycles_per_op) {
    using nv::fail;
    if (!ns_per_op || !cycles_per_op) return fail(NV_ERR_INVALID_ARG, "NULL output");
    if (ops < 1024 || ops % 64 != 0)
        return fail(NV_ERR_INVALID_ARG, "ops must be >= 1024 and a multiple of 64");
    if (precision != NV_FP64 && precision != NV_FP32)
        return fail(NV_ERR_INVALID_ARG, "unknown precision %d", precision);
    hipStream_t st = static_cast<hipStream_t>(stream);
    // [ticks][64 results of the widest type]
    void *buf = nullptr;
    const size_t bytes = sizeof(long long) + 64 * sizeof(double);
    if (hipMalloc(&buf, bytes) != hipSuccess) return fail(NV_ERR_OOM, "hipMalloc failed");
    long long *ticks = static_cast<long long *>(buf);
    void *out = static_cast<char *>(buf) + sizeof(long long);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) {
        // a = 1 - 2^-20 and b = 2^-30 keep x bounded and never subnormal
        if (precision == NV_FP64)
            hipLaunchKernelGGL(nv::fma_chain_kernel<double>, dim3(1), dim3(64), 0, st, ops,
                               1.0 - 0x1p-20, 0x1p-30, 1.0, ticks, static_cast<double *>(out));
        else
            hipLaunchKernelGGL(nv::fma_chain_kernel<float>, dim3(1), dim3(64), 0, st, ops,
                               1.0f - 0x1p-20f, 0x1p-30f, 1.0f, ticks, static_cast<float *>(out));
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    long long t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess) e = hipMemcpy(&t, ticks, sizeof t, hipMemcpyDeviceToHost);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(buf);
    if (e != hipSuccess) return fail(NV_ERR_HIP, "latency probe failed: %s", hipGetErrorString(e));
    *ns_per_op = 1e6 * double(ms) / double(ops);
    *cycles_per_op = double(t) / double(ops);
    return NV_OK;
}
