// The issue time of the vector FMA for one wave (include/nv_probe.h): one
// wave, 1, 2 or 4 independent chains of dependent FMAs per lane, timed with
// HIP events around the launch and with the shader clock counter inside the
// kernel.
#include "nv_probe.h"
#include "nv_internal.h"

#include <hip/hip_runtime.h>

namespace nv {
namespace {

// C independent chains of dependent FMAs per lane, interleaved; ticks[0]:
// clock ticks over the chains (lane 0); out: the chains' sum per lane, stored
// so that no chain can be removed.
template <class R, int C>
__global__ __launch_bounds__(64) void fma_chain_kernel(long long ops, R a, R b, R x0,
                                                       long long *ticks, R *out) {
    R x[C];
#pragma unroll
    for (int c = 0; c < C; ++c) x[c] = x0 + R(threadIdx.x + 64 * c) * b;
    const long long t0 = clock64();
    for (long long i = 0; i < ops; i += 64) {
#pragma unroll
        for (int k = 0; k < 64; ++k) {
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if constexpr (sizeof(R) == 8)
                    x[c] = __builtin_fma(x[c], a, b);
                else
                    x[c] = __builtin_fmaf(x[c], a, b);
            }
        }
    }
    const long long t1 = clock64();
    if (threadIdx.x == 0) ticks[0] = t1 - t0;
    R sum = R(0);
#pragma unroll
    for (int c = 0; c < C; ++c) sum += x[c];
    out[threadIdx.x] = sum;
}

template <class R>
hipError_t launch_chains(int chains, long long ops, R a, R b, R x0, long long *ticks, R *out,
                         hipStream_t st) {
    switch (chains) {
    case 1: hipLaunchKernelGGL((fma_chain_kernel<R, 1>), dim3(1), dim3(64), 0, st, ops, a, b, x0, ticks, out); break;
    case 2: hipLaunchKernelGGL((fma_chain_kernel<R, 2>), dim3(1), dim3(64), 0, st, ops, a, b, x0, ticks, out); break;
    case 4: hipLaunchKernelGGL((fma_chain_kernel<R, 4>), dim3(1), dim3(64), 0, st, ops, a, b, x0, ticks, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace
}  // namespace nv

extern "C" NV_API nv_status nv_probe_fma_chains(int precision, long long ops, int chains,
                                                void *stream, double *ns_per_fma,
                                                double *cycles_per_fma) {
    using nv::fail;
    if (!ns_per_fma || !cycles_per_fma) return fail(NV_ERR_INVALID_ARG, "NULL output");
    if (ops < 1024 || ops % 64 != 0)
        return fail(NV_ERR_INVALID_ARG, "ops must be >= 1024 and a multiple of 64");
    if (chains != 1 && chains != 2 && chains != 4)
        return fail(NV_ERR_INVALID_ARG, "chains must be 1, 2 or 4 (got %d)", chains);
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
            e = nv::launch_chains<double>(chains, ops, 1.0 - 0x1p-20, 0x1p-30, 1.0, ticks,
                                          static_cast<double *>(out), st);
        else
            e = nv::launch_chains<float>(chains, ops, 1.0f - 0x1p-20f, 0x1p-30f, 1.0f, ticks,
                                         static_cast<float *>(out), st);
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
    if (e != hipSuccess) return fail(NV_ERR_HIP, "FMA probe failed: %s", hipGetErrorString(e));
    const double fmas = double(ops) * double(chains);
    *ns_per_fma = 1e6 * double(ms) / fmas;
    *cycles_per_fma = double(t) / fmas;
    return NV_OK;
}

extern "C" NV_API nv_status nv_probe_fma_latency(int precision, long long ops, void *stream,
                                                 double *ns_per_op, double *cycles_per_op) {
    return nv_probe_fma_chains(precision, ops, 1, stream, ns_per_op, cycles_per_op);
}
