/*
 * nv_probe.h — a measurement of libnv's: the dependent-issue latency of the
 * vector fused multiply-add on the current device.
 *
 * Builds too small to fill the chip (the logistic workload: 16,384
 * trajectories, one wave per SIMD on 64 CUs) are bound by the latency of
 * each trajectory's chain of dependent operations, not by issue rate: the
 * (Mn/N) tau_F term of the GPU cost model of sec. 4 then has tau_F = (the
 * dependent operations on one step's critical path) x (this latency).  This
 * call measures the latency so that such builds can be reported against that
 * bound.
 *
 * Conventions as in nv.h.
 */
#ifndef NV_PROBE_H
#define NV_PROBE_H

#include "nv.h"

#ifdef __cplusplus
extern "C" {
#endif

/* One wave runs, in every lane, a chain of `ops` dependent FMAs
 * x <- x a + b (a, b runtime values, FP64 for precision NV_FP64, FP32 for
 * NV_FP32) on `stream` (NULL = null stream).  *ns_per_op: HIP-event time of the
 * launch over ops (launch overhead included, negligible for ops >= 2^20);
 * *cycles_per_op: the shader clock counter's ticks over the chain, read in the
 * kernel, over ops.  Synchronous; allocates and frees a 64-byte device buffer.
 * Errors: NV_ERR_INVALID_ARG (ops < 1024 or not a multiple of 64, NULL
 * outputs, unknown precision), NV_ERR_OOM, NV_ERR_HIP. */
NV_API nv_status nv_probe_fma_latency(int precision, long long ops, void *stream,
                                      double *ns_per_op, double *cycles_per_op);

#ifdef __cplusplus
}
#endif
#endif /* NV_PROBE_H */
