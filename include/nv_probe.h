/*
 * nv_probe.h — a measurement of libnv's: how fast one wave issues vector fused
 * multiply-adds on the current device, dependent or not.
 *
 * Builds too small to fill the chip (the logistic workload: 16,384
 * trajectories, one wave per SIMD on 64 CUs) run each wave alone on its SIMD;
 * the (Mn/N) tau_F term of the GPU cost model of sec. 4 then has tau_F = the
 * longer of (the step's VALU instructions) x (one wave's time per independent
 * FMA) and (the dependent operations on the step's critical path) x (its time
 * per dependent FMA).  These calls measure both times so that such builds can
 * be reported against that bound.
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

/* The same with `chains` (1, 2 or 4) independent chains of `ops` dependent
 * FMAs per lane, interleaved in one wave: *ns_per_fma and *cycles_per_fma are
 * per FMA issued (ops x chains of them).  With one chain this is the dependent
 * latency above; with several, the rate at which one wave issues FMAs that do
 * not wait for each other, so that a single wave's loop can be bounded by its
 * instruction count where that, and not its dependent path, decides.
 * Errors as above, and NV_ERR_INVALID_ARG for another chain count. */
NV_API nv_status nv_probe_fma_chains(int precision, long long ops, int chains, void *stream,
                                     double *ns_per_fma, double *cycles_per_fma);

#ifdef __cplusplus
}
#endif
#endif /* NV_PROBE_H */
