#!/usr/bin/env python3
"""Benchmark: trajectory-steps/s of the Nievergelt propagator build on one GPU.

One step = one pass of the whole hot path over the forced-cubic workload
(y' = sin 3t - y^3 on [0, 100], 4096 slices x 4096 grid points x 2000 RK4
steps, FP32 build with compensated update, FP64 cubic-Hermite composition):
forcing precompute + ensemble integration + table write + composition down to
y(T) and the 4097 boundary states on the host, through nv_solve (the
composition of each slice chunk runs as soon as its tables are complete).
Inputs (problem parameters) are resident; the table and scratch buffers are
allocated before the timed region.

Prints one JSON line.  `value` = trajectory-steps per second of whole steps.
`roofline` describes the dominant kernel (the ensemble integrator), timed with
HIP events on the stream it is launched on.  `cpu_baseline` times the CPU
oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_1304_6514_amd import workloads as W  # noqa: E402

# MI355X published peaks used as denominators
PEAK_FP32_VECTOR_TFLOPS = 157.3          # 256 CU x 128 FMA lanes x 2 FLOP x 2.4 GHz
PEAK_FP64_VECTOR_TFLOPS = 78.6

# algorithmic FLOPs per trajectory-step (FMA = 2): RK4 = 12*dim + 4*c_f with c_f
# the right-hand side's cost; the compensated FP32 update adds 3 per component
RHS_FLOPS = {"linear": 1, "logistic": 2, "forced_cubic": 3, "vdp": 5, "square": 1}

WORKLOADS = {"forced_cubic": W.FORCED_CUBIC_FP32, "logistic": W.LOGISTIC_FP64,
             "vdp": W.VDP_FP32}


def flops_per_step(w: W.Workload, compensated: bool) -> int:
    if w.scheme == "rk4":
        f = 12 * w.dim + 4 * RHS_FLOPS[w.rhs]
    else:
        f = 2 * w.dim + RHS_FLOPS[w.rhs]
    if w.precision == "fp32" and compensated:
        f += 3 * w.dim
    return f


def cpu_baseline(w: W.Workload, n_slices_sample: int):
    """The oracle (as it is, single-threaded C) on the first slices of w."""
    import numpy as np
    import oracle

    oracle._load()
    g = oracle.make_grid(w.grid_n, w.grid_lo, w.grid_hi)
    sl = np.repeat(np.arange(n_slices_sample, dtype=np.int64), w.points_per_slice)
    pt = np.tile(np.arange(w.points_per_slice, dtype=np.int64), n_slices_sample)
    t = time.perf_counter()
    oracle.table_entries(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices, g,
                         w.steps_per_slice, sl, pt)
    dt = time.perf_counter() - t
    steps = sl.size * w.steps_per_slice
    return {"value": steps / dt, "unit": "trajectory-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"slices 0..{n_slices_sample - 1} of {w.name}: "
                      f"{sl.size} trajectories x {w.steps_per_slice} steps "
                      f"({steps:.3g} trajectory-steps, {dt:.1f} s, FP64, one thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="forced_cubic", choices=sorted(WORKLOADS))
    ap.add_argument("--traj-per-lane", type=int, default=0)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default=None,
                    help="override the workload's build precision")
    ap.add_argument("--compensated", type=int, default=1, choices=[0, 1, 2],
                    help="FP32 state accumulation: 0 plain, 1 Kahan, 2 blocked summation")
    ap.add_argument("--two-phase", action="store_true",
                    help="time nv_build_propagators + nv_compose instead of nv_solve")
    ap.add_argument("--solve-chunks", type=int, default=0)
    ap.add_argument("--cpu-slices", type=int, default=32,
                    help="slices of the workload the CPU oracle baseline integrates")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one elementwise copy kernel (reads and writes this many "
                         "MiB) so that profiler byte counters can be scaled against it")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the build shards "
              "by contiguous slice blocks with no communication, which this one-GPU "
              "benchmark does not exercise", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1304_6514_amd import nv
    from paper_1304_6514_amd.propagator import Propagator

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    nv.load()
    w = WORKLOADS[args.workload]
    if args.precision:
        w = w.with_(precision=args.precision)
    dev = torch.device("cuda:0")
    prop = Propagator(dev, traj_per_lane=args.traj_per_lane, compensated=args.compensated,
                      solve_chunks=args.solve_chunks)

    def step():
        if args.two_phase:
            prop.build(w)
            r = prop.compose()
        else:
            r = prop.solve(w)
        if r.status != nv.NV_OK:
            raise RuntimeError(f"composition failed: {nv.status_name(r.status)}")
        return r

    if args.calibrate_copy_mib > 0:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        flush = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        flush.fill_(1)                      # evict x from the 256 MB last-level cache
        torch.cuda.synchronize()
        torch.add(x, 0.0, out=y)            # reads n*4 bytes, writes n*4 bytes
        torch.cuda.synchronize()
        del x, y, flush

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps

    # kernel durations (HIP events on the library's stream), same workload
    prop.set_timing(True)
    build_ms, compose_ms = [], []
    for _ in range(args.steps):
        rr = step()
        b, c = prop.last_timing()
        build_ms.append(b)
        compose_ms.append(c)
    prop.set_timing(False)
    launches = rr.n_chunks if not args.two_phase else 1
    avg_build_ms = sum(build_ms) / len(build_ms)          # all build launches of a step
    avg_compose_ms = sum(compose_ms) / len(compose_ms)

    steps_per_launch = w.trajectory_steps / launches
    fps = flops_per_step(w, compensated=args.compensated != 0)
    if w.precision == "fp32" and args.compensated == 2:
        fps = flops_per_step(w, compensated=False) + w.dim   # one extra add per component
    achieved_tflops = w.trajectory_steps * fps / (avg_build_ms * 1e-3) / 1e12
    peak = PEAK_FP64_VECTOR_TFLOPS if w.precision == "fp64" else PEAK_FP32_VECTOR_TFLOPS
    roofline = {
        "bound": "alu", "achieved": round(achieved_tflops, 3), "peak": peak,
        "unit": "TFLOP/s", "frac": round(achieved_tflops / peak, 4), "traffic": None,
        "kernel": "build_kernel (ensemble RK4 integration + table write)",
        "kernel_ms": round(avg_build_ms / launches, 4),
        "launches_per_step": launches,
        "flops_per_trajectory_step": fps,
        "trajectory_steps_per_launch": steps_per_launch,
    }

    value = w.trajectory_steps * args.steps / elapsed
    out = {
        "metric": "trajectory-steps/s in propagator build; time-to-y(T) vs serial at fixed error",
        "value": value,
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "rhs": w.rhs, "n_slices": w.n_slices,
                   "points_per_slice": w.points_per_slice,
                   "steps_per_slice": w.steps_per_slice, "interp": w.interp,
                   "compose": "fp64", "parallelism": "single-gpu"},
        "build_kernel_trajectory_steps_per_s": w.trajectory_steps / (avg_build_ms * 1e-3),
        "mode": "two-phase" if args.two_phase else "solve",
        "accumulation": ["plain", "kahan", "blocked"][args.compensated]
        if w.precision == "fp32" else "fp64",
        "compose_exposed_ms" if not args.two_phase else "compose_ms": round(avg_compose_ms, 4),
        "yT": float(r.yT[0]),
        "tau_N_us": None,
        "roofline": roofline,
    }
    # tau_N: the composition alone (one launch over all slices), HIP events
    prop.set_timing(True)
    prop.build(w)
    taus = []
    for _ in range(3):
        prop.compose()
        taus.append(prop.last_timing()[1])
    prop.set_timing(False)
    out["compose_alone_ms"] = round(min(taus), 4)
    out["tau_N_us"] = round(1e3 * min(taus) / w.n_slices, 4)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, min(args.cpu_slices, w.n_slices))
    prop.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
