#!/usr/bin/env python3
"""Benchmark: trajectory-steps/s of the Nievergelt propagator build on one GPU.

One step = one pass of the whole hot path over the forced-cubic workload
(y' = sin 3t - y^3 on [0, 100], 4096 slices x 4096 grid points x 2000 RK4
steps, FP32 build with blocked summation of the state, FP64 cubic-Hermite
composition):
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
# the variational term df/dy * v of a 1-D right-hand side, given the value's own
# intermediates (y^2 of the cubic): p v; (1 - 2 y) v; (-3 y^2) v; (2 y) v
TANGENT_FLOPS = {"linear": 1, "logistic": 3, "forced_cubic": 2, "square": 2}

WORKLOADS = {"forced_cubic": W.FORCED_CUBIC_FP32, "logistic": W.LOGISTIC_FP64,
             "vdp": W.VDP_FP32}

# HBM bytes per timed step of the build launches, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (raw counters, summed over the step's build dispatches; the
# profile files under profiles/ give the commands).  Keyed by workload,
# accumulation, mode, build launches per step and the SHA-1 of the kernel
# sources and build flags they were taken with; any other source gives
# traffic = null.
MEASURED_TRAFFIC = {
    ("forced-cubic-fp32-4096sl-4096pt-2000st", "blocked", "solve", 32,
     "fee9a34e4dc49e22641d8dc8c2681de47a273c25"): (65152.0 + 65664.0) * 1024,
    ("forced-cubic-fp32-4096sl-4096pt-2000st-hermite_slopes", "blocked", "solve", 32,
     "fee9a34e4dc49e22641d8dc8c2681de47a273c25"): (65520.0 + 131200.0) * 1024,
}

# builds too small to fill the chip (one wave per SIMD): per RK4 step, the FP64
# VALU instructions of the compiled loop and the dependent operations on its
# critical path (FP64 logistic: k1..k4 as fma(-u, u, u), three stage values,
# four FMAs adding the weighted stages into the state, the last after k4)
SINGLE_WAVE_STEP = {"logistic-fp64-64sl-256pt-1000st": {"valu": 11, "dependent": 8}}

KERNEL_SOURCES = [os.path.join(ROOT, "paper_1304_6514_amd", f)
                  for f in ("csrc/integrate.h", "csrc/build_kernels.hip", "_build.py")]


def kernel_source_sha1() -> str:
    import hashlib
    h = hashlib.sha1()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def algorithmic_bytes(w: W.Workload) -> float:
    """Table write plus the per-slice forcing rows read (non-autonomous only)."""
    elem = 4 if w.precision == "fp32" else 8
    comps = w.dim + (1 if w.interp == "hermite_slopes" else 0)     # the slope table
    tables = comps * w.n_slices * w.points_per_slice * elem
    forcing = (2 * w.steps_per_slice + 1) * w.n_slices * elem if w.rhs == "forced_cubic" else 0
    return float(tables + forcing)


def flops_per_step(w: W.Workload, compensated: bool) -> int:
    """Algorithmic FLOPs of one trajectory-step: the scheme's stage and
    combination arithmetic per state component plus its right-hand side
    evaluations; with stored slopes, the same for the derivative v."""
    comps = w.dim + (1 if w.interp == "hermite_slopes" else 0)
    if w.scheme == "rk4":
        f = 12 * comps + 4 * RHS_FLOPS[w.rhs]
        if w.interp == "hermite_slopes":
            f += 4 * TANGENT_FLOPS[w.rhs]
    else:
        f = 2 * comps + RHS_FLOPS[w.rhs]
        if w.interp == "hermite_slopes":
            f += TANGENT_FLOPS[w.rhs]
    if w.precision == "fp32" and compensated:
        f += 3 * comps
    return f


def host_description():
    """nproc, the CPUs this process may run on, and the CPU model name."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": os.cpu_count(), "usable_cpus": usable, "model": model}


def cpu_threads(host) -> int:
    """Host threads for the CPU baselines: every usable CPU, at most 16 (the
    host share of one GPU)."""
    return max(1, min(16, int(host["usable_cpus"] or 1)))


def cpu_baseline(w: W.Workload, threads: int, steps_per_thread: float = 1.5e8):
    """The oracle as it is (plain serial C, FP64) on `threads` host threads at
    once, each integrating its own whole slices of w (ctypes releases the
    interpreter lock during each call): a bounded sample of the workload."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    import oracle

    oracle._load()
    g = oracle.make_grid(w.grid_n, w.grid_lo, w.grid_hi)
    per_slice = w.points_per_slice * w.steps_per_slice
    per_thread = int(max(1, min(w.n_slices // threads, round(steps_per_thread / per_slice))))
    per_thread = max(per_thread, 1)
    threads = min(threads, w.n_slices)

    def run(i):
        sl = np.repeat(np.arange(i * per_thread, (i + 1) * per_thread, dtype=np.int64),
                       w.points_per_slice)
        pt = np.tile(np.arange(w.points_per_slice, dtype=np.int64), per_thread)
        entries = (oracle.table_entries_slopes if w.interp == "hermite_slopes"
                   else oracle.table_entries)
        entries(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices, g, w.steps_per_slice, sl, pt)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        t = time.perf_counter()
        list(ex.map(run, range(threads)))
        dt = time.perf_counter() - t
    steps = threads * per_thread * per_slice
    return {"value": steps / dt, "unit": "trajectory-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": f"slices 0..{threads * per_thread - 1} of {w.name} "
                      f"({threads} threads x {per_thread} slices, {steps:.3g} "
                      f"trajectory-steps, {dt:.1f} s, FP64 serial oracle per thread)"}


def cpu_parallel_build(w: W.Workload, threads: int, slices_per_thread: int = 64):
    """The CPU throughput baseline of the table build (OpenMP over `threads`
    host threads, forcing hoisted per slice, vectorised over trajectories) in
    FP64 and FP32 on a bounded number of the workload's slices."""
    import oracle

    if w.interp == "hermite_slopes":
        return {"what": "not built: the OpenMP CPU build integrates values only"}
    ns = min(w.n_slices, threads * slices_per_thread)
    out = {"threads": threads, "slices": ns,
           "what": "table build of the first slices, OpenMP over host threads, 64 "
                   "trajectories per vectorised block; FP64 = the oracle's operations, FP32 "
                   "with blocked summation"}
    for prec in ("fp64", "fp32"):
        oracle.cpu_build(w.rhs, w.params, w.t0, w.T, w.n_slices, w.grid_n, w.grid_lo,
                         w.grid_hi, w.steps_per_slice, prec, slices=(0, min(ns, threads)),
                         threads=threads)                       # warm-up
        # repeated until 0.3 s have passed (small workloads take milliseconds)
        reps, t = 0, time.perf_counter()
        while reps == 0 or time.perf_counter() - t < 0.3:
            oracle.cpu_build(w.rhs, w.params, w.t0, w.T, w.n_slices, w.grid_n, w.grid_lo,
                             w.grid_hi, w.steps_per_slice, prec, slices=(0, ns), threads=threads)
            reps += 1
        dt = (time.perf_counter() - t) / reps
        out[prec] = {"trajectory_steps_per_s": ns * w.points_per_slice * w.steps_per_slice / dt,
                     "s_per_build": round(dt, 4), "repetitions": reps}
    return out


def method_equal_error(prop, w: W.Workload, ref, target):
    """The method's own cheapest configuration of the same problem (same
    right-hand side, interval, initial value, grid range and interpolation)
    whose error at T is no larger than ``target``: slice counts, grid sizes
    and steps per slice from small to the fixed configuration's, each run once
    through nv_solve for its error, and those meeting the target timed (best of
    three whole solves, host clock, synchronized)."""
    import numpy as np
    import torch

    from paper_1304_6514_amd import nv

    tried, meeting, best = 0, 0, None
    # grids: 1-D point counts, or square 2-D grids on the same box
    grids = ([(M,) for M in (256, 512, 1024, 2048, 4096)] if w.dim == 1 else
             [(n, n) for n in (16, 32, 64, 128)])
    for N in (8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096):
        for gn in grids:
            for S in (10, 20, 50, 100, 200, 500):
                M = int(np.prod(gn))
                if N > w.n_slices or M > w.points_per_slice or S > w.steps_per_slice:
                    continue
                c = w.with_(name=f"{w.name}-eq-{N}x{'x'.join(map(str, gn))}x{S}", n_slices=N,
                            grid_n=gn, steps_per_slice=S)
                tried += 1
                r = prop.solve(c)
                if r.status != nv.NV_OK:
                    continue
                e = float(np.max(np.abs(np.asarray(r.yT) - ref)))
                if not (e <= target):
                    continue
                meeting += 1
                ts = []
                for _ in range(3):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    prop.solve(c)
                    torch.cuda.synchronize()
                    ts.append(time.perf_counter() - t)
                ms = 1e3 * min(ts)
                if best is None or ms < best["gpu_ms"]:
                    best = {"n_slices": N, "grid": list(gn), "points_per_slice": M,
                            "steps_per_slice": S,
                            "error": e, "gpu_ms": round(ms, 4),
                            "trajectory_steps": N * M * S}
    return {"configs_tried": tried, "configs_meeting_error": meeting, "fastest": best}


def fixed_error(w: W.Workload, yT_method, gpu_ms, prop=None):
    """Time-to-y(T) of the method on the GPU against the serial oracle on one
    host core: at the method's own step (N*S steps) and at equal error (the
    fewest serial steps whose error at T is no larger than the method's); with
    ``prop``, also the method's own cheapest configuration at that error."""
    import numpy as np
    import oracle

    oracle._load()
    S_ref = 4 * w.n_slices * w.steps_per_slice
    ref = oracle.serial_steps(w.rhs, w.params, w.scheme, w.t0, w.T, S_ref, w.y0)
    method_err = float(np.max(np.abs(np.asarray(yT_method) - ref)))
    n_same = w.n_slices * w.steps_per_slice
    t = time.perf_counter()
    oracle.serial_steps(w.rhs, w.params, w.scheme, w.t0, w.T, n_same, w.y0)
    t_same = time.perf_counter() - t

    def err(n):
        e = np.abs(oracle.serial_steps(w.rhs, w.params, w.scheme, w.t0, w.T, n, w.y0) - ref)
        return float(np.max(e)) if np.all(np.isfinite(e)) else float("inf")

    # geometric grid of step counts; the answer is the first count from which
    # the next three grid points also meet the method's error (so that a lucky
    # zero crossing of the error does not count)
    grid, n = [], 8
    while n < n_same:
        grid.append(n)
        n = max(n + 1, int(n * 1.1))
    grid.append(n_same)
    ok = [None] * len(grid)
    hi = n_same
    for i in range(len(grid)):
        ok[i] = err(grid[i]) <= method_err
        if i >= 3 and all(ok[i - 3:i + 1]):
            hi = grid[i - 3]
            break
    t = time.perf_counter()
    reps = 0
    while time.perf_counter() - t < 0.2:
        oracle.serial_steps(w.rhs, w.params, w.scheme, w.t0, w.T, hi, w.y0)
        reps += 1
    t_eq = (time.perf_counter() - t) / reps
    out = {"method_error_at_T": method_err, "reference": f"serial RK4, {S_ref} steps",
           "gpu_time_to_yT_ms": gpu_ms,
           "serial_same_step": {"steps": n_same, "ms": round(1e3 * t_same, 3)},
           "serial_equal_error": {"steps": hi, "error": err(hi), "ms": round(1e3 * t_eq, 4)},
           "cores": 1}
    if prop is not None:
        out["method_equal_error"] = method_equal_error(prop, w, ref, method_err)
    return out


def bench_batched(args):
    """96 seeded uneven problems in one persistent, graph-captured launch,
    against the plain form (each problem alone through nv_solve)."""
    import numpy as np
    import torch

    from paper_1304_6514_amd import nv
    from paper_1304_6514_amd.propagator import Batch, Propagator

    probs = W.batched_problems()
    total_steps = sum(w.trajectory_steps for w in probs)
    flops = sum(w.trajectory_steps * flops_per_step(w, compensated=False) for w in probs)
    b = Batch(probs)
    t = time.perf_counter()
    sched = b.autotune(reps=2)
    tune_s = time.perf_counter() - t
    for _ in range(args.warmup):
        b.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st, yT, _ = b.run()
        if st != nv.NV_OK:
            raise RuntimeError(f"batch failed: {nv.status_name(st)}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    run_ms, _ = b.last_timing()
    b.close()

    # the plain form: the same problems one after another, same options
    plain_y = []
    with Propagator("cuda:0") as p:
        for w in probs:                      # warm-up of every shape
            p.solve(w, want_boundary=False)
        # best of three timed passes: a single pass has been seen to catch a
        # one-off stall of ~30 ms on the host side
        plain_s = float("inf")
        for rep in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ys = []
            for w in probs:
                r = p.solve(w, want_boundary=False)
                ys.append(r.yT)
            torch.cuda.synchronize()
            plain_s = min(plain_s, time.perf_counter() - t1)
            if rep == 0:
                plain_y = ys
    same = all(np.array_equal(yT[i, :w.dim], plain_y[i]) for i, w in enumerate(probs))

    ms = 1e3 * elapsed / args.steps
    achieved = flops / (ms * 1e-3) / 1e12
    return {
        "metric": "trajectory-steps/s in propagator build; time-to-y(T) vs serial at fixed error",
        "value": total_steps * args.steps / elapsed, "unit": "trajectory-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched-96-uneven-seed3", "problems": len(probs),
                   "trajectory_steps": total_steps, "interp": "linear/bilinear",
                   "compose": "fp64", "parallelism": "single-gpu"},
        "graph_run_ms": round(run_ms, 4),
        "schedule": {"traj_per_lane": list(sched.traj_per_lane),
                     "workgroups_per_cu": sched.workgroups_per_cu,
                     "order": ["longest-first", "natural"][sched.order],
                     "autotune_s": round(tune_s, 2)},
        "plain_form": {"value": total_steps / plain_s, "ms": round(1e3 * plain_s, 3),
                       "what": "each problem alone through nv_solve, same options; best of "
                               "three timed passes",
                       "identical_results": bool(same)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3),
                     "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_VECTOR_TFLOPS, 4), "traffic": None,
                     "kernel": "whole batched step (persistent build + compositions + copy)",
                     "flops_per_step_total": flops},
    }


def bench_paper_table3(args):
    """The nine shapes of the paper's Table 3 (sec. 4): y' = y^2 on [0, 1/2],
    backward Euler with step dt, M Chebyshev nodes, N slices, single precision.
    Time to solution of nv_solve (buffers already allocated), the serial CPU
    oracle at the same dt, and a least-squares fit of the cost model."""
    import numpy as np
    import torch

    from paper_1304_6514_amd import costmodel
    from paper_1304_6514_amd import nv
    from paper_1304_6514_amd.propagator import Propagator

    # the paper's Table 3 rows: (T_total microseconds, speedup), Tesla C2075
    printed = {(2.0 ** -14, 32): 193.6, (2.0 ** -14, 64): 187.5, (2.0 ** -14, 128): 208.4,
               (2.0 ** -15, 32): 253.7, (2.0 ** -15, 64): 228.5, (2.0 ** -15, 128): 257.8,
               (2.0 ** -16, 32): 388.3, (2.0 ** -16, 64): 338.9, (2.0 ** -16, 128): 392.0}
    rows, fit_rows = [], []
    ours_steps = ours_time = paper_time = 0.0
    with Propagator("cuda:0") as p:
        for dt, N, M in W.PAPER_TABLE3:
            w = W.paper_model(N, M, dt, "fp32")
            p.set_timing(True)
            kb, kc = [], []
            for _ in range(max(3, args.warmup)):
                p.solve(w)
                b_ms, c_ms = p.last_timing()
                kb.append(b_ms)
                kc.append(c_ms)
            p.set_timing(False)
            reps = max(20, args.steps)
            torch.cuda.synchronize()
            times = []
            for _ in range(reps):
                t = time.perf_counter()
                r = p.solve(w)
                times.append(time.perf_counter() - t)
            if r.status != nv.NV_OK:
                raise RuntimeError("paper-mode solve failed")
            t_us = 1e6 * float(np.median(times))
            n = round(0.5 / dt)
            rows.append({"dt": dt, "N": N, "M": M, "T_total_us": round(t_us, 2),
                         "build_kernel_us": round(1e3 * min(kb), 2),
                         "compose_kernel_us": round(1e3 * min(kc), 2),
                         "error": abs(float(r.yT[0]) - 2.0),
                         "paper_T_total_us": printed[(dt, N)],
                         "trajectory_steps_per_s": M * n / (t_us * 1e-6)})
            fit_rows.append((M, n, N, t_us))
            ours_steps += M * n
            ours_time += t_us
            paper_time += printed[(dt, N)]
    tau_F, tau_N, tau_K = costmodel.fit(fit_rows)
    out = {
        "metric": "trajectory-steps/s in propagator build; time-to-y(T) vs serial at fixed error",
        "value": ours_steps / (ours_time * 1e-6), "unit": "trajectory-steps/s", "n_gpus": 1,
        "steps": max(20, args.steps), "warmup": max(3, args.warmup),
        "ms_per_step": round(ours_time / 1e3 / len(rows), 4), "higher_is_better": True,
        "scaling": "weak", "dtype": "f32", "data": "synthetic",
        "vs_baseline": round((ours_steps / ours_time) / (ours_steps / paper_time), 3),
        "vs_baseline_note": "against the trajectory-steps/s derived from the paper's Table 3 "
                            "(Tesla C2075 + Opteron, same nine shapes)",
        "config": {"workload": "paper-table3-square-be-chebyshev", "shapes": len(rows),
                   "parallelism": "single-gpu"},
        "rows": rows,
        "cost_model_fit_us": {"tau_F": tau_F, "tau_N": tau_N, "tau_K": tau_K},
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle._load()
        for row in rows:
            t = time.perf_counter()
            reps = 0
            while time.perf_counter() - t < 0.05:
                oracle.paper_serial(0.5, row["dt"], 1.0)
                reps += 1
            t_cpu = (time.perf_counter() - t) / reps * 1e6
            row["serial_cpu_us"] = round(t_cpu, 2)
            row["speedup_vs_serial"] = round(t_cpu / row["T_total_us"], 3)
        out["cpu_baseline"] = {"value": sum(0.5 / r["dt"] for r in rows) /
                               (1e-6 * sum(r["serial_cpu_us"] for r in rows)),
                               "unit": "time-steps/s", "cores": 1, "kind": "oracle",
                               "sample": "serial backward Euler of y' = y^2 over [0, 1/2] at "
                                         "each of the nine dt (FP64, one thread)"}
    return out


# algorithmic FLOPs per training sample of the surrogate network (FMA = 2):
# forward 2 (4*128 + 2*128*128 + 128*2) = 67,072; back-propagation through the
# two 128 x 128 layers 2 * 2 * 128*128; weight gradients 2 (128*4 + 2*128*128
# + 2*128); the matrix-core part is the three 128 x 128 products of each layer
SUR_FWD_FLOPS = 2 * (4 * 128 + 2 * 128 * 128 + 128 * 2)
SUR_TRAIN_FLOPS = SUR_FWD_FLOPS + 2 * 2 * 128 * 128 + 2 * (128 * 4 + 2 * 128 * 128 + 2 * 128)
SUR_MFMA_FLOPS = 3 * 2 * 2 * 128 * 128
PEAK_BF16_MFMA_TFLOPS = 2500.0


def bench_surrogate(args):
    """The learned slice-map surrogate of the Van der Pol problem: the training
    build (1024 one-slice problems, slice j with its own mu_j, 128 x 128 grid,
    500 RK4 steps: 16.7M endpoints), the training-set gather, Adam training on
    the matrix cores, then the composition with the network for held-out mu
    against the plain method (bilinear tables) at equal max final-state error."""
    import numpy as np
    import torch

    from paper_1304_6514_amd import nv
    from paper_1304_6514_amd.propagator import Batch, Propagator
    from paper_1304_6514_amd.surrogate import Surrogate

    B = 65536
    probs = W.surrogate_training_problems()
    b = Batch(probs)
    st, _, _ = b.run()                       # first run: graph capture and warm-up
    st, _, _ = b.run()
    if st != nv.NV_OK:
        raise RuntimeError(f"training build failed: {nv.status_name(st)}")
    build_ms, build_steps = b.last_timing()
    coarse = args.sur_coarse
    base = W.VDP_FP32
    # the step-doubling form: phi ~ G1 + d (16/15 + out_scale g out)
    sur = Surrogate("cuda:0", max_batch=B, coarse_steps=coarse, correction="step-doubling",
                    out_scale=W.SUR_SD_OUT_SCALE, gate=W.SUR_SD_GATE,
                    loss_scale=W.SUR_SD_LOSS_SCALE)
    # visit weights: the states Richardson chains (the untrained form) visit
    mug = np.linspace(1.0, 5.0, W.SUR_VISIT_MUS)
    t = time.perf_counter()
    st, _, vis, _ = sur.compose(np.tile(base.y0, (len(mug), 1)), mug, base.t0, base.T,
                                base.n_slices, want_boundary=True)
    visit_ms = 1e3 * (time.perf_counter() - t)
    sur.set_visits(vis, 1.0, 5.0, W.SUR_VISIT_SIGMA, W.SUR_VISIT_FLOOR)
    total = nv.nv_sur_dataset_from_batch(sur.h, b.batch)
    perm = W.surrogate_perm(total)
    t = time.perf_counter()
    x, tg = sur.dataset_from_batch(b, perm)
    gather_ms = 1e3 * (time.perf_counter() - t)
    b.close()
    del perm

    steps_per_epoch = total // B
    steps = args.sur_epochs * steps_per_epoch
    sur.set_params(W.surrogate_init_params(0))
    sur.train(x, tg, batch=B, steps=args.warmup)           # warm-up (then start afresh)
    sur.set_params(W.surrogate_init_params(0))
    torch.cuda.synchronize()
    t = time.perf_counter()
    losses = sur.train(x, tg, batch=B, steps=steps, lr=args.sur_lr, lr_final=args.sur_lr_final)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t
    train_ms_events = sur.last_ms()
    losses = losses.cpu().numpy()
    del x, tg

    # the kernels of one training step, timed alone (HIP events inside the call)
    xs, ts = W.surrogate_samples(B, seed=31)
    ts = np.concatenate([ts, np.ones_like(ts)])      # rho, and unit weights
    sur.loss_grad(xs, ts)
    step_ms = []
    xd = torch.from_numpy(xs).cuda()
    td = torch.from_numpy(ts).cuda()
    for _ in range(5):
        t1 = time.perf_counter()
        sur.loss_grad(xd, td)
        step_ms.append(1e3 * (time.perf_counter() - t1))

    if args.sur_train_only:
        sur.close()
        return {"what": "surrogate training only", "steps": steps,
                "train_s": round(train_s, 4), "samples_per_s": steps * B / train_s,
                "step_ms_loss_grad": round(min(step_ms), 4),
                "loss_last": float(losses[-1])}

    # evaluation on held-out mu: truth = the library's FP64 integration of the
    # whole interval from y0 (a one-slice build whose first grid point is y0)
    mus = W.surrogate_eval_mus(8)
    truth = []
    with Propagator("cuda:0") as pr:
        for mu in mus:
            wt = base.with_(name="vdp-serial-fp64", params=(float(mu),), n_slices=1,
                            grid_n=(2, 2), grid_lo=base.y0, grid_hi=(base.y0[0] + 1.0,
                                                                    base.y0[1] + 1.0),
                            steps_per_slice=base.n_slices * base.steps_per_slice,
                            precision="fp64")
            pr.build(wt)
            torch.cuda.synchronize()
            truth.append([float(pr.table(0)[0, 0]), float(pr.table(1)[0, 0])])
    truth = np.array(truth)

    y0 = np.tile(base.y0, (len(mus), 1))
    sur.compose(y0, mus, base.t0, base.T, base.n_slices)          # warm-up
    st, fin, _, info = sur.compose(y0, mus, base.t0, base.T, base.n_slices)
    sur_ms = info.ms
    err_sur = np.max(np.abs(fin.cpu().numpy() - truth), axis=1)
    trained = sur.params()
    off = trained.copy()
    off[-258:] = 0.0                          # W4 = 0, b4 = 0: Richardson alone
    sur.set_params(off)
    _, fin0, _, _ = sur.compose(y0, mus, base.t0, base.T, base.n_slices)
    err_rich = np.max(np.abs(fin0.cpu().numpy() - truth), axis=1)
    sur.set_params(trained)
    with Surrogate("cuda:0", max_batch=16, coarse_steps=coarse) as g1:   # zero network: G1
        _, fin1, _, _ = g1.compose(y0, mus, base.t0, base.T, base.n_slices)
        err_coarse = np.max(np.abs(fin1.cpu().numpy() - truth), axis=1)
    st1, _, _, info1 = sur.compose(y0[:1], mus[:1], base.t0, base.T, base.n_slices)
    many = 16384
    stq, _, _, infoq = sur.compose(np.tile(base.y0, (many, 1)), np.resize(mus, many), base.t0,
                                   base.T, base.n_slices)

    plain = []
    with Propagator("cuda:0") as pr:
        for n in (32, 48, 64, 96, 128, 192, 256):
            errs, ms = [], []
            for mu in mus:
                wp = base.with_(params=(float(mu),), grid_n=(n, n))
                pr.solve(wp, want_boundary=False)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                r = pr.solve(wp, want_boundary=False)
                ms.append(1e3 * (time.perf_counter() - t1))
                errs.append(float(np.max(np.abs(np.asarray(r.yT) - truth[len(errs)]))))
            plain.append({"grid": n, "max_error": max(errs), "errors": errs,
                          "ms_per_mu": round(float(np.mean(ms)), 3),
                          "table_bytes": base.n_slices * n * n * 2 * 4})
        # the network with the 128 x 128 table of the first mu as fallback and check
        wf = base.with_(params=(float(mus[0]),))
        pr.build(wf)
        torch.cuda.synchronize()
        stf, finf, _, infof = sur.compose(base.y0, [mus[0]], base.t0, base.T, base.n_slices,
                                          fallback=pr, guard=args.sur_guard)
        err_fb = float(np.max(np.abs(finf.cpu().numpy()[0] - truth[0])))

    e_sur = float(np.max(err_sur))
    eq = next((p for p in plain if p["max_error"] <= e_sur), None)
    train_samples = steps * B
    value = train_samples / train_s
    achieved = train_samples * SUR_MFMA_FLOPS / train_s / 1e12
    out = {
        "metric": "surrogate: training samples/s; composition at equal max final-state error",
        "value": value, "unit": "samples/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * train_s / max(steps, 1), 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "vdp-surrogate-1024x128x128x500-perslice-mu",
                   "network": "4-128-128-128-2 exact GELU", "batch": B, "epochs": args.sur_epochs,
                   "form": "step-doubling (G1 + d (16/15 + s g out)), visit-weighted loss",
                   "coarse_rk4_steps": coarse,
                   "samples": total, "lr": [args.sur_lr, args.sur_lr_final],
                   "parallelism": "single-gpu"},
        "training_build": {"ms": round(build_ms, 3), "trajectory_steps": build_steps,
                           "trajectory_steps_per_s": build_steps / (build_ms * 1e-3)},
        "gather_ms": round(gather_ms, 3), "visit_chains_ms": round(visit_ms, 3),
        "train_s": round(train_s, 3), "train_events_ms": round(train_ms_events, 2),
        "loss": {"first": float(losses[0]), "last": float(losses[-1]),
                 "last_epoch_mean": float(losses[-steps_per_epoch:].mean())},
        "step_ms_loss_grad": round(min(step_ms), 4),
        "eval": {"mus": [float(m) for m in mus], "truth": "library FP64 serial RK4, 512000 steps",
                 "surrogate_errors": [float(e) for e in err_sur], "surrogate_max_error": e_sur,
                 "richardson_alone_errors": [float(e) for e in err_rich],
                 "richardson_alone_max_error": float(np.max(err_rich)),
                 "coarse_alone_errors": [float(e) for e in err_coarse],
                 "coarse_alone_max_error": float(np.max(err_coarse)),
                 "surrogate_compose_ms_8_chains": round(sur_ms, 3),
                 "surrogate_compose_ms_1_chain": round(info1.ms, 3),
                 "surrogate_compose_ms_16384_chains": round(infoq.ms, 3),
                 "plain": plain,
                 "equal_error_grid": eq["grid"] if eq else None,
                 "equal_error_plain_ms_per_mu": eq["ms_per_mu"] if eq else None,
                 "with_fallback": {"guard": args.sur_guard, "n_fallback": infof.n_fallback,
                                   "max_deviation": infof.max_deviation, "error": err_fb},
                 "network_bytes_bf16": 33922 * 2},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3),
                     "peak": PEAK_BF16_MFMA_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_BF16_MFMA_TFLOPS, 5), "traffic": None,
                     "kernel": "whole training step (forward/back-propagation, gradient sums, "
                               "Adam); matrix-core FLOPs only",
                     "mfma_flops_per_sample": SUR_MFMA_FLOPS,
                     "train_flops_per_sample": SUR_TRAIN_FLOPS},
    }
    sur.close()
    return out


# Sec. 6, Tables 5, 7 and 8: the heat equation on [0, 10] with backward Euler,
# the largest slice count of each table, and the paper's cluster timings at
# that count and at one processor (seconds; context, other hardware).
HEAT_SHAPES = [  # (dx, dt, N, paper T_total at N, paper serial T_total)
    (0.1, 0.005, 128, 0.01763, 0.2870),
    (0.05, 0.001, 256, 0.0984, 1.641),
    (0.01, 0.0005, 1024, 1.595, 16.166),
]


def bench_heat(args):
    """The affine basis propagator on the three heat-equation shapes of sec. 6:
    time to y(T) of build + composition on the GPU (buffers allocated by a
    warm-up build), against serial backward Euler on one host core (the CPU
    oracle) and the paper's cluster timings as context."""
    import numpy as np

    from paper_1304_6514_amd.linear import HeatWorkload, LinearPropagator

    rows = []
    with LinearPropagator() as lp:
        for dx, dt, N, paper_t, paper_serial in HEAT_SHAPES:
            M = int(round(1.0 / dx)) - 1
            w = HeatWorkload(f"heat-M{M}-dt{dt:g}-N{N}", M, dt, N)
            y0 = np.sin(np.pi * dx * np.arange(1, M + 1))
            lp.build(w)
            lp.compose(y0, want_boundary=False)
            ts, bk, ck = [], [], []
            for _ in range(max(args.steps, 1)):
                t = time.perf_counter()
                lp.build(w)
                st, yT, _ = lp.compose(y0, want_boundary=False)
                ts.append(time.perf_counter() - t)
                b, c = lp.last_timing()
                bk.append(b)
                ck.append(c)
            L = 10.0 / N
            S = int(np.floor(L / dt + 1e-9))
            s_tot = S + (1 if L - S * dt > 1e-12 * L else 0)
            solve_steps = N * s_tot * (M + 1)
            err = float(np.max(np.abs(yT - np.cos(10.0) * y0)))
            rows.append({"shape": w.name, "M": M, "dt": dt, "N": N, "steps_per_slice": s_tot,
                         "T_total_us": round(1e6 * min(ts), 2),
                         "build_kernels_ms": round(min(bk), 4),
                         "compose_kernel_ms": round(min(ck), 4),
                         "tau_N_us": round(1e3 * min(ck) / N, 4),
                         "solve_steps": solve_steps,
                         "error_vs_closed_form": err,
                         "paper_T_total_s": paper_t, "paper_serial_s": paper_serial})
        # many initial values at once on the matrix cores (the last shape's tables)
        import torch
        M, N = rows[-1]["M"], rows[-1]["N"]
        single_ms = rows[-1]["compose_kernel_ms"]
        many = []
        rng = np.random.default_rng(3)
        for Q in (1, 16, 256, 1024, 4096, 16384):
            y0q = torch.from_numpy(rng.normal(0.0, 1.0, (Q, M))).cuda()
            lp.compose_many(y0q)                                   # warm-up
            ms = []
            for _ in range(3):
                st, _, _ = lp.compose_many(y0q)
                ms.append(lp.last_timing()[1])
            best = min(ms)
            flops = 2.0 * M * M * Q * N
            tf = flops / (best * 1e-3) / 1e12
            many.append({"Q": Q, "kernel_ms": round(best, 4), "chains_per_s": Q / (best * 1e-3),
                         "fp64_tflops": round(tf, 3),
                         "frac_fp64_peak": round(tf / PEAK_FP64_VECTOR_TFLOPS, 4),
                         "single_chains_ms": round(Q * single_ms, 3),
                         "gain_over_single_chains": round(Q * single_ms / best, 2)})
            del y0q
    big = rows[-1]
    out = {
        "metric": "affine basis propagator (heat equation): backward-Euler solve-steps/s, "
                  "time to y(T)",
        "value": big["solve_steps"] / (big["T_total_us"] * 1e-6), "unit": "solve-steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": round(big["T_total_us"] / 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "heat-sec6-tables-5-7-8", "parallelism": "single-gpu"},
        "rows": rows,
        "many_initial_values": {
            "what": f"nv_lin_compose_many on the M = {M}, N = {N} tables: Q chains as FP64 "
                    "matrix products (v_mfma_f64_16x16x4f64), 16 chains per workgroup; "
                    "FLOPs 2 M^2 Q N; single_chains_ms = Q x one nv_lin_compose",
            "runs": many},
        "vs_baseline_note": "the paper's heat timings are cluster runs (context only)",
    }
    if not args.no_cpu_baseline:
        from oracle import linear_oracle as lo
        dx, dt, N, _, _ = HEAT_SHAPES[0]
        M = int(round(1.0 / dx)) - 1
        t = time.perf_counter()
        lo.serial(M, 1.0, 0.25, True, 0.0, 10.0, N, dt, np.sin(np.pi * dx * np.arange(1, M + 1)))
        el = time.perf_counter() - t
        out["cpu_baseline"] = {"value": (10.0 / dt) / el, "unit": "BE steps/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"serial backward Euler, M = {M}, dt = {dt}, [0, 10] "
                                         f"({el:.2f} s, FP64, Python, one thread)"}
    return out


def end_to_end_cold(w: W.Workload, prop, repeats: int = 3):
    """The paper's T_total of the whole method: a fresh context whose nv_solve
    allocates its tables and scratch with hipMalloc, builds, composes, brings
    the boundary states to the host, then the context is destroyed (device
    memory freed); best of `repeats`, host clock, synchronized."""
    import torch

    from paper_1304_6514_amd import nv

    g = prop.grid(w)
    rhs = nv.RHS_IDS[w.rhs]
    ts = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t = time.perf_counter()
        ctx = nv.nv_ctx_create()
        try:
            nv.nv_set_options(ctx, prop.options(w))
            st, _, _, _ = nv.nv_solve(ctx, rhs, w.params, w.t0, w.T, w.n_slices, g,
                                      w.steps_per_slice, w.y0, w.dim, True)
        finally:
            nv.nv_ctx_destroy(ctx)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
        if st != nv.NV_OK:
            return {"status": nv.status_name(st)}
    return {"ms": round(1e3 * min(ts), 4),
            "what": "fresh context: nv_solve allocating tables and scratch (hipMalloc), "
                    "build, composition, boundary states to host, context destroyed "
                    "(device memory freed): the paper's end-to-end T_total"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="forced_cubic",
                    choices=sorted(WORKLOADS) + ["batched", "paper-table3", "surrogate", "heat"])
    ap.add_argument("--traj-per-lane", type=int, default=0)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default=None,
                    help="override the workload's build precision")
    ap.add_argument("--interp", choices=["linear", "hermite", "hermite_slopes"], default=None,
                    help="override the interpolation of a 1-D workload (hermite_slopes: the "
                         "build also stores each entry's slope)")
    ap.add_argument("--compensated", type=int, default=2, choices=[0, 1, 2],
                    help="FP32 state accumulation: 0 plain, 1 Kahan, 2 blocked summation")
    ap.add_argument("--two-phase", action="store_true",
                    help="time nv_build_propagators + nv_compose instead of nv_solve")
    ap.add_argument("--solve-chunks", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one elementwise copy kernel (reads and writes this many "
                         "MiB) so that profiler byte counters can be scaled against it")
    ap.add_argument("--sur-epochs", type=int, default=20,
                    help="surrogate: passes over the 16.7M-sample training set")
    ap.add_argument("--sur-lr", type=float, default=2e-3)
    ap.add_argument("--sur-lr-final", type=float, default=2e-5)
    ap.add_argument("--sur-coarse", type=int, default=1,
                    help="surrogate: RK4 steps of the coarse propagator the network corrects")
    ap.add_argument("--sur-train-only", action="store_true",
                    help="surrogate: stop after training (for profiling the training kernels)")
    ap.add_argument("--sur-guard", type=float, default=0.05,
                    help="surrogate: deviation from the table above which the table is used")
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
    if args.workload == "batched":
        print(json.dumps(bench_batched(args)), flush=True)
        return
    if args.workload == "paper-table3":
        print(json.dumps(bench_paper_table3(args)), flush=True)
        return
    if args.workload == "surrogate":
        print(json.dumps(bench_surrogate(args)), flush=True)
        return
    if args.workload == "heat":
        print(json.dumps(bench_heat(args)), flush=True)
        return
    w = WORKLOADS[args.workload]
    if args.precision:
        w = w.with_(precision=args.precision)
    if args.interp:
        if w.dim != 1:
            print(f"--interp applies to 1-D workloads; {w.name} is {w.dim}-D", file=sys.stderr)
            sys.exit(2)
        w = w.with_(interp=args.interp)
        if args.interp != WORKLOADS[args.workload].interp:
            w = w.with_(name=f"{w.name}-{args.interp}")
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

    # HIP events bracket the build launches of every step (in solve mode the
    # span from before the first chunk launch to after the last one, on the
    # stream they are launched on) and the composition
    prop.set_timing(True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K whole steps; each step's build span is read once the
    # step has returned (its events are complete by then)
    span_ms, exposed_ms = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = step()
        b, c = prop.last_timing()
        span_ms.append(b)
        exposed_ms.append(c)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1e3 * elapsed / args.steps
    launches = r.n_chunks if not args.two_phase else 1

    # for comparison: one launch of the integration kernel over the whole
    # workload, and one composition launch over all slices (tau_N)
    kern_ms, comp_ms = [], []
    for _ in range(args.steps):
        prop.build(w)
        prop.compose()
        b, c = prop.last_timing()
        kern_ms.append(b)
        comp_ms.append(c)
    prop.set_timing(False)
    avg_single_ms = sum(kern_ms) / len(kern_ms)
    avg_compose_ms = sum(comp_ms) / len(comp_ms)
    avg_span_ms = sum(span_ms) / len(span_ms)

    # algorithmic FLOPs of the method's RK4 step (the accumulation mode's extra
    # operations are not counted)
    fps = flops_per_step(w, compensated=False)
    achieved_tflops = w.trajectory_steps * fps / (avg_span_ms * 1e-3) / 1e12
    peak = PEAK_FP64_VECTOR_TFLOPS if w.precision == "fp64" else PEAK_FP32_VECTOR_TFLOPS
    chunking = "solve" if not args.two_phase else "two-phase"
    traffic = MEASURED_TRAFFIC.get((w.name, ["plain", "kahan", "blocked"][args.compensated],
                                    chunking, launches, kernel_source_sha1()))
    roofline = {
        "bound": "alu", "achieved": round(achieved_tflops, 3), "peak": peak,
        "unit": "TFLOP/s", "frac": round(achieved_tflops / peak, 4),
        "traffic": traffic,
        "traffic_unit": "HBM bytes per step (raw FETCH_SIZE + WRITE_SIZE over the step's "
                        "build launches)",
        "algorithmic_bytes": algorithmic_bytes(w),
        "kernel": f"build_kernel (ensemble RK4 integration + table write): the {launches} "
                  f"build launches of the timed step, HIP-event span",
        "kernel_ms": round(avg_span_ms, 4),
        "flops_per_trajectory_step": fps,
        "trajectory_steps_per_span": w.trajectory_steps,
        "single_launch_ms": round(avg_single_ms, 4),
    }
    if w.name in SINGLE_WAVE_STEP:
        # too few trajectories to fill the chip: each wave runs alone on its
        # SIMD, so a step takes the longer of its instructions' issue and its
        # dependent chain, both measured for one wave by the FMA probe
        st = SINGLE_WAVE_STEP[w.name]
        ns_lat, cyc_lat = nv.nv_probe_fma_chains(w.precision, 1 << 22, 1,
                                                 prop.stream.cuda_stream)
        ns_iss, cyc_iss = nv.nv_probe_fma_chains(w.precision, 1 << 22, 4,
                                                 prop.stream.cuda_stream)
        issue_ms = w.steps_per_slice * st["valu"] * ns_iss * 1e-6
        chain_ms = w.steps_per_slice * st["dependent"] * ns_lat * 1e-6
        bound_ms = max(issue_ms, chain_ms)
        roofline["single_wave_bound"] = {
            "valu_per_step": st["valu"], "dependent_ops_per_step": st["dependent"],
            "ns_per_fma_independent": round(ns_iss, 4),
            "ns_per_fma_dependent": round(ns_lat, 4),
            "clock_ticks_per_fma": [round(cyc_iss, 3), round(cyc_lat, 3)],
            "issue_bound_ms": round(issue_ms, 5), "chain_bound_ms": round(chain_ms, 5),
            "bound_ms": round(bound_ms, 5), "frac": round(bound_ms / avg_span_ms, 4),
            "what": "steps x max(VALU instructions per step x one wave's time per "
                    "independent FMA, dependent operations per step x its time per "
                    "dependent FMA): every trajectory is one lane of a wave that runs "
                    "alone on its SIMD (64 workgroups on 64 CUs), and one wave issues an "
                    "FP64 FMA every ~2.1 ns whether or not it waits on the last"}

    cold = end_to_end_cold(w, prop)

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
        "mode": "two-phase" if args.two_phase else "solve",
        "accumulation": ["plain", "kahan", "blocked"][args.compensated]
        if w.precision == "fp32" else "fp64",
        "build_launches_per_step": launches,
        "build_span_ms": round(avg_span_ms, 4),
        "compose_exposed_ms": round(sum(exposed_ms) / len(exposed_ms), 4)
        if not args.two_phase else None,
        "build_trajectory_steps_per_s": w.trajectory_steps / (avg_span_ms * 1e-3),
        "compose_alone_ms": round(avg_compose_ms, 4),
        "tau_N_us": round(1e3 * avg_compose_ms / w.n_slices, 4),
        "yT": [float(v) for v in r.yT],
        "end_to_end_cold": cold,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        host = host_description()
        threads = cpu_threads(host)
        out["cpu_baseline"] = cpu_baseline(w, threads)
        out["cpu_baseline"]["host"] = host
        out["cpu_parallel_build"] = cpu_parallel_build(w, threads)
        out["time_to_yT_vs_serial"] = fixed_error(w, r.yT, round(ms_per_step, 4), prop)
    prop.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
