"""PyTorch-owned device memory and streams around the libnv C ABI.

``Propagator`` allocates the table and scratch buffers as torch tensors on the
device, hands their addresses to the library (nv_set_buffers) and launches on
torch's current stream of that device.  All arithmetic runs in libnv's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import nv
from .workloads import Workload


@dataclass
class ComposeResult:
    status: int
    yT: np.ndarray
    boundary: np.ndarray | None
    n_out_of_grid: int
    bad_slice: int
    n_chunks: int = 1


class Propagator:
    def __init__(self, device="cuda:0", traj_per_lane=0, compensated=2, stream=None,
                 solve_chunks=0):
        import torch

        self.torch = torch
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("Propagator needs a GPU device")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.traj_per_lane = traj_per_lane
        self.compensated = compensated
        self.solve_chunks = solve_chunks
        self._calls, self._calls_for = {}, None
        self._compose_calls = {}
        self.ctx = nv.nv_ctx_create()
        self._tables = None
        self._work = None
        self.workload: Workload | None = None

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if self.ctx is not None:
            nv.nv_ctx_destroy(self.ctx)
            self.ctx = None
        self._tables = self._work = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers -------------------------------------------------------------
    def options(self, w: Workload) -> nv.nv_options:
        return nv.make_options(w.scheme, w.precision, self.compensated, self.traj_per_lane,
                               self.stream.cuda_stream, self.solve_chunks, w.dt)

    @staticmethod
    def grid(w: Workload) -> nv.nv_ic_grid:
        return nv.make_grid(w.grid_n, w.grid_lo, w.grid_hi, w.interp)

    def _ensure_buffers(self, table_bytes, work_bytes):
        t = self.torch
        if (self._tables is None or self._tables.numel() < table_bytes or
                self._work is None or self._work.numel() < work_bytes):
            with t.cuda.device(self.device):
                self._tables = t.empty(max(table_bytes, 256), dtype=t.uint8, device=self.device)
                self._work = t.empty(max(work_bytes, 256), dtype=t.uint8, device=self.device)
            nv.nv_set_buffers(self.ctx, self._tables.data_ptr(), self._tables.numel(),
                              self._work.data_ptr(), self._work.numel())

    # -- the two phases --------------------------------------------------------
    def _prepare(self, w: Workload):
        # options, grid and buffer sizes are set once per workload
        if getattr(self, "_prepared_for", None) is w:
            return self._prepared
        opt = self.options(w)
        nv.nv_set_options(self.ctx, opt)
        g = self.grid(w)
        rhs = nv.RHS_IDS[w.rhs]
        tb, wb = nv.nv_required_bytes(rhs, w.n_slices, g, w.steps_per_slice, opt)
        self._ensure_buffers(tb, wb)
        self._prepared_for, self._prepared = w, (g, rhs)
        return g, rhs

    def _key(self, w: Workload, params, *extra):
        # per workload (its identity) and parameters: the calls marshalled for it
        if self._calls_for is not w:
            self._calls, self._calls_for = {}, w
        return (params if isinstance(params, tuple)
                else tuple(np.asarray(params, dtype=np.float64).reshape(-1)),) + extra

    def build(self, w: Workload, params=None):
        """Computation phase: tables of every slice (asynchronous on the stream)."""
        g, rhs = self._prepare(w)
        params = params if params is not None else w.params
        key = ("build",) + self._key(w, params)
        call = self._calls.get(key)
        if call is None:
            call = self._calls[key] = nv.BuildCall(rhs, params, w.t0, w.T, w.n_slices, g,
                                                   w.steps_per_slice)
        call(self.ctx)
        self.workload = w

    def solve(self, w: Workload, y0=None, params=None, want_boundary=True) -> ComposeResult:
        """Both phases, the composition pipelined behind the build (synchronous)."""
        g, rhs = self._prepare(w)
        self.workload = None
        params = params if params is not None else w.params
        # the call's arguments are marshalled once per workload, parameters and
        # boundary choice (the binding's share of a small solve's latency)
        key = ("solve",) + self._key(w, params, bool(want_boundary))
        call = self._calls.get(key)
        if call is None:
            call = self._calls[key] = nv.SolveCall(rhs, params, w.t0, w.T, w.n_slices, g,
                                                   w.steps_per_slice, w.dim, want_boundary)
        st, yT, b, info = call(self.ctx, w.y0 if y0 is None else y0)
        self.workload = w
        return ComposeResult(st, yT, b, info.n_out_of_grid, info.bad_slice, info.n_chunks)

    def compose(self, y0=None, want_boundary=True) -> ComposeResult:
        """Communication phase (synchronous)."""
        w = self.workload
        key = (w.n_slices, w.dim, bool(want_boundary))
        call = self._compose_calls.get(key)
        if call is None:
            call = self._compose_calls[key] = nv.ComposeCall(w.n_slices, w.dim, want_boundary)
        st, yT, b, info = call(self.ctx, w.y0 if y0 is None else y0)
        return ComposeResult(st, yT, b, info.n_out_of_grid, info.bad_slice, info.n_chunks)

    # -- inspection ------------------------------------------------------------
    def table(self, component=0) -> np.ndarray:
        w = self.workload
        return nv.nv_get_table(self.ctx, component, w.n_slices, w.points_per_slice, w.precision)

    def table_tensor(self, component=0):
        """Device view of one component's table, shape (n_slices, points)."""
        t = self.torch
        w = self.workload
        ptr = nv.nv_table_device_ptr(self.ctx, component)
        off = ptr - self._tables.data_ptr()
        dt = t.float64 if w.precision == "fp64" else t.float32
        nbytes = w.n_slices * w.points_per_slice * (8 if w.precision == "fp64" else 4)
        return self._tables[off:off + nbytes].view(dt).view(w.n_slices, w.points_per_slice)

    def nonfinite_counts(self) -> np.ndarray:
        return nv.nv_get_nonfinite_counts(self.ctx, self.workload.n_slices)

    def set_timing(self, enable=True):
        nv.nv_set_timing(self.ctx, enable)

    def last_timing(self):
        return nv.nv_last_timing(self.ctx)


class Batch:
    """Many problems (Workloads) built in one persistent launch and composed in
    one launch, replayed from a captured HIP graph (nv_batch_*)."""

    def __init__(self, workloads, precision="fp32", compensated=2):
        self.workloads = list(workloads)
        if any(w.scheme != "rk4" for w in self.workloads):
            raise ValueError("batches integrate with RK4")
        self.precision = precision
        self.ctx = nv.nv_ctx_create()
        nv.nv_set_options(self.ctx, nv.make_options("rk4", precision, compensated))
        probs = [nv.make_problem(w.rhs, w.params, w.t0, w.T, w.n_slices,
                                 nv.make_grid(w.grid_n, w.grid_lo, w.grid_hi, w.interp),
                                 w.steps_per_slice, w.y0) for w in self.workloads]
        try:
            self.batch = nv.nv_batch_create(self.ctx, probs)
        except Exception:
            nv.nv_ctx_destroy(self.ctx)
            self.ctx = None
            raise

    def close(self):
        if getattr(self, "batch", None) is not None:
            nv.nv_batch_destroy(self.batch)
            self.batch = None
        if getattr(self, "ctx", None) is not None:
            nv.nv_ctx_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self):
        """(status, yT array (count, dim max 2), list of ComposeResult-like infos)."""
        st, yT, infos = nv.nv_batch_run(self.batch, len(self.workloads))
        return st, yT, [(i.n_out_of_grid, i.bad_slice) for i in infos]

    def schedule(self):
        return nv.nv_batch_get_schedule(self.batch)

    def set_schedule(self, traj_per_lane=None, workgroups_per_cu=8, order=0):
        s = nv.nv_batch_schedule()
        for r in range(5):
            s.traj_per_lane[r] = (traj_per_lane or {}).get(r, 1)
        s.workgroups_per_cu = workgroups_per_cu
        s.order = order
        nv.nv_batch_set_schedule(self.batch, s)

    def autotune(self, reps=2):
        return nv.nv_batch_autotune(self.batch, reps)

    def last_timing(self):
        return nv.nv_batch_last_timing(self.batch)

    def table(self, i, component=0):
        w = self.workloads[i]
        return nv.nv_batch_get_table(self.batch, i, component, w.n_slices, w.points_per_slice,
                                     self.precision)

    def boundary(self, i):
        w = self.workloads[i]
        return nv.nv_batch_get_boundary(self.batch, i, w.n_slices, w.dim)
