"""The affine basis propagator of libnv (include/nv_linear.h) for the heat
equation of sec. 6.  Argument marshalling only: the M + 1 backward Euler
solves per slice and the chain of affine maps run in the library's kernels."""
from __future__ import annotations

from dataclasses import dataclass

from . import nv


@dataclass(frozen=True)
class HeatWorkload:
    """y_t = a(t) y_xx + b(t, x) on [0, 1], M interior points, backward Euler
    with step dt, N slices over [t0, T]; a(t) = a0 + a1 sin t; forcing: the
    one under which cos(t) sin(pi x) is the solution."""
    name: str
    M: int
    dt: float
    n_slices: int
    t0: float = 0.0
    T: float = 10.0
    a0: float = 1.0
    a1: float = 0.25
    forcing: bool = True

    @property
    def dx(self) -> float:
        return 1.0 / (self.M + 1)


class LinearPropagator:
    def __init__(self, stream=None):
        self.h = nv.nv_lin_create(stream)
        self.workload: HeatWorkload | None = None

    def close(self):
        if getattr(self, "h", None) is not None:
            nv.nv_lin_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build(self, w: HeatWorkload):
        self.workload = None
        nv.nv_lin_build(self.h, nv.make_heat(w.M, w.a0, w.a1, w.forcing), w.t0, w.T, w.n_slices,
                        w.dt)
        self.workload = w

    def compose(self, y0, want_boundary=True):
        w = self.workload
        return nv.nv_lin_compose(self.h, y0, w.M, w.n_slices, want_boundary)

    def compose_many(self, y0, want_boundary=False, device="cuda:0"):
        """Many chains at once on the matrix cores: y0 (Q, M) (numpy or a torch
        tensor) -> (status, yT (Q, M), boundary (Q, N+1, M) or None), torch FP64
        device tensors."""
        import numpy as np
        import torch

        w = self.workload
        y = y0 if isinstance(y0, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(y0))
        y = y.to(device=device, dtype=torch.float64).contiguous()
        if y.dim() != 2 or y.shape[1] != w.M:
            raise ValueError(f"y0 must be (Q, {w.M})")
        Q = y.shape[0]
        yT = torch.empty_like(y)
        b = (torch.empty((Q, w.n_slices + 1, w.M), dtype=torch.float64, device=device)
             if want_boundary else None)
        torch.cuda.synchronize(device)
        st = nv.nv_lin_compose_many(self.h, y.data_ptr(), Q, yT.data_ptr(),
                                    b.data_ptr() if b is not None else None)
        return st, yT, b

    def tables(self):
        w = self.workload
        return nv.nv_lin_get_tables(self.h, w.M, w.n_slices)

    def last_timing(self):
        return nv.nv_lin_last_timing(self.h)
