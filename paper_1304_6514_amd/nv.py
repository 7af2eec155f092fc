"""ctypes binding of libnv (include/nv.h), with the C ABI's names.

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  If libnv.so has not been built this module raises on first use; there
is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnv.so")

# nv_status
NV_OK = 0
NV_ERR_INVALID_ARG = -1
NV_ERR_NOT_BUILT = -2
NV_ERR_NONFINITE = -3
NV_ERR_OOM = -4
NV_ERR_HIP = -5
NV_ERR_UNSUPPORTED = -6
NV_ERR_BUFFER_TOO_SMALL = -7
# nv_rhs_id
NV_RHS_LINEAR, NV_RHS_LOGISTIC, NV_RHS_FORCED_CUBIC, NV_RHS_VDP, NV_RHS_SQUARE = range(5)
# nv_scheme, nv_precision, nv_interp
NV_SCHEME_RK4, NV_SCHEME_EULER, NV_SCHEME_BACKWARD_EULER = 0, 1, 2
NV_FP64, NV_FP32 = 0, 1
NV_INTERP_LINEAR, NV_INTERP_HERMITE, NV_INTERP_BILINEAR, NV_INTERP_CHEBYSHEV = 0, 1, 2, 3
NV_INTERP_HERMITE_SLOPES = 4

RHS_IDS = {"linear": NV_RHS_LINEAR, "logistic": NV_RHS_LOGISTIC,
           "forced_cubic": NV_RHS_FORCED_CUBIC, "vdp": NV_RHS_VDP, "square": NV_RHS_SQUARE}
SCHEMES = {"rk4": NV_SCHEME_RK4, "euler": NV_SCHEME_EULER, "be": NV_SCHEME_BACKWARD_EULER}
PRECISIONS = {"fp64": NV_FP64, "fp32": NV_FP32}
INTERPS = {"linear": NV_INTERP_LINEAR, "hermite": NV_INTERP_HERMITE,
           "bilinear": NV_INTERP_BILINEAR, "chebyshev": NV_INTERP_CHEBYSHEV,
           "hermite_slopes": NV_INTERP_HERMITE_SLOPES}


class nv_ic_grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 2), ("lo", ctypes.c_double * 2),
                ("hi", ctypes.c_double * 2), ("interp", ctypes.c_int)]


class nv_options(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("precision", ctypes.c_int),
                ("compensated", ctypes.c_int), ("traj_per_lane", ctypes.c_int),
                ("stream", ctypes.c_void_p), ("solve_chunks", ctypes.c_int),
                ("dt", ctypes.c_double)]


class nv_compose_info(ctypes.Structure):
    _fields_ = [("n_out_of_grid", ctypes.c_longlong), ("bad_slice", ctypes.c_int),
                ("n_chunks", ctypes.c_int)]


class nv_solve_status(ctypes.Structure):
    _fields_ = [("n_out_of_grid", ctypes.c_longlong), ("bad_slice", ctypes.c_int),
                ("done", ctypes.c_int)]


NV_STATIC_SCRATCH_BYTES = 64 << 20


class nv_problem(ctypes.Structure):
    _fields_ = [("rhs_id", ctypes.c_int), ("params", ctypes.c_double * 2),
                ("t0", ctypes.c_double), ("T", ctypes.c_double), ("n_slices", ctypes.c_int),
                ("grid", nv_ic_grid), ("steps_per_slice", ctypes.c_int),
                ("y0", ctypes.c_double * 2)]


class nv_batch_schedule(ctypes.Structure):
    _fields_ = [("traj_per_lane", ctypes.c_int * 5), ("workgroups_per_cu", ctypes.c_int),
                ("order", ctypes.c_int)]


class NvError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{status_name(status)}: {message}")
        self.status = status


_lib = None

_P = ctypes.c_void_p
_SIGNATURES = {
    "nv_ctx_create": [ctypes.POINTER(ctypes.c_void_p)],
    "nv_ctx_destroy": [_P],
    "nv_set_options": [_P, ctypes.POINTER(nv_options)],
    "nv_get_options": [_P, ctypes.POINTER(nv_options)],
    "nv_required_bytes": [ctypes.c_int, ctypes.c_int, ctypes.POINTER(nv_ic_grid), ctypes.c_int,
                          ctypes.POINTER(nv_options), ctypes.POINTER(ctypes.c_size_t),
                          ctypes.POINTER(ctypes.c_size_t)],
    "nv_set_buffers": [_P, _P, ctypes.c_size_t, _P, ctypes.c_size_t],
    "nv_build_propagators": [_P, ctypes.c_int, _P, ctypes.c_double, ctypes.c_double,
                             ctypes.c_int, ctypes.POINTER(nv_ic_grid), ctypes.c_int],
    "nv_compose": [_P, _P, _P, _P, ctypes.POINTER(nv_compose_info)],
    "nv_solve": [_P, ctypes.c_int, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                 ctypes.POINTER(nv_ic_grid), ctypes.c_int, _P, _P, _P,
                 ctypes.POINTER(nv_compose_info)],
    "nv_solve_static": [ctypes.c_int, _P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                        ctypes.POINTER(nv_ic_grid), ctypes.c_int, ctypes.POINTER(nv_options),
                        _P, ctypes.c_size_t, _P, _P, _P],
    "nv_get_table": [_P, ctypes.c_int, _P, ctypes.c_size_t],
    "nv_table_device_ptr": [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)],
    "nv_get_nonfinite_counts": [_P, _P, ctypes.c_int],
    "nv_locate": [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int, _P, ctypes.c_longlong,
                  _P, _P, _P],
    "nv_set_timing": [_P, ctypes.c_int],
    "nv_last_timing": [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
    "nv_batch_create": [_P, ctypes.POINTER(nv_problem), ctypes.c_int,
                        ctypes.POINTER(ctypes.c_void_p)],
    "nv_batch_destroy": [_P],
    "nv_batch_set_schedule": [_P, ctypes.POINTER(nv_batch_schedule)],
    "nv_batch_get_schedule": [_P, ctypes.POINTER(nv_batch_schedule)],
    "nv_batch_autotune": [_P, ctypes.c_int, ctypes.POINTER(nv_batch_schedule)],
    "nv_batch_run": [_P, _P, ctypes.POINTER(nv_compose_info)],
    "nv_batch_last_timing": [_P, ctypes.POINTER(ctypes.c_float),
                             ctypes.POINTER(ctypes.c_longlong)],
    "nv_batch_get_table": [_P, ctypes.c_int, ctypes.c_int, _P, ctypes.c_size_t],
    "nv_batch_get_boundary": [_P, ctypes.c_int, _P, ctypes.c_size_t],
    "nv_probe_fma_latency": [ctypes.c_int, ctypes.c_longlong, _P,
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "nv_probe_fma_chains": [ctypes.c_int, ctypes.c_longlong, ctypes.c_int, _P,
                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
    "nv_last_error": [],
    "nv_status_string": [ctypes.c_int],
}


def load():
    """Load libnv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("nv_last_error", "nv_status_string") \
            else ctypes.c_int
    _lib = lib
    return lib


def status_name(status: int) -> str:
    return load().nv_status_string(int(status)).decode()


def nv_last_error() -> str:
    return load().nv_last_error().decode()


def _check(status: int):
    if status != NV_OK:
        raise NvError(status, nv_last_error())
    return status


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_grid(n, lo, hi, interp) -> nv_ic_grid:
    n = list(np.atleast_1d(n))
    lo = list(np.atleast_1d(lo))
    hi = list(np.atleast_1d(hi))
    g = nv_ic_grid()
    g.dim = len(n)
    for a in range(len(n)):
        g.n[a], g.lo[a], g.hi[a] = int(n[a]), float(lo[a]), float(hi[a])
    g.interp = INTERPS[interp] if isinstance(interp, str) else int(interp)
    return g


def make_options(scheme="rk4", precision="fp64", compensated=2, traj_per_lane=0,
                 stream=None, solve_chunks=0, dt=0.0) -> nv_options:
    o = nv_options()
    o.scheme = SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.compensated = int(compensated)
    o.traj_per_lane = int(traj_per_lane)
    o.stream = stream
    o.solve_chunks = int(solve_chunks)
    o.dt = float(dt)
    return o


# ---- the C ABI, one wrapper per entry point -------------------------------

def nv_ctx_create():
    h = ctypes.c_void_p()
    _check(load().nv_ctx_create(ctypes.byref(h)))
    return h


def nv_ctx_destroy(ctx):
    return _check(load().nv_ctx_destroy(ctx))


def nv_set_options(ctx, opt: nv_options):
    return _check(load().nv_set_options(ctx, ctypes.byref(opt)))


def nv_get_options(ctx) -> nv_options:
    o = nv_options()
    _check(load().nv_get_options(ctx, ctypes.byref(o)))
    return o


def nv_required_bytes(rhs_id, n_slices, grid: nv_ic_grid, steps_per_slice, opt=None):
    tb, wb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().nv_required_bytes(int(rhs_id), int(n_slices), ctypes.byref(grid),
                                    int(steps_per_slice),
                                    ctypes.byref(opt) if opt is not None else None,
                                    ctypes.byref(tb), ctypes.byref(wb)))
    return tb.value, wb.value


def nv_set_buffers(ctx, tables_dev, table_bytes, work_dev, work_bytes):
    return _check(load().nv_set_buffers(ctx, tables_dev, int(table_bytes), work_dev,
                                        int(work_bytes)))


def nv_build_propagators(ctx, rhs_id, params, t0, T, n_slices, grid: nv_ic_grid,
                         steps_per_slice):
    p = np.ascontiguousarray(np.asarray(params if params is not None else [0.0],
                                        dtype=np.float64).reshape(-1))
    if p.size == 0:
        p = np.zeros(1)
    return _check(load().nv_build_propagators(ctx, int(rhs_id), _ptr(p), float(t0), float(T),
                                              int(n_slices), ctypes.byref(grid),
                                              int(steps_per_slice)))


def nv_compose(ctx, y0, dim, n_slices, want_boundary=True):
    """Returns (status, yT, boundary or None, info).  Raises on every status
    other than NV_OK and NV_ERR_NONFINITE."""
    y0 = np.ascontiguousarray(np.asarray(y0, dtype=np.float64).reshape(-1))
    yT = np.full(dim, np.nan)
    boundary = np.full((n_slices + 1, dim), np.nan) if want_boundary else None
    info = nv_compose_info()
    st = load().nv_compose(ctx, _ptr(y0), _ptr(yT),
                           _ptr(boundary) if boundary is not None else None,
                           ctypes.byref(info))
    if st not in (NV_OK, NV_ERR_NONFINITE):
        _check(st)
    return st, yT, boundary, info


def nv_solve(ctx, rhs_id, params, t0, T, n_slices, grid: nv_ic_grid, steps_per_slice, y0,
             dim, want_boundary=True):
    """Returns (status, yT, boundary or None, info).  Raises on every status
    other than NV_OK and NV_ERR_NONFINITE."""
    p = np.ascontiguousarray(np.asarray(params if params is not None else [0.0],
                                        dtype=np.float64).reshape(-1))
    if p.size == 0:
        p = np.zeros(1)
    y0 = np.ascontiguousarray(np.asarray(y0, dtype=np.float64).reshape(-1))
    yT = np.full(dim, np.nan)
    boundary = np.full((n_slices + 1, dim), np.nan) if want_boundary else None
    info = nv_compose_info()
    st = load().nv_solve(ctx, int(rhs_id), _ptr(p), float(t0), float(T), int(n_slices),
                         ctypes.byref(grid), int(steps_per_slice), _ptr(y0), _ptr(yT),
                         _ptr(boundary) if boundary is not None else None, ctypes.byref(info))
    if st not in (NV_OK, NV_ERR_NONFINITE):
        _check(st)
    return st, yT, boundary, info


class _Outputs:
    """y0, yT, boundary and info buffers of one prepared composition call."""

    def __init__(self, n_slices, dim, want_boundary):
        self._y0 = np.zeros(dim)
        self._yT = np.full(dim, np.nan)
        self._boundary = np.full((n_slices + 1, dim), np.nan) if want_boundary else None
        self._info = nv_compose_info()
        self._out = (_ptr(self._y0), _ptr(self._yT),
                     _ptr(self._boundary) if self._boundary is not None else None,
                     ctypes.byref(self._info))

    def _finish(self, st):
        if st not in (NV_OK, NV_ERR_NONFINITE):
            _check(st)
        info = nv_compose_info.from_buffer_copy(self._info)
        b = None
        if self._boundary is not None:
            b = self._boundary.copy()
            if st != NV_OK:             # rows past the failing slice were not written
                b[info.bad_slice + 1:] = np.nan
        return st, self._yT.copy(), b, info


class SolveCall(_Outputs):
    """nv_solve's arguments for one problem, marshalled once.  Repeated solves
    of the same problem (a serving loop, the benchmark) then pay for the
    foreign call and the copies of the outputs only, not for building the
    argument arrays and pointers again.  Call it with the context and y0;
    it returns what nv_solve returns, the outputs copied out of its buffers.
    One call at a time: concurrent calls of one SolveCall share its buffers."""

    def __init__(self, rhs_id, params, t0, T, n_slices, grid: nv_ic_grid, steps_per_slice,
                 dim, want_boundary=True):
        super().__init__(n_slices, dim, want_boundary)
        p = np.ascontiguousarray(np.asarray(params if params is not None else [0.0],
                                            dtype=np.float64).reshape(-1))
        self._p = p if p.size else np.zeros(1)
        self._grid = grid
        y0, yT, b, info = self._out
        self._args = (int(rhs_id), _ptr(self._p), float(t0), float(T), int(n_slices),
                      ctypes.byref(grid), int(steps_per_slice), y0, yT, b, info)
        self._fn = load().nv_solve

    def __call__(self, ctx, y0):
        self._y0[:] = y0
        return self._finish(self._fn(ctx, *self._args))


class BuildCall:
    """nv_build_propagators' arguments for one problem, marshalled once (the
    same contract as SolveCall); call it with the context."""

    def __init__(self, rhs_id, params, t0, T, n_slices, grid: nv_ic_grid, steps_per_slice):
        p = np.ascontiguousarray(np.asarray(params if params is not None else [0.0],
                                            dtype=np.float64).reshape(-1))
        self._p = p if p.size else np.zeros(1)
        self._grid = grid
        self._args = (int(rhs_id), _ptr(self._p), float(t0), float(T), int(n_slices),
                      ctypes.byref(grid), int(steps_per_slice))
        self._fn = load().nv_build_propagators

    def __call__(self, ctx):
        return _check(self._fn(ctx, *self._args))


class ComposeCall(_Outputs):
    """nv_compose's arguments for one built problem, marshalled once (many
    initial values queried one after another through the same tables).  The
    same contract as SolveCall."""

    def __init__(self, n_slices, dim, want_boundary=True):
        super().__init__(n_slices, dim, want_boundary)
        self._fn = load().nv_compose

    def __call__(self, ctx, y0):
        self._y0[:] = y0
        return self._finish(self._fn(ctx, *self._out))


def nv_solve_static(rhs_id, params, t0, T, n_slices, grid: nv_ic_grid, steps_per_slice,
                    opt: nv_options, tables_dev, table_bytes, y0, boundary_dev, status_dev):
    """Queues the build and the composition on opt.stream with the library's
    static scratch; the outputs are device addresses (read them after the
    stream).  Raises on every status other than NV_OK."""
    p = np.ascontiguousarray(np.asarray(params if params is not None else [0.0],
                                        dtype=np.float64).reshape(-1))
    if p.size == 0:
        p = np.zeros(1)
    y0 = np.ascontiguousarray(np.asarray(y0, dtype=np.float64).reshape(-1))
    return _check(load().nv_solve_static(int(rhs_id), _ptr(p), float(t0), float(T),
                                         int(n_slices), ctypes.byref(grid),
                                         int(steps_per_slice), ctypes.byref(opt), tables_dev,
                                         int(table_bytes), _ptr(y0), boundary_dev, status_dev))


def nv_get_table(ctx, component, n_slices, points, precision):
    dt = np.float64 if precision in ("fp64", NV_FP64) else np.float32
    out = np.empty((n_slices, points), dtype=dt)
    _check(load().nv_get_table(ctx, int(component), _ptr(out), out.nbytes))
    return out


def nv_table_device_ptr(ctx, component):
    p = ctypes.c_void_p()
    _check(load().nv_table_device_ptr(ctx, int(component), ctypes.byref(p)))
    return p.value


def nv_get_nonfinite_counts(ctx, n_slices):
    out = np.zeros(n_slices, dtype=np.uint32)
    _check(load().nv_get_nonfinite_counts(ctx, _ptr(out), int(n_slices)))
    return out


def nv_locate(ctx, lo, hi, n, x_dev, count, cell_dev, w_dev, out_dev):
    return _check(load().nv_locate(ctx, float(lo), float(hi), int(n), x_dev, int(count),
                                   cell_dev, w_dev, out_dev))


def nv_set_timing(ctx, enable):
    return _check(load().nv_set_timing(ctx, int(bool(enable))))


def nv_last_timing(ctx):
    b, c = ctypes.c_float(), ctypes.c_float()
    _check(load().nv_last_timing(ctx, ctypes.byref(b), ctypes.byref(c)))
    return b.value, c.value


def nv_probe_fma_latency(precision="fp64", ops=1 << 22, stream=None):
    """(ns, shader-clock cycles) per dependent FMA of one wave's chain."""
    ns, cyc = ctypes.c_double(), ctypes.c_double()
    _check(load().nv_probe_fma_latency(PRECISIONS.get(precision, precision), int(ops), stream,
                                       ctypes.byref(ns), ctypes.byref(cyc)))
    return ns.value, cyc.value


def nv_probe_fma_chains(precision="fp64", ops=1 << 22, chains=4, stream=None):
    """(ns, shader-clock cycles) per FMA of one wave running `chains`
    independent chains of `ops` dependent FMAs per lane."""
    ns, cyc = ctypes.c_double(), ctypes.c_double()
    _check(load().nv_probe_fma_chains(PRECISIONS.get(precision, precision), int(ops),
                                      int(chains), stream, ctypes.byref(ns), ctypes.byref(cyc)))
    return ns.value, cyc.value


# ---- batches ----------------------------------------------------------------

def make_problem(rhs, params, t0, T, n_slices, grid: nv_ic_grid, steps_per_slice, y0):
    p = nv_problem()
    p.rhs_id = RHS_IDS[rhs] if isinstance(rhs, str) else int(rhs)
    for i, v in enumerate(list(params or [])[:2]):
        p.params[i] = float(v)
    p.t0, p.T, p.n_slices = float(t0), float(T), int(n_slices)
    p.grid = grid
    p.steps_per_slice = int(steps_per_slice)
    for i, v in enumerate(list(y0)[:2]):
        p.y0[i] = float(v)
    return p


def nv_batch_create(ctx, problems):
    arr = (nv_problem * len(problems))(*problems)
    h = ctypes.c_void_p()
    _check(load().nv_batch_create(ctx, arr, len(problems), ctypes.byref(h)))
    return h


def nv_batch_destroy(batch):
    return _check(load().nv_batch_destroy(batch))


def nv_batch_set_schedule(batch, sched: nv_batch_schedule):
    return _check(load().nv_batch_set_schedule(batch, ctypes.byref(sched)))


def nv_batch_get_schedule(batch) -> nv_batch_schedule:
    s = nv_batch_schedule()
    _check(load().nv_batch_get_schedule(batch, ctypes.byref(s)))
    return s


def nv_batch_autotune(batch, reps=2) -> nv_batch_schedule:
    s = nv_batch_schedule()
    _check(load().nv_batch_autotune(batch, int(reps), ctypes.byref(s)))
    return s


def nv_batch_run(batch, count):
    """Returns (status, yT of shape (count, 2), infos).  Raises on statuses
    other than NV_OK and NV_ERR_NONFINITE."""
    yT = np.full((count, 2), np.nan)
    infos = (nv_compose_info * count)()
    st = load().nv_batch_run(batch, _ptr(yT), infos)
    if st not in (NV_OK, NV_ERR_NONFINITE):
        _check(st)
    return st, yT, infos


def nv_batch_last_timing(batch):
    ms, steps = ctypes.c_float(), ctypes.c_longlong()
    _check(load().nv_batch_last_timing(batch, ctypes.byref(ms), ctypes.byref(steps)))
    return ms.value, steps.value


def nv_batch_get_table(batch, problem, component, n_slices, points, precision):
    dt = np.float64 if precision in ("fp64", NV_FP64) else np.float32
    out = np.empty((n_slices, points), dtype=dt)
    _check(load().nv_batch_get_table(batch, int(problem), int(component), _ptr(out),
                                     out.nbytes))
    return out


def nv_batch_get_boundary(batch, problem, n_slices, dim):
    out = np.empty((n_slices + 1, dim))
    _check(load().nv_batch_get_boundary(batch, int(problem), _ptr(out), out.size))
    return out


# ---- learned surrogate (include/nv_surrogate.h) ------------------------------

NV_SUR_PARAMS = 33922


class nv_sur_config(ctypes.Structure):
    _fields_ = [("in_shift", ctypes.c_float * 4), ("in_scale", ctypes.c_float * 4),
                ("out_scale", ctypes.c_double * 2), ("slice_length", ctypes.c_double),
                ("coarse_steps", ctypes.c_int), ("max_batch", ctypes.c_longlong),
                ("stream", ctypes.c_void_p), ("correction", ctypes.c_int),
                ("gate", ctypes.c_double * 2), ("loss_scale", ctypes.c_double * 2)]


NV_SUR_ADDITIVE, NV_SUR_STEP_DOUBLING = 0, 1


class nv_sur_train_opts(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_longlong), ("steps", ctypes.c_longlong),
                ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("lr_final", ctypes.c_float)]


class nv_sur_chains(ctypes.Structure):
    _fields_ = [("count", ctypes.c_longlong), ("y0", ctypes.c_void_p), ("mu", ctypes.c_void_p),
                ("t0", ctypes.c_double), ("T", ctypes.c_double), ("n_slices", ctypes.c_int),
                ("final_state", ctypes.c_void_p), ("boundary", ctypes.c_void_p),
                ("fb_tab0", ctypes.c_void_p), ("fb_tab1", ctypes.c_void_p),
                ("fb_precision", ctypes.c_int), ("fb_grid", nv_ic_grid),
                ("guard", ctypes.c_double), ("box_lo", ctypes.c_double * 2),
                ("box_hi", ctypes.c_double * 2)]


class nv_sur_compose_info(ctypes.Structure):
    _fields_ = [("n_fallback", ctypes.c_longlong), ("n_outside", ctypes.c_longlong),
                ("max_deviation", ctypes.c_double), ("bad_chain", ctypes.c_longlong),
                ("ms", ctypes.c_float)]


_SIGNATURES.update({
    "nv_sur_create": [ctypes.POINTER(nv_sur_config), ctypes.POINTER(ctypes.c_void_p)],
    "nv_sur_destroy": [_P],
    "nv_sur_set_params": [_P, _P],
    "nv_sur_get_params": [_P, _P],
    "nv_sur_forward": [_P, _P, ctypes.c_longlong, _P],
    "nv_sur_loss_grad": [_P, _P, _P, ctypes.c_longlong, ctypes.POINTER(ctypes.c_float), _P],
    "nv_sur_train": [_P, _P, _P, ctypes.c_longlong, ctypes.POINTER(nv_sur_train_opts), _P],
    "nv_sur_dataset_from_batch": [_P, _P, _P, _P, _P, ctypes.c_longlong,
                                  ctypes.POINTER(ctypes.c_longlong)],
    "nv_sur_compose": [_P, ctypes.POINTER(nv_sur_chains), ctypes.POINTER(nv_sur_compose_info)],
    "nv_sur_last_ms": [_P, ctypes.POINTER(ctypes.c_float)],
    "nv_sur_set_visits": [_P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, ctypes.c_double],
})


def make_sur_config(in_shift, in_scale, out_scale, slice_length, coarse_steps=0, max_batch=0,
                    stream=None, correction=NV_SUR_ADDITIVE, gate=(1.0, 1.0),
                    loss_scale=(1.0, 1.0)) -> nv_sur_config:
    c = nv_sur_config()
    for k in range(4):
        c.in_shift[k], c.in_scale[k] = float(in_shift[k]), float(in_scale[k])
    c.out_scale[0], c.out_scale[1] = float(out_scale[0]), float(out_scale[1])
    c.slice_length, c.coarse_steps = float(slice_length), int(coarse_steps)
    c.max_batch = int(max_batch)
    c.stream = stream
    c.correction = int(correction)
    for k in range(2):
        c.gate[k], c.loss_scale[k] = float(gate[k]), float(loss_scale[k])
    return c


def nv_sur_set_visits(sur, states_dev, n_mu, n_states, mu_lo, mu_hi, sigma, floor_weight):
    return _check(load().nv_sur_set_visits(sur, states_dev, int(n_mu), int(n_states),
                                           float(mu_lo), float(mu_hi), float(sigma),
                                           float(floor_weight)))


def nv_sur_create(cfg: nv_sur_config):
    h = ctypes.c_void_p()
    _check(load().nv_sur_create(ctypes.byref(cfg), ctypes.byref(h)))
    return h


def nv_sur_destroy(sur):
    return _check(load().nv_sur_destroy(sur))


def nv_sur_set_params(sur, params):
    p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(-1))
    if p.size != NV_SUR_PARAMS:
        raise ValueError(f"expected {NV_SUR_PARAMS} parameters, got {p.size}")
    return _check(load().nv_sur_set_params(sur, _ptr(p)))


def nv_sur_get_params(sur):
    out = np.empty(NV_SUR_PARAMS, dtype=np.float32)
    _check(load().nv_sur_get_params(sur, _ptr(out)))
    return out


def nv_sur_forward(sur, x_dev, n, out_dev):
    return _check(load().nv_sur_forward(sur, x_dev, int(n), out_dev))


def nv_sur_loss_grad(sur, x_dev, t_dev, n, want_grad=True):
    loss = ctypes.c_float()
    grad = np.empty(NV_SUR_PARAMS, dtype=np.float32) if want_grad else None
    _check(load().nv_sur_loss_grad(sur, x_dev, t_dev, int(n), ctypes.byref(loss),
                                   _ptr(grad) if grad is not None else None))
    return loss.value, grad


def make_train_opts(batch, steps, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                    lr_final=0.0) -> nv_sur_train_opts:
    o = nv_sur_train_opts()
    o.batch, o.steps = int(batch), int(steps)
    o.lr, o.beta1, o.beta2, o.eps, o.lr_final = lr, beta1, beta2, eps, lr_final
    return o


def nv_sur_train(sur, x_dev, t_dev, n_samples, opts: nv_sur_train_opts, loss_dev=None):
    return _check(load().nv_sur_train(sur, x_dev, t_dev, int(n_samples), ctypes.byref(opts),
                                      loss_dev))


def nv_sur_dataset_from_batch(sur, batch, perm_dev=None, x_dev=None, t_dev=None, cap=0):
    total = ctypes.c_longlong()
    _check(load().nv_sur_dataset_from_batch(sur, batch, perm_dev, x_dev, t_dev, int(cap),
                                            ctypes.byref(total)))
    return total.value


def nv_sur_compose(sur, chains: nv_sur_chains):
    """Returns (status, info); raises on statuses other than NV_OK and
    NV_ERR_NONFINITE."""
    info = nv_sur_compose_info()
    st = load().nv_sur_compose(sur, ctypes.byref(chains), ctypes.byref(info))
    if st not in (NV_OK, NV_ERR_NONFINITE):
        _check(st)
    return st, info


def nv_sur_last_ms(sur):
    ms = ctypes.c_float()
    _check(load().nv_sur_last_ms(sur, ctypes.byref(ms)))
    return ms.value


# ---- affine basis propagator for linear systems (include/nv_linear.h) ---------

NV_LIN_MAX_POINTS = 127


class nv_heat(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int), ("a0", ctypes.c_double), ("a1", ctypes.c_double),
                ("forcing", ctypes.c_int)]


_SIGNATURES.update({
    "nv_lin_create": [_P, ctypes.POINTER(ctypes.c_void_p)],
    "nv_lin_destroy": [_P],
    "nv_lin_build": [_P, ctypes.POINTER(nv_heat), ctypes.c_double, ctypes.c_double,
                     ctypes.c_int, ctypes.c_double],
    "nv_lin_compose": [_P, _P, _P, _P],
    "nv_lin_compose_many": [_P, _P, ctypes.c_longlong, _P, _P],
    "nv_lin_get_tables": [_P, _P, _P],
    "nv_lin_last_timing": [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
})


def make_heat(M, a0=1.0, a1=0.25, forcing=True) -> nv_heat:
    h = nv_heat()
    h.M, h.a0, h.a1, h.forcing = int(M), float(a0), float(a1), int(bool(forcing))
    return h


def nv_lin_create(stream=None):
    h = ctypes.c_void_p()
    _check(load().nv_lin_create(stream, ctypes.byref(h)))
    return h


def nv_lin_destroy(lin):
    return _check(load().nv_lin_destroy(lin))


def nv_lin_build(lin, heat: nv_heat, t0, T, n_slices, dt):
    return _check(load().nv_lin_build(lin, ctypes.byref(heat), float(t0), float(T),
                                      int(n_slices), float(dt)))


def nv_lin_compose(lin, y0, M, n_slices, want_boundary=True):
    """Returns (status, yT, boundary or None); raises on statuses other than
    NV_OK and NV_ERR_NONFINITE."""
    y0 = np.ascontiguousarray(np.asarray(y0, dtype=np.float64).reshape(-1))
    if y0.size != M:
        raise ValueError(f"y0 has {y0.size} values, the problem {M}")
    yT = np.full(M, np.nan)
    b = np.full((n_slices + 1, M), np.nan) if want_boundary else None
    st = load().nv_lin_compose(lin, _ptr(y0), _ptr(yT), _ptr(b) if b is not None else None)
    if st not in (NV_OK, NV_ERR_NONFINITE):
        _check(st)
    return st, yT, b


def nv_lin_compose_many(lin, y0_dev, count, yT_dev, boundary_dev=None):
    """Status (NV_OK or NV_ERR_NONFINITE); raises on every other status."""
    st = load().nv_lin_compose_many(lin, y0_dev, int(count), yT_dev, boundary_dev)
    if st not in (NV_OK, NV_ERR_NONFINITE):
        _check(st)
    return st


def nv_lin_get_tables(lin, M, n_slices):
    G = np.empty((n_slices, M, M))
    c = np.empty((n_slices, M))
    _check(load().nv_lin_get_tables(lin, _ptr(G), _ptr(c)))
    return G, c


def nv_lin_last_timing(lin):
    b, c = ctypes.c_float(), ctypes.c_float()
    _check(load().nv_lin_last_timing(lin, ctypes.byref(b), ctypes.byref(c)))
    return b.value, c.value
