"""Plain serial CPU oracle for Nievergelt's method (Barker, arXiv:1304.6514).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It never imports
the GPU package and the GPU package never imports it; both are written from the
paper independently.  The arithmetic lives in ``nv_oracle.c`` (plain C, FP64,
no contraction); this module only marshals arguments.

Problems are named by string: ``"linear"`` (y'=p0*y), ``"logistic"``,
``"forced_cubic"`` (y'=sin 3t - y^3), ``"vdp"`` (Van der Pol, p0=mu) and
``"square"`` (y'=y^2, the model problem of sec. 3).  Schemes: ``"rk4"``,
``"euler"``.  Interpolation: ``"linear"``, ``"hermite"``, ``"bilinear"``.

Every function here is pinned, independently of itself, by
``tests/test_oracle_pins.py`` and ``tests/test_oracle_paper.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nv_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_CB_SRC = os.path.join(_HERE, "cpu_build.c")
_CB_LIB = os.path.join(_HERE, "libcpubuild.so")

_RHS = {"linear": 10, "logistic": 11, "forced_cubic": 12, "vdp": 13, "square": 14}
_SCHEME = {"rk4": 1, "euler": 2}
_INTERP = {"linear": 1, "hermite": 2, "bilinear": 3, "hermite_slopes": 4}
OK, BAD_ARG, NONFINITE = 0, 1, 2

_lib = None


def build() -> str:
    """Compile the oracle with gcc (FP64, one rounding per operation), and the
    CPU throughput baseline beside it (cpu_build.c, OpenMP)."""
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    cmd = ["gcc", "-std=c99", "-O3", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", _CB_LIB + ".tmp", _CB_SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_CB_LIB + ".tmp", _CB_LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 2),
                ("lo", ctypes.c_double * 2), ("hi", ctypes.c_double * 2)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    D, I, LL = ctypes.c_double, ctypes.c_int, ctypes.c_longlong
    P = ctypes.c_void_p
    G = ctypes.POINTER(_Grid)
    sig = {
        "orc_rhs_dim": (I, [I]),
        "orc_integrate": (I, [I, P, I, D, D, LL, P]),
        "orc_serial": (I, [I, P, I, D, D, I, I, P, P]),
        "orc_serial_steps": (I, [I, P, I, D, D, LL, P, P]),
        "orc_grid_point": (I, [G, LL, P]),
        "orc_build_tables": (I, [I, P, I, D, D, I, G, I, P]),
        "orc_table_entries": (I, [I, P, I, D, D, I, G, I, LL, P, P, P]),
        "orc_integrate_tangent": (I, [I, P, I, D, D, LL, ctypes.POINTER(D),
                                      ctypes.POINTER(D)]),
        "orc_build_tables_slopes": (I, [I, P, I, D, D, I, G, I, P]),
        "orc_table_entries_slopes": (I, [I, P, I, D, D, I, G, I, LL, P, P, P]),
        "orc_locate": (I, [D, D, I, D, ctypes.POINTER(LL), ctypes.POINTER(D)]),
        "orc_compose_tables": (I, [G, I, I, P, P, P, P, P, ctypes.POINTER(LL),
                                   ctypes.POINTER(I)]),
        "orc_method_lazy": (I, [I, P, I, D, D, I, G, I, I, P, P, ctypes.POINTER(LL),
                                ctypes.POINTER(I)]),
        "orc_paper_method": (I, [D, I, I, D, D, D, D, I, I, ctypes.POINTER(D)]),
        "orc_paper_nodes": (I, [I, D, D, P]),
        "orc_paper_tables": (I, [D, I, I, D, D, D, I, I, P]),
        "orc_paper_compose": (I, [I, I, D, D, P, D, P, ctypes.POINTER(LL), ctypes.POINTER(I)]),
        "orc_paper_serial": (I, [D, D, D, I, I, ctypes.POINTER(D)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


_cb = None


def _load_cpu_build():
    global _cb
    if _cb is not None:
        return _cb
    if not os.path.exists(_CB_LIB):
        build()
    lib = ctypes.CDLL(_CB_LIB)
    D, I, P = ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    for name in ("cb_build_f64", "cb_build_f32"):
        fn = getattr(lib, name)
        fn.restype = I
        fn.argtypes = [I, D, D, D, I, I, I, I, P, P, P, I, I, P]
    lib.cb_max_threads.restype = I
    lib.cb_max_threads.argtypes = []
    _cb = lib
    return lib


_CB_RHS = {"logistic": 1, "forced_cubic": 2, "vdp": 3}


def cpu_build(rhs, params, t0, T, n_slices, grid_n, grid_lo, grid_hi, steps_per_slice,
              precision="fp64", slices=None, threads=None):
    """NOT the oracle: the CPU throughput baseline of cpu_build.c (OpenMP over
    all host cores, forcing hoisted per slice, FP64 = the oracle's operations
    in its order, FP32 with blocked summation).  Tables of slices
    [slices[0], slices[1]) as an array (dim, slices, points)."""
    lib = _load_cpu_build()
    n = np.ascontiguousarray(np.atleast_1d(grid_n), dtype=np.int32)
    lo = _f64(grid_lo)
    hi = _f64(grid_hi)
    dim = n.size
    s0, s1 = slices if slices is not None else (0, n_slices)
    M = int(np.prod(n))
    dt = np.float64 if precision == "fp64" else np.float32
    tab = np.empty((dim, s1 - s0, M), dtype=dt)
    fn = lib.cb_build_f64 if precision == "fp64" else lib.cb_build_f32
    mu = float(params[0]) if params else 0.0
    th = int(threads) if threads else lib.cb_max_threads()
    rc = fn(_CB_RHS[rhs], mu, float(t0), float(T), int(n_slices), int(s0), int(s1), dim,
            _ptr(n), _ptr(lo), _ptr(hi), int(steps_per_slice), th, _ptr(tab))
    if rc != 0:
        raise OracleError(f"cpu_build: status {rc}")
    return tab


class OracleError(RuntimeError):
    pass


def _check(rc, what):
    if rc == BAD_ARG:
        raise OracleError(f"{what}: invalid argument")
    return rc


def _f64(a, n=None):
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(-1))
    if n is not None and arr.size < n:
        arr = np.concatenate([arr, np.zeros(n - arr.size)])
    return arr


def _ptr(arr):
    return arr.ctypes.data_as(ctypes.c_void_p)


def make_grid(n, lo, hi) -> _Grid:
    """Uniform grid, endpoints included; n, lo, hi are scalars (1-D) or pairs (2-D)."""
    n = np.atleast_1d(n).astype(int)
    lo = np.atleast_1d(lo).astype(float)
    hi = np.atleast_1d(hi).astype(float)
    g = _Grid()
    g.dim = len(n)
    for a in range(len(n)):
        g.n[a] = int(n[a])
        g.lo[a] = float(lo[a])
        g.hi[a] = float(hi[a])
    return g


def rhs_dim(rhs: str) -> int:
    return _load().orc_rhs_dim(_RHS[rhs])


def _params(params):
    return _f64(params if params is not None else [], 4)


def integrate(rhs, params, scheme, t_base, h, nsteps, y):
    """Integrate y over nsteps steps of h; step s runs at t_base + s h."""
    lib = _load()
    y = _f64(y).copy()
    p = _params(params)
    _check(lib.orc_integrate(_RHS[rhs], _ptr(p), _SCHEME[scheme], t_base, h, nsteps,
                             _ptr(y)), "integrate")
    return y


def serial(rhs, params, scheme, t0, T, n_slices, steps_per_slice, y0):
    """O1: the whole interval in n_slices*steps_per_slice steps of the method's h."""
    lib = _load()
    p = _params(params)
    y0 = _f64(y0)
    out = np.zeros(rhs_dim(rhs))
    _check(lib.orc_serial(_RHS[rhs], _ptr(p), _SCHEME[scheme], t0, T, n_slices,
                          steps_per_slice, _ptr(y0), _ptr(out)), "serial")
    return out


def serial_steps(rhs, params, scheme, t0, T, nsteps, y0):
    lib = _load()
    p = _params(params)
    y0 = _f64(y0)
    out = np.zeros(rhs_dim(rhs))
    _check(lib.orc_serial_steps(_RHS[rhs], _ptr(p), _SCHEME[scheme], t0, T, nsteps,
                                _ptr(y0), _ptr(out)), "serial_steps")
    return out


def grid_points(grid: _Grid):
    """All grid points, shape (Mtot, dim)."""
    lib = _load()
    M = grid.n[0] * (grid.n[1] if grid.dim == 2 else 1)
    out = np.zeros((M, grid.dim))
    buf = np.zeros(2)
    for k in range(M):
        _check(lib.orc_grid_point(ctypes.byref(grid), k, _ptr(buf)), "grid_point")
        out[k] = buf[: grid.dim]
    return out


def build_tables(rhs, params, scheme, t0, T, n_slices, grid: _Grid, steps_per_slice):
    """O2 computation phase: tables of shape (dim, n_slices, Mtot), FP64."""
    lib = _load()
    p = _params(params)
    M = grid.n[0] * (grid.n[1] if grid.dim == 2 else 1)
    tab = np.zeros((grid.dim, n_slices, M))
    _check(lib.orc_build_tables(_RHS[rhs], _ptr(p), _SCHEME[scheme], t0, T, n_slices,
                                ctypes.byref(grid), steps_per_slice, _ptr(tab)),
           "build_tables")
    return tab


def build_tables_slopes(rhs, params, scheme, t0, T, n_slices, grid: _Grid, steps_per_slice):
    """Computation phase with slopes (1-D problems): shape (2, n_slices, M), [0] the
    values, [1] their derivatives with respect to the grid point."""
    lib = _load()
    p = _params(params)
    M = grid.n[0]
    tab = np.zeros((2, n_slices, M))
    _check(lib.orc_build_tables_slopes(_RHS[rhs], _ptr(p), _SCHEME[scheme], t0, T, n_slices,
                                       ctypes.byref(grid), steps_per_slice, _ptr(tab)),
           "build_tables_slopes")
    return tab


def table_entries_slopes(rhs, params, scheme, t0, T, n_slices, grid: _Grid, steps_per_slice,
                         slices, points):
    """Selected values and slopes (1-D problems): shape (2, count)."""
    lib = _load()
    p = _params(params)
    sl = np.ascontiguousarray(np.asarray(slices, dtype=np.int64))
    pt = np.ascontiguousarray(np.asarray(points, dtype=np.int64))
    out = np.zeros((2, sl.size))
    _check(lib.orc_table_entries_slopes(_RHS[rhs], _ptr(p), _SCHEME[scheme], t0, T, n_slices,
                                        ctypes.byref(grid), steps_per_slice, sl.size, _ptr(sl),
                                        _ptr(pt), _ptr(out)), "table_entries_slopes")
    return out


def integrate_tangent(rhs, params, scheme, t_base, h, nsteps, y, v=1.0):
    """(y, dy/dy0) after nsteps steps of a 1-D problem from (y, v)."""
    lib = _load()
    p = _params(params)
    yy = ctypes.c_double(float(y))
    vv = ctypes.c_double(float(v))
    _check(lib.orc_integrate_tangent(_RHS[rhs], _ptr(p), _SCHEME[scheme], float(t_base),
                                     float(h), int(nsteps), ctypes.byref(yy), ctypes.byref(vv)),
           "integrate_tangent")
    return yy.value, vv.value


def table_entries(rhs, params, scheme, t0, T, n_slices, grid: _Grid, steps_per_slice,
                  slices, points):
    """Selected table entries: shape (dim, count)."""
    lib = _load()
    p = _params(params)
    sl = np.ascontiguousarray(np.asarray(slices, dtype=np.int64))
    pt = np.ascontiguousarray(np.asarray(points, dtype=np.int64))
    out = np.zeros((grid.dim, sl.size))
    _check(lib.orc_table_entries(_RHS[rhs], _ptr(p), _SCHEME[scheme], t0, T, n_slices,
                                 ctypes.byref(grid), steps_per_slice, sl.size, _ptr(sl),
                                 _ptr(pt), _ptr(out)), "table_entries")
    return out


def locate(lo, hi, n, x):
    """(cell, w, outside) for one query on one axis."""
    lib = _load()
    cell = ctypes.c_longlong()
    w = ctypes.c_double()
    oog = lib.orc_locate(float(lo), float(hi), int(n), float(x), ctypes.byref(cell),
                         ctypes.byref(w))
    return cell.value, w.value, bool(oog)


class ComposeResult:
    def __init__(self, status, boundary, cells, weights, n_out_of_grid, bad_slice):
        self.status = status
        self.boundary = boundary
        self.cells = cells
        self.weights = weights
        self.n_out_of_grid = n_out_of_grid
        self.bad_slice = bad_slice

    @property
    def yT(self):
        return self.boundary[-1]


def compose_tables(grid: _Grid, interp, tab, y0):
    """O2 communication phase over given FP64 tables of shape (dim, N, Mtot)."""
    lib = _load()
    tab = np.ascontiguousarray(np.asarray(tab, dtype=np.float64))
    N = tab.shape[1]
    d = grid.dim
    y0 = _f64(y0)
    boundary = np.full((N + 1, d), np.nan)
    cells = np.full((N, d), -1, dtype=np.int64)
    weights = np.full((N, d), np.nan)
    oog = ctypes.c_longlong(0)
    bad = ctypes.c_int(-1)
    rc = _check(lib.orc_compose_tables(ctypes.byref(grid), _INTERP[interp], N, _ptr(tab),
                                       _ptr(y0), _ptr(boundary), _ptr(cells),
                                       _ptr(weights), ctypes.byref(oog),
                                       ctypes.byref(bad)), "compose_tables")
    return ComposeResult(rc, boundary, cells, weights, oog.value, bad.value)


def method_lazy(rhs, params, scheme, t0, T, n_slices, grid: _Grid, steps_per_slice,
                interp, y0):
    """O2 with only the table entries the lookups touch, integrated on demand."""
    lib = _load()
    p = _params(params)
    y0 = _f64(y0)
    d = grid.dim
    boundary = np.full((n_slices + 1, d), np.nan)
    oog = ctypes.c_longlong(0)
    bad = ctypes.c_int(-1)
    rc = _check(lib.orc_method_lazy(_RHS[rhs], _ptr(p), _SCHEME[scheme], t0, T, n_slices,
                                    ctypes.byref(grid), steps_per_slice, _INTERP[interp],
                                    _ptr(y0), _ptr(boundary), ctypes.byref(oog),
                                    ctypes.byref(bad)), "method_lazy")
    return ComposeResult(rc, boundary, None, None, oog.value, bad.value)


def paper_method(T, n_slices, M, a, b, dt, y0, be_exact=False, equal_substeps=False):
    """Paper mode: y'=y^2, backward Euler, Lagrange on M Chebyshev extrema of [a,b]."""
    lib = _load()
    out = ctypes.c_double()
    _check(lib.orc_paper_method(T, n_slices, M, a, b, dt, y0, int(be_exact),
                                int(equal_substeps), ctypes.byref(out)), "paper_method")
    return out.value


def paper_nodes(M, a, b):
    lib = _load()
    out = np.zeros(M)
    _check(lib.orc_paper_nodes(M, a, b, _ptr(out)), "paper_nodes")
    return out


def paper_tables(T, n_slices, M, a, b, dt, be_exact=False, equal_substeps=False):
    """Paper mode, computation phase: tables of shape (n_slices, M)."""
    lib = _load()
    tab = np.zeros((n_slices, M))
    _check(lib.orc_paper_tables(T, n_slices, M, a, b, dt, int(be_exact), int(equal_substeps),
                                _ptr(tab)), "paper_tables")
    return tab


def paper_compose(M, a, b, tab, y0):
    """Paper mode, communication phase over given tables of shape (N, M)."""
    lib = _load()
    tab = np.ascontiguousarray(np.asarray(tab, dtype=np.float64))
    N = tab.shape[0]
    boundary = np.full(N + 1, np.nan)
    oog = ctypes.c_longlong(0)
    bad = ctypes.c_int(-1)
    rc = _check(lib.orc_paper_compose(N, M, a, b, _ptr(tab), float(y0), _ptr(boundary),
                                      ctypes.byref(oog), ctypes.byref(bad)), "paper_compose")
    return ComposeResult(rc, boundary[:, None], None, None, oog.value, bad.value)


def paper_serial(T, dt, y0, be_exact=False, equal_substeps=False):
    lib = _load()
    out = ctypes.c_double()
    _check(lib.orc_paper_serial(T, dt, y0, int(be_exact), int(equal_substeps),
                                ctypes.byref(out)), "paper_serial")
    return out.value
