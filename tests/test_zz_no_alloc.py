"""nv_solve_static (the entry point that allocates nothing) against nv_solve.

Both run the same build and composition kernels; nv_solve_static keeps its
scratch in the library's static device array instead of context memory.  The
bar is bit-exactness of the tables, the boundary states and the status, on
consecutive calls that shrink (the static scratch keeps the previous call's
contents), plus the host-side rejections that launch nothing.
"""
import ctypes
import sys

import numpy as np
import pytest

from paper_1304_6514_amd import nv
from paper_1304_6514_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nv.load()          # raises when libnv.so is missing: no fallback
    return torch


def _options(torch, w):
    return nv.make_options(w.scheme, w.precision, 2, 0,
                           torch.cuda.current_stream().cuda_stream, 0, w.dt)


def _grid(w):
    return nv.make_grid(w.grid_n, w.grid_lo, w.grid_hi, w.interp)


def components(w):
    """Tables of a build: one per state component, plus the slopes."""
    return w.dim + (1 if w.interp == "hermite_slopes" else 0)


def solve_static(torch, w, sentinel=-7.0):
    """Tables (one tensor per component), boundary (N+1, dim) and the status
    of one nv_solve_static call; every output starts filled with a sentinel."""
    opt = _options(torch, w)
    g = _grid(w)
    rhs = nv.RHS_IDS[w.rhs]
    tb, wb = nv.nv_required_bytes(rhs, w.n_slices, g, w.steps_per_slice, opt)
    assert wb <= nv.NV_STATIC_SCRATCH_BYTES
    tables = torch.full((tb,), 0xA5, dtype=torch.uint8, device="cuda:0")
    boundary = torch.full(((w.n_slices + 1) * w.dim,), sentinel, dtype=torch.float64,
                          device="cuda:0")
    status = torch.full((2,), -1, dtype=torch.int64, device="cuda:0")
    say("nv_solve_static", w.name, "table bytes", tb, "scratch bytes", wb)
    nv.nv_solve_static(rhs, w.params, w.t0, w.T, w.n_slices, g, w.steps_per_slice, opt,
                       tables.data_ptr(), tb, w.y0, boundary.data_ptr(), status.data_ptr())
    torch.cuda.synchronize()
    elem = 8 if w.precision == "fp64" else 4
    n = w.n_slices * w.points_per_slice
    comp = (n * elem + 255) // 256 * 256
    dt = torch.float64 if w.precision == "fp64" else torch.float32
    tabs = [tables[c * comp:c * comp + n * elem].view(dt).view(w.n_slices, w.points_per_slice)
            for c in range(components(w))]
    st = status.cpu().numpy()
    n_oog = int(st[0])
    bad_slice, done = (int(v) for v in st[1:2].view(np.int32))
    return tabs, boundary.cpu().numpy().reshape(w.n_slices + 1, w.dim), (n_oog, bad_slice, done)


def solve_ctx(torch, w):
    from paper_1304_6514_amd.propagator import Propagator
    p = Propagator("cuda:0")
    say("nv_solve", w.name)
    res = p.solve(w)
    torch.cuda.synchronize()
    return p, res


# consecutive calls, each smaller than the one before: the full forced-cubic
# workload (its forcing rows precomputed into the static scratch), a small
# forced build whose workgroups form their rows in LDS, a ragged 2-D Van der
# Pol build, a forced build with stored slopes, a 1-D FP64 logistic build
SEQUENCE = [
    W.FORCED_CUBIC_FP32,
    W.small(W.FORCED_CUBIC_FP32, 64, (1000,), 30),
    W.small(W.VDP_FP32, 16, (37, 29), 20),
    W.small(W.FORCED_CUBIC_FP32, 12, (700,), 25).with_(interp="hermite_slopes"),
    W.small(W.LOGISTIC_FP64, 8, (301,), 40),
]


def test_static_solve_equals_solve_on_shrinking_calls(torch):
    for w in SEQUENCE:
        p, ref = solve_ctx(torch, w)
        try:
            assert ref.status == nv.NV_OK
            tabs, boundary, (n_oog, bad_slice, done) = solve_static(torch, w)
            iv = torch.int64 if w.precision == "fp64" else torch.int32
            for c in range(components(w)):
                # bit for bit, NaN patterns included
                assert torch.equal(tabs[c].view(iv), p.table_tensor(c).view(iv)), \
                    f"{w.name}: component {c} table differs"
            assert np.array_equal(boundary.view(np.int64), ref.boundary.view(np.int64)), \
                f"{w.name}: boundary states differ"
            assert (n_oog, bad_slice, done) == (ref.n_out_of_grid, ref.bad_slice, 1)
            say(w.name, "bit-exact; y(T) =", boundary[-1].tolist(), "out of grid", n_oog)
        finally:
            p.close()


def test_static_solve_reports_a_failing_chain_like_solve(torch):
    # y' = y^2 blows up at t = 1/y0 inside the interval (and grid points above
    # 1/L within a slice): both chains stop at the same slice
    w = W.Workload("square-blowup-static", "square", (), 0.0, 6.0, 6, (8,), (0.0,), (4.0,),
                   100, (0.3,), "fp64", "linear")
    p, ref = solve_ctx(torch, w)
    try:
        assert ref.status == nv.NV_ERR_NONFINITE and ref.bad_slice >= 0
        tabs, boundary, (n_oog, bad_slice, done) = solve_static(torch, w)
        assert (n_oog, bad_slice, done) == (ref.n_out_of_grid, ref.bad_slice, 1)
        k = ref.bad_slice + 1
        assert np.array_equal(boundary[:k].view(np.int64), ref.boundary[:k].view(np.int64))
        for c in range(w.dim):
            want = p.table_tensor(c)
            assert torch.equal(tabs[c].view(torch.int64), want.view(torch.int64))
    finally:
        p.close()


def test_static_solve_rejections_launch_nothing(torch):
    t = torch.empty(1 << 20, dtype=torch.uint8, device="cuda:0")
    b = torch.empty(1 << 16, dtype=torch.float64, device="cuda:0")
    s = torch.empty(2, dtype=torch.int64, device="cuda:0")

    def call(w, tables_ptr, table_bytes):
        opt = _options(torch, w)
        return nv.load().nv_solve_static(
            nv.RHS_IDS[w.rhs], nv._ptr(np.asarray(w.params or (0.0,), dtype=np.float64)),
            w.t0, w.T, w.n_slices, ctypes.byref(_grid(w)), w.steps_per_slice,
            ctypes.byref(opt), tables_ptr, table_bytes,
            nv._ptr(np.asarray(w.y0, dtype=np.float64)), b.data_ptr(), s.data_ptr())

    # scratch beyond the static array: FP64 forcing rows of the full forced cubic
    # (the table size passes; the scratch check comes before any launch)
    big = W.FORCED_CUBIC_FP32.with_(precision="fp64")
    assert call(big, t.data_ptr(), 1 << 40) == nv.NV_ERR_BUFFER_TOO_SMALL
    assert "static scratch" in nv.nv_last_error()
    small = W.small(W.FORCED_CUBIC_FP32, 64, (1000,), 30)
    # tables larger than the caller's buffer
    assert call(small, t.data_ptr(), 1024) == nv.NV_ERR_BUFFER_TOO_SMALL
    # a table address that is not 256-byte aligned
    assert call(small, t.data_ptr() + 8, t.numel() - 8) == nv.NV_ERR_INVALID_ARG
    # paper mode's Chebyshev nodes come from host memory
    cheb = W.paper_model(4, 5, 2.0 ** -10)
    assert call(cheb, t.data_ptr(), t.numel()) == nv.NV_ERR_UNSUPPORTED
    torch.cuda.synchronize()
