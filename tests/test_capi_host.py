"""Host-side checks of the C ABI: the library loads, exports every entry point
the headers under include/ declare, and its argument checking answers without
a GPU (every call here returns before touching the HIP runtime)."""
import ctypes
import glob
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(glob.glob(os.path.join(ROOT, "include", "*.h")))


@pytest.fixture(scope="module")
def nvmod():
    from paper_1304_6514_amd import nv
    if not os.path.exists(nv.LIB_PATH):
        from paper_1304_6514_amd import _build
        _build.build()
    nv.load()
    return nv


def declared_entry_points():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"NV_API\s+[^;(]*?\b(nv_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for must in ("nv_build_propagators", "nv_compose", "nv_solve", "nv_ctx_create",
                 "nv_ctx_destroy",
                 "nv_set_options", "nv_set_buffers", "nv_required_bytes", "nv_get_table",
                 "nv_locate", "nv_last_error", "nv_sur_create", "nv_sur_train",
                 "nv_sur_loss_grad", "nv_sur_compose", "nv_sur_dataset_from_batch"):
        assert must in names


def test_library_exports_every_declared_symbol(nvmod):
    lib = ctypes.CDLL(nvmod.LIB_PATH)
    missing = [n for n in declared_entry_points() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_every_entry_point(nvmod):
    for name in declared_entry_points():
        assert name in nvmod._SIGNATURES, name


def test_status_strings(nvmod):
    assert nvmod.status_name(0) == "NV_OK"
    assert nvmod.status_name(-3) == "NV_ERR_NONFINITE"
    assert nvmod.status_name(-7) == "NV_ERR_BUFFER_TOO_SMALL"


def _grid(nvmod, n=(256,), lo=(-0.1,), hi=(1.2,), interp="linear"):
    return nvmod.make_grid(n, lo, hi, interp)


def test_required_bytes_layout(nvmod):
    g = _grid(nvmod, (4096,), (-3.0,), (3.0,), "hermite")
    o = nvmod.make_options("rk4", "fp32")
    tb, wb = nvmod.nv_required_bytes(nvmod.NV_RHS_FORCED_CUBIC, 4096, g, 2000, o)
    assert tb == 4096 * 4096 * 4                         # 64 MiB, one FP32 component
    # forcing values + one non-finite count per tile (8 tiles of 512 points per slice; the
    # boundary states go to mapped host memory)
    assert 4096 * 4001 * 4 + 4096 * 8 * 4 <= wb < 4096 * 4001 * 4 + 4096 * 8 * 4 + 4097 * 8 + 4096
    g2 = _grid(nvmod, (128, 128), (-3.0, -8.0), (3.0, 8.0), "bilinear")
    tb2, _ = nvmod.nv_required_bytes(nvmod.NV_RHS_VDP, 1024, g2, 500, o)
    assert tb2 == 2 * 1024 * 128 * 128 * 4               # two 64 MiB tables
    tb3, _ = nvmod.nv_required_bytes(nvmod.NV_RHS_LOGISTIC, 64, _grid(nvmod), 1000,
                                     nvmod.make_options("rk4", "fp64"))
    assert tb3 == 64 * 256 * 8
    # stored slopes: a second table of the same size
    gs = _grid(nvmod, (4096,), (-3.0,), (3.0,), "hermite_slopes")
    tb4, wb4 = nvmod.nv_required_bytes(nvmod.NV_RHS_FORCED_CUBIC, 4096, gs, 2000, o)
    assert tb4 == 2 * tb and wb4 == wb


def test_slopes_configurations_need_no_gpu(nvmod):
    # a 2-D problem or a 2-D grid has no stored-slope lookup
    g2 = _grid(nvmod, (8, 8), (0.0, 0.0), (1.0, 1.0), "hermite_slopes")
    with pytest.raises(nvmod.NvError) as e:
        nvmod.nv_required_bytes(nvmod.NV_RHS_VDP, 4, g2, 10)
    assert e.value.status == nvmod.NV_ERR_INVALID_ARG
    g1 = _grid(nvmod, (8,), (0.0,), (1.0,), "hermite_slopes")
    with pytest.raises(nvmod.NvError) as e:
        nvmod.nv_required_bytes(nvmod.NV_RHS_VDP, 4, g1, 10)
    assert e.value.status == nvmod.NV_ERR_INVALID_ARG
    # the slopes are integrated with RK4 or forward Euler only
    with pytest.raises(nvmod.NvError) as e:
        nvmod.nv_required_bytes(nvmod.NV_RHS_SQUARE, 4, g1, 10, nvmod.make_options("be", "fp64"))
    assert e.value.status == nvmod.NV_ERR_UNSUPPORTED
    tb, _ = nvmod.nv_required_bytes(nvmod.NV_RHS_SQUARE, 4, g1, 10,
                                    nvmod.make_options("euler", "fp64"))
    assert tb == 2 * 256            # two tables of 4 x 8 doubles, each aligned to 256 bytes


@pytest.mark.parametrize("case", [
    dict(rhs=99), dict(n_slices=0), dict(steps=0), dict(n=(1,)),
    dict(lo=(1.0,), hi=(1.0,)), dict(lo=(float("nan"),)), dict(interp="bilinear"),
    dict(n=(2,), interp="hermite"), dict(rhs=3),                 # vdp needs a 2-D grid
    dict(n=(70000, 70000), lo=(0, 0), hi=(1, 1), interp="bilinear", rhs=3),  # > 2^31 points
])
def test_required_bytes_rejects_bad_shapes(nvmod, case):
    rhs = case.get("rhs", nvmod.NV_RHS_LOGISTIC)
    g = _grid(nvmod, case.get("n", (256,)), case.get("lo", (-0.1,)), case.get("hi", (1.2,)),
              case.get("interp", "linear"))
    with pytest.raises(nvmod.NvError) as e:
        nvmod.nv_required_bytes(rhs, case.get("n_slices", 64), g, case.get("steps", 1000))
    assert e.value.status == nvmod.NV_ERR_INVALID_ARG


def test_options_validation(nvmod):
    ctx = nvmod.nv_ctx_create()
    try:
        for bad in (dict(scheme=5), dict(precision=7), dict(traj_per_lane=3),
                    dict(compensated=3), dict(solve_chunks=-1), dict(solve_chunks=65)):
            o = nvmod.make_options(**{**dict(scheme=0, precision=0), **bad})
            with pytest.raises(nvmod.NvError) as e:
                nvmod.nv_set_options(ctx, o)
            assert e.value.status == nvmod.NV_ERR_INVALID_ARG
        good = nvmod.make_options("euler", "fp32", 2, 4, None, 7)
        nvmod.nv_set_options(ctx, good)
        back = nvmod.nv_get_options(ctx)
        assert (back.scheme, back.precision, back.compensated, back.traj_per_lane,
                back.solve_chunks) == (1, 1, 2, 4, 7)
    finally:
        nvmod.nv_ctx_destroy(ctx)


def test_build_argument_errors_need_no_gpu(nvmod):
    ctx = nvmod.nv_ctx_create()
    try:
        g = _grid(nvmod)
        cases = [
            (nvmod.NV_RHS_LOGISTIC, None, 0.0, 10.0, 0, g, 1000),
            (nvmod.NV_RHS_LOGISTIC, None, 10.0, 0.0, 64, g, 1000),          # T <= t0
            (nvmod.NV_RHS_LOGISTIC, None, 0.0, float("inf"), 64, g, 1000),
            (nvmod.NV_RHS_LINEAR, [float("nan")], 0.0, 1.0, 4, g, 10),      # bad parameter
        ]
        for args in cases:
            with pytest.raises(nvmod.NvError) as e:
                nvmod.nv_build_propagators(ctx, *args)
            assert e.value.status == nvmod.NV_ERR_INVALID_ARG
            assert nvmod.nv_last_error()
        # nothing built: compose and inspection refuse
        assert nvmod.load().nv_compose(ctx, None, None, None, None) == nvmod.NV_ERR_NOT_BUILT
        with pytest.raises(nvmod.NvError) as e:
            nvmod.nv_compose(ctx, [0.1], 1, 64)
        assert e.value.status == nvmod.NV_ERR_NOT_BUILT
        with pytest.raises(nvmod.NvError) as e:
            nvmod.nv_get_table(ctx, 0, 64, 256, "fp64")
        assert e.value.status == nvmod.NV_ERR_NOT_BUILT
    finally:
        nvmod.nv_ctx_destroy(ctx)


def test_null_context_and_destroy_null(nvmod):
    lib = nvmod.load()
    assert lib.nv_ctx_destroy(None) == 0
    assert lib.nv_set_timing(None, 1) == nvmod.NV_ERR_INVALID_ARG
    assert lib.nv_build_propagators(None, 0, None, 0.0, 1.0, 1, None, 1) == \
        nvmod.NV_ERR_INVALID_ARG
    assert lib.nv_solve(None, 0, None, 0.0, 1.0, 1, None, 1, None, None, None, None) == \
        nvmod.NV_ERR_INVALID_ARG


def test_solve_static_argument_errors_need_no_gpu(nvmod):
    # every rejection happens before the library looks up its static scratch
    # (its first HIP call): the device addresses below are never touched
    lib = nvmod.load()
    fake_tab, fake_b, fake_s = 0x10000, 0x20000, 0x30000
    y0 = np.array([0.1])
    p0 = np.zeros(1)

    def call(grid, n_slices=64, steps=1000, opt=None, tab=fake_tab, tab_bytes=1 << 40,
             y=y0, rhs=nvmod.NV_RHS_LOGISTIC, t0=0.0, T=10.0):
        o = opt if opt is not None else nvmod.make_options(precision="fp32")
        return lib.nv_solve_static(rhs, nvmod._ptr(p0), t0, T, n_slices, ctypes.byref(grid),
                                   steps, ctypes.byref(o), tab, tab_bytes,
                                   nvmod._ptr(y) if y is not None else None, fake_b, fake_s)

    g = _grid(nvmod)
    assert lib.nv_solve_static(1, None, 0.0, 1.0, 1, ctypes.byref(g), 1, None, fake_tab, 1,
                               nvmod._ptr(y0), fake_b, fake_s) == nvmod.NV_ERR_INVALID_ARG
    assert call(g, y=None) == nvmod.NV_ERR_INVALID_ARG
    assert call(g, tab=fake_tab + 8) == nvmod.NV_ERR_INVALID_ARG       # not 256-byte aligned
    assert call(g, n_slices=0) == nvmod.NV_ERR_INVALID_ARG
    assert call(g, t0=1.0, T=1.0) == nvmod.NV_ERR_INVALID_ARG
    assert call(_grid(nvmod, n=(5,), lo=(0.0,), hi=(2.0,), interp="chebyshev"),
                rhs=nvmod.NV_RHS_SQUARE) == nvmod.NV_ERR_UNSUPPORTED
    assert call(g, tab_bytes=1024) == nvmod.NV_ERR_BUFFER_TOO_SMALL     # tables too small
    assert "tables need" in nvmod.nv_last_error()
    # FP64 forcing rows of 4096 slices x 2000 steps: 131 MB > the static scratch
    big = _grid(nvmod, n=(4096,), lo=(-3.0,), hi=(3.0,), interp="hermite")
    assert call(big, n_slices=4096, steps=2000, rhs=nvmod.NV_RHS_FORCED_CUBIC, T=100.0,
                opt=nvmod.make_options(precision="fp64")) == nvmod.NV_ERR_BUFFER_TOO_SMALL
    assert "static scratch" in nvmod.nv_last_error()
    # the FP32 build of the same shape fits
    _, wb = nvmod.nv_required_bytes(nvmod.NV_RHS_FORCED_CUBIC, 4096, big, 2000,
                                    nvmod.make_options(precision="fp32"))
    assert wb <= nvmod.NV_STATIC_SCRATCH_BYTES


def test_product_path_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1304_6514_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "nv_oracle" not in text, f


def test_batch_argument_errors_need_no_gpu(nvmod):
    ctx = nvmod.nv_ctx_create()
    try:
        g = _grid(nvmod)
        good = nvmod.make_problem("logistic", [], 0.0, 10.0, 64, g, 100, [0.1])
        forced = nvmod.make_problem("forced_cubic", [], 0.0, 10.0, 64,
                                    _grid(nvmod, (100,), (-3.0,), (3.0,), "hermite"), 100, [1.0])
        bad = nvmod.make_problem("logistic", [], 0.0, 10.0, 0, g, 100, [0.1])
        with pytest.raises(nvmod.NvError) as e:
            nvmod.nv_batch_create(ctx, [good, forced])
        assert e.value.status == nvmod.NV_ERR_UNSUPPORTED and "problem 1" in str(e.value)
        with pytest.raises(nvmod.NvError) as e:
            nvmod.nv_batch_create(ctx, [good, good, bad])
        assert e.value.status == nvmod.NV_ERR_INVALID_ARG and "problem 2" in str(e.value)
        slopes = nvmod.make_problem("logistic", [], 0.0, 10.0, 64,
                                    _grid(nvmod, interp="hermite_slopes"), 100, [0.1])
        with pytest.raises(nvmod.NvError) as e:
            nvmod.nv_batch_create(ctx, [good, slopes])
        assert e.value.status == nvmod.NV_ERR_UNSUPPORTED and "problem 1" in str(e.value)
        lib = nvmod.load()
        assert lib.nv_batch_create(ctx, None, 0, None) == nvmod.NV_ERR_INVALID_ARG
        assert lib.nv_batch_destroy(None) == 0
        assert lib.nv_batch_run(None, None, None) == nvmod.NV_ERR_INVALID_ARG
    finally:
        nvmod.nv_ctx_destroy(ctx)


def test_batched_workload_recipe():
    from paper_1304_6514_amd import workloads as W
    probs = W.batched_problems()
    assert len(probs) == 96 and probs == W.batched_problems()       # seeded
    assert {w.rhs for w in probs} == {"linear", "logistic", "vdp"}
    for w in probs:
        assert 16 <= w.n_slices <= 2048 and 100 <= w.steps_per_slice <= 2000
        if w.dim == 1:
            assert 64 <= w.grid_n[0] <= 8192
        else:
            assert all(16 <= n <= 256 for n in w.grid_n)
        if w.rhs == "linear":
            assert -2.0 <= w.params[0] <= 0.5
        if w.rhs == "vdp":
            assert 1.0 <= w.params[0] <= 5.0


def test_surrogate_argument_errors_need_no_gpu(nvmod):
    from paper_1304_6514_amd import workloads as W
    lib = nvmod.load()
    good = dict(in_shift=W.SUR_IN_SHIFT, in_scale=W.SUR_IN_SCALE, out_scale=W.SUR_OUT_SCALE,
                slice_length=W.SUR_SLICE_LENGTH, coarse_steps=0, max_batch=0)
    for bad in (dict(out_scale=(0.2, 0.0)), dict(out_scale=(float("nan"), 1.0)),
                dict(in_scale=(1.0, float("inf"), 1.0, 1.0)), dict(max_batch=24),
                dict(max_batch=(1 << 20) + 16), dict(slice_length=0.0),
                dict(slice_length=float("inf")), dict(coarse_steps=-1), dict(coarse_steps=17)):
        kw = dict(good, **bad)
        cfg = nvmod.make_sur_config(kw["in_shift"], kw["in_scale"], kw["out_scale"],
                                    kw["slice_length"], kw["coarse_steps"], kw["max_batch"])
        h = ctypes.c_void_p()
        assert lib.nv_sur_create(ctypes.byref(cfg), ctypes.byref(h)) == nvmod.NV_ERR_INVALID_ARG
        assert h.value is None
    assert lib.nv_sur_create(None, None) == nvmod.NV_ERR_INVALID_ARG
    assert lib.nv_sur_destroy(None) == 0
    for fn, args in (("nv_sur_set_params", (None, None)), ("nv_sur_get_params", (None, None)),
                     ("nv_sur_forward", (None, None, 1, None)),
                     ("nv_sur_loss_grad", (None, None, None, 16, None, None)),
                     ("nv_sur_train", (None, None, None, 16, None, None)),
                     ("nv_sur_compose", (None, None, None)),
                     ("nv_sur_last_ms", (None, None))):
        assert getattr(lib, fn)(*args) == nvmod.NV_ERR_INVALID_ARG, fn
    assert "NULL" in nvmod.nv_last_error()


def test_surrogate_input_recipe():
    from paper_1304_6514_amd import workloads as W
    probs = W.surrogate_training_problems()
    assert len(probs) == 1024
    assert sum(p.points_per_slice * p.n_slices for p in probs) == 16777216
    mus = np.array([p.params[0] for p in probs])
    assert mus.min() >= 1.0 and mus.max() <= 5.0 and abs(mus.mean() - 3.0) < 0.15
    L = 50.0 / 1024
    assert all(abs(p.t0 - j * L) < 1e-12 and abs(p.T - p.t0 - L) < 1e-12
               for j, p in enumerate(probs))
    p = W.surrogate_init_params(0)
    assert p.dtype == np.float32 and p.size == 33922
    assert np.abs(p[:512]).max() <= 0.5 and np.abs(p[640:640 + 16384]).max() <= 1 / np.sqrt(128)
    perm = W.surrogate_perm(1000, seed=1)
    assert np.array_equal(np.sort(perm), np.arange(1000))


def test_linear_argument_errors_need_no_gpu(nvmod):
    lib = nvmod.load()
    assert lib.nv_lin_create(None, None) == nvmod.NV_ERR_INVALID_ARG
    assert lib.nv_lin_destroy(None) == 0
    h = nvmod.make_heat(9)
    assert lib.nv_lin_build(None, ctypes.byref(h), 0.0, 1.0, 4, 0.01) == nvmod.NV_ERR_INVALID_ARG
    assert lib.nv_lin_compose(None, None, None, None) == nvmod.NV_ERR_INVALID_ARG
    assert lib.nv_lin_compose_many(None, None, 4, None, None) == nvmod.NV_ERR_INVALID_ARG
    assert lib.nv_lin_get_tables(None, None, None) == nvmod.NV_ERR_INVALID_ARG
    assert lib.nv_lin_last_timing(None, None, None) == nvmod.NV_ERR_INVALID_ARG


def test_probe_argument_errors_need_no_gpu(nvmod):
    lib = nvmod.load()
    ns, cyc = ctypes.c_double(), ctypes.c_double()
    for prec, ops, chains in [(nvmod.NV_FP64, 1000, 1), (nvmod.NV_FP64, 1 << 20, 3),
                              (7, 1 << 20, 1), (nvmod.NV_FP32, 1 << 20, 0)]:
        assert lib.nv_probe_fma_chains(prec, ops, chains, None, ctypes.byref(ns),
                                       ctypes.byref(cyc)) == nvmod.NV_ERR_INVALID_ARG
    assert lib.nv_probe_fma_chains(nvmod.NV_FP64, 1 << 20, 1, None, None,
                                   ctypes.byref(cyc)) == nvmod.NV_ERR_INVALID_ARG


def test_prepared_solve_call_marshals_once_and_reports_errors(nvmod):
    # nv_solve's arguments marshalled once (no GPU needed: a NULL context is
    # rejected before any HIP call, and the error is raised like nv_solve's)
    from paper_1304_6514_amd import workloads as W
    nv = nvmod
    w = W.LOGISTIC_FP64
    g = nv.make_grid(w.grid_n, w.grid_lo, w.grid_hi, w.interp)
    call = nv.SolveCall(nv.RHS_IDS[w.rhs], w.params, w.t0, w.T, w.n_slices, g,
                        w.steps_per_slice, w.dim)
    assert call._boundary.shape == (w.n_slices + 1, w.dim)
    for _ in range(2):
        with pytest.raises(nv.NvError) as e:
            call(None, w.y0)
        assert e.value.status == nv.NV_ERR_INVALID_ARG
    assert np.array_equal(call._y0, np.asarray(w.y0))
    assert nv.SolveCall(nv.RHS_IDS[w.rhs], w.params, w.t0, w.T, w.n_slices, g,
                        w.steps_per_slice, w.dim, want_boundary=False)._boundary is None
    comp = nv.ComposeCall(w.n_slices, w.dim)
    with pytest.raises(nv.NvError) as e:
        comp(None, w.y0)
    assert e.value.status == nv.NV_ERR_INVALID_ARG
