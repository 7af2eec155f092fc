"""GPU parity of the slope tables and of cubic Hermite with stored slopes
(NV_INTERP_HERMITE_SLOPES), through the C ABI, against the CPU oracle.

Bars (as for the value tables):
  - values and slopes: |gpu - oracle| <= tol * max(|oracle|, 1), tol = 1e-12
    for FP64 builds and 1e-5 for FP32 builds (the slope is integrated with the
    value, in the same precision and with the same state accumulation);
  - the value table of a slope build equals the plain build's to the bit (the
    value component is formed by the same operations);
  - the composition over the GPU's own values and slopes: bit-exact against the
    oracle's (same basis, same sum, one rounding per operation).
"""
import sys

import numpy as np
import pytest

from paper_1304_6514_amd import nv
from paper_1304_6514_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def say(*a):
    print("[gpu-test]", *a, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nv.load()          # raises when libnv.so is missing: no fallback
    return torch


@pytest.fixture(scope="module")
def prop(torch):
    from paper_1304_6514_amd.propagator import Propagator
    p = Propagator("cuda:0")
    yield p
    p.close()


def ogrid(orc, w):
    return orc.make_grid(w.grid_n, w.grid_lo, w.grid_hi)


def mixed_err(g, o):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1.0)))


def slope_tables(prop, w):
    return np.stack([prop.table(0).astype(np.float64), prop.table(1).astype(np.float64)])


def check_compose(orc, prop, w, tab, y0):
    g = prop.compose(y0)
    o = orc.compose_tables(ogrid(orc, w), "hermite_slopes", tab, y0)
    assert g.status == (nv.NV_OK if o.status == 0 else nv.NV_ERR_NONFINITE)
    assert g.n_out_of_grid == o.n_out_of_grid
    if o.status == 0:
        assert np.array_equal(g.boundary.view(np.int64), o.boundary.view(np.int64)), \
            np.max(np.abs(g.boundary - o.boundary))
    else:
        assert g.bad_slice == o.bad_slice
    return g, o


SMALL = [
    # ragged grids (not multiples of 256), several tiles, offset slices
    W.Workload("logistic-slopes", "logistic", (), 0.0, 3.0, 5, (700,), (-0.1,), (1.2,), 60,
               (0.1,), "fp64", "hermite_slopes"),
    W.Workload("linear-slopes", "linear", (-1.3,), 0.25, 2.25, 6, (301,), (-2.0,), (2.0,), 40,
               (1.5,), "fp64", "hermite_slopes"),
    W.Workload("fcub-slopes-32", "forced_cubic", (), 0.5, 4.5, 7, (1000,), (-3.0,), (3.0,), 80,
               (1.0,), "fp32", "hermite_slopes"),
    W.Workload("fcub-slopes-64", "forced_cubic", (), 0.5, 4.5, 7, (1000,), (-3.0,), (3.0,), 80,
               (1.0,), "fp64", "hermite_slopes"),
    W.Workload("square-slopes", "square", (), 0.0, 0.5, 4, (257,), (0.0,), (2.0,), 100,
               (1.0,), "fp64", "hermite_slopes"),
    W.Workload("logistic-slopes-2pt", "logistic", (), 0.0, 1.0, 3, (2,), (0.2,), (0.9,), 30,
               (0.5,), "fp64", "hermite_slopes"),
]


@pytest.mark.parametrize("scheme", ["rk4", "euler"])
@pytest.mark.parametrize("w", SMALL, ids=[w.name for w in SMALL])
def test_slope_tables_and_compose(orc, prop, w, scheme):
    w = w.with_(scheme=scheme)
    say("slopes", w.name, scheme, w.n_slices, w.grid_n, w.steps_per_slice)
    prop.build(w)
    tab = slope_tables(prop, w)
    ref = orc.build_tables_slopes(w.rhs, w.params, scheme, w.t0, w.T, w.n_slices, ogrid(orc, w),
                                  w.steps_per_slice)
    assert np.all(np.isfinite(ref))
    ev, es = mixed_err(tab[0], ref[0]), mixed_err(tab[1], ref[1])
    say(f"  value error {ev:.3g}, slope error {es:.3g}")
    assert ev <= TOL[w.precision] and es <= TOL[w.precision], (ev, es)
    assert np.all(prop.nonfinite_counts() == 0)
    # the value table is the plain build's, to the bit
    plain = prop.table(0).copy()
    prop.build(w.with_(interp="hermite" if w.grid_n[0] >= 3 else "linear"))
    assert np.array_equal(prop.table(0), plain)
    prop.build(w)
    for y0 in [w.y0, tuple(v + 0.37 for v in w.y0), tuple(hi + 0.5 for hi in w.grid_hi)]:
        check_compose(orc, prop, w, tab, y0)


@pytest.mark.parametrize("chunks", [3, 0])
def test_slopes_solve_equals_build_then_compose(orc, torch, chunks):
    from paper_1304_6514_amd.propagator import Propagator
    w = SMALL[2]
    say("slopes solve", w.name, chunks)
    with Propagator("cuda:0") as a, Propagator("cuda:0", solve_chunks=chunks) as b:
        a.build(w)
        ra = a.compose()
        rb = b.solve(w)
        assert rb.status == ra.status == nv.NV_OK
        assert np.array_equal(ra.boundary, rb.boundary)
        for c in range(2):
            assert np.array_equal(a.table(c), b.table(c))


def test_slopes_blowup_is_reported_like_the_oracle(orc, prop):
    # y' = y^2 from y0 beyond the grid's blow-up time: non-finite values and slopes
    w = W.Workload("square-slopes-blowup", "square", (), 0.0, 6.0, 6, (8,), (0.0,), (4.0,), 100,
                   (0.3,), "fp64", "hermite_slopes")
    say("slopes blowup")
    prop.build(w)
    tab = slope_tables(prop, w)
    assert np.any(prop.nonfinite_counts() > 0)
    g, o = check_compose(orc, prop, w, tab, w.y0)
    assert o.status == orc.NONFINITE


def test_logistic_full_size_slopes_beat_finite_differences(orc, prop):
    # the logistic workload's shape (64 slices, 256 points, 1000 steps, FP64)
    base = W.LOGISTIC_FP64
    w = base.with_(name=base.name + "-slopes", interp="hermite_slopes")
    say("full", w.name)
    prop.build(w)
    tab = slope_tables(prop, w)
    g = ogrid(orc, w)
    ref = orc.build_tables_slopes(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices, g,
                                  w.steps_per_slice)
    assert mixed_err(tab[0], ref[0]) <= TOL["fp64"]
    assert mixed_err(tab[1], ref[1]) <= TOL["fp64"]
    gres, _ = check_compose(orc, prop, w, tab, w.y0)
    ser = orc.serial(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices, w.steps_per_slice,
                     w.y0)[0]
    errs = {"hermite_slopes": abs(gres.yT[0] - ser)}
    for interp in ("linear", "hermite"):
        prop.build(w.with_(interp=interp))
        errs[interp] = abs(prop.compose().yT[0] - ser)
    say("logistic method error vs serial by interpolant", errs)
    # order 4 against order 3 against order 2 on the same 256-point grid
    assert errs["hermite_slopes"] < errs["hermite"] / 10 < errs["linear"] / 100


def test_forced_cubic_fp32_slopes_sampled(orc, prop):
    w = W.Workload("fcub-slopes-mid", "forced_cubic", (), 0.0, 100.0, 512, (4096,), (-3.0,),
                   (3.0,), 500, (1.0,), "fp32", "hermite_slopes")
    say("mid", w.name)
    prop.build(w)
    sl, pt = W.sample_entries(w, 4096, seed=21)
    ref = orc.table_entries_slopes(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices,
                                   ogrid(orc, w), w.steps_per_slice, sl, pt)
    got = np.stack([prop.table_tensor(c)[sl, pt].double().cpu().numpy() for c in range(2)])
    ev, es = mixed_err(got[0], ref[0]), mixed_err(got[1], ref[1])
    say(f"  sampled value error {ev:.3g}, slope error {es:.3g}")
    assert ev <= TOL["fp32"] and es <= TOL["fp32"]
    tab = slope_tables(prop, w)
    check_compose(orc, prop, w, tab, w.y0)


def test_slopes_argument_errors(prop, torch):
    from paper_1304_6514_amd.propagator import Propagator
    # backward Euler has no slope build
    w = SMALL[0].with_(scheme="be")
    with pytest.raises(nv.NvError) as e:
        prop.build(w)
    assert e.value.status == nv.NV_ERR_UNSUPPORTED
    # a 2-D problem has no stored-slope lookup
    v = W.Workload("vdp-slopes", "vdp", (1.0,), 0.0, 1.0, 2, (8, 8), (-1.0, -1.0), (1.0, 1.0), 10,
                   (0.5, 0.5), "fp64", "hermite_slopes")
    with pytest.raises(nv.NvError) as e:
        prop.build(v)
    assert e.value.status == nv.NV_ERR_INVALID_ARG
    # the slope table is component 1; there is no component 2
    prop.build(SMALL[1])
    with pytest.raises(nv.NvError):
        nv.nv_get_table(prop.ctx, 2, SMALL[1].n_slices, SMALL[1].points_per_slice, "fp64")
