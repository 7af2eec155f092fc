"""A seeded sweep of small configurations through the C ABI, against the oracle.

Each case draws a right-hand side and its parameter, the build precision, the
scheme (RK4 or forward Euler), the FP32 accumulation mode, the trajectories per
lane, the lookup, the slice count, a grid (ragged sizes, offset boxes), the
steps per slice, the start time, y0 (inside or outside the grid) and a chunk
count for nv_solve, then checks, as the hand-written parity tests do:
  - every table entry against the oracle's: |g - o| <= tol * max(|o|, 1) with
    tol = 1e-12 for FP64 builds and 1e-5 for FP32 builds (with stored slopes,
    the slope table too), and non-finite entries in the same places;
  - the composition over the GPU's own tables against the oracle's over the
    same tables: the same status, failing slice and out-of-grid count, and the
    boundary states bit for bit;
  - nv_solve with the drawn chunk count gives the same tables and states as
    the build followed by the composition, bit for bit.
The draws are the test's own (numpy, seed = case number); none of the method's
arithmetic is here.
"""
import sys

import numpy as np
import pytest

from paper_1304_6514_amd import nv
from paper_1304_6514_amd import workloads as W

TOL = {"fp64": 1e-12, "fp32": 1e-5}
N_CASES = 96


def say(*a):
    print("[gpu-test]", *a, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nv.load()          # raises when libnv.so is missing: no fallback
    return torch


def draw(case):
    """One configuration: (workload, traj_per_lane, compensated, solve_chunks)."""
    rng = np.random.default_rng(case)
    rhs = ["linear", "logistic", "forced_cubic", "vdp", "square"][case % 5]
    precision = "fp64" if rng.random() < 0.5 else "fp32"
    scheme = "rk4" if rng.random() < 0.75 else "euler"
    n_slices = int(rng.integers(1, 25))
    steps = int(rng.integers(1, 81))
    t0 = float(np.round(rng.uniform(0.0, 1.0), 3))
    L = float(np.round(rng.uniform(0.05, 0.5), 3))
    params = ()
    if rhs == "linear":
        params = (float(np.round(rng.uniform(-2.0, 1.0), 3)),)
    elif rhs == "vdp":
        params = (float(np.round(rng.uniform(0.0, 3.0), 3)),)
    elif rhs == "square":
        L = min(L, 0.5 / n_slices)      # y' = y^2 from y <= 1.5 stays below 6
    if rhs == "vdp":
        n = (int(rng.integers(2, 25)), int(rng.integers(2, 25)))
        lo = (float(np.round(rng.uniform(-3.0, -1.0), 2)), float(np.round(rng.uniform(-4.0, -1.0), 2)))
        hi = (float(np.round(rng.uniform(1.0, 3.0), 2)), float(np.round(rng.uniform(1.0, 4.0), 2)))
        interp = "bilinear"
        y0 = tuple(float(np.round(rng.uniform(l, h), 3)) for l, h in zip(lo, hi))
    else:
        n = (int(rng.integers(2, 701)),)
        lo = (float(np.round(rng.uniform(-2.0, 0.0), 2)),)
        hi = (lo[0] + float(np.round(rng.uniform(0.5, 3.0), 2)),)
        if rhs == "square":
            lo, hi = (0.0,), (1.5,)
        choices = ["linear", "hermite_slopes"] + (["hermite"] if n[0] >= 3 else [])
        interp = choices[int(rng.integers(0, len(choices)))]
        inside = rng.random() < 0.8
        y0 = (float(np.round(rng.uniform(lo[0], hi[0]) if inside
                             else hi[0] + rng.uniform(0.0, 1.0), 3)),)
        if rhs == "square":
            y0 = (min(y0[0], 1.5),)
    compensated = 2
    if precision == "fp32":
        compensated = int(rng.integers(0, 3)) if steps <= 40 else int(rng.integers(1, 3))
    traj_per_lane = [0, 1, 2, 4][int(rng.integers(0, 4))]
    chunks = int(rng.integers(0, min(8, n_slices) + 1))
    w = W.Workload(f"sweep-{case}-{rhs}-{precision}-{scheme}-{interp}", rhs, params, t0,
                   t0 + n_slices * L, n_slices, n, lo, hi, steps, y0, precision, interp, scheme)
    return w, traj_per_lane, compensated, chunks


def mixed_err(g, o):
    fin = np.isfinite(o)
    assert np.array_equal(np.isfinite(g), fin)
    if not fin.any():
        return 0.0
    g, o = g[fin], o[fin]
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1.0)))


def same_states(g, e):
    fin = np.isfinite(e)
    assert np.array_equal(np.isfinite(g), fin)
    assert np.array_equal(g[fin].view(np.int64), e[fin].view(np.int64))


def test_sweep_draws_cover_the_options():
    # the draws reach every right-hand side, lookup, scheme, precision, FP32
    # accumulation mode, trajectories per lane and chunking, and both sides of
    # the grid for y0 (a test of the sweep itself, on the CPU)
    seen = {k: set() for k in ("rhs", "interp", "scheme", "precision", "comp", "p", "chunks",
                               "outside")}
    for case in range(N_CASES):
        w, p, comp, chunks = draw(case)
        seen["rhs"].add(w.rhs)
        seen["interp"].add(w.interp)
        seen["scheme"].add(w.scheme)
        seen["precision"].add(w.precision)
        if w.precision == "fp32":
            seen["comp"].add(comp)
        seen["p"].add(p)
        seen["chunks"].add(min(chunks, 2))
        seen["outside"].add(any(y > h for y, h in zip(w.y0, w.grid_hi)))
    assert seen["rhs"] == {"linear", "logistic", "forced_cubic", "vdp", "square"}
    assert seen["interp"] == {"linear", "hermite", "hermite_slopes", "bilinear"}
    assert seen["scheme"] == {"rk4", "euler"} and seen["precision"] == {"fp64", "fp32"}
    assert seen["comp"] == {0, 1, 2} and seen["p"] == {0, 1, 2, 4}
    assert seen["chunks"] == {0, 1, 2} and seen["outside"] == {False, True}


@pytest.mark.gpu
@pytest.mark.parametrize("case", range(N_CASES))
def test_sweep_case(orc, torch, case):
    from paper_1304_6514_amd.propagator import Propagator
    w, p, comp, chunks = draw(case)
    say("sweep", case, w.name, w.n_slices, w.grid_n, w.steps_per_slice, "P", p, "comp", comp,
        "chunks", chunks)
    g = orc.make_grid(w.grid_n, w.grid_lo, w.grid_hi)
    if w.interp == "hermite_slopes":
        ref = orc.build_tables_slopes(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices, g,
                                      w.steps_per_slice)
    else:
        ref = orc.build_tables(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices, g,
                               w.steps_per_slice)
    comps = ref.shape[0]
    with Propagator("cuda:0", traj_per_lane=p, compensated=comp) as a:
        a.build(w)
        tab = np.stack([a.table(c).astype(np.float64) for c in range(comps)])
        err = mixed_err(tab, ref)
        assert err <= TOL[w.precision], err
        ra = a.compose()
    o = orc.compose_tables(g, w.interp, tab, w.y0)
    assert ra.status == (nv.NV_OK if o.status == 0 else nv.NV_ERR_NONFINITE)
    assert ra.bad_slice == o.bad_slice and ra.n_out_of_grid == o.n_out_of_grid
    n = (o.bad_slice if o.status != 0 else w.n_slices) + 1
    same_states(ra.boundary[:n], o.boundary[:n])
    with Propagator("cuda:0", traj_per_lane=p, compensated=comp, solve_chunks=chunks) as b:
        rb = b.solve(w)
        tb = np.stack([b.table(c).astype(np.float64) for c in range(comps)])
    assert np.array_equal(tb.view(np.int64), tab.view(np.int64))
    assert rb.status == ra.status and rb.bad_slice == ra.bad_slice
    assert rb.n_out_of_grid == ra.n_out_of_grid
    same_states(rb.boundary[:n], ra.boundary[:n])
    say(f"  table error {err:.3g}, status {o.status}, out of grid {o.n_out_of_grid}")
