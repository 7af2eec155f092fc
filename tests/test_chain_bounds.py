"""CPU checks of the error recursion the GPU tests use (tests/chain_bounds.py):
its interpolant weights reproduce the oracle's interpolants, and the bound it
gives holds, and is not vacuous, for tables perturbed entry by entry within
the parity bar."""
import numpy as np
import pytest

from chain_bounds import _hermite_terms, chain_bound
from paper_1304_6514_amd import workloads as W


@pytest.mark.parametrize("n", [3, 4, 9])
def test_hermite_weights_reproduce_the_oracle_interpolant(orc, n):
    rng = np.random.default_rng(n)
    t = rng.standard_normal(n)
    g = orc.make_grid((n,), (-1.0,), (1.0,))
    dxi = 2.0 / (n - 1)
    for x in np.concatenate([rng.uniform(-1.0, 1.0, 20), [-1.0, 1.0, -1.2, 1.3]]):
        o = orc.compose_tables(g, "hermite", t[None, None, :], (x,))
        cell, w = int(o.cells[0, 0]), float(o.weights[0, 0])
        idx, coef, dcoef = _hermite_terms(n, cell, w)
        assert abs(float(np.dot(coef, t[idx])) - o.boundary[1, 0]) <= 1e-14
        # derivative in x against a central difference of the oracle's interpolant
        e = 1e-6
        hi = orc.compose_tables(g, "hermite", t[None, None, :], (x + e,)).boundary[1, 0]
        lo = orc.compose_tables(g, "hermite", t[None, None, :], (x - e,)).boundary[1, 0]
        if 0.0 < w + e / dxi and w - e / dxi < 1.0:          # stays in the cell
            assert abs(float(np.dot(dcoef, t[idx])) / dxi - (hi - lo) / (2 * e)) <= 1e-6


CASES = [
    W.Workload("fcub-bound", "forced_cubic", (), 0.0, 6.0, 60, (200,), (-3.0,), (3.0,), 40,
               (1.0,), "fp64", "hermite"),
    W.Workload("logistic-bound", "logistic", (), 0.0, 10.0, 64, (64,), (-0.1,), (1.2,), 50,
               (0.1,), "fp64", "linear"),
    W.Workload("vdp-bound", "vdp", (3.5,), 0.0, 10.0, 100, (40, 40), (-3.0, -8.0), (3.0, 8.0),
               40, (2.0, 0.0), "fp64", "bilinear"),
]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_bound_holds_for_perturbed_tables(orc, w):
    g = orc.make_grid(w.grid_n, w.grid_lo, w.grid_hi)
    tab = orc.build_tables(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices, g,
                           w.steps_per_slice)
    tol = 1e-5
    o = orc.compose_tables(g, w.interp, tab, w.y0)
    assert o.status == 0
    bound = chain_bound(w, tab, o, tol)
    worst = 0.0
    for seed in range(4):
        rng = np.random.default_rng(seed)
        # worst-case-like: every entry moved by the full bar, random sign
        pert = tab + tol * np.maximum(np.abs(tab), 1.0) * rng.choice([-1.0, 1.0], tab.shape)
        p = orc.compose_tables(g, w.interp, pert, w.y0)
        assert p.status == 0
        d = np.abs(p.boundary - o.boundary)
        assert np.all(d <= bound)
        worst = max(worst, float(np.max(d[1:] / bound[1:])))
    # the bound is a real constraint, not orders of magnitude above what happens
    assert worst > 1e-2, worst
