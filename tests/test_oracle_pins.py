"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against a closed form, an exact invariant, an
independent library integrator (scipy), or an exactness property the
interpolation rules must have, so that a dropped term, wrong sign, wrong stage
time, transposed index or wrong interpolation basis fails at least one test.
"""
import math

import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_1304_6514_amd import workloads as W


def rk4_poly(z):
    """Stability polynomial of classical RK4: the exact one-step factor on y'=lambda y."""
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


# --------------------------------------------------------------------------
# Time integration (O1)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lam,y0", [(-2.0, 1.3), (0.5, -0.7), (-7.5, 2.0)])
def test_rk4_linear_is_stability_polynomial_power(orc, lam, y0):
    # T = 5 in 5 slices of 10 steps: h = 0.1 (large, so coefficient errors show)
    got = orc.serial("linear", [lam], "rk4", 0.0, 5.0, 5, 10, [y0])[0]
    want = y0 * rk4_poly(lam * 0.1) ** 50
    assert got == pytest.approx(want, rel=1e-12)
    # and it approximates the exact solution to RK4 accuracy
    assert abs(got - y0 * math.exp(lam * 5.0)) <= 1e-2 * abs(y0 * math.exp(lam * 5.0)) + 1e-9


@pytest.mark.parametrize("lam", [-2.0, 0.5])
def test_euler_linear_is_power(orc, lam):
    got = orc.serial("linear", [lam], "euler", 0.0, 5.0, 5, 10, [1.0])[0]
    assert got == pytest.approx((1 + lam * 0.1) ** 50, rel=1e-12)


def test_logistic_closed_form(orc):
    w = W.LOGISTIC_FP64
    got = orc.serial("logistic", None, "rk4", w.t0, w.T, w.n_slices, w.steps_per_slice,
                     w.y0)[0]
    y0 = w.y0[0]
    exact = 1.0 / (1.0 + (1.0 / y0 - 1.0) * math.exp(-(w.T - w.t0)))
    assert abs(got - exact) < 1e-13
    # the decreasing branch, with a nonzero start time
    got2 = orc.serial("logistic", None, "rk4", 1.5, 4.5, 3, 300, [1.7])[0]
    exact2 = 1.0 / (1.0 + (1.0 / 1.7 - 1.0) * math.exp(-3.0))
    assert abs(got2 - exact2) < 1e-12


def test_square_model_closed_form_and_orders(orc):
    # y' = y^2, y(0) = 1: y = 1/(1 - t), y(1/2) = 2 (sec. 3)
    got = orc.serial_steps("square", None, "rk4", 0.0, 0.5, 2000, [1.0])[0]
    assert abs(got - 2.0) < 1e-11
    e1 = abs(orc.serial_steps("square", None, "euler", 0.0, 0.5, 1000, [1.0])[0] - 2.0)
    e2 = abs(orc.serial_steps("square", None, "euler", 0.0, 0.5, 2000, [1.0])[0] - 2.0)
    assert 1.9 < e1 / e2 < 2.1


def _scipy_solution(fun, t0, T, y0):
    sol = solve_ivp(fun, (t0, T), y0, method="DOP853", rtol=1e-13, atol=1e-15)
    assert sol.success
    return sol.y[:, -1]


def test_forced_cubic_matches_library_integrator(orc):
    t0, T = 2.3, 7.3
    ref = _scipy_solution(lambda t, y: [math.sin(3 * t) - y[0] ** 3], t0, T, [0.8])
    got = orc.serial("forced_cubic", None, "rk4", t0, T, 10, 500, [0.8])  # h = 1e-3
    assert abs(got[0] - ref[0]) < 1e-10


def test_forced_cubic_is_fourth_order(orc):
    # a wrong stage time (e.g. k2 evaluated at t instead of t + h/2) drops the order
    t0, T = 0.0, 4.0
    ref = _scipy_solution(lambda t, y: [math.sin(3 * t) - y[0] ** 3], t0, T, [1.0])[0]
    e1 = abs(orc.serial("forced_cubic", None, "rk4", t0, T, 1, 40, [1.0])[0] - ref)
    e2 = abs(orc.serial("forced_cubic", None, "rk4", t0, T, 1, 80, [1.0])[0] - ref)
    assert 12.0 < e1 / e2 < 20.0
    f1 = abs(orc.serial("forced_cubic", None, "euler", t0, T, 1, 4000, [1.0])[0] - ref)
    f2 = abs(orc.serial("forced_cubic", None, "euler", t0, T, 1, 8000, [1.0])[0] - ref)
    assert 1.8 < f1 / f2 < 2.2


def test_harmonic_state_is_complex_power(orc):
    # mu = 0: y1' = y2, y2' = -y1, i.e. z = y1 + i y2 obeys z' = -i z, so RK4
    # gives z_n = R(-i h)^n z_0 exactly (up to rounding); energy factor per step
    # is |R(ih)|^2 = 1 - h^6/72 + h^8/576.
    h, n = 0.1, 1000
    got = orc.serial("vdp", [0.0], "rk4", 0.0, h * n, 10, 100, [2.0, 0.0])
    z = 2.0 * rk4_poly(-1j * h) ** n
    assert got[0] == pytest.approx(z.real, abs=1e-12)
    assert got[1] == pytest.approx(z.imag, abs=1e-12)
    energy_ratio = (got[0] ** 2 + got[1] ** 2) / 4.0
    assert energy_ratio == pytest.approx((1 - h ** 6 / 72 + h ** 8 / 576) ** n, rel=1e-12)


def test_vdp_matches_library_integrator(orc):
    mu = 3.5
    ref = _scipy_solution(lambda t, y: [y[1], mu * (1 - y[0] ** 2) * y[1] - y[0]],
                          0.0, 10.0, [2.0, 0.0])
    got = orc.serial("vdp", [mu], "rk4", 0.0, 10.0, 10, 2000, [2.0, 0.0])  # h = 5e-4
    assert np.max(np.abs(got - ref)) < 1e-8


# --------------------------------------------------------------------------
# Grid and tables (O2 computation phase)
# --------------------------------------------------------------------------

def test_grid_points_uniform_and_axis0_major(orc):
    g1 = orc.make_grid(7, -0.1, 1.2)
    np.testing.assert_allclose(orc.grid_points(g1)[:, 0], np.linspace(-0.1, 1.2, 7),
                               rtol=0, atol=1e-15)
    g2 = orc.make_grid((3, 4), (-3.0, -8.0), (3.0, 8.0))
    pts = orc.grid_points(g2)
    a, b = np.meshgrid(np.linspace(-3, 3, 3), np.linspace(-8, 8, 4), indexing="ij")
    np.testing.assert_allclose(pts[:, 0], a.reshape(-1), atol=1e-15)
    np.testing.assert_allclose(pts[:, 1], b.reshape(-1), atol=1e-15)


def test_logistic_tables_are_exact_flow_map(orc):
    w = W.small(W.LOGISTIC_FP64, 8, (33,), 1000)   # L = 10/8, h = L/1000
    g = orc.make_grid(w.grid_n, w.grid_lo, w.grid_hi)
    tab = orc.build_tables("logistic", None, "rk4", w.t0, w.T, w.n_slices, g,
                           w.steps_per_slice)
    L = (w.T - w.t0) / w.n_slices
    xi = np.linspace(w.grid_lo[0], w.grid_hi[0], w.grid_n[0])
    exact = xi / (xi + (1 - xi) * math.exp(-L))
    for j in range(w.n_slices):
        assert np.max(np.abs(tab[0, j] - exact)) < 1e-13
    # autonomous problem: every slice holds bit-identical tables
    assert all(np.array_equal(tab[0, 0], tab[0, j]) for j in range(w.n_slices))


def test_linear_tables_are_polynomial_power(orc):
    g = orc.make_grid(9, -2.0, 2.0)
    tab = orc.build_tables("linear", [-1.5], "rk4", 0.0, 3.0, 6, g, 25)
    h = 3.0 / 6 / 25
    xi = np.linspace(-2.0, 2.0, 9)
    np.testing.assert_allclose(tab[0], np.tile(xi * rk4_poly(-1.5 * h) ** 25, (6, 1)),
                               rtol=1e-13, atol=1e-15)


def test_nonautonomous_tables_follow_slice_start_times(orc):
    # slice j starts at T_j = t0 + j (T - t0)/N; checked against scipy per entry
    t0, T, N, S = 1.0, 3.0, 4, 400
    g = orc.make_grid(5, -1.5, 1.5)
    tab = orc.build_tables("forced_cubic", None, "rk4", t0, T, N, g, S)
    L = (T - t0) / N
    for j in range(N):
        for k, x in enumerate(np.linspace(-1.5, 1.5, 5)):
            ref = _scipy_solution(lambda t, y: [math.sin(3 * t) - y[0] ** 3],
                                  t0 + j * L, t0 + (j + 1) * L, [x])[0]
            assert abs(tab[0, j, k] - ref) < 1e-9, (j, k)


def test_vdp_tables_component_layout(orc):
    g = orc.make_grid((3, 4), (-1.0, -2.0), (1.0, 2.0))
    mu, N, S = 1.7, 3, 200
    tab = orc.build_tables("vdp", [mu], "rk4", 0.0, 1.5, N, g, S)
    pts = orc.grid_points(g)
    for j in range(N):
        for k in range(12):
            ref = _scipy_solution(lambda t, y: [y[1], mu * (1 - y[0] ** 2) * y[1] - y[0]],
                                  0.5 * j, 0.5 * (j + 1), pts[k])
            assert abs(tab[0, j, k] - ref[0]) < 1e-9 and abs(tab[1, j, k] - ref[1]) < 1e-9


def test_sampled_entries_equal_full_tables(orc):
    g = orc.make_grid((5, 6), (-3.0, -8.0), (3.0, 8.0))
    tab = orc.build_tables("vdp", [2.0], "rk4", 0.0, 4.0, 7, g, 20)
    rng = np.random.default_rng(3)
    sl = rng.integers(0, 7, 50)
    pt = rng.integers(0, 30, 50)
    ent = orc.table_entries("vdp", [2.0], "rk4", 0.0, 4.0, 7, g, 20, sl, pt)
    assert np.array_equal(ent[0], tab[0, sl, pt]) and np.array_equal(ent[1], tab[1, sl, pt])


# --------------------------------------------------------------------------
# Lookup
# --------------------------------------------------------------------------

def test_locate_on_integer_grid(orc):
    n = 9                       # lo = 0, hi = 8: u = x exactly
    for x in range(0, 8):
        assert orc.locate(0.0, 8.0, n, float(x)) == (x, 0.0, False)
    assert orc.locate(0.0, 8.0, n, 8.0) == (7, 1.0, False)           # last node
    assert orc.locate(0.0, 8.0, n, 2.25) == (2, 0.25, False)
    assert orc.locate(0.0, 8.0, n, -0.5) == (0, -0.5, True)          # below: extrapolate
    assert orc.locate(0.0, 8.0, n, 8.5) == (7, 1.5, True)            # above: extrapolate
    assert orc.locate(0.0, 8.0, n, -0.0) == (0, 0.0, False)
    c, w, out = orc.locate(0.0, 8.0, n, 1e300)
    assert c == 7 and out and w > 1e299
    c, w, out = orc.locate(0.0, 8.0, n, float("-inf"))
    assert c == 0 and out and w == float("-inf")
    c, w, out = orc.locate(0.0, 8.0, n, float("nan"))
    assert c == 0 and out and w != w


def test_locate_brackets_random_queries(orc):
    rng = np.random.default_rng(0)
    for lo, hi, n in [(-3.0, 3.0, 4096), (-0.1, 1.2, 256), (-8.0, 8.0, 128), (0.3, 0.7, 2)]:
        d = (hi - lo) / (n - 1)
        for x in rng.uniform(lo, hi, 500):
            c, w, out = orc.locate(lo, hi, n, x)
            assert not out and 0 <= c <= n - 2
            assert -1e-12 <= w <= 1 + 1e-12
            assert abs(lo + (c + w) * d - x) <= 1e-13 * max(1.0, abs(x))


# --------------------------------------------------------------------------
# Interpolation rules (O2 communication phase), via one-slice compositions
# --------------------------------------------------------------------------

def _one_slice(orc, g, interp, values, query):
    tab = np.asarray(values, dtype=float).reshape(g.dim, 1, -1)
    r = orc.compose_tables(g, interp, tab, query)
    assert r.status == 0
    return r.boundary[1]


def test_linear_interp_reproduces_lines_including_extrapolation(orc):
    g = orc.make_grid(11, -1.0, 2.0)
    xi = np.linspace(-1.0, 2.0, 11)
    for q in [-1.0, -0.37, 0.5, 1.9999, 2.0, -3.0, 5.5]:
        assert _one_slice(orc, g, "linear", 3 * xi - 1, [q])[0] == pytest.approx(
            3 * q - 1, abs=1e-13)


def test_hermite_reproduces_quadratics_and_nodes(orc):
    # centred and one-sided second-order slopes are exact for quadratics, and a
    # cubic Hermite piece with exact slopes reproduces them everywhere
    g = orc.make_grid(9, -3.0, 3.0)
    xi = np.linspace(-3.0, 3.0, 9)
    vals = 0.7 * xi * xi - 1.3 * xi + 0.4
    for q in [-3.0, -2.9, -1.1, 0.0, 0.123, 2.5, 3.0, -3.4, 3.3]:
        assert _one_slice(orc, g, "hermite", vals, [q])[0] == pytest.approx(
            0.7 * q * q - 1.3 * q + 0.4, abs=1e-12)
    rng = np.random.default_rng(1)
    vals = rng.standard_normal(9)
    for k in range(9):
        assert _one_slice(orc, g, "hermite", vals, [xi[k]])[0] == pytest.approx(
            vals[k], abs=1e-14)


def test_bilinear_reproduces_bilinear_functions(orc):
    g = orc.make_grid((4, 6), (-3.0, -8.0), (3.0, 8.0))
    pts = orc.grid_points(g)
    f0 = 1.0 + 2.0 * pts[:, 0] - 0.5 * pts[:, 1] + 0.25 * pts[:, 0] * pts[:, 1]
    f1 = -2.0 + 0.1 * pts[:, 0] + 3.0 * pts[:, 1] - 0.125 * pts[:, 0] * pts[:, 1]
    for q in [(-3.0, -8.0), (0.3, 1.7), (2.9, -7.9), (3.0, 8.0), (-4.0, 9.0)]:
        out = _one_slice(orc, g, "bilinear", np.stack([f0, f1]), list(q))
        a, b = q
        assert out[0] == pytest.approx(1 + 2 * a - 0.5 * b + 0.25 * a * b, abs=1e-12)
        assert out[1] == pytest.approx(-2 + 0.1 * a + 3 * b - 0.125 * a * b, abs=1e-12)


def _logistic_one_slice_error(orc, n, interp, L=0.5):
    g = orc.make_grid(n, -0.1, 1.2)
    tab = orc.build_tables("logistic", None, "rk4", 0.0, L, 1, g, 200)
    qs = np.linspace(-0.1, 1.2, 1001)
    exact = qs / (qs + (1 - qs) * math.exp(-L))
    got = np.array([orc.compose_tables(g, interp, tab, [q]).boundary[1, 0] for q in qs])
    return np.max(np.abs(got - exact))


def test_interpolation_orders(orc):
    # sec. 5: interpolation error O(dxi^l); l = 2 for linear, 3 for Hermite
    # with finite-difference slopes
    lin = [_logistic_one_slice_error(orc, n, "linear") for n in (17, 33, 65)]
    her = [_logistic_one_slice_error(orc, n, "hermite") for n in (17, 33, 65)]
    for a, b in zip(lin, lin[1:]):
        assert 3.5 < a / b < 4.5
    for a, b in zip(her, her[1:]):
        assert 6.0 < a / b < 10.0


def test_bilinear_order_on_nonlinear_map(orc):
    rng = np.random.default_rng(5)
    qs = np.stack([rng.uniform(-1.9, 1.9, 600), rng.uniform(-1.9, 1.9, 600)], axis=1)
    refs = [orc.integrate("vdp", [1.0], "rk4", 0.0, 0.25 / 50, 50, q) for q in qs]
    errs = []
    for n in (9, 17, 33):
        g = orc.make_grid((n, n), (-2.0, -2.0), (2.0, 2.0))
        tab = orc.build_tables("vdp", [1.0], "rk4", 0.0, 0.25, 1, g, 50)
        err = 0.0
        for q, ref in zip(qs, refs):
            got = orc.compose_tables(g, "bilinear", tab, q).boundary[1]
            err = max(err, np.max(np.abs(got - ref)))
        errs.append(err)
    for a, b in zip(errs, errs[1:]):
        assert 3.0 < a / b < 5.0


# --------------------------------------------------------------------------
# Whole method (O2) against the serial run (O1)
# --------------------------------------------------------------------------

def test_linear_problem_method_equals_serial(orc):
    # sec. 5: for a linear ODE the map is linear in the initial value and the
    # interpolation adds no error beyond rounding; the states leave the grid
    # box (extrapolation), which must still be exact
    g = orc.make_grid(5, 0.5, 1.5)
    tab = orc.build_tables("linear", [-0.8], "rk4", 0.0, 4.0, 8, g, 50)
    r = orc.compose_tables(g, "linear", tab, [0.7])
    ser = orc.serial("linear", [-0.8], "rk4", 0.0, 4.0, 8, 50, [0.7])
    assert r.status == 0 and r.n_out_of_grid > 0
    assert r.yT[0] == pytest.approx(ser[0], rel=1e-13)
    for j in range(9):
        assert r.boundary[j, 0] == pytest.approx(0.7 * rk4_poly(-0.8 * 0.01) ** (50 * j),
                                                 rel=1e-13)


def test_harmonic_bilinear_method_equals_serial(orc):
    w = W.small(W.HARMONIC, 64, (16, 16), 500)
    g = orc.make_grid(w.grid_n, w.grid_lo, w.grid_hi)
    r = orc.method_lazy("vdp", w.params, "rk4", w.t0, w.T, w.n_slices, g,
                        w.steps_per_slice, "bilinear", w.y0)
    ser = orc.serial("vdp", w.params, "rk4", w.t0, w.T, w.n_slices, w.steps_per_slice,
                     w.y0)
    assert r.status == 0 and r.n_out_of_grid == 0
    assert np.max(np.abs(r.yT - ser)) < 1e-12
    energy = r.boundary[:, 0] ** 2 + r.boundary[:, 1] ** 2
    assert np.max(np.abs(energy - 4.0)) < 1e-6     # RK4 energy drift h^6/72 per step


def test_logistic_method_error_within_linear_interpolation_bound(orc):
    # sec. 5 error splitting: with phi'' of the exact slice map bounded by B and
    # Lipschitz constant K <= e^L, the method error is below
    # sum_j K^(N-j) * dxi^2/8 * B (interpolation) + RK4 error (negligible here)
    w = W.LOGISTIC_FP64
    g = orc.make_grid(w.grid_n, w.grid_lo, w.grid_hi)
    tab = orc.build_tables("logistic", None, "rk4", w.t0, w.T, w.n_slices, g,
                           w.steps_per_slice)
    r = orc.compose_tables(g, "linear", tab, w.y0)
    ser = orc.serial("logistic", None, "rk4", w.t0, w.T, w.n_slices, w.steps_per_slice,
                     w.y0)
    err = abs(r.yT[0] - ser[0])
    L = (w.T - w.t0) / w.n_slices
    xs = np.linspace(0.0, 1.0, 20001)
    E = math.exp(-L)
    d2 = np.abs(np.gradient(np.gradient(xs / (xs + (1 - xs) * E), xs), xs))
    dxi = (w.grid_hi[0] - w.grid_lo[0]) / (w.grid_n[0] - 1)
    bound = w.n_slices * math.exp(L) * dxi ** 2 / 8 * d2.max()
    assert r.status == 0 and r.n_out_of_grid == 0
    assert 1e-7 < err < bound
    # halving the grid spacing keeps the error under the bound, which scales
    # with dxi^2 (the theorem of sec. 5 with l = 2)
    g2 = orc.make_grid(2 * w.grid_n[0] - 1, w.grid_lo, w.grid_hi)
    tab2 = orc.build_tables("logistic", None, "rk4", w.t0, w.T, w.n_slices, g2,
                            w.steps_per_slice)
    err2 = abs(orc.compose_tables(g2, "linear", tab2, w.y0).yT[0] - ser[0])
    assert err2 < bound / 4 and err2 < err / 2


def test_lazy_method_equals_full_tables(orc):
    for rhs, params, grid, interp in [
        ("forced_cubic", None, ((33,), (-3.0,), (3.0,)), "hermite"),
        ("logistic", None, ((20,), (-0.1,), (1.2,)), "linear"),
        ("vdp", [2.5], ((9, 11), (-3.0, -8.0), (3.0, 8.0)), "bilinear"),
    ]:
        g = orc.make_grid(*grid)
        y0 = [2.0, 0.0] if rhs == "vdp" else [0.3]
        tab = orc.build_tables(rhs, params, "rk4", 0.0, 6.0, 12, g, 40)
        full = orc.compose_tables(g, interp, tab, y0)
        lazy = orc.method_lazy(rhs, params, "rk4", 0.0, 6.0, 12, g, 40, interp, y0)
        assert np.array_equal(full.boundary, lazy.boundary)
        assert full.n_out_of_grid == lazy.n_out_of_grid


def test_out_of_grid_counted_on_square_vdp_box(orc):
    # the [-3,3]^2 box does not contain the mu ~ 3.5 limit cycle (|y2| up to ~5.5)
    w = W.small(W.VDP_SQUARE_BOX, 256, (32, 32), 100)
    g = orc.make_grid(w.grid_n, w.grid_lo, w.grid_hi)
    r = orc.method_lazy("vdp", w.params, "rk4", w.t0, w.T, w.n_slices, g,
                        w.steps_per_slice, "bilinear", w.y0)
    assert r.status == 0 and r.n_out_of_grid > 0
    w2 = W.small(W.VDP_FP32, 256, (32, 32), 100)
    g2 = orc.make_grid(w2.grid_n, w2.grid_lo, w2.grid_hi)
    r2 = orc.method_lazy("vdp", w2.params, "rk4", w2.t0, w2.T, w2.n_slices, g2,
                         w2.steps_per_slice, "bilinear", w2.y0)
    assert r2.status == 0 and r2.n_out_of_grid == 0


def test_nonfinite_detection(orc):
    g = orc.make_grid(5, 0.0, 1.0)
    tab = np.tile(np.linspace(0.0, 1.0, 5), (1, 6, 1))  # identity maps
    tab[0, 3, :] = np.nan
    r = orc.compose_tables(g, "linear", tab, [0.4])
    assert r.status == orc.NONFINITE and r.bad_slice == 3
    assert np.all(np.isfinite(r.boundary[:4])) and r.boundary[3, 0] == pytest.approx(0.4)
    r = orc.compose_tables(g, "linear", tab[:, :3], [float("nan")])
    assert r.status == orc.NONFINITE and r.bad_slice == 0
    # a non-finite entry the lookup does not touch is not an error
    tab2 = np.tile(np.linspace(0.0, 1.0, 5), (1, 2, 1))
    tab2[0, 1, 4] = np.inf
    assert orc.compose_tables(g, "linear", tab2, [0.1]).status == 0


def test_bad_arguments_rejected(orc):
    g = orc.make_grid(1, 0.0, 1.0)
    with pytest.raises(orc.OracleError):
        orc.build_tables("logistic", None, "rk4", 0.0, 1.0, 2, g, 10)
    g = orc.make_grid(2, 0.0, 1.0)
    with pytest.raises(orc.OracleError):
        orc.compose_tables(g, "hermite", np.zeros((1, 1, 2)), [0.5])
    with pytest.raises(orc.OracleError):
        orc.build_tables("vdp", [1.0], "rk4", 0.0, 1.0, 2, g, 10)   # dim mismatch
