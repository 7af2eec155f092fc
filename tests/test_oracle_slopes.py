"""Pins of the oracle's slope tables and of cubic Hermite with stored slopes.

The slope table holds, for every entry, the derivative of the slice's
discrete map with respect to the grid point (the derivative of the RK4 or
Euler map that produced the entry, carried through every stage by the chain
rule).  The paper's computation phase tabulates values only; the slopes are
an optional second table for cubic Hermite lookup, which the paper leaves out.
Pins, each independent of the oracle's tangent code:
  - y' = lambda y: the derivative of S steps is the one-step factor to the
    power S, for every grid point, and equals value / grid point;
  - fourth-order central differences of the oracle's own value map (with
    forcing, offset slices and both schemes): a term dropped from a stage, a
    stage's Jacobian taken at the wrong state or a wrong weight in the
    combination moves the slope by far more than the difference formula's
    error;
  - the logistic equation's exact flow derivative exp(L)/(1 + xi (exp(L) - 1))^2,
    which RK4's derivative approaches at fourth order;
  - cubic Hermite with exact slopes reproduces every cubic polynomial, inside
    the grid and when extrapolating from an edge cell;
  - its error falls by 2^4 per halving of the grid spacing (order 4), and
    stays far below that of the finite-difference slopes;
  - the lazily integrated method equals the method over the full tables.
"""
import math

import numpy as np
import pytest


def rk4_poly(z):
    return 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24


@pytest.mark.parametrize("scheme", ["rk4", "euler"])
@pytest.mark.parametrize("lam", [-1.3, 0.7])
def test_linear_slopes_are_the_one_step_factor_to_the_power(orc, scheme, lam):
    n_slices, steps, t0, T = 3, 20, 0.25, 1.75
    g = orc.make_grid((9,), (-2.0,), (2.0,))
    tab = orc.build_tables_slopes("linear", (lam,), scheme, t0, T, n_slices, g, steps)
    h = (T - t0) / n_slices / steps
    z = lam * h
    factor = (rk4_poly(z) if scheme == "rk4" else 1 + z) ** steps
    np.testing.assert_allclose(tab[1], factor, rtol=1e-13, atol=0)
    xi = np.linspace(-2.0, 2.0, 9)
    nz = xi != 0
    np.testing.assert_allclose(tab[0][:, nz] / xi[nz], tab[1][:, nz], rtol=1e-13)
    # the values are those of the plain build, to the bit
    plain = orc.build_tables("linear", (lam,), scheme, t0, T, n_slices, g, steps)
    assert np.array_equal(tab[0], plain[0])


def _fd4(orc, rhs, params, scheme, t0, T, n_slices, steps, xi, delta):
    """Fourth-order central difference of the value map at xi, per slice, from
    a five-point grid xi - 2 delta .. xi + 2 delta (exact binary points)."""
    g = orc.make_grid((5,), (xi - 2 * delta,), (xi + 2 * delta,))
    v = orc.build_tables(rhs, params, scheme, t0, T, n_slices, g, steps)[0]
    return (8.0 * (v[:, 3] - v[:, 1]) - (v[:, 4] - v[:, 0])) / (12.0 * delta)


CASES = [
    ("logistic", (), 0.0, 2.0, [0.125, 0.5, 0.875]),
    ("forced_cubic", (), 0.375, 2.375, [-1.5, 0.25, 1.25]),
    ("square", (), 0.0, 0.5, [0.25, 0.5, 0.75]),
]


@pytest.mark.parametrize("scheme", ["rk4", "euler"])
@pytest.mark.parametrize("rhs,params,t0,T,points", CASES, ids=[c[0] for c in CASES])
def test_slopes_equal_differences_of_the_value_map(orc, rhs, params, t0, T, points, scheme):
    n_slices, steps, delta = 4, 25, 2.0 ** -9
    for xi in points:
        g = orc.make_grid((3,), (xi - 1.0,), (xi + 1.0,))       # xi is the middle node
        tab = orc.build_tables_slopes(rhs, params, scheme, t0, T, n_slices, g, steps)
        fd = _fd4(orc, rhs, params, scheme, t0, T, n_slices, steps, xi, delta)
        got = tab[1][:, 1]
        assert np.all(np.isfinite(got))
        # difference error ~ delta^4 f^(5) / 30 plus rounding ~ 1e-16 / delta
        np.testing.assert_allclose(got, fd, rtol=2e-9, atol=2e-11)


def test_logistic_slopes_approach_the_flow_derivative(orc):
    n_slices, steps, T = 5, 100, 2.5
    xi = np.linspace(0.05, 0.95, 10)
    g = orc.make_grid((10,), (0.05,), (0.95,))
    tab = orc.build_tables_slopes("logistic", (), "rk4", 0.0, T, n_slices, g, steps)
    L = T / n_slices
    exact = math.exp(L) / (1.0 + xi * (math.exp(L) - 1.0)) ** 2
    err = np.max(np.abs(tab[1] - exact[None, :]))
    # RK4 with h = 5e-3: the derivative of the map is fourth-order accurate
    assert err < 1e-10, err
    # and the error is that of the scheme, not of the tangent: halving h
    tab2 = orc.build_tables_slopes("logistic", (), "rk4", 0.0, T, n_slices, g, 2 * steps)
    err2 = np.max(np.abs(tab2[1] - exact[None, :]))
    assert 10.0 < err / err2 < 22.0, (err, err2)


def _cubic_table(coef, n, lo, hi):
    xi = lo + np.arange(n) * ((hi - lo) / (n - 1))
    p = np.polynomial.polynomial.polyval(xi, coef)
    dp = np.polynomial.polynomial.polyval(xi, np.polynomial.polynomial.polyder(coef))
    return np.stack([p[None, :], dp[None, :]])


def test_hermite_with_slopes_reproduces_cubics(orc):
    coef = [0.3, -1.1, 0.7, 0.45]
    lo, hi, n = -1.0, 2.0, 7
    g = orc.make_grid((n,), (lo,), (hi,))
    tab = _cubic_table(coef, n, lo, hi)
    for y0 in [-1.0, -0.37, 0.0, 0.51, 1.49999, 2.0, -1.3, 2.4]:   # last two: extrapolation
        r = orc.compose_tables(g, "hermite_slopes", tab, (y0,))
        want = np.polynomial.polynomial.polyval(y0, coef)
        assert r.status == 0
        assert abs(r.yT[0] - want) <= 1e-13 * max(1.0, abs(want)), (y0, r.yT[0], want)
    # a slope mistake is not invisible: the finite-difference form misses a cubic
    fd = orc.compose_tables(g, "hermite", tab[:1], (0.51,))
    assert abs(fd.yT[0] - np.polynomial.polynomial.polyval(0.51, coef)) > 1e-6


def _max_interp_error(orc, interp, n):
    lo, hi = 0.0, 1.0
    xi = lo + np.arange(n) * ((hi - lo) / (n - 1))
    tab = np.stack([np.sin(3 * xi)[None, :], (3 * np.cos(3 * xi))[None, :]])
    g = orc.make_grid((n,), (lo,), (hi,))
    q = np.linspace(0.013, 0.987, 97)
    t = tab if interp == "hermite_slopes" else tab[:1]
    return max(abs(orc.compose_tables(g, interp, t, (y,)).yT[0] - math.sin(3 * y)) for y in q)


def test_hermite_with_slopes_is_fourth_order(orc):
    e = [_max_interp_error(orc, "hermite_slopes", n) for n in (17, 33, 65)]
    r = [e[0] / e[1], e[1] / e[2]]
    assert all(12.0 < x < 20.0 for x in r), (e, r)
    # the finite-difference slopes (order 3 inside, second-order one-sided
    # slopes in the end cells) are far less accurate at every spacing
    f = [_max_interp_error(orc, "hermite", n) for n in (17, 33, 65)]
    assert all(a < b / 50 for a, b in zip(e, f)), (e, f)


@pytest.mark.parametrize("rhs,params,t0,T,y0", [("logistic", (), 0.0, 3.0, 0.2),
                                                ("forced_cubic", (), 0.5, 3.5, 0.8)])
def test_lazy_method_with_slopes_equals_full_tables(orc, rhs, params, t0, T, y0):
    g = orc.make_grid((41,), (-1.5,), (1.5,))
    tab = orc.build_tables_slopes(rhs, params, "rk4", t0, T, 6, g, 30)
    full = orc.compose_tables(g, "hermite_slopes", tab, (y0,))
    lazy = orc.method_lazy(rhs, params, "rk4", t0, T, 6, g, 30, "hermite_slopes", (y0,))
    assert full.status == 0 and lazy.status == 0
    assert np.array_equal(full.boundary, lazy.boundary)
    # the entries for a list of pairs are the table's
    sl, pt = np.array([0, 2, 5, 5]), np.array([0, 17, 40, 3])
    ent = orc.table_entries_slopes(rhs, params, "rk4", t0, T, 6, g, 30, sl, pt)
    assert np.array_equal(ent, tab[:, sl, pt])


def test_slopes_argument_errors(orc):
    g2 = orc.make_grid((4, 4), (0.0, 0.0), (1.0, 1.0))
    with pytest.raises(Exception):
        orc.build_tables_slopes("vdp", (1.0,), "rk4", 0.0, 1.0, 2, g2, 10)
