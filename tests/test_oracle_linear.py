"""Pins of the linear-system oracle (affine basis propagator, heat equation of
sec. 6) against facts fixed outside it: a dense library solve, the
eigen-decomposition of the second-difference matrix (discrete sine basis), the
closed-form solution cos(t) sin(pi x), and the paper's statement that the
affine reconstruction adds no error beyond rounding."""
import math

import numpy as np
import pytest

from oracle import linear_oracle as lo


def _dst(M):
    dx = 1.0 / (M + 1)
    i = np.arange(1, M + 1)
    V = np.sqrt(2 * dx) * np.sin(np.outer(i, i) * math.pi * dx)     # orthonormal, symmetric
    mu = (4.0 / dx ** 2) * np.sin(i * math.pi * dx / 2) ** 2          # D v_k = -mu_k v_k
    return dx, V, mu


def test_thomas_matches_dense_solve():
    rng = np.random.default_rng(0)
    for M in (1, 2, 9, 40):
        r = rng.uniform(0.01, 50.0)
        f = rng.normal(size=M)
        w, c = lo.thomas_coefficients(r, M)
        y = lo.thomas_solve(r, f, w, c)
        A = np.diag(np.full(M, 1 + 2 * r)) + np.diag(np.full(M - 1, -r), 1) \
            + np.diag(np.full(M - 1, -r), -1)
        ref = np.linalg.solve(A, f)
        assert np.max(np.abs(y - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


def test_dst_basis_diagonalises_the_second_difference():
    M = 11
    dx, V, mu = _dst(M)
    D = (np.diag(np.full(M, -2.0)) + np.diag(np.ones(M - 1), 1) + np.diag(np.ones(M - 1), -1)) / dx ** 2
    assert np.allclose(V @ V, np.eye(M), atol=1e-13)
    assert np.allclose(D @ V, V * -mu, atol=1e-9)


@pytest.mark.parametrize("dt,N", [(0.005, 8), (0.003, 7)])     # 0.003: a remainder step per slice
def test_homogeneous_maps_equal_sine_basis_closed_form(dt, N):
    M, a0, a1, t0, T = 9, 1.0, 0.25, 0.0, 1.0
    G, c = lo.build_tables(M, a0, a1, True, t0, T, N, dt)
    dx, V, mu = _dst(M)
    L, S, rem = lo.slice_steps(t0, T, N, dt)
    for j in range(N):
        d = np.ones(M)
        gamma = 0.0
        for h, te in lo.step_list(t0 + j * L, S, dt, rem):
            a = a0 + a1 * math.sin(te)
            d = d / (1.0 + h * a * mu)
            beta = math.pi ** 2 * a * math.cos(te) - math.sin(te)
            gamma = (gamma + h * beta) / (1.0 + h * a * mu[0])
        assert np.max(np.abs(G[j] - (V * d) @ V)) < 1e-13
        # sin(pi x_i) is the first sine basis vector up to scale: the forced
        # response stays along it
        _, _, s = lo.grid(M)
        assert np.max(np.abs(c[j] - gamma * s)) < 1e-13


def test_affine_reconstruction_adds_no_error_beyond_rounding():
    M, a0, a1, t0, T, N, dt = 9, 1.0, 0.25, 0.0, 2.0, 16, 0.005
    y0 = lo.exact(0.0, M)
    G, c = lo.build_tables(M, a0, a1, True, t0, T, N, dt)
    method = lo.compose(G, c, y0)[-1]
    serial = lo.serial(M, a0, a1, True, t0, T, N, dt, y0)
    assert np.max(np.abs(method - serial)) < 1e-13


def test_serial_backward_euler_converges_to_the_closed_form():
    a0, a1, T = 1.0, 0.25, 1.0

    def run(M, dt):
        return lo.serial(M, a0, a1, True, 0.0, T, 1, dt, lo.exact(0.0, M))

    # first order in time (self-convergence isolates the time error)
    y1, y2, y4 = run(9, 0.01), run(9, 0.005), run(9, 0.0025)
    r = np.max(np.abs(y1 - y2)) / np.max(np.abs(y2 - y4))
    assert 1.8 < r < 2.2, r
    # second order in space against the closed form cos(t) sin(pi x)
    e9 = np.max(np.abs(run(9, 0.0025) - lo.exact(T, 9)))
    e19 = np.max(np.abs(run(19, 0.0025) - lo.exact(T, 19)))
    assert 3.0 < e9 / e19 < 5.0, (e9, e19)
    assert e9 < 0.01
