"""Plain FP64 oracle of the method for linear systems: the affine basis
propagator (the closing discussion of linear problems in sec. 5, equations
`lineardiscrete` and `linearreconstruct`) on the heat equation of sec. 6.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library.

Problem (sec. 6, equation `heatequation`): y_t = a(t) y_xx + b(t, x) on
x in [0, 1] with y = 0 at both ends, a(t) = a0 + a1 sin t (the paper:
a0 = 1, a1 = 1/4).  With ``forcing=True``, b(t, x) = beta(t) sin(pi x),
beta(t) = pi^2 a(t) cos t - sin t, the forcing under which the exact solution
is y = cos(t) sin(pi x) (from y(0, x) = sin(pi x)).

Space: M interior points x_i = i dx, dx = 1/(M+1), centred second differences,
giving y' = a(t) D y + b(t) (`lineardiscrete`), D = tridiag(1, -2, 1) / dx^2.
Time: backward Euler, (I - h a(t+h) D) y_new = y + h b(t+h).

The tridiagonal system (1 + 2r) on the diagonal, -r off it, r = h a / dx^2, is
solved by the Thomas algorithm in this exact form (both sides of the parity
tests follow it operation for operation):
    w_1 = 1 / (1 + 2r),            c_1 = (-r) w_1
    w_i = 1 / ((1 + 2r) - (-r) c_{i-1}),  c_i = (-r) w_i          i = 2..M
    f'_1 = f_1 w_1,   f'_i = (f_i - (-r) f'_{i-1}) w_i
    y_M = f'_M,       y_i = f'_i - c_i y_{i+1}
with f = y + (h beta) s, s_i = sin(pi x_i) (the forcing term only in the
inhomogeneous solve).

Slices: [T_j, T_{j+1}], T_j = t0 + j L, L = (T - t0)/N, each integrated with
floor(L/dt + 1e-9) steps of dt plus one step of the remainder when it exceeds
1e-12 L; step s of slice j ends at T_j + (s+1) dt, the remainder step at
T_j + S dt + rem.

The affine propagator of slice j (`linearreconstruct`): c_j = the slice's
solve from y = 0 with the forcing, column k of G_j = the homogeneous solve
from the unit vector e_k; then phi_j(y) = c_j + G_j y exactly (no
interpolation error), and the composition is lambda_{j+1} = c_j + G_j
lambda_j, each component summed in index order starting from c_i.  The paper
fixes the affine map, not a summation order; any other order differs from
this one by rounding only (tests bound that difference).
"""
from __future__ import annotations

import math

import numpy as np


def grid(M):
    dx = 1.0 / (M + 1)
    x = np.array([(i + 1) * dx for i in range(M)])
    s = np.array([math.sin(math.pi * xi) for xi in x])
    return dx, x, s


def a_of(t, a0, a1):
    return a0 + a1 * math.sin(t)


def beta_of(t, a0, a1):
    """Forcing amplitude under which y = cos(t) sin(pi x) solves the PDE."""
    return (math.pi * math.pi) * a_of(t, a0, a1) * math.cos(t) - math.sin(t)


def slice_steps(t0, T, n_slices, dt):
    """(L, S, rem): slice length, whole steps of dt, remainder step (0: none)."""
    L = (T - t0) / n_slices
    S = int(math.floor(L / dt + 1e-9))
    rem = L - S * dt
    if not rem > 1e-12 * L:
        rem = 0.0
    return L, S, rem


def step_list(Tj, S, dt, rem):
    """(h, end time) of every step of a slice starting at Tj."""
    out = [(dt, Tj + (s + 1) * dt) for s in range(S)]
    if rem > 0.0:
        out.append((rem, (Tj + S * dt) + rem))
    return out


def thomas_coefficients(r, M):
    w = np.empty(M)
    c = np.empty(M)
    diag, off = 1.0 + 2.0 * r, -r
    for i in range(M):
        den = diag if i == 0 else diag - off * c[i - 1]
        w[i] = 1.0 / den
        c[i] = off * w[i]
    return w, c


def thomas_solve(r, f, w, c):
    """Solve (I - r D dx^2) y = f with the coefficients of thomas_coefficients."""
    M = len(f)
    off = -r
    fp = np.empty(M)
    for i in range(M):
        fp[i] = f[i] * w[i] if i == 0 else (f[i] - off * fp[i - 1]) * w[i]
    y = np.empty(M)
    y[M - 1] = fp[M - 1]
    for i in range(M - 2, -1, -1):
        y[i] = fp[i] - c[i] * y[i + 1]
    return y


def be_step(y, h, t_end, a0, a1, dx, s, forcing):
    """One backward Euler step of the semi-discrete heat equation."""
    r = (h * a_of(t_end, a0, a1)) / (dx * dx)
    w, c = thomas_coefficients(r, len(y))
    if forcing:
        hb = h * beta_of(t_end, a0, a1)
        f = y + hb * s
    else:
        f = np.array(y, dtype=np.float64)
    return thomas_solve(r, f, w, c)


def serial(M, a0, a1, forcing, t0, T, n_slices, dt, y0):
    """Backward Euler over [t0, T] with the method's own steps (slice by slice)."""
    dx, _, s = grid(M)
    L, S, rem = slice_steps(t0, T, n_slices, dt)
    y = np.array(y0, dtype=np.float64)
    for j in range(n_slices):
        for h, te in step_list(t0 + j * L, S, dt, rem):
            y = be_step(y, h, te, a0, a1, dx, s, forcing)
    return y


def build_tables(M, a0, a1, forcing, t0, T, n_slices, dt, slices=None):
    """The computation phase: G (N, M, M) and c (N, M); M+1 solves per slice.
    With ``slices``, only those slices (in that order)."""
    dx, _, s = grid(M)
    L, S, rem = slice_steps(t0, T, n_slices, dt)
    which = list(range(n_slices)) if slices is None else list(slices)
    G = np.empty((len(which), M, M))
    cvec = np.empty((len(which), M))
    for jj, j in enumerate(which):
        steps = step_list(t0 + j * L, S, dt, rem)
        y = np.zeros(M)
        for h, te in steps:
            y = be_step(y, h, te, a0, a1, dx, s, forcing)
        cvec[jj] = y
        for k in range(M):
            y = np.zeros(M)
            y[k] = 1.0
            for h, te in steps:
                y = be_step(y, h, te, a0, a1, dx, s, False)
            G[jj, :, k] = y
    return G, cvec


def compose(G, cvec, y0):
    """The communication phase: lambda_{j+1} = c_j + G_j lambda_j, every
    component summed left to right from c.  Returns lambda_0 .. lambda_N."""
    N, M, _ = G.shape
    lam = np.array(y0, dtype=np.float64)
    out = [lam.copy()]
    for j in range(N):
        # all components at once, each still c_i + G_i0 l_0 + G_i1 l_1 + ...
        # in that order: one elementwise product and one elementwise sum per k
        acc = np.array(cvec[j], dtype=np.float64)
        for k in range(M):
            acc = acc + G[j, :, k] * lam[k]
        lam = acc
        out.append(lam.copy())
    return np.array(out)


def exact(t, M):
    """The closed-form solution cos(t) sin(pi x) at the interior points."""
    _, x, _ = grid(M)
    return math.cos(t) * np.sin(math.pi * x)
