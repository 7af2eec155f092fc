"""Error recursion of sec. 5 evaluated along one composition chain.

Used by the GPU tests to bound the difference between the method run over the
GPU's FP32 tables and the same method over FP64 tables (the oracle's), when
every FP32 entry meets the parity bar |t32 - t64| <= tol * max(|t64|, 1).

Sec. 5 splits the global error into the error each slice adds and the error
earlier slices carry through the later slice maps (their Lipschitz constants).
Here the per-slice term is the interpolant's amplification of the table error
at the lookup (the sum of the absolute weights it gives the table values it
reads), and the carrying factor is the interpolant's own Jacobian at each
lookup instead of a global Lipschitz constant.  The recursion is linearised,
so the result is doubled.
"""
from __future__ import annotations

import numpy as np


def _hermite_terms(n, cell, w):
    """Weights of the table values in the cubic Hermite interpolant with
    finite-difference slopes (slope times spacing: (t[i+1] - t[i-1]) / 2
    inside, ((4 t1 - 3 t0) - t2) / 2 and ((3 t[n-1] - 4 t[n-2]) + t[n-3]) / 2 at
    the ends) at weight w of the cell, and their derivatives in w."""
    h = np.array([2 * w**3 - 3 * w**2 + 1, w**3 - 2 * w**2 + w, -2 * w**3 + 3 * w**2,
                  w**3 - w**2])
    dh = np.array([6 * w**2 - 6 * w, 3 * w**2 - 4 * w + 1, -6 * w**2 + 6 * w,
                   3 * w**2 - 2 * w])

    def slope(i):
        if i == 0:
            return {0: -1.5, 1: 2.0, 2: -0.5}
        if i == n - 1:
            return {n - 1: 1.5, n - 2: -2.0, n - 3: 0.5}
        return {i + 1: 0.5, i - 1: -0.5}

    coef, dcoef = {}, {}
    parts = [({cell: 1.0}, 0), (slope(cell), 1), ({cell + 1: 1.0}, 2), (slope(cell + 1), 3)]
    for terms, b in parts:
        for k, v in terms.items():
            coef[k] = coef.get(k, 0.0) + h[b] * v
            dcoef[k] = dcoef.get(k, 0.0) + dh[b] * v
    idx = np.array(sorted(coef))
    return idx, np.array([coef[k] for k in idx]), np.array([dcoef[k] for k in idx])


def _slice_terms(w, tabs, j, cell, wt):
    """(Jacobian of slice j's interpolant at the lookup, amplification of a
    table error, largest table value read)."""
    n = w.grid_n
    dxi = [(hi - lo) / (m - 1) for lo, hi, m in zip(w.grid_lo, w.grid_hi, n)]
    if w.dim == 1:
        t, i, x = tabs[0, j], int(cell[0]), float(wt[0])
        if w.interp == "linear":
            idx = np.array([i, i + 1])
            coef = np.array([1.0 - x, x])
            dcoef = np.array([-1.0, 1.0])
        elif w.interp == "hermite":
            idx, coef, dcoef = _hermite_terms(n[0], i, x)
        else:
            raise ValueError(w.interp)
        vals = t[idx]
        J = np.array([[float(np.dot(dcoef, vals)) / dxi[0]]])
        return J, float(np.sum(np.abs(coef))), float(np.max(np.abs(vals)))
    if w.interp != "bilinear":
        raise ValueError(w.interp)
    i0, i1 = (int(c) for c in cell)
    w0, w1 = (float(v) for v in wt)
    J, ymax = np.zeros((2, 2)), 0.0
    for c in range(2):
        t = tabs[c, j].reshape(n)
        t00, t01, t10, t11 = t[i0, i1], t[i0, i1 + 1], t[i0 + 1, i1], t[i0 + 1, i1 + 1]
        J[c, 0] = ((t10 - t00) * (1 - w1) + (t11 - t01) * w1) / dxi[0]
        J[c, 1] = ((t01 - t00) * (1 - w0) + (t11 - t10) * w0) / dxi[1]
        ymax = max(ymax, abs(t00), abs(t01), abs(t10), abs(t11))
    amp = (abs(1.0 - w0) + abs(w0)) * (abs(1.0 - w1) + abs(w1))
    return J, amp, ymax


def chain_bound(w, tabs, o, tol):
    """Componentwise bound, per boundary state (shape (N + 1, dim)), on the
    difference between the chain over ``tabs`` (whose lookups ``o`` records:
    the oracle's composition over those tables) and the chain over tables
    that differ from them entry by entry by at most tol * max(|t|, 1).

    Slice j adds an error delta_j = tol * max(|t|, 1) * amplification in any
    direction; later slices carry it through their Jacobians."""
    V = np.zeros((0, w.dim))
    out = np.zeros((w.n_slices + 1, w.dim))
    for j in range(w.n_slices):
        J, amp, ymax = _slice_terms(w, tabs, j, o.cells[j], o.weights[j])
        delta = tol * max(1.0, ymax) * amp
        if len(V):
            V = V @ J.T
        V = np.vstack([V, delta * np.eye(w.dim)])
        out[j + 1] = 2.0 * np.sum(np.abs(V), axis=0)
    return out
