"""The cost model of sec. 4.

GPU time to solution, eq. (gpucostmodel): C_G = (M n / N) tau_F + N tau_N + tau_K,
with n = T / dt time steps in all, M initial values per slice, N slices;
serial time, eq. (serialcostmodel): C_C = n tau_F^cpu.  `fit` recovers
(tau_F, tau_N, tau_K) from measured times by least squares, as the paper does
for its Table 4.
"""
from __future__ import annotations

import numpy as np


def gpu_cost(M, n, N, tau_F, tau_N, tau_K):
    return M * n / N * tau_F + N * tau_N + tau_K


def serial_cost(n, tau_F_cpu):
    return n * tau_F_cpu


def fit(rows):
    """rows: iterable of (M, n, N, time).  Returns (tau_F, tau_N, tau_K) in the
    unit of time, least squares over all rows."""
    rows = np.asarray(list(rows), dtype=np.float64)
    M, n, N, t = rows.T
    A = np.stack([M * n / N, N, np.ones_like(N)], axis=1)
    coef, *_ = np.linalg.lstsq(A, t, rcond=None)
    return tuple(float(c) for c in coef)
