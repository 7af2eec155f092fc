"""The cost model of sec. 4 against the numbers the paper prints (Tables 3, 4)."""
import os

import numpy as np
import pytest

from paper_1304_6514_amd import costmodel

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if line:
            out.append([float(v) for v in line.split()])
    return out


def test_table3_estimates_follow_from_table4():
    tau_F, tau_N, tau_K, tau_cpu = _rows("paper_table4.txt")[0]
    for dt, N, M, total, speedup, est in _rows("paper_table3.txt"):
        n = 0.5 / dt
        assert costmodel.gpu_cost(M, n, N, tau_F, tau_N, tau_K) == pytest.approx(est, rel=0.006)
        # the printed speedup is the serial model time over the measured total
        assert costmodel.serial_cost(n, tau_cpu) / total == pytest.approx(speedup, rel=0.06)


def test_fit_recovers_known_parameters():
    rng = np.random.default_rng(0)
    rows = [(M, 0.5 / dt, N, costmodel.gpu_cost(M, 0.5 / dt, N, 0.04, 0.7, 137.0))
            for dt in (2.0 ** -14, 2.0 ** -15, 2.0 ** -16) for N in (32, 64, 128)
            for M in (4, int(rng.integers(5, 8)))]
    assert costmodel.fit(rows) == pytest.approx((0.04, 0.7, 137.0), rel=1e-9)


def test_fit_of_the_printed_totals():
    # the printed Table 4 values were not fitted to Table 3's totals alone: a
    # least-squares fit of those totals gives different, but same-order, values
    rows = [(M, 0.5 / dt, N, total) for dt, N, M, total, _, _ in _rows("paper_table3.txt")]
    tau_F, tau_N, tau_K = costmodel.fit(rows)
    assert 0.02 < tau_F < 0.06 and 0.3 < tau_N < 2.0 and 50 < tau_K < 200
