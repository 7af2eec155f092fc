"""The CPU throughput baseline (oracle/cpu_build.c) against the oracle.

It is not the oracle: it reorders the work (forcing per slice, 64
trajectories at a time, OpenMP threads).  Its FP64 tables must still equal the
oracle's bit for bit, since each entry takes the oracle's operations in the
oracle's order; its FP32 tables must meet the FP32 bar (1e-5 mixed)."""
import numpy as np
import pytest

CASES = [
    # rhs, params, t0, T, slices, grid n, lo, hi, steps
    ("logistic", (), 0.0, 10.0, 3, (37,), (-0.1,), (1.2,), 50),
    ("forced_cubic", (), 0.3, 2.3, 6, (21,), (-3.0,), (3.0,), 40),
    ("vdp", (3.5,), 0.0, 5.0, 3, (5, 7), (-3.0, -8.0), (3.0, 8.0), 30),
]


def oracle_tables(orc, case):
    rhs, params, t0, T, N, n, lo, hi, S = case
    g = orc.make_grid(n, lo, hi)
    return orc.build_tables(rhs, params, "rk4", t0, T, N, g, S)


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
@pytest.mark.parametrize("threads", [1, 3])
def test_fp64_build_equals_oracle_bit_for_bit(orc, case, threads):
    rhs, params, t0, T, N, n, lo, hi, S = case
    ref = oracle_tables(orc, case)
    got = orc.cpu_build(rhs, params, t0, T, N, n, lo, hi, S, "fp64", threads=threads)
    assert got.shape == ref.shape
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fp32_build_within_the_fp32_bar(orc, case):
    rhs, params, t0, T, N, n, lo, hi, S = case
    ref = oracle_tables(orc, case)
    got = orc.cpu_build(rhs, params, t0, T, N, n, lo, hi, S, "fp32", threads=2)
    # grid points that blow up within a slice (the logistic below 0) do so on both
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    err = np.max(np.abs(got[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1.0))
    assert err <= 1e-5, err


def test_slice_range_is_the_same_slices(orc):
    rhs, params, t0, T, N, n, lo, hi, S = CASES[1]
    full = orc.cpu_build(rhs, params, t0, T, N, n, lo, hi, S, "fp64")
    part = orc.cpu_build(rhs, params, t0, T, N, n, lo, hi, S, "fp64", slices=(2, 5))
    assert np.array_equal(part, full[:, 2:5])
