"""The paper's own configuration on the GPU: y' = y^2, backward Euler with the
paper's fixed step, Lagrange interpolation on Chebyshev extrema (sec. 3 and 4)."""
import os
import sys

import numpy as np
import pytest

from paper_1304_6514_amd import nv
from paper_1304_6514_amd import workloads as W

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print("[gpu-test]", *a, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def prop():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nv.load()
    from paper_1304_6514_amd.propagator import Propagator
    p = Propagator("cuda:0")
    yield p
    p.close()


def _rows(name):
    out = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.split("#", 1)[0].strip()
        if line:
            out.append([float(v) for v in line.split()])
    return out


def mixed_err(g, o):
    return float(np.max(np.abs(np.asarray(g, float) - o) / np.maximum(np.abs(o), 1.0)))


def _check_against_oracle(orc, prop, w, tol):
    r = prop.solve(w)
    tab = prop.table(0).astype(np.float64)
    M = w.grid_n[0]
    ref = orc.paper_tables(w.T, w.n_slices, M, w.grid_lo[0], w.grid_hi[0], w.dt)
    assert mixed_err(tab, ref) <= tol
    o = orc.paper_compose(M, w.grid_lo[0], w.grid_hi[0], tab, w.y0[0])
    assert r.status == nv.NV_OK and o.status == 0
    assert np.array_equal(r.boundary[:, 0], o.boundary[:, 0])       # bit-exact
    assert r.n_out_of_grid == o.n_out_of_grid
    return r


def test_table1_reproduced_on_gpu(orc, prop):
    worst = 0.0
    for row in _rows("paper_table1.txt"):
        dt, printed = row[0], row[1:]
        for M, want in zip(range(3, 8), printed):
            w = W.paper_model(4, M, dt, "fp64")
            r = _check_against_oracle(orc, prop, w, 1e-12)
            got = abs(r.yT[0] - 2.0)
            worst = max(worst, abs(got - want) / want)
            assert got == pytest.approx(want, rel=0.02), (dt, M, got, want)
    say("Table 1 on the GPU: worst relative deviation from the printed cells", worst)


def test_table3_shapes_in_single_precision(orc, prop):
    for dt, N, M in W.PAPER_TABLE3:
        w = W.paper_model(N, M, dt, "fp32")
        r = _check_against_oracle(orc, prop, w, 1e-5)
        err = abs(r.yT[0] - 2.0)
        serial = abs(orc.paper_serial(0.5, dt, 1.0) - 2.0)
        say("Table 3 shape", dt, N, M, "error", err, "serial BE error", serial)
        # sec. 4: the method's error is comparable to the time-stepping error
        assert err <= 2.0 * serial


def test_fixed_step_mode_matches_equal_steps(prop):
    w = W.small(W.LOGISTIC_FP64, 8, (300,), 125).with_(T=1.0)    # L = 0.125, h = 0.001
    prop.build(w)
    a = prop.table(0)
    prop.build(w.with_(dt=0.001))
    b = prop.table(0)
    assert np.array_equal(a, b)


def test_backward_euler_on_linear_problem_is_exact(prop):
    # one Newton step solves the linear implicit equation exactly:
    # y_{n+1} = y_n / (1 - lambda h), so a slice maps xi to xi / (1 - lambda h)^S
    lam, S = -1.7, 40
    w = W.Workload("be-linear", "linear", (lam,), 0.0, 2.0, 5, (101,), (-2.0,), (2.0,), S,
                   (1.0,), "fp64", "linear", scheme="be")
    prop.build(w)
    h = (2.0 / 5) / S
    xi = np.linspace(-2.0, 2.0, 101)
    np.testing.assert_allclose(prop.table(0), np.tile(xi / (1 - lam * h) ** S, (5, 1)),
                               rtol=1e-13, atol=1e-15)


def test_paper_mode_argument_errors(prop):
    with pytest.raises(nv.NvError) as e:
        prop.build(W.small(W.VDP_FP32, 2, (4, 4), 3).with_(scheme="be"))
    assert e.value.status == nv.NV_ERR_UNSUPPORTED
    with pytest.raises(nv.NvError) as e:
        prop.build(W.paper_model(4, 65, 1e-3))
    assert e.value.status == nv.NV_ERR_INVALID_ARG
    with pytest.raises(nv.NvError) as e:
        prop.build(W.small(W.FORCED_CUBIC_FP32, 2, (16,), 3).with_(dt=0.01))
    assert e.value.status == nv.NV_ERR_INVALID_ARG


def test_chebyshev_nodes_survive_other_builds_in_between(prop):
    # a forced build writes its forcing values over the start of the scratch,
    # where a Chebyshev build of 32 slices keeps its nodes; the next Chebyshev
    # build must not take the overwritten values for its nodes
    forced = W.small(W.FORCED_CUBIC_FP32, 64, (256,), 50)
    cheb = W.paper_model(32, 5, 2.0 ** -14, "fp64")
    prop.build(forced)                 # scratch large enough for both from here on
    first = prop.solve(cheb)
    prop.build(forced)
    again = prop.solve(cheb)
    assert np.array_equal(first.boundary, again.boundary)
    prop.build(W.small(W.LOGISTIC_FP64, 512, (64,), 10))   # counters and carry over the nodes
    third = prop.solve(cheb)
    assert np.array_equal(first.boundary, third.boundary)
