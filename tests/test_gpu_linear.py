"""GPU parity of the affine basis propagator (heat equation of sec. 6): the
tables equal the oracle's to the bit (FP64, one rounding per operation, the
same Thomas form on both sides); the composition lambda_{j+1} = c_j + G_j
lambda_j (sec. 5, equation `linearreconstruct`) stays within a rounding bound
of the oracle's index-order sums (the paper fixes the map, not the order of
its sums); and the method equals serial backward Euler up to rounding, as the
paper states for linear problems."""
import math
import sys

import numpy as np
import pytest

from oracle import linear_oracle as lo
from paper_1304_6514_amd import nv
from paper_1304_6514_amd.linear import HeatWorkload

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-test]", *a, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def lin():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1304_6514_amd.linear import LinearPropagator
    nv.load()
    p = LinearPropagator()
    yield p
    p.close()


U64 = 2.0 ** -53


def chain_bound(G, c, lam_a, lam_b):
    """Componentwise bound on |lam_a - lam_b| for two FP64 evaluations of the
    same affine chain lambda_{j+1} = c_j + G_j lambda_j that differ only in
    the order of each component's M + 1 terms.  One evaluation of
    c_i + sum_k G_ik l_k in any order rounds each product once and each term
    passes through at most M additions, so it is within
    gamma_{M+1} (|c_i| + sum_k |G_ik| |l_k|) of the exact value,
    gamma_n = n u / (1 - n u) (the standard inner-product bound).  The two
    chains' difference d_j then obeys
        d_{j+1} <= |G_j| d_j + gamma_{M+1} (2 |c_j| + |G_j| (|lam_a,j| + |lam_b,j|)).
    Evaluated in FP64 and widened by 1 % for the bound's own rounding."""
    N, M, _ = G.shape
    g = (M + 1) * U64 / (1.0 - (M + 1) * U64)
    d = np.zeros(M)
    out = [d.copy()]
    for j in range(N):
        A = np.abs(G[j])
        d = A @ d + g * (2.0 * np.abs(c[j]) + A @ (np.abs(lam_a[j]) + np.abs(lam_b[j])))
        out.append(d * 1.01)
    return np.array(out)


def check_chain(G, c, got, ref, what):
    """got and ref are lambda_0 .. lambda_N of the same chain over (G, c)."""
    assert got.shape == ref.shape and np.array_equal(got[0], ref[0])
    bound = chain_bound(G, c, got, ref)
    diff = np.abs(got - ref)
    assert np.all(np.isfinite(got))
    ok = diff <= bound
    worst = float(np.max(diff[1:] / np.maximum(bound[1:], 1e-300)))
    say(f"  {what}: max |gpu - oracle| = {float(np.max(diff)):.3g}, "
        f"max bound = {float(np.max(bound)):.3g}, worst diff/bound = {worst:.3g}, "
        f"bit-equal components {int(np.sum(diff[1:] == 0))}/{diff[1:].size}")
    assert np.all(ok), f"{what}: outside the rounding bound at {np.argwhere(~ok)[:5]}"


CASES = [HeatWorkload("heat-M9-dt0.005-N8", 9, 0.005, 8, T=1.0),
         HeatWorkload("heat-M9-dt0.003-N7-remainder", 9, 0.003, 7, T=1.0),
         HeatWorkload("heat-M1", 1, 0.01, 3, T=0.5),
         HeatWorkload("heat-M63-two-waves", 63, 0.002, 5, T=0.1),
         HeatWorkload("heat-M70-unforced", 70, 0.001, 4, T=0.05, forcing=False),
         HeatWorkload("heat-M127-max", 127, 0.001, 3, T=0.02)]


@pytest.mark.parametrize("w", CASES, ids=lambda w: w.name)
def test_tables_bit_exact_and_composition_within_rounding(lin, w):
    say("linear", w.name)
    lin.build(w)
    G, c = lin.tables()
    Go, co = lo.build_tables(w.M, w.a0, w.a1, w.forcing, w.t0, w.T, w.n_slices, w.dt)
    assert np.array_equal(G, Go) and np.array_equal(c, co)
    y0 = lo.exact(w.t0, w.M) + 0.1 * np.cos(np.arange(w.M))
    st, yT, bnd = lin.compose(y0)
    assert st == nv.NV_OK
    ref = lo.compose(Go, co, y0)
    assert np.array_equal(yT, bnd[-1])
    check_chain(Go, co, bnd, ref, w.name)


@pytest.mark.parametrize("M,dt,N", [(9, 0.005, 128), (19, 0.001, 256), (99, 0.0005, 1024)])
def test_paper_sizes_method_equals_serial_backward_euler(lin, M, dt, N):
    """Tables 5, 7 and 8 of sec. 6 (dx = 0.1, 0.05, 0.01; T = 10): the method's
    y(T) equals serial backward Euler with the same steps to rounding, and
    sampled slices' tables equal the oracle's to the bit."""
    w = HeatWorkload(f"heat-M{M}", M, dt, N)
    say(f"linear paper size M={M} dt={dt} N={N}")
    lin.build(w)
    b_ms, _ = lin.last_timing()
    y0 = lo.exact(0.0, M)
    st, yT, bnd = lin.compose(y0)
    _, c_ms = lin.last_timing()
    assert st == nv.NV_OK and np.array_equal(yT, bnd[-1])
    serial = lo.serial(M, w.a0, w.a1, True, w.t0, w.T, N, dt, y0)
    diff = float(np.max(np.abs(yT - serial)))
    err = float(np.max(np.abs(yT - lo.exact(w.T, M))))
    say(f"  build {b_ms:.3f} ms, compose {c_ms:.3f} ms, |method - serial BE| = {diff:.3g}, "
        f"|method - cos(t) sin(pi x)| = {err:.3g}")
    assert diff <= 1e-12 * max(1.0, float(np.max(np.abs(serial))))
    assert err < 0.02
    G, c = lin.tables()
    pick = [0, N // 2, N - 1]
    Go, co = lo.build_tables(M, w.a0, w.a1, True, w.t0, w.T, N, dt, slices=pick)
    assert np.array_equal(G[pick], Go) and np.array_equal(c[pick], co)
    # the whole chain against the oracle's composition over the GPU's tables
    check_chain(G, c, bnd, lo.compose(G, c, y0), f"chain M={M} N={N}")


def test_linear_argument_errors(lin):
    with pytest.raises(nv.NvError) as e:
        lin.build(HeatWorkload("bad-M", 128, 0.01, 4))
    assert e.value.status == nv.NV_ERR_INVALID_ARG
    with pytest.raises(nv.NvError) as e:
        lin.build(HeatWorkload("bad-a", 9, 0.01, 4, a0=-1.0, a1=0.25))
    assert e.value.status == nv.NV_ERR_INVALID_ARG and "not positive" in str(e.value)
    with pytest.raises(nv.NvError) as e:
        lin.build(HeatWorkload("bad-dt", 9, 0.0, 4))
    assert e.value.status == nv.NV_ERR_INVALID_ARG
    # a failed build leaves nothing to compose
    with pytest.raises(nv.NvError) as e:
        nv.nv_lin_compose(lin.h, np.zeros(9), 9, 4)
    assert e.value.status == nv.NV_ERR_NOT_BUILT


def test_linear_first_nonpositive_diffusion_is_named_over_many_steps(lin):
    """With many steps the library evaluates the per-step scalars on several
    host threads; the error still names the first step end (in time order)
    where a(t) = a0 + a1 sin t is not positive, as the oracle's step list
    finds it."""
    w = HeatWorkload("bad-a-late", 9, 0.0005, 1024, a0=0.1, a1=1.0)
    L, S, rem = lo.slice_steps(w.t0, w.T, w.n_slices, w.dt)
    first = None
    for j in range(w.n_slices):
        for _, te in lo.step_list(w.t0 + j * L, S, w.dt, rem):
            if not lo.a_of(te, w.a0, w.a1) > 0.0:
                first = te
                break
        if first is not None:
            break
    assert first is not None and 3.0 < first < 3.5
    say("first non-positive a(t) at", first)
    with pytest.raises(nv.NvError) as e:
        lin.build(w)
    assert e.value.status == nv.NV_ERR_INVALID_ARG
    assert f"at t = {first:g}" in str(e.value), str(e.value)


def test_linear_nonfinite_state_is_reported(lin):
    w = HeatWorkload("heat-M9-nan", 9, 0.01, 5, T=0.5)
    lin.build(w)
    y0 = lo.exact(0.0, 9)
    y0[3] = np.nan
    st, yT, bnd = lin.compose(y0)
    assert st == nv.NV_ERR_NONFINITE
    assert not np.all(np.isfinite(bnd[1]))


def test_linear_single_slice_equals_serial(lin):
    w = HeatWorkload("heat-M19-N1", 19, 0.01, 1, T=0.7)
    lin.build(w)
    y0 = lo.exact(0.0, 19)
    st, yT, _ = lin.compose(y0, want_boundary=False)
    G, c = lo.build_tables(19, 1.0, 0.25, True, 0.0, 0.7, 1, 0.01)
    assert st == nv.NV_OK
    ref = lo.compose(G, c, y0)
    check_chain(G, c, np.stack([y0, yT]), ref, "one slice")


# ---- many initial values on the matrix cores --------------------------------

@pytest.mark.parametrize("w", CASES + [HeatWorkload("heat-M99-N40", 99, 0.0005, 40, T=0.5)],
                         ids=lambda w: w.name)
def test_compose_many_within_rounding_bound_of_oracle(lin, w):
    """nv_lin_compose_many: 37 chains (two full groups of 16 and a ragged
    third) through the same tables; every chain's boundary states stay within
    the FP64 inner-product rounding bound of the oracle's index-order chain."""
    import torch
    say("linear many", w.name)
    lin.build(w)
    G, c = lin.tables()
    Q = 37
    rng = np.random.default_rng(71)
    y0 = rng.normal(0.0, 1.0, (Q, w.M))
    st, yT, bnd = lin.compose_many(y0, want_boundary=True)
    torch.cuda.synchronize()
    assert st == nv.NV_OK
    yT, bnd = yT.cpu().numpy(), bnd.cpu().numpy()
    assert np.array_equal(yT, bnd[:, -1]) and np.array_equal(bnd[:, 0], y0)
    for q in (0, 15, 16, 31, 32, 36):
        check_chain(G, c, bnd[q], lo.compose(G, c, y0[q]), f"{w.name} chain {q}")
    # without boundary states: the same final states
    st, yT2, _ = lin.compose_many(y0)
    assert st == nv.NV_OK and np.array_equal(yT2.cpu().numpy(), yT)


@pytest.mark.parametrize("w", [HeatWorkload("heat-M19-N30", 19, 0.001, 30, T=0.3),
                               HeatWorkload("heat-M99-N12", 99, 0.0005, 12, T=0.12),
                               HeatWorkload("heat-M120-N8", 120, 0.0005, 8, T=0.08)],
                         ids=lambda w: w.name)
def test_compose_many_large_counts_equal_small_ones(lin, w):
    """With chains enough for two workgroups per CU (16,384 on 256 CUs), a
    workgroup carries two blocks of 16 chains that share its table reads
    (M <= 116; M = 120 keeps one block): every chain's states are those of the
    same chain in a small run, to the bit, and within the rounding bound of the
    oracle's chain."""
    import torch
    say("linear many, large count", w.name)
    lin.build(w)
    G, c = lin.tables()
    Q = 16384 + 37
    rng = np.random.default_rng(72)
    y0 = rng.normal(0.0, 1.0, (Q, w.M))
    st, yT, bnd = lin.compose_many(y0, want_boundary=True)
    torch.cuda.synchronize()
    assert st == nv.NV_OK
    yT, bnd = yT.cpu().numpy(), bnd.cpu().numpy()
    assert np.array_equal(yT, bnd[:, -1]) and np.array_equal(bnd[:, 0], y0)
    pick = [0, 15, 16, 31, 32, 33, 47, 8191, 16383, 16384, 16399, 16400, Q - 1]
    st, yT_s, bnd_s = lin.compose_many(y0[pick], want_boundary=True)
    torch.cuda.synchronize()
    assert st == nv.NV_OK
    assert np.array_equal(bnd_s.cpu().numpy().view(np.int64), bnd[pick].view(np.int64))
    for q in (0, 31, 16383, Q - 1):
        check_chain(G, c, bnd[q], lo.compose(G, c, y0[q]), f"{w.name} chain {q}")


def test_compose_many_reports_a_nonfinite_chain(lin):
    import torch
    w = HeatWorkload("heat-M9-nan-many", 9, 0.01, 5, T=0.5)
    lin.build(w)
    y0 = np.tile(lo.exact(0.0, 9), (20, 1))
    y0[17, 3] = np.nan
    st, yT, _ = lin.compose_many(y0)
    torch.cuda.synchronize()
    assert st == nv.NV_ERR_NONFINITE and "slice 0" in nv.nv_last_error()
    yT = yT.cpu().numpy()
    assert not np.all(np.isfinite(yT[17])) and np.all(np.isfinite(np.delete(yT, 17, 0)))
    with pytest.raises(nv.NvError) as e:
        nv.nv_lin_compose_many(lin.h, None, 4, None)
    assert e.value.status == nv.NV_ERR_INVALID_ARG
