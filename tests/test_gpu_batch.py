"""GPU parity of the batched path (one persistent, graph-captured launch for
many uneven problems) against the single-problem path and the CPU oracle."""
import sys

import numpy as np
import pytest

from chain_bounds import chain_bound
from paper_1304_6514_amd import nv
from paper_1304_6514_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


def say(*a):
    print("[gpu-test]", *a, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nv.load()
    return torch


def small_batch():
    probs = W.batched_problems(count=12, seed=7, scale=0.08)
    # add the other autonomous right-hand side and a Hermite lookup
    probs.append(W.Workload("batch-square", "square", (), 0.0, 0.5, 5, (77,), (0.0,), (2.0,), 40,
                            (1.0,), "fp32", "hermite"))
    return probs


def mixed_err(g, o):
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), 1.0)))


def single_path(w):
    from paper_1304_6514_amd.propagator import Propagator
    with Propagator("cuda:0", traj_per_lane=1) as p:
        p.build(w)
        r = p.compose()
        tabs = [p.table(c) for c in range(w.dim)]
    return r, tabs


def test_batch_equals_single_problem_path(torch):
    from paper_1304_6514_amd.propagator import Batch
    probs = small_batch()
    say("batch vs single", len(probs))
    with Batch(probs) as b:
        st, yT, infos = b.run()
        assert st == nv.NV_OK
        for i, w in enumerate(probs):
            r, tabs = single_path(w)
            for c in range(w.dim):
                assert np.array_equal(b.table(i, c), tabs[c]), (i, w.name)
            assert np.array_equal(b.boundary(i), r.boundary), (i, w.name)
            assert np.array_equal(yT[i, :w.dim], r.yT)
            assert infos[i][0] == r.n_out_of_grid


def test_batch_schedules_give_identical_results(torch):
    from paper_1304_6514_amd.propagator import Batch
    probs = small_batch()
    with Batch(probs) as b:
        _, ref, _ = b.run()
        tabs = [b.table(i) for i in range(len(probs))]
        for P, wpc, order in [({0: 2, 1: 4, 3: 2, 4: 1}, 4, 1), ({0: 4, 1: 2, 3: 4, 4: 2}, 8, 0),
                              ({0: 1, 1: 1, 3: 1, 4: 4}, 1, 0)]:
            say("schedule", P, wpc, order)
            b.set_schedule(P, wpc, order)
            st, yT, _ = b.run()
            assert st == nv.NV_OK and np.array_equal(yT, ref)
            assert all(np.array_equal(b.table(i), tabs[i]) for i in range(len(probs)))
        chosen = b.autotune(reps=1)
        say("autotuned", list(chosen.traj_per_lane), chosen.workgroups_per_cu, chosen.order)
        st, yT, _ = b.run()
        assert st == nv.NV_OK and np.array_equal(yT, ref)


def test_batch_graph_replays_match_eager_results(torch):
    # the graph is replayed several times with other eager GPU work and
    # synchronisations in between; every replay must equal the eager path
    from paper_1304_6514_amd.propagator import Batch, Propagator
    probs = small_batch()[:6]
    eager = [single_path(w)[0] for w in probs]
    with Batch(probs) as b, Propagator("cuda:0") as other:
        for rep in range(4):
            say("replay", rep)
            st, yT, _ = b.run()
            assert st == nv.NV_OK
            for i, w in enumerate(probs):
                assert np.array_equal(yT[i, :w.dim], eager[i].yT), (rep, i)
                assert np.array_equal(b.boundary(i), eager[i].boundary)
            other.build(W.small(W.FORCED_CUBIC_FP32, 8, (300,), 50))
            other.compose()
            torch.cuda.synchronize()


def test_batch_oracle_parity_full_size(orc, torch):
    from paper_1304_6514_amd.propagator import Batch
    probs = W.batched_problems()
    say("full batch", len(probs), "problems", sum(w.trajectory_steps for w in probs))
    with Batch(probs) as b:
        chosen = b.autotune(reps=1)
        say("autotuned", list(chosen.traj_per_lane), chosen.workgroups_per_cu, chosen.order)
        st, yT, infos = b.run()
        ms, steps = b.last_timing()
        say("batch run ms", ms, "traj-steps/s", steps / (ms * 1e-3))
        assert st == nv.NV_OK
        worst_tab, worst_d = 0.0, 0.0
        for i, w in enumerate(probs):
            g = orc.make_grid(w.grid_n, w.grid_lo, w.grid_hi)
            tabs = np.stack([b.table(i, c).astype(np.float64) for c in range(w.dim)])
            # sampled table entries against the oracle's FP64 integration
            sl, pt = W.sample_entries(w, 28, seed=100 + i)
            ref = orc.table_entries(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices, g,
                                    w.steps_per_slice, sl, pt)
            err = mixed_err(tabs[:, sl, pt], ref)
            worst_tab = max(worst_tab, err)
            assert err <= TOL32, (i, w.name, err)
            # composition over the batch's own tables: bit-exact
            o = orc.compose_tables(g, w.interp, tabs, w.y0)
            assert o.status == 0
            assert np.array_equal(b.boundary(i), o.boundary), (i, w.name)
            assert infos[i][0] == o.n_out_of_grid
            # the same method with FP64 tables, within the error recursion of
            # sec. 5 evaluated along this chain (chain_bound)
            lazy = orc.method_lazy(w.rhs, w.params, w.scheme, w.t0, w.T, w.n_slices, g,
                                   w.steps_per_slice, w.interp, w.y0)
            d = np.abs(o.boundary - lazy.boundary)
            bound = chain_bound(w, tabs, o, TOL32)
            worst_d = max(worst_d, float(np.max(d[1:] / bound[1:])))
            assert np.all(d <= bound), (i, w.name, float(np.max(d)), float(np.max(bound)))
        say("batch worst sampled table error", worst_tab,
            "worst fp32-vs-fp64 method difference as a fraction of its bound", worst_d)


def test_batch_errors(torch):
    from paper_1304_6514_amd.propagator import Batch
    with pytest.raises(nv.NvError) as e:
        Batch([W.small(W.FORCED_CUBIC_FP32, 4, (64,), 10)])
    assert e.value.status == nv.NV_ERR_UNSUPPORTED
    bad = small_batch()[:3] + [W.Workload("bad", "logistic", (), 0.0, 1.0, 0, (10,), (0.0,),
                                          (1.0,), 5, (0.5,), "fp32", "linear")]
    with pytest.raises(nv.NvError) as e:
        Batch(bad)
    assert e.value.status == nv.NV_ERR_INVALID_ARG and "problem 3" in str(e.value)
    with Batch(small_batch()[:2]) as b:
        for get in (lambda: b.table(0), lambda: b.boundary(1)):
            with pytest.raises(nv.NvError) as e:
                get()                   # nothing to hand out before the first run
            assert e.value.status == nv.NV_ERR_NOT_BUILT
        s = nv.nv_batch_schedule()
        for r in range(5):
            s.traj_per_lane[r] = 3
        s.workgroups_per_cu = 8
        with pytest.raises(nv.NvError):
            nv.nv_batch_set_schedule(b.batch, s)
        st, _, _ = b.run()          # the batch still runs with its old schedule
        assert st == nv.NV_OK
