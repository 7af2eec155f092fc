"""GPU parity of the learned slice-map surrogate against its FP64 oracle: the
network's forward pass, the loss and gradient of a minibatch, the Adam update,
a short training run, the training-set gather and the composition with the
network, with and without the table fallback.

Tolerances.  The oracle is run twice: in FP64 throughout, and with bfloat16
rounding at the points where the kernels feed the matrix cores (operands of
the two 128 x 128 layers, of their back-propagation and of every gradient sum).
Against the second the only differences left are FP32 against FP64
accumulation, the FP32 evaluation of erf (absolute error below 1.5e-7) and the
rare bfloat16 rounding that these flip; against the first, the bfloat16
rounding itself (unit roundoff 2^-9 = 2.0e-3 per operand) bounds the relative
error of every matrix product, which gives the looser bars below."""
import sys

import numpy as np
import pytest

from oracle import mlp_oracle as mo
from paper_1304_6514_amd import nv
from paper_1304_6514_amd import workloads as W

pytestmark = pytest.mark.gpu

SHIFT = np.array(W.SUR_IN_SHIFT)
SCALE = np.array(W.SUR_IN_SCALE, dtype=np.float32).astype(np.float64)
OUT_SCALE = np.array(W.SUR_OUT_SCALE)
# the step-doubling form of the workload
SD_KW = dict(correction="step-doubling", coarse_steps=1, out_scale=W.SUR_SD_OUT_SCALE,
             gate=W.SUR_SD_GATE, loss_scale=W.SUR_SD_LOSS_SCALE)


def say(*a):
    print("[gpu-test]", *a, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    nv.load()
    return torch


@pytest.fixture(scope="module")
def sur(torch):
    from paper_1304_6514_amd.surrogate import Surrogate
    s = Surrogate("cuda:0", max_batch=8192)
    yield s
    s.close()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def test_forward_matches_oracle(sur):
    p = W.surrogate_init_params(1)
    sur.set_params(p)
    x, _ = W.surrogate_samples(1000, seed=2)          # 1000: not a multiple of 16 or 64
    say("forward n=1000")
    out = sur.forward(x).cpu().numpy().T
    emu, _ = mo.forward(p.astype(np.float64), x.T.astype(np.float64), SHIFT, SCALE,
                        emulate_bf16=True)
    ref, _ = mo.forward(p.astype(np.float64), x.T.astype(np.float64), SHIFT, SCALE)
    e_emu, e_ref = np.max(np.abs(out - emu)), np.max(np.abs(out - ref))
    say(f"forward: max |gpu - oracle(bf16)| = {e_emu:.3g}, |gpu - oracle(fp64)| = {e_ref:.3g}, "
        f"max |out| = {np.max(np.abs(ref)):.3g}")
    assert e_emu < 1e-4
    assert e_ref < 2e-2 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [16, 4112])
def test_loss_and_gradient_match_oracle(sur, n):
    p = W.surrogate_init_params(3)
    sur.set_params(p)
    x, t = W.surrogate_samples(n, seed=4)
    say(f"loss_grad n={n}")
    loss, g = sur.loss_grad(x, t)
    p64 = p.astype(np.float64)
    l_emu, g_emu = mo.loss_and_grad(p64, x.T.astype(np.float64), t.T.astype(np.float64), SHIFT,
                                    SCALE, emulate_bf16=True)
    l_ref, g_ref = mo.loss_and_grad(p64, x.T.astype(np.float64), t.T.astype(np.float64), SHIFT,
                                    SCALE)
    assert abs(loss - l_emu) <= 1e-5 * l_emu, (loss, l_emu)
    assert abs(loss - l_ref) <= 1e-3 * l_ref, (loss, l_ref)
    gu = mo.unflatten(g)
    worst = []
    for name, _ in mo.SHAPES:
        r_emu, r_ref = _rel(gu[name], g_emu[name]), _rel(gu[name], g_ref[name])
        worst.append((name, r_emu, r_ref))
        assert r_emu < 2e-3, (name, r_emu)
        assert r_ref < 3e-2, (name, r_ref)
    say("gradient rel. L2 error vs oracle (bf16-emulating, fp64): " +
        ", ".join(f"{k} {a:.2g}/{b:.2g}" for k, a, b in worst))


def test_adam_update_matches_oracle(sur, torch):
    p = W.surrogate_init_params(5)
    sur.set_params(p)
    x, t = W.surrogate_samples(2048, seed=6)
    opt = mo.Adam(mo.N_PARAMS, lr=2e-3, beta1=0.9, beta2=0.99, eps=1e-8)
    theta = p.astype(np.float64)
    for k in range(3):
        _, g = sur.loss_grad(x, t)                    # gradient at the current parameters
        theta = opt.step(theta, g.astype(np.float64))
        sur.train(x, t, batch=2048, steps=1, lr=2e-3, beta1=0.9, beta2=0.99, eps=1e-8)
        got = sur.params().astype(np.float64)
        err = np.max(np.abs(got - theta))
        say(f"adam step {k + 1}: max |gpu - oracle| = {err:.3g}")
        assert err < 1e-6
    # the bf16 copies of the weights follow the update
    out = sur.forward(x[:, :256]).cpu().numpy().T
    emu, _ = mo.forward(sur.params().astype(np.float64), x[:, :256].T.astype(np.float64), SHIFT,
                        SCALE, emulate_bf16=True)
    assert np.max(np.abs(out - emu)) < 1e-4


def test_training_run_tracks_oracle(sur, torch):
    """Twelve Adam steps over a 4-minibatch data set: the GPU's per-step losses
    follow the oracle's (bf16-emulating) training run."""
    p = W.surrogate_init_params(7)
    sur.set_params(p)
    B, steps = 1024, 12
    x, t = W.surrogate_samples(4 * B, seed=8)
    say("training run 12 steps")
    losses = sur.train(x, t, batch=B, steps=steps, lr=3e-3).cpu().numpy()
    opt = mo.Adam(mo.N_PARAMS, lr=3e-3)
    theta = p.astype(np.float64)
    ref = []
    for k in range(steps):
        sl = slice((k * B) % (4 * B), (k * B) % (4 * B) + B)
        l, g = mo.loss_and_grad(theta, x[:, sl].T.astype(np.float64),
                                t[:, sl].T.astype(np.float64), SHIFT, SCALE, emulate_bf16=True)
        ref.append(l)
        theta = opt.step(theta, mo.flatten(g))
    ref = np.array(ref)
    say("losses gpu  ", np.array2string(losses, precision=5))
    say("losses oracle", np.array2string(ref, precision=5))
    assert np.max(np.abs(losses - ref) / ref) < 2e-3
    assert losses[-1] < losses[0]


def test_weighted_loss_gradient_and_training_match_oracle(torch):
    """The step-doubling form's training loss, e = w out - rho with per-sample
    weights: loss and gradient of one minibatch, then a 12-step training run,
    against the oracle's weighted least squares (bf16-emulating)."""
    from paper_1304_6514_amd.surrogate import Surrogate
    with Surrogate("cuda:0", max_batch=4112, **SD_KW) as s2:
        p = W.surrogate_init_params(3)
        s2.set_params(p)
        n = 4112
        x, t = W.surrogate_samples(n, seed=4)
        wts = np.random.default_rng(41).uniform(-2.0, 2.0, (2, n)).astype(np.float32)
        tg = np.concatenate([t, wts]).astype(np.float32)      # rows rho_0, rho_1, w_0, w_1
        say("weighted loss_grad n=4112")
        loss, g = s2.loss_grad(x, tg)
        p64 = p.astype(np.float64)
        args = (x.T.astype(np.float64), t.T.astype(np.float64), SHIFT, SCALE)
        l_emu, g_emu = mo.loss_and_grad(p64, *args, emulate_bf16=True,
                                        weights=wts.T.astype(np.float64))
        l_ref, g_ref = mo.loss_and_grad(p64, *args, weights=wts.T.astype(np.float64))
        assert abs(loss - l_emu) <= 1e-5 * l_emu, (loss, l_emu)
        assert abs(loss - l_ref) <= 1e-3 * l_ref, (loss, l_ref)
        gu = mo.unflatten(g)
        for name, _ in mo.SHAPES:
            assert _rel(gu[name], g_emu[name]) < 2e-3, name
            assert _rel(gu[name], g_ref[name]) < 3e-2, name

        B, steps = 1024, 12
        p = W.surrogate_init_params(7)
        s2.set_params(p)
        x, t = W.surrogate_samples(4 * B, seed=8)
        wts = np.random.default_rng(42).uniform(0.0, 2.0, (2, 4 * B)).astype(np.float32)
        losses = s2.train(x, np.concatenate([t, wts]), batch=B, steps=steps,
                          lr=3e-3).cpu().numpy()
        opt = mo.Adam(mo.N_PARAMS, lr=3e-3)
        theta = p.astype(np.float64)
        ref = []
        for k in range(steps):
            sl = slice((k * B) % (4 * B), (k * B) % (4 * B) + B)
            l, gk = mo.loss_and_grad(theta, x[:, sl].T.astype(np.float64),
                                     t[:, sl].T.astype(np.float64), SHIFT, SCALE,
                                     emulate_bf16=True, weights=wts[:, sl].T.astype(np.float64))
            ref.append(l)
            theta = opt.step(theta, mo.flatten(gk))
        ref = np.array(ref)
        say("weighted losses gpu   ", np.array2string(losses, precision=5))
        say("weighted losses oracle", np.array2string(ref, precision=5))
        assert np.max(np.abs(losses - ref) / ref) < 2e-3
        assert losses[-1] < losses[0]


def _train_batch(torch):
    from paper_1304_6514_amd.propagator import Batch
    # eight slices of the training build's length 50/1024
    probs = W.surrogate_training_problems(n_slices=8, grid_n=(12, 10), steps=40, seed=9,
                                          T=8 * 50.0 / 1024)
    b = Batch(probs, precision="fp32")
    st, _, _ = b.run()
    assert st == nv.NV_OK
    return probs, b


@pytest.mark.parametrize("coarse", [0, 2])
def test_training_set_gather_is_exact(sur, torch, coarse):
    from paper_1304_6514_amd.surrogate import Surrogate
    probs, b = _train_batch(torch)
    os_ = OUT_SCALE if coarse == 0 else np.array(W.SUR_OUT_SCALE_COARSE)
    s2 = Surrogate("cuda:0", max_batch=1024, out_scale=os_, coarse_steps=coarse)
    try:
        M = 12 * 10
        total = len(probs) * M
        perm = W.surrogate_perm(total, seed=10)
        x, t = s2.dataset_from_batch(b, perm)
        x, t = x.cpu().numpy(), t.cpu().numpy()
        for i, w in enumerate(probs):
            tabs = [nv.nv_batch_get_table(b.batch, i, c, 1, M, "fp32")[0] for c in range(2)]
            k = np.arange(M)
            k0, k1 = k // 10, k % 10
            d0 = (w.grid_hi[0] - w.grid_lo[0]) / 11
            d1 = (w.grid_hi[1] - w.grid_lo[1]) / 9
            y0 = (w.grid_lo[0] + k0 * d0).astype(np.float32)
            y1 = (w.grid_lo[1] + k1 * d1).astype(np.float32)
            pos = perm[i * M + k]
            assert np.array_equal(x[0, pos], y0) and np.array_equal(x[1, pos], y1)
            assert np.all(x[2, pos] == np.float32(w.t0))
            assert np.all(x[3, pos] == np.float32(w.params[0]))
            g = mo.coarse_step(np.stack([y0, y1], -1).astype(np.float64), w.params[0],
                               w.T - w.t0, coarse)
            e0 = ((tabs[0].astype(np.float64) - g[:, 0]) / os_[0]).astype(np.float32)
            e1 = ((tabs[1].astype(np.float64) - g[:, 1]) / os_[1]).astype(np.float32)
            if coarse == 0:
                assert np.array_equal(t[0, pos], e0) and np.array_equal(t[1, pos], e1)
            else:   # the coarse RK4 step: FP64 on both sides, one FP32 rounding at the end
                assert np.max(np.abs(t[0, pos] - e0) / np.maximum(np.abs(e0), 1e-3)) < 1e-6
                assert np.max(np.abs(t[1, pos] - e1) / np.maximum(np.abs(e1), 1e-3)) < 1e-6
        say(f"training-set gather (coarse steps {coarse}): {total} samples checked")
    finally:
        s2.close()
        b.close()


@pytest.mark.parametrize("visits", [False, True])
def test_step_doubling_gather_matches_oracle(torch, visits):
    """The step-doubling training set: inputs bit for bit, the targets rho and
    weights w against the oracle's (FP64 on both sides, one fp32 rounding at
    the end; the visit weight's fp32 exponential may differ in its last bit)."""
    from paper_1304_6514_amd.surrogate import Surrogate
    probs, b = _train_batch(torch)
    s2 = Surrogate("cuda:0", max_batch=1024, **SD_KW)
    try:
        M = 12 * 10
        total = len(probs) * M
        states = None
        if visits:
            rng = np.random.default_rng(61)
            n_mu, n_states = 5, 37
            states = np.stack([np.column_stack([rng.uniform(-2.5, 2.5, n_states),
                                                rng.uniform(-7.0, 7.0, n_states)])
                               for _ in range(n_mu)])
            s2.set_visits(states, 1.0, 5.0, 0.3, 0.02)
        perm = W.surrogate_perm(total, seed=10)
        x, t = s2.dataset_from_batch(b, perm)
        x, t = x.cpu().numpy(), t.cpu().numpy()
        assert t.shape == (4, total)
        worst = 0.0
        for i, w in enumerate(probs):
            tabs = [nv.nv_batch_get_table(b.batch, i, c, 1, M, "fp32")[0] for c in range(2)]
            k = np.arange(M)
            k0, k1 = k // 10, k % 10
            d0 = (w.grid_hi[0] - w.grid_lo[0]) / 11
            d1 = (w.grid_hi[1] - w.grid_lo[1]) / 9
            y0 = (w.grid_lo[0] + k0 * d0).astype(np.float32)
            y1 = (w.grid_lo[1] + k1 * d1).astype(np.float32)
            pos = perm[i * M + k]
            assert np.array_equal(x[0, pos], y0) and np.array_equal(x[1, pos], y1)
            assert np.all(x[2, pos] == np.float32(w.t0))
            assert np.all(x[3, pos] == np.float32(w.params[0]))
            xi = np.stack([y0, y1], -1)
            v = None
            if visits:
                ci = int(np.clip(np.rint((w.params[0] - 1.0) / 1.0), 0, 4))
                v = mo.visit_weight(mo.visit_d2(xi, states[ci], SCALE), 0.3, 0.02)
            rho, wt = mo.step_doubling_targets(
                np.stack([tb.astype(np.float64) for tb in tabs], -1), xi.astype(np.float64),
                w.params[0], w.T - w.t0, 1, W.SUR_SD_GATE, W.SUR_SD_OUT_SCALE,
                W.SUR_SD_LOSS_SCALE, v)
            for row, ref in ((0, rho[:, 0]), (1, rho[:, 1]), (2, wt[:, 0]), (3, wt[:, 1])):
                scale = max(float(np.max(np.abs(ref))), 1e-30)
                err = float(np.max(np.abs(t[row, pos] - ref)) / scale)
                worst = max(worst, err)
                assert err < 1e-6, (i, row, err)
        say(f"step-doubling gather (visits {visits}): {total} samples, worst relative "
            f"difference {worst:.3g}")
    finally:
        s2.close()
        b.close()


def test_step_doubling_chain_matches_oracle(torch):
    from paper_1304_6514_amd.surrogate import Surrogate
    p = W.surrogate_init_params(11)
    with Surrogate("cuda:0", max_batch=1024, **SD_KW) as s2:
        s2.set_params(p)
        rng = np.random.default_rng(12)
        Q, N = 37, 16
        y0 = np.column_stack([rng.uniform(-2, 2, Q), rng.uniform(-4, 4, Q)])
        mu = rng.uniform(1, 5, Q)
        say(f"step-doubling compose Q={Q} N={N}")
        st, final, bnd, info = s2.compose(y0, mu, 0.0, 50.0 * N / 1024, N, want_boundary=True)
        assert st == nv.NV_OK and info.bad_chain == -1
        bnd = bnd.cpu().numpy()
        worst = 0.0
        for q in range(Q):
            ref = mo.surrogate_chain(p.astype(np.float64), SHIFT, SCALE, W.SUR_SD_OUT_SCALE,
                                     y0[q], mu[q], 0.0, 50.0 * N / 1024, N, emulate_bf16=True,
                                     coarse_steps=1, correction="step-doubling",
                                     gate=W.SUR_SD_GATE)
            worst = max(worst, float(np.max(np.abs(bnd[q] - ref))))
        say(f"step-doubling chains: max |gpu - oracle(bf16)| = {worst:.3g}")
        # the network's output enters scaled by d (about 1e-3 at most here) x 0.05
        assert worst < 1e-7


@pytest.mark.parametrize("coarse", [0, 1])
def test_compose_matches_oracle_chain(sur, torch, coarse):
    from paper_1304_6514_amd.surrogate import Surrogate
    p = W.surrogate_init_params(11)
    p[mo.N_PARAMS - 258:] *= 0.2                      # a gentle map: small W4, b4
    os_ = OUT_SCALE if coarse == 0 else np.array(W.SUR_OUT_SCALE_COARSE)
    s2 = sur if coarse == 0 else Surrogate("cuda:0", max_batch=1024, out_scale=os_,
                                           coarse_steps=coarse)
    s2.set_params(p)
    rng = np.random.default_rng(12)
    Q, N = 37, 16
    y0 = np.column_stack([rng.uniform(-2, 2, Q), rng.uniform(-4, 4, Q)])
    mu = rng.uniform(1, 5, Q)
    say(f"surrogate compose Q={Q} N={N} coarse={coarse}")
    st, final, bnd, info = s2.compose(y0, mu, 0.0, 50.0 * N / 1024, N, want_boundary=True)
    assert st == nv.NV_OK and info.bad_chain == -1
    final, bnd = final.cpu().numpy(), bnd.cpu().numpy()
    worst = 0.0
    for q in range(Q):
        ref = mo.surrogate_chain(p.astype(np.float64), SHIFT, SCALE, os_, y0[q], mu[q], 0.0,
                                 50.0 * N / 1024, N, emulate_bf16=True, coarse_steps=coarse)
        worst = max(worst, float(np.max(np.abs(bnd[q] - ref))))
        assert np.array_equal(bnd[q, -1], final[q])
    say(f"chains: max |gpu - oracle(bf16)| over boundary states = {worst:.3g}")
    assert worst < 1e-4
    if s2 is not sur:
        s2.close()


def test_compose_rejects_other_slice_lengths(sur, torch):
    with pytest.raises(nv.NvError) as e:
        sur.compose([[2.0, 0.0]], [3.0], 0.0, 50.0, 100)
    assert e.value.status == nv.NV_ERR_INVALID_ARG


def test_compose_fallback_reproduces_bilinear_composition(sur, torch):
    """With guard < 0 every step takes the table's value: the result is the
    library's bilinear composition over the same table, to the bit."""
    from paper_1304_6514_amd.propagator import Propagator
    w = W.small(W.VDP_FP32, 24, (20, 20), 60).with_(T=24 * W.SUR_SLICE_LENGTH)
    sur.set_params(W.surrogate_init_params(13))
    with Propagator("cuda:0") as prop:
        prop.build(w)
        res = prop.compose()
        y_ref = np.asarray(res.yT)
        Q = 3
        st, final, _, info = sur.compose(np.tile(w.y0, (Q, 1)), np.full(Q, w.params[0]), w.t0,
                                         w.T, w.n_slices, fallback=prop, guard=-1.0)
        assert st == nv.NV_OK
        assert info.n_fallback == Q * w.n_slices
        assert np.array_equal(final.cpu().numpy(), np.tile(y_ref, (Q, 1)))
        # guard = inf: no step falls back inside the box, and the deviation is reported
        st, final2, _, info2 = sur.compose(np.tile(w.y0, (Q, 1)), np.full(Q, w.params[0]),
                                           w.t0, w.T, w.n_slices, fallback=prop,
                                           guard=float("inf"))
        assert info2.max_deviation > 0.0
        say(f"fallback: {info.n_fallback} steps reproduce the bilinear chain; guard=inf: "
            f"{info2.n_fallback} fallbacks, max deviation {info2.max_deviation:.3g}")


def test_trained_network_gains_over_the_method_without_it(torch, orc):
    """The whole learned path at full size, in the step-doubling form: the
    training build (1024 one-slice Van der Pol problems with their own mu,
    128 x 128 grid, 500 RK4 steps: 16.7M endpoints), the visit weights from
    Richardson chains of the untrained form for 81 mu, 20 epochs of Adam, then
    the composition over [0, 50] (1024 slices) for eight held-out mu that no
    table was built for.  Truth: the oracle's serial RK4 run (512,000 steps).
    The trained network's max final-state error must be below each method
    without it: the same form with the network's output zeroed (Richardson
    extrapolation of one RK4 step per slice), the coarse step alone (one RK4
    step per slice), and the plain method with a fresh 128 x 128 table build
    per mu."""
    from paper_1304_6514_amd.propagator import Batch, Propagator
    from paper_1304_6514_amd.surrogate import Surrogate
    B = 65536
    base = W.VDP_FP32
    probs = W.surrogate_training_problems()
    b = Batch(probs)
    st, _, _ = b.run()
    assert st == nv.NV_OK
    sur = Surrogate("cuda:0", max_batch=B, **SD_KW)
    g1 = Surrogate("cuda:0", max_batch=16, coarse_steps=1, out_scale=(1.0, 1.0))
    try:
        # the states the composition visits: the untrained form (zero network:
        # Richardson) from the workload's y0 for a grid of mu
        mug = np.linspace(1.0, 5.0, W.SUR_VISIT_MUS)
        st, _, vis, _ = sur.compose(np.tile(base.y0, (len(mug), 1)), mug, base.t0, base.T,
                                    base.n_slices, want_boundary=True)
        assert st == nv.NV_OK
        sur.set_visits(vis, 1.0, 5.0, W.SUR_VISIT_SIGMA, W.SUR_VISIT_FLOOR)
        total = nv.nv_sur_dataset_from_batch(sur.h, b.batch)
        x, t = sur.dataset_from_batch(b, W.surrogate_perm(total))
        b.close()
        sur.set_params(W.surrogate_init_params(0))
        losses = sur.train(x, t, batch=B, steps=20 * (total // B), lr=2e-3,
                           lr_final=2e-5).cpu().numpy()
        del x, t
        say(f"training: {len(losses)} steps, loss {losses[0]:.3g} -> {losses[-1]:.3g}, "
            f"{sur.last_ms():.0f} ms")

        mus = W.surrogate_eval_mus(8)
        y0 = np.tile(base.y0, (len(mus), 1))
        truth = np.array([orc.serial("vdp", [float(mu)], "rk4", base.t0, base.T, base.n_slices,
                                     base.steps_per_slice, base.y0) for mu in mus])

        def errors(s):
            st, fin, _, _ = s.compose(y0, mus, base.t0, base.T, base.n_slices)
            assert st == nv.NV_OK
            return np.max(np.abs(fin.cpu().numpy() - truth), axis=1)

        e_net = errors(sur)
        trained = sur.params()
        off = trained.copy()
        off[mo.N_PARAMS - 258:] = 0.0                # W4 = 0, b4 = 0: Richardson alone
        sur.set_params(off)
        e_rich = errors(sur)
        e_g1 = errors(g1)                            # untrained additive form: G alone
        plain = []
        with Propagator("cuda:0") as pr:
            for i, mu in enumerate(mus):
                r = pr.solve(base.with_(params=(float(mu),)), want_boundary=False)
                plain.append(float(np.max(np.abs(np.asarray(r.yT) - truth[i]))))
        plain = np.array(plain)
        say("held-out mu          ", np.array2string(mus, precision=3))
        say("network error        ", np.array2string(e_net, precision=3))
        say("Richardson alone     ", np.array2string(e_rich, precision=3))
        say("one RK4 step alone   ", np.array2string(e_g1, precision=3))
        say("plain 128x128 build  ", np.array2string(plain, precision=3))
        assert losses[-1] < 0.1 * losses[0]
        assert np.max(e_net) < np.max(e_rich)
        assert np.max(e_net) < np.max(e_g1)
        assert np.max(e_net) < np.max(plain)
    finally:
        sur.close()
        g1.close()


def test_surrogate_error_paths(sur, torch):
    """Argument checks of the surrogate's entry points on a live object, the
    out-of-box count, and a chain that starts non-finite."""
    sur.set_params(W.surrogate_init_params(21))
    x, t = W.surrogate_samples(64, seed=22)
    with pytest.raises(nv.NvError) as e:
        sur.loss_grad(x[:, :40], t[:, :40])                 # not a multiple of 16
    assert e.value.status == nv.NV_ERR_INVALID_ARG
    with pytest.raises(nv.NvError) as e:
        sur.train(x[:, :48], t[:, :48], batch=32, steps=1)  # 48 not a multiple of 32
    assert e.value.status == nv.NV_ERR_INVALID_ARG
    with pytest.raises(nv.NvError) as e:
        sur.train(x, t, batch=16384, steps=1)               # above max_batch
    assert e.value.status == nv.NV_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        sur.set_params(np.zeros(10, np.float32))
    bad = W.surrogate_init_params(21)
    bad[5] = np.nan
    with pytest.raises(nv.NvError) as e:
        sur.set_params(bad)
    assert e.value.status == nv.NV_ERR_INVALID_ARG
    N = 8
    T = N * W.SUR_SLICE_LENGTH
    # chain 1 starts outside the box: counted once per slice it spends outside
    st, fin, _, info = sur.compose([[0.5, 0.0], [2.0, 30.0], [0.0, 1.0]], [2.0, 2.0, 2.0], 0.0, T,
                                   N)
    assert st == nv.NV_OK and info.n_outside >= 1 and info.bad_chain == -1
    # chain 2 starts at NaN: reported, the others still complete
    st, fin, _, info = sur.compose([[0.5, 0.0], [1.0, 0.0], [np.nan, 0.0]], [2.0, 2.0, 2.0], 0.0,
                                   T, N)
    assert st == nv.NV_ERR_NONFINITE and info.bad_chain == 2
    f = fin.cpu().numpy()
    assert np.all(np.isfinite(f[:2])) and not np.all(np.isfinite(f[2]))


def test_gather_rejects_foreign_problems_and_bad_permutations(sur, torch):
    from paper_1304_6514_amd.propagator import Batch
    b = Batch([W.small(W.LOGISTIC_FP64, 4, (64,), 50)])
    try:
        assert b.run()[0] == nv.NV_OK
        with pytest.raises(nv.NvError) as e:
            nv.nv_sur_dataset_from_batch(sur.h, b.batch)
        assert e.value.status == nv.NV_ERR_INVALID_ARG
    finally:
        b.close()
    probs, b = _train_batch(torch)
    try:
        total = len(probs) * 120
        perm = np.arange(total, dtype=np.int64)
        perm[7] = total + 5                                     # outside [0, cap)
        with pytest.raises(nv.NvError) as e:
            sur.dataset_from_batch(b, perm)
        assert e.value.status == nv.NV_ERR_INVALID_ARG
    finally:
        b.close()
