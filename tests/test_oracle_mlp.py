"""Pins of the surrogate network's FP64 oracle against facts fixed outside it:
textbook values of the normal distribution, finite differences, torch's own
GELU/linear/Adam implementations, and affine special cases."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp_oracle as mo


def _params(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, mo.N_PARAMS)


SHIFT = np.array([0.0, 0.0, 25.0, 3.0])
SCALE = np.array([1 / 3, 1 / 8, 1 / 25, 1 / 2])


def _inputs(seed, n):
    rng = np.random.default_rng(seed)
    x = np.column_stack([rng.uniform(-3, 3, n), rng.uniform(-8, 8, n), rng.uniform(0, 50, n),
                         rng.uniform(1, 5, n)])
    t = rng.normal(0.0, 1.0, (n, 2))
    return x, t


def test_param_count_matches_architecture():
    # 4->128, 128->128, 128->128, 128->2 with biases
    assert mo.N_PARAMS == (4 * 128 + 128) + 2 * (128 * 128 + 128) + (128 * 2 + 2) == 33922
    p = _params(0)
    assert np.array_equal(mo.flatten(mo.unflatten(p)), p)


def test_bf16_rounding_ties_and_library():
    one = 1.0
    # spacing of bfloat16 near 1 is 2^-7: halfway points round to the even neighbour
    assert mo.bf16(one + 2.0 ** -8) == 1.0
    assert mo.bf16(one + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert mo.bf16(one + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert mo.bf16(-2.5) == -2.5
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.normal(0, 1, 20000), rng.normal(0, 1e-6, 2000),
                        rng.normal(0, 1e6, 2000)]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mo.bf16(v), ref)


def test_gelu_textbook_values():
    # Phi(1) and Phi(-1) of the standard normal distribution
    assert mo.gelu(np.array(1.0)) == pytest.approx(0.8413447460685429, rel=1e-15)
    assert mo.gelu(np.array(-1.0)) == pytest.approx(-0.15865525393145707, rel=1e-14)
    assert mo.gelu(np.array(0.0)) == 0.0
    assert mo.gelu(np.array(12.0)) == 12.0
    assert mo.gelu_prime(np.array(0.0)) == 0.5
    z = np.linspace(-6, 6, 97)
    h = 1e-5
    fd = (mo.gelu(z + h) - mo.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mo.gelu_prime(z))) < 1e-9
    tz = torch.from_numpy(z)
    assert np.allclose(mo.gelu(z), torch.nn.functional.gelu(tz, approximate="none").numpy(),
                       rtol=0, atol=1e-15)


def test_forward_matches_torch_layers():
    p = mo.unflatten(_params(2))
    x, _ = _inputs(3, 33)
    out, _ = mo.forward(p, x, SHIFT, SCALE)
    T = lambda a: torch.from_numpy(np.asarray(a, np.float64))
    F = torch.nn.functional
    u = (T(x) - T(SHIFT)) * T(SCALE)
    a = F.gelu(F.linear(u, T(p["W1"]), T(p["b1"])))
    a = F.gelu(F.linear(a, T(p["W2"]), T(p["b2"])))
    a = F.gelu(F.linear(a, T(p["W3"]), T(p["b3"])))
    ref = F.linear(a, T(p["W4"]), T(p["b4"])).numpy()
    assert np.max(np.abs(out - ref)) < 1e-13


def test_gradient_matches_central_differences():
    flat = _params(4)
    x, t = _inputs(5, 9)
    loss, g = mo.loss_and_grad(flat, x, t, SHIFT, SCALE)
    gf = mo.flatten(g)
    rng = np.random.default_rng(6)
    # a few coordinates of every tensor, including both ends of each
    idx, off = [], 0
    for _, shape in mo.SHAPES:
        n = int(np.prod(shape))
        idx += [off, off + n - 1] + list(off + rng.integers(0, n, 4))
        off += n
    h = 1e-6
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = h
        lp, _ = mo.loss_and_grad(flat + e, x, t, SHIFT, SCALE)
        lm, _ = mo.loss_and_grad(flat - e, x, t, SHIFT, SCALE)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gf[i]) <= 1e-7 * max(1.0, abs(gf[i])), (i, fd, gf[i])
    assert loss > 0


def test_gradient_matches_torch_autograd():
    flat = _params(7)
    x, t = _inputs(8, 50)
    loss, g = mo.loss_and_grad(flat, x, t, SHIFT, SCALE)
    p = {k: torch.tensor(v, requires_grad=True) for k, v in mo.unflatten(flat).items()}
    F = torch.nn.functional
    u = (torch.from_numpy(x) - torch.from_numpy(SHIFT)) * torch.from_numpy(SCALE)
    a = F.gelu(u @ p["W1"].T + p["b1"])
    a = F.gelu(a @ p["W2"].T + p["b2"])
    a = F.gelu(a @ p["W3"].T + p["b3"])
    out = a @ p["W4"].T + p["b4"]
    L = ((out - torch.from_numpy(t)) ** 2).sum(dim=1).mean()
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    for k in p:
        assert np.max(np.abs(p[k].grad.numpy() - g[k])) < 1e-12 * max(1.0, np.abs(g[k]).max())


def test_emulated_gradient_close_to_exact():
    flat = _params(9)
    x, t = _inputs(10, 256)
    _, g = mo.loss_and_grad(flat, x, t, SHIFT, SCALE)
    _, ge = mo.loss_and_grad(flat, x, t, SHIFT, SCALE, emulate_bf16=True)
    for k in g:
        rel = np.linalg.norm(ge[k] - g[k]) / np.linalg.norm(g[k])
        assert 0 < rel < 3e-2, (k, rel)


def test_adam_matches_torch_and_first_step_sign():
    rng = np.random.default_rng(11)
    theta0 = rng.normal(0, 1, 40)
    grads = [rng.normal(0, 1, 40) for _ in range(6)]
    opt = mo.Adam(40, lr=3e-3, beta1=0.9, beta2=0.99, eps=1e-8)
    th = torch.tensor(theta0, requires_grad=True)
    topt = torch.optim.Adam([th], lr=3e-3, betas=(0.9, 0.99), eps=1e-8)
    theta = theta0.copy()
    for k, gk in enumerate(grads):
        new = opt.step(theta, gk)
        if k == 0:
            # first step: m_hat / sqrt(v_hat) = g / |g|, a step of lr against the sign
            assert np.allclose(new - theta, -3e-3 * np.sign(gk), rtol=1e-6, atol=0)
        theta = new
        th.grad = torch.from_numpy(gk.copy())
        topt.step()
    assert np.max(np.abs(theta - th.detach().numpy())) < 1e-14


def _affine_params(seed):
    """A network whose every hidden pre-activation exceeds 10, where
    gelu(z) = z to FP64 precision, so the network is an affine map."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.uniform(-0.1, 0.1, (128, 4)), "b1": np.full(128, 20.0),
         "W2": rng.uniform(-0.02, 0.02, (128, 128)), "b2": np.full(128, 60.0),
         "W3": rng.uniform(-0.02, 0.02, (128, 128)), "b3": np.full(128, 100.0),
         "W4": rng.uniform(-0.01, 0.01, (2, 128)), "b4": rng.uniform(-0.1, 0.1, 2)}
    A = p["W4"] @ p["W3"] @ p["W2"] @ p["W1"]
    c = p["W4"] @ (p["W3"] @ (p["W2"] @ p["b1"] + p["b2"]) + p["b3"]) + p["b4"]
    return p, A, c


def test_chain_of_affine_network_is_linear_recurrence():
    p, A, c = _affine_params(12)
    x, _ = _inputs(13, 20)
    _, cache = mo.forward(p, x, SHIFT, SCALE)
    assert min(cache["z1"].min(), cache["z2"].min(), cache["z3"].min()) > 10
    out_scale = np.array([0.05, 0.2])
    y0, mu, t0, T, N = np.array([2.0, 0.0]), 2.7, 0.0, 5.0, 40
    bnd = mo.surrogate_chain(p, SHIFT, SCALE, out_scale, y0, mu, t0, T, N)
    # out = A u + c with u = (x - shift) * scale: write the recurrence in matrix form
    As = A * SCALE[None, :]
    M = np.eye(2) + out_scale[:, None] * As[:, :2]
    lam = y0.copy()
    for j in range(N):
        tj = t0 + j * (T - t0) / N
        drive = As[:, 2] * tj + As[:, 3] * mu - As @ SHIFT + c
        lam = M @ lam + out_scale * drive
    assert np.max(np.abs(bnd[-1] - lam)) < 1e-11
    assert bnd.shape == (N + 1, 2) and np.array_equal(bnd[0], y0)


def test_chain_zero_network_keeps_state_and_constant_network_drifts():
    p = mo.unflatten(_params(14))
    p["W4"][:] = 0.0
    p["b4"][:] = 0.0
    bnd = mo.surrogate_chain(p, SHIFT, SCALE, np.array([1.0, 1.0]), [0.5, -1.0], 3.0, 0, 10, 16)
    assert np.all(bnd == np.array([0.5, -1.0]))
    p["b4"][:] = [0.25, -0.5]
    bnd = mo.surrogate_chain(p, SHIFT, SCALE, np.array([0.5, 2.0]), [0.5, -1.0], 3.0, 0, 10, 16)
    assert np.allclose(bnd[-1], [0.5 + 16 * 0.125, -1.0 - 16 * 1.0], rtol=0, atol=1e-13)


def test_coarse_step_is_the_rk4_of_the_library_oracle(orc):
    """G of the surrogate is classical RK4 of the Van der Pol field: the same
    steps as the C oracle's integrator (written separately)."""
    rng = np.random.default_rng(15)
    for _ in range(5):
        y, mu, k = rng.uniform(-3, 3, 2), rng.uniform(1, 5), int(rng.integers(1, 4))
        L = 50.0 / 1024
        ref = orc.integrate("vdp", [mu], "rk4", 0.0, L / k, k, y)
        assert np.max(np.abs(mo.coarse_step(y, mu, L, k) - ref)) < 1e-15
    assert np.array_equal(mo.coarse_step([0.3, -1.0], 2.0, 0.1, 0), [0.3, -1.0])


# ---- the step-doubling form ------------------------------------------------

def test_weighted_gradient_matches_torch_autograd_and_differences():
    """e_c = w_c out_c - target_c: the weighted least-squares loss's gradient
    against torch autograd and, for a few parameters, central differences."""
    flat = _params(31)
    x, t = _inputs(32, 40)
    w = np.random.default_rng(33).uniform(-2.0, 2.0, (40, 2))
    loss, g = mo.loss_and_grad(flat, x, t, SHIFT, SCALE, weights=w)
    p = {k: torch.tensor(v, requires_grad=True) for k, v in mo.unflatten(flat).items()}
    F = torch.nn.functional
    u = (torch.from_numpy(x) - torch.from_numpy(SHIFT)) * torch.from_numpy(SCALE)
    a = F.gelu(u @ p["W1"].T + p["b1"])
    a = F.gelu(a @ p["W2"].T + p["b2"])
    a = F.gelu(a @ p["W3"].T + p["b3"])
    out = a @ p["W4"].T + p["b4"]
    L = ((torch.from_numpy(w) * out - torch.from_numpy(t)) ** 2).sum(dim=1).mean()
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    for k in p:
        assert np.max(np.abs(p[k].grad.numpy() - g[k])) < 1e-12 * max(1.0, np.abs(g[k]).max())
    gf = mo.flatten(g)
    h = 1e-6
    for i in (3, 600, 17000, 33921):
        e = np.zeros(mo.N_PARAMS)
        e[i] = h
        lp, _ = mo.loss_and_grad(flat + e, x, t, SHIFT, SCALE, weights=w)
        lm, _ = mo.loss_and_grad(flat - e, x, t, SHIFT, SCALE, weights=w)
        assert abs((lp - lm) / (2 * h) - gf[i]) <= 1e-7 * max(1.0, abs(gf[i]))
    # unit weights are the plain loss
    l1, g1 = mo.loss_and_grad(flat, x, t, SHIFT, SCALE, weights=np.ones((40, 2)))
    l0, g0 = mo.loss_and_grad(flat, x, t, SHIFT, SCALE)
    assert l1 == l0 and all(np.array_equal(g1[k], g0[k]) for k in g0)


def _vdp_flow(y, mu, L):
    """The Van der Pol slice map from a library integrator (DOP853, tight tolerances)."""
    from scipy.integrate import solve_ivp
    r = solve_ivp(lambda t, v: [v[1], mu * (1 - v[0] ** 2) * v[1] - v[0]], (0.0, L), y,
                  method="DOP853", rtol=1e-13, atol=1e-14)
    return r.y[:, -1]


def test_richardson_map_is_fifth_order_and_step_doubling_difference_estimates_the_error():
    """With out = 0 the step-doubling map is Richardson extrapolation of RK4:
    its one-slice error falls by about 2^6 when L halves (RK4's by 2^5), and
    16/15 (G2 - G1) estimates G1's error to leading order."""
    y, mu = np.array([1.2, -0.7]), 2.5
    errs_r, errs_1 = [], []
    for L in (0.2, 0.1, 0.05):
        phi = _vdp_flow(y, mu, L)
        g1, d, _ = mo.step_doubling(y, mu, L, 1, (1.0, 1.0))
        rich = mo.step_doubling_map(y, np.zeros(2), mu, L, 1, (1.0, 1.0), (1.0, 1.0))
        errs_r.append(np.max(np.abs(rich - phi)))
        errs_1.append(np.max(np.abs(g1 - phi)))
        # the leading term of G1's error is 16/15 d
        assert np.max(np.abs((phi - g1) - mo.RICHARDSON * d)) < 0.2 * np.max(np.abs(phi - g1))
    r_rich = [errs_r[i] / errs_r[i + 1] for i in range(2)]
    r_one = [errs_1[i] / errs_1[i + 1] for i in range(2)]
    assert all(40.0 < r < 90.0 for r in r_rich), r_rich
    assert all(24.0 < r < 40.0 for r in r_one), r_one
    # the same extrapolation written the other way round: G2 + (G2 - G1)/15
    g1 = mo.coarse_step(y, mu, 0.1, 1)
    g2 = mo.coarse_step(y, mu, 0.1, 2)
    rich = mo.step_doubling_map(y, np.zeros(2), mu, 0.1, 1, (1.0, 1.0), (1.0, 1.0))
    assert np.max(np.abs(rich - (g2 + (g2 - g1) / 15.0))) < 1e-15


def test_gate_values_and_network_scaling():
    """g = d^2 / (d^2 + gate^2): 0 at d = 0, 1/2 at |d| = gate, 4/5 at 2 gate;
    the network's output enters as d * out_scale * g * out."""
    y, mu, L = np.array([0.4, 1.5]), 3.0, 50.0 / 1024
    g1, d, _ = mo.step_doubling(y, mu, L, 1, (1.0, 1.0))
    for k in (1.0, 2.0, 0.5):
        gate = np.abs(d) / k
        _, _, g = mo.step_doubling(y, mu, L, 1, gate)
        assert np.allclose(g, k * k / (k * k + 1.0), rtol=1e-14)
    out = np.array([0.3, -0.7])
    os_ = np.array([0.05, 0.1])
    gate = np.abs(d)
    m = mo.step_doubling_map(y, out, mu, L, 1, gate, os_)
    m0 = mo.step_doubling_map(y, np.zeros(2), mu, L, 1, gate, os_)
    # (the difference of two states near 1 resolves to about 1e-16)
    assert np.allclose(m - m0, d * os_ * 0.5 * out, rtol=1e-6, atol=4e-16)
    assert np.all(np.abs(d * os_ * 0.5 * out) > 1e-12)


def test_step_doubling_targets_make_the_weighted_error_the_map_error():
    """w out - rho = sqrt(v) (surrogate map - endpoint) / loss_scale for any out."""
    rng = np.random.default_rng(41)
    n = 200
    xi = np.column_stack([rng.uniform(-3, 3, n), rng.uniform(-8, 8, n)])
    mu, L = 2.2, 50.0 / 1024
    tab = np.array([_vdp_flow(p, mu, L) for p in xi[:20]])
    xi = xi[:20]
    gate, os_, q = (1e-4, 3e-3), (0.05, 0.05), (2e-5, 7e-4)
    v = rng.uniform(0.02, 1.02, 20)
    rho, w = mo.step_doubling_targets(tab, xi, mu, L, 1, gate, os_, q, v)
    out = rng.normal(0, 1, (20, 2))
    surrogate = np.array([mo.step_doubling_map(xi[i], out[i], mu, L, 1, gate, os_)
                          for i in range(20)])
    want = np.sqrt(v)[:, None] * (surrogate - tab) / np.array(q)
    assert np.allclose(w * out - rho, want, rtol=1e-7, atol=1e-9)


def test_visit_distance_is_the_nearest_neighbour_distance():
    """D^2 against scipy's k-d tree on the scaled coordinates, and the weight's
    value at D = 0, D = sigma."""
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(51)
    states = np.column_stack([rng.uniform(-2.5, 2.5, 300), rng.uniform(-7, 7, 300)])
    xi = np.column_stack([rng.uniform(-3, 3, 500), rng.uniform(-8, 8, 500)]).astype(np.float32)
    sc = np.array([1 / 3, 1 / 8, 1 / 25, 1 / 2], dtype=np.float32)
    d2 = mo.visit_d2(xi, states, sc)
    tree = cKDTree(states * sc[:2].astype(np.float64))
    ref = tree.query(xi.astype(np.float64) * sc[:2].astype(np.float64))[0] ** 2
    assert np.allclose(d2, ref, rtol=2e-6, atol=1e-7)
    v = mo.visit_weight(np.array([0.0, 0.05 ** 2], np.float32), 0.05, 0.02)
    assert np.allclose(v, [1.02, math.exp(-0.5) + 0.02], rtol=1e-6)
