"""Plain FP64 oracle of the learned slice-map surrogate.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  It shares no code
with the GPU library.

The surrogate replaces the table lookup of the sequential pass (sec. 3: the
composition lambda_{j+1} = phi^j(lambda_j)) by a small network that learns the
slice map from the endpoints the computation phase tabulates.  The network is a
multilayer perceptron

    u   = (x - shift) * scale                x = (y1, y2, slice start time, mu)
    a1  = gelu(W1 u  + b1)                   W1: 128 x 4
    a2  = gelu(W2 a1 + b2)                   W2: 128 x 128
    a3  = gelu(W3 a2 + b3)                   W3: 128 x 128
    out = W4 a3 + b4                         W4: 2 x 128

with the exact GELU, gelu(z) = z Phi(z), Phi the standard normal distribution
function.  Its output corrects a coarse propagator: additively,
phi^j(y) ~ G(y) + out_scale * out, G the identity or a few RK4 steps over the
slice (``coarse_step``); or in the step-doubling form, phi^j(y) ~ G1 +
d (16/15 + out_scale g out) with d the difference of one coarse step to two of
half the length and g a gate in d (``step_doubling_map``; with out = 0 this is
Richardson extrapolation of the coarse step).  The training loss is the mean
over samples of the squared error summed over the two outputs (weighted per
sample in the step-doubling form); the optimiser is Adam (Kingma and Ba,
"Adam: a method for stochastic optimization", Algorithm 1).

Flat parameter order: W1 (row-major, out x in), b1, W2, b2, W3, b3, W4, b4;
33,922 numbers.

``emulate_bf16=True`` rounds to bfloat16 at the points where the GPU kernels
feed their matrix cores (inputs of the two 128 x 128 layers, their weights, the
back-propagated errors and the operands of every weight-gradient sum), so that
both sides take the same roundings; everything else stays FP64.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

IN, WIDTH, OUT = 4, 128, 2
SHAPES = (("W1", (WIDTH, IN)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (OUT, WIDTH)), ("b4", (OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(flat):
    """Flat parameter vector -> dict of FP64 arrays (copies)."""
    flat = np.asarray(flat, dtype=np.float64)
    if flat.size != N_PARAMS:
        raise ValueError(f"expected {N_PARAMS} parameters, got {flat.size}")
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[off:off + n].reshape(shape).copy()
        off += n
    return out


def flatten(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), through binary32 first, as a
    float-to-bfloat16 conversion of a binary32 value does.  Returns FP64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(f)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, out)


def gelu(z):
    """gelu(z) = z Phi(z), Phi(z) = (1 + erf(z / sqrt 2)) / 2."""
    return z * 0.5 * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    """d/dz gelu = Phi(z) + z phi(z), phi the standard normal density."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def normalise(x, shift, scale):
    """x: (n, 4) raw inputs -> u = (x - shift) * scale."""
    return (np.asarray(x, np.float64) - np.asarray(shift, np.float64)) * np.asarray(scale, np.float64)


def forward(params, x, shift, scale, emulate_bf16=False):
    """Network output (n, 2) and the intermediate values of the pass."""
    p = params if isinstance(params, dict) else unflatten(params)
    r = bf16 if emulate_bf16 else (lambda v: v)
    u = normalise(x, shift, scale)
    z1 = u @ p["W1"].T + p["b1"]
    a1 = gelu(z1)
    h1 = r(a1)
    z2 = h1 @ r(p["W2"]).T + p["b2"]
    a2 = gelu(z2)
    h2 = r(a2)
    z3 = h2 @ r(p["W3"]).T + p["b3"]
    a3 = gelu(z3)
    out = a3 @ p["W4"].T + p["b4"]
    cache = dict(u=u, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, a3=a3, out=out)
    return out, cache


def loss_and_grad(params, x, target, shift, scale, emulate_bf16=False, weights=None):
    """Loss = mean over the n samples of sum_c e_c^2, e_c = out_c - target_c, or
    with per-sample weights w (n, 2) the weighted least-squares error
    e_c = w_c out_c - target_c; and its gradient by the chain rule, layer by
    layer from the output back."""
    p = params if isinstance(params, dict) else unflatten(params)
    r = bf16 if emulate_bf16 else (lambda v: v)
    out, c = forward(p, x, shift, scale, emulate_bf16)
    n = out.shape[0]
    w = np.ones_like(out) if weights is None else np.asarray(weights, np.float64)
    err = w * out - np.asarray(target, np.float64)
    loss = float(np.sum(err * err) / n)
    dout = 2.0 * err * w / n                               # dL/d out
    g = {}
    dq = r(dout)
    g["W4"] = dq.T @ r(c["a3"])
    g["b4"] = dq.sum(axis=0)
    d3 = (dout @ p["W4"]) * gelu_prime(c["z3"])            # dL/d z3
    d3q = r(d3)
    g["W3"] = d3q.T @ c["h2"]
    g["b3"] = d3q.sum(axis=0)
    d2 = (d3q @ r(p["W3"])) * gelu_prime(c["z2"])
    d2q = r(d2)
    g["W2"] = d2q.T @ c["h1"]
    g["b2"] = d2q.sum(axis=0)
    d1 = (d2q @ r(p["W2"])) * gelu_prime(c["z1"])
    d1q = r(d1)
    g["W1"] = d1q.T @ r(c["u"])
    g["b1"] = d1q.sum(axis=0)
    return loss, g


class Adam:
    """Adam with bias correction (Kingma and Ba, Algorithm 1), FP64 state."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0

    def step(self, theta, grad):
        """Return the updated parameters (theta is not modified)."""
        self.t += 1
        g = np.asarray(grad, np.float64)
        self.m = self.beta1 * self.m + (1.0 - self.beta1) * g
        self.v = self.beta2 * self.v + (1.0 - self.beta2) * g * g
        m_hat = self.m / (1.0 - self.beta1 ** self.t)
        v_hat = self.v / (1.0 - self.beta2 ** self.t)
        return np.asarray(theta, np.float64) - self.lr * m_hat / (np.sqrt(v_hat) + self.eps)


def coarse_step(y, mu, L, k):
    """The coarse propagator G over a slice of length L: k classical RK4 steps
    of h = L / k of the Van der Pol field y1' = y2, y2' = mu (1 - y1^2) y2 - y1
    (k = 0: the identity).  y: (..., 2)."""
    y = np.array(y, dtype=np.float64)
    if k == 0:
        return y

    def f(v):
        return np.stack([v[..., 1], mu * (1.0 - v[..., 0] ** 2) * v[..., 1] - v[..., 0]], -1)

    h = L / k
    for _ in range(k):
        k1 = f(y)
        k2 = f(y + 0.5 * h * k1)
        k3 = f(y + 0.5 * h * k2)
        k4 = f(y + h * k3)
        y = y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return y


# Richardson's constant of a fourth-order step: G1's error is about 16/15 of
# the step-doubling difference G2 - G1.
RICHARDSON = 16.0 / 15.0


def step_doubling(y, mu, L, k, gate):
    """The step-doubling form's pieces at y (..., 2): G1 = k RK4 steps of L / k,
    d = G2 - G1 with G2 = 2k RK4 steps of L / (2k), and the gate
    g_c = d_c^2 / (d_c^2 + gate_c^2).  Returns (G1, d, g)."""
    g1 = coarse_step(y, mu, L, k)
    g2 = coarse_step(y, mu, L, 2 * k)
    d = g2 - g1
    tau2 = np.asarray(gate, np.float64) ** 2
    dd = d * d
    return g1, d, dd / (dd + tau2)


def step_doubling_map(y, out, mu, L, k, gate, out_scale):
    """phi(y)_c ~ G1_c + d_c (16/15 + (out_scale_c g_c) out_c)."""
    g1, d, g = step_doubling(y, mu, L, k, gate)
    return g1 + d * (RICHARDSON + (np.asarray(out_scale, np.float64) * g) * out)


def visit_d2(xi, states, in_scale):
    """Squared distance, in the network's input units, from points xi (n, 2) to
    the nearest of a chain's states (m, 2); fp32, one rounding per operation."""
    xi = np.asarray(xi, np.float32)
    st = np.asarray(states, np.float64).astype(np.float32)
    sc = np.asarray(in_scale, np.float32)[:2]
    best = np.full(xi.shape[0], np.inf, np.float32)
    for s in st:
        e0 = (xi[:, 0] - s[0]) * sc[0]
        e1 = (xi[:, 1] - s[1]) * sc[1]
        best = np.minimum(best, e0 * e0 + e1 * e1)
    return best


def visit_weight(d2, sigma, floor_weight):
    """v = exp(-D^2 / (2 sigma^2)) + floor, in fp32."""
    inv = np.float32(1.0 / (2.0 * sigma * sigma))
    return np.exp(-(np.asarray(d2, np.float32) * inv)) + np.float32(floor_weight)


def step_doubling_targets(tab, xi, mu, L, k, gate, out_scale, loss_scale, v=None):
    """Training targets of the step-doubling form for endpoints tab (n, 2) of
    the slice map from xi (n, 2): rho_c = sqrt(v) r_c / q_c with
    r = (tab - G1) - 16/15 d, and w_c = sqrt(v) (d_c out_scale_c) g_c / q_c,
    q = loss_scale, so that w out - rho is sqrt(v) times the surrogate map's
    error in units of q.  Returns (rho, w), (n, 2) each, FP64."""
    g1, d, g = step_doubling(np.asarray(xi, np.float64), mu, L, k, gate)
    sv = np.ones((d.shape[0], 1)) if v is None else \
        np.sqrt(np.asarray(v, np.float64))[:, None]
    q = np.asarray(loss_scale, np.float64)
    r = (np.asarray(tab, np.float64) - g1) - RICHARDSON * d
    return (sv * r) / q, (sv * ((d * np.asarray(out_scale, np.float64)) * g)) / q


def surrogate_chain(params, shift, scale, out_scale, y0, mu, t0, T, n_slices,
                    emulate_bf16=False, coarse_steps=0, correction="additive",
                    gate=(1.0, 1.0)):
    """The sequential pass with the network in place of the lookup:
    lambda_0 = y0, lambda_{j+1} = the surrogate map at (lambda_j, T_j, mu),
    T_j = t0 + j (T - t0) / n_slices: G(lambda_j) + out_scale * net (additive,
    G the coarse propagator of coarse_step) or step_doubling_map.
    Returns lambda_0 .. lambda_N, (N+1, 2)."""
    L = (T - t0) / n_slices
    lam = np.array(y0, np.float64)
    bnd = [lam.copy()]
    for j in range(n_slices):
        x = np.array([[lam[0], lam[1], t0 + j * L, mu]])
        out, _ = forward(params, x, shift, scale, emulate_bf16)
        if correction == "step-doubling":
            lam = step_doubling_map(lam, out[0], mu, L, coarse_steps, gate, out_scale)
        else:
            lam = coarse_step(lam, mu, L, coarse_steps) + \
                np.asarray(out_scale, np.float64) * out[0]
        bnd.append(lam.copy())
    return np.array(bnd)
