"""Seeded synthetic workloads shaped like the paper's problems.

This module holds problem descriptions and seeded draws only: no step of the
method's arithmetic.  Both the GPU library and the CPU oracle are fed from it.

A workload names a right-hand side, the time interval [t0, T], the number of
slices N (sec. 3: slice j covers [T_j, T_{j+1}], T_j = t0 + j (T - t0)/N), a
uniform grid of the initial value space (endpoints included), the RK4 steps
per slice, the true initial value y0, the working precision of the table build
and the interpolation rule of the composition.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

RHS_DIM = {"linear": 1, "logistic": 1, "forced_cubic": 1, "vdp": 2, "square": 1}


@dataclass(frozen=True)
class Workload:
    name: str
    rhs: str
    params: tuple
    t0: float
    T: float
    n_slices: int
    grid_n: tuple
    grid_lo: tuple
    grid_hi: tuple
    steps_per_slice: int
    y0: tuple
    precision: str          # "fp64" or "fp32" (the table build's arithmetic)
    interp: str             # "linear", "hermite", "hermite_slopes", "bilinear" or "chebyshev"
    scheme: str = "rk4"     # "rk4", "euler" or "be" (backward Euler)
    dt: float = 0.0         # > 0: fixed step dt per slice (plus a shorter last step)

    @property
    def dim(self) -> int:
        return RHS_DIM[self.rhs]

    @property
    def points_per_slice(self) -> int:
        return int(np.prod(self.grid_n))

    @property
    def trajectories(self) -> int:
        return self.n_slices * self.points_per_slice

    @property
    def trajectory_steps(self) -> int:
        return self.trajectories * self.steps_per_slice

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def vdp_mu(seed: int = 0) -> float:
    """Van der Pol damping mu ~ U[1, 5] from a seed."""
    return float(np.random.default_rng(seed).uniform(1.0, 5.0))


# Plain method in FP64: logistic y'=y(1-y), t in [0,10], y0 = 0.1; 64 slices,
# 256 uniform points on [-0.1, 1.2], 1000 RK4 steps per slice, linear lookup.
LOGISTIC_FP64 = Workload(
    name="logistic-fp64-64sl-256pt-1000st", rhs="logistic", params=(), t0=0.0, T=10.0,
    n_slices=64, grid_n=(256,), grid_lo=(-0.1,), grid_hi=(1.2,), steps_per_slice=1000,
    y0=(0.1,), precision="fp64", interp="linear")

# Forced scalar ODE y'=sin(3t)-y^3, t in [0,100], y0 = 1; 4096 slices, 4096
# points on [-3, 3], 2000 RK4 steps per slice; FP32 build, FP64 Hermite compose.
FORCED_CUBIC_FP32 = Workload(
    name="forced-cubic-fp32-4096sl-4096pt-2000st", rhs="forced_cubic", params=(),
    t0=0.0, T=100.0, n_slices=4096, grid_n=(4096,), grid_lo=(-3.0,), grid_hi=(3.0,),
    steps_per_slice=2000, y0=(1.0,), precision="fp32", interp="hermite")

# Van der Pol, mu ~ U[1,5] (seed 0), t in [0,50], y0 = (2, 0); 1024 slices,
# 128 x 128 tensor grid, 500 RK4 steps per slice; FP32 build, FP64 bilinear
# compose.  The y2 axis spans [-8, 8] so that the limit cycle of every mu in
# [1, 5] lies inside the grid; the [-3, 3]^2 box is kept as VDP_SQUARE_BOX.
VDP_FP32 = Workload(
    name="vdp-fp32-1024sl-128x128pt-500st", rhs="vdp", params=(vdp_mu(0),), t0=0.0,
    T=50.0, n_slices=1024, grid_n=(128, 128), grid_lo=(-3.0, -8.0), grid_hi=(3.0, 8.0),
    steps_per_slice=500, y0=(2.0, 0.0), precision="fp32", interp="bilinear")

VDP_SQUARE_BOX = VDP_FP32.with_(name="vdp-fp32-1024sl-128x128pt-500st-box3",
                                grid_lo=(-3.0, -3.0), grid_hi=(3.0, 3.0))

# Harmonic oscillator (Van der Pol with mu = 0): the slice map is linear, so
# bilinear lookup reproduces it up to rounding.
HARMONIC = VDP_FP32.with_(name="harmonic-1024sl-128x128pt-500st", params=(0.0,),
                          grid_lo=(-3.0, -3.0), grid_hi=(3.0, 3.0))

# The model problem of sec. 3: y' = y^2, y(0) = 1 on [0, 1/2].
SQUARE_MODEL = Workload(
    name="square-fp64-4sl-64pt-1250st", rhs="square", params=(), t0=0.0, T=0.5,
    n_slices=4, grid_n=(64,), grid_lo=(0.0,), grid_hi=(2.0,), steps_per_slice=1250,
    y0=(1.0,), precision="fp64", interp="hermite")

FULL_SIZE = {w.name: w for w in (LOGISTIC_FP64, FORCED_CUBIC_FP32, VDP_FP32)}


def small(w: Workload, n_slices: int, grid_n: tuple, steps: int, **kw) -> Workload:
    """A reduced copy of a workload (same problem, interval and grid box)."""
    return w.with_(name=f"{w.name}-small-{n_slices}x{'x'.join(map(str, grid_n))}x{steps}",
                   n_slices=n_slices, grid_n=tuple(grid_n), steps_per_slice=steps, **kw)


def sample_entries(w: Workload, count: int, seed: int):
    """Seeded (slice, point) pairs covering the first/last slice and grid edges."""
    rng = np.random.default_rng(seed)
    sl = rng.integers(0, w.n_slices, size=count, dtype=np.int64)
    pt = rng.integers(0, w.points_per_slice, size=count, dtype=np.int64)
    edge_s = np.array([0, 0, w.n_slices - 1, w.n_slices - 1], dtype=np.int64)
    edge_p = np.array([0, w.points_per_slice - 1, 0, w.points_per_slice - 1],
                      dtype=np.int64)
    return np.concatenate([edge_s, sl]), np.concatenate([edge_p, pt])


def _log_uniform_int(rng, lo, hi):
    return int(round(float(np.exp(rng.uniform(np.log(lo), np.log(hi))))))


def batched_problems(count: int = 96, seed: int = 3, scale: float = 1.0):
    """The batched uneven workload: count seeded problems mixing y' = lambda y
    (lambda ~ U[-2, 0.5], [0, 10], grid [-2, 2]), the logistic problem ([0, 10],
    grid [-0.1, 1.2]) and Van der Pol (mu ~ U[1, 5], [0, 50], grid
    [-3, 3] x [-8, 8]); slices log-uniform in [16, 2048], 1-D grids log-uniform
    in [64, 8192] points, 2-D grids log-uniform in [16, 256] per axis, steps per
    slice uniform in [100, 2000].  scale < 1 shrinks slices, grids and steps
    proportionally (same draws) for tests, and the interval with them so that
    every problem keeps its step size."""
    rng = np.random.default_rng(seed)
    out = []
    fams = ("linear", "logistic", "vdp")
    for i in range(count):
        fam = fams[int(rng.integers(0, 3))]
        n_slices = _log_uniform_int(rng, 16, 2048)
        steps = int(rng.integers(100, 2001))
        if fam == "vdp":
            grid_n = (_log_uniform_int(rng, 16, 256), _log_uniform_int(rng, 16, 256))
            params, T, lo, hi, y0, interp = ((float(rng.uniform(1.0, 5.0)),), 50.0,
                                             (-3.0, -8.0), (3.0, 8.0), (2.0, 0.0), "bilinear")
        elif fam == "linear":
            grid_n = (_log_uniform_int(rng, 64, 8192),)
            params, T, lo, hi, y0, interp = ((float(rng.uniform(-2.0, 0.5)),), 10.0, (-2.0,),
                                             (2.0,), (1.0,), "linear")
        else:
            grid_n = (_log_uniform_int(rng, 64, 8192),)
            params, T, lo, hi, y0, interp = ((), 10.0, (-0.1,), (1.2,), (0.1,), "linear")
        if scale != 1.0:
            n_s, s_s = max(2, int(n_slices * scale)), max(2, int(steps * scale))
            T = T * (n_s * s_s) / (n_slices * steps)
            n_slices, steps = n_s, s_s
            grid_n = tuple(max(3, int(n * scale)) for n in grid_n)
        out.append(Workload(name=f"batch{i:02d}-{fam}", rhs=fam, params=params, t0=0.0, T=T,
                            n_slices=n_slices, grid_n=grid_n, grid_lo=lo, grid_hi=hi,
                            steps_per_slice=steps, y0=y0, precision="fp32", interp=interp))
    return out


def paper_model(n_slices: int, M: int, dt: float, precision: str = "fp64") -> Workload:
    """The model problem of sec. 3 as the paper runs it: y' = y^2, y(0) = 1 on
    [0, 1/2], backward Euler with step dt, Lagrange on the M Chebyshev extrema
    of [0, 2] (Tables 1 to 4)."""
    return Workload(name=f"paper-square-be-{precision}-{n_slices}sl-{M}cheb-dt{dt:g}",
                    rhs="square", params=(), t0=0.0, T=0.5, n_slices=n_slices, grid_n=(M,),
                    grid_lo=(0.0,), grid_hi=(2.0,), steps_per_slice=1, y0=(1.0,),
                    precision=precision, interp="chebyshev", scheme="be", dt=dt)


# Table 3 of the paper (sec. 4): dt in {2^-14, 2^-15, 2^-16} with M = 4, 5, 7
# Chebyshev nodes, N in {32, 64, 128} slices, single precision.
PAPER_TABLE3 = [(dt, n, M) for dt, M in ((2.0 ** -14, 4), (2.0 ** -15, 5), (2.0 ** -16, 7))
                for n in (32, 64, 128)]


# ---- learned surrogate of the Van der Pol slice map ---------------------------
# Network input x = (y1, y2, slice start time, mu), normalised as
# (x - shift) * scale so that the box [-3, 3] x [-8, 8], the interval [0, 50] and
# mu in [1, 5] map to [-1, 1]; outputs are slice displacements in units of
# SUR_OUT_SCALE (about their standard deviation over the box for slices of
# length 50/1024).
SUR_IN_SHIFT = (0.0, 0.0, 25.0, 3.0)
SUR_IN_SCALE = (1.0 / 3.0, 1.0 / 8.0, 1.0 / 25.0, 0.5)
SUR_OUT_SCALE = (0.2, 1.6)
SUR_SLICE_LENGTH = 50.0 / 1024
# With one coarse RK4 step over the slice the network learns only the
# correction to it: about 1/20 and 1/8 of the displacement's scale.
SUR_OUT_SCALE_COARSE = (0.01, 0.2)


# The step-doubling form (phi ~ G1 + d (16/15 + out_scale g out), G1 one RK4
# step over the slice, d the difference to two half steps): the gate scale per
# component (0.1 of d's spread over the visited training states), the unit of
# the training residual (its spread there) and the output scale; the training
# samples are weighted by their distance to the states that Richardson chains
# from y0 = (2, 0) visit for SUR_VISIT_MUS values of mu on [1, 5] (Gaussian of
# width SUR_VISIT_SIGMA in the network's input units, plus a floor).
SUR_SD_GATE = (5.7e-5, 2.0e-3)
SUR_SD_LOSS_SCALE = (1.8e-5, 7.4e-4)
SUR_SD_OUT_SCALE = (0.05, 0.05)
SUR_VISIT_MUS = 81
SUR_VISIT_SIGMA = 0.05
SUR_VISIT_FLOOR = 0.02


def surrogate_training_problems(n_slices: int = 1024, grid_n=(128, 128), steps: int = 500,
                                seed: int = 17, T: float = 50.0):
    """The training build: Van der Pol on [0, T] cut into n_slices slices, slice j
    integrated with its own mu_j ~ U[1, 5] (seeded), each slice a one-slice
    problem of a batch.  With the defaults: 1024 x 128 x 128 = 16.7M endpoints."""
    rng = np.random.default_rng(seed)
    mus = rng.uniform(1.0, 5.0, n_slices)
    L = T / n_slices
    return [Workload(name=f"sur-train-{j:04d}", rhs="vdp", params=(float(mus[j]),), t0=j * L,
                     T=(j + 1) * L, n_slices=1, grid_n=tuple(grid_n), grid_lo=(-3.0, -8.0),
                     grid_hi=(3.0, 8.0), steps_per_slice=steps, y0=(2.0, 0.0),
                     precision="fp32", interp="bilinear") for j in range(n_slices)]


def surrogate_init_params(seed: int = 0) -> np.ndarray:
    """Initial network parameters, flat (W1, b1, W2, b2, W3, b3, W4, b4): each
    layer's weights and biases uniform in +-1/sqrt(fan_in)."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((128, 4), (128, 128), (128, 128), (2, 128)):
        bound = 1.0 / np.sqrt(cols)
        parts.append(rng.uniform(-bound, bound, rows * cols))
        parts.append(rng.uniform(-bound, bound, rows))
    return np.concatenate(parts).astype(np.float32)


def surrogate_perm(total: int, seed: int = 5) -> np.ndarray:
    """The one-time shuffle of the training set (int64 permutation)."""
    return np.random.default_rng(seed).permutation(total).astype(np.int64)


def surrogate_eval_mus(count: int = 8, seed: int = 23) -> np.ndarray:
    """Held-out Van der Pol parameters for evaluating the surrogate."""
    return np.random.default_rng(seed).uniform(1.0, 5.0, count)


def surrogate_samples(n: int, seed: int):
    """Seeded network inputs over the training box and targets of unit scale,
    (4, n) and (2, n) float32, for parity checks of the network itself."""
    rng = np.random.default_rng(seed)
    x = np.stack([rng.uniform(-3, 3, n), rng.uniform(-8, 8, n), rng.uniform(0, 50, n),
                  rng.uniform(1, 5, n)]).astype(np.float32)
    t = rng.normal(0.0, 1.0, (2, n)).astype(np.float32)
    return x, t
