// Device code of the computation phase of Nievergelt's method (sec. 3,
// pseudocode figure): right-hand sides, the RK4 / forward Euler step with the
// FP32 accumulation modes, the grid point of a lane, and the integration of
// one tile of one slice.  Included by the kernels that launch it.
#pragma once

#include "nv_internal.h"

#include <cmath>

namespace nv {
namespace dev {

// ---------------------------------------------------------------------------
// Right-hand sides.  F is the wave-uniform forcing value of the stage time
// (used by non-autonomous problems only), p the parameter.
// ---------------------------------------------------------------------------
template <class R>
struct RhsLinear {              // y' = p y
    static constexpr int dim = 1;
    static constexpr bool forced = false;
    static constexpr bool tangent = false;
    static constexpr int rhs_id = 0;
    __device__ static void f(R, R p, const R *y, R *k) { k[0] = p * y[0]; }
    __device__ static R df(R, R p, R) { return p; }
    // f and (df/dy) v together (the variational term of slope builds)
    __device__ static void fjv(R, R p, R y, R v, R &k, R &kv) {
        k = p * y;
        kv = p * v;
    }
};

template <class R>
struct RhsLogistic {            // y' = y (1 - y)
    static constexpr int dim = 1;
    static constexpr bool forced = false;
    static constexpr bool tangent = false;
    static constexpr int rhs_id = 1;
    __device__ static void f(R, R, const R *y, R *k) { k[0] = y[0] - y[0] * y[0]; }
    __device__ static R df(R, R, R y) { return R(1) - R(2) * y; }
    __device__ static void fjv(R, R, R y, R v, R &k, R &kv) {
        k = y - y * y;
        kv = (R(1) - R(2) * y) * v;
    }
};

template <class R>
struct RhsForcedCubic {         // y' = sin(3t) - y^3, F = sin(3t)
    static constexpr int dim = 1;
    static constexpr bool forced = true;
    static constexpr bool tangent = false;
    static constexpr int rhs_id = 2;  // nv_rhs_id, for forcing_value
    __device__ static void f(R F, R, const R *y, R *k) {
        R y2 = y[0] * y[0];
        k[0] = F - y2 * y[0];
    }
    __device__ static R df(R, R, R y) { return R(-3) * y * y; }
    // the square serves both terms: -3 y^2 is formed from it
    __device__ static void fjv(R F, R, R y, R v, R &k, R &kv) {
        const R y2 = y * y;
        k = F - y2 * y;
        kv = (R(-3) * y2) * v;
    }
};

template <class R>
struct RhsVdp {                 // y1' = y2, y2' = mu (1 - y1^2) y2 - y1
    static constexpr int dim = 2;
    static constexpr bool forced = false;
    static constexpr bool tangent = false;
    static constexpr int rhs_id = 3;
    __device__ static void f(R, R mu, const R *y, R *k) {
        R a = R(1) - y[0] * y[0];
        k[0] = y[1];
        k[1] = (mu * a) * y[1] - y[0];
    }
};

template <class R>
struct RhsSquare {              // y' = y^2
    static constexpr int dim = 1;
    static constexpr bool forced = false;
    static constexpr bool tangent = false;
    static constexpr int rhs_id = 4;
    __device__ static void f(R, R, const R *y, R *k) { k[0] = y[0] * y[0]; }
    __device__ static R df(R, R, R y) { return R(2) * y; }
    __device__ static void fjv(R, R, R y, R v, R &k, R &kv) {
        k = y * y;
        kv = (R(2) * y) * v;
    }
};

// A one-dimensional right-hand side together with its variational equation:
// state (y, v), y' = f(t, y), v' = df/dy(t, y) v.  A scheme applied to this
// pair gives, in v, the derivative of the scheme's own map for y with respect
// to y's initial value when v starts at 1 (a Runge-Kutta method commutes with
// differentiation with respect to the initial value), and the y component is
// formed by exactly the operations of the plain build.
template <template <class> class Base, class R>
struct RhsTangent {
    static_assert(Base<R>::dim == 1, "slopes are built for one-dimensional right-hand sides");
    static constexpr int dim = 2;
    static constexpr bool forced = Base<R>::forced;
    static constexpr bool tangent = true;
    static constexpr int rhs_id = Base<R>::rhs_id;
    // k[0] by the operations of Base::f, k[1] = df/dy(y[0]) y[1]
    __device__ static void f(R F, R p, const R *y, R *k) { Base<R>::fjv(F, p, y[0], y[1], k[0], k[1]); }
};

// The forcing function of non-autonomous right-hand sides.
__device__ inline double forcing_value(int rhs, double t) {
    return rhs == 2 ? sin(3.0 * t) : 0.0;
}

// Workgroup id -> logical tile id such that XCD x (which receives workgroups
// x, x+8, x+16, ...) processes one contiguous range of logical tiles.
__device__ inline int xcd_remap(int b, int nblocks) {
    const int q = nblocks / kNumXcd, r = nblocks % kNumXcd;
    const int x = b % kNumXcd, local = b / kNumXcd;
    return (x < r) ? x * (q + 1) + local : r * (q + 1) + (x - r) * q + local;
}

// Grid point of flat index k: xi = lo + k * dxi per axis, in FP64 (one
// rounding per operation), then rounded to the working precision.
template <class R, int D>
__device__ inline void grid_point(const BuildArgs &a, long long k, R *y) {
#pragma clang fp contract(off)
    if constexpr (D == 1) {
        y[0] = a.nodes ? R(a.nodes[k]) : R(a.lo0 + double(k) * a.dxi0);
    } else {
        const unsigned kk = unsigned(k), n1 = unsigned(a.n1);
        const unsigned k0 = kk / n1, k1 = kk - k0 * n1;
        y[0] = R(a.lo0 + double(k0) * a.dxi0);
        y[1] = R(a.lo1 + double(k1) * a.dxi1);
    }
}

// State accumulation of the FP32 build (Acc):
//   kPlain    y <- y + dy, one rounding per step;
//   kKahan    compensated summation: c carries the low-order part the rounded
//             state lost in earlier updates (3 extra operations per step);
//   kBlocked  blocked summation: the state is y (fixed for a block of
//             kSumBlock steps) plus a small accumulator a of the block's
//             increments, z = y + a is the state the stages see; a is folded
//             into y once per block (1 extra operation per step).
enum Acc { kPlain = 0, kKahan = 1, kBlocked = 2 };
constexpr int kSumBlock = 64;

// One step of the scheme for P trajectories.  Fa, Fb, Fc: forcing at the
// step's start, midpoint and end times.
template <class Rhs, class R, int Scheme, int A, int P>
__device__ inline void step(R (&y)[P][Rhs::dim], R (&c)[P][Rhs::dim], R (&z)[P][Rhs::dim],
                            R Fa, R Fb, R Fc, R h, R h2, R h6, R p) {
    constexpr int D = Rhs::dim;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        R k1[D], k2[D], k3[D], k4[D], u[D], dy[D];
        // the state the right-hand side sees
        R (&x)[D] = A == kBlocked ? z[q] : y[q];
        if constexpr (Scheme == 1) {                 // forward Euler
            Rhs::f(Fa, p, x, k1);
#pragma unroll
            for (int d = 0; d < D; ++d) dy[d] = h * k1[d];
        } else if constexpr (Scheme == 2) {          // backward Euler, one Newton step
            static_assert(D == 1, "backward Euler is built for 1-D right-hand sides");
            Rhs::f(Fc, p, x, k1);
            const R den = R(1) - h * Rhs::df(Fc, p, x[0]);
            if constexpr (sizeof(R) == 4)
                // FP32: the hardware reciprocal (about 1 ulp) instead of the
                // correctly rounded division sequence, which would dominate the
                // latency of this strictly sequential step
                dy[0] = (h * k1[0]) * __builtin_amdgcn_rcpf(den);
            else
                dy[0] = (h * k1[0]) / den;
        } else if constexpr (sizeof(R) == 8 && A == kPlain) {
            // classical RK4 for FP64 builds, which are small and bound by the
            // latency of each trajectory's chain: the weights are folded into
            // a running sum one stage at a time, y + h/6 k1 + h/3 k2 + h/3 k3
            // + h/6 k4 (h/3 = 2 (h/6) exactly), each partial sum formed right
            // after its stage and beside the next stage value, so the step's
            // chain is its seven stage operations and the final update (three
            // roundings more per step than one update by the weighted sum)
            const R h3 = R(2) * h6;
            R acc[D];
            Rhs::f(Fa, p, x, k1);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                u[d] = x[d] + h2 * k1[d];
                acc[d] = x[d] + h6 * k1[d];
            }
            Rhs::f(Fb, p, u, k2);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                u[d] = x[d] + h2 * k2[d];
                acc[d] = acc[d] + h3 * k2[d];
            }
            Rhs::f(Fb, p, u, k3);
#pragma unroll
            for (int d = 0; d < D; ++d) {
                u[d] = x[d] + h * k3[d];
                acc[d] = acc[d] + h3 * k3[d];
            }
            Rhs::f(Fc, p, u, k4);
#pragma unroll
            for (int d = 0; d < D; ++d) y[q][d] = acc[d] + h6 * k4[d];
            continue;
        } else {                                     // classical RK4
            Rhs::f(Fa, p, x, k1);
#pragma unroll
            for (int d = 0; d < D; ++d) u[d] = x[d] + h2 * k1[d];
            Rhs::f(Fb, p, u, k2);
#pragma unroll
            for (int d = 0; d < D; ++d) u[d] = x[d] + h2 * k2[d];
            Rhs::f(Fb, p, u, k3);
#pragma unroll
            for (int d = 0; d < D; ++d) u[d] = x[d] + h * k3[d];
            Rhs::f(Fc, p, u, k4);
#pragma unroll
            for (int d = 0; d < D; ++d) dy[d] = h6 * ((k1[d] + k4[d]) + R(2) * (k2[d] + k3[d]));
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            if constexpr (A == kKahan) {
                const R yk = dy[d] - c[q][d];
                const R t = y[q][d] + yk;
                c[q][d] = (t - y[q][d]) - yk;
                y[q][d] = t;
            } else if constexpr (A == kBlocked) {
                c[q][d] = c[q][d] + dy[d];           // block accumulator
                z[q][d] = y[q][d] + c[q][d];
            } else {
                y[q][d] = y[q][d] + dy[d];
            }
        }
    }
}

// Fold the block accumulator into the state (blocked summation only).
template <int D, class R, int A, int P>
__device__ inline void end_block(R (&y)[P][D], R (&c)[P][D], R (&z)[P][D]) {
    if constexpr (A == kBlocked) {
#pragma unroll
        for (int q = 0; q < P; ++q)
#pragma unroll
            for (int d = 0; d < D; ++d) {
                y[q][d] = y[q][d] + c[q][d];
                c[q][d] = R(0);
                z[q][d] = y[q][d];
            }
    }
}

// Integrate and store one tile: 256*P consecutive grid points of slice j, F
// the slice's forcing row (right-hand sides with forcing).  Returns how many
// non-finite end states (per trajectory: either component) this lane stored.
template <class Rhs, class R, int Scheme, int A, int P>
__device__ inline unsigned build_tile_rows(const BuildArgs &a, int j, int tile,
                                           const R *__restrict__ F) {
    constexpr int D = Rhs::dim;
    const long long base = (long long)tile * (kBuildBlock * P) + threadIdx.x;

    R y[P][D], c[P][D], z[P][D];
#pragma unroll
    for (int q = 0; q < P; ++q) {
        long long k = base + (long long)q * kBuildBlock;
        if (k >= a.M) k = a.M - 1;           // ragged tail: compute, do not store
        if constexpr (Rhs::tangent) {
            grid_point<R, 1>(a, k, y[q]);    // the grid is one-dimensional
            y[q][1] = R(1);                  // d y0 / d xi
        } else {
            grid_point<R, D>(a, k, y[q]);
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
            c[q][d] = R(0);
            z[q][d] = y[q][d];
        }
    }

    const R h = R(a.h), h2 = R(a.h * 0.5), h6 = R(a.h / 6.0), p = R(a.p0);
    const int S = a.steps;
    // Builds small enough to leave one wave per SIMD are bound by that wave's
    // own instruction stream, in which the loop's counter, compare and branch
    // take issue slots; large builds hide them behind other waves.  Unrolling
    // 8 steps (with the loop aligned to the instruction cache line, a build
    // flag of the files that include this one) measured fastest for the small
    // builds and equal for the large ones.
    constexpr int kUnroll = 8;
    for (int s0 = 0; s0 < S; s0 += kSumBlock) {
        const int s1 = min(s0 + kSumBlock, S);
#pragma unroll kUnroll
        for (int s = s0; s < s1; ++s) {
            if constexpr (Rhs::forced)
                step<Rhs, R, Scheme, A, P>(y, c, z, F[2 * s], F[2 * s + 1], F[2 * s + 2], h, h2,
                                           h6, p);
            else
                step<Rhs, R, Scheme, A, P>(y, c, z, R(0), R(0), R(0), h, h2, h6, p);
        }
        end_block<D, R, A, P>(y, c, z);
    }
    if (a.h_last > 0.0) {      // the shorter final step of a fixed-step slice
        if constexpr (!Rhs::forced) {
            step<Rhs, R, Scheme, A, P>(y, c, z, R(0), R(0), R(0), R(a.h_last),
                                       R(a.h_last * 0.5), R(a.h_last / 6.0), p);
            end_block<D, R, A, P>(y, c, z);
        }
    }

    R *t0 = static_cast<R *>(a.tab0) + (long long)j * a.M;
    R *t1 = D == 2 ? static_cast<R *>(a.tab1) + (long long)j * a.M : nullptr;
    unsigned bad = 0;
#pragma unroll
    for (int q = 0; q < P; ++q) {
        const long long k = base + (long long)q * kBuildBlock;
        if (k < a.M) {
            t0[k] = y[q][0];
            bad += !isfinite(y[q][0]);
            if constexpr (D == 2) {
                t1[k] = y[q][1];
                bad += !isfinite(y[q][1]) && isfinite(y[q][0]);
            }
        }
    }
    return bad;
}

// The same, the forcing row taken from the build's forcing array.
template <class Rhs, class R, int Scheme, int A, int P>
__device__ inline unsigned build_tile(const BuildArgs &a, int j, int tile) {
    const R *F = Rhs::forced
                     ? static_cast<const R *>(a.forcing) + (long long)j * (2 * a.steps + 1)
                     : nullptr;
    return build_tile_rows<Rhs, R, Scheme, A, P>(a, j, tile, F);
}

}  // namespace dev
}  // namespace nv
