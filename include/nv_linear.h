/*
 * nv_linear.h — C ABI of libnv's affine basis propagator for linear systems.
 *
 * For a linear system y' = A(t) y + b(t) the slice map is affine in the
 * initial value, so the method needs no interpolation at all (the closing
 * discussion of linear problems in sec. 5, equations `lineardiscrete` and
 * `linearreconstruct`): on every slice solve once from y = 0 with the forcing
 * and once without it from each unit vector e_k; then
 *     phi_j(y) = c_j + G_j y,     c_j = g(0),  column k of G_j = g(e_k),
 * exactly, and the sequential pass is the chain lambda_{j+1} = c_j + G_j lambda_j.
 *
 * The system is the heat equation of sec. 6 (equation `heatequation`):
 *     y_t = a(t) y_xx + b(t, x),  x in [0, 1],  y = 0 at both ends,
 *     a(t) = a0 + a1 sin t,
 *     b(t, x) = beta(t) sin(pi x), beta(t) = pi^2 a(t) cos t - sin t (forcing on),
 * the forcing under which y = cos(t) sin(pi x) is the exact solution.  Space:
 * M interior points x_i = i/(M+1), centred second differences.  Time:
 * backward Euler (the paper's scheme), each step a tridiagonal solve by the
 * Thomas algorithm:
 *     r = (h a(t+h)) / (dx dx),  dx = 1/(M+1),
 *     w_1 = 1/(1+2r), c_1 = (-r) w_1;  w_i = 1/((1+2r) - (-r) c_{i-1}), c_i = (-r) w_i,
 *     f'_1 = f_1 w_1;  f'_i = (f_i - (-r) f'_{i-1}) w_i;
 *     y_M = f'_M;  y_i = f'_i - c_i y_{i+1},
 * f = y + (h beta(t+h)) sin(pi x_i), x_i = i dx, for the forced solve, f = y
 * otherwise; a(t) = a0 + a1 sin t and beta(t) = ((pi pi) a(t)) cos t - sin t.
 * Slices: L = (T - t0)/N; each slice takes floor(L/dt + 1e-9) steps of dt and
 * one step of the remainder when it exceeds 1e-12 L (step s of slice j ends at
 * T_j + (s+1) dt).  Everything is FP64 with one rounding per operation, and
 * a(t), beta(t) and sin(pi x_i) are evaluated on the host, so the tables and the
 * composition are specified to the bit.
 *
 * Conventions as in nv.h (status codes, nv_last_error, one thread per object).
 */
#ifndef NV_LINEAR_H
#define NV_LINEAR_H

#include "nv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define NV_LIN_MAX_POINTS 127

typedef struct {
    int M;                      /* interior points, 1 .. NV_LIN_MAX_POINTS */
    double a0, a1;              /* a(t) = a0 + a1 sin t; a(t) > 0 on the interval */
    int forcing;                /* 1: the forcing of the closed-form solution; 0: b = 0 */
} nv_heat;

typedef struct nv_lin nv_lin;

/* Create / destroy.  stream: hipStream_t of every kernel (NULL = null
 * stream).  Device memory is allocated by nv_lin_build and kept for builds of
 * the same or smaller size.  Errors: INVALID_ARG, HIP. */
NV_API nv_status nv_lin_create(void *stream, nv_lin **out);
NV_API nv_status nv_lin_destroy(nv_lin *lin);

/* Computation phase: the tables G (n_slices x M x M, G[j][i][k] = component i
 * of slice j's solve from e_k) and c (n_slices x M), kept in device memory in
 * a layout internal to the library (nv_lin_get_tables returns them in plain
 * order), M + 1 backward Euler solves per slice, all slices in one launch.
 * dt > 0.  Asynchronous with respect to the host.  Errors: INVALID_ARG
 * (M out of range, n_slices < 1, non-finite or empty interval, dt <= 0, a(t)
 * not positive at a step), OOM, HIP. */
NV_API nv_status nv_lin_build(nv_lin *lin, const nv_heat *problem, double t0, double T,
                              int n_slices, double dt);

/* Communication phase: lambda_0 = y0 (host, M values), lambda_{j+1} = c_j +
 * G_j lambda_j, component i formed as c_i + (((p0 + p1) + (p2 + p3)) + ((p4 +
 * p5) + (p6 + p7))) with p_r = G_i,r l_r + G_i,r+8 l_r+8 + ... summed left to
 * right from 0 (k counted from 0): eight independent chains instead of one.  yT (host, M) receives lambda_N; boundary (host, (N+1) x M, may be
 * NULL) every lambda_j.  Synchronous.  Errors: INVALID_ARG, NOT_BUILT,
 * NONFINITE (a state became non-finite), HIP. */
NV_API nv_status nv_lin_compose(nv_lin *lin, const double *y0, double *yT, double *boundary);

/* Communication phase for many initial values (sec. 5, equation
 * `linearreconstruct`, applied to count independent initial values): the
 * chains lambda^q_{j+1} = c_j + G_j lambda^q_j, q = 0..count-1, evaluated as
 * FP64 matrix products G_j [lambda^q ... lambda^{q+15}] on the matrix cores,
 * 16 chains per workgroup (32, sharing the workgroup's table reads, when
 * count fills two such workgroups per compute unit and M <= 116).  Each component's sum c_i + sum_k G_ik l_k is
 * formed by the matrix cores in an order this interface does not fix (so
 * results are within the FP64 inner-product rounding bound of any order, not
 * bit-equal to nv_lin_compose).
 *   y0_dev        device, count x M doubles (chain q's initial value at q M)
 *   yT_dev        device, count x M doubles: lambda^q_N
 *   boundary_dev  device, count x (N + 1) x M doubles, chain-major
 *                 (lambda^q_j at (q (N + 1) + j) M), or NULL
 * Synchronous.  Errors: INVALID_ARG (NULL pointers, count < 1), NOT_BUILT,
 * NONFINITE (some chain's state became non-finite; the message names the
 * first such slice), HIP. */
NV_API nv_status nv_lin_compose_many(nv_lin *lin, const double *y0_dev, long long count,
                                     double *yT_dev, double *boundary_dev);

/* Copy the tables of the last build to host memory (G: n_slices*M*M values,
 * c: n_slices*M values; either may be NULL).  Errors: NOT_BUILT, HIP. */
NV_API nv_status nv_lin_get_tables(nv_lin *lin, double *G, double *c);

/* Milliseconds of the last build's and the last composition's kernels (HIP
 * events on the object's stream). */
NV_API nv_status nv_lin_last_timing(nv_lin *lin, float *build_ms, float *compose_ms);

#ifdef __cplusplus
}
#endif
#endif
