/*
 * Plain serial CPU oracle for Nievergelt's parallel-in-time method
 * (A. T. Barker, arXiv:1304.6514).  TEST INFRASTRUCTURE ONLY: see nv_oracle.h.
 *
 * Written to be read against the paper:
 *   - the time partition T_j and the two phases follow the pseudocode figure
 *     of sec. 3 (Fig. 4): every slice solves the IVP from every sample point,
 *     then the boundary values are obtained one after the other by
 *     lambda_j = phi^j(lambda_{j-1}), starting from y0 (slice 1 is
 *     interpolated too);
 *   - the interpolation rules (linear, cubic Hermite with finite-difference
 *     slopes or with stored slopes, bilinear) and the lookup are the plain
 *     definitions written out;
 *   - the optional slope table holds the derivative of each entry's discrete
 *     map with respect to its grid point, carried through every stage by the
 *     chain rule (one-dimensional problems);
 *   - paper mode is backward Euler plus Lagrange interpolation on Chebyshev
 *     nodes, as in sec. 3 and Table 1.
 * No blocking, no reordering, no vectorisation.
 */
#include "nv_oracle.h"

#include <math.h>
#include <stdlib.h>

int orc_rhs_dim(int rhs) {
    switch (rhs) {
    case ORC_LIN:
    case ORC_LOG:
    case ORC_FCUB:
    case ORC_SQR:
        return 1;
    case ORC_VDP:
        return 2;
    default:
        return 0;
    }
}

/* f(t, y) for the problem families. */
static void rhs_eval(int rhs, const double *p, double t, const double *y, double *f) {
    switch (rhs) {
    case ORC_LIN:
        f[0] = p[0] * y[0];
        break;
    case ORC_LOG:
        f[0] = y[0] * (1.0 - y[0]);
        break;
    case ORC_FCUB:
        f[0] = sin(3.0 * t) - y[0] * y[0] * y[0];
        break;
    case ORC_VDP:
        f[0] = y[1];
        f[1] = p[0] * (1.0 - y[0] * y[0]) * y[1] - y[0];
        break;
    case ORC_SQR:
        f[0] = y[0] * y[0];
        break;
    }
}

/* One step from time ta to tc = ta + h (tb = midpoint), state y in place. */
static void one_step(int rhs, const double *p, int scheme, double ta, double tb,
                     double tc, double h, double *y) {
    int d = orc_rhs_dim(rhs);
    double k1[2], k2[2], k3[2], k4[2], z[2];
    int c;
    if (scheme == ORC_EULER) {
        rhs_eval(rhs, p, ta, y, k1);
        for (c = 0; c < d; ++c) y[c] = y[c] + h * k1[c];
        return;
    }
    /* classical Runge-Kutta */
    rhs_eval(rhs, p, ta, y, k1);
    for (c = 0; c < d; ++c) z[c] = y[c] + (h / 2.0) * k1[c];
    rhs_eval(rhs, p, tb, z, k2);
    for (c = 0; c < d; ++c) z[c] = y[c] + (h / 2.0) * k2[c];
    rhs_eval(rhs, p, tb, z, k3);
    for (c = 0; c < d; ++c) z[c] = y[c] + h * k3[c];
    rhs_eval(rhs, p, tc, z, k4);
    for (c = 0; c < d; ++c)
        y[c] = y[c] + (h / 6.0) * (k1[c] + 2.0 * k2[c] + 2.0 * k3[c] + k4[c]);
}

/* df/dy of a one-dimensional right-hand side at (t, y). */
static double rhs_jacobian(int rhs, const double *p, double y) {
    switch (rhs) {
    case ORC_LIN:
        return p[0];
    case ORC_LOG:
        return 1.0 - 2.0 * y;
    case ORC_FCUB:
        return -3.0 * y * y;
    case ORC_SQR:
        return 2.0 * y;
    default:
        return 0.0;
    }
}

/* One step of a one-dimensional problem together with the derivative of the
 * step's result with respect to the initial value of the trajectory: v holds
 * dy/dxi before the step and afterwards the derivative of the new y, by the
 * chain rule through every stage of the step (the derivative of the discrete
 * map, not of the exact flow).  y follows exactly the operations of one_step. */
static void one_step_tangent(int rhs, const double *p, int scheme, double ta, double tb,
                             double tc, double h, double *y, double *v) {
    double k1, k2, k3, k4, z, d1, d2, d3, d4, dz, yy = *y, vv = *v;
    if (scheme == ORC_EULER) {
        rhs_eval(rhs, p, ta, &yy, &k1);
        d1 = rhs_jacobian(rhs, p, yy) * vv;
        *y = yy + h * k1;
        *v = vv + h * d1;
        return;
    }
    rhs_eval(rhs, p, ta, &yy, &k1);
    d1 = rhs_jacobian(rhs, p, yy) * vv;
    z = yy + (h / 2.0) * k1;
    dz = vv + (h / 2.0) * d1;
    rhs_eval(rhs, p, tb, &z, &k2);
    d2 = rhs_jacobian(rhs, p, z) * dz;
    z = yy + (h / 2.0) * k2;
    dz = vv + (h / 2.0) * d2;
    rhs_eval(rhs, p, tb, &z, &k3);
    d3 = rhs_jacobian(rhs, p, z) * dz;
    z = yy + h * k3;
    dz = vv + h * d3;
    rhs_eval(rhs, p, tc, &z, &k4);
    d4 = rhs_jacobian(rhs, p, z) * dz;
    *y = yy + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4);
    *v = vv + (h / 6.0) * (d1 + 2.0 * d2 + 2.0 * d3 + d4);
}

static int valid_problem(int rhs, int scheme) {
    return orc_rhs_dim(rhs) > 0 && (scheme == ORC_RK4 || scheme == ORC_EULER);
}

int orc_integrate(int rhs, const double *p, int scheme, double t_base, double h,
                  long long nsteps, double *y) {
    long long s;
    if (!valid_problem(rhs, scheme) || nsteps < 0) return ORC_BAD_ARG;
    for (s = 0; s < nsteps; ++s) {
        double ta = t_base + (double)s * h;
        double tb = ta + h / 2.0;
        double tc = t_base + (double)(s + 1) * h;
        one_step(rhs, p, scheme, ta, tb, tc, h, y);
    }
    return ORC_OK;
}

int orc_integrate_tangent(int rhs, const double *p, int scheme, double t_base, double h,
                          long long nsteps, double *y, double *v) {
    long long s;
    if (!valid_problem(rhs, scheme) || orc_rhs_dim(rhs) != 1 || nsteps < 0) return ORC_BAD_ARG;
    for (s = 0; s < nsteps; ++s) {
        double ta = t_base + (double)s * h;
        double tb = ta + h / 2.0;
        double tc = t_base + (double)(s + 1) * h;
        one_step_tangent(rhs, p, scheme, ta, tb, tc, h, y, v);
    }
    return ORC_OK;
}

/* Slice length L = (T - t0)/N, slice start T_j = t0 + j L, step h = L / S. */
static double slice_length(double t0, double T, int n_slices) {
    return (T - t0) / (double)n_slices;
}
static double slice_start(double t0, double L, long long j) {
    return t0 + (double)j * L;
}

int orc_serial(int rhs, const double *p, int scheme, double t0, double T,
               int n_slices, int steps_per_slice, const double *y0, double *yT) {
    double L, h;
    int c, d = orc_rhs_dim(rhs);
    if (!valid_problem(rhs, scheme) || n_slices < 1 || steps_per_slice < 1)
        return ORC_BAD_ARG;
    L = slice_length(t0, T, n_slices);
    h = L / (double)steps_per_slice;
    for (c = 0; c < d; ++c) yT[c] = y0[c];
    return orc_integrate(rhs, p, scheme, t0, h,
                         (long long)n_slices * (long long)steps_per_slice, yT);
}

int orc_serial_steps(int rhs, const double *p, int scheme, double t0, double T,
                     long long nsteps, const double *y0, double *yT) {
    int c, d = orc_rhs_dim(rhs);
    if (!valid_problem(rhs, scheme) || nsteps < 1) return ORC_BAD_ARG;
    for (c = 0; c < d; ++c) yT[c] = y0[c];
    return orc_integrate(rhs, p, scheme, t0, (T - t0) / (double)nsteps, nsteps, yT);
}

static int valid_grid(const orc_grid *g) {
    int a;
    if (g->dim < 1 || g->dim > 2) return 0;
    for (a = 0; a < g->dim; ++a)
        if (g->n[a] < 2 || !(g->hi[a] > g->lo[a])) return 0;
    return 1;
}

static long long grid_size(const orc_grid *g) {
    return g->dim == 1 ? (long long)g->n[0] : (long long)g->n[0] * (long long)g->n[1];
}

/* point k of one axis: lo + k (hi - lo)/(n - 1) */
static double axis_point(double lo, double hi, int n, long long k) {
    double dxi = (hi - lo) / (double)(n - 1);
    return lo + (double)k * dxi;
}

int orc_grid_point(const orc_grid *g, long long k, double *xi) {
    if (!valid_grid(g) || k < 0 || k >= grid_size(g)) return ORC_BAD_ARG;
    if (g->dim == 1) {
        xi[0] = axis_point(g->lo[0], g->hi[0], g->n[0], k);
    } else {
        long long k0 = k / g->n[1], k1 = k % g->n[1];
        xi[0] = axis_point(g->lo[0], g->hi[0], g->n[0], k0);
        xi[1] = axis_point(g->lo[1], g->hi[1], g->n[1], k1);
    }
    return ORC_OK;
}

/* Solve the IVP on slice j from grid point k: the value lambda_j^k. */
static void table_entry(int rhs, const double *p, int scheme, double t0, double L,
                        double h, int steps, const orc_grid *g, long long j,
                        long long k, double *out) {
    orc_grid_point(g, k, out);
    orc_integrate(rhs, p, scheme, slice_start(t0, L, j), h, steps, out);
}

static int check_method_args(int rhs, int scheme, int n_slices, const orc_grid *g,
                             int steps) {
    if (!valid_problem(rhs, scheme) || n_slices < 1 || steps < 1) return 0;
    if (!valid_grid(g) || g->dim != orc_rhs_dim(rhs)) return 0;
    return 1;
}

int orc_build_tables(int rhs, const double *p, int scheme, double t0, double T,
                     int n_slices, const orc_grid *g, int steps_per_slice,
                     double *tab) {
    long long j, k, M;
    int c, d;
    double L, h, y[2];
    if (!check_method_args(rhs, scheme, n_slices, g, steps_per_slice)) return ORC_BAD_ARG;
    d = g->dim;
    M = grid_size(g);
    L = slice_length(t0, T, n_slices);
    h = L / (double)steps_per_slice;
    for (j = 0; j < n_slices; ++j)
        for (k = 0; k < M; ++k) {
            table_entry(rhs, p, scheme, t0, L, h, steps_per_slice, g, j, k, y);
            for (c = 0; c < d; ++c) tab[((long long)c * n_slices + j) * M + k] = y[c];
        }
    return ORC_OK;
}

/* The value and the slope (its derivative with respect to the grid point) of
 * entry (slice j, grid point k) of a one-dimensional problem. */
static void table_entry_tangent(int rhs, const double *p, int scheme, double t0, double L,
                                double h, int steps, const orc_grid *g, long long j,
                                long long k, double *value, double *slope) {
    orc_grid_point(g, k, value);
    *slope = 1.0;
    orc_integrate_tangent(rhs, p, scheme, slice_start(t0, L, j), h, steps, value, slope);
}

int orc_build_tables_slopes(int rhs, const double *p, int scheme, double t0, double T,
                            int n_slices, const orc_grid *g, int steps_per_slice,
                            double *tab) {
    long long j, k, M;
    double L, h, v, m;
    if (!check_method_args(rhs, scheme, n_slices, g, steps_per_slice) || g->dim != 1)
        return ORC_BAD_ARG;
    M = grid_size(g);
    L = slice_length(t0, T, n_slices);
    h = L / (double)steps_per_slice;
    for (j = 0; j < n_slices; ++j)
        for (k = 0; k < M; ++k) {
            table_entry_tangent(rhs, p, scheme, t0, L, h, steps_per_slice, g, j, k, &v, &m);
            tab[j * M + k] = v;
            tab[((long long)n_slices + j) * M + k] = m;
        }
    return ORC_OK;
}

int orc_table_entries(int rhs, const double *p, int scheme, double t0, double T,
                      int n_slices, const orc_grid *g, int steps_per_slice,
                      long long count, const long long *slice,
                      const long long *point, double *out) {
    long long q, M;
    int c, d;
    double L, h, y[2];
    if (!check_method_args(rhs, scheme, n_slices, g, steps_per_slice)) return ORC_BAD_ARG;
    d = g->dim;
    M = grid_size(g);
    L = slice_length(t0, T, n_slices);
    h = L / (double)steps_per_slice;
    for (q = 0; q < count; ++q) {
        if (slice[q] < 0 || slice[q] >= n_slices || point[q] < 0 || point[q] >= M)
            return ORC_BAD_ARG;
        table_entry(rhs, p, scheme, t0, L, h, steps_per_slice, g, slice[q], point[q], y);
        for (c = 0; c < d; ++c) out[(long long)c * count + q] = y[c];
    }
    return ORC_OK;
}

int orc_table_entries_slopes(int rhs, const double *p, int scheme, double t0, double T,
                             int n_slices, const orc_grid *g, int steps_per_slice,
                             long long count, const long long *slice,
                             const long long *point, double *out) {
    long long q, M;
    double L, h;
    if (!check_method_args(rhs, scheme, n_slices, g, steps_per_slice) || g->dim != 1)
        return ORC_BAD_ARG;
    M = grid_size(g);
    L = slice_length(t0, T, n_slices);
    h = L / (double)steps_per_slice;
    for (q = 0; q < count; ++q) {
        if (slice[q] < 0 || slice[q] >= n_slices || point[q] < 0 || point[q] >= M)
            return ORC_BAD_ARG;
        table_entry_tangent(rhs, p, scheme, t0, L, h, steps_per_slice, g, slice[q], point[q],
                            &out[q], &out[count + q]);
    }
    return ORC_OK;
}

/* u = (x - lo) * (n - 1)/(hi - lo); cell = floor(u) limited to [0, n-2];
 * w = u - cell.  Outside the grid w leaves [0, 1] (extrapolation).  A NaN
 * query gives cell 0, w = NaN, and counts as outside. */
int orc_locate(double lo, double hi, int n, double x, long long *cell, double *w) {
    double inv = (double)(n - 1) / (hi - lo);
    double u = (x - lo) * inv;
    double f;
    long long i;
    if (isnan(u)) {
        *cell = 0;
        *w = u;
        return 1;
    }
    f = floor(u);
    if (f < 0.0)
        i = 0;
    else if (f > (double)(n - 2))
        i = n - 2;
    else
        i = (long long)f;
    *cell = i;
    *w = u - (double)i;
    return (u < 0.0 || u > (double)(n - 1)) ? 1 : 0;
}

/* Source of table values for the communication phase: component c of the
 * entry (slice j, grid point k). */
typedef struct {
    const double *tab; /* full tables, or NULL for on-demand integration */
    long long M;
    int n_slices;
    /* on-demand integration */
    int rhs, scheme, steps;
    const double *p;
    double t0, L, h;
    const orc_grid *g;
    /* component 1 is the slope table of a one-dimensional problem */
    int slopes;
    /* one-entry memo so that a 2-D entry is integrated once for both components */
    long long memo_j, memo_k;
    double memo[2];
} entry_source;

static double entry_value(entry_source *src, int c, long long j, long long k) {
    if (src->tab) return src->tab[((long long)c * src->n_slices + j) * src->M + k];
    if (src->memo_j != j || src->memo_k != k) {
        if (src->slopes)
            table_entry_tangent(src->rhs, src->p, src->scheme, src->t0, src->L, src->h,
                                src->steps, src->g, j, k, &src->memo[0], &src->memo[1]);
        else
            table_entry(src->rhs, src->p, src->scheme, src->t0, src->L, src->h, src->steps,
                        src->g, j, k, src->memo);
        src->memo_j = j;
        src->memo_k = k;
    }
    return src->memo[c];
}

/* Delta-xi times the slope at node i, from the table by finite differences:
 * centred inside, one-sided second order at the two ends. */
static double hermite_node_slope(entry_source *src, long long j, long long i, int n) {
    if (i == 0) {
        double t0 = entry_value(src, 0, j, 0), t1 = entry_value(src, 0, j, 1),
               t2 = entry_value(src, 0, j, 2);
        return 0.5 * ((4.0 * t1 - 3.0 * t0) - t2);
    }
    if (i == n - 1) {
        double a = entry_value(src, 0, j, n - 1), b = entry_value(src, 0, j, n - 2),
               c = entry_value(src, 0, j, n - 3);
        return 0.5 * ((3.0 * a - 4.0 * b) + c);
    }
    return 0.5 * (entry_value(src, 0, j, i + 1) - entry_value(src, 0, j, i - 1));
}

/* The interpolants.  Any non-finite value they read sets *bad. */
static double interp_linear(entry_source *src, long long j, long long i, double w, int *bad) {
    double a = entry_value(src, 0, j, i), b = entry_value(src, 0, j, i + 1);
    if (!isfinite(a) || !isfinite(b)) *bad = 1;
    return a + w * (b - a);
}

static double interp_hermite(entry_source *src, long long j, long long i, double w, int n,
                             int *bad) {
    double a = entry_value(src, 0, j, i), b = entry_value(src, 0, j, i + 1);
    double da = hermite_node_slope(src, j, i, n), db = hermite_node_slope(src, j, i + 1, n);
    double w2 = w * w, w3 = w2 * w;
    double h00 = (2.0 * w3 - 3.0 * w2) + 1.0;
    double h10 = (w3 - 2.0 * w2) + w;
    double h01 = 3.0 * w2 - 2.0 * w3;
    double h11 = w3 - w2;
    if (!isfinite(a) || !isfinite(b) || !isfinite(da) || !isfinite(db)) *bad = 1;
    return ((h00 * a + h10 * da) + h01 * b) + h11 * db;
}

/* Cubic Hermite with the stored slopes (component 1): the same basis and
 * sum as interp_hermite, Delta-xi times the slope at each node taken from the
 * slope table, Delta-xi = (hi - lo)/(n - 1). */
static double interp_hermite_slopes(entry_source *src, long long j, long long i, double w,
                                    double dxi, int *bad) {
    double a = entry_value(src, 0, j, i), b = entry_value(src, 0, j, i + 1);
    double da = dxi * entry_value(src, 1, j, i), db = dxi * entry_value(src, 1, j, i + 1);
    double w2 = w * w, w3 = w2 * w;
    double h00 = (2.0 * w3 - 3.0 * w2) + 1.0;
    double h10 = (w3 - 2.0 * w2) + w;
    double h01 = 3.0 * w2 - 2.0 * w3;
    double h11 = w3 - w2;
    if (!isfinite(a) || !isfinite(b) || !isfinite(da) || !isfinite(db)) *bad = 1;
    return ((h00 * a + h10 * da) + h01 * b) + h11 * db;
}

static void interp_bilinear(entry_source *src, long long j, long long i0, double w0,
                            long long i1, double w1, int n1, double *out, int *bad) {
    int c;
    for (c = 0; c < 2; ++c) {
        double t00 = entry_value(src, c, j, i0 * n1 + i1);
        double t01 = entry_value(src, c, j, i0 * n1 + i1 + 1);
        double t10 = entry_value(src, c, j, (i0 + 1) * n1 + i1);
        double t11 = entry_value(src, c, j, (i0 + 1) * n1 + i1 + 1);
        double r0 = t00 + w1 * (t01 - t00);
        double r1 = t10 + w1 * (t11 - t10);
        if (!isfinite(t00) || !isfinite(t01) || !isfinite(t10) || !isfinite(t11)) *bad = 1;
        out[c] = r0 + w0 * (r1 - r0);
    }
}

static int interp_fits(const orc_grid *g, int interp) {
    if (interp == ORC_I_LINEAR) return g->dim == 1;
    if (interp == ORC_I_HERMITE) return g->dim == 1 && g->n[0] >= 3;
    if (interp == ORC_I_BILINEAR) return g->dim == 2;
    if (interp == ORC_I_HERMITE_SLOPES) return g->dim == 1;
    return 0;
}

/* Communication phase: lambda_0 = y0, lambda_{j+1} = phi^j(lambda_j). */
static int compose(entry_source *src, const orc_grid *g, int interp, int n_slices,
                   const double *y0, double *boundary, long long *cells,
                   double *weights, long long *n_out_of_grid, int *bad_slice) {
    int d = g->dim, c, a;
    long long j, oog = 0;
    double lam[2], next[2];
    for (c = 0; c < d; ++c) lam[c] = y0[c];
    if (boundary)
        for (c = 0; c < d; ++c) boundary[c] = lam[c];
    if (bad_slice) *bad_slice = -1;
    for (j = 0; j < n_slices; ++j) {
        long long cell[2];
        double w[2];
        int bad = 0;
        for (c = 0; c < d; ++c)
            if (!isfinite(lam[c])) bad = 1;
        if (bad) {
            if (bad_slice) *bad_slice = (int)j;
            if (n_out_of_grid) *n_out_of_grid = oog;
            return ORC_NONFINITE;
        }
        for (a = 0; a < d; ++a) {
            oog += orc_locate(g->lo[a], g->hi[a], g->n[a], lam[a], &cell[a], &w[a]);
            if (cells) cells[j * d + a] = cell[a];
            if (weights) weights[j * d + a] = w[a];
        }
        if (interp == ORC_I_LINEAR)
            next[0] = interp_linear(src, j, cell[0], w[0], &bad);
        else if (interp == ORC_I_HERMITE)
            next[0] = interp_hermite(src, j, cell[0], w[0], g->n[0], &bad);
        else if (interp == ORC_I_HERMITE_SLOPES)
            next[0] = interp_hermite_slopes(src, j, cell[0], w[0],
                                            (g->hi[0] - g->lo[0]) / (double)(g->n[0] - 1), &bad);
        else
            interp_bilinear(src, j, cell[0], w[0], cell[1], w[1], g->n[1], next, &bad);
        if (bad) {
            if (bad_slice) *bad_slice = (int)j;
            if (n_out_of_grid) *n_out_of_grid = oog;
            return ORC_NONFINITE;
        }
        for (c = 0; c < d; ++c) lam[c] = next[c];
        if (boundary)
            for (c = 0; c < d; ++c) boundary[(j + 1) * d + c] = lam[c];
    }
    if (n_out_of_grid) *n_out_of_grid = oog;
    return ORC_OK;
}

int orc_compose_tables(const orc_grid *g, int interp, int n_slices, const double *tab,
                       const double *y0, double *boundary, long long *cells,
                       double *weights, long long *n_out_of_grid, int *bad_slice) {
    entry_source src = {0};
    if (!valid_grid(g) || n_slices < 1 || !interp_fits(g, interp)) return ORC_BAD_ARG;
    src.tab = tab;
    src.M = grid_size(g);
    src.n_slices = n_slices;
    return compose(&src, g, interp, n_slices, y0, boundary, cells, weights,
                   n_out_of_grid, bad_slice);
}

int orc_method_lazy(int rhs, const double *p, int scheme, double t0, double T,
                    int n_slices, const orc_grid *g, int steps_per_slice, int interp,
                    const double *y0, double *boundary, long long *n_out_of_grid,
                    int *bad_slice) {
    entry_source src = {0};
    if (!check_method_args(rhs, scheme, n_slices, g, steps_per_slice) ||
        !interp_fits(g, interp))
        return ORC_BAD_ARG;
    src.tab = NULL;
    src.M = grid_size(g);
    src.n_slices = n_slices;
    src.rhs = rhs;
    src.scheme = scheme;
    src.steps = steps_per_slice;
    src.p = p;
    src.t0 = t0;
    src.L = slice_length(t0, T, n_slices);
    src.h = src.L / (double)steps_per_slice;
    src.g = g;
    src.slopes = interp == ORC_I_HERMITE_SLOPES;
    src.memo_j = -1;
    src.memo_k = -1;
    return compose(&src, g, interp, n_slices, y0, boundary, NULL, NULL, n_out_of_grid,
                   bad_slice);
}

/* ---------------------------------------------------------------------------
 * Paper mode: y' = y^2, backward Euler, Chebyshev-Lagrange interpolation.
 * ------------------------------------------------------------------------- */

/* One backward Euler step z = y + dt z^2.  Either one Newton step on
 * F(z) = z - y - dt z^2 from z = y, or the root of the quadratic that tends to
 * y as dt -> 0. */
static double be_step_square(double y, double dt, int exact) {
    if (exact) return (1.0 - sqrt(1.0 - 4.0 * dt * y)) / (2.0 * dt);
    return y + dt * y * y / (1.0 - 2.0 * dt * y);
}

/* Backward Euler over an interval of length L with nominal step dt. */
static double be_interval(double y, double L, double dt, int exact, int equal_substeps) {
    long long n, s;
    if (equal_substeps) {
        double step;
        n = (long long)ceil(L / dt - 1e-9);
        if (n < 1) n = 1;
        step = L / (double)n;
        for (s = 0; s < n; ++s) y = be_step_square(y, step, exact);
        return y;
    } else {
        double rem;
        n = (long long)floor(L / dt + 1e-9);
        rem = L - (double)n * dt;
        for (s = 0; s < n; ++s) y = be_step_square(y, dt, exact);
        if (rem > 1e-12 * L) y = be_step_square(y, rem, exact);
        return y;
    }
}

/* The M Chebyshev extrema of [a, b], k = 0..M-1. */
static double cheb_node(double a, double b, int M, int k) {
    const double pi = 3.14159265358979323846;
    return (a + b) / 2.0 + (b - a) / 2.0 * cos((double)k * pi / (double)(M - 1));
}

/* Lagrange interpolation polynomial through (x_k, v_k), evaluated at x. */
static double lagrange(const double *xs, const double *vs, int M, double x) {
    double s = 0.0;
    int k, m;
    for (k = 0; k < M; ++k) {
        double term = vs[k];
        for (m = 0; m < M; ++m)
            if (m != k) term *= (x - xs[m]) / (xs[k] - xs[m]);
        s += term;
    }
    return s;
}

int orc_paper_nodes(int M, double a, double b, double *xs) {
    int k;
    if (M < 2 || !(b > a)) return ORC_BAD_ARG;
    for (k = 0; k < M; ++k) xs[k] = cheb_node(a, b, M, k);
    return ORC_OK;
}

/* Computation phase of paper mode: tab[j * M + k] = backward Euler over slice j
 * (length T / N) from the node xi_k. */
int orc_paper_tables(double T, int n_slices, int M, double a, double b, double dt,
                     int be_exact, int equal_substeps, double *tab) {
    double L, xs[64];
    int j, k;
    if (n_slices < 1 || M < 2 || M > 64 || !(b > a) || !(dt > 0.0)) return ORC_BAD_ARG;
    L = T / (double)n_slices;
    orc_paper_nodes(M, a, b, xs);
    for (j = 0; j < n_slices; ++j)
        for (k = 0; k < M; ++k)
            tab[(long long)j * M + k] = be_interval(xs[k], L, dt, be_exact, equal_substeps);
    return ORC_OK;
}

/* Communication phase of paper mode over given tables: lambda_0 = y0,
 * lambda_{j+1} = Lagrange interpolant of row j at lambda_j.  Lookups at points
 * outside [a, b] are counted; a non-finite lambda_j or table value read stops
 * the chain with ORC_NONFINITE and *bad_slice = j. */
int orc_paper_compose(int n_slices, int M, double a, double b, const double *tab, double y0,
                      double *boundary, long long *n_out_of_grid, int *bad_slice) {
    double xs[64], lam = y0;
    long long oog = 0;
    int j, k;
    if (n_slices < 1 || M < 2 || M > 64 || !(b > a)) return ORC_BAD_ARG;
    orc_paper_nodes(M, a, b, xs);
    if (boundary) boundary[0] = lam;
    if (bad_slice) *bad_slice = -1;
    for (j = 0; j < n_slices; ++j) {
        const double *row = tab + (long long)j * M;
        int bad = !isfinite(lam);
        for (k = 0; k < M; ++k)
            if (!isfinite(row[k])) bad = 1;
        if (bad) {
            if (bad_slice) *bad_slice = j;
            if (n_out_of_grid) *n_out_of_grid = oog;
            return ORC_NONFINITE;
        }
        if (lam < a || lam > b) ++oog;
        lam = lagrange(xs, row, M, lam);
        if (boundary) boundary[j + 1] = lam;
    }
    if (n_out_of_grid) *n_out_of_grid = oog;
    return ORC_OK;
}

int orc_paper_method(double T, int n_slices, int M, double a, double b, double dt,
                     double y0, int be_exact, int equal_substeps, double *yT) {
    double *tab, *boundary;
    int rc;
    if (n_slices < 1 || M < 2 || M > 64 || !(b > a) || !(dt > 0.0)) return ORC_BAD_ARG;
    tab = (double *)malloc(sizeof(double) * (size_t)n_slices * (size_t)M);
    boundary = (double *)malloc(sizeof(double) * ((size_t)n_slices + 1));
    if (!tab || !boundary) {
        free(tab);
        free(boundary);
        return ORC_BAD_ARG;
    }
    orc_paper_tables(T, n_slices, M, a, b, dt, be_exact, equal_substeps, tab);
    rc = orc_paper_compose(n_slices, M, a, b, tab, y0, boundary, NULL, NULL);
    *yT = rc == ORC_OK ? boundary[n_slices] : NAN;
    free(tab);
    free(boundary);
    return rc == ORC_NONFINITE ? ORC_OK : rc;
}

int orc_paper_serial(double T, double dt, double y0, int be_exact, int equal_substeps,
                     double *yT) {
    if (!(dt > 0.0)) return ORC_BAD_ARG;
    *yT = be_interval(y0, T, dt, be_exact, equal_substeps);
    return ORC_OK;
}
