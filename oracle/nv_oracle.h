/*
 * Plain serial CPU oracle for Nievergelt's parallel-in-time method
 * (A. T. Barker, "A minimal communication approach to parallel time
 * integration", arXiv:1304.6514).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header,
 * constant or helper with the GPU library; both are written from the paper and
 * from the written interpolation/lookup rules independently.
 *
 * Everything is IEEE binary64, one rounding per operation (compiled with
 * -ffp-contract=off; x86-64 without -mfma has no fused multiply-add anyway).
 *
 * Problem codes used by this oracle (its own numbering):
 *   ORC_LIN   y' = p0 * y                 (dim 1)
 *   ORC_LOG   y' = y (1 - y)              (dim 1)
 *   ORC_FCUB  y' = sin(3 t) - y^3         (dim 1)
 *   ORC_VDP   y1' = y2, y2' = p0 (1 - y1^2) y2 - y1   (dim 2; p0 = mu)
 *   ORC_SQR   y' = y^2                    (dim 1; the model problem of sec. 3)
 * Schemes: ORC_RK4 (classical fourth-order Runge-Kutta), ORC_EULER (forward
 * Euler, the scheme of Nievergelt's own analysis, sec. 5).
 * Interpolation: ORC_I_LINEAR, ORC_I_HERMITE (cubic Hermite, slopes by finite
 * differences of the table), ORC_I_BILINEAR (2-D tensor grid),
 * ORC_I_HERMITE_SLOPES (cubic Hermite with the slopes of a slope table: the
 * derivative of each entry with respect to its grid point).
 */
#ifndef NV_ORACLE_H
#define NV_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_LIN = 10, ORC_LOG = 11, ORC_FCUB = 12, ORC_VDP = 13, ORC_SQR = 14 };
enum { ORC_RK4 = 1, ORC_EULER = 2 };
enum { ORC_I_LINEAR = 1, ORC_I_HERMITE = 2, ORC_I_BILINEAR = 3, ORC_I_HERMITE_SLOPES = 4 };
enum { ORC_OK = 0, ORC_BAD_ARG = 1, ORC_NONFINITE = 2 };

/* A uniform grid of the initial value space, endpoints included:
 * axis a has n[a] points lo[a] + k (hi[a]-lo[a])/(n[a]-1), k = 0..n[a]-1.
 * A 2-D grid is flattened axis-0 major: k = k0 * n[1] + k1. */
typedef struct {
    int dim;
    int n[2];
    double lo[2];
    double hi[2];
} orc_grid;

int orc_rhs_dim(int rhs);

/* Integrate y (in place) over nsteps steps of size h.  Step s takes the
 * stage times ta = t_base + s h, tb = ta + h/2, tc = t_base + (s+1) h. */
int orc_integrate(int rhs, const double *p, int scheme, double t_base, double h,
                  long long nsteps, double *y);

/* The same for a one-dimensional problem, with v (in place) the derivative of
 * y with respect to its initial value, carried through every stage of every
 * step by the chain rule (the derivative of the discrete map). */
int orc_integrate_tangent(int rhs, const double *p, int scheme, double t_base, double h,
                          long long nsteps, double *y, double *v);

/* O1, serial truth: the whole interval [t0, T] from y0 in n_slices *
 * steps_per_slice steps of h = ((T - t0) / n_slices) / steps_per_slice. */
int orc_serial(int rhs, const double *p, int scheme, double t0, double T,
               int n_slices, int steps_per_slice, const double *y0, double *yT);

/* Serial run with nsteps equal steps of (T - t0) / nsteps. */
int orc_serial_steps(int rhs, const double *p, int scheme, double t0, double T,
                     long long nsteps, const double *y0, double *yT);

/* Grid point k (flat index) into xi[dim]. */
int orc_grid_point(const orc_grid *g, long long k, double *xi);

/* O2 computation phase, full tables: tab[(c * N + j) * Mtot + k] = component c
 * of the state at T_{j+1} reached from grid point k at T_j. */
int orc_build_tables(int rhs, const double *p, int scheme, double t0, double T,
                     int n_slices, const orc_grid *g, int steps_per_slice,
                     double *tab);

/* The computation phase with slopes (one-dimensional problems): tab[j * Mtot
 * + k] as orc_build_tables, tab[(N + j) * Mtot + k] the derivative of that
 * entry with respect to grid point k (orc_integrate_tangent from slope 1).
 * This two-component layout is what ORC_I_HERMITE_SLOPES composes. */
int orc_build_tables_slopes(int rhs, const double *p, int scheme, double t0, double T,
                            int n_slices, const orc_grid *g, int steps_per_slice,
                            double *tab);

/* The same entries for a list of (slice, grid point) pairs:
 * out[c * count + q] for pair q. */
int orc_table_entries(int rhs, const double *p, int scheme, double t0, double T,
                      int n_slices, const orc_grid *g, int steps_per_slice,
                      long long count, const long long *slice,
                      const long long *point, double *out);

/* Values and slopes for a list of pairs (one-dimensional problems):
 * out[q] the value, out[count + q] the slope of pair q. */
int orc_table_entries_slopes(int rhs, const double *p, int scheme, double t0, double T,
                             int n_slices, const orc_grid *g, int steps_per_slice,
                             long long count, const long long *slice,
                             const long long *point, double *out);

/* Lookup on one axis: cell index and local coordinate of x.
 * Returns 1 when x lies outside [lo, hi], else 0. */
int orc_locate(double lo, double hi, int n, double x, long long *cell, double *w);

/* O2 communication phase over given tables (same layout as orc_build_tables;
 * for ORC_I_HERMITE_SLOPES that of orc_build_tables_slopes).
 *   boundary[(j) * dim + c], j = 0..N : the states lambda_j
 *   cells[j * dim + a], weights[j * dim + a], j = 0..N-1 : lookup of lambda_j
 *   (either may be NULL).  *n_out_of_grid counts lookups outside the grid.
 * Returns ORC_NONFINITE with *bad_slice set when lambda_j or a table entry the
 * lookup touches is not finite. */
int orc_compose_tables(const orc_grid *g, int interp, int n_slices,
                       const double *tab, const double *y0, double *boundary,
                       long long *cells, double *weights,
                       long long *n_out_of_grid, int *bad_slice);

/* O2 with entries integrated on demand: only the entries the lookups touch. */
int orc_method_lazy(int rhs, const double *p, int scheme, double t0, double T,
                    int n_slices, const orc_grid *g, int steps_per_slice,
                    int interp, const double *y0, double *boundary,
                    long long *n_out_of_grid, int *bad_slice);

/* Paper mode (sec. 3, Tables 1 and 2): y' = y^2 on [0, T], backward Euler,
 * Lagrange interpolation on the M Chebyshev extrema of [a, b].
 * be_exact = 0: each implicit step solved by one Newton step from y_n;
 * be_exact = 1: the exact root of the step's quadratic.
 * equal_substeps = 0: steps of dt plus one shorter final step per slice;
 * equal_substeps = 1: ceil(L / dt) equal steps per slice.
 * Returns lambda_N in *yT. */
int orc_paper_method(double T, int n_slices, int M, double a, double b,
                     double dt, double y0, int be_exact, int equal_substeps,
                     double *yT);
/* The two phases of paper mode separately.  Nodes: the M Chebyshev extrema of
 * [a, b], xs[k] = (a+b)/2 + (b-a)/2 cos(k pi/(M-1)), 2 <= M <= 64.  Tables:
 * tab[j * M + k], slice j, node k.  Compose: boundary[0..N], Lagrange
 * interpolation of row j at lambda_j (points outside [a, b] are counted). */
int orc_paper_nodes(int M, double a, double b, double *xs);
int orc_paper_tables(double T, int n_slices, int M, double a, double b, double dt,
                     int be_exact, int equal_substeps, double *tab);
int orc_paper_compose(int n_slices, int M, double a, double b, const double *tab, double y0,
                      double *boundary, long long *n_out_of_grid, int *bad_slice);
/* Plain backward Euler over [0, T] (no slicing, no interpolation). */
int orc_paper_serial(double T, double dt, double y0, int be_exact,
                     int equal_substeps, double *yT);

#ifdef __cplusplus
}
#endif
#endif
