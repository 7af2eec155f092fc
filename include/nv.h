/*
 * nv.h — C ABI of the MI355X (gfx950) propagator-build library for
 * Nievergelt's parallel-in-time method, as framed in A. T. Barker,
 * "A minimal communication approach to parallel time integration",
 * arXiv:1304.6514.
 *
 * The method (sec. 3, pseudocode figure): cut [t0, T] into N slices; on every
 * slice, solve the initial value problem from every point of a sample of the
 * initial value space (computation phase, embarrassingly parallel); then, from
 * the true y0, obtain the slice-boundary states one after the other by
 * evaluating each slice's tabulated initial-to-final map at the previous
 * boundary state (communication phase).
 *
 *   nv_build_propagators  — computation phase: writes the map tables.
 *   nv_compose            — communication phase: y(T) and the boundary states.
 *
 * Conventions
 *   - Every call returns an nv_status; nothing aborts.  On failure,
 *     nv_last_error() returns a message for the calling thread.
 *   - "host" pointers are ordinary CPU memory owned by the caller; "device"
 *     pointers are GPU memory on the context's device.
 *   - A context is not thread-safe: one thread drives it at a time.
 *   - All kernels of a context run on its stream (nv_options.stream).  The
 *     build is asynchronous with respect to the host.  nv_compose and nv_solve
 *     return once the composition has written its outputs into host memory
 *     (the kernel's own exit may still be queued; it is ordered before later
 *     work on the stream); the copy-out calls synchronize the stream.
 *   - Floating-point parameters and time values are IEEE binary64.
 */
#ifndef NV_H
#define NV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NV_API __attribute__((visibility("default")))

typedef enum {
    NV_OK = 0,
    NV_ERR_INVALID_ARG = -1,      /* an argument is out of its documented range */
    NV_ERR_NOT_BUILT = -2,        /* compose/inspect before any successful build */
    NV_ERR_NONFINITE = -3,        /* the composition met a non-finite value */
    NV_ERR_OOM = -4,              /* a device (or host) allocation failed */
    NV_ERR_HIP = -5,              /* a HIP runtime call failed */
    NV_ERR_UNSUPPORTED = -6,      /* a combination this library does not build */
    NV_ERR_BUFFER_TOO_SMALL = -7  /* caller-provided memory is too small */
} nv_status;

/* Right-hand sides f(t, y).  params[] holds the listed parameters. */
typedef enum {
    NV_RHS_LINEAR = 0,        /* y' = p0 y                           dim 1, 1 param */
    NV_RHS_LOGISTIC = 1,      /* y' = y (1 - y)                      dim 1          */
    NV_RHS_FORCED_CUBIC = 2,  /* y' = sin(3 t) - y^3                 dim 1          */
    NV_RHS_VDP = 3,           /* y1' = y2, y2' = p0 (1 - y1^2) y2 - y1   dim 2, p0 = mu
                                 (mu = 0: harmonic oscillator)                      */
    NV_RHS_SQUARE = 4         /* y' = y^2, the model problem of sec. 3   dim 1      */
} nv_rhs_id;

/* Time-stepping scheme of the computation phase.  Forward Euler is the scheme
 * of the error analysis of sec. 5; classical RK4 is the default; backward
 * Euler is the scheme of every experiment of the paper (sec. 3, Table 1;
 * sec. 4), each implicit step solved by one Newton step from the current value
 * (y_{n+1} = y_n + h f(y_n) / (1 - h f'(y_n))), 1-D right-hand sides only. */
typedef enum { NV_SCHEME_RK4 = 0, NV_SCHEME_EULER = 1, NV_SCHEME_BACKWARD_EULER = 2 } nv_scheme;

/* Arithmetic of the table build.  The composition is always FP64. */
typedef enum { NV_FP64 = 0, NV_FP32 = 1 } nv_precision;

/* Interpolation of the tabulated slice maps (the "approximating function" of
 * the pseudocode):
 *   LINEAR     1-D piecewise linear (Nievergelt's own choice, sec. 5)
 *   HERMITE    1-D cubic Hermite; node slopes from the table by finite
 *              differences (centred inside, one-sided second order at the ends)
 *   BILINEAR   2-D tensor-grid bilinear
 *   CHEBYSHEV  1-D Lagrange interpolation on the n Chebyshev extrema of
 *              [lo, hi], xi_k = (lo+hi)/2 + (hi-lo)/2 cos(k pi/(n-1)),
 *              k = 0..n-1 (sec. 3, Table 1), 2 <= n <= 64; the nodes REPLACE
 *              the uniform grid.  phi(x) = sum_k t[k] prod_{m != k}
 *              ((x - xi_m) / (xi_k - xi_m)), k and m ascending, in FP64.
 *   HERMITE_SLOPES  1-D cubic Hermite with stored slopes: the build also
 *              integrates, for every trajectory, the derivative of its state
 *              with respect to its grid point (the scheme applied to the
 *              variational equation v' = df/dy v, v = 1 at the grid point:
 *              exactly the derivative of the scheme's own map) and stores it
 *              as a second table, component 1.  Order 4 in the grid spacing
 *              instead of 3; twice the table memory and about twice the
 *              build's arithmetic.  RK4 or forward Euler, 1-D right-hand
 *              sides, n >= 2.  With d = (hi - lo)/(n - 1), values a, b and
 *              slopes ma, mb of cell i, the same basis and sum as HERMITE with
 *              da = d * ma, db = d * mb.                                      */
typedef enum {
    NV_INTERP_LINEAR = 0,
    NV_INTERP_HERMITE = 1,
    NV_INTERP_BILINEAR = 2,
    NV_INTERP_CHEBYSHEV = 3,
    NV_INTERP_HERMITE_SLOPES = 4
} nv_interp;

/* Sample Xi_h of the initial value space (sec. 3): a uniform tensor grid with
 * endpoints included.  Axis a has n[a] >= 2 points
 *     xi = lo[a] + k (hi[a] - lo[a]) / (n[a] - 1),   k = 0 .. n[a]-1,
 * (n[0] >= 3 for HERMITE).  dim must equal the right-hand side's dimension.
 * A 2-D point has the flat index k = k0 * n[1] + k1 (axis 0 major). */
typedef struct {
    int dim;
    int n[2];
    double lo[2];
    double hi[2];
    int interp;               /* nv_interp; LINEAR/HERMITE need dim 1, BILINEAR dim 2 */
} nv_ic_grid;

typedef struct {
    int scheme;               /* nv_scheme (default RK4) */
    int precision;            /* nv_precision (default FP64) */
    int compensated;          /* FP32 only, accumulation of the state update:
                                 0 plain (one rounding per step),
                                 1 Kahan-compensated,
                                 2 blocked summation (default: the step increments of a
                                   block of 64 steps are summed apart from the state and
                                   added to it once per block) */
    int traj_per_lane;        /* trajectories per GPU lane: 1, 2 or 4; 0 = chosen by the
                                 library (2 for builds of at least 2^21 trajectories) */
    void *stream;             /* hipStream_t the context launches on; NULL = null stream */
    int solve_chunks;         /* nv_solve: slice chunks the build is cut into so that the
                                 composition of chunk c overlaps the build of chunk c+1;
                                 0 = chosen by the library, 1 = no overlap */
    double dt;                /* 0: steps_per_slice equal steps per slice.  > 0: steps of
                                 dt, floor(L/dt + 1e-9) of them, plus one final step of
                                 the remainder L - floor(..) dt when it exceeds 1e-12 L
                                 (the paper's fixed time step, sec. 3); steps_per_slice is
                                 then ignored.  Autonomous right-hand sides only. */
} nv_options;

/* Result details of a composition. */
typedef struct {
    long long n_out_of_grid;  /* lookups whose point lay outside the grid box; those
                                 are extrapolated from the edge cell, not clamped */
    int bad_slice;            /* first slice whose lookup met a non-finite value, or -1 */
    int n_chunks;             /* slice chunks the composition ran in (1 for nv_compose) */
} nv_compose_info;

typedef struct nv_ctx nv_ctx;

/* Create a context on the current HIP device with default options.
 * *out receives the handle; free it with nv_ctx_destroy. */
NV_API nv_status nv_ctx_create(nv_ctx **out);

/* Free the context and every device buffer the library allocated for it.
 * Caller-provided buffers (nv_set_buffers) are not freed.  NULL is accepted. */
NV_API nv_status nv_ctx_destroy(nv_ctx *ctx);

/* Replace the context's options.  Takes effect at the next build.  Invalid
 * values give NV_ERR_INVALID_ARG and leave the options unchanged. */
NV_API nv_status nv_set_options(nv_ctx *ctx, const nv_options *opt);
NV_API nv_status nv_get_options(const nv_ctx *ctx, nv_options *opt);

/* Device memory a build of this shape needs.
 *   *table_bytes: the map tables, dim x N x (points per slice) values of the
 *                 working precision, 256-byte aligned per component;
 *   *work_bytes:  scratch (per-slice forcing values of non-autonomous
 *                 right-hand sides, one non-finite count per build tile, the
 *                 composition's running status and carried state, the
 *                 Chebyshev nodes).  The boundary states and the final status
 *                 go to pinned, device-mapped host memory that the context
 *                 allocates itself.
 * Pure host arithmetic: no device call. */
NV_API nv_status nv_required_bytes(int rhs_id, int n_slices, const nv_ic_grid *grid,
                                   int steps_per_slice, const nv_options *opt,
                                   size_t *table_bytes, size_t *work_bytes);

/* Hand the context caller-owned device memory (e.g. from PyTorch) for the
 * tables and the scratch.  The library never frees it; it must stay valid
 * until the next nv_set_buffers, or nv_ctx_destroy.  Passing NULL pointers
 * returns to library-owned memory (allocated on demand by the build).  If a
 * build needs more than the given sizes it fails with NV_ERR_BUFFER_TOO_SMALL. */
NV_API nv_status nv_set_buffers(nv_ctx *ctx, void *tables_dev, size_t table_bytes,
                                void *work_dev, size_t work_bytes);

/* Computation phase (sec. 3 pseudocode, "computation phase"; the (Mn/N) tau_F
 * term of the GPU cost model of sec. 4).
 *
 * For every slice j = 0..n_slices-1 and every grid point k, integrate the
 * problem from xi_k at T_j = t0 + j (T - t0)/n_slices over steps_per_slice
 * steps of h = ((T - t0)/n_slices)/steps_per_slice and store the end state in
 * the table: tab[c][j][k] for state component c (see nv_get_table).  Step s of
 * a slice evaluates the right-hand side at T_j + s h, T_j + s h + h/2 and
 * T_j + (s+1) h.
 *
 *   rhs_id          nv_rhs_id
 *   params          host array with the right-hand side's parameters (may be
 *                   NULL when it takes none); must be finite
 *   t0 < T          finite
 *   n_slices        >= 1
 *   grid            host struct, see nv_ic_grid
 *   steps_per_slice >= 1
 *
 * Asynchronous on the context's stream.  Per-slice counts of trajectories that
 * ended non-finite are kept (nv_get_nonfinite_counts).  Errors:
 * NV_ERR_INVALID_ARG, NV_ERR_UNSUPPORTED, NV_ERR_OOM, NV_ERR_BUFFER_TOO_SMALL,
 * NV_ERR_HIP.  A failed build leaves the context unbuilt. */
NV_API nv_status nv_build_propagators(nv_ctx *ctx, int rhs_id, const double *params,
                                      double t0, double T, int n_slices,
                                      const nv_ic_grid *grid, int steps_per_slice);

/* Communication phase (sec. 3 pseudocode, "communication phase"; the N tau_N
 * term of the cost model of sec. 4): lambda_0 = y0 and
 * lambda_{j+1} = phi^j(lambda_j) for j = 0..N-1, each phi^j the interpolant of
 * slice j's table (every slice, the first included), in FP64 on the GPU.
 *
 * Lookup on axis a: inv = (n-1)/(hi-lo), u = (x-lo) inv, cell = floor(u)
 * limited to [0, n-2], w = u - cell, each an IEEE binary64 operation.
 * Interpolants (t = the table row, widened exactly to FP64):
 *   LINEAR    t[i] + w (t[i+1] - t[i])
 *   HERMITE   ((h00 t[i] + h10 d[i]) + h01 t[i+1]) + h11 d[i+1] with
 *             h00 = (2w^3 - 3w^2) + 1, h10 = (w^3 - 2w^2) + w, h01 = 3w^2 - 2w^3,
 *             h11 = w^3 - w^2, d[i] = (t[i+1] - t[i-1])/2 inside,
 *             d[0] = ((4t[1] - 3t[0]) - t[2])/2,
 *             d[n-1] = ((3t[n-1] - 4t[n-2]) + t[n-3])/2
 *   BILINEAR  per component: r0 = t00 + w1 (t01 - t00), r1 = t10 + w1 (t11 - t10),
 *             r0 + w0 (r1 - r0), t_ab the corner (cell0 + a, cell1 + b)
 *
 *   y0        host array, dim values (the true initial value)
 *   yT        host array, dim values: lambda_N = the method's y(T)
 *   boundary  host array of (n_slices + 1) * dim values, lambda_j at
 *             boundary[j * dim + c], or NULL
 *   info      host struct, or NULL
 *
 * Synchronous.  NV_ERR_NOT_BUILT before a build; NV_ERR_NONFINITE when
 * lambda_j or a table entry the lookup reads is not finite (info->bad_slice =
 * j; boundary holds lambda_0..lambda_j).  Lookups outside the grid box
 * extrapolate from the edge cell and are counted, not treated as errors. */
NV_API nv_status nv_compose(nv_ctx *ctx, const double *y0, double *yT, double *boundary,
                            nv_compose_info *info);

/* Both phases in one call, pipelined as in the paper's scheduling figure for
 * the method (sec. 3): a processor interpolates as soon as its own map is
 * built and the previous boundary value has arrived, while later slices are
 * still being built.  The slices are cut into contiguous chunks; the build of
 * each chunk is launched on the context's stream, and the composition of
 * chunk c runs on a second, library-owned stream as soon as chunk c's tables
 * are complete, concurrently with the build of the chunks after it.
 *
 * Arguments and results are those of nv_build_propagators followed by
 * nv_compose, and so are the tables and the boundary states, bit for bit.
 * The context is built afterwards (nv_compose may be called again with other
 * initial values).  Synchronous.  Errors: those of both calls. */
NV_API nv_status nv_solve(nv_ctx *ctx, int rhs_id, const double *params, double t0,
                          double T, int n_slices, const nv_ic_grid *grid,
                          int steps_per_slice, const double *y0, double *yT,
                          double *boundary, nv_compose_info *info);

/* Copy component c's table of the last build to host memory: n_slices rows of
 * (points per slice) values in the build's precision (double or float),
 * row j at offset j * points.  bytes must be at least that size.  Components:
 * one per state component; with HERMITE_SLOPES, 0 the values and 1 the slopes. */
NV_API nv_status nv_get_table(nv_ctx *ctx, int component, void *host_dst, size_t bytes);

/* Device address of component c's table (same layout as nv_get_table). */
NV_API nv_status nv_table_device_ptr(nv_ctx *ctx, int component, void **dev_ptr);

/* Copy the per-slice counts of trajectories that ended non-finite (n_slices
 * uint32 values) to host memory; n is the capacity of host_counts.  Waits on
 * the context's stream.  Errors: NV_ERR_INVALID_ARG (NULL argument),
 * NV_ERR_NOT_BUILT, NV_ERR_BUFFER_TOO_SMALL (n < n_slices), NV_ERR_OOM (no
 * host memory to gather the per-tile counts), NV_ERR_HIP. */
NV_API nv_status nv_get_nonfinite_counts(nv_ctx *ctx, uint32_t *host_counts, int n);

/* The lookup of nv_compose applied to count device-resident queries x_dev:
 * cell_dev[q] (int64) and w_dev[q] (double); out_dev[q] = 1 when outside the
 * grid box.  Runs on the context's stream and synchronizes.  For checking the
 * lookup bit for bit. */
NV_API nv_status nv_locate(nv_ctx *ctx, double lo, double hi, int n, const double *x_dev,
                           long long count, long long *cell_dev, double *w_dev,
                           int32_t *out_dev);

/* Kernel timing with HIP events on the context's streams.  When enabled, the
 * last build's integration kernel(s) and the last composition are bracketed by
 * events; nv_last_timing waits for them and returns milliseconds (-1 when not
 * measured).  After nv_solve, build_ms spans all build launches and
 * compose_ms the part of the composition that ran after the last build launch
 * had finished. */
NV_API nv_status nv_set_timing(nv_ctx *ctx, int enable);
NV_API nv_status nv_last_timing(nv_ctx *ctx, float *build_ms, float *compose_ms);

/* ------------------------------------------------------------------------
 * Batches: many independent problems of uneven shape in one persistent,
 * graph-captured launch.
 *
 * Every problem is the method of sec. 3 on its own (own right-hand side,
 * interval, slices, grid and steps); the batch builds all their tables in ONE
 * launch of a persistent kernel whose workgroups take work items (a tile of
 * 256 x P grid points of one slice of one problem) from a shared counter,
 * longest items first, then composes every problem in one launch (one wave per
 * problem).  The reset, the two launches and the copy of the results to host
 * memory are captured once into a HIP graph and replayed by nv_batch_run.
 * Results equal those of nv_build_propagators + nv_compose on each problem
 * alone, bit for bit (same options).  Batches take the autonomous right-hand
 * sides (LINEAR, LOGISTIC, VDP, SQUARE); FORCED_CUBIC gives NV_ERR_UNSUPPORTED.
 * ------------------------------------------------------------------------ */

/* One problem of a batch: the arguments of nv_build_propagators plus y0. */
typedef struct {
    int rhs_id;
    double params[2];
    double t0, T;
    int n_slices;
    nv_ic_grid grid;
    int steps_per_slice;
    double y0[2];
} nv_problem;

/* How the batch's build is scheduled.  traj_per_lane[r] is P for the problems
 * of right-hand side r (1, 2 or 4); workgroups_per_cu sets the persistent
 * grid (256 CUs x this many workgroups of 256 lanes, 1..8); order 0 hands out
 * items longest first, order 1 in problem/slice/tile order. */
typedef struct {
    int traj_per_lane[5];
    int workgroups_per_cu;
    int order;
} nv_batch_schedule;

typedef struct nv_batch nv_batch;

/* Create a batch of count problems (host array, copied).  Precision and FP32
 * accumulation come from ctx's options; the batch owns its device memory, its
 * stream and its graph.  The default schedule is P = 1 for every right-hand
 * side, 8 workgroups per CU, longest items first.  Errors: NV_ERR_INVALID_ARG
 * (with the offending problem's index in the message), NV_ERR_UNSUPPORTED,
 * NV_ERR_OOM, NV_ERR_HIP. */
NV_API nv_status nv_batch_create(nv_ctx *ctx, const nv_problem *problems, int count,
                                 nv_batch **out);
NV_API nv_status nv_batch_destroy(nv_batch *batch);

/* Replace / read the schedule (a new schedule is captured at the next run). */
NV_API nv_status nv_batch_set_schedule(nv_batch *batch, const nv_batch_schedule *sched);
NV_API nv_status nv_batch_get_schedule(const nv_batch *batch, nv_batch_schedule *sched);

/* Project autotuner: times candidate schedules on this batch with HIP events
 * (per right-hand side, P in {1, 2, 4} on that right-hand side's items alone;
 * then workgroups per CU in {4, 8} and both item orders on the whole batch),
 * keeps the fastest, sets it and returns it in *chosen (may be NULL).  reps
 * timed launches per candidate (>= 1). */
NV_API nv_status nv_batch_autotune(nv_batch *batch, int reps, nv_batch_schedule *chosen);

/* Run the whole batch (replays the captured graph) and wait.  yT: host array
 * of count x 2 values (problem i's final state at yT[2i], yT[2i+1]; the second
 * is 0 for 1-D problems); info: host array of count entries, or NULL.
 * Returns NV_ERR_NONFINITE if any problem's composition met a non-finite value
 * (see its info entry), else NV_OK. */
NV_API nv_status nv_batch_run(nv_batch *batch, double *yT, nv_compose_info *info);

/* Milliseconds of the last nv_batch_run (HIP events around the graph launch),
 * and the trajectory-steps one run integrates. */
NV_API nv_status nv_batch_last_timing(nv_batch *batch, float *run_ms, long long *traj_steps);

/* Copy problem p's component c table (layout of nv_get_table) or its boundary
 * states ((n_slices + 1) x dim doubles) of the last run to host memory;
 * NV_ERR_NOT_BUILT before the first nv_batch_run. */
NV_API nv_status nv_batch_get_table(nv_batch *batch, int problem, int component,
                                    void *host_dst, size_t bytes);
NV_API nv_status nv_batch_get_boundary(nv_batch *batch, int problem, double *host_dst,
                                       size_t count);

/* ------------------------------------------------------------------------
 * nv_solve for callers that cannot allocate: code under HIP graph capture,
 * serving loops that must not call hipMalloc, harnesses that forbid it.
 *
 * The build and the composition of nv_solve (same kernels, same options, one
 * slice chunk: no overlap) with no context and no allocation of any kind:
 * the caller passes every input and output, and the scratch (forcing rows,
 * per-tile non-finite counts, the composition's running status and carried
 * state) is a library-owned static array of NV_STATIC_SCRATCH_BYTES on each
 * device, held from the library's first use on that device until the process
 * ends.  The scratch a build needs is nv_required_bytes' *work_bytes; builds
 * that need more are rejected with NV_ERR_BUFFER_TOO_SMALL (the forced cubic
 * in FP32 fits up to (2 steps + 1) x slices x 4 bytes of forcing rows, about
 * 63 MiB with its per-tile counts at 4096 slices x 2000 steps x 4096 points).
 *
 *   opt           host; scheme, precision, accumulation, trajectories per lane,
 *                 dt and the stream to launch on (solve_chunks is ignored)
 *   tables_dev    device, 256-byte aligned, table_bytes >= nv_required_bytes'
 *                 *table_bytes; receives the tables (layout of nv_get_table,
 *                 component c at c x the 256-byte-aligned component size)
 *   y0            host, dim values (read before the call returns)
 *   boundary_dev  device, (n_slices + 1) x dim doubles, 8-byte aligned:
 *                 lambda_j at [j * dim + c]; lambda_N is the method's y(T)
 *   status_dev    device, 8-byte aligned: n_out_of_grid, bad_slice (-1 when
 *                 none; then boundary_dev holds lambda_0..lambda_bad_slice) and
 *                 done = 1, written by the composition when it ends
 *
 * Asynchronous: returns once the launches are queued on opt->stream (no
 * synchronization, no memset, no copy); read the outputs after the stream.
 * Every call on one device uses that device's one scratch, which keeps the
 * last call's contents (nothing in it needs to start at zero): calls that
 * may overlap on one device race and must be ordered by the caller (e.g. one
 * stream).  Chebyshev (paper-mode) grids give NV_ERR_UNSUPPORTED (their nodes
 * come from host memory).  Errors: those of nv_solve, found before anything is
 * launched, and NV_ERR_HIP. */
#define NV_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

typedef struct {
    long long n_out_of_grid;
    int bad_slice;
    int done;
} nv_solve_status;

NV_API nv_status nv_solve_static(int rhs_id, const double *params, double t0, double T,
                                 int n_slices, const nv_ic_grid *grid, int steps_per_slice,
                                 const nv_options *opt, void *tables_dev, size_t table_bytes,
                                 const double *y0, double *boundary_dev,
                                 nv_solve_status *status_dev);

/* Message of the last failure on the calling thread ("" if none). */
NV_API const char *nv_last_error(void);

/* Name of a status code. */
NV_API const char *nv_status_string(int status);

#ifdef __cplusplus
}
#endif
#endif /* NV_H */
