// C ABI of libnv (declared in include/nv.h): argument checking, device-buffer
// planning and ownership, kernel launches on the context's stream, timing and
// error reporting.  No arithmetic of the method happens here apart from the
// FP64 scalars of the slice partition and grid (T_j, h, grid spacing, the
// lookup's (n-1)/(hi-lo)), which are computed once on the host.
#include "nv.h"
#include "nv_internal.h"

#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

namespace {
// a fixed buffer, so that reporting an error allocates nothing
thread_local char g_last_error[512];
}  // namespace

nv_status nv::fail(nv_status s, const char *fmt, ...) {
    // formatted apart first: an argument may be the current message itself
    char buf[sizeof g_last_error];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::memcpy(g_last_error, buf, sizeof buf);
    return s;
}

namespace {
using nv::fail;

#define NV_HIP(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(NV_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

constexpr size_t kAlign = 256;
constexpr int kMaxChunks = 64;
constexpr int kMaxChebyshev = 64;
// a build of a right-hand side with forcing forms each slice's forcing row in
// its workgroups' LDS (no forcing launch) when it has at most this many
// workgroups and a row fits in this many bytes
constexpr long long kLocalForcingBlocks = 2048;
constexpr size_t kLocalForcingBytes = 16384;
// automatic chunking of nv_solve: about this many workgroups per build launch
// (half a round of 256 CUs x 8 resident workgroups; consecutive chunks overlap)
constexpr long long kBlocksPerChunk = 1024;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int rhs_dim(int rhs) {
    switch (rhs) {
    case NV_RHS_LINEAR: case NV_RHS_LOGISTIC: case NV_RHS_FORCED_CUBIC: case NV_RHS_SQUARE:
        return 1;
    case NV_RHS_VDP:
        return 2;
    default:
        return 0;
    }
}
int rhs_nparams(int rhs) { return (rhs == NV_RHS_LINEAR || rhs == NV_RHS_VDP) ? 1 : 0; }
bool rhs_forced(int rhs) { return rhs == NV_RHS_FORCED_CUBIC; }

nv_options default_options() {
    nv_options o;
    o.scheme = NV_SCHEME_RK4;
    o.precision = NV_FP64;
    o.compensated = 2;
    o.traj_per_lane = 0;
    o.stream = nullptr;
    o.solve_chunks = 0;
    o.dt = 0.0;
    return o;
}

// Trajectories per lane: the caller's choice, else 2 when the build still
// fills the chip twice over with 2 per lane (256 CUs x 8 resident workgroups
// of 256 lanes, two rounds), else 1.
int effective_p(const nv_options &o, long long trajectories) {
    if (o.traj_per_lane != 0) return o.traj_per_lane;
    const long long two_rounds_at_p2 = 2LL * 256 * 8 * nv::kBuildBlock * 2;
    return trajectories >= two_rounds_at_p2 ? 2 : 1;
}

nv_status check_options(const nv_options *o) {
    if (!o) return fail(NV_ERR_INVALID_ARG, "options pointer is NULL");
    if (o->scheme != NV_SCHEME_RK4 && o->scheme != NV_SCHEME_EULER &&
        o->scheme != NV_SCHEME_BACKWARD_EULER)
        return fail(NV_ERR_INVALID_ARG, "unknown scheme %d", o->scheme);
    if (!std::isfinite(o->dt) || o->dt < 0.0)
        return fail(NV_ERR_INVALID_ARG, "dt must be finite and >= 0");
    if (o->precision != NV_FP64 && o->precision != NV_FP32)
        return fail(NV_ERR_INVALID_ARG, "unknown precision %d", o->precision);
    if (o->compensated < 0 || o->compensated > 2)
        return fail(NV_ERR_INVALID_ARG, "compensated must be 0, 1 or 2");
    if (o->traj_per_lane != 0 && o->traj_per_lane != 1 && o->traj_per_lane != 2 &&
        o->traj_per_lane != 4)
        return fail(NV_ERR_INVALID_ARG, "traj_per_lane must be 0, 1, 2 or 4");
    if (o->solve_chunks < 0 || o->solve_chunks > kMaxChunks)
        return fail(NV_ERR_INVALID_ARG, "solve_chunks must be in [0, %d]", kMaxChunks);
    return NV_OK;
}

// Where everything lives for one build shape.
struct Plan {
    int dim = 0;                  // state dimension
    int components = 0;           // tables: one per state component, plus the slopes
    long long M = 0;              // points per slice
    size_t elem = 0;              // bytes per table value
    size_t comp_bytes = 0;        // one component's table, aligned
    size_t table_bytes = 0;
    size_t forcing_off = 0, forcing_bytes = 0;
    size_t nonfinite_off = 0;
    size_t status_off = 0, carry_off = 0;   // device: running status, carried state
    size_t boundary_bytes = 0;     // in the mapped host stage, from offset 0
    size_t stage_status_off = 0;   // the final status, in the mapped host stage
    size_t nodes_off = 0;
    size_t work_bytes = 0;
    int tiles_per_slice = 0;
    long long total_blocks = 0;
    int traj_per_lane = 1;
};

nv_status make_plan(int rhs, int n_slices, const nv_ic_grid *g, int steps,
                    const nv_options &o, Plan *p) {
    if (rhs_dim(rhs) == 0) return fail(NV_ERR_INVALID_ARG, "unknown rhs_id %d", rhs);
    if (!g) return fail(NV_ERR_INVALID_ARG, "ic_grid is NULL");
    if (n_slices < 1) return fail(NV_ERR_INVALID_ARG, "n_slices must be >= 1 (got %d)", n_slices);
    if (o.dt == 0.0 && steps < 1)
        return fail(NV_ERR_INVALID_ARG, "steps_per_slice must be >= 1 (got %d)", steps);
    if (o.dt > 0.0) {
        if (rhs_forced(rhs))
            return fail(NV_ERR_INVALID_ARG, "a fixed step dt needs an autonomous right-hand side");
        steps = 0;                                 // counted per slice from dt
    }
    if (o.scheme == NV_SCHEME_BACKWARD_EULER && rhs_dim(rhs) != 1)
        return fail(NV_ERR_UNSUPPORTED, "backward Euler is built for 1-D right-hand sides");
    if (g->dim != rhs_dim(rhs))
        return fail(NV_ERR_INVALID_ARG, "grid dim %d does not match the rhs dimension %d",
                    g->dim, rhs_dim(rhs));
    long long M = 1;
    for (int a = 0; a < g->dim; ++a) {
        if (g->n[a] < 2) return fail(NV_ERR_INVALID_ARG, "grid axis %d needs n >= 2", a);
        if (!std::isfinite(g->lo[a]) || !std::isfinite(g->hi[a]) || !(g->hi[a] > g->lo[a]))
            return fail(NV_ERR_INVALID_ARG, "grid axis %d needs finite lo < hi", a);
        M *= g->n[a];
    }
    if (M > 0x7fffffffLL)
        return fail(NV_ERR_INVALID_ARG, "grid has %lld points; at most 2^31-1 per slice", M);
    switch (g->interp) {
    case NV_INTERP_LINEAR:
        if (g->dim != 1) return fail(NV_ERR_INVALID_ARG, "LINEAR interpolation needs dim 1");
        break;
    case NV_INTERP_HERMITE:
        if (g->dim != 1) return fail(NV_ERR_INVALID_ARG, "HERMITE interpolation needs dim 1");
        if (g->n[0] < 3) return fail(NV_ERR_INVALID_ARG, "HERMITE interpolation needs n >= 3");
        break;
    case NV_INTERP_BILINEAR:
        if (g->dim != 2) return fail(NV_ERR_INVALID_ARG, "BILINEAR interpolation needs dim 2");
        break;
    case NV_INTERP_HERMITE_SLOPES:
        if (g->dim != 1)
            return fail(NV_ERR_INVALID_ARG, "HERMITE_SLOPES interpolation needs dim 1");
        if (o.scheme == NV_SCHEME_BACKWARD_EULER)
            return fail(NV_ERR_UNSUPPORTED, "slopes are integrated with RK4 or forward Euler");
        break;
    case NV_INTERP_CHEBYSHEV:
        if (g->dim != 1) return fail(NV_ERR_INVALID_ARG, "CHEBYSHEV interpolation needs dim 1");
        if (g->n[0] > kMaxChebyshev)
            return fail(NV_ERR_INVALID_ARG, "CHEBYSHEV interpolation takes at most %d nodes",
                        kMaxChebyshev);
        break;
    default:
        return fail(NV_ERR_INVALID_ARG, "unknown interpolation %d", g->interp);
    }
    const int P = effective_p(o, M * (long long)n_slices);
    const long long per_tile = (long long)nv::kBuildBlock * P;
    const long long tiles = (M + per_tile - 1) / per_tile;
    const long long blocks = tiles * n_slices;
    if (blocks > 0x7fffffffLL)
        return fail(NV_ERR_INVALID_ARG, "build needs %lld workgroups; at most 2^31-1", blocks);

    p->dim = g->dim;
    p->components = g->interp == NV_INTERP_HERMITE_SLOPES ? 2 : g->dim;
    p->M = M;
    p->elem = o.precision == NV_FP64 ? sizeof(double) : sizeof(float);
    p->comp_bytes = align_up(size_t(M) * size_t(n_slices) * p->elem);
    p->table_bytes = p->comp_bytes * size_t(p->components);
    size_t off = 0;
    p->forcing_off = off;
    p->forcing_bytes = rhs_forced(rhs) ? (2 * size_t(steps) + 1) * size_t(n_slices) * p->elem : 0;
    off = align_up(off + p->forcing_bytes);
    // one non-finite count per tile, stored by its workgroup (the host sums a
    // slice's tiles)
    p->nonfinite_off = off;
    off = align_up(off + size_t(n_slices) * size_t(tiles) * sizeof(uint32_t));
    // the running status and the state carried from one range of slices to
    // the next stay in device memory; the boundary states and a copy of the
    // final status go to the context's mapped host memory:
    // [boundary][status at stage_status_off]
    p->status_off = off;
    off = align_up(off + sizeof(nv::ComposeStatus));
    p->carry_off = off;
    off = align_up(off + 2 * sizeof(double));
    p->boundary_bytes = (size_t(n_slices) + 1) * size_t(g->dim) * sizeof(double);
    p->stage_status_off = align_up(p->boundary_bytes);
    p->nodes_off = off;
    off = align_up(off + kMaxChebyshev * sizeof(double));
    p->work_bytes = off;
    p->tiles_per_slice = int(tiles);
    p->total_blocks = blocks;
    p->traj_per_lane = P;
    return NV_OK;
}

}  // namespace

nv_status nv::check_problem(int rhs_id, const double *params, double t0, double T, int n_slices,
                            const nv_ic_grid *grid, int steps_per_slice) {
    Plan p;
    nv_status s = make_plan(rhs_id, n_slices, grid, steps_per_slice, default_options(), &p);
    if (s != NV_OK) return s;
    if (!std::isfinite(t0) || !std::isfinite(T) || !(T > t0))
        return fail(NV_ERR_INVALID_ARG, "need finite t0 < T (got %g, %g)", t0, T);
    if (rhs_nparams(rhs_id) > 0 && (!params || !std::isfinite(params[0])))
        return fail(NV_ERR_INVALID_ARG, "rhs %d needs a finite parameter", rhs_id);
    return NV_OK;
}

struct nv_ctx {
    nv_options opt = default_options();
    // device memory
    void *tables = nullptr;
    size_t tables_cap = 0;
    bool tables_owned = true;
    void *work = nullptr;
    size_t work_cap = 0;
    bool work_owned = true;
    // pinned, device-mapped memory that the composition writes its boundary
    // states and status into (host and device addresses)
    void *host_stage = nullptr;
    void *host_stage_dev = nullptr;
    double nodes_host[kMaxChebyshev] = {};
    // what the scratch's node array holds (uploaded once per grid and buffer)
    const void *nodes_dev = nullptr;
    int nodes_n = 0;
    double nodes_lo = 0.0, nodes_hi = 0.0;
    size_t host_stage_cap = 0;
    // last build
    bool built = false;
    Plan plan;
    int rhs = -1;
    int precision = NV_FP64;
    int n_slices = 0;
    nv_ic_grid grid{};
    // nv_solve: composition stream, second build stream, per-chunk events
    hipStream_t aux = nullptr;
    hipStream_t aux2 = nullptr;
    hipEvent_t chunk_ev[kMaxChunks] = {};
    hipEvent_t ready_ev = nullptr;
    // timing
    bool timing = false;
    bool build_timed = false, compose_timed = false, solve_timed = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

hipStream_t stream_of(const nv_ctx *c) { return static_cast<hipStream_t>(c->opt.stream); }

nv_status ensure_device(void **ptr, size_t *cap, bool owned, size_t need, const char *what) {
    if (!owned) {
        if (*ptr == nullptr && need > 0)
            return fail(NV_ERR_BUFFER_TOO_SMALL, "no %s buffer was given", what);
        if (need > *cap)
            return fail(NV_ERR_BUFFER_TOO_SMALL, "%s buffer holds %zu bytes, build needs %zu",
                        what, *cap, need);
        return NV_OK;
    }
    if (need <= *cap && *ptr) return NV_OK;
    if (*ptr) {
        NV_HIP(hipFree(*ptr));
        *ptr = nullptr;
        *cap = 0;
    }
    hipError_t e = hipMalloc(ptr, need);
    if (e != hipSuccess) {
        *ptr = nullptr;
        return fail(NV_ERR_OOM, "hipMalloc of %zu bytes for %s failed: %s", need, what,
                    hipGetErrorString(e));
    }
    *cap = need;
    return NV_OK;
}

nv_status ensure_host_stage(nv_ctx *c, size_t need) {
    if (need <= c->host_stage_cap && c->host_stage) return NV_OK;
    if (c->host_stage) {
        NV_HIP(hipHostFree(c->host_stage));
        c->host_stage = c->host_stage_dev = nullptr;
        c->host_stage_cap = 0;
    }
    hipError_t e = hipHostMalloc(&c->host_stage, need, hipHostMallocMapped);
    if (e != hipSuccess) {
        c->host_stage = nullptr;
        return fail(NV_ERR_OOM, "hipHostMalloc of %zu bytes failed: %s", need,
                    hipGetErrorString(e));
    }
    e = hipHostGetDevicePointer(&c->host_stage_dev, c->host_stage, 0);
    if (e != hipSuccess) {
        (void)hipHostFree(c->host_stage);
        c->host_stage = c->host_stage_dev = nullptr;
        return fail(NV_ERR_HIP, "hipHostGetDevicePointer failed: %s", hipGetErrorString(e));
    }
    c->host_stage_cap = need;
    return NV_OK;
}

// The timing events only measure: nothing waits on them and no result is read
// through them (the composition hands its states to the host through its own
// system-scope flag), so they are recorded without the system-scope fence,
// whose cache writeback would otherwise sit between the build and the
// composition of every timed solve (about 10 us on a small build).
nv_status ensure_events(nv_ctx *c) {
    for (auto &e : c->ev)
        if (!e) NV_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    return NV_OK;
}

char *work_at(const nv_ctx *c, size_t off) { return static_cast<char *>(c->work) + off; }

// The n Chebyshev extrema of [a, b] (sec. 3, Table 1), one rounding per
// operation: (a+b)/2 + (b-a)/2 cos(k pi/(n-1)), k = 0..n-1.
void chebyshev_nodes(int n, double a, double b, double *xs) {
#pragma clang fp contract(off)
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < n; ++k)
        xs[k] = (a + b) / 2.0 + (b - a) / 2.0 * std::cos(double(k) * pi / double(n - 1));
}


// One build: its configuration and the integration kernel's arguments.
struct PreparedBuild {
    nv::BuildConfig cfg;
    nv::BuildArgs args;
};

// Checks of one build and every argument of its integration kernel but the
// device addresses (place_build): the plan, the slice partition and the grid.
nv_status describe_build(const nv_options &o, int rhs_id, const double *params, double t0,
                         double T, int n_slices, const nv_ic_grid *grid, int steps_per_slice,
                         Plan *pp, PreparedBuild *pb) {
    Plan &p = *pp;
    nv_status s = make_plan(rhs_id, n_slices, grid, steps_per_slice, o, &p);
    if (s != NV_OK) return s;
    if (!std::isfinite(t0) || !std::isfinite(T) || !(T > t0))
        return fail(NV_ERR_INVALID_ARG, "need finite t0 < T (got %g, %g)", t0, T);
    double p0 = 0.0;
    if (rhs_nparams(rhs_id) > 0) {
        if (!params) return fail(NV_ERR_INVALID_ARG, "rhs %d needs a parameter", rhs_id);
        if (!std::isfinite(params[0])) return fail(NV_ERR_INVALID_ARG, "parameter not finite");
        p0 = params[0];
    }
    nv::BuildConfig cfg{rhs_id, o.scheme, o.precision, o.compensated, p.traj_per_lane,
                        grid->interp == NV_INTERP_HERMITE_SLOPES ? 1 : 0};
    if (!nv::build_supported(cfg)) return fail(NV_ERR_UNSUPPORTED, "unsupported configuration");

    // slice partition (sec. 3): L = (T - t0)/N, T_j = t0 + j L; either S equal
    // steps h = L / S, or steps of the fixed dt plus one shorter final step
    const double L = (T - t0) / double(n_slices);
    double h, h_last = 0.0;
    int S = steps_per_slice;
    if (o.dt > 0.0) {
        const double n = std::floor(L / o.dt + 1e-9);
        if (n > 2147483647.0) return fail(NV_ERR_INVALID_ARG, "dt gives too many steps");
        S = int(n);
        h = o.dt;
        const double rem = L - double(S) * o.dt;
        if (rem > 1e-12 * L) h_last = rem;
    } else {
        h = L / double(steps_per_slice);
    }

    nv::BuildArgs &a = pb->args;
    a = nv::BuildArgs{};
    a.lo0 = grid->lo[0];
    a.dxi0 = (grid->hi[0] - grid->lo[0]) / double(grid->n[0] - 1);
    a.lo1 = p.dim == 2 ? grid->lo[1] : 0.0;
    a.dxi1 = p.dim == 2 ? (grid->hi[1] - grid->lo[1]) / double(grid->n[1] - 1) : 0.0;
    a.h = h;
    a.h_last = h_last;
    a.p0 = p0;
    a.nodes = nullptr;
    a.M = p.M;
    a.n1 = p.dim == 2 ? grid->n[1] : 1;
    a.n_slices = n_slices;
    a.slice0 = 0;
    a.steps = S;
    a.tiles_per_slice = p.tiles_per_slice;
    a.total_blocks = int(p.total_blocks);
    a.t0 = t0;
    a.L = L;
    a.local_forcing = rhs_forced(rhs_id) && p.total_blocks <= kLocalForcingBlocks &&
                      (2 * size_t(steps_per_slice) + 1) * p.elem <= kLocalForcingBytes;
    pb->cfg = cfg;
    return NV_OK;
}

// The device addresses of a described build: its tables at `tables`, its
// scratch (laid out by the plan) at `work`.
void place_build(PreparedBuild *pb, const Plan &p, void *tables, char *work) {
    nv::BuildArgs &a = pb->args;
    a.tab0 = tables;
    a.tab1 = p.components == 2 ? static_cast<char *>(tables) + p.comp_bytes : nullptr;
    a.forcing = rhs_forced(pb->cfg.rhs) ? work + p.forcing_off : nullptr;
    a.nonfinite = reinterpret_cast<uint32_t *>(work + p.nonfinite_off);
}

// The forcing rows of a placed build, unless its workgroups form them themselves.
hipError_t launch_forcing_rows(const PreparedBuild &pb, const Plan &p, char *work,
                               hipStream_t st) {
    const nv::BuildArgs &a = pb.args;
    if (!a.forcing || a.local_forcing) return hipSuccess;
    return nv::launch_forcing(pb.cfg.rhs, pb.cfg.precision, work + p.forcing_off, a.n_slices,
                              a.steps, a.t0, a.L, a.h, st);
}

// Checks, buffers, the pre-launch kernels (forcing values, Chebyshev nodes) on
// the context's stream and the integration kernel's arguments; records the
// build's description in the context (marked built by the caller once the
// integration is launched).
nv_status prepare_build(nv_ctx *ctx, int rhs_id, const double *params, double t0, double T,
                        int n_slices, const nv_ic_grid *grid, int steps_per_slice,
                        PreparedBuild *pb) {
    if (!ctx) return fail(NV_ERR_INVALID_ARG, "ctx is NULL");
    ctx->built = false;
    Plan p;
    nv_status s = describe_build(ctx->opt, rhs_id, params, t0, T, n_slices, grid,
                                 steps_per_slice, &p, pb);
    if (s != NV_OK) return s;

    s = ensure_device(&ctx->tables, &ctx->tables_cap, ctx->tables_owned, p.table_bytes, "table");
    if (s != NV_OK) return s;
    const size_t work_cap_before = ctx->work_cap;
    s = ensure_device(&ctx->work, &ctx->work_cap, ctx->work_owned, p.work_bytes, "work");
    if (s != NV_OK) return s;
    if (ctx->work_cap != work_cap_before) ctx->nodes_dev = nullptr;   // a new allocation
    s = ensure_host_stage(ctx, p.stage_status_off + sizeof(nv::ComposeStatus));
    if (s != NV_OK) return s;
    if (ctx->timing) {
        s = ensure_events(ctx);
        if (s != NV_OK) return s;
    }
    place_build(pb, p, ctx->tables, work_at(ctx, 0));

    hipStream_t st = stream_of(ctx);
    if (grid->interp == NV_INTERP_CHEBYSHEV) {
        double *dn = reinterpret_cast<double *>(work_at(ctx, p.nodes_off));
        if (ctx->nodes_dev != dn || ctx->nodes_n != grid->n[0] ||
            ctx->nodes_lo != grid->lo[0] || ctx->nodes_hi != grid->hi[0]) {
            chebyshev_nodes(grid->n[0], grid->lo[0], grid->hi[0], ctx->nodes_host);
            NV_HIP(hipMemcpyAsync(dn, ctx->nodes_host, size_t(grid->n[0]) * sizeof(double),
                                  hipMemcpyHostToDevice, st));
            ctx->nodes_dev = dn;
            ctx->nodes_n = grid->n[0];
            ctx->nodes_lo = grid->lo[0];
            ctx->nodes_hi = grid->hi[0];
        }
        pb->args.nodes = dn;
    } else {
        // the new table build's forcing values, counters and carried state may cover
        // the place where an earlier build kept its nodes
        ctx->nodes_dev = nullptr;
    }
    NV_HIP(launch_forcing_rows(*pb, p, work_at(ctx, 0), st));

    ctx->plan = p;
    ctx->rhs = rhs_id;
    ctx->precision = ctx->opt.precision;
    ctx->n_slices = n_slices;
    ctx->grid = *grid;
    return NV_OK;
}

// Arguments of the composition kernel over slices [j0, j1) of a build with
// tables at `tables` and scratch at `work`; it writes the boundary states to
// `boundary` and, when the chain ends, the final status to `status_out`.
nv::ComposeArgs compose_args_at(const Plan &p, const nv_ic_grid &g, int n_slices,
                                const void *tables, char *work, double *boundary,
                                nv::ComposeStatus *status_out, const double *y0, int j0,
                                int j1) {
    nv::ComposeArgs a{};
    a.tab0 = tables;
    a.tab1 = p.components == 2 ? static_cast<const char *>(tables) + p.comp_bytes : nullptr;
    a.boundary = boundary;
    a.status = reinterpret_cast<nv::ComposeStatus *>(work + p.status_off);
    a.carry = reinterpret_cast<double *>(work + p.carry_off);
    a.status_host = status_out;
    a.M = p.M;
    a.n_slices = n_slices;
    a.j_begin = j0;
    a.j_end = j1;
    a.n0 = g.n[0];
    a.n1 = p.dim == 2 ? g.n[1] : 1;
    a.lo0 = g.lo[0];
    a.inv0 = double(g.n[0] - 1) / (g.hi[0] - g.lo[0]);
    a.lo1 = p.dim == 2 ? g.lo[1] : 0.0;
    a.inv1 = p.dim == 2 ? double(g.n[1] - 1) / (g.hi[1] - g.lo[1]) : 0.0;
    a.hi0 = g.hi[0];
    a.dxi0 = (g.hi[0] - g.lo[0]) / double(g.n[0] - 1);
    a.nodes = g.interp == NV_INTERP_CHEBYSHEV
                  ? reinterpret_cast<const double *>(work + p.nodes_off)
                  : nullptr;
    a.y00 = y0[0];
    a.y01 = p.dim == 2 ? y0[1] : 0.0;
    return a;
}

// ... over slices [j0, j1) of the context's last build, writing into the
// context's mapped host memory.
nv::ComposeArgs compose_args(const nv_ctx *ctx, const double *y0, int j0, int j1) {
    return compose_args_at(
        ctx->plan, ctx->grid, ctx->n_slices, ctx->tables, work_at(ctx, 0),
        static_cast<double *>(ctx->host_stage_dev),
        reinterpret_cast<nv::ComposeStatus *>(static_cast<char *>(ctx->host_stage_dev) +
                                              ctx->plan.stage_status_off),
        y0, j0, j1);
}

volatile nv::ComposeStatus *host_status(const nv_ctx *ctx) {
    return reinterpret_cast<volatile nv::ComposeStatus *>(static_cast<char *>(ctx->host_stage) +
                                                          ctx->plan.stage_status_off);
}

// Cleared before a composition is launched; its last range sets it once the
// outputs are in host memory.
void clear_host_done(const nv_ctx *ctx) { host_status(ctx)->done = 0; }

// Wait until the composition on stream st has written the boundary states and
// the status into the context's mapped host memory, and hand them out.  The
// chain's last range sets the status's done flag after a system-scope fence,
// so the host polls that flag instead of waiting for the stream's completion
// signal (the kernel's exit, still queued on the stream, is ordered before any
// later work on it).  The stream is queried now and then, so a launch that
// fails or ends without the flag ends the wait: the stream is then
// synchronized, which reports its error.
nv_status finish_compose(nv_ctx *ctx, hipStream_t st, double *yT, double *boundary,
                         nv_compose_info *info, int n_chunks) {
    const Plan &p = ctx->plan;
    volatile nv::ComposeStatus *hs = host_status(ctx);
    bool seen = false;
    for (unsigned n = 1;; ++n) {
        if (hs->done) {
            seen = true;
            break;
        }
        if ((n & 1023u) == 0 && hipStreamQuery(st) != hipErrorNotReady) {
            seen = hs->done != 0;
            break;
        }
    }
    if (!seen) NV_HIP(hipStreamSynchronize(st));
    std::atomic_thread_fence(std::memory_order_acquire);
    const double *hb = static_cast<const double *>(ctx->host_stage);
    nv::ComposeStatus cs;
    cs.n_out_of_grid = hs->n_out_of_grid;
    cs.bad_slice = hs->bad_slice;
    cs.done = hs->done;
    if (!cs.done) return fail(NV_ERR_HIP, "composition kernel did not complete");
    // a range that fails sets the flag while the later ranges of an nv_solve
    // may still be queued (each returns at once on seeing the failure); they
    // are drained here, before a later call can reset the running status they
    // read
    if (cs.bad_slice >= 0) NV_HIP(hipStreamSynchronize(st));
    const int n_done = cs.bad_slice < 0 ? ctx->n_slices : cs.bad_slice;
    if (boundary) std::memcpy(boundary, hb, size_t(n_done + 1) * p.dim * sizeof(double));
    for (int c = 0; c < p.dim; ++c) yT[c] = hb[size_t(n_done) * p.dim + c];
    if (info) {
        info->n_out_of_grid = cs.n_out_of_grid;
        info->bad_slice = cs.bad_slice;
        info->n_chunks = n_chunks;
    }
    if (cs.bad_slice >= 0)
        return fail(NV_ERR_NONFINITE, "composition met a non-finite value in slice %d",
                    cs.bad_slice);
    return NV_OK;
}

}  // namespace

// The scratch of nv_solve_static: one build's scratch, laid out as a
// context's (the plan's offsets).  Each device that runs the library holds
// its own copy until the process ends.  In host code this name stands for no
// device address: the kernels get the address hipGetSymbolAddress gives for
// the current device (static_scratch below).
constexpr size_t kStaticScratchBytes = NV_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_dev[kMaxDevices] = {};

// The current device's address of the scratch, looked up once per device.
nv_status static_scratch(char **out) {
    int dev = -1;
    NV_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(NV_ERR_UNSUPPORTED, "device %d: the static scratch serves devices 0..%d",
                    dev, kMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(NV_ERR_HIP, "hipGetSymbolAddress of the static scratch failed on "
                        "device %d: %s", dev, hipGetErrorString(e));
        g_scratch_dev[dev] = ptr;
    }
    *out = static_cast<char *>(g_scratch_dev[dev]);
    return NV_OK;
}

static_assert(sizeof(nv_solve_status) == sizeof(nv::ComposeStatus) &&
                  offsetof(nv_solve_status, n_out_of_grid) ==
                      offsetof(nv::ComposeStatus, n_out_of_grid) &&
                  offsetof(nv_solve_status, bad_slice) == offsetof(nv::ComposeStatus, bad_slice) &&
                  offsetof(nv_solve_status, done) == offsetof(nv::ComposeStatus, done),
              "nv_solve_status is the composition's final status");

}  // namespace

extern "C" {

NV_API nv_status nv_ctx_create(nv_ctx **out) {
    if (!out) return fail(NV_ERR_INVALID_ARG, "out is NULL");
    *out = new (std::nothrow) nv_ctx();
    if (!*out) return fail(NV_ERR_OOM, "out of host memory");
    return NV_OK;
}

NV_API nv_status nv_ctx_destroy(nv_ctx *ctx) {
    if (!ctx) return NV_OK;
    // every stream that may still use the buffers is drained before they go
    (void)hipStreamSynchronize(stream_of(ctx));
    if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
    if (ctx->aux2) (void)hipStreamSynchronize(ctx->aux2);
    if (ctx->tables_owned && ctx->tables) (void)hipFree(ctx->tables);
    if (ctx->work_owned && ctx->work) (void)hipFree(ctx->work);
    if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
    for (auto e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto e : ctx->chunk_ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->ready_ev) (void)hipEventDestroy(ctx->ready_ev);
    if (ctx->aux) (void)hipStreamDestroy(ctx->aux);
    if (ctx->aux2) (void)hipStreamDestroy(ctx->aux2);
    delete ctx;
    return NV_OK;
}

NV_API nv_status nv_set_options(nv_ctx *ctx, const nv_options *opt) {
    if (!ctx) return fail(NV_ERR_INVALID_ARG, "ctx is NULL");
    nv_status s = check_options(opt);
    if (s != NV_OK) return s;
    ctx->opt = *opt;
    return NV_OK;
}

NV_API nv_status nv_get_options(const nv_ctx *ctx, nv_options *opt) {
    if (!ctx || !opt) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    *opt = ctx->opt;
    return NV_OK;
}

NV_API nv_status nv_required_bytes(int rhs_id, int n_slices, const nv_ic_grid *grid,
                                   int steps_per_slice, const nv_options *opt,
                                   size_t *table_bytes, size_t *work_bytes) {
    nv_options o = default_options();
    if (opt) {
        nv_status s = check_options(opt);
        if (s != NV_OK) return s;
        o = *opt;
    }
    Plan p;
    nv_status s = make_plan(rhs_id, n_slices, grid, steps_per_slice, o, &p);
    if (s != NV_OK) return s;
    if (table_bytes) *table_bytes = p.table_bytes;
    if (work_bytes) *work_bytes = p.work_bytes;
    return NV_OK;
}

NV_API nv_status nv_set_buffers(nv_ctx *ctx, void *tables_dev, size_t table_bytes,
                                void *work_dev, size_t work_bytes) {
    if (!ctx) return fail(NV_ERR_INVALID_ARG, "ctx is NULL");
    if ((tables_dev == nullptr) != (work_dev == nullptr))
        return fail(NV_ERR_INVALID_ARG, "give both buffers or neither");
    NV_HIP(hipStreamSynchronize(stream_of(ctx)));
    if (ctx->aux) NV_HIP(hipStreamSynchronize(ctx->aux));
    if (ctx->aux2) NV_HIP(hipStreamSynchronize(ctx->aux2));
    if (ctx->tables_owned && ctx->tables) NV_HIP(hipFree(ctx->tables));
    if (ctx->work_owned && ctx->work) NV_HIP(hipFree(ctx->work));
    ctx->built = false;
    ctx->nodes_dev = nullptr;
    if (tables_dev) {
        ctx->tables = tables_dev;
        ctx->tables_cap = table_bytes;
        ctx->tables_owned = false;
        ctx->work = work_dev;
        ctx->work_cap = work_bytes;
        ctx->work_owned = false;
    } else {
        ctx->tables = nullptr;
        ctx->tables_cap = 0;
        ctx->tables_owned = true;
        ctx->work = nullptr;
        ctx->work_cap = 0;
        ctx->work_owned = true;
    }
    return NV_OK;
}

NV_API nv_status nv_build_propagators(nv_ctx *ctx, int rhs_id, const double *params,
                                      double t0, double T, int n_slices,
                                      const nv_ic_grid *grid, int steps_per_slice) {
    PreparedBuild pb;
    nv_status s = prepare_build(ctx, rhs_id, params, t0, T, n_slices, grid, steps_per_slice, &pb);
    if (s != NV_OK) return s;
    hipStream_t st = stream_of(ctx);
    ctx->build_timed = ctx->compose_timed = ctx->solve_timed = false;
    if (ctx->timing) NV_HIP(hipEventRecord(ctx->ev[0], st));
    NV_HIP(nv::launch_build(pb.cfg, pb.args, st));
    if (ctx->timing) {
        NV_HIP(hipEventRecord(ctx->ev[1], st));
        ctx->build_timed = true;
    }
    ctx->built = true;
    return NV_OK;
}

NV_API nv_status nv_compose(nv_ctx *ctx, const double *y0, double *yT, double *boundary,
                            nv_compose_info *info) {
    if (!ctx) return fail(NV_ERR_INVALID_ARG, "ctx is NULL");
    if (!ctx->built) return fail(NV_ERR_NOT_BUILT, "nv_compose before a successful build");
    if (!y0 || !yT) return fail(NV_ERR_INVALID_ARG, "y0 and yT must not be NULL");
    hipStream_t st = stream_of(ctx);
    ctx->compose_timed = ctx->solve_timed = false;
    if (ctx->timing) {
        nv_status s = ensure_events(ctx);
        if (s != NV_OK) return s;
        NV_HIP(hipEventRecord(ctx->ev[2], st));
    }
    clear_host_done(ctx);
    NV_HIP(nv::launch_compose(ctx->grid.interp, ctx->precision,
                              compose_args(ctx, y0, 0, ctx->n_slices), st));
    if (ctx->timing) {
        NV_HIP(hipEventRecord(ctx->ev[3], st));
        ctx->compose_timed = true;
    }
    return finish_compose(ctx, st, yT, boundary, info, 1);
}

NV_API nv_status nv_solve(nv_ctx *ctx, int rhs_id, const double *params, double t0, double T,
                          int n_slices, const nv_ic_grid *grid, int steps_per_slice,
                          const double *y0, double *yT, double *boundary,
                          nv_compose_info *info) {
    if (!ctx) return fail(NV_ERR_INVALID_ARG, "ctx is NULL");
    if (!y0 || !yT) return fail(NV_ERR_INVALID_ARG, "y0 and yT must not be NULL");
    PreparedBuild pb;
    nv_status s = prepare_build(ctx, rhs_id, params, t0, T, n_slices, grid, steps_per_slice, &pb);
    if (s != NV_OK) return s;
    // chunks of whole slices
    int chunks = ctx->opt.solve_chunks;
    if (chunks == 0) {
        const long long c = ctx->plan.total_blocks / kBlocksPerChunk;
        chunks = int(c < 1 ? 1 : (c > kMaxChunks ? kMaxChunks : c));
    }
    if (chunks > n_slices) chunks = n_slices;
    const int per = (n_slices + chunks - 1) / chunks;
    chunks = (n_slices + per - 1) / per;

    if (chunks == 1) {
        // nothing to overlap: build and compose back to back on the context's
        // stream, without the second streams and their events
        hipStream_t st = stream_of(ctx);
        ctx->build_timed = ctx->compose_timed = ctx->solve_timed = false;
        if (ctx->timing) NV_HIP(hipEventRecord(ctx->ev[0], st));
        NV_HIP(nv::launch_build(pb.cfg, pb.args, st));
        if (ctx->timing) NV_HIP(hipEventRecord(ctx->ev[1], st));
        clear_host_done(ctx);
        NV_HIP(nv::launch_compose(ctx->grid.interp, ctx->precision,
                                  compose_args(ctx, y0, 0, n_slices), st));
        if (ctx->timing) {
            NV_HIP(hipEventRecord(ctx->ev[3], st));
            ctx->build_timed = ctx->compose_timed = ctx->solve_timed = true;
        }
        ctx->built = true;
        return finish_compose(ctx, st, yT, boundary, info, 1);
    }

    if (!ctx->aux) NV_HIP(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    if (!ctx->aux2) NV_HIP(hipStreamCreateWithFlags(&ctx->aux2, hipStreamNonBlocking));
    if (!ctx->ready_ev) NV_HIP(hipEventCreateWithFlags(&ctx->ready_ev, hipEventDisableTiming));
    for (int c = 0; c < chunks; ++c)
        if (!ctx->chunk_ev[c])
            NV_HIP(hipEventCreateWithFlags(&ctx->chunk_ev[c], hipEventDisableTiming));

    // build chunks alternate between the context's stream and a second one, so
    // that one chunk's last workgroups overlap the next chunk's first ones; the
    // second stream starts after the counter reset and the forcing values
    hipStream_t st = stream_of(ctx), aux = ctx->aux, st2 = ctx->aux2;
    ctx->build_timed = ctx->compose_timed = ctx->solve_timed = false;
    NV_HIP(hipEventRecord(ctx->ready_ev, st));
    NV_HIP(hipStreamWaitEvent(st2, ctx->ready_ev, 0));
    if (ctx->timing) NV_HIP(hipEventRecord(ctx->ev[0], st));
    for (int c = 0; c < chunks; ++c) {
        hipStream_t bs = (c % 2 == 0) ? st : st2;
        nv::BuildArgs a = pb.args;
        a.slice0 = c * per;
        const int ns = (a.slice0 + per <= n_slices ? per : n_slices - a.slice0);
        a.total_blocks = ns * a.tiles_per_slice;
        NV_HIP(nv::launch_build(pb.cfg, a, bs));
        NV_HIP(hipEventRecord(ctx->chunk_ev[c], bs));
    }
    // the context's stream waits for every build chunk
    if (chunks > 1) NV_HIP(hipStreamWaitEvent(st, ctx->chunk_ev[chunks % 2 == 0 ? chunks - 1
                                                                            : chunks - 2], 0));
    if (ctx->timing) NV_HIP(hipEventRecord(ctx->ev[1], st));
    clear_host_done(ctx);
    for (int c = 0; c < chunks; ++c) {
        const int j0 = c * per, j1 = (j0 + per <= n_slices ? j0 + per : n_slices);
        NV_HIP(hipStreamWaitEvent(aux, ctx->chunk_ev[c], 0));
        NV_HIP(nv::launch_compose(ctx->grid.interp, ctx->precision,
                                  compose_args(ctx, y0, j0, j1), aux));
    }
    if (ctx->timing) {
        NV_HIP(hipEventRecord(ctx->ev[3], aux));
        ctx->build_timed = true;
    }
    ctx->built = true;
    s = finish_compose(ctx, aux, yT, boundary, info, chunks);
    if (ctx->timing) {
        ctx->compose_timed = true;
        ctx->solve_timed = true;
    }
    return s;
}

NV_API nv_status nv_solve_static(int rhs_id, const double *params, double t0, double T,
                                 int n_slices, const nv_ic_grid *grid, int steps_per_slice,
                                 const nv_options *opt, void *tables_dev, size_t table_bytes,
                                 const double *y0, double *boundary_dev,
                                 nv_solve_status *status_dev) {
    nv_status s = check_options(opt);
    if (s != NV_OK) return s;
    if (!y0 || !tables_dev || !boundary_dev || !status_dev)
        return fail(NV_ERR_INVALID_ARG, "y0, tables_dev, boundary_dev and status_dev must not "
                    "be NULL");
    if (reinterpret_cast<uintptr_t>(tables_dev) % kAlign != 0 ||
        reinterpret_cast<uintptr_t>(boundary_dev) % alignof(double) != 0 ||
        reinterpret_cast<uintptr_t>(status_dev) % alignof(nv_solve_status) != 0)
        return fail(NV_ERR_INVALID_ARG, "tables_dev must be 256-byte aligned, boundary_dev and "
                    "status_dev 8-byte aligned");
    if (grid && grid->interp == NV_INTERP_CHEBYSHEV)
        return fail(NV_ERR_UNSUPPORTED, "nv_solve_static takes no Chebyshev grid (its nodes "
                    "are uploaded from host memory)");
    Plan p;
    PreparedBuild pb;
    s = describe_build(*opt, rhs_id, params, t0, T, n_slices, grid, steps_per_slice, &p, &pb);
    if (s != NV_OK) return s;
    if (p.table_bytes > table_bytes)
        return fail(NV_ERR_BUFFER_TOO_SMALL, "tables need %zu bytes, %zu given", p.table_bytes,
                    table_bytes);
    if (p.work_bytes > kStaticScratchBytes)
        return fail(NV_ERR_BUFFER_TOO_SMALL, "this build needs %zu bytes of scratch; the static "
                    "scratch holds %zu (NV_STATIC_SCRATCH_BYTES)", p.work_bytes,
                    kStaticScratchBytes);
    char *work = nullptr;
    s = static_scratch(&work);
    if (s != NV_OK) return s;
    place_build(&pb, p, tables_dev, work);
    hipStream_t st = static_cast<hipStream_t>(opt->stream);
    NV_HIP(launch_forcing_rows(pb, p, work, st));
    NV_HIP(nv::launch_build(pb.cfg, pb.args, st));
    NV_HIP(nv::launch_compose(grid->interp, opt->precision,
                              compose_args_at(p, *grid, n_slices, tables_dev, work, boundary_dev,
                                              reinterpret_cast<nv::ComposeStatus *>(status_dev),
                                              y0, 0, n_slices),
                              st));
    return NV_OK;
}

NV_API nv_status nv_get_table(nv_ctx *ctx, int component, void *host_dst, size_t bytes) {
    if (!ctx) return fail(NV_ERR_INVALID_ARG, "ctx is NULL");
    if (!ctx->built) return fail(NV_ERR_NOT_BUILT, "no table before a successful build");
    if (component < 0 || component >= ctx->plan.components || !host_dst)
        return fail(NV_ERR_INVALID_ARG, "bad component or NULL destination");
    const size_t need = size_t(ctx->plan.M) * size_t(ctx->n_slices) * ctx->plan.elem;
    if (bytes < need) return fail(NV_ERR_BUFFER_TOO_SMALL, "need %zu bytes", need);
    hipStream_t st = stream_of(ctx);
    const char *src = static_cast<const char *>(ctx->tables) + component * ctx->plan.comp_bytes;
    NV_HIP(hipMemcpyAsync(host_dst, src, need, hipMemcpyDeviceToHost, st));
    NV_HIP(hipStreamSynchronize(st));
    return NV_OK;
}

NV_API nv_status nv_table_device_ptr(nv_ctx *ctx, int component, void **dev_ptr) {
    if (!ctx || !dev_ptr) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (!ctx->built) return fail(NV_ERR_NOT_BUILT, "no table before a successful build");
    if (component < 0 || component >= ctx->plan.components)
        return fail(NV_ERR_INVALID_ARG, "bad component %d", component);
    *dev_ptr = static_cast<char *>(ctx->tables) + component * ctx->plan.comp_bytes;
    return NV_OK;
}

NV_API nv_status nv_get_nonfinite_counts(nv_ctx *ctx, uint32_t *host_counts, int n) {
    if (!ctx || !host_counts) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (!ctx->built) return fail(NV_ERR_NOT_BUILT, "no counts before a successful build");
    if (n < ctx->n_slices) return fail(NV_ERR_BUFFER_TOO_SMALL, "need %d counts", ctx->n_slices);
    hipStream_t st = stream_of(ctx);
    // one count per tile: the slice's count is their sum
    const size_t tiles = size_t(ctx->plan.tiles_per_slice), ns = size_t(ctx->n_slices);
    std::vector<uint32_t> per_tile;
    try {
        per_tile.resize(ns * tiles);
    } catch (const std::bad_alloc &) {
        return fail(NV_ERR_OOM, "no host memory for %zu per-tile counts", ns * tiles);
    }
    NV_HIP(hipMemcpyAsync(per_tile.data(), work_at(ctx, ctx->plan.nonfinite_off),
                          per_tile.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    NV_HIP(hipStreamSynchronize(st));
    for (size_t j = 0; j < ns; ++j) {
        uint32_t sum = 0;
        for (size_t t = 0; t < tiles; ++t) sum += per_tile[j * tiles + t];
        host_counts[j] = sum;
    }
    return NV_OK;
}

NV_API nv_status nv_locate(nv_ctx *ctx, double lo, double hi, int n, const double *x_dev,
                           long long count, long long *cell_dev, double *w_dev,
                           int32_t *out_dev) {
    if (!ctx) return fail(NV_ERR_INVALID_ARG, "ctx is NULL");
    if (n < 2 || !std::isfinite(lo) || !std::isfinite(hi) || !(hi > lo))
        return fail(NV_ERR_INVALID_ARG, "need n >= 2 and finite lo < hi");
    if (count < 0) return fail(NV_ERR_INVALID_ARG, "negative count");
    if (count > 0 && (!x_dev || !cell_dev || !w_dev || !out_dev))
        return fail(NV_ERR_INVALID_ARG, "NULL device array");
    const double inv = double(n - 1) / (hi - lo);
    hipStream_t st = stream_of(ctx);
    NV_HIP(nv::launch_locate(lo, inv, n, x_dev, count, cell_dev, w_dev, out_dev, st));
    NV_HIP(hipStreamSynchronize(st));
    return NV_OK;
}

NV_API nv_status nv_set_timing(nv_ctx *ctx, int enable) {
    if (!ctx) return fail(NV_ERR_INVALID_ARG, "ctx is NULL");
    ctx->timing = enable != 0;
    ctx->build_timed = ctx->compose_timed = ctx->solve_timed = false;
    return NV_OK;
}

NV_API nv_status nv_last_timing(nv_ctx *ctx, float *build_ms, float *compose_ms) {
    if (!ctx) return fail(NV_ERR_INVALID_ARG, "ctx is NULL");
    if (build_ms) {
        *build_ms = -1.0f;
        if (ctx->build_timed) {
            NV_HIP(hipEventSynchronize(ctx->ev[1]));
            NV_HIP(hipEventElapsedTime(build_ms, ctx->ev[0], ctx->ev[1]));
        }
    }
    if (compose_ms) {
        *compose_ms = -1.0f;
        if (ctx->compose_timed) {
            // after nv_solve: the composition left once the last build launch ended
            hipEvent_t from = ctx->solve_timed ? ctx->ev[1] : ctx->ev[2];
            NV_HIP(hipEventSynchronize(ctx->ev[3]));
            NV_HIP(hipEventElapsedTime(compose_ms, from, ctx->ev[3]));
        }
    }
    return NV_OK;
}

NV_API const char *nv_last_error(void) { return g_last_error; }

NV_API const char *nv_status_string(int status) {
    switch (status) {
    case NV_OK: return "NV_OK";
    case NV_ERR_INVALID_ARG: return "NV_ERR_INVALID_ARG";
    case NV_ERR_NOT_BUILT: return "NV_ERR_NOT_BUILT";
    case NV_ERR_NONFINITE: return "NV_ERR_NONFINITE";
    case NV_ERR_OOM: return "NV_ERR_OOM";
    case NV_ERR_HIP: return "NV_ERR_HIP";
    case NV_ERR_UNSUPPORTED: return "NV_ERR_UNSUPPORTED";
    case NV_ERR_BUFFER_TOO_SMALL: return "NV_ERR_BUFFER_TOO_SMALL";
    default: return "unknown status";
    }
}

}  // extern "C"
