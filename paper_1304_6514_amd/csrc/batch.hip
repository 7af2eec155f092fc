// Batches of independent problems of uneven shape (include/nv.h, nv_batch_*).
//
// Computation phase: ONE persistent launch.  256 CUs x W workgroups of 256
// lanes loop: workgroup takes the next work item from a shared counter (a tile
// of 256*P grid points of one slice of one problem, longest items first), runs
// the same integration body as the single-problem build (build_tile), and
// exits when the list is exhausted -- every workgroup reaches that exit.
// Communication phase: one launch, one wave per problem, each running its own
// dependent chain.  Counter reset, both launches and the copy of the results
// are captured once into a HIP graph and replayed.
#include "compose.h"
#include "integrate.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

namespace nv {
namespace {
using namespace dev;

// Integration cost of one step of one trajectory, in VALU operations, used to
// order the work list (longest items first).
int step_cost(int rhs) {
    switch (rhs) {
    case NV_RHS_VDP: return 28;
    case NV_RHS_LOGISTIC: return 12;
    default: return 11;
    }
}

template <class R, int A, int P>
__device__ inline void run_tile(const BuildArgs &a, int rhs, int j, int tile) {
    unsigned bad = 0;
    switch (rhs) {
    case NV_RHS_LINEAR: bad = build_tile<RhsLinear<R>, R, 0, A, P>(a, j, tile); break;
    case NV_RHS_LOGISTIC: bad = build_tile<RhsLogistic<R>, R, 0, A, P>(a, j, tile); break;
    case NV_RHS_VDP: bad = build_tile<RhsVdp<R>, R, 0, A, P>(a, j, tile); break;
    case NV_RHS_SQUARE: bad = build_tile<RhsSquare<R>, R, 0, A, P>(a, j, tile); break;
    default: break;
    }
    if (bad) atomicAdd(&a.nonfinite[j], bad);      // counters cleared in the graph
}

template <class R, int A>
__global__ void __launch_bounds__(kBuildBlock)
    batch_build_kernel(const BatchProblem *__restrict__ probs,
                       const BatchItem *__restrict__ items, int n_items, unsigned *counter) {
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = int(atomicAdd(counter, 1u));
        __syncthreads();
        // the item index is the same for the whole workgroup: keep it scalar
        const int it = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (it >= n_items) return;
        const BatchItem item = items[it];
        const BatchProblem &pr = probs[item.problem];
        switch (pr.traj_per_lane) {
        case 1: run_tile<R, A, 1>(pr.build, pr.rhs, item.slice, item.tile); break;
        case 2: run_tile<R, A, 2>(pr.build, pr.rhs, item.slice, item.tile); break;
        default: run_tile<R, A, 4>(pr.build, pr.rhs, item.slice, item.tile); break;
        }
    }
}

template <class T>
__global__ void batch_compose_kernel(const BatchProblem *__restrict__ probs, int count) {
    const int b = int(blockIdx.x);
    if (b >= count) return;
    const BatchProblem &pr = probs[b];
    double fin[2] = {0.0, 0.0};
    switch (pr.interp) {
    case NV_INTERP_LINEAR: compose_range<T, 0>(pr.compose, fin); break;
    case NV_INTERP_HERMITE: compose_range<T, 1>(pr.compose, fin); break;
    default: compose_range<T, 2>(pr.compose, fin); break;
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < pr.dim; ++d) pr.result[d] = fin[d];
}

}  // namespace

hipError_t launch_batch_build(int precision, int accumulation, const BatchProblem *probs,
                              const BatchItem *items, int n_items, unsigned *counter,
                              int n_workgroups, hipStream_t s) {
    const dim3 grid{unsigned(n_workgroups), 1, 1}, block{unsigned(kBuildBlock), 1, 1};
    if (precision == NV_FP64)
        hipLaunchKernelGGL((batch_build_kernel<double, kPlain>), grid, block, 0, s, probs, items,
                           n_items, counter);
    else if (accumulation == 0)
        hipLaunchKernelGGL((batch_build_kernel<float, kPlain>), grid, block, 0, s, probs, items,
                           n_items, counter);
    else if (accumulation == 1)
        hipLaunchKernelGGL((batch_build_kernel<float, kKahan>), grid, block, 0, s, probs, items,
                           n_items, counter);
    else
        hipLaunchKernelGGL((batch_build_kernel<float, kBlocked>), grid, block, 0, s, probs,
                           items, n_items, counter);
    return hipGetLastError();
}

hipError_t launch_batch_compose(int precision, const BatchProblem *probs, int count,
                                hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (precision == NV_FP64)
        hipLaunchKernelGGL((batch_compose_kernel<double>), dim3(unsigned(count)), dim3(64), 0, s,
                           probs, count);
    else
        hipLaunchKernelGGL((batch_compose_kernel<float>), dim3(unsigned(count)), dim3(64), 0, s,
                           probs, count);
    return hipGetLastError();
}

}  // namespace nv

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

using nv::fail;

#define NV_HIP(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(NV_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int kCus = 256;

struct Item {
    nv::BatchItem it;
    long long cost;
};

}  // namespace

struct nv_batch {
    int count = 0;
    std::vector<nv_problem> problems;
    int precision = NV_FP32, accumulation = 2, scheme = NV_SCHEME_RK4;
    nv_batch_schedule sched{};
    // device memory
    char *tables = nullptr;
    char *work = nullptr;
    size_t off_probs = 0, off_items = 0, off_counter = 0, off_nonfinite = 0, off_boundary = 0,
           off_status = 0, off_result = 0, work_bytes = 0, tables_bytes = 0;
    long long max_items = 0, total_slices = 0;
    std::vector<size_t> tab_off, comp_bytes, bnd_off, elems;
    std::vector<nv::BatchProblem> hp;
    int n_items = 0;
    long long traj_steps = 0;
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *stage = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    bool ran = false;          // a run has written the tables
};

namespace {

int dim_of(const nv_problem &p) { return p.rhs_id == NV_RHS_VDP ? 2 : 1; }

long long points_of(const nv_problem &p) {
    return p.grid.dim == 2 ? (long long)p.grid.n[0] * p.grid.n[1] : (long long)p.grid.n[0];
}

// The work list for the batch's schedule (all problems, or one right-hand side).
std::vector<nv::BatchItem> make_items(const nv_batch *b, const nv_batch_schedule &s,
                                      int only_rhs) {
    std::vector<Item> v;
    for (int i = 0; i < b->count; ++i) {
        const nv_problem &p = b->problems[i];
        if (only_rhs >= 0 && p.rhs_id != only_rhs) continue;
        const int P = s.traj_per_lane[p.rhs_id];
        const long long per = (long long)nv::kBuildBlock * P;
        const int tiles = int((points_of(p) + per - 1) / per);
        const long long cost = (long long)p.steps_per_slice * nv::step_cost(p.rhs_id) * per *
                               dim_of(p);
        for (int j = 0; j < p.n_slices; ++j)
            for (int t = 0; t < tiles; ++t) v.push_back({{i, j, t, 0}, cost});
    }
    if (s.order == 0)
        std::stable_sort(v.begin(), v.end(),
                         [](const Item &a, const Item &c) { return a.cost > c.cost; });
    std::vector<nv::BatchItem> out(v.size());
    for (size_t k = 0; k < v.size(); ++k) out[k] = v[k].it;
    return out;
}

nv_status check_schedule(const nv_batch_schedule *s) {
    if (!s) return fail(NV_ERR_INVALID_ARG, "schedule is NULL");
    for (int r = 0; r < 5; ++r)
        if (s->traj_per_lane[r] != 1 && s->traj_per_lane[r] != 2 && s->traj_per_lane[r] != 4)
            return fail(NV_ERR_INVALID_ARG, "traj_per_lane[%d] must be 1, 2 or 4", r);
    if (s->workgroups_per_cu < 1 || s->workgroups_per_cu > 8)
        return fail(NV_ERR_INVALID_ARG, "workgroups_per_cu must be in [1, 8]");
    if (s->order != 0 && s->order != 1) return fail(NV_ERR_INVALID_ARG, "order must be 0 or 1");
    return NV_OK;
}

void drop_graph(nv_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

// Apply a schedule: per-problem P and tiles, the work list, and upload both.
nv_status apply_schedule(nv_batch *b, const nv_batch_schedule &s) {
    for (int i = 0; i < b->count; ++i) {
        const nv_problem &p = b->problems[i];
        const int P = s.traj_per_lane[p.rhs_id];
        const long long per = (long long)nv::kBuildBlock * P;
        b->hp[i].traj_per_lane = P;
        b->hp[i].build.tiles_per_slice = int((points_of(p) + per - 1) / per);
    }
    const std::vector<nv::BatchItem> items = make_items(b, s, -1);
    b->n_items = int(items.size());
    NV_HIP(hipMemcpyAsync(b->work + b->off_probs, b->hp.data(),
                          b->hp.size() * sizeof(nv::BatchProblem), hipMemcpyHostToDevice,
                          b->stream));
    NV_HIP(hipMemcpyAsync(b->work + b->off_items, items.data(),
                          items.size() * sizeof(nv::BatchItem), hipMemcpyHostToDevice,
                          b->stream));
    NV_HIP(hipStreamSynchronize(b->stream));
    b->sched = s;
    drop_graph(b);
    return NV_OK;
}

// The build of a list of items alone (no graph), timed with events; ms < 0 on error.
nv_status time_build(nv_batch *b, const std::vector<nv::BatchItem> &items, int wpc, int reps,
                     float *ms) {
    NV_HIP(hipMemcpyAsync(b->work + b->off_items, items.data(),
                          items.size() * sizeof(nv::BatchItem), hipMemcpyHostToDevice,
                          b->stream));
    NV_HIP(hipMemcpyAsync(b->work + b->off_probs, b->hp.data(),
                          b->hp.size() * sizeof(nv::BatchProblem), hipMemcpyHostToDevice,
                          b->stream));
    auto *counter = reinterpret_cast<unsigned *>(b->work + b->off_counter);
    const auto *probs = reinterpret_cast<const nv::BatchProblem *>(b->work + b->off_probs);
    const auto *dit = reinterpret_cast<const nv::BatchItem *>(b->work + b->off_items);
    float best = 1e30f;
    for (int r = 0; r <= reps; ++r) {            // the first launch is a warm-up
        NV_HIP(nv::launch_fill_u32(counter, 1, 0u, b->stream));
        NV_HIP(hipEventRecord(b->ev0, b->stream));
        NV_HIP(nv::launch_batch_build(b->precision, b->accumulation, probs, dit, int(items.size()),
                                      counter, kCus * wpc, b->stream));
        NV_HIP(hipEventRecord(b->ev1, b->stream));
        NV_HIP(hipEventSynchronize(b->ev1));
        float t = 0.f;
        NV_HIP(hipEventElapsedTime(&t, b->ev0, b->ev1));
        if (r > 0) best = std::min(best, t);
    }
    *ms = best;
    return NV_OK;
}

nv_status ensure_graph(nv_batch *b) {
    if (b->exec) return NV_OK;
    auto *counter = reinterpret_cast<unsigned *>(b->work + b->off_counter);
    auto *nonfinite = reinterpret_cast<uint32_t *>(b->work + b->off_nonfinite);
    const auto *probs = reinterpret_cast<const nv::BatchProblem *>(b->work + b->off_probs);
    const auto *items = reinterpret_cast<const nv::BatchItem *>(b->work + b->off_items);
    NV_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    // counters are cleared by a fill kernel, never by a memset node
    hipError_t e = nv::launch_fill_u32(counter, 1, 0u, b->stream);
    if (e == hipSuccess) e = nv::launch_fill_u32(nonfinite, b->total_slices, 0u, b->stream);
    if (e == hipSuccess)
        e = nv::launch_batch_build(b->precision, b->accumulation, probs, items, b->n_items, counter,
                                   kCus * b->sched.workgroups_per_cu, b->stream);
    if (e == hipSuccess) e = nv::launch_batch_compose(b->precision, probs, b->count, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->stage, b->work + b->off_status,
                           b->off_result - b->off_status + size_t(b->count) * 2 * sizeof(double),
                           hipMemcpyDeviceToHost, b->stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(NV_ERR_HIP, "graph capture failed: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    b->graph = g;
    NV_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return NV_OK;
}

void free_batch(nv_batch *b) {
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    drop_graph(b);
    if (b->tables) (void)hipFree(b->tables);
    if (b->work) (void)hipFree(b->work);
    if (b->stage) (void)hipHostFree(b->stage);
    if (b->ev0) (void)hipEventDestroy(b->ev0);
    if (b->ev1) (void)hipEventDestroy(b->ev1);
    if (b->stream) (void)hipStreamDestroy(b->stream);
    delete b;
}

}  // namespace

namespace {

// The tuning itself; it overwrites the device work list and descriptors while
// timing candidates (the caller restores a consistent schedule on failure).
nv_status autotune(nv_batch *b, int reps, nv_batch_schedule *chosen) {
    drop_graph(b);
    nv_batch_schedule best = b->sched;
    const int cands[3] = {1, 2, 4};
    // 1. P per right-hand side, on that right-hand side's items alone
    for (int r = 0; r < 5; ++r) {
        bool present = false;
        for (const nv_problem &p : b->problems) present = present || p.rhs_id == r;
        if (!present) continue;
        float best_ms = 1e30f;
        int best_p = best.traj_per_lane[r];
        for (int P : cands) {
            nv_batch_schedule s = best;
            s.traj_per_lane[r] = P;
            for (int i = 0; i < b->count; ++i) {
                const long long per = (long long)nv::kBuildBlock * s.traj_per_lane[b->problems[i].rhs_id];
                b->hp[i].traj_per_lane = s.traj_per_lane[b->problems[i].rhs_id];
                b->hp[i].build.tiles_per_slice = int((points_of(b->problems[i]) + per - 1) / per);
            }
            float ms = 0.f;
            nv_status st = time_build(b, make_items(b, s, r), best.workgroups_per_cu, reps, &ms);
            if (st != NV_OK) return st;
            if (ms < best_ms) {
                best_ms = ms;
                best_p = P;
            }
        }
        best.traj_per_lane[r] = best_p;
    }
    // 2. persistent grid size and item order, on the whole batch
    for (int i = 0; i < b->count; ++i) {
        const long long per = (long long)nv::kBuildBlock * best.traj_per_lane[b->problems[i].rhs_id];
        b->hp[i].traj_per_lane = best.traj_per_lane[b->problems[i].rhs_id];
        b->hp[i].build.tiles_per_slice = int((points_of(b->problems[i]) + per - 1) / per);
    }
    float best_ms = 1e30f;
    nv_batch_schedule pick = best;
    for (int wpc : {4, 8})
        for (int order : {0, 1}) {
            nv_batch_schedule s = best;
            s.workgroups_per_cu = wpc;
            s.order = order;
            float ms = 0.f;
            nv_status st = time_build(b, make_items(b, s, -1), wpc, reps, &ms);
            if (st != NV_OK) return st;
            if (ms < best_ms) {
                best_ms = ms;
                pick = s;
            }
        }
    nv_status st = apply_schedule(b, pick);
    if (st != NV_OK) return st;
    if (chosen) *chosen = pick;
    return NV_OK;
}

}  // namespace

extern "C" {

NV_API nv_status nv_batch_create(nv_ctx *ctx, const nv_problem *problems, int count,
                                 nv_batch **out) try {
    if (!ctx || !problems || !out) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (count < 1) return fail(NV_ERR_INVALID_ARG, "count must be >= 1");
    *out = nullptr;
    nv_options opt;
    nv_status s = nv_get_options(ctx, &opt);
    if (s != NV_OK) return s;
    for (int i = 0; i < count; ++i) {
        const nv_problem &p = problems[i];
        if (p.rhs_id == NV_RHS_FORCED_CUBIC)
            return fail(NV_ERR_UNSUPPORTED, "problem %d: batches take autonomous right-hand sides",
                        i);
        if (p.grid.interp == NV_INTERP_CHEBYSHEV)
            return fail(NV_ERR_UNSUPPORTED, "problem %d: batches take uniform grids", i);
        if (p.grid.interp == NV_INTERP_HERMITE_SLOPES)
            return fail(NV_ERR_UNSUPPORTED, "problem %d: batches build no slope tables", i);
        s = nv::check_problem(p.rhs_id, p.params, p.t0, p.T, p.n_slices, &p.grid,
                              p.steps_per_slice);
        if (s != NV_OK) {
            char msg[512];
            snprintf(msg, sizeof msg, "problem %d: %s", i, nv_last_error());
            return fail(s, "%s", msg);
        }
    }
    // owned by the guard until the batch is complete: every failure below,
    // a host allocation that throws included, frees what was set up so far
    std::unique_ptr<nv_batch, void (*)(nv_batch *)> guard(new (std::nothrow) nv_batch(),
                                                          free_batch);
    nv_batch *b = guard.get();
    if (!b) return fail(NV_ERR_OOM, "out of host memory");
    b->count = count;
    b->problems.assign(problems, problems + count);
    b->precision = opt.precision;
    b->accumulation = opt.compensated;
    b->scheme = opt.scheme;
    if (b->scheme != NV_SCHEME_RK4 || opt.dt != 0.0) {
        return fail(NV_ERR_UNSUPPORTED, "batches integrate with RK4 and equal steps per slice");
    }
    const size_t elem = b->precision == NV_FP64 ? sizeof(double) : sizeof(float);

    // layout: tables (per problem, per component), then scratch
    b->tab_off.resize(count);
    b->comp_bytes.resize(count);
    b->bnd_off.resize(count);
    b->elems.resize(count);
    size_t toff = 0, boff = 0;
    long long nf = 0;
    for (int i = 0; i < count; ++i) {
        const nv_problem &p = problems[i];
        const long long M = points_of(p);
        b->tab_off[i] = toff;
        b->elems[i] = size_t(M) * size_t(p.n_slices);
        b->comp_bytes[i] = align_up(b->elems[i] * elem);
        toff += b->comp_bytes[i] * size_t(dim_of(p));
        b->bnd_off[i] = boff;
        boff += (size_t(p.n_slices) + 1) * size_t(dim_of(p)) * sizeof(double);
        nf += p.n_slices;
        b->max_items += (long long)p.n_slices * ((M + nv::kBuildBlock - 1) / nv::kBuildBlock);
        b->traj_steps += M * p.n_slices * (long long)p.steps_per_slice;
    }
    b->total_slices = nf;
    b->tables_bytes = toff;
    if (b->max_items > 0x7fffffffLL) {
        return fail(NV_ERR_INVALID_ARG, "batch has more than 2^31-1 work items");
    }
    size_t off = 0;
    b->off_probs = off;
    off = align_up(off + size_t(count) * sizeof(nv::BatchProblem));
    b->off_items = off;
    off = align_up(off + size_t(b->max_items) * sizeof(nv::BatchItem));
    b->off_counter = off;
    off = align_up(off + sizeof(unsigned));
    b->off_nonfinite = off;
    off = align_up(off + size_t(nf) * sizeof(uint32_t));
    b->off_boundary = off;
    off = align_up(off + boff);
    b->off_status = off;                              // statuses, then results, adjacent
    b->off_result = align_up(off + size_t(count) * sizeof(nv::ComposeStatus));
    off = align_up(b->off_result + size_t(count) * 2 * sizeof(double));
    b->work_bytes = off;

    hipError_t e = hipMalloc(reinterpret_cast<void **>(&b->tables), b->tables_bytes);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&b->work), b->work_bytes);
    if (e != hipSuccess) {
        return fail(NV_ERR_OOM, "device allocation of %zu + %zu bytes failed", b->tables_bytes,
                    b->work_bytes);
    }
    e = hipHostMalloc(&b->stage, b->work_bytes - b->off_status, hipHostMallocDefault);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&b->ev0);
    if (e == hipSuccess) e = hipEventCreate(&b->ev1);
    if (e != hipSuccess) {
        return fail(NV_ERR_HIP, "batch set-up failed: %s", hipGetErrorString(e));
    }

    // device descriptors of every problem
    b->hp.resize(count);
    size_t nf_off = 0;
    for (int i = 0; i < count; ++i) {
        const nv_problem &p = problems[i];
        const int D = dim_of(p);
        nv::BatchProblem &q = b->hp[i];
        std::memset(&q, 0, sizeof q);
        char *t0 = b->tables + b->tab_off[i];
        char *t1 = D == 2 ? t0 + b->comp_bytes[i] : nullptr;
        // slice partition (sec. 3): L = (T - t0)/N, h = L / S
        const double L = (p.T - p.t0) / double(p.n_slices);
        nv::BuildArgs &a = q.build;
        a.tab0 = t0;
        a.tab1 = t1;
        a.forcing = nullptr;
        a.nonfinite = reinterpret_cast<uint32_t *>(b->work + b->off_nonfinite) + nf_off;
        a.lo0 = p.grid.lo[0];
        a.dxi0 = (p.grid.hi[0] - p.grid.lo[0]) / double(p.grid.n[0] - 1);
        a.lo1 = D == 2 ? p.grid.lo[1] : 0.0;
        a.dxi1 = D == 2 ? (p.grid.hi[1] - p.grid.lo[1]) / double(p.grid.n[1] - 1) : 0.0;
        a.h = L / double(p.steps_per_slice);
        a.h_last = 0.0;
        a.nodes = nullptr;
        a.p0 = (p.rhs_id == NV_RHS_LINEAR || p.rhs_id == NV_RHS_VDP) ? p.params[0] : 0.0;
        a.M = points_of(p);
        a.n1 = D == 2 ? p.grid.n[1] : 1;
        a.n_slices = p.n_slices;
        a.slice0 = 0;
        a.steps = p.steps_per_slice;
        nv::ComposeArgs &c = q.compose;
        c.tab0 = t0;
        c.tab1 = t1;
        c.boundary = reinterpret_cast<double *>(b->work + b->off_boundary + b->bnd_off[i]);
        c.status = reinterpret_cast<nv::ComposeStatus *>(b->work + b->off_status) + i;
        c.carry = nullptr;                  // one range per problem: nothing to carry
        c.status_host = nullptr;
        c.M = a.M;
        c.n_slices = p.n_slices;
        c.j_begin = 0;
        c.j_end = p.n_slices;
        c.n0 = p.grid.n[0];
        c.n1 = a.n1;
        c.lo0 = p.grid.lo[0];
        c.inv0 = double(p.grid.n[0] - 1) / (p.grid.hi[0] - p.grid.lo[0]);
        c.lo1 = a.lo1;
        c.inv1 = D == 2 ? double(p.grid.n[1] - 1) / (p.grid.hi[1] - p.grid.lo[1]) : 0.0;
        c.hi0 = p.grid.hi[0];
        c.nodes = nullptr;
        c.y00 = p.y0[0];
        c.y01 = D == 2 ? p.y0[1] : 0.0;
        q.rhs = p.rhs_id;
        q.interp = p.grid.interp;
        q.dim = D;
        q.result = reinterpret_cast<double *>(b->work + b->off_result) + 2 * size_t(i);
        nf_off += size_t(p.n_slices);
    }
    nv_batch_schedule def{};
    for (int r = 0; r < 5; ++r) def.traj_per_lane[r] = 1;
    def.workgroups_per_cu = 8;
    def.order = 0;
    s = apply_schedule(b, def);
    if (s != NV_OK) return s;
    *out = guard.release();
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_batch_create: host allocation failed");
}

NV_API nv_status nv_batch_destroy(nv_batch *batch) {
    if (batch) free_batch(batch);
    return NV_OK;
}

NV_API nv_status nv_batch_set_schedule(nv_batch *batch, const nv_batch_schedule *sched) try {
    if (!batch) return fail(NV_ERR_INVALID_ARG, "batch is NULL");
    nv_status s = check_schedule(sched);
    if (s != NV_OK) return s;
    return apply_schedule(batch, *sched);
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_batch_set_schedule: host allocation failed");
}

NV_API nv_status nv_batch_get_schedule(const nv_batch *batch, nv_batch_schedule *sched) {
    if (!batch || !sched) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    *sched = batch->sched;
    return NV_OK;
}

NV_API nv_status nv_batch_autotune(nv_batch *b, int reps, nv_batch_schedule *chosen) try {
    if (!b) return fail(NV_ERR_INVALID_ARG, "batch is NULL");
    if (reps < 1) return fail(NV_ERR_INVALID_ARG, "reps must be >= 1");
    const nv_batch_schedule before = b->sched;
    nv_status s = autotune(b, reps, chosen);
    if (s != NV_OK) {
        const std::string msg = nv_last_error();
        (void)apply_schedule(b, before);
        return fail(s, "%s", msg.c_str());
    }
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_batch_autotune: host allocation failed");
}

NV_API nv_status nv_batch_run(nv_batch *b, double *yT, nv_compose_info *info) try {
    if (!b || !yT) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    nv_status s = ensure_graph(b);
    if (s != NV_OK) return s;
    b->timed = false;
    NV_HIP(hipEventRecord(b->ev0, b->stream));
    NV_HIP(hipGraphLaunch(b->exec, b->stream));
    NV_HIP(hipEventRecord(b->ev1, b->stream));
    NV_HIP(hipStreamSynchronize(b->stream));
    b->timed = true;
    b->ran = true;
    const auto *st = static_cast<const nv::ComposeStatus *>(b->stage);
    const auto *res = reinterpret_cast<const double *>(static_cast<const char *>(b->stage) +
                                                       (b->off_result - b->off_status));
    int first_bad = -1;
    for (int i = 0; i < b->count; ++i) {
        yT[2 * i] = res[2 * i];
        yT[2 * i + 1] = dim_of(b->problems[i]) == 2 ? res[2 * i + 1] : 0.0;
        if (info) {
            info[i].n_out_of_grid = st[i].n_out_of_grid;
            info[i].bad_slice = st[i].bad_slice;
            info[i].n_chunks = 1;
        }
        if (!st[i].done) return fail(NV_ERR_HIP, "problem %d: composition did not complete", i);
        if (st[i].bad_slice >= 0 && first_bad < 0) first_bad = i;
    }
    if (first_bad >= 0)
        return fail(NV_ERR_NONFINITE, "problem %d met a non-finite value in slice %d", first_bad,
                    st[first_bad].bad_slice);
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_batch_run: host allocation failed");
}

NV_API nv_status nv_batch_last_timing(nv_batch *b, float *run_ms, long long *traj_steps) {
    if (!b) return fail(NV_ERR_INVALID_ARG, "batch is NULL");
    if (run_ms) {
        *run_ms = -1.0f;
        if (b->timed) NV_HIP(hipEventElapsedTime(run_ms, b->ev0, b->ev1));
    }
    if (traj_steps) *traj_steps = b->traj_steps;
    return NV_OK;
}

NV_API nv_status nv_batch_get_table(nv_batch *b, int problem, int component, void *host_dst,
                                    size_t bytes) try {
    if (!b || !host_dst) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (problem < 0 || problem >= b->count) return fail(NV_ERR_INVALID_ARG, "bad problem index");
    if (component < 0 || component >= dim_of(b->problems[problem]))
        return fail(NV_ERR_INVALID_ARG, "bad component");
    if (!b->ran) return fail(NV_ERR_NOT_BUILT, "the batch has not been run");
    const size_t need = b->elems[problem] * (b->precision == NV_FP64 ? 8 : 4);
    if (bytes < need) return fail(NV_ERR_BUFFER_TOO_SMALL, "need %zu bytes", need);
    NV_HIP(hipMemcpyAsync(host_dst,
                          b->tables + b->tab_off[problem] + component * b->comp_bytes[problem],
                          need, hipMemcpyDeviceToHost, b->stream));
    NV_HIP(hipStreamSynchronize(b->stream));
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_batch_get_table: host allocation failed");
}

NV_API nv_status nv_batch_get_boundary(nv_batch *b, int problem, double *host_dst,
                                       size_t count) try {
    if (!b || !host_dst) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (problem < 0 || problem >= b->count) return fail(NV_ERR_INVALID_ARG, "bad problem index");
    const nv_problem &p = b->problems[problem];
    const size_t need = (size_t(p.n_slices) + 1) * size_t(dim_of(p));
    if (count < need) return fail(NV_ERR_BUFFER_TOO_SMALL, "need %zu values", need);
    if (!b->ran) return fail(NV_ERR_NOT_BUILT, "the batch has not been run");
    NV_HIP(hipMemcpyAsync(host_dst, b->work + b->off_boundary + b->bnd_off[problem],
                          need * sizeof(double), hipMemcpyDeviceToHost, b->stream));
    NV_HIP(hipStreamSynchronize(b->stream));
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_batch_get_boundary: host allocation failed");
}

}  // extern "C"

nv_status nv::batch_slice_sources(nv_batch *b, std::vector<SliceMapSource> &out,
                                  int *precision) {
    if (!b) return fail(NV_ERR_INVALID_ARG, "batch is NULL");
    if (!b->ran) return fail(NV_ERR_NOT_BUILT, "the batch has not been run");
    out.clear();
    long long first = 0;
    for (int i = 0; i < b->count; ++i) {
        const nv_problem &p = b->problems[i];
        if (p.rhs_id != NV_RHS_VDP || p.grid.dim != 2)
            return fail(NV_ERR_INVALID_ARG, "problem %d is not a 2-D Van der Pol problem", i);
        const BuildArgs &a = b->hp[i].build;
        SliceMapSource s{};
        s.tab0 = a.tab0;
        s.tab1 = a.tab1;
        s.M = a.M;
        s.n1 = a.n1;
        s.n_slices = p.n_slices;
        s.lo0 = a.lo0;
        s.dxi0 = a.dxi0;
        s.lo1 = a.lo1;
        s.dxi1 = a.dxi1;
        s.t0 = p.t0;
        s.L = (p.T - p.t0) / double(p.n_slices);
        s.mu = p.params[0];
        s.first = first;
        first += a.M * (long long)p.n_slices;
        out.push_back(s);
    }
    *precision = b->precision;
    return NV_OK;
}
