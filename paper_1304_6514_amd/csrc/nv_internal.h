// Library-internal declarations shared by the C ABI and the kernels of libnv.
// Not installed; the public interface is include/nv.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "nv.h"

namespace nv {

constexpr int kBuildBlock = 256;   // lanes per build workgroup (4 wave64s)
constexpr int kNumXcd = 8;         // MI355X: 8 XCDs, workgroups dispatched round-robin

// Arguments of the ensemble-integration kernel (one launch = the whole build).
struct BuildArgs {
    void *tab0;               // component 0 table, [n_slices][M] of the working type
    void *tab1;               // component 1 table (2-D problems, or the slopes) or null
    const void *forcing;      // [n_slices][2*steps+1] forcing values, or null
    uint32_t *nonfinite;      // single-problem build: [n_slices][tiles_per_slice] counts, one
                              // per tile, stored; batch: [n_slices] counters, added to
    double lo0, dxi0;         // axis 0: xi = lo0 + k0 * dxi0
    double lo1, dxi1;         // axis 1 (2-D)
    double h;                 // step
    double h_last;            // > 0: one more step of this size after the `steps` steps
    double p0;                // right-hand side parameter
    const double *nodes;      // Chebyshev nodes of axis 0 (replace lo0 + k dxi0), or null
    long long M;              // points per slice
    int n1;                   // points on axis 1 (1 for 1-D)
    int n_slices;             // slices of the whole build (forcing row count)
    int slice0;               // first slice of this launch
    int steps;
    int tiles_per_slice;      // workgroups per slice
    int total_blocks;         // (slices of this launch) * tiles_per_slice
    int local_forcing;        // 1: each workgroup forms its slice's forcing row in LDS
    double t0, L;             // T_j = t0 + j L (for local_forcing)
};

struct BuildConfig {
    int rhs;                  // nv_rhs_id
    int scheme;               // nv_scheme
    int precision;            // nv_precision
    int compensated;          // FP32 only: 0 plain, 1 Kahan, 2 blocked summation
    int traj_per_lane;        // 1, 2, 4
    int slopes;               // 1: also integrate the derivative with respect to the
                              // grid point and store it as component 1 (1-D problems)
};

// Status the composition kernel leaves in device memory.
struct ComposeStatus {
    long long n_out_of_grid;
    int bad_slice;
    int done;
};

struct ComposeArgs {
    const void *tab0;
    const void *tab1;
    double *boundary;         // [(n_slices+1) * dim], written only (may be host-mapped)
    ComposeStatus *status;    // device: the running status of the whole chain
    double *carry;            // device [2]: the state a range ends with, or null
    ComposeStatus *status_host;  // a copy of the final status, or null (may be host-mapped)
    long long M;
    int n_slices;
    int j_begin, j_end;       // slices this launch composes; lambda_{j_begin} is y0 when
                              // j_begin == 0, else the carry the previous range left
    int n0, n1;
    double lo0, inv0, lo1, inv1;   // inv = (n-1)/(hi-lo), computed on the host
    double hi0;                    // Chebyshev: the interval's upper end
    double dxi0;                   // stored slopes: the grid spacing (hi - lo)/(n - 1)
    const double *nodes;           // Chebyshev nodes (Lagrange lookup), or null
    double y00, y01;
};

// One problem of a batch, as the batched kernels see it.
struct BatchProblem {
    BuildArgs build;          // slice0 = 0; tables, counters and grid of this problem
    ComposeArgs compose;      // whole range of slices, this problem's y0
    int rhs;                  // nv_rhs_id (autonomous right-hand sides only)
    int interp;               // nv_interp
    int traj_per_lane;        // P of this problem's tiles
    int dim;
    double *result;           // [dim]: lambda_N, written after the composition
};

// One work item of the persistent build: a tile of 256*P grid points of one
// slice of one problem.
struct BatchItem {
    int problem;
    int slice;
    int tile;
    int reserved;
};

// One problem's tables seen as samples of its slice maps: sample (j, k) is
// grid point k of slice j, the slice starting at t0 + j L (training set of the
// learned surrogate).  first = number of the problem's first sample.
struct SliceMapSource {
    const void *tab0, *tab1;
    long long M;
    int n1, n_slices;
    double lo0, dxi0, lo1, dxi1;
    double t0, L, mu;
    long long first;
};

// The tables of a run batch of 2-D Van der Pol problems, problem by problem.
nv_status batch_slice_sources(nv_batch *b, std::vector<SliceMapSource> &out, int *precision);

bool build_supported(const BuildConfig &c);
hipError_t launch_build(const BuildConfig &c, const BuildArgs &a, hipStream_t s);
// The forcing rows of every slice (right-hand sides with forcing).
hipError_t launch_forcing(int rhs, int precision, void *F, int n_slices, int steps,
                          double t0, double L, double h, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, long long n, uint32_t v, hipStream_t s);
hipError_t launch_compose(int interp, int precision, const ComposeArgs &a, hipStream_t s);
hipError_t launch_locate(double lo, double inv, int n, const double *x, long long count,
                         long long *cell, double *w, int32_t *out, hipStream_t s);
hipError_t launch_batch_build(int precision, int accumulation, const BatchProblem *probs,
                              const BatchItem *items, int n_items, unsigned *counter,
                              int n_workgroups, hipStream_t s);
hipError_t launch_batch_compose(int precision, const BatchProblem *probs, int count,
                                hipStream_t s);

// Shared by the C-ABI translation units: record the calling thread's error
// message and return s; check one problem's description (host only).
nv_status fail(nv_status s, const char *fmt, ...);
nv_status check_problem(int rhs_id, const double *params, double t0, double T, int n_slices,
                        const nv_ic_grid *grid, int steps_per_slice);

}  // namespace nv
