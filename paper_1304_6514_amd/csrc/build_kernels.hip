// Computation phase of Nievergelt's method (sec. 3, pseudocode figure): every
// (slice, grid point) pair integrates its own initial value problem over the
// slice, fully independently, and stores the end state in the slice's table.
//
// gfx950 mapping
//   - one trajectory per lane (P trajectories per lane for instruction-level
//     parallelism), state in VGPRs, no LDS, no inter-lane traffic;
//   - one workgroup covers 256*P consecutive grid points of ONE slice, so the
//     slice index, its start time and its forcing values are wave-uniform and
//     live in SGPRs (scalar loads from the per-slice forcing row);
//   - workgroup ids are remapped so that each of the 8 XCDs runs a contiguous
//     range of slices (its L2 then holds those slices' forcing rows);
//   - the grid point is computed from the lane's index (no load); the only
//     HBM traffic is the coalesced table store at the end.
//
// The inner loop is VALU-bound: RK4 on y' = F(t) - y^3 costs 15 VALU ops per
// step (+3 with Kahan-compensated FP32 accumulation, +1 with blocked
// summation), Van der Pol 26 (+6, +2).
#include "integrate.h"

namespace nv {
namespace {
using namespace dev;

// The workgroup's count of non-finite end states, stored in its tile's own
// word (the host sums a slice's tiles), so no counter is cleared before a
// build.
__device__ inline void store_tile_count(const BuildArgs &a, int j, int tile, unsigned bad) {
    __shared__ unsigned count;
    if (threadIdx.x == 0) count = 0;
    __syncthreads();
    if (bad) atomicAdd(&count, bad);
    __syncthreads();
    if (threadIdx.x == 0) a.nonfinite[(long long)j * a.tiles_per_slice + tile] = count;
}

// Start time of slice j, T_j = t0 + j L: the product rounded, then the sum,
// never one fused operation, so that every kernel that forms a forcing row
// sees the same T_j.
__device__ inline double slice_start(double t0, long long j, double L) {
#pragma clang fp contract(off)
    return t0 + double(j) * L;
}

// Entry m of slice j's forcing row: the right-hand side's forcing at
// T_j + (m/2) h, plus h/2 for odd m (the step's start, midpoint and end times),
// in FP64, rounded once.
template <class R>
__device__ inline R forcing_entry(int rhs, double Tj, long long m, double h) {
#pragma clang fp contract(off)
    double t = Tj + double(m >> 1) * h;
    if (m & 1) t = t + h / 2.0;
    return R(forcing_value(rhs, t));
}

template <class Rhs, class R, int Scheme, int A, int P>
__global__ void __launch_bounds__(kBuildBlock) build_kernel(BuildArgs a) {
    const int lid = xcd_remap(int(blockIdx.x), a.total_blocks);
    const int j = a.slice0 + lid / a.tiles_per_slice, tile = lid % a.tiles_per_slice;
    const unsigned bad = build_tile<Rhs, R, Scheme, A, P>(a, j, tile);
    store_tile_count(a, j, tile, bad);
}

// The same for small builds of a right-hand side with forcing: each workgroup
// forms its slice's forcing row in LDS (dynamic, 2 steps + 1 values) before
// integrating, so no forcing launch precedes the build.  The values are those
// of forcing_kernel, entry for entry.
template <class Rhs, class R, int Scheme, int A, int P>
__global__ void __launch_bounds__(kBuildBlock) build_local_forcing_kernel(BuildArgs a) {
    extern __shared__ unsigned char forcing_lds[];
    R *F = reinterpret_cast<R *>(forcing_lds);
    const int lid = xcd_remap(int(blockIdx.x), a.total_blocks);
    const int j = a.slice0 + lid / a.tiles_per_slice, tile = lid % a.tiles_per_slice;
    const long long per = 2LL * a.steps + 1;
    const double Tj = slice_start(a.t0, j, a.L);
    for (long long m = threadIdx.x; m < per; m += kBuildBlock)
        F[m] = forcing_entry<R>(Rhs::rhs_id, Tj, m, a.h);
    __syncthreads();
    const unsigned bad = build_tile_rows<Rhs, R, Scheme, A, P>(a, j, tile, F);
    store_tile_count(a, j, tile, bad);
}

// Forcing values of slice j at the stage times of its steps:
// F[j][2s] = g(T_j + s h), F[j][2s+1] = g((T_j + s h) + h/2), F[j][2S] = g(T_j + S h).
template <class R>
__global__ void forcing_kernel(int rhs, R *F, int n_slices, int steps, double t0, double L,
                               double h) {
#pragma clang fp contract(off)
    const long long per = 2LL * steps + 1;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= per * n_slices) return;
    const long long j = idx / per, m = idx - j * per;
    F[idx] = forcing_entry<R>(rhs, slice_start(t0, j, L), m, h);
}

__global__ void fill_u32_kernel(uint32_t *p, long long n, uint32_t v) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <class Rhs, class R, int Scheme, int A, int P>
hipError_t launch_one(const BuildArgs &a, hipStream_t s) {
    if constexpr (Rhs::forced) {
        if (a.local_forcing) {
            const size_t lds = size_t(2LL * a.steps + 1) * sizeof(R);
            hipLaunchKernelGGL((build_local_forcing_kernel<Rhs, R, Scheme, A, P>),
                               dim3(a.total_blocks), dim3(kBuildBlock), lds, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((build_kernel<Rhs, R, Scheme, A, P>), dim3(a.total_blocks),
                       dim3(kBuildBlock), 0, s, a);
    return hipGetLastError();
}

template <template <class> class Rhs, class R, int Scheme, int A>
hipError_t by_p(int P, const BuildArgs &a, hipStream_t s) {
    switch (P) {
    case 1: return launch_one<Rhs<R>, R, Scheme, A, 1>(a, s);
    case 2: return launch_one<Rhs<R>, R, Scheme, A, 2>(a, s);
    case 4: return launch_one<Rhs<R>, R, Scheme, A, 4>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <template <class> class Rhs, class R, int A>
hipError_t by_scheme(const BuildConfig &c, const BuildArgs &a, hipStream_t s) {
    switch (c.scheme) {
    case 0: return by_p<Rhs, R, 0, A>(c.traj_per_lane, a, s);
    case 1: return by_p<Rhs, R, 1, A>(c.traj_per_lane, a, s);
    case 2:
        if constexpr (Rhs<R>::dim == 1) return by_p<Rhs, R, 2, A>(c.traj_per_lane, a, s);
        return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
    }
}

template <template <class> class Rhs>
hipError_t by_config(const BuildConfig &c, const BuildArgs &a, hipStream_t s) {
    if (c.precision == 0) return by_scheme<Rhs, double, kPlain>(c, a, s);
    switch (c.compensated) {
    case 0: return by_scheme<Rhs, float, kPlain>(c, a, s);
    case 1: return by_scheme<Rhs, float, kKahan>(c, a, s);
    case 2: return by_scheme<Rhs, float, kBlocked>(c, a, s);
    default: return hipErrorInvalidValue;
    }
}

// The one-dimensional right-hand sides with their variational equations
// (builds that also store slopes).
template <class R> using LinearSlopes = RhsTangent<RhsLinear, R>;
template <class R> using LogisticSlopes = RhsTangent<RhsLogistic, R>;
template <class R> using ForcedCubicSlopes = RhsTangent<RhsForcedCubic, R>;
template <class R> using SquareSlopes = RhsTangent<RhsSquare, R>;

}  // namespace

bool build_supported(const BuildConfig &c) {
    return c.rhs >= 0 && c.rhs <= 4 && (c.scheme >= 0 && c.scheme <= 2) &&
           !(c.scheme == 2 && c.rhs == 3) &&
           (c.precision == 0 || c.precision == 1) &&
           (c.compensated >= 0 && c.compensated <= 2) &&
           (c.traj_per_lane == 1 || c.traj_per_lane == 2 || c.traj_per_lane == 4) &&
           !(c.slopes && (c.rhs == 3 || c.scheme == 2));
}

hipError_t launch_build(const BuildConfig &c, const BuildArgs &a, hipStream_t s) {
    if (c.slopes) {
        switch (c.rhs) {
        case 0: return by_config<LinearSlopes>(c, a, s);
        case 1: return by_config<LogisticSlopes>(c, a, s);
        case 2: return by_config<ForcedCubicSlopes>(c, a, s);
        case 4: return by_config<SquareSlopes>(c, a, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (c.rhs) {
    case 0: return by_config<RhsLinear>(c, a, s);
    case 1: return by_config<RhsLogistic>(c, a, s);
    case 2: return by_config<RhsForcedCubic>(c, a, s);
    case 3: return by_config<RhsVdp>(c, a, s);
    case 4: return by_config<RhsSquare>(c, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forcing(int rhs, int precision, void *F, int n_slices, int steps,
                          double t0, double L, double h, hipStream_t s) {
    const long long n = (2LL * steps + 1) * n_slices;
    const int block = 256;
    const long long grid = (n + block - 1) / block;
    if (precision == 0)
        hipLaunchKernelGGL(forcing_kernel<double>, dim3(unsigned(grid)), dim3(block), 0, s, rhs,
                           static_cast<double *>(F), n_slices, steps, t0, L, h);
    else
        hipLaunchKernelGGL(forcing_kernel<float>, dim3(unsigned(grid)), dim3(block), 0, s, rhs,
                           static_cast<float *>(F), n_slices, steps, t0, L, h);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, long long n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int block = 256;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(unsigned((n + block - 1) / block)), dim3(block), 0,
                       s, p, n, v);
    return hipGetLastError();
}

}  // namespace nv
