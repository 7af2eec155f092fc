// Communication phase of Nievergelt's method (sec. 3, pseudocode figure):
// lambda_0 = y0, lambda_{j+1} = phi^j(lambda_j), one slice after the other.
//
// This is a chain of N dependent lookups (the N tau_N term of the cost model
// of sec. 4), so one wave runs it, in FP64, directly on the tables the build
// left in HBM; nothing is copied to the host but the N+1 boundary states.
//
// Every floating-point operation here is a single IEEE binary64 operation
// with no contraction: the lookup and the interpolants are specified bit for
// bit (see include/nv.h), so that a composition over given tables is exactly
// reproducible.
#include "compose.h"

namespace nv {
namespace {
using namespace dev;

template <class T, int Interp>
__global__ void compose_kernel(ComposeArgs a) {
    if (blockIdx.x != 0) return;
    // The chain usually shares its SIMD with waves of a build still running
    // (nv_solve overlaps them); the highest wave priority lets its dependent
    // instructions issue first instead of waiting behind those waves.
    __builtin_amdgcn_s_setprio(3);
    if constexpr (Interp == 3)
        compose_range_lagrange<T>(a);
    else
        compose_range<T, Interp>(a);
}

// The 1-D chain with its table windows staged in LDS by helper waves: one
// workgroup of 1 + kPfHelpers waves.
template <class T, int Interp>
__global__ __launch_bounds__(64 * (1 + kPfHelpers)) void compose_staged_kernel(ComposeArgs a) {
    __shared__ PfShared<Interp> sh;
    if (blockIdx.x != 0) return;
    compose_range_staged<T, Interp>(a, sh);
}

// The bilinear chain with its windows staged in LDS: one workgroup of
// 1 + kPfHelpers waves.
template <class T>
__global__ __launch_bounds__(64 * (1 + kPfHelpers)) void compose_staged2_kernel(ComposeArgs a) {
    __shared__ PfShared2 sh;
    if (blockIdx.x != 0) return;
    compose_range_staged2<T>(a, sh);
}

__global__ void locate_kernel(double lo, double inv, int n, const double *x, long long count,
                              long long *cell, double *w, int32_t *out) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    long long c;
    double ww;
    out[q] = locate(lo, inv, n, x[q], c, ww);
    cell[q] = c;
    w[q] = ww;
}

}  // namespace

hipError_t launch_compose(int interp, int precision, const ComposeArgs &a, hipStream_t s) {
    const dim3 grid(1), block(64), staged(64 * (1 + kPfHelpers));
    // cells and window origins of the staged bilinear chain are packed 16 bits per axis
    const bool staged2 = a.n0 <= kPf2MaxAxis && a.n1 <= kPf2MaxAxis;
    if (precision == 0) {
        switch (interp) {
        case 0: hipLaunchKernelGGL((compose_staged_kernel<double, 0>), grid, staged, 0, s, a); break;
        case 1: hipLaunchKernelGGL((compose_staged_kernel<double, 1>), grid, staged, 0, s, a); break;
        case 2:
            if (staged2)
                hipLaunchKernelGGL((compose_staged2_kernel<double>), grid, staged, 0, s, a);
            else
                hipLaunchKernelGGL((compose_kernel<double, 2>), grid, block, 0, s, a);
            break;
        case 3: hipLaunchKernelGGL((compose_kernel<double, 3>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((compose_staged_kernel<double, 4>), grid, staged, 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    } else {
        switch (interp) {
        case 0: hipLaunchKernelGGL((compose_staged_kernel<float, 0>), grid, staged, 0, s, a); break;
        case 1: hipLaunchKernelGGL((compose_staged_kernel<float, 1>), grid, staged, 0, s, a); break;
        case 2:
            if (staged2)
                hipLaunchKernelGGL((compose_staged2_kernel<float>), grid, staged, 0, s, a);
            else
                hipLaunchKernelGGL((compose_kernel<float, 2>), grid, block, 0, s, a);
            break;
        case 3: hipLaunchKernelGGL((compose_kernel<float, 3>), grid, block, 0, s, a); break;
        case 4: hipLaunchKernelGGL((compose_staged_kernel<float, 4>), grid, staged, 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t launch_locate(double lo, double inv, int n, const double *x, long long count,
                         long long *cell, double *w, int32_t *out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int block = 256;
    hipLaunchKernelGGL(locate_kernel, dim3(unsigned((count + block - 1) / block)), dim3(block),
                       0, s, lo, inv, n, x, count, cell, w, out);
    return hipGetLastError();
}

}  // namespace nv
