// Affine basis propagator for the heat equation of sec. 6 (include/nv_linear.h).
//
// Computation phase, two launches:
//   lin_coef_kernel   one thread per (slice, step): the Thomas coefficients
//                     w_i, c_i of that step's tridiagonal matrix (a chain of M
//                     divisions that every solve of the slice shares);
//   lin_build_kernel  one workgroup per slice, one lane per solve: lane 0 the
//                     forced solve from 0, lane k the homogeneous solve from
//                     e_k; each lane's vector lives in LDS (column-major, so
//                     the lanes' accesses are consecutive), and no lane ever
//                     waits for another.
// Communication phase: lin_compose_kernel, one workgroup; lane i owns
// component i of lambda and forms c_i + G_i1 l_1 + ... from the table stored
// column by column (coalesced reads); boundary states are collected in LDS
// and written out per chunk so that no store sits in the chain.
#include "nv_internal.h"
#include "nv_linear.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

using nv::fail;

#define NV_HIP(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(NV_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

namespace {

constexpr int kMaxM = NV_LIN_MAX_POINTS;

struct CoefArgs {
    const double *step;         // [n_slices * S_tot][2]: r, h beta
    double *w, *c;              // [n_slices * S_tot][M]
    long long count;            // n_slices * S_tot
    int M;
};

__global__ __launch_bounds__(256) void lin_coef_kernel(CoefArgs a) {
#pragma clang fp contract(off)
    const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
    if (q >= a.count) return;
    const double r = a.step[2 * q];
    const double diag = 1.0 + 2.0 * r, off = -r;
    double cp = 0.0;
    for (int i = 0; i < a.M; ++i) {
        const double den = i == 0 ? diag : diag - off * cp;
        const double w = 1.0 / den;
        cp = off * w;
        a.w[q * a.M + i] = w;
        a.c[q * a.M + i] = cp;
    }
}

// Device table of slice j: T[j][k M + i] = G_j[i][k] (column-major), then
// T[j][M M + i] = c_j[i]; one contiguous block of M (M + 1) values per slice.
struct BuildArgs {
    const double *step;         // [n_slices * S_tot][2]
    const double *w, *c;        // [n_slices * S_tot][M]
    const double *s;            // [M] sin(pi x_i)
    double *T;                  // [n_slices][M (M + 1)]
    int M, S_tot, forcing;
};

__global__ __launch_bounds__(256) void lin_build_kernel(BuildArgs a) {
#pragma clang fp contract(off)
    extern __shared__ double xs[];           // [M][ncol]
    const int ncol = int(blockDim.x), lane = int(threadIdx.x), M = a.M;
    const int j = int(blockIdx.x);
    const bool live = lane <= M;             // lane 0: forced solve; lane k: from e_k
    const bool forced = lane == 0 && a.forcing;
    for (int i = 0; i < M; ++i) xs[i * ncol + lane] = (lane >= 1 && i == lane - 1) ? 1.0 : 0.0;
    for (int st = 0; st < a.S_tot; ++st) {
        const long long q = (long long)j * a.S_tot + st;
        const double off = -a.step[2 * q], hb = a.step[2 * q + 1];
        const double *w = a.w + q * M, *c = a.c + q * M;
        // forward elimination, in place
        double fp = 0.0;
        for (int i = 0; i < M; ++i) {
            double f = xs[i * ncol + lane];
            if (forced) f = f + hb * a.s[i];
            fp = i == 0 ? f * w[0] : (f - off * fp) * w[i];
            xs[i * ncol + lane] = fp;
        }
        // back substitution, in place
        double y = fp;
        for (int i = M - 2; i >= 0; --i) {
            y = xs[i * ncol + lane] - c[i] * y;
            xs[i * ncol + lane] = y;
        }
    }
    if (!live) return;
    double *blk = a.T + (long long)j * M * (M + 1);
    double *col = lane == 0 ? blk + M * M : blk + (lane - 1) * M;
    for (int i = 0; i < M; ++i) col[i] = xs[i * ncol + lane];
}

struct ComposeArgs {
    const double *T;            // [N][M (M + 1)]
    const double *y0;           // device [M]
    double *boundary;           // device [(N+1)][M]
    int *bad;                   // first slice whose state is not finite, or -1
    int M, N;
};

// The chain reads every table value once, in slice order, so the tables of a
// chunk of CH slices (CH M (M + 1) values) are staged in LDS and the next
// chunk is loaded into registers while the current one is composed: no
// global memory operation sits in the dependent chain.  Lane i < M owns
// component i, formed from eight interleaved partial sums (the order written
// in include/nv_linear.h), every term read from LDS (the table column-major,
// so lanes read consecutive words).  The state is
// double-buffered in LDS, so one barrier per slice suffices; a single wave
// serves M <= 63.
constexpr int kLinRegs = 64;                           // per-thread share of a chunk
constexpr int kLinMaxChunk = 16;                       // slices per chunk (boundary buffer)

template <int NT>
__global__ __launch_bounds__(NT) void lin_compose_kernel(ComposeArgs a) {
#pragma clang fp contract(off)
    constexpr int kStage = NT * kLinRegs;              // doubles
    __shared__ double stage[kStage];
    __shared__ double lam[2][kMaxM];
    __shared__ double bnd[kLinMaxChunk][kMaxM];
    __shared__ int bad_s;
    const int tid = int(threadIdx.x), M = a.M, N = a.N;
    const int MM = M * M, per = MM + M;
    const int CH = kStage / per < kLinMaxChunk ? kStage / per : kLinMaxChunk;
    const bool row = tid < M;
    if (row) {
        lam[0][tid] = a.y0[tid];
        a.boundary[tid] = a.y0[tid];
    }
    if (tid == 0) bad_s = 0x7fffffff;
    {
        const int count = (CH < N ? CH : N) * per;
        for (int v = tid; v < count; v += NT) stage[v] = a.T[v];
    }
    double regs[kLinRegs];
    for (int c0 = 0; c0 < N; c0 += CH) {
        const int cn = c0 + CH <= N ? CH : N - c0;
        const int n0 = c0 + CH, nn = n0 < N ? (n0 + CH <= N ? CH : N - n0) : 0;
        const int nT = nn * per;
        __syncthreads();                               // chunk c0 is in LDS
        if (nT > 0) {
            // the next chunk, in flight meanwhile: every load unconditional from a
            // clamped index, so that no wait separates them
            const double *src = a.T + (long long)n0 * per;
#pragma unroll
            for (int r = 0; r < kLinRegs; ++r) {
                const int v = tid + r * NT;
                regs[r] = src[v < nT ? v : nT - 1];
            }
        }
        for (int js = 0; js < cn; ++js) {
            const int cur = (c0 + js) & 1;
            if (row) {
                const double *G = stage + js * per;
                const double *l = lam[cur];
                // eight interleaved partial sums (k mod 8), then a fixed tree
                double p[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
                int k = 0;
                for (; k + 8 <= M; k += 8) {
#pragma unroll
                    for (int r = 0; r < 8; ++r) p[r] = p[r] + G[(k + r) * M + tid] * l[k + r];
                }
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (k + r < M) p[r] = p[r] + G[(k + r) * M + tid] * l[k + r];
                const double acc =
                    G[MM + tid] + (((p[0] + p[1]) + (p[2] + p[3])) + ((p[4] + p[5]) + (p[6] + p[7])));
                lam[cur ^ 1][tid] = acc;
                bnd[js][tid] = acc;
            }
            __syncthreads();                           // the new state is complete
        }
        if (row) {
            for (int js = 0; js < cn; ++js) {
                const double v = bnd[js][tid];
                a.boundary[(long long)(c0 + js + 1) * M + tid] = v;
                if (!isfinite(v)) atomicMin(&bad_s, c0 + js);
            }
        }
        __syncthreads();                               // chunk c0 is consumed
        if (nT > 0) {
#pragma unroll
            for (int r = 0; r < kLinRegs; ++r) {
                const int v = tid + r * NT;
                if (v < nT) stage[v] = regs[r];
            }
        }
    }
    __syncthreads();
    if (tid == 0) *a.bad = bad_s == 0x7fffffff ? -1 : bad_s;
}

}  // namespace

struct nv_lin {
    hipStream_t stream = nullptr;
    char *mem = nullptr;
    size_t mem_bytes = 0;
    // layout of the last build
    double *step = nullptr, *w = nullptr, *c = nullptr, *s = nullptr, *T = nullptr,
           *y0 = nullptr, *boundary = nullptr;
    int *bad = nullptr;
    int M = 0, N = 0, S_tot = 0;
    bool built = false;
    hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
    float build_ms = 0.f, compose_ms = 0.f;
};

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// FP64 host evaluations with one rounding per operation.
double a_of(const nv_heat &p, double t) {
#pragma clang fp contract(off)
    return p.a0 + p.a1 * std::sin(t);
}

double beta_of(const nv_heat &p, double t) {
#pragma clang fp contract(off)
    return ((M_PI * M_PI) * a_of(p, t)) * std::cos(t) - std::sin(t);
}

}  // namespace

extern "C" {

NV_API nv_status nv_lin_create(void *stream, nv_lin **out) {
    if (!out) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    nv_lin *l = new (std::nothrow) nv_lin();
    if (!l) return fail(NV_ERR_OOM, "out of host memory");
    l->stream = static_cast<hipStream_t>(stream);
    hipError_t e = hipEventCreate(&l->e0);
    if (e == hipSuccess) e = hipEventCreate(&l->e1);
    if (e == hipSuccess) e = hipEventCreate(&l->e2);
    if (e == hipSuccess) e = hipEventCreate(&l->e3);
    if (e != hipSuccess) {
        nv_lin_destroy(l);
        return fail(NV_ERR_HIP, "event creation failed: %s", hipGetErrorString(e));
    }
    *out = l;
    return NV_OK;
}

NV_API nv_status nv_lin_destroy(nv_lin *l) {
    if (!l) return NV_OK;
    if (l->mem) {
        (void)hipStreamSynchronize(l->stream);
        (void)hipFree(l->mem);
    }
    for (hipEvent_t ev : {l->e0, l->e1, l->e2, l->e3})
        if (ev) (void)hipEventDestroy(ev);
    delete l;
    return NV_OK;
}

NV_API nv_status nv_lin_build(nv_lin *l, const nv_heat *p, double t0, double T, int n_slices,
                              double dt) {
#pragma clang fp contract(off)
    if (!l || !p) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    l->built = false;                        // a failed build leaves nothing to compose
    if (p->M < 1 || p->M > kMaxM)
        return fail(NV_ERR_INVALID_ARG, "M = %d: need 1..%d interior points", p->M, kMaxM);
    if (n_slices < 1) return fail(NV_ERR_INVALID_ARG, "n_slices = %d", n_slices);
    if (!std::isfinite(t0) || !std::isfinite(T) || !(T > t0))
        return fail(NV_ERR_INVALID_ARG, "need finite t0 < T");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(NV_ERR_INVALID_ARG, "dt must be > 0");
    if (!std::isfinite(p->a0) || !std::isfinite(p->a1))
        return fail(NV_ERR_INVALID_ARG, "a0, a1 must be finite");
    const int M = p->M;
    const double L = (T - t0) / double(n_slices);
    const double Sd = std::floor(L / dt + 1e-9);
    if (Sd > 1e7) return fail(NV_ERR_INVALID_ARG, "more than 1e7 steps per slice");
    const int S = int(Sd);
    double rem = L - double(S) * dt;
    if (!(rem > 1e-12 * L)) rem = 0.0;
    const int S_tot = S + (rem > 0.0 ? 1 : 0);
    if (S_tot < 1) return fail(NV_ERR_INVALID_ARG, "a slice takes no step");
    const long long nq = (long long)n_slices * S_tot;
    // per-step scalars on the host: r = (h a(t_end)) / (dx dx), h beta(t_end)
    const double dx = 1.0 / double(M + 1);
    std::vector<double> step(size_t(nq) * 2), sv(M);
    for (int j = 0; j < n_slices; ++j) {
        const double Tj = t0 + double(j) * L;
        for (int st = 0; st < S_tot; ++st) {
            const bool last = st == S;
            const double h = last ? rem : dt;
            const double te = last ? (Tj + double(S) * dt) + rem : Tj + double(st + 1) * dt;
            const double a = a_of(*p, te);
            if (!(a > 0.0))
                return fail(NV_ERR_INVALID_ARG, "a(t) = %g is not positive at t = %g", a, te);
            const size_t q = size_t(j) * S_tot + st;
            step[2 * q] = (h * a) / (dx * dx);
            step[2 * q + 1] = p->forcing ? h * beta_of(*p, te) : 0.0;
        }
    }
    for (int i = 0; i < M; ++i) sv[i] = std::sin(M_PI * (double(i + 1) * dx));

    // device layout
    size_t off = 0;
    const size_t o_step = off; off = al(off + size_t(nq) * 2 * 8);
    const size_t o_w = off;    off = al(off + size_t(nq) * M * 8);
    const size_t o_c = off;    off = al(off + size_t(nq) * M * 8);
    const size_t o_s = off;    off = al(off + size_t(M) * 8);
    const size_t o_T = off;    off = al(off + size_t(n_slices) * M * (M + 1) * 8);
    const size_t o_y0 = off;   off = al(off + size_t(M) * 8);
    const size_t o_b = off;    off = al(off + (size_t(n_slices) + 1) * M * 8);
    const size_t o_bad = off;  off = al(off + sizeof(int));
    if (off > l->mem_bytes) {
        if (l->mem) {
            NV_HIP(hipStreamSynchronize(l->stream));
            NV_HIP(hipFree(l->mem));
            l->mem = nullptr;
            l->mem_bytes = 0;
        }
        if (hipMalloc(reinterpret_cast<void **>(&l->mem), off) != hipSuccess) {
            l->built = false;
            return fail(NV_ERR_OOM, "device allocation of %zu bytes failed", off);
        }
        l->mem_bytes = off;
    }
    l->step = reinterpret_cast<double *>(l->mem + o_step);
    l->w = reinterpret_cast<double *>(l->mem + o_w);
    l->c = reinterpret_cast<double *>(l->mem + o_c);
    l->s = reinterpret_cast<double *>(l->mem + o_s);
    l->T = reinterpret_cast<double *>(l->mem + o_T);
    l->y0 = reinterpret_cast<double *>(l->mem + o_y0);
    l->boundary = reinterpret_cast<double *>(l->mem + o_b);
    l->bad = reinterpret_cast<int *>(l->mem + o_bad);
    l->M = M;
    l->N = n_slices;
    l->S_tot = S_tot;
    l->built = false;

    NV_HIP(hipMemcpyAsync(l->step, step.data(), step.size() * 8, hipMemcpyHostToDevice,
                          l->stream));
    NV_HIP(hipMemcpyAsync(l->s, sv.data(), sv.size() * 8, hipMemcpyHostToDevice, l->stream));
    NV_HIP(hipEventRecord(l->e0, l->stream));
    CoefArgs ca{l->step, l->w, l->c, nq, M};
    hipLaunchKernelGGL(lin_coef_kernel, dim3(unsigned((nq + 255) / 256)), dim3(256), 0,
                       l->stream, ca);
    NV_HIP(hipGetLastError());
    BuildArgs ba{l->step, l->w, l->c, l->s, l->T, M, S_tot, p->forcing ? 1 : 0};
    const int ncol = 64 * ((M + 1 + 63) / 64);
    const size_t lds = size_t(M) * ncol * sizeof(double);     // at most 127 x 128 x 8 bytes
    NV_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(lin_build_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
    hipLaunchKernelGGL(lin_build_kernel, dim3(unsigned(n_slices)), dim3(ncol), lds, l->stream,
                       ba);
    NV_HIP(hipGetLastError());
    NV_HIP(hipEventRecord(l->e1, l->stream));
    // the host vectors must outlive the copies
    NV_HIP(hipStreamSynchronize(l->stream));
    NV_HIP(hipEventElapsedTime(&l->build_ms, l->e0, l->e1));
    l->built = true;
    return NV_OK;
}

NV_API nv_status nv_lin_compose(nv_lin *l, const double *y0, double *yT, double *boundary) {
    if (!l || !y0 || !yT) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (!l->built) return fail(NV_ERR_NOT_BUILT, "no successful nv_lin_build");
    const int M = l->M, N = l->N;
    NV_HIP(hipMemcpyAsync(l->y0, y0, size_t(M) * 8, hipMemcpyHostToDevice, l->stream));
    NV_HIP(hipEventRecord(l->e2, l->stream));
    ComposeArgs a{l->T, l->y0, l->boundary, l->bad, M, N};
    if (M <= 63)
        hipLaunchKernelGGL(lin_compose_kernel<64>, dim3(1), dim3(64), 0, l->stream, a);
    else
        hipLaunchKernelGGL(lin_compose_kernel<256>, dim3(1), dim3(256), 0, l->stream, a);
    NV_HIP(hipGetLastError());
    NV_HIP(hipEventRecord(l->e3, l->stream));
    int bad = -1;
    NV_HIP(hipMemcpyAsync(&bad, l->bad, sizeof(int), hipMemcpyDeviceToHost, l->stream));
    NV_HIP(hipMemcpyAsync(yT, l->boundary + size_t(N) * M, size_t(M) * 8, hipMemcpyDeviceToHost,
                          l->stream));
    if (boundary)
        NV_HIP(hipMemcpyAsync(boundary, l->boundary, (size_t(N) + 1) * M * 8,
                              hipMemcpyDeviceToHost, l->stream));
    NV_HIP(hipStreamSynchronize(l->stream));
    NV_HIP(hipEventElapsedTime(&l->compose_ms, l->e2, l->e3));
    if (bad >= 0) return fail(NV_ERR_NONFINITE, "the state became non-finite in slice %d", bad);
    return NV_OK;
}

NV_API nv_status nv_lin_get_tables(nv_lin *l, double *G, double *c) {
    if (!l) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (!l->built) return fail(NV_ERR_NOT_BUILT, "no successful nv_lin_build");
    const size_t M = size_t(l->M), N = size_t(l->N), per = M * (M + 1);
    std::vector<double> t(N * per);
    NV_HIP(hipMemcpyAsync(t.data(), l->T, t.size() * 8, hipMemcpyDeviceToHost, l->stream));
    NV_HIP(hipStreamSynchronize(l->stream));
    for (size_t j = 0; j < N; ++j) {
        const double *b = t.data() + j * per;
        if (G)
            for (size_t k = 0; k < M; ++k)
                for (size_t i = 0; i < M; ++i) G[(j * M + i) * M + k] = b[k * M + i];
        if (c)
            for (size_t i = 0; i < M; ++i) c[j * M + i] = b[M * M + i];
    }
    return NV_OK;
}

NV_API nv_status nv_lin_last_timing(nv_lin *l, float *build_ms, float *compose_ms) {
    if (!l) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (build_ms) *build_ms = l->build_ms;
    if (compose_ms) *compose_ms = l->compose_ms;
    return NV_OK;
}

}  // extern "C"
