// Affine basis propagator for the heat equation of sec. 6 (include/nv_linear.h).
//
// Computation phase, two launches:
//   lin_coef_kernel   one thread per (slice, step): the Thomas coefficients
//                     w_i, c_i of that step's tridiagonal matrix (a chain of M
//                     divisions that every solve of the slice shares);
//   lin_build_reg_kernel<MP> (M <= 104) / lin_build_kernel (larger M)
//                     one workgroup per slice, one lane per solve: lane 0 the
//                     forced solve from 0, lane k the homogeneous solve from
//                     e_k; each lane's vector lives in registers (the sweeps
//                     unrolled over MP rows) or, for the largest M, in LDS,
//                     and the step's coefficients are staged in LDS.
// Communication phase: lin_chain_kernel, one workgroup of eight waves, wave r
// forming the partial sums of residue r of the fixed summation order for
// every component from table values prefetched into its registers several
// slices ahead; one LDS exchange and one barrier per slice.
#include "nv_internal.h"
#include "nv_linear.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <utility>
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

// Device table of slice j: T[j][k Ms + i] = G_j[i][k] (column-major), then
// T[j][M Ms + i] = c_j[i], with the column stride Ms = M rounded up to even
// (the padding row holds 0.0): one contiguous block of Ms (M + 1) values per
// slice, every column 16-byte aligned.
struct BuildArgs {
    const double *step;         // [n_slices * S_tot][2]
    const double *w, *c;        // [n_slices * S_tot][M]
    const double *s;            // [M] sin(pi x_i)
    double *T;                  // [n_slices][Ms (M + 1)]
    int M, S_tot, forcing;
};

__host__ __device__ inline int lin_stride(int M) { return M + (M & 1); }

// LDS of lin_build_kernel, in doubles: the lanes' vectors xs[M][M + 1]
// (lane k's vector is column k, so the lanes of a wave touch consecutive
// words), two buffers of one step's Thomas coefficients (w then c, M each)
// and sin(pi x_i).
inline size_t lin_build_lds_bytes(int M) { return size_t(M) * (M + 6) * sizeof(double); }

// The coefficients of the step being solved are read from LDS (a broadcast
// read whose address does not depend on the recurrence, so it can be issued
// ahead of it); those of the next step are loaded into registers meanwhile
// and published to the other buffer at the end of the step.
__global__ __launch_bounds__(128) void lin_build_kernel(BuildArgs a) {
#pragma clang fp contract(off)
    constexpr int kPre = 2;                  // ceil(M / 64) for M <= 127
    constexpr int kLook = 4;                 // rows read ahead of the recurrences
    extern __shared__ double lds[];
    const int nt = int(blockDim.x), lane = int(threadIdx.x), M = a.M, ncol = M + 1;
    double *xs = lds, *wc = lds + M * ncol, *ss = wc + 4 * M;
    const int j = int(blockIdx.x);
    const bool live = lane <= M;             // lane 0: forced solve; lane k: from e_k
    const bool forced = lane == 0 && a.forcing;
    const long long q0 = (long long)j * a.S_tot;
    if (live)
        for (int i = 0; i < M; ++i) xs[i * ncol + lane] = (lane >= 1 && i == lane - 1) ? 1.0 : 0.0;
    for (int v = lane; v < M; v += nt) {
        ss[v] = a.s[v];
        wc[v] = a.w[q0 * M + v];
        wc[M + v] = a.c[q0 * M + v];
    }
    __syncthreads();
    for (int st = 0; st < a.S_tot; ++st) {
        const long long q = q0 + st;
        const double off = -a.step[2 * q], hb = a.step[2 * q + 1];
        // the next step's coefficients (the last step reloads its own), every
        // load unconditional from a clamped index
        const long long qn = st + 1 < a.S_tot ? q + 1 : q;
        double pw[kPre], pc[kPre];
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int v = lane + u * nt < M ? lane + u * nt : M - 1;
            pw[u] = a.w[qn * M + v];
            pc[u] = a.c[qn * M + v];
        }
        const double *w = wc + (st & 1) * 2 * M, *c = w + M;
        if (live) {
            // Both sweeps read the rows, coefficients and sin values kLook rows
            // ahead of the recurrence into a register ring (the row read ahead
            // is written only later, when the sweep reaches it; a clamped index
            // past the end reads a value that is never used).
            double fr[kLook], wr[kLook], sr[kLook];
#pragma unroll
            for (int u = 0; u < kLook; ++u) {
                const int iu = u < M ? u : M - 1;
                fr[u] = xs[iu * ncol + lane];
                wr[u] = w[iu];
                sr[u] = ss[iu];
            }
            // forward elimination, in place
            double fp = 0.0;
            for (int i0 = 0; i0 < M; i0 += kLook) {
#pragma unroll
                for (int u = 0; u < kLook; ++u) {
                    const int i = i0 + u;
                    if (i < M) {
                        double f = fr[u];
                        const double wi = wr[u], si = sr[u];
                        const int in = i + kLook < M ? i + kLook : M - 1;
                        fr[u] = xs[in * ncol + lane];
                        wr[u] = w[in];
                        sr[u] = ss[in];
                        if (forced) f = f + hb * si;
                        fp = i == 0 ? f * wi : (f - off * fp) * wi;
                        xs[i * ncol + lane] = fp;
                    }
                }
            }
            // back substitution, in place, rows M - 2 down to 0
#pragma unroll
            for (int u = 0; u < kLook; ++u) {
                const int iu = M - 2 - u >= 0 ? M - 2 - u : 0;
                fr[u] = xs[iu * ncol + lane];
                wr[u] = c[iu];
            }
            double y = fp;
            for (int i0 = M - 2; i0 >= 0; i0 -= kLook) {
#pragma unroll
                for (int u = 0; u < kLook; ++u) {
                    const int i = i0 - u;
                    if (i >= 0) {
                        const double xi = fr[u], ci = wr[u];
                        const int in = i - kLook >= 0 ? i - kLook : 0;
                        fr[u] = xs[in * ncol + lane];
                        wr[u] = c[in];
                        y = xi - ci * y;
                        xs[i * ncol + lane] = y;
                    }
                }
            }
        }
        double *wn = wc + ((st + 1) & 1) * 2 * M;
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int v = lane + u * nt;
            if (v < M) {
                wn[v] = pw[u];
                wn[M + v] = pc[u];
            }
        }
        __syncthreads();
    }
    if (!live) return;
    const int Ms = lin_stride(M);
    double *blk = a.T + (long long)j * Ms * (M + 1);
    double *col = lane == 0 ? blk + Ms * M : blk + (lane - 1) * Ms;
    for (int i = 0; i < M; ++i) col[i] = xs[i * ncol + lane];
    if (Ms > M) col[M] = 0.0;
}

// The same solves with each lane's vector in registers, for M <= MP: the
// sweeps are unrolled over MP rows, so every row is a register of its own,
// and LDS holds only the coefficients, which lets four workgroups share a CU
// instead of one.  The staged coefficients are padded with zeros to MP rows,
// so that every row reads its coefficient at a fixed offset; rows M .. MP-1 of
// the forward sweep then hold zeros that no row below M reads, and the back
// substitution starts at row M - 1 by a test on the wave-uniform M.  The
// operations on rows 0 .. M-1 are those of lin_build_kernel, in the same order.
template <int MP>
__global__ __launch_bounds__(128) void lin_build_reg_kernel(BuildArgs a) {
#pragma clang fp contract(off)
    constexpr int kPre = (MP + 63) / 64;     // staged rows per lane
    __shared__ double wc[2][2][MP];          // [buffer][w, c][row]
    __shared__ double ss[MP];
    const int nt = int(blockDim.x), lane = int(threadIdx.x), M = a.M;
    const int j = int(blockIdx.x);
    const bool live = lane <= M;             // lane 0: forced solve; lane k: from e_k
    const bool forced = lane == 0 && a.forcing;
    const long long q0 = (long long)j * a.S_tot;
    double x[MP];
#pragma unroll
    for (int i = 0; i < MP; ++i) x[i] = (lane >= 1 && i == lane - 1) ? 1.0 : 0.0;
    for (int v = lane; v < MP; v += nt) {
        ss[v] = v < M ? a.s[v] : 0.0;
        wc[0][0][v] = v < M ? a.w[q0 * M + v] : 0.0;
        wc[0][1][v] = v < M ? a.c[q0 * M + v] : 0.0;
    }
    __syncthreads();
    for (int st = 0; st < a.S_tot; ++st) {
        const long long q = q0 + st;
        const double off = -a.step[2 * q], hb = a.step[2 * q + 1];
        const long long qn = st + 1 < a.S_tot ? q + 1 : q;
        double pw[kPre], pc[kPre];
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int v = lane + u * nt < M ? lane + u * nt : M - 1;
            pw[u] = a.w[qn * M + v];
            pc[u] = a.c[qn * M + v];
        }
        const double *w = wc[st & 1][0], *c = wc[st & 1][1];
        // forward elimination
        double fp = 0.0;
#pragma unroll
        for (int i = 0; i < MP; ++i) {
            double f = x[i];
            if (forced) f = f + hb * ss[i];
            fp = i == 0 ? f * w[0] : (f - off * fp) * w[i];
            x[i] = fp;
        }
        // back substitution from row M - 1
        double y = 0.0;
#pragma unroll
        for (int i = MP - 1; i >= 0; --i) {
            if (i == M - 1) {
                y = x[i];
            } else if (i < M - 1) {
                y = x[i] - c[i] * y;
                x[i] = y;
            }
        }
        double(*wn)[MP] = wc[(st + 1) & 1];
#pragma unroll
        for (int u = 0; u < kPre; ++u) {
            const int v = lane + u * nt;
            if (v < MP) {
                wn[0][v] = v < M ? pw[u] : 0.0;
                wn[1][v] = v < M ? pc[u] : 0.0;
            }
        }
        __syncthreads();
    }
    if (!live) return;
    const int Ms = lin_stride(M);
    double *blk = a.T + (long long)j * Ms * (M + 1);
    double *col = lane == 0 ? blk + Ms * M : blk + (lane - 1) * Ms;
#pragma unroll
    for (int i = 0; i < MP; ++i)
        if (i < M) col[i] = x[i];
    if (Ms > M) col[M] = 0.0;
}

struct ComposeArgs {
    const double *T;            // [N][Ms (M + 1)]
    const double *y0;           // device [M]
    double *boundary;           // device [(N+1)][M]
    int *bad;                   // first slice whose state is not finite, or -1
    int M, N;
};

__device__ inline double lin_readlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(b & 0xffffffffLL), l));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(b >> 32), l));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// third word of a buffer resource on gfx9-family chips (32-bit data format,
// no swizzle): raw buffer loads then read num_records bytes from the base
constexpr int kBufferWord3 = 0x00020000;

// The chain, built around the summation order itself.  Wave r (r = 0..7)
// forms the partial sums p_r = G_i,r l_r + G_i,r+8 l_r+8 + ... (left to right
// from 0) of every component i, lane l taking the two rows 2l and 2l + 1 (so
// one wave covers M <= 128), from table values that were loaded straight into
// its registers D slices ahead: per slice, KM = ceil(M/8) 16-byte loads of a
// row pair (column fragments of 128 consecutive doubles per wave: coalesced,
// and no table value passes through LDS).  The partial sums go to LDS; after
// the one barrier of the slice, lane m < KM of wave r combines the eight
// partial sums of component r + 8m in the fixed tree and adds c, which yields
// exactly the new state components that wave r needs for the next slice, and
// v_readlane hands them to the whole wave.  The partial-sum buffer is double
// buffered, so one barrier per slice suffices.  Each wave stores its own
// components of the boundary states; a store is always younger than the loads
// the next slices wait for, so it never delays them (the memory counter is in
// order).
template <int KM, int D>
__global__ __launch_bounds__(512) void lin_chain_kernel(ComposeArgs a) {
#pragma clang fp contract(off)
    constexpr int kRow = 128;
    __shared__ double part[2][8][kRow];
    __shared__ int bad_s;
    const int tid = int(threadIdx.x), lane = tid & 63;
    const int r = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int M = a.M, N = a.N, Ms = lin_stride(M), per = Ms * (M + 1);
    const int mr = r < M ? (M - r + 7) / 8 : 0;        // components k = r + 8m < M
    const int i2 = 2 * lane;                           // the lane's first row
    // byte offsets within a slice block: column k starts at the wave-uniform
    // k Ms, the lane adds its (16-byte aligned) row pair; c of component
    // r + 8 lane for lanes < mr
    const unsigned row_b = unsigned(i2 < M ? i2 : Ms - 2) * 8u;
    const unsigned c_b = unsigned(Ms * M + (lane < mr ? r + 8 * lane : M - 1)) * 8u;
    // Terms past mr (components r + 8m >= M; only when KM > mr) take the state
    // value +0.0 (here, and from the broadcast of lanes >= mr, whose v stays
    // 0.0) and the table value of column M - 1; their product is then +-0.0 for
    // a finite table, and since p starts at +0.0 it is never -0.0, so adding
    // +-0.0 leaves p unchanged to the bit: no per-term condition is needed.  (A
    // non-finite value in column M - 1 makes that row non-finite in the exact
    // sum as well, in the same slice.)
    double lam[KM];
#pragma unroll
    for (int m = 0; m < KM; ++m) {
        const int k = r + 8 * m;
        lam[m] = k < M ? a.y0[k] : 0.0;
    }
    if (tid < M) a.boundary[tid] = a.y0[tid];
    if (tid == 0) bad_s = 0x7fffffff;

    double2 g[D][KM];
    double cv[D];
    // Raw buffer loads over the slice's block, every one unconditional, from a
    // clamped slice index: the column offset k Ms is a scalar operand and the
    // lane's row pair a 32-bit vector offset, so no load needs an address
    // register of its own (and the hardware checks the block's bounds).  The
    // slice index passes through readfirstlane so that the compiler keeps one
    // scalar base instead of strength-reducing every load into an address
    // register.
#define NV_LIN_FETCH(slot, s)                                                            \
    do {                                                                                 \
        const int s_ = __builtin_amdgcn_readfirstlane((s) < N ? (s) : N - 1);            \
        const __amdgpu_buffer_rsrc_t rs_ = __builtin_amdgcn_make_buffer_rsrc(            \
            (void *)(a.T + (long long)s_ * per), 0, per * 8, kBufferWord3);              \
        _Pragma("unroll") for (int m = 0; m < KM; ++m) {                                 \
            const int col_ = (r + 8 * m < M ? r + 8 * m : M - 1) * Ms * 8;               \
            g[slot][m] = __builtin_bit_cast(                                             \
                double2, __builtin_amdgcn_raw_buffer_load_b128(rs_, int(row_b), col_, 0)); \
        }                                                                                \
        cv[slot] = __builtin_bit_cast(double,                                            \
                                      __builtin_amdgcn_raw_buffer_load_b64(rs_, int(c_b), 0, 0)); \
    } while (0)
    // first half of a slice: the partial sums of the lane's two rows, to LDS
#define NV_LIN_PARTIAL(slot, j)                                                          \
    do {                                                                                 \
        double p0 = 0.0, p1 = 0.0;                                                       \
        _Pragma("unroll") for (int m = 0; m < KM; ++m) {                                 \
            p0 = p0 + g[slot][m].x * lam[m];                                             \
            p1 = p1 + g[slot][m].y * lam[m];                                             \
        }                                                                                \
        if (i2 < M) part[(j) & 1][r][i2] = p0;                                           \
        if (i2 + 1 < M) part[(j) & 1][r][i2 + 1] = p1;                                   \
    } while (0)
    // second half: after the barrier, the new components r + 8m and their
    // broadcast; nothing is stored for the slices past N
#define NV_LIN_COMBINE(c_now, j)                                                         \
    do {                                                                                 \
        __syncthreads();                                                                 \
        double v = 0.0;                                                                  \
        if (lane < mr) {                                                                 \
            const int k = r + 8 * lane;                                                  \
            const double *q = &part[(j) & 1][0][k];                                      \
            const double s = ((q[0] + q[kRow]) + (q[2 * kRow] + q[3 * kRow])) +          \
                             ((q[4 * kRow] + q[5 * kRow]) + (q[6 * kRow] + q[7 * kRow])); \
            v = (c_now) + s;                                                             \
            if ((j) < N) {                                                               \
                a.boundary[(long long)((j) + 1) * M + k] = v;                            \
                if (!isfinite(v)) atomicMin(&bad_s, (j));                                \
            }                                                                            \
        }                                                                                \
        _Pragma("unroll") for (int m = 0; m < KM; ++m) lam[m] = lin_readlane(v, m);      \
    } while (0)

#pragma unroll
    for (int d = 0; d < D; ++d) NV_LIN_FETCH(d, d);
    // whole groups of D slices: the up to D - 1 slices past N of the last group
    // repeat the clamped table of slice N - 1 and store nothing, which keeps
    // the loop free of a tail (a tail's extra copy of the body doubles the
    // register demand)
    for (int j0 = 0; j0 < N; j0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            NV_LIN_PARTIAL(d, j0 + d);
            const double c_now = cv[d];
            // slot d is consumed: refill it while the other waves reach the
            // barrier (not hoisted above the products, which would hold old and
            // new values of the slot at once)
            __builtin_amdgcn_sched_barrier(0);
            NV_LIN_FETCH(d, j0 + d + D);
            NV_LIN_COMBINE(c_now, j0 + d);
        }
    }
#undef NV_LIN_FETCH
#undef NV_LIN_PARTIAL
#undef NV_LIN_COMBINE
    __syncthreads();
    if (tid == 0) *a.bad = bad_s == 0x7fffffff ? -1 : bad_s;
}

// prefetch depth for KM loads per slice: a ring of about 72 doubles per lane
// (120 for the largest tables, KM >= 10, where a deeper ring measured faster),
// at least 2 and at most 8 slices ahead
constexpr int lin_depth(int KM) {
    const int ring = KM >= 10 ? 120 : 72, d = ring / (2 * KM + 1);
    return d < 2 ? 2 : (d > 8 ? 8 : d);
}

template <int KM>
void lin_launch_chain(const ComposeArgs &a, hipStream_t st) {
    hipLaunchKernelGGL((lin_chain_kernel<KM, lin_depth(KM)>), dim3(1), dim3(512), 0, st, a);
}

using LinLaunch = void (*)(const ComposeArgs &, hipStream_t);
template <int... K>
constexpr void lin_fill(LinLaunch *t, std::integer_sequence<int, K...>) {
    ((t[K] = &lin_launch_chain<K + 1>), ...);
}

// lin_chain[KM - 1] launches the chain for ceil(M/8) = KM
struct LinChainTable {
    LinLaunch f[16];
    LinChainTable() { lin_fill(f, std::make_integer_sequence<int, 16>{}); }
};
const LinChainTable lin_chain;

// ---- many initial values: the chain as FP64 matrix products -------------
//
// Q chains lambda^q_{j+1} = c_j + G_j lambda^q_j are independent, so workgroup
// b carries the 16 CB chains q = 16 CB b .. 16 CB b + 16 CB - 1 through every
// slice alone (no synchronisation between workgroups): per slice the product
// G_j Lambda_j of the M x M table with the M x 16 CB block of states, on the
// matrix cores (v_mfma_f64_16x16x4f64: wave w forms rows 16 w .. 16 w + 15 of
// the product, k = 0 .. 4 KP - 1 in steps of four, each A fragment of G
// multiplied with the CB 16-column blocks of states), then c_j added.
// Lambda_j lives in LDS, double buffered (rows k >= M are zero), one barrier
// per slice; every wave holds the A fragments of its rows of G_{j+1} in
// registers while it computes slice j.  Every workgroup reads all N tables, so
// the tables' traffic from the caches is (Q / 16 CB) x N x M (M + 1) doubles:
// CB = 2 halves it for large Q.
struct ManyArgs {
    const double *T;            // [N][Ms (M + 1)]
    const double *y0;           // [Q][M]
    double *yT;                 // [Q][M]
    double *boundary;           // [Q][N+1][M] or null
    int *bad;                   // first slice whose state is not finite (atomic min), or -1
    long long Q;
    int M, N;
};

typedef double v4d __attribute__((ext_vector_type(4)));

template <int KP, int CB>
__global__ __launch_bounds__(512) void lin_many_kernel(ManyArgs a) {
#pragma clang fp contract(off)
    constexpr int K = 4 * KP;                    // rows of Lambda in LDS (M <= K)
    constexpr int C = 16 * CB;                   // chains of the workgroup
    __shared__ double lam[2][K][C];
    const int tid = int(threadIdx.x), lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int M = a.M, N = a.N, Ms = lin_stride(M), per = Ms * (M + 1);
    const int col = lane & 15, kq = lane >> 4;
    const long long q0 = (long long)blockIdx.x * C;
    for (int e = tid; e < 2 * K * C; e += 512) {
        const int buf = e / (K * C), k = (e / C) % K, c = e % C;
        const long long qq = q0 + c < a.Q ? q0 + c : a.Q - 1;
        lam[buf][k][c] = (buf == 0 && k < M) ? a.y0[qq * M + k] : 0.0;
        if (a.boundary && buf == 0 && k < M && q0 + c < a.Q)
            a.boundary[(q0 + c) * (long long)(N + 1) * M + k] = a.y0[qq * M + k];
    }
    // the lane's A operand: row 16 w + col of G, columns 4 kk + kq (A[i][k] in
    // lane i + 16 k), B[k][j] in lane j + 16 k; the FP64 16 x 16 accumulator
    // interleaves its rows: lane l holds D[4 i + l/16][l % 16] (i = 0..3,
    // measured on the device), so the lane's outputs are rows 16 w + 4 i + kq
    // of chain column col of each column block
    const int arow = 16 * w + col;
    const bool active = 16 * w < M;
    bool live[CB];
    long long q[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        q[cb] = q0 + 16 * cb + col;
        live[cb] = q[cb] < a.Q;
    }
    // the A fragments and the c values of a slice, loaded unconditionally from
    // clamped (in-block) addresses, with no select after the load (which would
    // wait for it): a column k >= M meets the zero row k of Lambda, a row
    // >= M of the product is never stored.  Two register sets in turn, so that
    // a slice's operands were loaded during the previous slice and nothing
    // waits for the prefetch.  (A non-finite table value in column M - 1 thus
    // also reaches the padded terms; it makes its row non-finite in the exact
    // sum as well.)
    double ga[KP], gb[KP], ca[4], cb4[4];
#define NV_LIN_LOAD(g, cv, j)                                                            \
    do {                                                                                 \
        const double *Tj_ = a.T + (long long)(j) * per;                                  \
        const int ar_ = arow < M ? arow : M - 1;                                         \
        _Pragma("unroll") for (int kk = 0; kk < KP; ++kk) {                              \
            const int k_ = 4 * kk + kq;                                                  \
            g[kk] = Tj_[(k_ < M ? k_ : M - 1) * Ms + ar_];                               \
        }                                                                                \
        _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                  \
            const int r_ = 16 * w + 4 * i + kq;                                          \
            cv[i] = Tj_[Ms * M + (r_ < M ? r_ : M - 1)];                                 \
        }                                                                                \
    } while (0)
    // one slice: the product on the matrix cores (even and odd k-steps in two
    // accumulators per column block), c added, the new states to LDS (and the
    // boundary), barrier
#define NV_LIN_SLICE(g, cv, j)                                                           \
    do {                                                                                 \
        if (active) {                                                                    \
            v4d acc[CB], acc1[CB];                                                       \
            _Pragma("unroll") for (int cb = 0; cb < CB; ++cb) {                          \
                acc[cb] = v4d{0.0, 0.0, 0.0, 0.0};                                       \
                acc1[cb] = v4d{0.0, 0.0, 0.0, 0.0};                                      \
            }                                                                            \
            _Pragma("unroll") for (int kk = 0; kk < KP; ++kk) {                          \
                _Pragma("unroll") for (int cb = 0; cb < CB; ++cb) {                      \
                    const double b_ = lam[cur][4 * kk + kq][16 * cb + col];              \
                    if (kk % 2 == 0)                                                     \
                        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[kk], b_, acc[cb],   \
                                                                       0, 0, 0);         \
                    else                                                                 \
                        acc1[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(g[kk], b_, acc1[cb], \
                                                                        0, 0, 0);        \
                }                                                                        \
            }                                                                            \
            _Pragma("unroll") for (int cb = 0; cb < CB; ++cb) {                          \
                const v4d s_ = acc[cb] + acc1[cb];                                       \
                _Pragma("unroll") for (int i = 0; i < 4; ++i) {                          \
                    const int r = 16 * w + 4 * i + kq;                                   \
                    const double v = cv[i] + s_[i];                                      \
                    if (r < M) {                                                         \
                        lam[cur ^ 1][r][16 * cb + col] = v;                              \
                        if (live[cb] && a.boundary)                                      \
                            a.boundary[(q[cb] * (N + 1) + (j) + 1) * (long long)M + r] = v;  \
                        if (live[cb] && !isfinite(v) && (j) < bad) bad = (j);            \
                    }                                                                    \
                }                                                                        \
            }                                                                            \
        }                                                                                \
        __syncthreads();                                                                 \
        cur ^= 1;                                                                        \
    } while (0)
    int cur = 0, bad = 0x7fffffff;
    if (active) NV_LIN_LOAD(ga, ca, 0);
    __syncthreads();
    for (int j = 0; j < N; j += 2) {
        if (active) NV_LIN_LOAD(gb, cb4, j + 1 < N ? j + 1 : N - 1);
        NV_LIN_SLICE(ga, ca, j);
        if (j + 1 >= N) break;
        if (active) NV_LIN_LOAD(ga, ca, j + 2 < N ? j + 2 : N - 1);
        NV_LIN_SLICE(gb, cb4, j + 1);
    }
#undef NV_LIN_LOAD
#undef NV_LIN_SLICE
    for (int e = tid; e < M * C; e += 512) {
        const int k = e / C, c = e % C;
        if (q0 + c < a.Q) a.yT[(q0 + c) * M + k] = lam[cur][k][c];
    }
    if (bad != 0x7fffffff) atomicMin(a.bad, bad);
}

// With enough chains for two workgroups of two column blocks on every CU, a
// workgroup carries two blocks that share its table reads; fewer chains keep
// one block per workgroup, for more workgroups (measured at M = 99, N = 1024:
// 16,384 chains 9.1 -> 7.4 ms paired, 4096 chains 2.5 -> 3.7 ms).  Two blocks
// need more registers: up to KP = 29 (M <= 116) the kernel holds them without
// spilling.
constexpr int kManyPairMaxKP = 29;

template <int KP>
void lin_launch_many(const ManyArgs &a, long long pair_from, hipStream_t st) {
    if constexpr (KP <= kManyPairMaxKP) {
        if (a.Q >= pair_from) {
            hipLaunchKernelGGL((lin_many_kernel<KP, 2>), dim3(unsigned((a.Q + 31) / 32)),
                               dim3(512), 0, st, a);
            return;
        }
    }
    hipLaunchKernelGGL((lin_many_kernel<KP, 1>), dim3(unsigned((a.Q + 15) / 16)), dim3(512), 0,
                       st, a);
}

using ManyLaunch = void (*)(const ManyArgs &, long long, hipStream_t);
template <int... K>
constexpr void many_fill(ManyLaunch *t, std::integer_sequence<int, K...>) {
    ((t[K] = &lin_launch_many<K + 1>), ...);
}

// lin_many[KP - 1] launches the product chain for ceil(M/4) = KP
struct LinManyTable {
    ManyLaunch f[32];
    LinManyTable() { many_fill(f, std::make_integer_sequence<int, 32>{}); }
};
const LinManyTable lin_many;

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
// a(t) = a0 + a1 sin t and beta(t) = ((pi pi) a(t)) cos t - sin t from one
// evaluation of sin t and cos t (the same values as evaluating them anew)
struct StepCoef {
    double a, beta;
};

StepCoef coef_at(const nv_heat &p, double t) {
#pragma clang fp contract(off)
    const double sn = std::sin(t), cs = std::cos(t);
    const double a = p.a0 + p.a1 * sn;
    return {a, ((M_PI * M_PI) * a) * cs - sn};
}

// The per-step scalars r = (h a(t_end)) / (dx dx) and h beta(t_end) of slices
// [j0, j1); returns the first step (global index) whose a(t) is not positive,
// or -1, with its time in *bad_t.
long long step_scalars(const nv_heat &p, double t0, double L, double dt, int S, double rem,
                       int S_tot, double dx, int j0, int j1, double *step, double *bad_t) {
#pragma clang fp contract(off)
    for (int j = j0; j < j1; ++j) {
        const double Tj = t0 + double(j) * L;
        for (int st = 0; st < S_tot; ++st) {
            const bool last = st == S;
            const double h = last ? rem : dt;
            const double te = last ? (Tj + double(S) * dt) + rem : Tj + double(st + 1) * dt;
            const StepCoef k = coef_at(p, te);
            const long long q = (long long)j * S_tot + st;
            if (!(k.a > 0.0)) {
                *bad_t = te;
                return q;
            }
            step[2 * q] = (h * k.a) / (dx * dx);
            step[2 * q + 1] = p.forcing ? h * k.beta : 0.0;
        }
    }
    return -1;
}

}  // namespace

extern "C" {

NV_API nv_status nv_lin_create(void *stream, nv_lin **out) try {
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
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_lin_create: host allocation failed");
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
                              double dt) try {
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
    {
        // slices split over a few host threads when there are many steps
        const unsigned hc = std::thread::hardware_concurrency();
        const int nth = nq < 8192 ? 1 : int(hc < 2 ? 1 : (hc > 8 ? 8 : hc));
        std::vector<long long> bad_q(size_t(nth), -1);
        std::vector<double> bad_t(size_t(nth), 0.0);
        auto part = [&](int k) {
            const int j0 = int((long long)n_slices * k / nth);
            const int j1 = int((long long)n_slices * (k + 1) / nth);
            bad_q[size_t(k)] = step_scalars(*p, t0, L, dt, S, rem, S_tot, dx, j0, j1, step.data(),
                                            &bad_t[size_t(k)]);
        };
        std::vector<std::thread> pool;
        for (int k = 1; k < nth; ++k) pool.emplace_back(part, k);
        part(0);
        for (std::thread &t : pool) t.join();
        for (int k = 0; k < nth; ++k)
            if (bad_q[size_t(k)] >= 0)
                return fail(NV_ERR_INVALID_ARG, "a(t) = %g is not positive at t = %g",
                            coef_at(*p, bad_t[size_t(k)]).a, bad_t[size_t(k)]);
    }
    for (int i = 0; i < M; ++i) sv[i] = std::sin(M_PI * (double(i + 1) * dx));

    // device layout
    size_t off = 0;
    const size_t o_step = off; off = al(off + size_t(nq) * 2 * 8);
    const size_t o_w = off;    off = al(off + size_t(nq) * M * 8);
    const size_t o_c = off;    off = al(off + size_t(nq) * M * 8);
    const size_t o_s = off;    off = al(off + size_t(M) * 8);
    const size_t o_T = off;    off = al(off + size_t(n_slices) * lin_stride(M) * (M + 1) * 8);
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
    const int ncol = 64 * ((M + 1 + 63) / 64);                // threads: one per solve
    const dim3 grid{unsigned(n_slices)}, block{unsigned(ncol)};
    if (M <= 8) hipLaunchKernelGGL(lin_build_reg_kernel<8>, grid, block, 0, l->stream, ba);
    else if (M <= 16) hipLaunchKernelGGL(lin_build_reg_kernel<16>, grid, block, 0, l->stream, ba);
    else if (M <= 24) hipLaunchKernelGGL(lin_build_reg_kernel<24>, grid, block, 0, l->stream, ba);
    else if (M <= 32) hipLaunchKernelGGL(lin_build_reg_kernel<32>, grid, block, 0, l->stream, ba);
    else if (M <= 48) hipLaunchKernelGGL(lin_build_reg_kernel<48>, grid, block, 0, l->stream, ba);
    else if (M <= 64) hipLaunchKernelGGL(lin_build_reg_kernel<64>, grid, block, 0, l->stream, ba);
    else if (M <= 80) hipLaunchKernelGGL(lin_build_reg_kernel<80>, grid, block, 0, l->stream, ba);
    else if (M <= 104) hipLaunchKernelGGL(lin_build_reg_kernel<104>, grid, block, 0, l->stream, ba);
    else {
        const size_t lds = lin_build_lds_bytes(M);             // at most 127 x 133 x 8 bytes
        NV_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(lin_build_kernel),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, int(lds)));
        hipLaunchKernelGGL(lin_build_kernel, grid, block, lds, l->stream, ba);
    }
    NV_HIP(hipGetLastError());
    NV_HIP(hipEventRecord(l->e1, l->stream));
    // the host vectors must outlive the copies
    NV_HIP(hipStreamSynchronize(l->stream));
    NV_HIP(hipEventElapsedTime(&l->build_ms, l->e0, l->e1));
    l->built = true;
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_lin_build: host allocation failed");
}

NV_API nv_status nv_lin_compose(nv_lin *l, const double *y0, double *yT, double *boundary) {
    if (!l || !y0 || !yT) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (!l->built) return fail(NV_ERR_NOT_BUILT, "no successful nv_lin_build");
    const int M = l->M, N = l->N;
    NV_HIP(hipMemcpyAsync(l->y0, y0, size_t(M) * 8, hipMemcpyHostToDevice, l->stream));
    NV_HIP(hipEventRecord(l->e2, l->stream));
    ComposeArgs a{l->T, l->y0, l->boundary, l->bad, M, N};
    lin_chain.f[(M + 7) / 8 - 1](a, l->stream);
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

NV_API nv_status nv_lin_compose_many(nv_lin *l, const double *y0_dev, long long count,
                                     double *yT_dev, double *boundary_dev) {
    if (!l || !y0_dev || !yT_dev) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (count < 1) return fail(NV_ERR_INVALID_ARG, "count = %lld", count);
    if ((count + 15) / 16 > 0x7fffffffLL) return fail(NV_ERR_INVALID_ARG, "too many chains");
    if (!l->built) return fail(NV_ERR_NOT_BUILT, "no successful nv_lin_build");
    const int M = l->M, N = l->N;
    const int init = 0x7fffffff;
    NV_HIP(hipMemcpyAsync(l->bad, &init, sizeof(int), hipMemcpyHostToDevice, l->stream));
    NV_HIP(hipEventRecord(l->e2, l->stream));
    ManyArgs a{l->T, y0_dev, yT_dev, boundary_dev, l->bad, count, M, N};
    int dev = 0, n_cu = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n_cu < 1)
        n_cu = 256;
    lin_many.f[(M + 3) / 4 - 1](a, 2LL * n_cu * 32, l->stream);
    NV_HIP(hipGetLastError());
    NV_HIP(hipEventRecord(l->e3, l->stream));
    int bad = init;
    NV_HIP(hipMemcpyAsync(&bad, l->bad, sizeof(int), hipMemcpyDeviceToHost, l->stream));
    NV_HIP(hipStreamSynchronize(l->stream));
    NV_HIP(hipEventElapsedTime(&l->compose_ms, l->e2, l->e3));
    if (bad != init)
        return fail(NV_ERR_NONFINITE, "a state became non-finite in slice %d", bad);
    return NV_OK;
}

NV_API nv_status nv_lin_get_tables(nv_lin *l, double *G, double *c) {
    if (!l) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (!l->built) return fail(NV_ERR_NOT_BUILT, "no successful nv_lin_build");
    const size_t M = size_t(l->M), N = size_t(l->N), Ms = size_t(lin_stride(l->M)),
                 per = Ms * (M + 1);
    std::vector<double> t(N * per);
    NV_HIP(hipMemcpyAsync(t.data(), l->T, t.size() * 8, hipMemcpyDeviceToHost, l->stream));
    NV_HIP(hipStreamSynchronize(l->stream));
    for (size_t j = 0; j < N; ++j) {
        const double *b = t.data() + j * per;
        if (G)
            for (size_t k = 0; k < M; ++k)
                for (size_t i = 0; i < M; ++i) G[(j * M + i) * M + k] = b[k * Ms + i];
        if (c)
            for (size_t i = 0; i < M; ++i) c[j * M + i] = b[Ms * M + i];
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
