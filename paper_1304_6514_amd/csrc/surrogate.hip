// Learned slice-map surrogate: training (forward and back-propagation on bf16
// matrix cores, weight-gradient sums, Adam), inference inside the composition,
// and the training set drawn from the tables of the computation phase.
#include "compose.h"
#include "mlp.h"
#include "nv_surrogate.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

using nv::fail;
using namespace nv::mlp;

#define NV_HIP(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(NV_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

namespace {

constexpr int kInferThreads = 256;       // 4 waves
constexpr int kMaxSplits = 128;          // weight-gradient sums: splits of the minibatch
constexpr long long kMinSplit = 512;      // samples per split, at least
constexpr long long kMaxBatch = 1LL << 20;

enum { kModeReduce = 1, kModeAdam = 2 };
constexpr int kMaxCoarse = 16;

// The coarse propagator G: k classical RK4 steps of length h of the Van der
// Pol field y1' = y2, y2' = mu (1 - y1^2) y2 - y1, in FP64 (k = 0: identity).
__host__ __device__ inline void coarse_rk4(double mu, double h, int k, double &y0, double &y1) {
#pragma clang fp contract(off)
    for (int s = 0; s < k; ++s) {
        const double a1 = y1, b1 = mu * (1.0 - y0 * y0) * y1 - y0;
        const double p0 = y0 + 0.5 * h * a1, p1 = y1 + 0.5 * h * b1;
        const double a2 = p1, b2 = mu * (1.0 - p0 * p0) * p1 - p0;
        const double q0 = y0 + 0.5 * h * a2, q1 = y1 + 0.5 * h * b2;
        const double a3 = q1, b3 = mu * (1.0 - q0 * q0) * q1 - q0;
        const double r0 = y0 + h * a3, r1 = y1 + h * b3;
        const double a4 = r1, b4 = mu * (1.0 - r0 * r0) * r1 - r0;
        y0 = y0 + (h / 6.0) * (((a1 + 2.0 * a2) + 2.0 * a3) + a4);
        y1 = y1 + (h / 6.0) * (((b1 + 2.0 * b2) + 2.0 * b3) + b4);
    }
}

// The step-doubling form's pieces at y: G1 (k RK4 steps of L / k), the
// difference d = G2 - G1 to 2k steps of half that length, and the gate
// g = d^2 / (d^2 + tau2), tau2 = gate^2, per component; FP64.
struct StepDoubling {
    double g0, g1, d0, d1, gt0, gt1;
};
__host__ __device__ inline StepDoubling step_doubling(double mu, double L, int k, double y0,
                                                      double y1, double tau2_0, double tau2_1) {
#pragma clang fp contract(off)
    StepDoubling r;
    double a0 = y0, a1 = y1, b0 = y0, b1 = y1;
    coarse_rk4(mu, L / double(k), k, a0, a1);
    coarse_rk4(mu, L / double(2 * k), 2 * k, b0, b1);
    r.g0 = a0;
    r.g1 = a1;
    r.d0 = b0 - a0;
    r.d1 = b1 - a1;
    const double dd0 = r.d0 * r.d0, dd1 = r.d1 * r.d1;
    r.gt0 = dd0 / (dd0 + tau2_0);
    r.gt1 = dd1 / (dd1 + tau2_1);
    return r;
}

// Richardson's constant of a fourth-order step: the error of G1 is about
// 16/15 (G2 - G1).
constexpr double kRichardson = 16.0 / 15.0;

// ---------------------------------------------------------------- kernels

struct TrainArgs {
    const float *x, *t;          // data set rows, ld samples each
    long long ld, start, n;      // minibatch = samples start .. start+n-1
    const float *params;
    const __bf16 *shadow;        // Wf2, Wf3, Wb2, Wb3 (permuted bf16)
    __bf16 *S;                   // workspace, kRowsS rows of ldS
    long long ldS;
    float *loss_part;            // one sum per 16 samples
    float shift[4], scale[4];
    float inv_n;
    int weighted;                // targets are rho_0, rho_1, w_0, w_1: e = w out - rho
};

// Weight-gradient sums G = A B^T over samples k0..k1-1 of the minibatch, A and
// B row blocks of S; blockIdx.y of the launch is the split of the sum.  In the
// small products each wave computes a 32 x 32 block (wave tiles
// kGemmSmallFirst.. of kGemmWaveTiles: D1 . XO^T, giving dW1 and db1, and
// XO . [H3; XO]^T, giving dW4 and db4; db2 and db3 are row sums that the
// 128 x 128 products form from the rows they stage anyway).
struct GemmArgs {
    const __bf16 *S;
    long long ldS, n, k_per_split;
    float *part;                 // [splits][kGradEntries]
};

__device__ inline void grad_small(const GemmArgs &a, int bx) {
    const int lane = int(threadIdx.x) & 63, r = lane & 15, g = lane >> 4;
    const int wt = kGemmSmallFirst + bx * 4 + (int(threadIdx.x) >> 6);
    if (wt >= kGemmWaveTiles) return;
    int a_row, b_row, M, N, out, t, tiles_n;
    if (wt < 16) {
        a_row = kRowD + 128; b_row = kRowH; M = N = 128; out = kG_W2; t = wt; tiles_n = 4;
    } else if (wt < 32) {
        a_row = kRowD + 256; b_row = kRowH + 128; M = N = 128; out = kG_W3; t = wt - 16;
        tiles_n = 4;
    } else if (wt < 36) {
        a_row = kRowD; b_row = kRowXO; M = 128; N = 16; out = kG_D_XO; t = wt - 32; tiles_n = 1;
    } else {
        a_row = kRowXO; b_row = kRowH + 256; M = 16; N = 144; out = kG_XO_H3; t = wt - 36;
        tiles_n = 5;
    }
    const int mt0 = 2 * (t / tiles_n), nt0 = 2 * (t % tiles_n);
    const bool m1 = mt0 + 1 < M / 16, n1 = nt0 + 1 < N / 16;
    const long long k0 = (long long)blockIdx.y * a.k_per_split;
    const long long k1 = std::min(k0 + a.k_per_split, a.n);
    const __bf16 *pa0 = a.S + (long long)(a_row + 16 * mt0 + r) * a.ldS + 8 * g;
    const __bf16 *pa1 = pa0 + 16 * a.ldS;
    const __bf16 *pb0 = a.S + (long long)(b_row + 16 * nt0 + r) * a.ldS + 8 * g;
    const __bf16 *pb1 = pb0 + 16 * a.ldS;
    f32x4 c00 = {0.f, 0.f, 0.f, 0.f}, c01 = c00, c10 = c00, c11 = c00;
    const bf16x8 zero = {};
    constexpr int U = 4;                         // k-steps of 32 samples per iteration
    long long k = k0;
    for (; k + 32 * U <= k1; k += 32 * U) {
        bf16x8 A0[U], A1[U], B0[U], B1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            A0[u] = *reinterpret_cast<const bf16x8 *>(pa0 + k + 32 * u);
            B0[u] = *reinterpret_cast<const bf16x8 *>(pb0 + k + 32 * u);
            A1[u] = m1 ? *reinterpret_cast<const bf16x8 *>(pa1 + k + 32 * u) : zero;
            B1[u] = n1 ? *reinterpret_cast<const bf16x8 *>(pb1 + k + 32 * u) : zero;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            c00 = mfma(A0[u], B0[u], c00);
            if (n1) c01 = mfma(A0[u], B1[u], c01);
            if (m1) c10 = mfma(A1[u], B0[u], c10);
            if (m1 && n1) c11 = mfma(A1[u], B1[u], c11);
        }
    }
    for (; k < k1; k += 32) {
        const bool ok = k + 8 * g < k1;          // the minibatch ends on a multiple of 16
        const bf16x8 A0 = ok ? *reinterpret_cast<const bf16x8 *>(pa0 + k) : zero;
        const bf16x8 B0 = ok ? *reinterpret_cast<const bf16x8 *>(pb0 + k) : zero;
        const bf16x8 A1 = (ok && m1) ? *reinterpret_cast<const bf16x8 *>(pa1 + k) : zero;
        const bf16x8 B1 = (ok && n1) ? *reinterpret_cast<const bf16x8 *>(pb1 + k) : zero;
        c00 = mfma(A0, B0, c00);
        if (n1) c01 = mfma(A0, B1, c01);
        if (m1) c10 = mfma(A1, B0, c10);
        if (m1 && n1) c11 = mfma(A1, B1, c11);
    }
    float *P = a.part + (long long)blockIdx.y * kGradEntries + out;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int row0 = 16 * mt0 + 4 * g + i, col0 = 16 * nt0 + r;
        P[row0 * N + col0] = c00[i];
        if (n1) P[row0 * N + col0 + 16] = c01[i];
        if (m1) P[(row0 + 16) * N + col0] = c10[i];
        if (m1 && n1) P[(row0 + 16) * N + col0 + 16] = c11[i];
    }
}

// The two 128 x 128 weight gradients, dW2 = D2 . H1^T and dW3 = D3 . H2^T
// (job 0, 1), over samples k0..k1-1 (blockIdx.y = split), and the
// bias gradients db2, db3, the row sums of D2 and D3.  The workgroup stages
// each 32-sample step of its 128 A rows and 128 B rows in LDS once (rows
// padded to 80 bytes: 16 lanes reading 16 bytes from 16 rows hit disjoint
// banks) and each wave multiplies a 64 x 64 quadrant; two threads per A row
// add its 32 staged values into FP32 row sums; the next step's rows are loaded
// into registers while the current one is multiplied.
constexpr int kGmPad = 40;                 // bf16 per LDS row

struct GradMatLds {
    __bf16 As[128 * kGmPad], Bs[128 * kGmPad];
};

__device__ inline void grad_mat(const GemmArgs &a, GradMatLds &L, int job) {
    __bf16 *As = L.As, *Bs = L.Bs;
    const int a_row = job == 0 ? kRowD + 128 : kRowD + 256;
    const int b_row = job == 0 ? kRowH : kRowH + 128;
    const int out = job == 0 ? kG_W2 : kG_W3;
    const int tid = int(threadIdx.x), lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4, mh = wave >> 1, nh = wave & 1;
    const long long k0 = (long long)blockIdx.y * a.k_per_split;
    const long long k1 = std::min(k0 + a.k_per_split, a.n);
    // this thread's share of a step: chunks tid and tid + 256 of 4 x 128 16-byte chunks
    const int row0 = tid >> 2, part0 = tid & 3, row1 = (tid + 256) >> 2, part1 = (tid + 256) & 3;
    const bf16x8 zero = {};
    auto load = [&](long long k, bf16x8 &a0, bf16x8 &a1, bf16x8 &b0, bf16x8 &b1) {
        const bool ok0 = k + 8 * part0 < k1, ok1 = k + 8 * part1 < k1;
        a0 = ok0 ? *reinterpret_cast<const bf16x8 *>(a.S + (long long)(a_row + row0) * a.ldS + k +
                                                     8 * part0) : zero;
        a1 = ok1 ? *reinterpret_cast<const bf16x8 *>(a.S + (long long)(a_row + row1) * a.ldS + k +
                                                     8 * part1) : zero;
        b0 = ok0 ? *reinterpret_cast<const bf16x8 *>(a.S + (long long)(b_row + row0) * a.ldS + k +
                                                     8 * part0) : zero;
        b1 = ok1 ? *reinterpret_cast<const bf16x8 *>(a.S + (long long)(b_row + row1) * a.ldS + k +
                                                     8 * part1) : zero;
    };
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    // row sum of A row tid / 2, samples 16 (tid & 1) .. + 15 of every step
    const int srow = tid >> 1, shalf = tid & 1;
    float bsum = 0.0f;
    bf16x8 ra0, ra1, rb0, rb1;
    if (k0 < k1) load(k0, ra0, ra1, rb0, rb1);
    for (long long k = k0; k < k1; k += 32) {
        *reinterpret_cast<bf16x8 *>(As + row0 * kGmPad + 8 * part0) = ra0;
        *reinterpret_cast<bf16x8 *>(As + row1 * kGmPad + 8 * part1) = ra1;
        *reinterpret_cast<bf16x8 *>(Bs + row0 * kGmPad + 8 * part0) = rb0;
        *reinterpret_cast<bf16x8 *>(Bs + row1 * kGmPad + 8 * part1) = rb1;
        __syncthreads();
        if (k + 32 < k1) load(k + 32, ra0, ra1, rb0, rb1);
        bf16x8 fa[4], fb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            fa[t] = *reinterpret_cast<const bf16x8 *>(As + (64 * mh + 16 * t + r) * kGmPad + 8 * g);
            fb[t] = *reinterpret_cast<const bf16x8 *>(Bs + (64 * nh + 16 * t + r) * kGmPad + 8 * g);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = mfma(fa[i], fb[j], acc[i][j]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const bf16x8 v = *reinterpret_cast<const bf16x8 *>(As + srow * kGmPad + 16 * shalf + 8 * h);
#pragma unroll
            for (int e = 0; e < 8; ++e) bsum += float(v[e]);
        }
        __syncthreads();
    }
    // the two halves of a row are adjacent lanes
    const float rsum = bsum + __shfl_xor(bsum, 1);
    if (shalf == 0)
        a.part[(long long)blockIdx.y * kGradEntries + kG_D_XO + (128 * (job + 1) + srow) * 16 + 4] =
            rsum;
    float *P = a.part + (long long)blockIdx.y * kGradEntries + out;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e)
                P[(64 * mh + 16 * i + 4 * g + e) * 128 + 64 * nh + 16 * j + r] = acc[i][j][e];
}

// All weight-gradient sums of one step in one launch: blockIdx.x 0 and 1 are
// the two 128 x 128 products (the long-running workgroups, dispatched first),
// the others the small products; blockIdx.y is the split of the sum.
constexpr int kGradSmallBlocks = (kGemmWaveTiles - kGemmSmallFirst + 3) / 4;

__global__ __launch_bounds__(256) void sur_grad_kernel(GemmArgs a) {
    __shared__ GradMatLds L;
    if (blockIdx.x < 2)
        grad_mat(a, L, int(blockIdx.x));
    else
        grad_small(a, int(blockIdx.x) - 2);
}

// Offset of parameter p's gradient in the partial vector.
__device__ inline int grad_source(int p) {
    if (p < kB1) return kG_D_XO + (p >> 2) * 16 + (p & 3);                 // W1[f][k]
    if (p < kW2) return kG_D_XO + (p - kB1) * 16 + 4;                      // b1
    if (p < kB2) return kG_W2 + (p - kW2);                                 // W2
    if (p < kW3) return kG_D_XO + (128 + p - kB2) * 16 + 4;                // b2
    if (p < kB3) return kG_W3 + (p - kW3);                                 // W3
    if (p < kW4) return kG_D_XO + (256 + p - kB3) * 16 + 4;                // b3
    if (p < kB4) return kG_XO_H3 + (5 + ((p - kW4) >> 7)) * 144 + ((p - kW4) & 127);  // W4
    return kG_XO_H3 + (5 + (p - kB4)) * 144 + 128 + 4;                     // b4
}

struct UpdateArgs {
    float *params, *m, *v, *grad;
    __bf16 *shadow;
    const float *part;
    int splits, mode;
    float lr, beta1, beta2, eps, inv_bc1, inv_bc2;
    const float *loss_part;
    long long n_loss;
    float inv_n;
    float *loss_out;
};

// 64 parameters per workgroup: wave q (q = 0..3) sums splits 32q .. 32q+31 of
// each parameter's gradient in split order (all 32 loads in flight at once);
// wave 0 then combines the four sums as ((s0 + s1) + (s2 + s3)), takes the Adam
// step and refreshes the permuted bf16 copies.
constexpr int kUpdateParams = 64;
constexpr int kUpdateGroups = 4;

__global__ __launch_bounds__(256) void sur_update_kernel(UpdateArgs a) {
    static_assert(kMaxSplits % kUpdateGroups == 0, "splits per group");
    constexpr int kPer = kMaxSplits / kUpdateGroups;
    if (int(blockIdx.x) == int(gridDim.x) - 1 && a.loss_out) {
        // the extra last workgroup: the minibatch loss from the per-tile sums
        __shared__ float red[256];
        float s = 0.0f;
#pragma unroll 16
        for (long long i = threadIdx.x; i < a.n_loss; i += 256) s += a.loss_part[i];
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) a.loss_out[0] = red[0] * a.inv_n;
        return;
    }
    __shared__ float sums[kUpdateGroups][kUpdateParams];
    const int pl = int(threadIdx.x) & (kUpdateParams - 1), grp = int(threadIdx.x) >> 6;
    const int p = int(blockIdx.x) * kUpdateParams + pl;
    const int pc = p < kParams ? p : kParams - 1;
    if (a.mode & kModeReduce) {
        const int src = grad_source(pc);
        float part[kPer];
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int sp = grp * kPer + u;
            part[u] = a.part[(long long)(sp < a.splits ? sp : a.splits - 1) * kGradEntries + src];
        }
        float gs = 0.0f;
#pragma unroll
        for (int u = 0; u < kPer; ++u)
            if (grp * kPer + u < a.splits) gs += part[u];
        sums[grp][pl] = gs;
    }
    __syncthreads();
    if (grp != 0 || p >= kParams) return;
    float th = a.params[p];
    if (a.mode & kModeReduce) {
        const float gsum = (sums[0][pl] + sums[1][pl]) + (sums[2][pl] + sums[3][pl]);
        a.grad[p] = gsum;
        if (a.mode & kModeAdam) {
            const float m = a.beta1 * a.m[p] + (1.0f - a.beta1) * gsum;
            const float v = a.beta2 * a.v[p] + (1.0f - a.beta2) * gsum * gsum;
            a.m[p] = m;
            a.v[p] = v;
            th -= a.lr * (m * a.inv_bc1) / (sqrtf(v * a.inv_bc2) + a.eps);
            a.params[p] = th;
        }
    }
    int base = -1, q = 0;
    if (p >= kW2 && p < kB2) { base = 0; q = p - kW2; }
    else if (p >= kW3 && p < kB3) { base = 1; q = p - kW3; }
    if (base >= 0) {
        const int o = q >> 7, i = q & 127;
        const __bf16 bv = __bf16(th);
        a.shadow[base * kMat + o * kWidth + 32 * (i >> 5) + perm32_inv(i & 31)] = bv;
        a.shadow[(2 + base) * kMat + i * kWidth + 32 * (o >> 5) + perm32_inv(o & 31)] = bv;
    }
}

struct InferLds {
    __bf16 w[2 * kWidth * kLdsRow];
    SmallParams sp;
};

struct ForwardArgs {
    const float *params;
    const __bf16 *shadow;
    const float *x;
    float *out;
    long long n;
    float shift[4], scale[4];
};

__global__ __launch_bounds__(kInferThreads) void sur_forward_kernel(ForwardArgs a) {
    __shared__ InferLds L;
    const int tid = int(threadIdx.x);
    load_mats<2, kInferThreads>(L.w, a.shadow, tid);
    load_small<kInferThreads>(L.sp, a.params, tid);
    __syncthreads();
    const int lane = tid & 63, s = lane & 15, g = lane >> 4;
    const long long n = ((long long)blockIdx.x * (kInferThreads / 64) + (tid >> 6)) * 16 + s;
    const long long nc = n < a.n ? n : a.n - 1;
    float u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = (a.x[k * a.n + nc] - a.shift[k]) * a.scale[k];
    Layer d1, d2, d3, a3;
    float o0, o1;
    forward<false>(L.sp, L.w, L.w + kWidth * kLdsRow, u, lane, d1, d2, d3, a3, o0, o1, nullptr);
    if (n < a.n && g == 0) {
        a.out[n] = o0;
        a.out[a.n + n] = o1;
    }
}

struct ChainArgs {
    const float *params;
    const __bf16 *shadow;
    float shift[4], scale[4];
    double os0, os1;
    const double *y0, *mu;
    long long count;
    double t0, L;
    int coarse;                  // coarse RK4 steps (0: identity)
    int step_doubling;           // 1: the step-doubling form
    double tau2_0, tau2_1;       // squared gate scales
    int n_slices;
    double *final_state, *boundary;
    const void *tab0, *tab1;
    int fb_fp64;
    long long M;
    int n0, n1;
    double lo0, inv0, lo1, inv1, guard;
    double blo0, blo1, bhi0, bhi1;
    unsigned long long *stats;   // fallbacks, outside, max deviation (bits), first bad chain
};

// The bilinear map of table row j at (l0, l1), with the operation sequence of
// the library's bilinear composition.
template <class T>
__device__ inline void bilinear_row(const ChainArgs &a, int j, double l0, double l1, double &p,
                                    double &q) {
#pragma clang fp contract(off)
    long long i0, i1;
    double w0, w1;
    nv::dev::locate(a.lo0, a.inv0, a.n0, l0, i0, w0);
    nv::dev::locate(a.lo1, a.inv1, a.n1, l1, i1, w1);
    const T *row0 = static_cast<const T *>(a.tab0) + (long long)j * a.M;
    const T *row1 = static_cast<const T *>(a.tab1) + (long long)j * a.M;
    const long long c00 = i0 * a.n1 + i1, c10 = (i0 + 1) * a.n1 + i1;
    const double p00 = double(row0[c00]), p01 = double(row0[c00 + 1]);
    const double p10 = double(row0[c10]), p11 = double(row0[c10 + 1]);
    const double q00 = double(row1[c00]), q01 = double(row1[c00 + 1]);
    const double q10 = double(row1[c10]), q11 = double(row1[c10 + 1]);
    const double r0 = p00 + w1 * (p01 - p00), r1 = p10 + w1 * (p11 - p10);
    const double s0 = q00 + w1 * (q01 - q00), s1 = q10 + w1 * (q11 - q10);
    p = r0 + w0 * (r1 - r0);
    q = s0 + w0 * (s1 - s0);
}

// The composition runs one dependent chain of network evaluations, so its
// latency matters more than its throughput: a workgroup of 4 waves evaluates
// the network for 16 chains together.  Wave w computes output tiles 2w and
// 2w+1 (features 32w .. 32w+31) of every 128-wide layer, which is exactly
// k-block w of the next layer's operand in the permuted order; the four blocks
// are exchanged through LDS, and the output layer's partial sums are added in
// wave order.
struct ChainLds {
    __bf16 w[2 * kWidth * kLdsRow];      // Wf2, Wf3
    SmallParams sp;
    bf16x8 xb[4][64];                    // operand k-block of each wave, by lane
    float part[4][2][16];                // output partial sums: wave, output, sample
};

// One 128 x 128 layer's tiles 2w, 2w+1 from the four operand blocks.
__device__ inline void layer_split(const __bf16 *M, const bf16x8 (&b)[4], int w, int lane,
                                   f32x4 (&out)[2]) {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        const __bf16 *row = M + (16 * (2 * w + t) + r) * kLdsRow + 8 * g;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb)
            acc = mfma(*reinterpret_cast<const bf16x8 *>(row + 32 * kb), b[kb], acc);
        out[t] = acc;
    }
}

// Publish this wave's block and gather all four (two barriers: the previous
// round's reads are complete before the block is overwritten).
__device__ inline void exchange(ChainLds &L, const bf16x8 &mine, int w, int lane,
                                bf16x8 (&b)[4]) {
    __syncthreads();
    L.xb[w][lane] = mine;
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) b[kb] = L.xb[kb][lane];
}

__device__ inline void forward_split(ChainLds &L, const float (&u)[4], int w, int lane,
                                     float &o0, float &o1) {
    const int s = lane & 15, g = lane >> 4;
    f32x4 x[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = 16 * (2 * w + t) + 4 * g + i;
            float z = L.sp.b1[f];
            z = fmaf(L.sp.w1[4 * f + 0], u[0], z);
            z = fmaf(L.sp.w1[4 * f + 1], u[1], z);
            z = fmaf(L.sp.w1[4 * f + 2], u[2], z);
            z = fmaf(L.sp.w1[4 * f + 3], u[3], z);
            float d;
            x[t][i] = gelu_d(z, d);
        }
    }
    bf16x8 b[4], blk;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        blk[e] = __bf16(x[0][e]);
        blk[e + 4] = __bf16(x[1][e]);
    }
    exchange(L, blk, w, lane, b);
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        const __bf16 *M = L.w + layer * kWidth * kLdsRow;
        const float *bias = layer == 0 ? L.sp.b2 : L.sp.b3;
        layer_split(M, b, w, lane, x);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float d;
                x[t][i] = gelu_d(x[t][i] + bias[16 * (2 * w + t) + 4 * g + i], d);
            }
        }
        if (layer == 0) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                blk[e] = __bf16(x[0][e]);
                blk[e + 4] = __bf16(x[1][e]);
            }
            exchange(L, blk, w, lane, b);
        }
    }
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = 16 * (2 * w + t) + 4 * g + i;
            s0 = fmaf(L.sp.w4[f], x[t][i], s0);
            s1 = fmaf(L.sp.w4[kWidth + f], x[t][i], s1);
        }
    }
    s0 += __shfl_xor(s0, 16);
    s1 += __shfl_xor(s1, 16);
    s0 += __shfl_xor(s0, 32);
    s1 += __shfl_xor(s1, 32);
    if (g == 0) {
        L.part[w][0][s] = s0;
        L.part[w][1][s] = s1;
    }
    __syncthreads();
    o0 = ((L.part[0][0][s] + L.part[1][0][s]) + (L.part[2][0][s] + L.part[3][0][s])) + L.sp.b4[0];
    o1 = ((L.part[0][1][s] + L.part[1][1][s]) + (L.part[2][1][s] + L.part[3][1][s])) + L.sp.b4[1];
}

__global__ __launch_bounds__(kInferThreads) void sur_chain_kernel(ChainArgs a) {
#pragma clang fp contract(off)
    __shared__ ChainLds L;
    const int tid = int(threadIdx.x);
    load_mats<2, kInferThreads>(L.w, a.shadow, tid);
    load_small<kInferThreads>(L.sp, a.params, tid);
    __syncthreads();
    const int lane = tid & 63, w = tid >> 6, s = lane & 15, g = lane >> 4;
    const long long q = (long long)blockIdx.x * 16 + s;        // the 4 waves share 16 chains
    const bool live = q < a.count;
    const long long qc = live ? q : a.count - 1;
    double l0 = a.y0[2 * qc], l1 = a.y0[2 * qc + 1];
    const float muf = float(a.mu[qc]);
    const bool writer = live && g == 0 && w == 0;
    const long long stride = (long long)a.n_slices + 1;
    if (writer && a.boundary) {
        a.boundary[(q * stride) * 2] = l0;
        a.boundary[(q * stride) * 2 + 1] = l1;
    }
    unsigned long long nfb = 0, nout = 0;
    double maxdev = 0.0;
    bool bad = false;
    for (int j = 0; j < a.n_slices; ++j) {
        asm volatile("" ::: "memory");  // keep the weight reads inside the loop
        if (!(isfinite(l0) && isfinite(l1))) bad = true;
        const float tj = float(a.t0 + double(j) * a.L);
        float u[4] = {(float(l0) - a.shift[0]) * a.scale[0], (float(l1) - a.shift[1]) * a.scale[1],
                      (tj - a.shift[2]) * a.scale[2], (muf - a.shift[3]) * a.scale[3]};
        float o0, o1;
        forward_split(L, u, w, lane, o0, o1);
        double n0, n1;
        if (a.step_doubling) {
            const StepDoubling sd = step_doubling(a.mu[qc], a.L, a.coarse, l0, l1, a.tau2_0,
                                                  a.tau2_1);
            n0 = sd.g0 + sd.d0 * (kRichardson + (a.os0 * sd.gt0) * double(o0));
            n1 = sd.g1 + sd.d1 * (kRichardson + (a.os1 * sd.gt1) * double(o1));
        } else {
            double g0 = l0, g1 = l1;
            coarse_rk4(double(a.mu[qc]), a.L / double(a.coarse), a.coarse, g0, g1);
            n0 = g0 + a.os0 * double(o0);
            n1 = g1 + a.os1 * double(o1);
        }
        const bool outside = !(l0 >= a.blo0 && l0 <= a.bhi0 && l1 >= a.blo1 && l1 <= a.bhi1);
        if (a.tab0) {
            double p, pq;
            if (a.fb_fp64)
                bilinear_row<double>(a, j, l0, l1, p, pq);
            else
                bilinear_row<float>(a, j, l0, l1, p, pq);
            const double d0 = fabs(n0 - p), dd1 = fabs(n1 - pq);
            const double dev = d0 > dd1 ? d0 : dd1;
            if (dev == dev && dev > maxdev) maxdev = dev;
            if (!(dev <= a.guard) || outside) {
                n0 = p;
                n1 = pq;
                ++nfb;
            }
        } else if (outside) {
            ++nout;
        }
        if (!bad) {
            l0 = n0;
            l1 = n1;
        }
        if (writer && a.boundary) {
            a.boundary[(q * stride + j + 1) * 2] = l0;
            a.boundary[(q * stride + j + 1) * 2 + 1] = l1;
        }
    }
    if (!(isfinite(l0) && isfinite(l1))) bad = true;
    if (writer) {
        a.final_state[2 * q] = l0;
        a.final_state[2 * q + 1] = l1;
        if (nfb) atomicAdd(&a.stats[0], nfb);
        if (nout) atomicAdd(&a.stats[1], nout);
        if (maxdev > 0.0) atomicMax(&a.stats[2], (unsigned long long)__double_as_longlong(maxdev));
        if (bad) atomicMin(&a.stats[3], (unsigned long long)q);
    }
}

// ---- training: forward pass, loss and back-propagation ------------------
//
// Four waves share a tile of 16 samples, as in the composition above: wave w
// of a group computes features 32 w .. 32 w + 31 (output tiles 2w, 2w+1) of
// every 128-wide layer, which is exactly k-block w of the next product's
// operand, and the four blocks are exchanged through LDS.  A wave so holds a
// quarter of each layer's values and GELU derivatives, which lets two groups
// (two waves per SIMD) share the workgroup's one copy of the four bf16
// weight matrices in LDS: the second group's instructions fill the first's
// latency.  Each product's output element is summed over the same k-blocks in
// the same order as a whole-layer product; the network's two outputs are the
// four waves' partial sums added in wave order.
constexpr int kTrainGroups = 3;                        // tiles in flight per workgroup
constexpr int kTrainThreads = 256 * kTrainGroups;
// Inputs and targets of kStageTiles tiles are staged in LDS before the tiles
// are processed: a global load inside the tile loop would have to wait for
// every store of the previous tile (the memory counter is in order).
constexpr int kStageTiles = 8;

struct TrainLds {
    __bf16 w[4 * kWidth * kLdsRow];         // Wf2, Wf3, Wb2, Wb3
    SmallParams sp;
    float xs[4 * kStageTiles * 16];
    float ts[4 * kStageTiles * 16];         // targets and weights (1 when unweighted)
    bf16x8 xb[kTrainGroups][4][64];         // per group: each wave's operand k-block
    float part[kTrainGroups][4][2][16];     // per group: the outputs' partial sums
};
static_assert(sizeof(TrainLds) <= 160 * 1024, "the training kernel's LDS exceeds 160 KiB");

// Publish this wave's block to its group and gather all four (two barriers:
// the group's previous reads are complete before the block is overwritten).
__device__ inline void train_exchange(TrainLds &L, int gi, const bf16x8 &mine, int w, int lane,
                                      bf16x8 (&b)[4]) {
    __syncthreads();
    L.xb[gi][w][lane] = mine;
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) b[kb] = L.xb[gi][kb][lane];
}

__device__ inline bf16x8 pack_block(const f32x4 (&x)[2]) {
    bf16x8 blk;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        blk[e] = __bf16(x[0][e]);
        blk[e + 4] = __bf16(x[1][e]);
    }
    return blk;
}

// Rows row0 + 32 w + (features of the block) of the tile: element e of the
// block is feature 4 g + e (e < 4) or 16 + 4 g + (e - 4) of the wave's 32.
__device__ inline void store_block(const RowSink &o, int row0, int w, const bf16x8 &blk,
                                   int lane) {
    const int s = lane & 15, g = lane >> 4;
    __bf16 *col = o.tile + (long long)(row0 + 32 * w + 4 * g) * o.ld + s;
#pragma unroll
    for (int e = 0; e < 8; ++e) col[(long long)(e < 4 ? e : 12 + e) * o.ld] = blk[e];
}

// One tile (16 samples, staged at li0 .. li0 + 15 of the chunk) by wave w of
// group gi.  When !live the group computes and stores nothing but passes the
// same barriers (every barrier below is outside the `live` conditions, so all
// waves of the workgroup meet the same sequence of them).
__device__ inline void train_tile(const TrainArgs &a, TrainLds &L, long long tile, int li0,
                                  bool live, int gi, int w, int lane) {
    const int s = lane & 15, g = lane >> 4, li = li0 + s;
    const __bf16 *Wf2 = L.w, *Wf3 = L.w + kWidth * kLdsRow;
    const __bf16 *Wb2 = L.w + 2 * kWidth * kLdsRow, *Wb3 = L.w + 3 * kWidth * kLdsRow;
    const RowSink sink{a.S + tile * 16, a.ldS};
    float u[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = (L.xs[k * kStageTiles * 16 + li] - a.shift[k]) * a.scale[k];
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    f32x4 x[2] = {zero, zero}, d1[2] = {zero, zero}, d2[2] = {zero, zero}, d3[2] = {zero, zero};
    bf16x8 b[4], blk = {};
    // layer 1 (FP32): the wave's 32 features
    if (live) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * (2 * w + t) + 4 * g + i;
                float z = L.sp.b1[f];
                z = fmaf(L.sp.w1[4 * f + 0], u[0], z);
                z = fmaf(L.sp.w1[4 * f + 1], u[1], z);
                z = fmaf(L.sp.w1[4 * f + 2], u[2], z);
                z = fmaf(L.sp.w1[4 * f + 3], u[3], z);
                float d;
                x[t][i] = gelu_d(z, d);
                d1[t][i] = d;
            }
        }
        blk = pack_block(x);
        store_block(sink, kRowH, w, blk, lane);
    }
    train_exchange(L, gi, blk, w, lane, b);
    // layers 2 and 3 on the matrix cores
#pragma unroll
    for (int layer = 0; layer < 2; ++layer) {
        if (live) {
            layer_split(layer == 0 ? Wf2 : Wf3, b, w, lane, x);
            const float *bias = layer == 0 ? L.sp.b2 : L.sp.b3;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float d;
                    x[t][i] = gelu_d(x[t][i] + bias[16 * (2 * w + t) + 4 * g + i], d);
                    if (layer == 0)
                        d2[t][i] = d;
                    else
                        d3[t][i] = d;
                }
            }
            blk = pack_block(x);
            store_block(sink, kRowH + 128 * (layer + 1), w, blk, lane);
        }
        if (layer == 0) train_exchange(L, gi, blk, w, lane, b);
    }
    // the two outputs: the wave's partial sums over its 32 features of a3
    if (live) {
        float s0 = 0.f, s1 = 0.f;
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * (2 * w + t) + 4 * g + i;
                s0 = fmaf(L.sp.w4[f], x[t][i], s0);
                s1 = fmaf(L.sp.w4[kWidth + f], x[t][i], s1);
            }
        }
        s0 += __shfl_xor(s0, 16);
        s1 += __shfl_xor(s1, 16);
        s0 += __shfl_xor(s0, 32);
        s1 += __shfl_xor(s1, 32);
        if (g == 0) {
            L.part[gi][w][0][s] = s0;
            L.part[gi][w][1][s] = s1;
        }
    }
    __syncthreads();
    float e0 = 0.f, e1 = 0.f, dout0 = 0.f, dout1 = 0.f;
    if (live) {
        const float o0 = ((L.part[gi][0][0][s] + L.part[gi][1][0][s]) +
                          (L.part[gi][2][0][s] + L.part[gi][3][0][s])) + L.sp.b4[0];
        const float o1 = ((L.part[gi][0][1][s] + L.part[gi][1][1][s]) +
                          (L.part[gi][2][1][s] + L.part[gi][3][1][s])) + L.sp.b4[1];
        // the error of the sample, e = w out - target (w = 1 unweighted, where
        // this is out - target to the bit), and dL/dout = 2 e w / n.  Rows 2 and 3
        // of the staged targets hold the weights, 1 when unweighted: an
        // unconditional read keeps the kernel within its register budget.
        const float t0 = L.ts[li], t1 = L.ts[kStageTiles * 16 + li];
        const float w0 = L.ts[2 * kStageTiles * 16 + li], w1 = L.ts[3 * kStageTiles * 16 + li];
        e0 = w0 * o0 - t0;
        e1 = w1 * o1 - t1;
        dout0 = 2.0f * e0 * w0 * a.inv_n;
        dout1 = 2.0f * e1 * w1 * a.inv_n;
        // back-propagation: dL/dz3 = (W4^T dout) * gelu'(z3) for the wave's features
#pragma unroll
        for (int t = 0; t < 2; ++t) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int f = 16 * (2 * w + t) + 4 * g + i;
                x[t][i] = (L.sp.w4[f] * dout0 + L.sp.w4[kWidth + f] * dout1) * d3[t][i];
            }
        }
        blk = pack_block(x);
        store_block(sink, kRowD + 256, w, blk, lane);
    }
    train_exchange(L, gi, blk, w, lane, b);
    if (live) {
        layer_split(Wb3, b, w, lane, x);                  // W3^T dL/dz3
#pragma unroll
        for (int t = 0; t < 2; ++t) x[t] *= d2[t];
        blk = pack_block(x);
        store_block(sink, kRowD + 128, w, blk, lane);
    }
    train_exchange(L, gi, blk, w, lane, b);
    if (live) {
        layer_split(Wb2, b, w, lane, x);                  // W2^T dL/dz2
#pragma unroll
        for (int t = 0; t < 2; ++t) x[t] *= d1[t];
        blk = pack_block(x);
        store_block(sink, kRowD, w, blk, lane);
    }

    if (live && w == 0) {
        // rows of XO: group 0 writes u0..u3, group 1 writes 1, dout0, dout1, 0,
        // groups 2 and 3 the zero rows
        __bf16 xo[4];
        if (g == 0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) xo[r] = __bf16(u[r]);
        } else if (g == 1) {
            xo[0] = __bf16(1.0f);
            xo[1] = __bf16(dout0);
            xo[2] = __bf16(dout1);
            xo[3] = __bf16(0.0f);
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) xo[r] = __bf16(0.0f);
        }
        store_rows16(sink, kRowXO, xo, lane);
        float sq = g == 0 ? e0 * e0 + e1 * e1 : 0.0f;
        sq += __shfl_xor(sq, 1);
        sq += __shfl_xor(sq, 2);
        sq += __shfl_xor(sq, 4);
        sq += __shfl_xor(sq, 8);
        if (lane == 0) a.loss_part[tile] = sq;
    }
}

__global__ __launch_bounds__(kTrainThreads) void sur_train_kernel(TrainArgs a) {
    __shared__ TrainLds L;
    const int tid = int(threadIdx.x);
    load_mats<4, kTrainThreads>(L.w, a.shadow, tid);
    load_small<kTrainThreads>(L.sp, a.params, tid);
    const int lane = tid & 63;
    const int gi = __builtin_amdgcn_readfirstlane(tid >> 8);        // group
    const int w = __builtin_amdgcn_readfirstlane((tid >> 6) & 3);   // wave in the group
    const long long tiles = a.n / 16;
    // workgroup b owns the contiguous tiles [b * per, (b+1) * per), staged in
    // chunks of kStageTiles; group gi takes tiles c0 + gi, c0 + gi + G, ...
    const long long per = (tiles + gridDim.x - 1) / gridDim.x;
    const long long tb = (long long)blockIdx.x * per;
    const long long te = tb + per < tiles ? tb + per : tiles;
    for (long long c0 = tb; c0 < te; c0 += kStageTiles) {
        const long long c1 = c0 + kStageTiles < te ? c0 + kStageTiles : te;
        const int cn = int(c1 - c0) * 16;
        __syncthreads();                              // the previous chunk is consumed
        for (int i = tid; i < cn; i += kTrainThreads) {
            const long long src = a.start + c0 * 16 + i;
#pragma unroll
            for (int k = 0; k < 4; ++k) L.xs[k * kStageTiles * 16 + i] = a.x[k * a.ld + src];
            L.ts[i] = a.t[src];
            L.ts[kStageTiles * 16 + i] = a.t[a.ld + src];
            L.ts[2 * kStageTiles * 16 + i] = a.weighted ? a.t[2 * a.ld + src] : 1.0f;
            L.ts[3 * kStageTiles * 16 + i] = a.weighted ? a.t[3 * a.ld + src] : 1.0f;
        }
        __syncthreads();
        // every group runs the same number of rounds (the barriers inside a
        // tile are the workgroup's); a group past the chunk's end only passes
        // the barriers
        const int rounds = (int(c1 - c0) + kTrainGroups - 1) / kTrainGroups;
        for (int r = 0; r < rounds; ++r) {
            asm volatile("" ::: "memory");            // keep the weight reads inside the loop
            const long long tile = c0 + r * kTrainGroups + gi;
            const bool live = tile < c1;
            const long long tt = live ? tile : c0;
            train_tile(a, L, tt, int(tt - c0) * 16, live, gi, w, lane);
        }
    }
}

struct DatasetArgs {
    const nv::SliceMapSource *src;
    int n_src, fp64;
    long long total, cap;
    const long long *perm;
    float *x, *t;
    double os0, os1;
    int coarse;
    int *error;
    int step_doubling;           // targets rho_0, rho_1, w_0, w_1 (4 rows)
    double tau2_0, tau2_1, q0, q1;
    // visit weights (step-doubling only; visits null: v = 1)
    const double *visits;        // [n_mu][n_states][2]
    int n_mu, n_states;
    double mu_lo, mu_step;       // chain i for mu_lo + i mu_step
    float sc0, sc1, inv2s2, floor_w;
};

constexpr int kMaxVisitStates = 4096;     // states of one chain staged in LDS (32 KiB)

// The source (problem) of sample n: the last whose first sample is <= n.
__device__ inline int source_of(const DatasetArgs &a, long long n) {
    int lo = 0, hi = a.n_src - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.src[mid].first <= n)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ inline int visit_chain(const DatasetArgs &a, double mu) {
    double c = rint((mu - a.mu_lo) / a.mu_step);
    c = c < 0.0 ? 0.0 : (c > double(a.n_mu - 1) ? double(a.n_mu - 1) : c);
    return int(c);
}

// Squared distance, in the network's input units, from (y0, y1) to the
// nearest state of a chain (fp32, one rounding per operation).
template <class Get>
__device__ inline float nearest_d2(const Get &state, int n, float y0, float y1, float sc0,
                                   float sc1) {
#pragma clang fp contract(off)
    float best = INFINITY;
    for (int i = 0; i < n; ++i) {
        const float2 v = state(i);
        const float e0 = (y0 - v.x) * sc0, e1 = (y1 - v.y) * sc1;
        const float d2 = e0 * e0 + e1 * e1;
        best = d2 < best ? d2 : best;
    }
    return best;
}

// Grid-stride over chunks of 256 consecutive samples (natural numbering, so
// that a chunk usually lies in one problem and shares its mu's visit chain,
// which the workgroup stages in LDS).
__global__ __launch_bounds__(256) void sur_dataset_kernel(DatasetArgs a) {
#pragma clang fp contract(off)
    __shared__ float2 vis[kMaxVisitStates];
    int staged = -1;                                      // workgroup-uniform
    const long long step = (long long)gridDim.x * 256;
    for (long long base = (long long)blockIdx.x * 256; base < a.total; base += step) {
        if (a.visits) {
            const int cf = visit_chain(a, a.src[source_of(a, base)].mu);
            if (cf != staged) {
                __syncthreads();                          // the previous chain is consumed
                const double *cs = a.visits + (long long)cf * a.n_states * 2;
                for (int i = int(threadIdx.x); i < a.n_states; i += 256)
                    vis[i] = make_float2(float(cs[2 * i]), float(cs[2 * i + 1]));
                __syncthreads();
                staged = cf;
            }
        }
        const long long n = base + threadIdx.x;
        if (n >= a.total) continue;
        const nv::SliceMapSource &s = a.src[source_of(a, n)];
        const long long r = n - s.first, j = r / s.M, k = r - j * s.M;
        const unsigned kk = unsigned(k), n1 = unsigned(s.n1);
        const unsigned k0 = kk / n1, k1 = kk - k0 * n1;
        const float y0 = float(s.lo0 + double(k0) * s.dxi0);
        const float y1 = float(s.lo1 + double(k1) * s.dxi1);
        double e0, e1;
        if (a.fp64) {
            e0 = static_cast<const double *>(s.tab0)[j * s.M + k];
            e1 = static_cast<const double *>(s.tab1)[j * s.M + k];
        } else {
            e0 = double(static_cast<const float *>(s.tab0)[j * s.M + k]);
            e1 = double(static_cast<const float *>(s.tab1)[j * s.M + k]);
        }
        const long long pos = a.perm ? a.perm[n] : n;
        if (pos < 0 || pos >= a.cap) {
            atomicOr(a.error, 1);
            continue;
        }
        if (!isfinite(e0) || !isfinite(e1)) atomicOr(a.error, 2);
        a.x[pos] = y0;
        a.x[a.cap + pos] = y1;
        a.x[2 * a.cap + pos] = float(s.t0 + double(j) * s.L);
        a.x[3 * a.cap + pos] = float(s.mu);
        if (!a.step_doubling) {
            double g0 = double(y0), g1 = double(y1);
            coarse_rk4(s.mu, s.L / double(a.coarse), a.coarse, g0, g1);
            a.t[pos] = float((e0 - g0) / a.os0);
            a.t[a.cap + pos] = float((e1 - g1) / a.os1);
            continue;
        }
        const StepDoubling sd =
            step_doubling(s.mu, s.L, a.coarse, double(y0), double(y1), a.tau2_0, a.tau2_1);
        double sv = 1.0;
        if (a.visits) {
            const int ci = visit_chain(a, s.mu);
            float d2;
            if (ci == staged) {
                d2 = nearest_d2([&](int i) { return vis[i]; }, a.n_states, y0, y1, a.sc0, a.sc1);
            } else {
                const double *cs = a.visits + (long long)ci * a.n_states * 2;
                d2 = nearest_d2(
                    [&](int i) { return make_float2(float(cs[2 * i]), float(cs[2 * i + 1])); },
                    a.n_states, y0, y1, a.sc0, a.sc1);
            }
            const float v = expf(-(d2 * a.inv2s2)) + a.floor_w;
            sv = sqrt(double(v));
        }
        const double r0 = (e0 - sd.g0) - kRichardson * sd.d0;
        const double r1 = (e1 - sd.g1) - kRichardson * sd.d1;
        a.t[pos] = float((sv * r0) / a.q0);
        a.t[a.cap + pos] = float((sv * r1) / a.q1);
        a.t[2 * a.cap + pos] = float((sv * ((sd.d0 * a.os0) * sd.gt0)) / a.q0);
        a.t[3 * a.cap + pos] = float((sv * ((sd.d1 * a.os1) * sd.gt1)) / a.q1);
    }
}

}  // namespace

// ---------------------------------------------------------------- host side

struct nv_sur {
    nv_sur_config cfg{};
    hipStream_t stream = nullptr;
    int n_cu = 256;
    long long max_batch = 0;
    char *mem = nullptr;         // one device allocation
    float *params = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    __bf16 *shadow = nullptr, *S = nullptr;
    float *part = nullptr, *loss_part = nullptr, *loss = nullptr;
    unsigned long long *stats = nullptr;
    int *error = nullptr;
    long long adam_t = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float last_ms = 0.f;
    // visit weights of the step-doubling training set (nv_sur_set_visits)
    const double *visits = nullptr;
    int n_mu = 0, n_states = 0;
    double mu_lo = 0.0, mu_hi = 0.0, sigma = 0.0, floor_w = 0.0;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

void fill_norm(const nv_sur *s, float (&shift)[4], float (&scale)[4]) {
    for (int k = 0; k < 4; ++k) {
        shift[k] = s->cfg.in_shift[k];
        scale[k] = s->cfg.in_scale[k];
    }
}

nv_status refresh_shadow(nv_sur *s) {
    UpdateArgs u{};
    u.params = s->params;
    u.shadow = s->shadow;
    u.mode = 0;
    hipLaunchKernelGGL(sur_update_kernel, dim3((kParams + kUpdateParams - 1) / kUpdateParams),
                       dim3(256), 0, s->stream, u);
    NV_HIP(hipGetLastError());
    return NV_OK;
}

long long k_per_split(long long n) {
    long long k = std::max(kMinSplit, (n + kMaxSplits - 1) / kMaxSplits);
    return (k + 31) / 32 * 32;
}

// One minibatch: forward and back-propagation, gradient sums, then the update
// kernel (mode: reduce only, or reduce and Adam step).
nv_status minibatch(nv_sur *s, const float *x, const float *t, long long ld, long long start,
                    long long n, int mode, float lr, float b1, float b2, float eps,
                    float *loss_out) {
    TrainArgs ta{};
    ta.x = x;
    ta.t = t;
    ta.ld = ld;
    ta.start = start;
    ta.n = n;
    ta.params = s->params;
    ta.shadow = s->shadow;
    ta.S = s->S;
    ta.ldS = s->max_batch;
    ta.loss_part = s->loss_part;
    fill_norm(s, ta.shift, ta.scale);
    ta.inv_n = float(1.0 / double(n));
    ta.weighted = s->cfg.correction == NV_SUR_STEP_DOUBLING;
    const long long tiles = n / 16;
    const int wpb = kTrainThreads / 64;                        // waves per workgroup
    const int blocks = int(std::min<long long>((tiles + wpb - 1) / wpb, s->n_cu));
    hipLaunchKernelGGL(sur_train_kernel, dim3(blocks), dim3(kTrainThreads), 0, s->stream, ta);
    NV_HIP(hipGetLastError());

    GemmArgs ga{};
    ga.S = s->S;
    ga.ldS = s->max_batch;
    ga.n = n;
    ga.k_per_split = k_per_split(n);
    ga.part = s->part;
    const int splits = int((n + ga.k_per_split - 1) / ga.k_per_split);
    hipLaunchKernelGGL(sur_grad_kernel, dim3(2 + kGradSmallBlocks, splits), dim3(256), 0,
                       s->stream, ga);
    NV_HIP(hipGetLastError());

    UpdateArgs ua{};
    ua.params = s->params;
    ua.m = s->m;
    ua.v = s->v;
    ua.grad = s->grad;
    ua.shadow = s->shadow;
    ua.part = s->part;
    ua.splits = splits;
    ua.mode = mode;
    if (mode & kModeAdam) {
        const long long t = ++s->adam_t;
        ua.lr = lr;
        ua.beta1 = b1;
        ua.beta2 = b2;
        ua.eps = eps;
        ua.inv_bc1 = float(1.0 / (1.0 - std::pow(double(b1), double(t))));
        ua.inv_bc2 = float(1.0 / (1.0 - std::pow(double(b2), double(t))));
    }
    ua.loss_part = s->loss_part;
    ua.n_loss = tiles;
    ua.inv_n = ta.inv_n;
    ua.loss_out = loss_out;
    // one workgroup per 64 parameters, plus one for the loss
    hipLaunchKernelGGL(sur_update_kernel,
                       dim3((kParams + kUpdateParams - 1) / kUpdateParams + (ua.loss_out ? 1 : 0)),
                       dim3(256), 0, s->stream, ua);
    NV_HIP(hipGetLastError());
    return NV_OK;
}

}  // namespace

extern "C" {

NV_API nv_status nv_sur_create(const nv_sur_config *cfg, nv_sur **out) try {
    if (!cfg || !out) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(cfg->in_shift[k]) || !std::isfinite(cfg->in_scale[k]))
            return fail(NV_ERR_INVALID_ARG, "input normalisation %d is not finite", k);
    for (int c = 0; c < 2; ++c)
        if (!(cfg->out_scale[c] > 0.0) || !std::isfinite(cfg->out_scale[c]))
            return fail(NV_ERR_INVALID_ARG, "out_scale[%d] must be positive and finite", c);
    if (!(cfg->slice_length > 0.0) || !std::isfinite(cfg->slice_length))
        return fail(NV_ERR_INVALID_ARG, "slice_length must be positive and finite");
    if (cfg->coarse_steps < 0 || cfg->coarse_steps > kMaxCoarse)
        return fail(NV_ERR_INVALID_ARG, "coarse_steps %d: need 0..%d", cfg->coarse_steps,
                    kMaxCoarse);
    if (cfg->correction != NV_SUR_ADDITIVE && cfg->correction != NV_SUR_STEP_DOUBLING)
        return fail(NV_ERR_INVALID_ARG, "unknown correction %d", cfg->correction);
    if (cfg->correction == NV_SUR_STEP_DOUBLING) {
        if (cfg->coarse_steps < 1)
            return fail(NV_ERR_INVALID_ARG, "the step-doubling form needs coarse_steps >= 1");
        for (int c = 0; c < 2; ++c)
            if (!(cfg->gate[c] > 0.0) || !std::isfinite(cfg->gate[c]) ||
                !(cfg->loss_scale[c] > 0.0) || !std::isfinite(cfg->loss_scale[c]))
                return fail(NV_ERR_INVALID_ARG, "gate[%d] and loss_scale[%d] must be positive "
                            "and finite", c, c);
    }
    const long long mb = cfg->max_batch == 0 ? 65536 : cfg->max_batch;
    if (mb < 16 || mb > kMaxBatch || mb % 16 != 0)
        return fail(NV_ERR_INVALID_ARG, "max_batch %lld: need a multiple of 16 in [16, 2^20]",
                    mb);
    nv_sur *s = new (std::nothrow) nv_sur();
    if (!s) return fail(NV_ERR_OOM, "out of host memory");
    s->cfg = *cfg;
    s->cfg.max_batch = mb;
    s->max_batch = mb;
    s->stream = static_cast<hipStream_t>(cfg->stream);
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            n > 0)
            s->n_cu = n;
    }
    // layout of the single allocation
    size_t off = 0;
    const size_t o_params = off; off = align256(off + kParams * sizeof(float));
    const size_t o_m = off;      off = align256(off + kParams * sizeof(float));
    const size_t o_v = off;      off = align256(off + kParams * sizeof(float));
    const size_t o_grad = off;   off = align256(off + kParams * sizeof(float));
    const size_t o_shadow = off; off = align256(off + 4 * kMat * sizeof(__bf16));
    const size_t o_part = off;   off = align256(off + size_t(kMaxSplits) * kGradEntries * 4);
    const size_t o_lp = off;     off = align256(off + size_t(mb / 16) * sizeof(float));
    const size_t o_loss = off;   off = align256(off + sizeof(float));
    const size_t o_stats = off;  off = align256(off + 4 * sizeof(unsigned long long));
    const size_t o_err = off;    off = align256(off + sizeof(int));
    const size_t o_S = off;      off = align256(off + size_t(kRowsS) * size_t(mb) * 2);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&s->mem), off);
    if (e != hipSuccess) {
        delete s;
        return fail(NV_ERR_OOM, "device allocation of %zu bytes failed", off);
    }
    s->params = reinterpret_cast<float *>(s->mem + o_params);
    s->m = reinterpret_cast<float *>(s->mem + o_m);
    s->v = reinterpret_cast<float *>(s->mem + o_v);
    s->grad = reinterpret_cast<float *>(s->mem + o_grad);
    s->shadow = reinterpret_cast<__bf16 *>(s->mem + o_shadow);
    s->part = reinterpret_cast<float *>(s->mem + o_part);
    s->loss_part = reinterpret_cast<float *>(s->mem + o_lp);
    s->loss = reinterpret_cast<float *>(s->mem + o_loss);
    s->stats = reinterpret_cast<unsigned long long *>(s->mem + o_stats);
    s->error = reinterpret_cast<int *>(s->mem + o_err);
    s->S = reinterpret_cast<__bf16 *>(s->mem + o_S);
    e = hipMemsetAsync(s->mem, 0, o_S, s->stream);
    if (e == hipSuccess) e = hipEventCreate(&s->ev0);
    if (e == hipSuccess) e = hipEventCreate(&s->ev1);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) {
        nv_sur_destroy(s);
        return fail(NV_ERR_HIP, "surrogate set-up failed: %s", hipGetErrorString(e));
    }
    *out = s;
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_sur_create: host allocation failed");
}

NV_API nv_status nv_sur_destroy(nv_sur *s) {
    if (!s) return NV_OK;
    if (s->stream || s->mem) (void)hipStreamSynchronize(s->stream);
    if (s->mem) (void)hipFree(s->mem);
    if (s->ev0) (void)hipEventDestroy(s->ev0);
    if (s->ev1) (void)hipEventDestroy(s->ev1);
    delete s;
    return NV_OK;
}

NV_API nv_status nv_sur_set_params(nv_sur *s, const float *host) {
    if (!s || !host) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    for (int i = 0; i < kParams; ++i)
        if (!std::isfinite(host[i])) return fail(NV_ERR_INVALID_ARG, "parameter %d is not finite", i);
    NV_HIP(hipMemcpyAsync(s->params, host, kParams * sizeof(float), hipMemcpyHostToDevice,
                          s->stream));
    NV_HIP(hipMemsetAsync(s->m, 0, kParams * sizeof(float), s->stream));
    NV_HIP(hipMemsetAsync(s->v, 0, kParams * sizeof(float), s->stream));
    s->adam_t = 0;
    nv_status st = refresh_shadow(s);
    if (st != NV_OK) return st;
    NV_HIP(hipStreamSynchronize(s->stream));
    return NV_OK;
}

NV_API nv_status nv_sur_get_params(nv_sur *s, float *host) {
    if (!s || !host) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    NV_HIP(hipMemcpyAsync(host, s->params, kParams * sizeof(float), hipMemcpyDeviceToHost,
                          s->stream));
    NV_HIP(hipStreamSynchronize(s->stream));
    return NV_OK;
}

NV_API nv_status nv_sur_forward(nv_sur *s, const float *x, long long n, float *out) {
    if (!s || !x || !out) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (n < 1) return fail(NV_ERR_INVALID_ARG, "n = %lld", n);
    ForwardArgs fa{};
    fa.params = s->params;
    fa.shadow = s->shadow;
    fa.x = x;
    fa.out = out;
    fa.n = n;
    fill_norm(s, fa.shift, fa.scale);
    const long long blocks = (n + 63) / 64;
    if (blocks > 0x7fffffffLL) return fail(NV_ERR_INVALID_ARG, "n = %lld is too large", n);
    NV_HIP(hipEventRecord(s->ev0, s->stream));
    hipLaunchKernelGGL(sur_forward_kernel, dim3(unsigned(blocks)), dim3(kInferThreads), 0,
                       s->stream, fa);
    NV_HIP(hipGetLastError());
    NV_HIP(hipEventRecord(s->ev1, s->stream));
    NV_HIP(hipStreamSynchronize(s->stream));
    NV_HIP(hipEventElapsedTime(&s->last_ms, s->ev0, s->ev1));
    return NV_OK;
}

NV_API nv_status nv_sur_loss_grad(nv_sur *s, const float *x, const float *t, long long n,
                                  float *loss_host, float *grad_host) {
    if (!s || !x || !t || !loss_host) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (n < 16 || n % 16 != 0 || n > s->max_batch)
        return fail(NV_ERR_INVALID_ARG, "n = %lld: need a multiple of 16 in [16, %lld]", n,
                    s->max_batch);
    nv_status st = minibatch(s, x, t, n, 0, n, kModeReduce, 0.f, 0.f, 0.f, 0.f, s->loss);
    if (st != NV_OK) return st;
    NV_HIP(hipMemcpyAsync(loss_host, s->loss, sizeof(float), hipMemcpyDeviceToHost, s->stream));
    if (grad_host)
        NV_HIP(hipMemcpyAsync(grad_host, s->grad, kParams * sizeof(float), hipMemcpyDeviceToHost,
                              s->stream));
    NV_HIP(hipStreamSynchronize(s->stream));
    return NV_OK;
}

NV_API nv_status nv_sur_train(nv_sur *s, const float *x, const float *t, long long n_samples,
                              const nv_sur_train_opts *o, float *loss_dev) try {
    if (!s || !x || !t || !o) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    const long long B = o->batch;
    if (B < 16 || B % 16 != 0 || B > s->max_batch)
        return fail(NV_ERR_INVALID_ARG, "batch %lld: need a multiple of 16 in [16, %lld]", B,
                    s->max_batch);
    if (n_samples < B || n_samples % B != 0)
        return fail(NV_ERR_INVALID_ARG, "n_samples %lld is not a positive multiple of batch %lld",
                    n_samples, B);
    if (o->steps < 0) return fail(NV_ERR_INVALID_ARG, "steps < 0");
    const float lr = o->lr > 0.f ? o->lr : 1e-3f;
    const float b1 = o->beta1 > 0.f ? o->beta1 : 0.9f;
    const float b2 = o->beta2 > 0.f ? o->beta2 : 0.999f;
    const float eps = o->eps > 0.f ? o->eps : 1e-8f;
    if (!(lr < 1.f) || !(b1 < 1.f) || !(b2 < 1.f) || !std::isfinite(o->lr_final) ||
        o->lr_final < 0.f)
        return fail(NV_ERR_INVALID_ARG, "Adam hyper-parameters out of range");
    NV_HIP(hipEventRecord(s->ev0, s->stream));
    const double decay = (o->lr_final > 0.f && o->steps > 1)
                             ? std::log(double(o->lr_final) / double(lr)) / double(o->steps - 1)
                             : 0.0;
    for (long long k = 0; k < o->steps; ++k) {
        const long long start = (s->adam_t * B) % n_samples;   // steps since set_params
        const float lrk = float(double(lr) * std::exp(decay * double(k)));
        nv_status st = minibatch(s, x, t, n_samples, start, B, kModeReduce | kModeAdam, lrk, b1,
                                 b2, eps, loss_dev ? loss_dev + k : nullptr);
        if (st != NV_OK) return st;
    }
    NV_HIP(hipEventRecord(s->ev1, s->stream));
    NV_HIP(hipStreamSynchronize(s->stream));
    NV_HIP(hipEventElapsedTime(&s->last_ms, s->ev0, s->ev1));
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_sur_train: host allocation failed");
}

NV_API nv_status nv_sur_dataset_from_batch(nv_sur *s, nv_batch *batch, const long long *perm,
                                           float *x, float *t, long long cap, long long *total) try {
    if (!s || !batch || !total) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    std::vector<nv::SliceMapSource> src;
    int precision = 0;
    nv_status st = nv::batch_slice_sources(batch, src, &precision);
    if (st != NV_OK) return st;
    long long n = 0;
    for (size_t i = 0; i < src.size(); ++i) {
        const double L = s->cfg.slice_length;
        if (std::fabs(src[i].L - L) > 1e-9 * L)
            return fail(NV_ERR_INVALID_ARG, "problem %zu has slices of length %.17g, the "
                        "network is configured for %.17g", i, src[i].L, L);
        n += src[i].M * src[i].n_slices;
    }
    *total = n;
    if (!x && !t) return NV_OK;
    if (!x || !t) return fail(NV_ERR_INVALID_ARG, "x and target must both be given");
    if (cap < n) return fail(NV_ERR_INVALID_ARG, "capacity %lld < %lld samples", cap, n);
    if (s->cfg.correction == NV_SUR_STEP_DOUBLING && s->cfg.coarse_steps < 1)
        return fail(NV_ERR_INVALID_ARG, "the step-doubling form needs coarse_steps >= 1");
    void *dsrc = nullptr;
    NV_HIP(hipMalloc(&dsrc, src.size() * sizeof(nv::SliceMapSource)));
    hipError_t e = hipMemcpyAsync(dsrc, src.data(), src.size() * sizeof(nv::SliceMapSource),
                                  hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(s->error, 0, sizeof(int), s->stream);
    if (e == hipSuccess) {
        DatasetArgs da{};
        da.src = static_cast<const nv::SliceMapSource *>(dsrc);
        da.n_src = int(src.size());
        da.fp64 = precision == NV_FP64;
        da.total = n;
        da.cap = cap;
        da.perm = perm;
        da.x = x;
        da.t = t;
        da.os0 = s->cfg.out_scale[0];
        da.os1 = s->cfg.out_scale[1];
        da.coarse = s->cfg.coarse_steps;
        da.error = s->error;
        if (s->cfg.correction == NV_SUR_STEP_DOUBLING) {
            da.step_doubling = 1;
            da.tau2_0 = s->cfg.gate[0] * s->cfg.gate[0];
            da.tau2_1 = s->cfg.gate[1] * s->cfg.gate[1];
            da.q0 = s->cfg.loss_scale[0];
            da.q1 = s->cfg.loss_scale[1];
            if (s->visits) {
                da.visits = s->visits;
                da.n_mu = s->n_mu;
                da.n_states = s->n_states;
                da.mu_lo = s->mu_lo;
                da.mu_step = (s->mu_hi - s->mu_lo) / double(s->n_mu - 1);
                da.sc0 = s->cfg.in_scale[0];
                da.sc1 = s->cfg.in_scale[1];
                da.inv2s2 = float(1.0 / (2.0 * s->sigma * s->sigma));
                da.floor_w = float(s->floor_w);
            }
        }
        const long long blocks = std::min<long long>((n + 255) / 256, 65536);
        hipLaunchKernelGGL(sur_dataset_kernel, dim3(unsigned(blocks)), dim3(256), 0, s->stream,
                           da);
        e = hipGetLastError();
    }
    int err = 0;
    if (e == hipSuccess)
        e = hipMemcpyAsync(&err, s->error, sizeof(int), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(dsrc);
    if (e != hipSuccess)
        return fail(NV_ERR_HIP, "training-set gather failed: %s", hipGetErrorString(e));
    if (err & 1) return fail(NV_ERR_INVALID_ARG, "perm holds a position outside [0, cap)");
    if (err & 2) return fail(NV_ERR_NONFINITE, "the batch's tables hold non-finite endpoints");
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_sur_dataset_from_batch: host allocation failed");
}

NV_API nv_status nv_sur_set_visits(nv_sur *s, const double *states, int n_mu, int n_states,
                                   double mu_lo, double mu_hi, double sigma, double floor_w) {
    if (!s) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (!states) {
        s->visits = nullptr;
        return NV_OK;
    }
    if (n_mu < 2 || n_states < 1 || n_states > kMaxVisitStates)
        return fail(NV_ERR_INVALID_ARG, "need n_mu >= 2 and 1 <= n_states <= %d",
                    kMaxVisitStates);
    if (!std::isfinite(mu_lo) || !std::isfinite(mu_hi) || !(mu_hi > mu_lo) ||
        !std::isfinite(sigma) || !(sigma > 0.0) || !std::isfinite(floor_w) || floor_w < 0.0)
        return fail(NV_ERR_INVALID_ARG, "need finite mu_lo < mu_hi, sigma > 0, floor >= 0");
    s->visits = states;
    s->n_mu = n_mu;
    s->n_states = n_states;
    s->mu_lo = mu_lo;
    s->mu_hi = mu_hi;
    s->sigma = sigma;
    s->floor_w = floor_w;
    return NV_OK;
}

NV_API nv_status nv_sur_compose(nv_sur *s, const nv_sur_chains *c, nv_sur_compose_info *info) try {
    if (!s || !c || !info) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    if (c->count < 1 || c->n_slices < 1 || !c->y0 || !c->mu || !c->final_state)
        return fail(NV_ERR_INVALID_ARG, "need count >= 1, n_slices >= 1, y0, mu, final_state");
    if (!std::isfinite(c->t0) || !std::isfinite(c->T) || !(c->T > c->t0))
        return fail(NV_ERR_INVALID_ARG, "need finite t0 < T");
    ChainArgs a{};
    a.params = s->params;
    a.shadow = s->shadow;
    fill_norm(s, a.shift, a.scale);
    a.os0 = s->cfg.out_scale[0];
    a.os1 = s->cfg.out_scale[1];
    a.y0 = c->y0;
    a.mu = c->mu;
    a.count = c->count;
    a.t0 = c->t0;
    a.L = (c->T - c->t0) / double(c->n_slices);
    if (std::fabs(a.L - s->cfg.slice_length) > 1e-9 * s->cfg.slice_length)
        return fail(NV_ERR_INVALID_ARG, "slices of length %.17g; the network is configured "
                    "for %.17g", a.L, s->cfg.slice_length);
    a.coarse = s->cfg.coarse_steps;
    a.step_doubling = s->cfg.correction == NV_SUR_STEP_DOUBLING;
    a.tau2_0 = s->cfg.gate[0] * s->cfg.gate[0];
    a.tau2_1 = s->cfg.gate[1] * s->cfg.gate[1];
    a.n_slices = c->n_slices;
    a.final_state = c->final_state;
    a.boundary = c->boundary;
    a.blo0 = c->box_lo[0];
    a.blo1 = c->box_lo[1];
    a.bhi0 = c->box_hi[0];
    a.bhi1 = c->box_hi[1];
    a.guard = c->guard;
    if (c->fb_tab0) {
        const nv_ic_grid &g = c->fb_grid;
        if (!c->fb_tab1 || g.dim != 2 || g.interp != NV_INTERP_BILINEAR || g.n[0] < 2 ||
            g.n[1] < 2 || !std::isfinite(g.lo[0]) || !std::isfinite(g.hi[0]) ||
            !std::isfinite(g.lo[1]) || !std::isfinite(g.hi[1]) || !(g.hi[0] > g.lo[0]) ||
            !(g.hi[1] > g.lo[1]) ||
            (c->fb_precision != NV_FP32 && c->fb_precision != NV_FP64))
            return fail(NV_ERR_INVALID_ARG, "the fallback needs two tables of a 2-D bilinear grid");
        a.tab0 = c->fb_tab0;
        a.tab1 = c->fb_tab1;
        a.fb_fp64 = c->fb_precision == NV_FP64;
        a.M = (long long)g.n[0] * g.n[1];
        a.n0 = g.n[0];
        a.n1 = g.n[1];
        a.lo0 = g.lo[0];
        a.lo1 = g.lo[1];
        a.inv0 = double(g.n[0] - 1) / (g.hi[0] - g.lo[0]);
        a.inv1 = double(g.n[1] - 1) / (g.hi[1] - g.lo[1]);
    }
    const unsigned long long init[4] = {0ull, 0ull, 0ull, ~0ull};
    NV_HIP(hipMemcpyAsync(s->stats, init, sizeof init, hipMemcpyHostToDevice, s->stream));
    a.stats = s->stats;
    const long long blocks = (c->count + 15) / 16;
    if (blocks > 0x7fffffffLL) return fail(NV_ERR_INVALID_ARG, "too many chains");
    NV_HIP(hipEventRecord(s->ev0, s->stream));
    hipLaunchKernelGGL(sur_chain_kernel, dim3(unsigned(blocks)), dim3(kInferThreads), 0,
                       s->stream, a);
    NV_HIP(hipGetLastError());
    NV_HIP(hipEventRecord(s->ev1, s->stream));
    unsigned long long st[4];
    NV_HIP(hipMemcpyAsync(st, s->stats, sizeof st, hipMemcpyDeviceToHost, s->stream));
    NV_HIP(hipStreamSynchronize(s->stream));
    NV_HIP(hipEventElapsedTime(&s->last_ms, s->ev0, s->ev1));
    info->n_fallback = (long long)st[0];
    info->n_outside = (long long)st[1];
    double md;
    std::memcpy(&md, &st[2], sizeof md);
    info->max_deviation = md;
    info->bad_chain = st[3] == ~0ull ? -1 : (long long)st[3];
    info->ms = s->last_ms;
    if (info->bad_chain >= 0)
        return fail(NV_ERR_NONFINITE, "chain %lld became non-finite", info->bad_chain);
    return NV_OK;
} catch (const std::bad_alloc &) {
    return fail(NV_ERR_OOM, "nv_sur_compose: host allocation failed");
}

NV_API nv_status nv_sur_last_ms(nv_sur *s, float *ms) {
    if (!s || !ms) return fail(NV_ERR_INVALID_ARG, "NULL argument");
    *ms = s->last_ms;
    return NV_OK;
}

}  // extern "C"
