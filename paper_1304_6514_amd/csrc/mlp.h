// Device code of the learned slice-map surrogate: a 4 -> 128 -> 128 -> 128 -> 2
// perceptron with the exact GELU, run by 64-lane waves on gfx950 matrix cores.
//
// Data layout inside a wave.  A wave works on 16 samples at a time; lane l
// holds sample l % 16 and, of every 128-wide layer, the 32 features
//     f = 16 mt + 4 g + i,     mt = 0..7, i = 0..3, g = l / 16,
// i.e. exactly the accumulator layout of v_mfma_f32_16x16x32_bf16 when the
// layer is computed transposed (features x samples = W x activations^T):
// accumulator register i of lane l is row 4 (l / 16) + i, column l % 16.
// The operand B of the next layer (32 features x 16 samples per instruction)
// must hold, in lane l, 8 features of sample l % 16; the lane already holds 8
// features of each 32-feature block -- {4g..4g+3} and {16+4g..16+4g+3} -- so
// the activations stay in registers from layer to layer provided the weight
// matrix (operand A) lists its columns in that order.  The library therefore
// keeps each 128 x 128 weight matrix as bfloat16 with the columns of every
// 32-block permuted by perm32 (forward: W, back-propagation: W^T).
#pragma once

#include "nv_internal.h"

#include <cmath>

namespace nv {
namespace mlp {

constexpr int kIn = 4, kWidth = 128, kOut = 2;
// flat parameter vector: W1, b1, W2, b2, W3, b3, W4, b4
constexpr int kW1 = 0, kB1 = 512, kW2 = 640, kB2 = kW2 + 16384, kW3 = kB2 + 128,
              kB3 = kW3 + 16384, kW4 = kB3 + 128, kB4 = kW4 + 256, kParams = kB4 + 2;
static_assert(kParams == 33922, "parameter count of the 4-128-128-128-2 network");

constexpr int kMat = kWidth * kWidth;  // elements of one 128 x 128 matrix
constexpr int kLdsRow = kWidth + 8;    // padded bf16 row in LDS: 272 bytes, 16-lane reads
                                       // of 16 bytes from 16 rows hit disjoint banks

// Training workspace S: bfloat16 rows of one value per sample of the minibatch.
constexpr int kRowD = 0;      // 384 rows: dL/dz of layers 1, 2, 3
constexpr int kRowH = 384;    // 384 rows: bf16 activations a1, a2, a3
constexpr int kRowXO = 768;   // 16 rows: u0..u3, 1, dL/dout0, dL/dout1, zeros
constexpr int kRowsS = 784;

// Weight-gradient sums G = A B^T over the minibatch, A and B row blocks of S.
// Their outputs, concatenated, form one partial vector per split of the sum.
constexpr int kG_W2 = 0;                    // [128 x 128]  D2 . H1^T
constexpr int kG_W3 = 16384;                // [128 x 128]  D3 . H2^T
constexpr int kG_D_XO = 32768;              // [384 x 16]   D . XO^T  (dW1, db1; db2, db3 in column 4)
constexpr int kG_XO_H3 = 32768 + 384 * 16;  // [16 x 144]   XO . [H3; XO]^T  (dW4, db4)
constexpr int kGradEntries = kG_XO_H3 + 16 * 144;
constexpr int kGemmWaveTiles = 16 + 16 + 4 + 5;
constexpr int kGemmSmallFirst = 32;         // wave tiles of the two small products

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Position kp (0..31) of a 32-block of the matrix-core k index -> feature
// offset inside the block, and back.
__host__ __device__ constexpr int perm32(int kp) {
    return (kp & 7) < 4 ? 4 * (kp >> 3) + (kp & 7) : 16 + 4 * (kp >> 3) + ((kp & 7) - 4);
}
__host__ __device__ constexpr int perm32_inv(int f) {
    return f < 16 ? 8 * (f >> 2) + (f & 3) : 8 * ((f - 16) >> 2) + 4 + ((f - 16) & 3);
}

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// gelu(z) = z Phi(z) and its derivative Phi(z) + z phi(z), Phi and phi the
// standard normal distribution and density.  erf is evaluated branch-free by
// the rational approximation of Abramowitz and Stegun, Handbook of
// Mathematical Functions, formula 7.1.26 (absolute error below 1.5e-7, the
// size of an FP32 rounding of Phi): for x >= 0, with t = 1 / (1 + p x),
//     erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-x^2),
// and erf(-x) = -erf(x), at x = |z| / sqrt 2.  The constants are folded so
// that one exponential gives the density itself: with u = |z| sqrt(log2(e)/2),
// phi(z) = 2^(L - u^2), L = log2(1/sqrt(2 pi)); t = 1 / (1 + (p / sqrt(log2 e)) u);
// and with b_k = a_k sqrt(2 pi) / 2, t (b1 + t (b2 + ...)) phi(z) is
// (1 - erf(|z|/sqrt 2)) / 2, the tail 1 - Phi(|z|).
__device__ inline float gelu_d(float z, float &d) {
    constexpr float c = 0.84932180028801904f;    // sqrt(log2(e) / 2)
    constexpr float pq = 0.27273748087922250f;   // 0.3275911 / sqrt(log2 e)
    constexpr float L = -1.32574806473615920f;   // log2(1 / sqrt(2 pi))
    constexpr float b1 = 0.31938153025994087f, b2 = -0.35656378124891560f,
                    b3 = 1.78147793656981280f, b4 = -1.82125597910777540f,
                    b5 = 1.33027442958912310f;   // a_k sqrt(2 pi) / 2
    const float u = fabsf(z) * c;
    const float t = __builtin_amdgcn_rcpf(fmaf(pq, u, 1.0f));
    const float phi = __builtin_amdgcn_exp2f(fmaf(-u, u, L));
    const float tail = (t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, b5, b4), b3), b2), b1)) * phi;
    const float P = z >= 0.0f ? 1.0f - tail : tail;
    d = fmaf(z, phi, P);
    return z * P;
}

// Per-lane values of one 128-wide layer for the lane's sample (see above).
struct Layer {
    f32x4 v[8];
};

// Layer values -> the four bfloat16 B operands of the next matrix product.
__device__ inline void pack(const Layer &x, bf16x8 (&b)[4]) {
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            b[kb][e] = __bf16(x.v[2 * kb][e]);
            b[kb][e + 4] = __bf16(x.v[2 * kb + 1][e]);
        }
    }
}

// out = M . act^T for a 128 x 128 matrix M held in LDS in the permuted layout
// (kLdsRow-padded rows); act given as B operands.
__device__ inline void matmul(const __bf16 *M, const bf16x8 (&b)[4], Layer &out, int lane) {
    const int r = lane & 15, g = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 8; mt += 2) {
        // two output tiles at a time: eight operand reads in flight, two
        // independent accumulation chains, and a bounded register footprint
        asm volatile("" ::: "memory");
        f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0;
        const __bf16 *row0 = M + (16 * mt + r) * kLdsRow + 8 * g;
        const __bf16 *row1 = row0 + 16 * kLdsRow;
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            acc0 = mfma(*reinterpret_cast<const bf16x8 *>(row0 + 32 * kb), b[kb], acc0);
            acc1 = mfma(*reinterpret_cast<const bf16x8 *>(row1 + 32 * kb), b[kb], acc1);
        }
        out.v[mt] = acc0;
        out.v[mt + 1] = acc1;
    }
}

// The small FP32 parameters every kernel keeps in LDS.
struct SmallParams {
    float w1[kWidth * kIn];
    float b1[kWidth], b2[kWidth], b3[kWidth];
    float w4[kOut * kWidth];
    float b4[kOut];
};

// The small parameters into LDS: every thread's loads are issued before the
// first store to LDS (a store right after each load would make each thread
// wait for its loads one at a time).
template <int kThreads>
__device__ inline void load_small(SmallParams &sp, const float *params, int tid) {
    constexpr int kN = kWidth * kIn + 3 * kWidth + kOut * kWidth + kOut;   // 1154 values
    constexpr int kIter = (kN + kThreads - 1) / kThreads;
    static_assert(sizeof(SmallParams) == kN * sizeof(float), "SmallParams is the flat list");
    // SmallParams holds w1, b1, b2, b3, w4, b4; in the flat parameter vector
    // the matrices W2, W3 sit between them
    float v[kIter];
#pragma unroll
    for (int i = 0; i < kIter; ++i) {
        int e = tid + i * kThreads;
        e = e < kN ? e : kN - 1;                   // in bounds, no select after the load
        const int b1 = kWidth * kIn, b2 = b1 + kWidth, b3 = b2 + kWidth, w4 = b3 + kWidth;
        const int src = e < b1   ? kW1 + e
                        : e < b2 ? kB1 + (e - b1)
                        : e < b3 ? kB2 + (e - b2)
                        : e < w4 ? kB3 + (e - b3)
                                 : kW4 + (e - w4);   // W4 then b4, adjacent in both
        v[i] = params[src];
    }
    float *dst = reinterpret_cast<float *>(&sp);
#pragma unroll
    for (int i = 0; i < kIter; ++i) {
        const int e = tid + i * kThreads;
        if (e < kN) dst[e] = v[i];
    }
}

// Copy kMats permuted bf16 matrices from global memory into padded LDS rows,
// every thread's 16-byte loads issued before its first store to LDS.
template <int kMats, int kThreads>
__device__ inline void load_mats(__bf16 *lds, const __bf16 *src, int tid) {
    constexpr int kChunks = kMats * kWidth * (kWidth / 8);      // 16-byte chunks
    constexpr int kIter = (kChunks + kThreads - 1) / kThreads;
    bf16x8 v[kIter];
#pragma unroll
    for (int i = 0; i < kIter; ++i) {
        int c = tid + i * kThreads;
        c = c < kChunks ? c : kChunks - 1;         // in bounds, no select after the load
        v[i] = *reinterpret_cast<const bf16x8 *>(src + size_t(c) * 8);
    }
#pragma unroll
    for (int i = 0; i < kIter; ++i) {
        const int c = tid + i * kThreads;
        if (c < kChunks) {
            const int m = c / (kWidth * 16), rem = c - m * kWidth * 16;
            const int row = rem >> 4, col = (rem & 15) * 8;
            *reinterpret_cast<bf16x8 *>(lds + (m * kWidth + row) * kLdsRow + col) = v[i];
        }
    }
}

// Where the training kernel writes a tile's rows: the workspace S (row r,
// sample n at S[r * ld + n]) at the tile's first sample.  Each lane writes its
// 32 features of its sample; the row offsets are the same in every lane, so
// they stay scalar instead of occupying vector registers.  (Routing the stores
// through an LDS transpose into 16-byte runs was measured slower.)
struct RowSink {
    __bf16 *tile;               // S + 16 * tile
    long long ld;
};

// Rows row0 + f (f = 0..127) of the tile from the lane's B operands b[kb]
// (element e of b[kb] is feature 32 kb + perm32(8 g + e)).
__device__ inline void store_rows(const RowSink &o, int row0, const bf16x8 (&b)[4], int lane) {
    const int s = lane & 15, g = lane >> 4;
    __bf16 *col = o.tile + (long long)(4 * g) * o.ld + s;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int f = 32 * kb + (e < 4 ? e : 16 + (e - 4));
            col[(long long)(row0 + f) * o.ld] = b[kb][e];
        }
    }
}

// The 16 rows starting at row0 from four values per lane (rows 4 g + r).
__device__ inline void store_rows16(const RowSink &o, int row0, const __bf16 (&v)[4], int lane) {
    const int s = lane & 15, g = lane >> 4;
    __bf16 *col = o.tile + (long long)(4 * g) * o.ld + s;
#pragma unroll
    for (int r = 0; r < 4; ++r) col[(long long)(row0 + r) * o.ld] = v[r];
}

// Forward pass of the lane's sample, u = normalised input.  Returns the two
// outputs (identical in the four lanes that share a sample) and a3.  When
// Train, also fills the hidden layers' GELU derivatives d1..d3 and stores the
// bf16 inputs of the two matrix layers (a1, a2) to the workspace rows kRowH
// and kRowH + 128 through the sink.
template <bool Train>
__device__ inline void forward(const SmallParams &sp, const __bf16 *Wf2, const __bf16 *Wf3,
                               const float (&u)[4], int lane, Layer &d1, Layer &d2, Layer &d3,
                               Layer &a3, float &o0, float &o1, const RowSink *sink) {
    const int g = lane >> 4;
    Layer x;
    bf16x8 b[4];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = 16 * mt + 4 * g + i;
            float z = sp.b1[f];
            z = fmaf(sp.w1[4 * f + 0], u[0], z);
            z = fmaf(sp.w1[4 * f + 1], u[1], z);
            z = fmaf(sp.w1[4 * f + 2], u[2], z);
            z = fmaf(sp.w1[4 * f + 3], u[3], z);
            float d;
            x.v[mt][i] = gelu_d(z, d);
            if (Train) d1.v[mt][i] = d;
        }
    }
    pack(x, b);
    if (Train) store_rows(*sink, kRowH, b, lane);
    matmul(Wf2, b, x, lane);
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = x.v[mt][i] + sp.b2[16 * mt + 4 * g + i];
            float d;
            x.v[mt][i] = gelu_d(z, d);
            if (Train) d2.v[mt][i] = d;
        }
    }
    pack(x, b);
    if (Train) store_rows(*sink, kRowH + 128, b, lane);
    matmul(Wf3, b, x, lane);
    float s0 = 0.f, s1 = 0.f;
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int f = 16 * mt + 4 * g + i;
            const float z = x.v[mt][i] + sp.b3[f];
            float d;
            const float a = gelu_d(z, d);
            if (Train) d3.v[mt][i] = d;
            a3.v[mt][i] = a;
            s0 = fmaf(sp.w4[f], a, s0);
            s1 = fmaf(sp.w4[kWidth + f], a, s1);
        }
    }
    // the four lanes of a sample hold disjoint quarters of the features
    s0 += __shfl_xor(s0, 16);
    s1 += __shfl_xor(s1, 16);
    s0 += __shfl_xor(s0, 32);
    s1 += __shfl_xor(s1, 32);
    o0 = s0 + sp.b4[0];
    o1 = s1 + sp.b4[1];
}

}  // namespace mlp
}  // namespace nv
