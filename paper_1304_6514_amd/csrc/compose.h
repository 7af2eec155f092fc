// Device code of the communication phase of Nievergelt's method (sec. 3,
// pseudocode figure): the lookup, the interpolants and the dependent chain
// lambda_{j+1} = phi^j(lambda_j) over a range of slices.  Every floating-point
// operation is one IEEE binary64 operation with no contraction, so that the
// result over given tables is specified bit for bit (include/nv.h).
#pragma once

#include "nv_internal.h"

#include <cmath>

namespace nv {
namespace dev {

// Cell and local coordinate of x on one axis.  Returns 1 when x lies outside
// [lo, hi] (the lookup then extrapolates from the edge cell).  A NaN query
// gives cell 0, w = NaN and counts as outside.
__device__ inline int locate(double lo, double inv, int n, double x, long long &cell,
                             double &w) {
#pragma clang fp contract(off)
    const double u = (x - lo) * inv;
    if (u != u) {
        cell = 0;
        w = u;
        return 1;
    }
    const double f = floor(u);
    long long i;
    if (f < 0.0)
        i = 0;
    else if (f > double(n - 2))
        i = n - 2;
    else
        i = (long long)f;
    cell = i;
    w = u - double(i);
    return (u < 0.0 || u > double(n - 1)) ? 1 : 0;
}

__device__ inline bool finite(double v) { return isfinite(v); }

// Delta-xi times the slope at node i of a 1-D table row, by finite differences;
// get(k) gives node k's table value.
template <class F>
__device__ inline double node_slope_f(const F &get, long long i, int n) {
#pragma clang fp contract(off)
    if (i == 0) {
        const double t0 = get(0), t1 = get(1), t2 = get(2);
        return 0.5 * ((4.0 * t1 - 3.0 * t0) - t2);
    }
    if (i == n - 1) {
        const double a = get(n - 1), b = get(n - 2), c = get(n - 3);
        return 0.5 * ((3.0 * a - 4.0 * b) + c);
    }
    return 0.5 * (get(i + 1) - get(i - 1));
}

template <class T>
__device__ inline double node_slope(const T *row, long long i, int n) {
    return node_slope_f([row](long long k) { return double(row[k]); }, i, n);
}

// The start of a range of slices: y0 (a range from slice 0 also resets the
// running status and writes lambda_0) or the state the previous range carried
// over.  Returns false when an earlier range already failed.  Everything the
// next range needs stays in device memory; the boundary states and the final
// status may live in host-mapped memory, which the chain only writes.
template <int D>
__device__ inline bool range_begin(const ComposeArgs &a, int lane, double &l0, double &l1) {
    if (a.j_begin == 0) {
        l0 = a.y00;
        l1 = a.y01;
        if (lane == 0) {
            a.boundary[0] = l0;
            if (D == 2) a.boundary[1] = l1;
            a.status->n_out_of_grid = 0;
            a.status->bad_slice = -1;
            a.status->done = 0;
        }
        return true;
    }
    if (a.status->bad_slice >= 0) return false;
    l0 = a.carry[0];
    l1 = a.carry[1];
    return true;
}

// The end of a range: the running status, the carried state and, when the
// chain ends here, a copy of the final status.
__device__ inline void range_end(const ComposeArgs &a, int lane, double l0, double l1,
                                 long long oog, int bad_slice) {
    if (lane != 0) return;
    const long long total = a.status->n_out_of_grid + oog;
    a.status->n_out_of_grid = total;
    if (bad_slice >= 0) a.status->bad_slice = bad_slice;
    const bool last = a.j_end == a.n_slices || bad_slice >= 0;
    if (last) a.status->done = 1;
    if (a.carry) {
        a.carry[0] = l0;
        a.carry[1] = l1;
    }
    if (last && a.status_host) {
        a.status_host->n_out_of_grid = total;
        a.status_host->bad_slice = bad_slice;
        a.status_host->done = 1;
    }
}

// Composes slices j_begin .. j_end-1, run by one whole wave: every lane takes
// the same chain (uniform values, uniform loads, so the result is that of one
// lane), and lane l keeps the boundary state of slice jb + l + 1 of the current
// block of 64 slices; a block is written out with one coalesced store.  No
// store then sits between one slice's loads and the next's (the memory counter
// is in order, so a load issued after a store would also wait for the store):
// the chain waits for a store once per 64 slices.  A launch that starts at
// slice 0 takes y0 from its arguments and resets the status; a later launch
// resumes from the boundary state the previous one left in memory and adds to
// the status.  With final_out, the last state (that of the failing slice's
// start when one fails) is also returned there ([dim]).
template <class T, int Interp>
__device__ inline void compose_range(const ComposeArgs &a, double *final_out = nullptr) {
#pragma clang fp contract(off)
    constexpr int D = Interp == 2 ? 2 : 1;
    const int lane = int(threadIdx.x) & 63;
    const T *tab0 = static_cast<const T *>(a.tab0);
    const T *tab1 = static_cast<const T *>(a.tab1);
    double lam0 = 0.0, lam1 = 0.0;
    if (!range_begin<D>(a, lane, lam0, lam1)) return;     // an earlier range already failed
    long long oog = 0;
    int bad_slice = -1;
    double keep0 = 0.0, keep1 = 0.0;
    int jb = a.j_begin;                           // first slice of the current block
    int j = a.j_begin;
    for (; j < a.j_end; ++j) {
        if (!finite(lam0) || (D == 2 && !finite(lam1))) {
            bad_slice = j;
            break;
        }
        const T *row0 = tab0 + (long long)j * a.M;
        long long i0, i1;
        double w0, w1;
        oog += locate(a.lo0, a.inv0, a.n0, lam0, i0, w0);
        double next0, next1 = 0.0;
        bool bad = false;
        if constexpr (Interp == 0) {
            const double ta = double(row0[i0]), tb = double(row0[i0 + 1]);
            bad = !finite(ta) || !finite(tb);
            next0 = ta + w0 * (tb - ta);
        } else if constexpr (Interp == 1) {
            const double ta = double(row0[i0]), tb = double(row0[i0 + 1]);
            const double da = node_slope(row0, i0, a.n0), db = node_slope(row0, i0 + 1, a.n0);
            const double w2 = w0 * w0, w3 = w2 * w0;
            const double h00 = (2.0 * w3 - 3.0 * w2) + 1.0;
            const double h10 = (w3 - 2.0 * w2) + w0;
            const double h01 = 3.0 * w2 - 2.0 * w3;
            const double h11 = w3 - w2;
            bad = !finite(ta) || !finite(tb) || !finite(da) || !finite(db);
            next0 = ((h00 * ta + h10 * da) + h01 * tb) + h11 * db;
        } else {
            oog += locate(a.lo1, a.inv1, a.n1, lam1, i1, w1);
            const long long c00 = i0 * a.n1 + i1, c10 = (i0 + 1) * a.n1 + i1;
            const T *row1 = tab1 + (long long)j * a.M;
            const double p00 = double(row0[c00]), p01 = double(row0[c00 + 1]);
            const double p10 = double(row0[c10]), p11 = double(row0[c10 + 1]);
            const double q00 = double(row1[c00]), q01 = double(row1[c00 + 1]);
            const double q10 = double(row1[c10]), q11 = double(row1[c10 + 1]);
            bad = !finite(p00) || !finite(p01) || !finite(p10) || !finite(p11) ||
                  !finite(q00) || !finite(q01) || !finite(q10) || !finite(q11);
            const double r0 = p00 + w1 * (p01 - p00), r1 = p10 + w1 * (p11 - p10);
            const double s0 = q00 + w1 * (q01 - q00), s1 = q10 + w1 * (q11 - q10);
            next0 = r0 + w0 * (r1 - r0);
            next1 = s0 + w0 * (s1 - s0);
        }
        if (bad) {
            bad_slice = j;
            break;
        }
        lam0 = next0;
        lam1 = next1;
        if (lane == j - jb) {
            keep0 = lam0;
            keep1 = lam1;
        }
        if (j - jb == 63) {
            a.boundary[(long long)(jb + lane + 1) * D] = keep0;
            if (D == 2) a.boundary[(long long)(jb + lane + 1) * D + 1] = keep1;
            jb += 64;
        }
    }
    // the states of the last, partial block (slices jb .. j-1)
    if (lane < j - jb) {
        a.boundary[(long long)(jb + lane + 1) * D] = keep0;
        if (D == 2) a.boundary[(long long)(jb + lane + 1) * D + 1] = keep1;
    }
    range_end(a, lane, lam0, lam1, oog, bad_slice);
    if (final_out) {
        final_out[0] = lam0;
        if (D == 2) final_out[1] = lam1;
    }
}

// The chain with Lagrange interpolation on Chebyshev nodes (paper mode), run
// by one wave of 64 lanes, lane k < M owning node k.  For each slice, lane k
// forms its term t[k] * prod_m f_km, f_km = (x - xi_m) / (xi_k - xi_m) (the
// diagonal factor is exactly 1, so multiplying by it changes nothing), with m
// ascending; its M divisions are independent of one another, so they overlap.
// The terms are then summed in ascending k by reading them lane by lane
// (v_readlane: no LDS, no barrier).  This is exactly the operation sequence of
// the written rule, so the result is the same to the bit.
constexpr int kMaxLagrange = 64;

__device__ inline double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(b & 0xffffffffLL), l));
    const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(b >> 32), l));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Table rows staged in LDS per refill: the rows of a range are loaded in
// chunks of kLagrangeStage values with all loads in flight at once, and the
// boundary states of a chunk are collected in LDS and written out after it, so
// that no global memory operation sits inside the dependent chain (a store in
// flight would make the next load wait: the memory counter is in order).
constexpr int kLagrangeStage = 4096;

// The Lagrange value of one slice: lane k < M holds node xk and table value
// vk; MC > 0 is the node count as a compile-time constant (its M independent
// divisions are then unrolled and overlap), MC = 0 a run-time M.
template <int MC>
__device__ inline double lagrange_value(double lam, double xk, double vk, int lane, int M) {
#pragma clang fp contract(off)
    constexpr int kUnroll = MC > 0 ? MC : 1;
    const int Mn = MC > 0 ? MC : M;
    double term = vk;
#pragma unroll kUnroll
    for (int m = 0; m < Mn; ++m) {
        const double xm = readlane_f64(xk, m);
        const double f = (lam - xm) / (xk - xm);
        term *= (m == lane) ? 1.0 : f;
    }
    double sum = 0.0;
#pragma unroll kUnroll
    for (int k = 0; k < Mn; ++k) sum += readlane_f64(term, k);
    return sum;
}

// The same value for a compile-time node count MC <= 8, with the M*M
// quotients spread over the wave: lane k*MC + m forms f_km = (lam - x_m) /
// den_km, den_km = x_k - x_m (the same operands as above, so the same
// quotient), all in one division step, where the form above takes M divisions
// one after another (each ends in v_div_fmas, which reads VCC, so two cannot
// overlap).  Lane k < MC then gathers f_k0 .. f_k(MC-1) and multiplies them into
// its term in ascending m, the factor with m = k replaced by 1 as above, and the
// terms are summed in ascending k: the operation sequence of lagrange_value.
template <int MC>
__device__ inline double lagrange_value_pairs(double lam, double x_m, double den, double vk,
                                              int lane) {
#pragma clang fp contract(off)
    static_assert(MC >= 1 && MC * MC <= 64, "one quotient per lane");
    const double f = (lam - x_m) / den;
    const int src0 = lane < MC ? lane * MC : 0;
    double term = vk;
#pragma unroll
    for (int m = 0; m < MC; ++m) {
        const double fm = __shfl(f, src0 + m);
        term *= (m == lane) ? 1.0 : fm;
    }
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < MC; ++k) sum += readlane_f64(term, k);
    return sum;
}

template <class T, int MC>
__device__ inline void lagrange_chain(const ComposeArgs &a, double *rows, double *bnd) {
#pragma clang fp contract(off)
    const int lane = int(threadIdx.x);
    const int M = a.n0;
    const double xk = lane < M ? a.nodes[lane] : 0.0;
    // lane k*MC + m (< MC*MC) of the spread quotients: x_m and x_k - x_m (zero
    // for k = m, whose quotient is never used)
    double pair_xm = 0.0, pair_den = 1.0;
    if (MC > 0 && MC <= 8 && lane < MC * MC) {
        const int pk = lane / (MC > 0 ? MC : 1), pm = lane - pk * MC;
        pair_xm = a.nodes[pm];
        pair_den = a.nodes[pk] - pair_xm;
    }
    const T *tab0 = static_cast<const T *>(a.tab0);
    double lam = 0.0, unused = 0.0;
    if (!range_begin<1>(a, lane, lam, unused)) return;    // an earlier range already failed
    long long oog = 0;
    int bad_slice = -1;
    const int rows_per_chunk = kLagrangeStage / M;
    for (int c0 = a.j_begin; c0 < a.j_end && bad_slice < 0; c0 += rows_per_chunk) {
        const int c1 = c0 + rows_per_chunk < a.j_end ? c0 + rows_per_chunk : a.j_end;
        __syncthreads();                          // the previous chunk is consumed
        const long long base = (long long)c0 * M, count = (long long)(c1 - c0) * M;
        // the chunk's first row holding a non-finite value, found while staging
        // it, so that the chain itself needs no vote per slice
        int first_bad = c1;
        for (long long i = lane; i < count; i += int(blockDim.x)) {
            const double v = double(tab0[base + i]);
            rows[i] = v;
            if (!finite(v) && c0 + int(i / M) < first_bad) first_bad = c0 + int(i / M);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const int other = __shfl_xor(first_bad, o);
            first_bad = other < first_bad ? other : first_bad;
        }
        __syncthreads();
        int done = c0;                            // boundary states bnd[0 .. done-c0) ready
        double vk = lane < M ? rows[lane] : 0.0;
        for (int j = c0; j < c1; ++j) {
            if (!finite(lam) || j == first_bad) {
                bad_slice = j;
                break;
            }
            // the next slice's table values, read ahead of the chain
            const double vnext = (lane < M && j + 1 < c1) ? rows[(j + 1 - c0) * M + lane] : 0.0;
            double next;
            if constexpr (MC > 0 && MC <= 8)
                next = lagrange_value_pairs<MC>(lam, pair_xm, pair_den, vk, lane);
            else
                next = lagrange_value<MC>(lam, xk, vk, lane, M);
            oog += (lam < a.lo0 || lam > a.hi0) ? 1 : 0;
            lam = next;
            if (lane == 0) bnd[j - c0] = lam;
            done = j + 1;
            vk = vnext;
        }
        __syncthreads();
        for (int i = lane; i < done - c0; i += int(blockDim.x)) a.boundary[c0 + 1 + i] = bnd[i];
    }
    range_end(a, lane, lam, 0.0, oog, bad_slice);
}

template <class T>
__device__ inline void compose_range_lagrange(const ComposeArgs &a) {
    __shared__ double rows[kLagrangeStage];
    __shared__ double bnd[kLagrangeStage / 2];
    switch (a.n0) {
    case 2: lagrange_chain<T, 2>(a, rows, bnd); break;
    case 3: lagrange_chain<T, 3>(a, rows, bnd); break;
    case 4: lagrange_chain<T, 4>(a, rows, bnd); break;
    case 5: lagrange_chain<T, 5>(a, rows, bnd); break;
    case 6: lagrange_chain<T, 6>(a, rows, bnd); break;
    case 7: lagrange_chain<T, 7>(a, rows, bnd); break;
    case 8: lagrange_chain<T, 8>(a, rows, bnd); break;
    default: lagrange_chain<T, 0>(a, rows, bnd); break;
    }
}

}  // namespace dev
}  // namespace nv
