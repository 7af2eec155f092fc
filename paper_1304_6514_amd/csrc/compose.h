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
// gives cell 0, w = NaN and counts as outside.  The cell is floor(u) clamped
// to [0, n-2], formed without branches as u clamped to [0, n-2] and truncated
// (the same integer: truncation is floor on [0, n-2], and fmax and fmin return
// the other operand for a NaN); w = u - cell, the cell converted back exactly.
__device__ inline int locate(double lo, double inv, int n, double x, long long &cell,
                             double &w) {
#pragma clang fp contract(off)
    const double u = (x - lo) * inv;
    const int i = int(fmin(fmax(u, 0.0), double(n - 2)));
    cell = i;
    w = u - double(i);
    return (u < 0.0 || u > double(n - 1) || u != u) ? 1 : 0;
}

__device__ inline bool finite(double v) { return isfinite(v); }

// Every argument finite; the tests are combined without short-circuit
// branches (as integers), so they issue side by side.
__device__ inline bool all_finite(double a, double b) {
    return (int(finite(a)) & int(finite(b))) != 0;
}
__device__ inline bool all_finite(double a, double b, double c, double d) {
    return (int(finite(a)) & int(finite(b)) & int(finite(c)) & int(finite(d))) != 0;
}

// The lanes of the wave on which v is not finite (one class test, its result
// left in a scalar register pair).
__device__ inline unsigned long long any_nonfinite(double v) {
    return __builtin_amdgcn_ballot_w64(!isfinite(v));
}

// The 1-D interpolants of one slice at cell i0, local coordinate w0: linear
// (Interp 0) or cubic Hermite (Interp 1) with Delta-xi times the slope at node
// i taken by finite differences, (t[i+1] - t[i-1])/2 inside the row and the
// second-order one-sided forms (4 t[1] - 3 t[0] - t[2])/2 and
// (3 t[n-1] - 4 t[n-2] + t[n-3])/2 at its ends; get(k) gives node k's table
// value.  Returns false when an entry it reads (or a slope) is not finite.
// The Hermite form reads the four nodes i0-1 .. i0+2 clamped to the row, all
// at once, and picks an end's one-sided slope by selection, so no branch sits
// between the reads.
// The cubic Hermite basis at w (h00, h10, h01, h11); it does not depend on
// the table, so the chain forms it while the table values are in flight.
struct HermiteBasis {
    double h00, h10, h01, h11;
};

__device__ inline HermiteBasis hermite_basis(double w) {
#pragma clang fp contract(off)
    const double w2 = w * w, w3 = w2 * w;
    HermiteBasis b;
    b.h00 = (2.0 * w3 - 3.0 * w2) + 1.0;
    b.h10 = (w3 - 2.0 * w2) + w;
    b.h01 = 3.0 * w2 - 2.0 * w3;
    b.h11 = w3 - w2;
    return b;
}

template <int Interp>
__device__ inline bool interp_1d_values(double tm, double ta, double tb, double tp, long long i0,
                                        double w0, const HermiteBasis &hb, int n,
                                        double &next) {
#pragma clang fp contract(off)
    if constexpr (Interp == 0) {
        next = ta + w0 * (tb - ta);
        return all_finite(ta, tb);
    } else {
        // node i0 (never the last): one-sided at the first node, else central;
        // node i0+1 (never the first): one-sided at the last node, else central.
        // Both forms are formed and one is selected (no branch).
        const double da_end = 0.5 * ((4.0 * tb - 3.0 * ta) - tp), da_in = 0.5 * (tb - tm);
        const double db_end = 0.5 * ((3.0 * tb - 4.0 * ta) + tm), db_in = 0.5 * (tp - ta);
        const double da = i0 == 0 ? da_end : da_in;
        const double db = i0 + 1 == n - 1 ? db_end : db_in;
        next = ((hb.h00 * ta + hb.h10 * da) + hb.h01 * tb) + hb.h11 * db;
        return all_finite(ta, tb, da, db);
    }
}

// The bilinear interpolant of the two components from the corner values
// p (component 0) and q (component 1) of cell (i0, i1), local coordinates
// (w0, w1).  Returns true when a corner value is not finite.  The eight class
// tests are wave masks ORed in scalar registers (every lane holds the same
// values); written as plain boolean logic the compiler packs them into a
// vector bit mask, several instructions per entry.
__device__ inline bool bilinear_values(double p00, double p01, double p10, double p11,
                                       double q00, double q01, double q10, double q11,
                                       double w0, double w1, double &next0, double &next1) {
#pragma clang fp contract(off)
    const bool bad = (any_nonfinite(p00) | any_nonfinite(p01) | any_nonfinite(p10) |
                      any_nonfinite(p11) | any_nonfinite(q00) | any_nonfinite(q01) |
                      any_nonfinite(q10) | any_nonfinite(q11)) != 0;
    const double r0 = p00 + w1 * (p01 - p00), r1 = p10 + w1 * (p11 - p10);
    const double s0 = q00 + w1 * (q01 - q00), s1 = q10 + w1 * (q11 - q10);
    next0 = r0 + w0 * (r1 - r0);
    next1 = s0 + w0 * (s1 - s0);
    return bad;
}

// Nodes i0-1 (clamped to 0) and i0+2 (clamped to n-1) for the Hermite form.
__device__ inline long long node_below(long long i0) { return i0 > 0 ? i0 - 1 : 0; }
__device__ inline long long node_above(long long i0, int n) { return i0 + 2 < n ? i0 + 2 : n - 1; }

template <int Interp, class F>
__device__ inline bool interp_1d(const F &get, long long i0, double w0, int n, double &next) {
    const double ta = get(i0), tb = get(i0 + 1);
    const double tm = Interp == 1 ? get(node_below(i0)) : 0.0;
    const double tp = Interp == 1 ? get(node_above(i0, n)) : 0.0;
    const HermiteBasis hb = Interp == 1 ? hermite_basis(w0) : HermiteBasis{};
    return interp_1d_values<Interp>(tm, ta, tb, tp, i0, w0, hb, n, next);
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
// chain ends here, a copy of the final status whose done flag is written last.
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
        // the wave's boundary states and the two fields above reach host memory
        // before the flag that the host polls
        __threadfence_system();
        __hip_atomic_store(&a.status_host->done, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
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
// Cubic Hermite with stored slopes (Interp 4): node values ta, tb of cell i0
// and the slopes ma, mb the build stored for them (component 1), each times
// the grid spacing, in the basis and order of the finite-difference form.
__device__ inline bool hermite_slopes_values(double ta, double tb, double ma, double mb,
                                             double dxi, const HermiteBasis &hb, double &next) {
#pragma clang fp contract(off)
    const double da = dxi * ma, db = dxi * mb;
    next = ((hb.h00 * ta + hb.h10 * da) + hb.h01 * tb) + hb.h11 * db;
    return all_finite(ta, tb, da, db);
}

template <class T, int Interp>
__device__ inline void compose_range(const ComposeArgs &a, double *final_out = nullptr) {
#pragma clang fp contract(off)
    static_assert(Interp != 4, "stored slopes compose through the staged chain");
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
        if constexpr (Interp == 0 || Interp == 1) {
            bad = !interp_1d<Interp>([row0](long long k) { return double(row0[k]); }, i0, w0,
                                     a.n0, next0);
        } else {
            oog += locate(a.lo1, a.inv1, a.n1, lam1, i1, w1);
            const long long c00 = i0 * a.n1 + i1, c10 = (i0 + 1) * a.n1 + i1;
            const T *row1 = tab1 + (long long)j * a.M;
            const double p00 = double(row0[c00]), p01 = double(row0[c00 + 1]);
            const double p10 = double(row0[c10]), p11 = double(row0[c10 + 1]);
            const double q00 = double(row1[c00]), q01 = double(row1[c00 + 1]);
            const double q10 = double(row1[c10]), q11 = double(row1[c10 + 1]);
            bad = bilinear_values(p00, p01, p10, p11, q00, q01, q10, q11, w0, w1, next0, next1);
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

// The 1-D chain with its table windows staged ahead in LDS.  Each slice's
// table read depends on the state the previous slice produced, so its latency
// is on the chain's path.  Helper waves therefore fetch, for each coming
// slice s, a window of kPfWin consecutive values of row s around the cell the
// chain is predicted to need (the chain's latest cell, moved on at its latest
// rate per slice), once the chain is within kPfAhead slices of s, into a ring
// of kPfSlots LDS slots; the chain then pays an LDS read instead of a global
// one.  The chain takes a slice's values from its slot when the slot holds
// that slice and every value the interpolant reads, and from global memory
// otherwise; it never waits for a helper, so the values it uses, and the
// result, are the same either way.  A helper waits only for the chain's
// progress, and gives up after a bounded number of polls.  What remains per
// slice is the issue of the chain's own instructions by its one wave (the
// cell, the weights, the interpolant, the checks), which is why the loop
// keeps them few: one branch between the LDS and the global reads, central
// slopes only on the LDS path, 32-bit offsets.
constexpr int kPfHelpers = 8;      // helper waves
constexpr int kPfSlots = 16;       // staged windows
constexpr int kPfWin = 256;        // table values per window
constexpr int kPfAhead = 8;        // a window is fetched this many slices ahead
constexpr int kPfSpinMax = 1 << 20;

// C = 2 for cubic Hermite with stored slopes: a slot holds the window of the
// value row (component 0) and the same window of the slope row (component 1).
template <int C>
struct PfSharedC {
    double win[C][kPfSlots][kPfWin];
    long long tag[kPfSlots];       // (slice << 32) | first cell of the window; -1 empty
    long long hist[2];             // (slice << 32) | cell, of the last two slices the chain
                                   // finished (slice j in hist[j & 1])
    int done;                      // the chain has ended
};

template <int Interp>
using PfShared = PfSharedC<Interp == 4 ? 2 : 1>;

// The value of the wave's first active lane, held in scalar registers.  The
// chain computes the same values in every lane; taking them from one lane
// tells the compiler so, and its branches then test scalar conditions instead
// of saving, masking and restoring the execution mask around each one (a lone
// wave pays an issue slot for every instruction it runs).
__device__ inline double uniform_f64(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = unsigned(__builtin_amdgcn_readfirstlane(int(b & 0xffffffffLL)));
    const unsigned hi = unsigned(__builtin_amdgcn_readfirstlane(int(b >> 32)));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ inline long long uniform_i64(long long v) {
    const unsigned lo = unsigned(__builtin_amdgcn_readfirstlane(int(v & 0xffffffffLL)));
    const unsigned hi = unsigned(__builtin_amdgcn_readfirstlane(int(v >> 32)));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ inline bool uniform_bool(bool v) {
    return __builtin_amdgcn_readfirstlane(v ? 1 : 0) != 0;
}

__device__ inline double pf_read(const double *w, unsigned k) {
    return __hip_atomic_load(w + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline long long pf_pack(int hi, long long lo) {
    return (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}

template <class T, int Interp>
__device__ inline void pf_chain(const ComposeArgs &a, PfShared<Interp> &sh) {
#pragma clang fp contract(off)
    const int lane = int(threadIdx.x) & 63;
    const T *tab0 = static_cast<const T *>(a.tab0);
    const T *tab1 = static_cast<const T *>(a.tab1);
    const int n = a.n0;
    double lam = 0.0, unused = 0.0;
    if (!range_begin<1>(a, lane, lam, unused)) return;    // an earlier range already failed
    int oog = 0;
    int bad_slice = -1;
    double keep = 0.0;
    int jb = a.j_begin;
    int j = a.j_begin;
    // nodes the interpolant reads: i0-1 .. i0+2 (Hermite on differences) or
    // i0 .. i0+1 (linear, Hermite on stored slopes)
    constexpr int kBelow = Interp == 1 ? 1 : 0, kSpan = Interp == 1 ? 4 : 2;
    // A state that is not finite fails the slice that starts from it.  Inside
    // the loop one test of the interpolated value stands for both checks: an
    // entry that is not finite (or a slope formed from one) makes the value
    // not finite (a product with zero gives NaN), so a finite value has finite
    // entries and is itself the next slice's finite start.  The loop leaves
    // at the first value that is not finite, and the code after it tells the
    // two cases apart.
    double next = 0.0;
    bool ok = true;
    if (j < a.j_end && !finite(lam)) {
        bad_slice = j;
    } else {
        for (; j < a.j_end; ++j) {
            // the slot's tag, read while the cell is located; the window's
            // values are read after it, at addresses that depend on it
            const unsigned slot = unsigned(j) % kPfSlots;
            const long long tg = uniform_i64(__hip_atomic_load(
                &sh.tag[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            // the slot's slice and first cell (-1 and -1 for an empty slot)
            const int tag_slice = int(tg >> 32), base = int(tg & 0xffffffffLL);
            const double *win = sh.win[0][slot];
            long long i0;
            double w0;
            oog += locate(a.lo0, a.inv0, n, lam, i0, w0);
            const int i = int(i0);
            // a hit needs nodes i-kBelow .. i-kBelow+kSpan-1 inside the window
            // and, for the Hermite form on differences, a cell away from the
            // row's ends (1 <= i <= n-3), where both slopes are central; every
            // other case reads global memory
            const unsigned o = unsigned(i - kBelow - base);
            const bool hit = tag_slice == j && o <= unsigned(kPfWin - kSpan) &&
                             (Interp != 1 || i <= n - 3);
            if (hit) {
                // offsets into the slot; atomic reads keep them LDS reads (a
                // pointer chosen between LDS and global memory would make them
                // flat loads)
                if constexpr (Interp == 1) {
                    const double tm = pf_read(win, o), ta = pf_read(win, o + 1);
                    const double tb = pf_read(win, o + 2), tp = pf_read(win, o + 3);
                    // the weights do not depend on the table: formed while the
                    // reads are in flight (the empty asm keeps them there)
                    HermiteBasis hb = hermite_basis(w0);
                    asm volatile("" : "+v"(hb.h00), "+v"(hb.h10), "+v"(hb.h01), "+v"(hb.h11));
                    const double da = 0.5 * (tb - tm), db = 0.5 * (tp - ta);
                    next = ((hb.h00 * ta + hb.h10 * da) + hb.h01 * tb) + hb.h11 * db;
                    ok = all_finite(ta, tb, da, db);
                } else if constexpr (Interp == 4) {
                    const double *win1 = sh.win[Interp == 4 ? 1 : 0][slot];
                    const double ta = pf_read(win, o), tb = pf_read(win, o + 1);
                    const double ma = pf_read(win1, o), mb = pf_read(win1, o + 1);
                    HermiteBasis hb = hermite_basis(w0);
                    asm volatile("" : "+v"(hb.h00), "+v"(hb.h10), "+v"(hb.h01), "+v"(hb.h11));
                    ok = hermite_slopes_values(ta, tb, ma, mb, a.dxi0, hb, next);
                } else {
                    const double ta = pf_read(win, o), tb = pf_read(win, o + 1);
                    next = ta + w0 * (tb - ta);
                    ok = all_finite(ta, tb);
                }
            } else if constexpr (Interp == 4) {
                const T *row0 = tab0 + (long long)j * a.M, *row1 = tab1 + (long long)j * a.M;
                const double ta = double(row0[i0]), tb = double(row0[i0 + 1]);
                const double ma = double(row1[i0]), mb = double(row1[i0 + 1]);
                ok = hermite_slopes_values(ta, tb, ma, mb, a.dxi0, hermite_basis(w0), next);
            } else {
                const T *row = tab0 + (long long)j * a.M;
                ok = interp_1d<Interp>([row](long long k) { return double(row[k]); }, i0, w0,
                                       n, next);
            }
            asm volatile("" : "+v"(next));   // formed before the branch, not after it
            next = uniform_f64(next);
            if (!finite(next)) break;
            lam = next;
            // slice j is done.  Its slot is reused for slice j + kPfSlots, which
            // no helper fetches before the chain is past slice j + kPfSlots -
            // kPfAhead.
            if (lane == 0)
                __hip_atomic_store(&sh.hist[j & 1], pf_pack(j, i0), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            if (lane == j - jb) keep = lam;
            if (j - jb == 63) {
                a.boundary[jb + lane + 1] = keep;
                jb += 64;
            }
        }
        if (j < a.j_end) {               // slice j gave a value that is not finite
            if (!uniform_bool(ok)) {     // from an entry that is not finite: j fails
                bad_slice = j;
            } else {                     // a state that is not finite: j + 1 fails
                lam = next;
                if (lane == j - jb) keep = lam;
                if (j - jb == 63) {
                    a.boundary[jb + lane + 1] = keep;
                    jb += 64;
                }
                ++j;
                if (j < a.j_end) bad_slice = j;
            }
        }
    }
    if (lane < j - jb) a.boundary[jb + lane + 1] = keep;
    range_end(a, lane, lam, 0.0, oog, bad_slice);
}

// Helper wave r (1..kPfHelpers) stages slices j_begin + r, j_begin + r + kPfHelpers, ...
template <class T, int C>
__device__ inline void pf_helper(const ComposeArgs &a, PfSharedC<C> &sh, int r) {
    const int lane = int(threadIdx.x) & 63;
    const T *tab0 = static_cast<const T *>(a.tab0);
    const T *tab1 = static_cast<const T *>(a.tab1);
    const int n = a.n0;
    const long long top = n > kPfWin ? n - kPfWin : 0;
    for (int s = a.j_begin + r; s < a.j_end; s += kPfHelpers) {
        // wait until the chain is within kPfAhead slices of s
        long long h0 = 0, h1 = 0;
        int p = 0;                  // the chain has finished every slice before p
        bool go = false;
        for (int spin = 0; spin < kPfSpinMax; ++spin) {
            if (__hip_atomic_load(&sh.done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP))
                return;
            h0 = __hip_atomic_load(&sh.hist[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            h1 = __hip_atomic_load(&sh.hist[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            p = int((h0 >> 32) > (h1 >> 32) ? h0 >> 32 : h1 >> 32) + 1;
            if (p >= s - kPfAhead) {
                go = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!go) return;            // the chain does not depend on the helpers
        if (p >= s) continue;       // the chain is already at or past slice s
        // the latest cell, moved on at the latest rate per slice
        const bool newer0 = (h0 >> 32) >= (h1 >> 32);
        const long long hn = newer0 ? h0 : h1, ho = newer0 ? h1 : h0;
        const long long jn = hn >> 32, in = hn & 0xffffffffLL;
        const long long jo = ho >> 32, io = ho & 0xffffffffLL;
        const long long rate = jn - jo == 1 ? in - io : 0;
        long long base = in + rate * ((long long)s - jn) - kPfWin / 2;
        base = base < 0 ? 0 : (base > top ? top : base);
        const int slot = s % kPfSlots;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const T *row = (c == 0 ? tab0 : tab1) + (long long)s * a.M;
#pragma unroll
            for (int q = 0; q < kPfWin / 64; ++q) {
                // past the row's end (a row shorter than a window) the last
                // value is read again; the chain never uses those entries
                const long long k = base + q * 64 + lane;
                sh.win[c][slot][q * 64 + lane] = double(row[k < n ? k : n - 1]);
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0)
            __hip_atomic_store(&sh.tag[slot], pf_pack(s, base), __ATOMIC_RELEASE,
                               __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

// The whole 1-D composition of a range: wave 0 runs the chain, waves
// 1..kPfHelpers stage windows for it.
template <class T, int Interp>
__device__ inline void compose_range_staged(const ComposeArgs &a, PfShared<Interp> &sh) {
    const int wave = int(threadIdx.x) >> 6;
    if (threadIdx.x < kPfSlots) sh.tag[threadIdx.x] = -1;
    if (threadIdx.x == 0) {
        // the cell of the range's first state seeds the helpers' prediction
        const double l = a.j_begin == 0 ? a.y00 : (a.carry ? a.carry[0] : a.y00);
        long long c;
        double w;
        (void)locate(a.lo0, a.inv0, a.n0, l, c, w);
        // as if the chain had just finished slice j_begin - 1 in that cell
        sh.hist[0] = sh.hist[1] = pf_pack(a.j_begin - 1, c);
        sh.done = 0;
    }
    __syncthreads();
    if (wave == 0) {
        // the chain usually shares its CU with waves of a build still running
        __builtin_amdgcn_s_setprio(3);
        pf_chain<T, Interp>(a, sh);
        if ((threadIdx.x & 63) == 0)
            __hip_atomic_store(&sh.done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        pf_helper<T>(a, sh, wave);
    }
}

// The bilinear (2-D) chain with staged windows, as the 1-D one above: a window
// is 16 x 16 grid cells' corner values of both table components of a coming
// slice, around the chain's predicted cell on each axis, fetched kPf2Ahead
// slices ahead (the state moves farther per slice, so the prediction reaches
// less far: on the Van der Pol workload 2 slices ahead measured best, 0.45 us
// per slice against 0.47, 0.48 and 0.51 us at 3, 4 and 6).  Cells and window origins are packed 16 bits per axis, so the path
// serves grids of at most 65,536 points per axis; larger ones take the plain
// chain.
constexpr int kPf2Side = 16;                 // window cells per axis
constexpr int kPf2Win = kPf2Side * kPf2Side;
constexpr int kPf2Ahead = 2;
constexpr int kPf2Slots = 15;                // the ring within 64 KB of LDS
constexpr int kPf2MaxAxis = 65536;

struct PfShared2 {
    double win[kPf2Slots][2][kPf2Win];       // [slot][component][row * 16 + column]
    long long tag[kPf2Slots];                // (slice << 32) | (base0 << 16) | base1; -1 empty
    long long hist[2];                       // (slice << 32) | (cell0 << 16) | cell1 of the
                                             // last two slices the chain finished
    int done;
};

template <class T>
__device__ inline void pf2_chain(const ComposeArgs &a, PfShared2 &sh) {
#pragma clang fp contract(off)
    const int lane = int(threadIdx.x) & 63;
    const T *tab0 = static_cast<const T *>(a.tab0);
    const T *tab1 = static_cast<const T *>(a.tab1);
    double lam0 = 0.0, lam1 = 0.0;
    if (!range_begin<2>(a, lane, lam0, lam1)) return;     // an earlier range already failed
    int oog = 0;
    int bad_slice = -1;
    double keep0 = 0.0, keep1 = 0.0;
    int jb = a.j_begin;
    int j = a.j_begin;
    // As in the 1-D chain: inside the loop one test of the two interpolated
    // values stands for the corners' tests and the next slice's start test (a
    // corner that is not finite makes its component's value not finite), and
    // the slice at which the loop leaves is told apart after it.
    double next0 = 0.0, next1 = 0.0;
    bool bad = false;
    if (j < a.j_end && (!finite(lam0) || !finite(lam1))) {
        bad_slice = j;
    } else {
        for (; j < a.j_end; ++j) {
            const unsigned slot = unsigned(j) % kPf2Slots;
            const long long tg = uniform_i64(__hip_atomic_load(
                &sh.tag[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP));
            const int tag_slice = int(tg >> 32);
            const int b0 = int((tg >> 16) & 0xffff), b1 = int(tg & 0xffff);
            long long i0, i1;
            double w0, w1;
            oog += locate(a.lo0, a.inv0, a.n0, lam0, i0, w0);
            oog += locate(a.lo1, a.inv1, a.n1, lam1, i1, w1);
            // a hit needs cells i0, i0+1 and i1, i1+1 inside the window
            const unsigned o0 = unsigned(int(i0) - b0), o1 = unsigned(int(i1) - b1);
            const bool hit = tag_slice == j && o0 <= unsigned(kPf2Side - 2) &&
                             o1 <= unsigned(kPf2Side - 2);
            double p00, p01, p10, p11, q00, q01, q10, q11;
            if (hit) {
                const double *u = sh.win[slot][0], *v = sh.win[slot][1];
                const unsigned e = o0 * kPf2Side + o1;
                p00 = pf_read(u, e);
                p01 = pf_read(u, e + 1);
                p10 = pf_read(u, e + kPf2Side);
                p11 = pf_read(u, e + kPf2Side + 1);
                q00 = pf_read(v, e);
                q01 = pf_read(v, e + 1);
                q10 = pf_read(v, e + kPf2Side);
                q11 = pf_read(v, e + kPf2Side + 1);
            } else {
                const long long c00 = i0 * a.n1 + i1, c10 = (i0 + 1) * a.n1 + i1;
                const T *row0 = tab0 + (long long)j * a.M, *row1 = tab1 + (long long)j * a.M;
                p00 = double(row0[c00]);
                p01 = double(row0[c00 + 1]);
                p10 = double(row0[c10]);
                p11 = double(row0[c10 + 1]);
                q00 = double(row1[c00]);
                q01 = double(row1[c00 + 1]);
                q10 = double(row1[c10]);
                q11 = double(row1[c10 + 1]);
            }
            bad = bilinear_values(p00, p01, p10, p11, q00, q01, q10, q11, w0, w1, next0, next1);
            asm volatile("" : "+v"(next0), "+v"(next1));   // formed before the branch
            next0 = uniform_f64(next0);
            next1 = uniform_f64(next1);
            if (!finite(next0) || !finite(next1)) break;
            lam0 = next0;
            lam1 = next1;
            // slice j is done (its slot is reused for slice j + kPf2Slots, which
            // no helper fetches before the chain is past slice j + kPf2Slots -
            // kPf2Ahead)
            if (lane == 0)
                __hip_atomic_store(&sh.hist[j & 1], pf_pack(j, (i0 << 16) | i1),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (lane == j - jb) {
                keep0 = lam0;
                keep1 = lam1;
            }
            if (j - jb == 63) {
                a.boundary[(long long)(jb + lane + 1) * 2] = keep0;
                a.boundary[(long long)(jb + lane + 1) * 2 + 1] = keep1;
                jb += 64;
            }
        }
        if (j < a.j_end) {               // slice j gave a value that is not finite
            if (bad) {                   // from a corner that is not finite: j fails
                bad_slice = j;
            } else {                     // a state that is not finite: j + 1 fails
                lam0 = next0;
                lam1 = next1;
                if (lane == j - jb) {
                    keep0 = lam0;
                    keep1 = lam1;
                }
                if (j - jb == 63) {
                    a.boundary[(long long)(jb + lane + 1) * 2] = keep0;
                    a.boundary[(long long)(jb + lane + 1) * 2 + 1] = keep1;
                    jb += 64;
                }
                ++j;
                if (j < a.j_end) bad_slice = j;
            }
        }
    }
    if (lane < j - jb) {
        a.boundary[(long long)(jb + lane + 1) * 2] = keep0;
        a.boundary[(long long)(jb + lane + 1) * 2 + 1] = keep1;
    }
    range_end(a, lane, lam0, lam1, oog, bad_slice);
}

// Helper wave r (1..kPfHelpers) stages slices j_begin + r, j_begin + r + kPfHelpers, ...
template <class T>
__device__ inline void pf2_helper(const ComposeArgs &a, PfShared2 &sh, int r) {
    const int lane = int(threadIdx.x) & 63;
    const T *tab0 = static_cast<const T *>(a.tab0);
    const T *tab1 = static_cast<const T *>(a.tab1);
    const int n0 = a.n0, n1 = a.n1;
    const long long top0 = n0 > kPf2Side ? n0 - kPf2Side : 0;
    const long long top1 = n1 > kPf2Side ? n1 - kPf2Side : 0;
    for (int s = a.j_begin + r; s < a.j_end; s += kPfHelpers) {
        long long h0 = 0, h1 = 0;
        int p = 0;                  // the chain has finished every slice before p
        bool go = false;
        for (int spin = 0; spin < kPfSpinMax; ++spin) {
            if (__hip_atomic_load(&sh.done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP))
                return;
            h0 = __hip_atomic_load(&sh.hist[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            h1 = __hip_atomic_load(&sh.hist[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            p = int((h0 >> 32) > (h1 >> 32) ? h0 >> 32 : h1 >> 32) + 1;
            if (p >= s - kPf2Ahead) {
                go = true;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!go) return;            // the chain does not depend on the helpers
        if (p >= s) continue;       // the chain is already at or past slice s
        // each axis's latest cell, moved on at its latest rate per slice
        const bool newer0 = (h0 >> 32) >= (h1 >> 32);
        const long long hn = newer0 ? h0 : h1, ho = newer0 ? h1 : h0;
        const long long jn = hn >> 32, jo = ho >> 32;
        const long long cn0 = (hn >> 16) & 0xffff, cn1 = hn & 0xffff;
        const long long co0 = (ho >> 16) & 0xffff, co1 = ho & 0xffff;
        const bool consecutive = jn - jo == 1;
        const long long ds = (long long)s - jn;
        long long base0 = cn0 + (consecutive ? cn0 - co0 : 0) * ds - (kPf2Side / 2 - 1);
        long long base1 = cn1 + (consecutive ? cn1 - co1 : 0) * ds - (kPf2Side / 2 - 1);
        base0 = base0 < 0 ? 0 : (base0 > top0 ? top0 : base0);
        base1 = base1 < 0 ? 0 : (base1 > top1 ? top1 : base1);
        const T *row0 = tab0 + (long long)s * a.M, *row1 = tab1 + (long long)s * a.M;
        const int slot = s % kPf2Slots;
#pragma unroll
        for (int q = 0; q < kPf2Win / 64; ++q) {
            // past the grid's end (an axis shorter than a window) the last cell
            // is read again; the chain never uses those entries
            const int e = q * 64 + lane;
            const long long k0 = base0 + e / kPf2Side, k1 = base1 + e % kPf2Side;
            const long long k = (k0 < n0 ? k0 : n0 - 1) * n1 + (k1 < n1 ? k1 : n1 - 1);
            sh.win[slot][0][e] = double(row0[k]);
            sh.win[slot][1][e] = double(row1[k]);
        }
        __builtin_amdgcn_wave_barrier();
        if (lane == 0)
            __hip_atomic_store(&sh.tag[slot], pf_pack(s, (base0 << 16) | base1),
                               __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

template <class T>
__device__ inline void compose_range_staged2(const ComposeArgs &a, PfShared2 &sh) {
    const int wave = int(threadIdx.x) >> 6;
    if (threadIdx.x < kPf2Slots) sh.tag[threadIdx.x] = -1;
    if (threadIdx.x == 0) {
        // the cells of the range's first state seed the helpers' prediction
        const bool first = a.j_begin == 0 || !a.carry;
        const double l0 = first ? a.y00 : a.carry[0], l1 = first ? a.y01 : a.carry[1];
        long long c0, c1;
        double w;
        (void)locate(a.lo0, a.inv0, a.n0, l0, c0, w);
        (void)locate(a.lo1, a.inv1, a.n1, l1, c1, w);
        // as if the chain had just finished slice j_begin - 1 in that cell
        sh.hist[0] = sh.hist[1] = pf_pack(a.j_begin - 1, (c0 << 16) | c1);
        sh.done = 0;
    }
    __syncthreads();
    if (wave == 0) {
        __builtin_amdgcn_s_setprio(3);
        pf2_chain<T>(a, sh);
        if ((threadIdx.x & 63) == 0)
            __hip_atomic_store(&sh.done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        pf2_helper<T>(a, sh, wave);
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
