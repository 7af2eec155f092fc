/*
 * CPU throughput baseline of the propagator build: the computation phase of
 * Nievergelt's method (sec. 3, pseudocode figure: every slice solves the
 * initial value problem from every grid point) over all host cores with
 * OpenMP, in FP64 or FP32, classical RK4.
 *
 * TEST AND MEASUREMENT INFRASTRUCTURE, NOT THE ORACLE: only tests/ and the
 * CPU baseline of bench.py use it.  It shares no code with the GPU library.
 * What differs from the oracle's plain table build is scheduling only:
 *   - the forcing of the non-autonomous problem (sin 3t at the step's start,
 *     midpoint and end times) is evaluated once per slice and stage time
 *     instead of once per trajectory;
 *   - trajectories are integrated 64 at a time, the step loop outside
 *     and the trajectory loop inside, one function per right-hand side, so
 *     that the compiler vectorises across trajectories (the block worker is
 *     built for AVX-512, AVX2 and baseline x86-64 and picked at load time);
 *   - slices and blocks of trajectories are spread over OpenMP threads.
 * Compiled without contraction: the FP64 variant keeps every operation of
 * the oracle in the oracle's order, so its entries equal the oracle's bit for
 * bit.  The FP32 variant evaluates in single precision and accumulates the
 * state by blocked summation: the increments of 64 steps are summed apart
 * from the state, which the stages see as state + partial sum, and added to
 * it once per block.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>

enum { CB_LOGISTIC = 1, CB_FORCED_CUBIC = 2, CB_VDP = 3 };
#define CB_BLOCK 64
#define CB_SUM_BLOCK 64

int cb_max_threads(void) { return omp_get_max_threads(); }

typedef struct {
    long long M;
    int n1, steps;
    double lo0, dxi0, lo1, dxi1, h, mu;
} cb_shape;

/* Stages of one RK4 step at state (x0, x1) (k_i[1] = 0 for 1-D problems):
 * the oracle's expressions, operation for operation. */
#define STAGES_LOGISTIC(R)                                                                \
    k1a = x0 * (1 - x0);                                                                  \
    u0 = x0 + h2 * k1a;                                                                   \
    k2a = u0 * (1 - u0);                                                                  \
    u0 = x0 + h2 * k2a;                                                                   \
    k3a = u0 * (1 - u0);                                                                  \
    u0 = x0 + hr * k3a;                                                                   \
    k4a = u0 * (1 - u0);

#define STAGES_FORCED_CUBIC(R)                                                            \
    k1a = Fa - x0 * x0 * x0;                                                              \
    u0 = x0 + h2 * k1a;                                                                   \
    k2a = Fb - u0 * u0 * u0;                                                              \
    u0 = x0 + h2 * k2a;                                                                   \
    k3a = Fb - u0 * u0 * u0;                                                              \
    u0 = x0 + hr * k3a;                                                                   \
    k4a = Fc - u0 * u0 * u0;

#define STAGES_VDP(R)                                                                     \
    k1a = x1;                                                                             \
    k1b = m * (1 - x0 * x0) * x1 - x0;                                                    \
    u0 = x0 + h2 * k1a;                                                                   \
    u1 = x1 + h2 * k1b;                                                                   \
    k2a = u1;                                                                             \
    k2b = m * (1 - u0 * u0) * u1 - u0;                                                    \
    u0 = x0 + h2 * k2a;                                                                   \
    u1 = x1 + h2 * k2b;                                                                   \
    k3a = u1;                                                                             \
    k3b = m * (1 - u0 * u0) * u1 - u0;                                                    \
    u0 = x0 + hr * k3a;                                                                   \
    u1 = x1 + hr * k3b;                                                                   \
    k4a = u1;                                                                             \
    k4b = m * (1 - u0 * u0) * u1 - u0;

/* Integrate the block of trajectories k0 .. k0+cnt-1 of one slice (F its
 * forcing row; FORCED = 0: none) and store their end states at out (component stride
 * cstride).  BLOCKED: 0 plain update y <- y + (h/6)(((k1 + 2k2) + 2k3) + k4),
 * 1 blocked summation. */
#define DEFINE_BLOCK(NAME, R, STAGES, DIM, BLOCKED, FORCED)                               \
__attribute__((target_clones("avx512f", "avx2", "default")))                              \
static void NAME(const cb_shape *sh, long long k0, int cnt, const R *F, R *out,           \
                 size_t cstride) {                                                        \
    R y0[CB_BLOCK], y1[CB_BLOCK], c0[CB_BLOCK], c1[CB_BLOCK], z0[CB_BLOCK],               \
        z1[CB_BLOCK];                                                                     \
    const R hr = (R)sh->h, h2 = (R)(sh->h / 2.0), h6 = (R)(sh->h / 6.0), m = (R)sh->mu;   \
    int q, s;                                                                             \
    (void)m;                                                                              \
    for (q = 0; q < CB_BLOCK; ++q) {                                                      \
        const long long k = k0 + (q < cnt ? q : cnt - 1);                                 \
        if (DIM == 1) {                                                                   \
            y0[q] = (R)(sh->lo0 + (double)k * sh->dxi0);                                  \
            y1[q] = 0;                                                                    \
        } else {                                                                          \
            y0[q] = (R)(sh->lo0 + (double)(k / sh->n1) * sh->dxi0);                       \
            y1[q] = (R)(sh->lo1 + (double)(k % sh->n1) * sh->dxi1);                       \
        }                                                                                 \
        c0[q] = c1[q] = 0;                                                                \
        z0[q] = y0[q];                                                                    \
        z1[q] = y1[q];                                                                    \
    }                                                                                     \
    for (s = 0; s < sh->steps; ++s) {                                                     \
        R Fa = 0, Fb = 0, Fc = 0;                                                         \
        if (FORCED) {                                                                     \
            Fa = F[2 * s];                                                                \
            Fb = F[2 * s + 1];                                                            \
            Fc = F[2 * s + 2];                                                            \
        }                                                                                 \
        (void)Fa; (void)Fb; (void)Fc;                                                     \
        for (q = 0; q < CB_BLOCK; ++q) {                                                  \
            const R x0 = z0[q], x1 = z1[q];                                               \
            R k1a, k2a, k3a, k4a, k1b = 0, k2b = 0, k3b = 0, k4b = 0, u0, u1;             \
            (void)x1; (void)u1;                                                           \
            STAGES(R)                                                                     \
            {                                                                             \
                const R da = h6 * (k1a + 2 * k2a + 2 * k3a + k4a);                        \
                const R db = h6 * (k1b + 2 * k2b + 2 * k3b + k4b);                        \
                if (BLOCKED) {                                                            \
                    c0[q] = c0[q] + da;                                                   \
                    z0[q] = y0[q] + c0[q];                                                \
                    if (DIM == 2) {                                                       \
                        c1[q] = c1[q] + db;                                               \
                        z1[q] = y1[q] + c1[q];                                            \
                    }                                                                     \
                } else {                                                                  \
                    y0[q] = y0[q] + da;                                                   \
                    z0[q] = y0[q];                                                        \
                    if (DIM == 2) {                                                       \
                        y1[q] = y1[q] + db;                                               \
                        z1[q] = y1[q];                                                    \
                    }                                                                     \
                }                                                                         \
            }                                                                             \
        }                                                                                 \
        if (BLOCKED && ((s + 1) % CB_SUM_BLOCK == 0 || s + 1 == sh->steps)) {             \
            for (q = 0; q < CB_BLOCK; ++q) {                                              \
                y0[q] = y0[q] + c0[q];                                                    \
                y1[q] = y1[q] + c1[q];                                                    \
                c0[q] = c1[q] = 0;                                                        \
                z0[q] = y0[q];                                                            \
                z1[q] = y1[q];                                                            \
            }                                                                             \
        }                                                                                 \
    }                                                                                     \
    for (q = 0; q < cnt; ++q) {                                                           \
        out[q] = y0[q];                                                                   \
        if (DIM == 2) out[cstride + q] = y1[q];                                           \
    }                                                                                     \
}

DEFINE_BLOCK(block_logistic_f64, double, STAGES_LOGISTIC, 1, 0, 0)
DEFINE_BLOCK(block_fcub_f64, double, STAGES_FORCED_CUBIC, 1, 0, 1)
DEFINE_BLOCK(block_vdp_f64, double, STAGES_VDP, 2, 0, 0)
DEFINE_BLOCK(block_logistic_f32, float, STAGES_LOGISTIC, 1, 1, 0)
DEFINE_BLOCK(block_fcub_f32, float, STAGES_FORCED_CUBIC, 1, 1, 1)
DEFINE_BLOCK(block_vdp_f32, float, STAGES_VDP, 2, 1, 0)

/* Tables of slices [slice_begin, slice_end) of the build (rhs, mu, [t0, T],
 * n_slices, grid, steps): tab[c][j - slice_begin][k].  Returns 0, 1 for a bad
 * argument, 2 when out of memory. */
#define DEFINE_BUILD(NAME, R, SUFFIX)                                                     \
int NAME(int rhs, double mu, double t0, double T, int n_slices, int slice_begin,         \
         int slice_end, int dim, const int *n, const double *lo, const double *hi,        \
         int steps, int threads, R *tab) {                                                \
    cb_shape sh;                                                                          \
    const int ns = slice_end - slice_begin;                                               \
    const double L = (T - t0) / (double)n_slices;                                         \
    long long blocks, item;                                                               \
    R *rows = NULL;                                                                       \
    int j;                                                                                \
    if (rhs != CB_LOGISTIC && rhs != CB_FORCED_CUBIC && rhs != CB_VDP) return 1;          \
    if ((rhs == CB_VDP) != (dim == 2) || ns < 1 || steps < 1 || threads < 1) return 1;    \
    sh.M = dim == 1 ? (long long)n[0] : (long long)n[0] * n[1];                           \
    sh.n1 = dim == 2 ? n[1] : 1;                                                          \
    sh.steps = steps;                                                                     \
    sh.h = L / (double)steps;                                                             \
    sh.lo0 = lo[0];                                                                       \
    sh.dxi0 = (hi[0] - lo[0]) / (double)(n[0] - 1);                                       \
    sh.lo1 = dim == 2 ? lo[1] : 0.0;                                                      \
    sh.dxi1 = dim == 2 ? (hi[1] - lo[1]) / (double)(n[1] - 1) : 0.0;                      \
    sh.mu = mu;                                                                           \
    blocks = (sh.M + CB_BLOCK - 1) / CB_BLOCK;                                            \
    if (rhs == CB_FORCED_CUBIC) {                                                         \
        /* forcing at T_j + s h (s = 0..S) and at the midpoints, per slice */             \
        rows = (R *)malloc(sizeof(R) * (size_t)ns * (size_t)(2 * steps + 1));             \
        if (!rows) return 2;                                                              \
        _Pragma("omp parallel for num_threads(threads) schedule(static)")                 \
        for (j = 0; j < ns; ++j) {                                                        \
            const double tj = t0 + (double)(slice_begin + j) * L;                         \
            R *F = rows + (size_t)j * (size_t)(2 * steps + 1);                            \
            int s;                                                                        \
            for (s = 0; s < steps; ++s) {                                                 \
                const double ta = tj + (double)s * sh.h;                                  \
                F[2 * s] = (R)sin(3.0 * ta);                                              \
                F[2 * s + 1] = (R)sin(3.0 * (ta + sh.h / 2.0));                           \
            }                                                                             \
            F[2 * steps] = (R)sin(3.0 * (tj + (double)steps * sh.h));                     \
        }                                                                                 \
    }                                                                                     \
    _Pragma("omp parallel for num_threads(threads) schedule(dynamic, 4)")                 \
    for (item = 0; item < (long long)ns * blocks; ++item) {                               \
        const int jj = (int)(item / blocks);                                              \
        const long long k0 = (item % blocks) * CB_BLOCK;                                  \
        const int cnt = (int)(sh.M - k0 < CB_BLOCK ? sh.M - k0 : CB_BLOCK);               \
        R *out = tab + (size_t)jj * (size_t)sh.M + (size_t)k0;                            \
        const size_t cstride = (size_t)ns * (size_t)sh.M;                                 \
        if (rhs == CB_LOGISTIC)                                                           \
            block_logistic_##SUFFIX(&sh, k0, cnt, NULL, out, cstride);                    \
        else if (rhs == CB_FORCED_CUBIC)                                                  \
            block_fcub_##SUFFIX(&sh, k0, cnt, rows + (size_t)jj * (size_t)(2 * steps + 1), \
                                out, cstride);                                            \
        else                                                                              \
            block_vdp_##SUFFIX(&sh, k0, cnt, NULL, out, cstride);                         \
    }                                                                                     \
    free(rows);                                                                           \
    return 0;                                                                             \
}

DEFINE_BUILD(cb_build_f64, double, f64)
DEFINE_BUILD(cb_build_f32, float, f32)
