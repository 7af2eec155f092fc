/*
 * nv_surrogate.h — C ABI of the learned slice-map surrogate of libnv.
 *
 * The communication phase of the method (sec. 3: lambda_{j+1} = phi^j(lambda_j),
 * each phi^j evaluated by interpolating the table the computation phase wrote)
 * is the only sequential part.  This interface trains a small network on the
 * endpoints that the computation phase itself tabulates, and runs the
 * composition with the network in place of the table lookup; a built table
 * stays available as the fallback and as the check on the network's error.
 *
 * The network (one per nv_sur), for x = (y1, y2, t, mu), t the slice start
 * time T_j and mu the Van der Pol parameter:
 *     u   = (x - in_shift) * in_scale
 *     a1  = gelu(W1 u  + b1)        W1: 128 x 4      (FP32 arithmetic)
 *     a2  = gelu(W2 a1 + b2)        W2: 128 x 128    (bf16 matrix cores, FP32 sums)
 *     a3  = gelu(W3 a2 + b3)        W3: 128 x 128    (bf16 matrix cores, FP32 sums)
 *     out = W4 a3 + b4              W4: 2 x 128      (FP32 arithmetic)
 * gelu(z) = z Phi(z) with Phi the standard normal distribution function (the
 * exact GELU of Hendrycks and Gimpel).  The surrogate slice map takes one of
 * two forms (correction), every operation of the state update in FP64:
 *
 *   NV_SUR_ADDITIVE       phi(y) ~ G(y) + out_scale * out(y, T_j, mu),
 *     G a cheap coarse propagator over the slice: coarse_steps = 0 gives
 *     G(y) = y (the network learns the whole displacement), coarse_steps = k > 0
 *     gives k classical RK4 steps of length slice_length / k of the Van der Pol
 *     field with the sample's mu (the network learns the correction to it);
 *
 *   NV_SUR_STEP_DOUBLING  phi(y)_c ~ G1_c + d_c (16/15 + (out_scale_c g_c) out_c),
 *     G1 = k RK4 steps of slice_length / k, G2 = 2k RK4 steps of half that
 *     length (k = coarse_steps >= 1), d = G2 - G1, and the gate
 *     g_c = (d_c d_c) / (d_c d_c + gate_c gate_c).  With out = 0 this is the
 *     Richardson extrapolation of the coarse step (RK4 is of order 4, so the
 *     error of G1 is about 16/15 d); the network learns what remains, in units
 *     of the step-doubling difference, and the gate switches its correction
 *     off where that difference is small against gate_c (the slices on which
 *     the extrapolation is already accurate), so that the network's own error
 *     floor is added only where the coarse step is inaccurate.
 *
 * Flat parameter order (NV_SUR_PARAMS fp32 numbers): W1 (row-major, output
 * row by input column), b1, W2, b2, W3, b3, W4, b4.
 *
 * Training minimises the mean over the samples of sum_c e_c^2 with Adam (Kingma
 * and Ba, Algorithm 1), where e_c = out_c - target_c (additive form: targets
 * are 2 rows) or e_c = w_c out_c - rho_c (step-doubling form: targets are the 4
 * rows rho_0, rho_1, w_0, w_1, a least-squares fit weighted per sample).  The operands of the two 128 x 128
 * layers, of their back-propagation and of every weight-gradient sum are
 * rounded to bfloat16 (nearest, ties to even); products are summed in FP32.
 *
 * Device data layouts are feature-major: an array of n samples with d features
 * is d rows of n fp32 values (row r holds feature r of every sample).
 *
 * Conventions as in nv.h: every call returns an nv_status and sets
 * nv_last_error() on failure; an nv_sur is driven by one thread at a time;
 * its kernels run on the stream given at creation, and every call below
 * synchronizes that stream before it returns.
 */
#ifndef NV_SURROGATE_H
#define NV_SURROGATE_H

#include "nv.h"

#ifdef __cplusplus
extern "C" {
#endif

#define NV_SUR_IN 4
#define NV_SUR_WIDTH 128
#define NV_SUR_OUT 2
#define NV_SUR_PARAMS 33922

typedef enum { NV_SUR_ADDITIVE = 0, NV_SUR_STEP_DOUBLING = 1 } nv_sur_correction;

typedef struct nv_sur nv_sur;

typedef struct {
    float in_shift[NV_SUR_IN];   /* input normalisation u = (x - in_shift) * in_scale */
    float in_scale[NV_SUR_IN];
    double out_scale[NV_SUR_OUT];/* correction per unit of network output, > 0 */
    double slice_length;         /* L the network is trained for (> 0): training sets and
                                    compositions must have slices of this length */
    int coarse_steps;            /* 0: G(y) = y; 1..16: RK4 steps of the coarse propagator */
    long long max_batch;         /* largest minibatch of nv_sur_loss_grad / nv_sur_train:
                                    a multiple of 16, 16 .. 2^20 (0 = 65536); sizes the
                                    library's training workspace (about 1.6 KB per sample) */
    void *stream;                /* hipStream_t of every kernel; NULL = null stream */
    int correction;              /* nv_sur_correction (0 = additive) */
    double gate[NV_SUR_OUT];     /* step-doubling: the gate's scale per component, > 0 */
    double loss_scale[NV_SUR_OUT]; /* step-doubling: the unit q_c of the training residual
                                    (rho and w are in units of q_c), > 0 */
} nv_sur_config;

/* Create a surrogate with zero parameters on the current device.  Allocates
 * the parameters, the Adam moments and the training workspace.
 * Errors: INVALID_ARG (cfg NULL, non-finite or non-positive scales or slice
 * length, max_batch or coarse_steps out of range, an unknown correction,
 * step-doubling with coarse_steps 0 or a non-positive gate or loss scale), OOM,
 * HIP. */
NV_API nv_status nv_sur_create(const nv_sur_config *cfg, nv_sur **out);
NV_API nv_status nv_sur_destroy(nv_sur *sur);

/* Copy NV_SUR_PARAMS fp32 parameters in (host memory, flat order above) and
 * reset the Adam state (moments zero, step count zero) / copy them out.
 * Errors: INVALID_ARG (NULL pointer or non-finite parameter), HIP. */
NV_API nv_status nv_sur_set_params(nv_sur *sur, const float *host_params);
NV_API nv_status nv_sur_get_params(nv_sur *sur, float *host_params);

/* Network output for n samples: x_dev is [4][n] raw inputs (device, fp32),
 * out_dev receives [2][n] fp32 outputs (device).  n >= 1, any value.
 * Errors: INVALID_ARG, HIP. */
NV_API nv_status nv_sur_forward(nv_sur *sur, const float *x_dev, long long n, float *out_dev);

/* Loss and gradient of one minibatch, without a parameter update: x_dev is
 * [4][n] raw inputs, target_dev [2][n] (additive) or [4][n] (step-doubling:
 * rho_0, rho_1, w_0, w_1) (device, fp32); n a multiple of 16 and
 * at most max_batch.  *loss_host receives the mean loss; grad_host (may be
 * NULL) receives NV_SUR_PARAMS fp32 values in the flat order.
 * Errors: INVALID_ARG, HIP. */
NV_API nv_status nv_sur_loss_grad(nv_sur *sur, const float *x_dev, const float *target_dev,
                                  long long n, float *loss_host, float *grad_host);

typedef struct {
    long long batch;             /* samples per step: a multiple of 16, <= max_batch */
    long long steps;             /* Adam steps */
    float lr, beta1, beta2, eps; /* Adam hyper-parameters (0 = 1e-3, 0.9, 0.999, 1e-8) */
    float lr_final;              /* > 0: learning rate decays geometrically from lr to
                                    lr_final over the steps; 0 = constant lr */
} nv_sur_train_opts;

/* Adam training on a device-resident data set of n_samples samples (x_dev
 * [4][n_samples] raw inputs, target_dev [2][n_samples] or, step-doubling,
 * [4][n_samples]), n_samples a multiple
 * of batch.  Step s (counting from the first step since nv_sur_set_params)
 * uses the samples [(s * batch) mod n_samples, + batch): shuffle the data set
 * once beforehand (nv_sur_dataset_from_batch takes a permutation).  When
 * loss_dev is not NULL it receives one fp32 minibatch loss per step (device,
 * opts->steps values).  Every step is three kernels: forward and
 * back-propagation, the weight-gradient sums, and the Adam update.
 * Errors: INVALID_ARG, HIP. */
NV_API nv_status nv_sur_train(nv_sur *sur, const float *x_dev, const float *target_dev,
                              long long n_samples, const nv_sur_train_opts *opts,
                              float *loss_dev);

/* The training set from the tables of a run batch (nv_batch_run): every
 * problem must be Van der Pol (NV_RHS_VDP) with a bilinear grid.  Sample
 * (problem i, slice j, grid point k), numbered problem by problem, slice by
 * slice, point by point from 0, is written to position perm_dev[number] (or to
 * its own number when perm_dev is NULL; perm_dev, device int64, must be a
 * permutation of 0 .. total-1): x = (xi_k, T_j, mu_i) and
 *   additive:       target_c = (tab[c][j][k] - G(xi_k)[c]) / out_scale[c];
 *   step-doubling:  with G1, G2, d and g_c at xi_k as in the network's form,
 *                   r_c = (tab[c][j][k] - G1_c) - (16/15) d_c and the sample
 *                   weight v (1, or the visit weight of nv_sur_set_visits),
 *                   rho_c = sqrt(v) r_c / loss_scale_c and
 *                   w_c = sqrt(v) ((d_c out_scale_c) g_c) / loss_scale_c
 *                   (FP64, rounded to fp32 once);
 * so that e_c = w_c out_c - rho_c is sqrt(v) times the error of the surrogate
 * map in units of loss_scale_c.  Every problem's slices must have the
 * configured slice_length (relative 1e-9).  *total receives the number of
 * samples; x_dev / target_dev (device, [4][cap] and [2][cap] fp32, [4][cap]
 * step-doubling) may be NULL to query it.  Errors: INVALID_ARG (foreign problem, cap < total, perm entry
 * outside [0, cap)), NOT_BUILT (the batch has not run), NONFINITE (a table
 * entry is not finite: the data set is written but unusable), HIP. */
NV_API nv_status nv_sur_dataset_from_batch(nv_sur *sur, nv_batch *batch,
                                           const long long *perm_dev, float *x_dev,
                                           float *target_dev, long long cap,
                                           long long *total);

/* Visit weights of the step-doubling training set: the samples near the states
 * the composition visits count more.  states_dev (device, FP64, caller-owned,
 * valid until the next nv_sur_dataset_from_batch has returned) holds n_mu
 * chains of n_states states (y1, y2), [n_mu][n_states][2], chain i for
 * mu_i = mu_lo + i (mu_hi - mu_lo) / (n_mu - 1).  A sample (xi, mu) takes the
 * chain i = nearest integer to (mu - mu_lo) (n_mu - 1) / (mu_hi - mu_lo),
 * limited to [0, n_mu - 1], and
 *     v = exp(-D^2 / (2 sigma^2)) + floor,
 *     D^2 = min over the chain's states s of sum_c ((xi_c - s_c) in_scale_c)^2
 * (in fp32).  states_dev NULL switches the weights off (v = 1).  Errors:
 * INVALID_ARG (n_mu < 2, n_states outside 1..4096, mu_hi <= mu_lo, sigma <= 0, floor < 0,
 * non-finite values). */
NV_API nv_status nv_sur_set_visits(nv_sur *sur, const double *states_dev, int n_mu,
                                   int n_states, double mu_lo, double mu_hi, double sigma,
                                   double floor_weight);

/* The composition with the network in place of the lookup, for count
 * independent chains q (device arrays): lambda_0 = y0[q], and for j = 0..N-1
 *     lambda_{j+1} = the surrogate map at (lambda_j, T_j, mu[q]) (the form the
 *                    configured correction gives; additive:
 *                    G(lambda_j) + out_scale * out(lambda_j, T_j, mu[q])),
 * T_j = t0 + j (T - t0) / N, the state kept in FP64; (T - t0) / N must equal
 * the configured slice_length (relative 1e-9).
 *
 * Fallback and check: when fb_tab0 is not NULL, (fb_tab0, fb_tab1) are the
 * two component tables of a built Van der Pol context for the same mu, t0, T
 * and N (nv_table_device_ptr; layout tab[j][k], fb_precision NV_FP32 or
 * NV_FP64, bilinear grid fb_grid).  Each step then also evaluates the table's
 * bilinear map; when the two differ by more than guard (max over components)
 * or lambda_j leaves the box [box_lo, box_hi], the table's value is taken
 * instead and counted in n_fallback.  Without a table, lambda_j outside the
 * box is counted in n_outside and the network extrapolates.
 *
 *   y0        device [count][2] FP64       mu        device [count] FP64
 *   final     device [count][2] FP64       boundary  device [count][N+1][2] FP64 or NULL
 * Errors: INVALID_ARG (count < 1, N < 1, bad grid or pointers), NONFINITE
 * (a state became non-finite; info->bad_chain names one), HIP. */
typedef struct {
    long long count;
    const double *y0;
    const double *mu;
    double t0, T;
    int n_slices;
    double *final_state;
    double *boundary;
    const void *fb_tab0, *fb_tab1;
    int fb_precision;
    nv_ic_grid fb_grid;
    double guard;
    double box_lo[2], box_hi[2];
} nv_sur_chains;

typedef struct {
    long long n_fallback;        /* steps that took the table's value */
    long long n_outside;         /* steps that started outside the box */
    double max_deviation;        /* max over steps of |network - table| (table given) */
    long long bad_chain;         /* -1, or a chain whose state became non-finite */
    float ms;                    /* kernel time (HIP events) */
} nv_sur_compose_info;

NV_API nv_status nv_sur_compose(nv_sur *sur, const nv_sur_chains *chains,
                                nv_sur_compose_info *info);

/* Milliseconds (HIP events on the surrogate's stream) of the kernels of the
 * last nv_sur_forward, nv_sur_train or nv_sur_compose call. */
NV_API nv_status nv_sur_last_ms(nv_sur *sur, float *ms);

#ifdef __cplusplus
}
#endif
#endif
