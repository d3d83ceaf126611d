/*
 * rsv_mlp.h -- C ABI of the learned diagonal-mass network (gfx950, BF16 MFMA).
 *
 * The HMC of Sec. 3 (arXiv:1603.08114) uses the kinetic energy 1/2 sum p_i^2.
 * The sampler here also accepts a diagonal mass, H = sum p_t^2/(2 m_t) - ln f,
 * which leaves the target f(h | theta) unchanged (the Metropolis test of
 * Sec. 3 is exact for any fixed positive m that does not depend on h).  This
 * network predicts log m_t per series-site from the data around t and theta:
 *
 *   inputs (27, padded to 32): ln(y_s^2 + 1e-8) and ln RV_s for
 *     s = t-5..t+5 (indices clamped to the series), then theta
 *     (phi, mu, xi, sigma_eta^2, sigma_u^2); each standardised as
 *     (raw - mean[i]) / std[i] with training-set statistics;
 *   layers: 32 -> 64 (GELU) -> 64 (GELU) -> 1, GELU(x) = x Phi(x);
 *   arithmetic: inputs, weights and hidden activations in bfloat16 (round to
 *     nearest even), products on the matrix cores with FP32 accumulation,
 *     biases and GELU in FP32.
 *
 * Parameters are one FP32 array of RSV_MLP_PARAMS values, in this order:
 *   W1[32][64] (row = input, rows 27..31 zero), b1[64], W2[64][64]
 *   (row = first hidden unit), b2[64], w3[64], b3[1].
 * Training minimises the mean squared error against a target (the log
 * posterior precision -ln Var(h_t) estimated from identity-mass chains).
 *
 * Conventions are those of rsv_hmc.h: device pointers are caller-owned HIP
 * memory, work is enqueued on `hip_stream`, nothing is allocated.
 */
#ifndef RSV_MLP_H
#define RSV_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "rsv_hmc.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { RSV_MLP_INPUTS = 27, RSV_MLP_INPUTS_PAD = 32, RSV_MLP_HIDDEN = 64, RSV_MLP_PARAMS = 6337 };

/* Standardised inputs of every site of S series, as bfloat16 bit patterns
 * (each FP64 value (raw - mean) / std rounded to FP32, then to bfloat16).
 *   offsets  device int64, S+1 (the layout of rsv_problem); max_T (host) is
 *            the longest series; y, log_rv device FP64 per site.
 *   theta    device, one rsv_theta per series.
 *   mean, std  device FP64, 27 each.
 *   x        device uint16 [offsets[S]][32], 16-byte aligned (columns 27..31
 *            written as 0). */
rsv_status rsv_mlp_features(int32_t n_series, const int64_t *offsets, const double *y,
                            const double *log_rv, const rsv_theta *theta, const double *mean,
                            const double *std, int64_t max_T, uint16_t *x, void *hip_stream);

/* Forward pass for n rows of x: out[i] = network output (FP32).  If clip is
 * non-zero a finite output is clipped to [-5, 5] (the log mass used by the
 * sampler); a non-finite one is written as it is, so that the caller's
 * identity fallback sees it (rsv_hmc_init also takes m_t = 1 at such a site). */
rsv_status rsv_mlp_forward(int64_t n, const uint16_t *x, const float *params, float *out,
                           int32_t clip, void *hip_stream);

/* Bytes of workspace rsv_mlp_grad needs for n rows. */
size_t rsv_mlp_grad_workspace_bytes(int64_t n);

/* Gradient of L = (1/n) sum_i (out(x_{r_i}) - target[r_i])^2 over the rows
 * r_i = rows[i] (rows may be NULL: r_i = i), written to grad (device FP32,
 * RSV_MLP_PARAMS); *loss (device FP64, may be NULL) receives L.  Reduction
 * order is fixed: the result does not depend on scheduling. */
rsv_status rsv_mlp_grad(int64_t n, const uint16_t *x, const float *target, const int32_t *rows,
                        const float *params, float *grad, double *loss, void *workspace,
                        size_t ws_bytes, void *hip_stream);

/* One Adam step (Kingma & Ba) on params with moments m, v (device FP32,
 * RSV_MLP_PARAMS each); step counts from 1. */
rsv_status rsv_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t step,
                        float lr, float beta1, float beta2, float eps, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
