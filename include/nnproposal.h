/*
 * nnproposal: a learned Gaussian proposal over the planner's controller parameters, with BF16
 * matrix-core (MFMA) training and inference kernels for MI355X (gfx950).
 *
 * The paper samples the controller parameters theta without a learned prior and names better-
 * guided sampling and warm starts from offline encodings as future work (Sect. V). This library
 * implements that extension: a network maps an encoding of one planning problem to a diagonal
 * Gaussian N(mu, diag(exp(2 s))) over theta and is trained on the plain planner's best samples
 * theta* (Gaussian negative log-likelihood, Adam). nnp_plan draws from it through the n_prop /
 * prop_mu / prop_log_sigma fields of nnp_problem (include/nnplan.h); uniform draws stay in the
 * same plan as the fallback.
 *
 * Definitions
 *  Encoding e[72] of a problem, in the vehicle frame at z0 (c = cos phi0, s = sin phi0;
 *  xi = c dx + s dy, eta = c dy - s dx for a world offset (dx, dy) from (x0, y0)):
 *    e[0:4]  = [v0 / norm_v, a_prev[0], a_prev[1], T / 100]
 *    e[4:8]  = [xi_goal / norm_xi, eta_goal / norm_eta, wrap(phi_goal - phi0) / norm_phi,
 *               v_goal / norm_v]
 *    e[8:72] = 16 blocks [xi_j / d_cap, eta_j / d_cap, vxi_j / norm_v, veta_j / norm_v] of the
 *              16 obstacle points nearest to (x0, y0), ascending squared distance (binary32
 *              fmaf(dx, dx, dy * dy)), lower index first on ties; missing points (P < 16) give the block
 *              [100 / d_cap, 0, 0, 0]. a_prev NULL means [0, a_idle] as in nnp_plan.
 *  Network: h1 = relu(W1 q(e) + b1), h2 = relu(W2 q(h1) + b2), y = W3 q(h2) + b3, widths
 *    72 -> 256 -> 256 -> 2 n_theta; mu = y[0:n_theta], log_sigma = y[n_theta:2 n_theta].
 *    q() rounds to bfloat16 (nearest, ties to even); products run on BF16 MFMA with binary32
 *    accumulation; biases, activations before rounding, the loss and all updates are binary32.
 *  Loss of a batch of B pairs (e_b, theta*_b): L = (1/B) sum_b sum_k [ (theta*_bk - mu_bk)^2
 *    exp(-2 s_bk) / 2 + s_bk ]. Back-propagated gradients are rounded to bfloat16 before each
 *    product, like the forward operands.
 *  Adam (Kingma and Ba, 2015): beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected.
 *  Parameter vector (n_params floats, the layout of get/set_params and of gradients):
 *    W1 [256][72], b1 [256], W2 [256][256], b2 [256], W3 [2 n_theta][256], b3 [2 n_theta],
 *    every matrix row-major [out][in].
 *
 * Conventions are those of include/nnplan.h: device pointers on the handle's device, host
 * pointers read before the call returns, asynchronous on the given hip_stream, negative NNP_E*
 * codes on failure with nothing enqueued, one handle per host thread.
 */
#ifndef NNPROPOSAL_H
#define NNPROPOSAL_H

#include <stdint.h>

#include "nnplan.h"

#ifdef __cplusplus
extern "C" {
#endif

#define NNP_PROP_ENC 72      /* encoding width                                               */
#define NNP_PROP_HIDDEN 256  /* hidden width                                                 */
#define NNP_PROP_NEAR 16     /* obstacle points in the encoding                              */

typedef struct nnp_proposal_config {
    int32_t n_theta;         /* controller parameters (the output has 2 n_theta values)      */
    int32_t max_batch;       /* largest batch B of forward / gradient / train calls, >= 1    */
    float norm_xi, norm_eta, norm_phi, norm_v; /* encoding normalisers (the planner's eq. (3) */
    float d_cap;             /* Delta values of Table II and its distance cap)                */
    float u_min, u_max;      /* acceleration range, for a_idle when a_prev is NULL            */
} nnp_proposal_config;

typedef struct nnp_proposal nnp_proposal;

/* Create a proposal network (parameters zero; set them with nnp_proposal_set_params) and its
 * workspace for batches up to max_batch. NNP_EINVAL / NNP_ENOMEM / NNP_EDEVICE on failure, with
 * *q set to NULL. */
int nnp_proposal_create(nnp_proposal **q, const nnp_proposal_config *c, int device);

/* Release the handle and its workspace (waits for its device work). NULL is accepted. */
void nnp_proposal_destroy(nnp_proposal *q);

/* Length of the parameter vector. */
int nnp_proposal_n_params(const nnp_proposal *q);

/* Load parameters from device params[n_params] (layout above); resets the Adam moments and the
 * step count. */
int nnp_proposal_set_params(nnp_proposal *q, const float *params, void *hip_stream);

/* Copy the current parameters to device params[n_params]. */
int nnp_proposal_get_params(nnp_proposal *q, float *params, void *hip_stream);

/* Training state, for checkpoint and resume: the parameters and both Adam moments (each device
 * [n_params] in the parameter layout) and the Adam step count t. get_state copies them out (m or v
 * may be NULL to skip them; params and step may not). set_state loads all of them, so that the
 * training steps after it continue bit for bit as they would have without the round trip.
 * NNP_EINVAL for NULL arguments or a step outside [0, 2^31). */
int nnp_proposal_get_state(nnp_proposal *q, float *params, float *m, float *v, int64_t *step,
                           void *hip_stream);
int nnp_proposal_set_state(nnp_proposal *q, const float *params, const float *m, const float *v,
                           int64_t step, void *hip_stream);

/* Encodings of `count` problems into device enc[count][72]. Reads z0, goal, a_prev, T, P and obst
 * of each problem (other fields are ignored). count in 1..65535. */
int nnp_proposal_encode(nnp_proposal *q, const nnp_problem *probs, int count, float *enc,
                        void *hip_stream);

/* Forward pass for B encodings (device enc[B][72]) into device mu[B][n_theta] and
 * log_sigma[B][n_theta] (either may be NULL). B in 1..max_batch. */
int nnp_proposal_forward(nnp_proposal *q, const float *enc, int B, float *mu, float *log_sigma,
                         void *hip_stream);

/* Loss and gradients for B pairs (enc[B][72], theta_star[B][n_theta], device) without updating
 * the parameters: grads (device [n_params], layout above) and loss (device [1]); either may be
 * NULL. */
int nnp_proposal_gradients(nnp_proposal *q, const float *enc, const float *theta_star, int B,
                           float *grads, float *loss, void *hip_stream);

/* One training step: forward, loss, backward and an Adam update with learning rate lr. loss
 * (device [1], may be NULL) receives the batch loss before the update. */
int nnp_proposal_train_step(nnp_proposal *q, const float *enc, const float *theta_star, int B,
                            float lr, float *loss, void *hip_stream);

/* The BF16 MFMA matrix product the network runs on, exported for direct use and testing:
 * C[m][n] = sum_k A(m, k) B(k, n) over bfloat16 operands (stored as uint16 bit patterns) with
 * binary32 accumulation, then the epilogue.
 *   a_layout 0: A(m, k) = A[m * lda + k];  1: A(m, k) = A[k * lda + m]
 *   b_layout 0: B(k, n) = B[n * ldb + k];  1: B(k, n) = B[k * ldb + n]
 *   epilogue 0: v = acc + bias[n] (bias may be NULL); C = v; Cq = bf16(v)
 *            1: v = acc + bias[n]; C = v; Cq = bf16(max(v, 0))
 *            2: v = mask[m * ldm + n] > 0 ? acc : 0; C = v; Cq = bf16(v)
 *   C (binary32, ldc) and Cq (bfloat16 bits, ldcq) may each be NULL.
 * M and N must be multiples of 128 and K a multiple of 32; leading dimensions multiples of 8
 * and operand pointers 16-byte aligned. */
int nnp_gemm_bf16(int a_layout, int b_layout, int M, int N, int K, const uint16_t *A, int lda,
                  const uint16_t *B, int ldb, int epilogue, const float *bias, const float *mask,
                  int ldm, float *C, int ldc, uint16_t *Cq, int ldcq, void *hip_stream);

/* Text of the handle's last error ("" if none); NULL: the last create failure. */
const char *nnp_proposal_last_error(const nnp_proposal *q);

#ifdef __cplusplus
}
#endif

#endif
