/* lbnet.h -- C ABI of the learned boundary upsampler (gfx950, BF16 MFMA).
 *
 * The boundary of a fine box is driven by the velocity of the flow around a
 * tracer, known only at coarse points and times (Sec. 2-3: sampled on a grid
 * of the coarse simulation every few steps and interpolated linearly in space
 * and time).  This library learns the correction to that interpolation: a
 * small convolutional network maps the coarse samples of one face (an R x R
 * corner-aligned grid at four sample times k-1 .. k+2) and the phase
 * theta = (n - t_k) / dt of step n inside the window [t_k, t_k+1) to the
 * 64 x 64 per-step face field
 *
 *   u = base + s r,   base = L(Sb),   Sb = (1 - theta) S_k + theta S_k+1,
 *
 * where L is the corner-aligned bilinear lift to 64 x 64 (base is the
 * interpolation the plain method uses), s the RMS of the sample's coarse
 * values and r the network output: 3 x 3 convolutions 15 -> 64 -> 64 -> 3,
 * ReLU between them, zero padding.  Its 15 input channels are L(Sb) / s,
 * L(Duu Sb) / s, L(Dvv Sb) / s (coarse second differences along the face's
 * u and v axes; edge nodes take the next node's), the temporal second
 * difference L(S_k+2 - S_k+1 - S_k + S_k-1) / s (three components each),
 * theta, and the position of the node inside its coarse cell, 4 a (1 - a)
 * and 4 b (1 - b).
 *
 * Precision: activations and weights bfloat16, FP32 accumulation, FP32 master
 * weights, Adam optimiser.  All pointers named *_dev are device pointers the
 * caller owns; host pointers are read before the call returns.  Every call
 * returns an lb_status of lbm.h (0 = LB_OK, negative = error, message in
 * lbn_last_error).  Calls are asynchronous on the configured stream except
 * those that return host results (loss, gradients, parameters).
 *
 * Parameter vector (host, FP32, LBN_PARAM_COUNT values, this order):
 *   W1[64][15][3][3], b1[64], W2[64][64][3][3], b2[64], W3[3][64][3][3], b3[3]
 * with out[co][y][x] = b[co] + sum_{ci,ky,kx} W[co][ci][ky][kx] in[ci][y+ky-1][x+kx-1].
 */
#ifndef LBNET_H
#define LBNET_H

#include <stddef.h>
#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

#define LBN_IMG 64          /* face field edge (nodes) */
#define LBN_PARAM_COUNT 47363

typedef struct lbn_ctx lbn_ctx;

typedef struct {
  int32_t coarse;      /* R, coarse samples per face edge, 2..32 */
  int32_t max_batch;   /* largest number of samples per call, >= 1 */
  void* stream;        /* hipStream_t; NULL = the null stream */
  void* (*dev_alloc)(size_t bytes, void* user);  /* NULL = hipMalloc */
  void (*dev_free)(void* ptr, void* user);
  void* alloc_user;
} lbn_config;

/* Creates a context with all parameters zero.  LB_ERR_ARG on a bad config. */
lb_status lbn_init(const lbn_config* cfg, lbn_ctx** out);

/* Host parameter vector in, or out (n must be LBN_PARAM_COUNT, else
 * LB_ERR_BUFSIZE).  Setting parameters resets the Adam moments and step. */
lb_status lbn_set_params(lbn_ctx* ctx, const float* params, size_t n);
lb_status lbn_get_params(lbn_ctx* ctx, float* params, size_t n);

/* Face fields of `batch` samples: coarse_dev [batch][4][3][R][R] (sample
 * time, component, row v, column u), theta_dev [batch]; out_dev
 * [batch][64][64][3].  1 <= batch <= max_batch. */
lb_status lbn_forward(lbn_ctx* ctx, const float* coarse_dev, const float* theta_dev, int32_t batch,
                      float* out_dev);

/* Face fields of one window for the LEARNED boundary of lbm.h.  samples_dev
 * holds a box's sampled face history [n_samples][6][R][R][3] (the SAMPLED
 * layout of lb_boundary); window k covers steps t_k .. t_k + dt - 1.  Writes
 * ring_dev [dt][6][64][64][3]: slot j = step t_k + j, faces in the order
 * -x, +x, -y, +y, -z, +z.  Sample times k-1 and k+2 are clamped to the
 * history; needs 0 <= k < n_samples - 1 and 6 dt <= max_batch. */
lb_status lbn_window_forward(lbn_ctx* ctx, const float* samples_dev, int32_t n_samples, int32_t k,
                             int32_t dt, float* ring_dev);

/* Loss L = mean over batch x 64 x 64 x 3 values of ((u - truth) / s)^2, the
 * squared error in units of each sample's coarse RMS s, against truth_dev
 * [batch][64][64][3], and its gradient with respect to the parameters (kept
 * for lbn_adam_step).  loss (host, may be NULL) receives L; grad (host, may
 * be NULL) the gradient in the parameter-vector order.  Either output makes
 * the call wait for the stream. */
lb_status lbn_loss_grad(lbn_ctx* ctx, const float* coarse_dev, const float* theta_dev,
                        const float* truth_dev, int32_t batch, double* loss, float* grad);

/* One Adam step (Kingma and Ba, bias-corrected) with the last gradient.
 * LB_ERR_STATE if no gradient was computed since the parameters were set. */
lb_status lbn_adam_step(lbn_ctx* ctx, float lr, float beta1, float beta2, float eps);

/* Intermediate buffers of the last forward pass, converted to FP32 on the host
 * (n values, LB_ERR_BUFSIZE if it does not match): 0 = lifted input
 * [batch][64][64][16], 1 = layer-1 output [batch][64][64][64], 2 = layer-2
 * output, 3 = network output r [batch][64][64][16], 4 = base [batch][64][64][3],
 * 5 = scale s [batch].  lbn_window_forward keeps 1, 4 and 5 only: it lifts
 * straight into layer 1, keeps the layer-2 output on chip and writes the
 * face field from the last layer, so 0, 2 and 3 still hold the last
 * lbn_forward or lbn_loss_grad. */
lb_status lbn_read_buffer(lbn_ctx* ctx, int32_t which, int32_t batch, float* out, size_t n);

lb_status lbn_sync(lbn_ctx* ctx);
const char* lbn_last_error(const lbn_ctx* ctx);
void lbn_free(lbn_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBNET_H */
