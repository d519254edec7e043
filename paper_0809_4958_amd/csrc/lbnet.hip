// lbnet.hip -- host side of the learned boundary upsampler (include/lbnet.h).
//
// The context owns the FP32 master parameters (device layout [tap][co][ci],
// channel counts padded to the MFMA tiles with zero weights), the Adam
// moments, the bfloat16 forward and backward-data weight copies, and the
// activation and gradient buffers for max_batch samples.  A training step is
// lift + layer 1 (k_head) -> layers 2 + 3 with the loss and dy (k_conv23)
// -> weight gradients of the three layers (k_wgrad) around the data
// gradients of layers 3 and 2 through their ReLUs (k_back32) -> the first
// stage of one fixed-order reduction of the weight-gradient partials -> Adam,
// which sums the stage's range sums; every step is a kernel of
// lbnet_kernels.hpp on the context stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lbnet.h"
#include "lbnet_kernels.hpp"

using namespace lbnet;

namespace {

// device parameter layout (floats)
constexpr size_t W1N = (size_t)NTAP * CH * CIN, W2N = (size_t)NTAP * CH * CH, W3N = (size_t)NTAP * COUT * CH;
constexpr size_t OFF_W1 = 0, OFF_B1 = OFF_W1 + W1N, OFF_W2 = OFF_B1 + CH, OFF_B2 = OFF_W2 + W2N,
                 OFF_W3 = OFF_B2 + CH, OFF_B3 = OFF_W3 + W3N, NDEV = OFF_B3 + COUT;
constexpr int IN_USED = 15, OUT_USED = 3;
constexpr int MAX_PART = 256;  // weight-gradient partials (workgroups)
constexpr int RSEG = ADAM_RANGES;  // first-stage ranges of the partial reduction

static_assert((size_t)CH * IN_USED * 9 + CH + (size_t)CH * CH * 9 + CH + (size_t)OUT_USED * CH * 9 +
                      OUT_USED ==
                  LBN_PARAM_COUNT,
              "parameter count");

}  // namespace

struct lbn_ctx {
  lbn_config cfg{};
  hipStream_t stream = nullptr;
  std::string err;
  // parameters
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  __bf16 *w1f = nullptr, *w1t = nullptr, *w2f = nullptr, *w2t = nullptr, *w3f = nullptr, *w3t = nullptr;
  bool weights_dirty = true, has_grad = false;
  int adam_t = 0;
  // activations for max_batch samples
  __bf16 *x0 = nullptr, *a1 = nullptr, *a2 = nullptr, *dy = nullptr, *dz1 = nullptr, *dz2 = nullptr;
  float *r = nullptr, *base = nullptr, *scale = nullptr, *part = nullptr;
  float* part_seg = nullptr;
  double* loss_part = nullptr;
  int last_batch = 0;
  int grad_parts = 0;  // weight-gradient partials of the last lbn_loss_grad
  std::vector<void*> owned;
};

namespace {

lb_status fail(lbn_ctx* c, lb_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIPCHK(call)                                                              \
  do {                                                                            \
    hipError_t e_ = (call);                                                       \
    if (e_ != hipSuccess) return fail(ctx, LB_ERR_HIP, std::string(#call) + ": " + \
                                                       hipGetErrorString(e_));    \
  } while (0)

void* dalloc(lbn_ctx* ctx, size_t bytes, bool* ok) {
  if (!*ok) return nullptr;
  bytes = std::max<size_t>(bytes, 256);
  void* ptr = nullptr;
  if (ctx->cfg.dev_alloc) {
    ptr = ctx->cfg.dev_alloc(bytes, ctx->cfg.alloc_user);
  } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
    ptr = nullptr;
  }
  if (!ptr) {
    *ok = false;
    return nullptr;
  }
  ctx->owned.push_back(ptr);
  return ptr;
}

template <typename T>
T* dalloc_t(lbn_ctx* ctx, size_t n, bool* ok) {
  return (T*)dalloc(ctx, n * sizeof(T), ok);
}

// canonical W[co][ci][ky][kx] of a layer <-> device [tap][co_pad][ci_pad]
void canon_to_dev(const float* src, int co_n, int ci_n, int co_pad, int ci_pad, float* dst) {
  for (int co = 0; co < co_n; co++)
    for (int ci = 0; ci < ci_n; ci++)
      for (int tap = 0; tap < 9; tap++)
        dst[((size_t)tap * co_pad + co) * ci_pad + ci] = src[((size_t)co * ci_n + ci) * 9 + tap];
}

void dev_to_canon(const float* src, int co_n, int ci_n, int co_pad, int ci_pad, float* dst) {
  for (int co = 0; co < co_n; co++)
    for (int ci = 0; ci < ci_n; ci++)
      for (int tap = 0; tap < 9; tap++)
        dst[((size_t)co * ci_n + ci) * 9 + tap] = src[((size_t)tap * co_pad + co) * ci_pad + ci];
}

void params_to_dev(const float* in, std::vector<float>& dev) {
  dev.assign(NDEV, 0.0f);
  const float* q = in;
  canon_to_dev(q, CH, IN_USED, CH, CIN, dev.data() + OFF_W1);
  q += (size_t)CH * IN_USED * 9;
  std::memcpy(dev.data() + OFF_B1, q, CH * sizeof(float));
  q += CH;
  canon_to_dev(q, CH, CH, CH, CH, dev.data() + OFF_W2);
  q += (size_t)CH * CH * 9;
  std::memcpy(dev.data() + OFF_B2, q, CH * sizeof(float));
  q += CH;
  canon_to_dev(q, OUT_USED, CH, COUT, CH, dev.data() + OFF_W3);
  q += (size_t)OUT_USED * CH * 9;
  std::memcpy(dev.data() + OFF_B3, q, OUT_USED * sizeof(float));
}

void dev_to_params(const std::vector<float>& dev, float* out) {
  float* q = out;
  dev_to_canon(dev.data() + OFF_W1, CH, IN_USED, CH, CIN, q);
  q += (size_t)CH * IN_USED * 9;
  std::memcpy(q, dev.data() + OFF_B1, CH * sizeof(float));
  q += CH;
  dev_to_canon(dev.data() + OFF_W2, CH, CH, CH, CH, q);
  q += (size_t)CH * CH * 9;
  std::memcpy(q, dev.data() + OFF_B2, CH * sizeof(float));
  q += CH;
  dev_to_canon(dev.data() + OFF_W3, OUT_USED, CH, COUT, CH, q);
  q += (size_t)OUT_USED * CH * 9;
  std::memcpy(q, dev.data() + OFF_B3, OUT_USED * sizeof(float));
}

// the three layers' weights and their bf16 copies
PrepLayers prep_layers(lbn_ctx* ctx) {
  return PrepLayers{{ctx->p + OFF_W1, ctx->p + OFF_W2, ctx->p + OFF_W3},
                    {ctx->w1f, ctx->w2f, ctx->w3f},
                    {ctx->w1t, ctx->w2t, ctx->w3t},
                    {CH, CH, COUT},
                    {CIN, CH, CH},
                    {(int)OFF_W1, (int)OFF_W2, (int)OFF_W3}};
}

lb_status prep_weights(lbn_ctx* ctx) {
  if (!ctx->weights_dirty) return LB_OK;
  const int n = (int)(W1N + W2N + W3N);
  hipLaunchKernelGGL(k_prep_weights, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, prep_layers(ctx));
  HIPCHK(hipGetLastError());
  ctx->weights_dirty = false;
  return LB_OK;
}

// workgroups (and partials) of a weight-gradient launch
int wgrad_grid(int batch) { return std::min(batch * IMG, MAX_PART); }

// bands per image of a convolution launch (one workgroup per band): the
// fewest (a power of two, at most 64 / TR) for which the grid reaches about
// per_cu workgroups per compute unit (per_cu by LDS and register use)
int conv_bands(int batch, int per_cu) {
  int bands = 1;
  while (bands < IMG / TR && batch * bands < 240 * per_cu) bands *= 2;
  return bands;
}

// win.samples != NULL: the window path (inputs gathered by the lift, the
// face field written by the last layer into u_out; r is not kept)
// loss.truth != NULL: the training forward, whose last layer also writes dy
// and the loss partials
lb_status forward(lbn_ctx* ctx, const float* coarse, const float* theta, int batch,
                  LiftWindow win = LiftWindow{nullptr, 0, 0, 1}, float* u_out = nullptr,
                  LossOut loss = LossOut{nullptr, 0.0f, nullptr, nullptr}) {
  lb_status s = prep_weights(ctx);
  if (s) return s;
  hipStream_t st = ctx->stream;
  const int R = ctx->cfg.coarse;
  // lift + layer 1 per (sample, band): bands so that the grid covers most of
  // the 256 compute units (each band repeats the sample's preparation, so a
  // grid of 240 for the 120-image window beats 480); x0 kept only outside
  // the window path (training and lbn_read_buffer read it)
  int bands = 1;
  while (bands < IMG / TR && batch * bands < 240) bands *= 2;
  hipLaunchKernelGGL(k_head, dim3(batch * bands), dim3(NBC), 24 * R * R * sizeof(float), st, coarse, theta, win,
                     R, ctx->w1f, ctx->p + OFF_B1, ctx->a1, u_out ? nullptr : ctx->x0, ctx->base, ctx->scale,
                     bands);
  // layers 2 and 3 in one pass; the layer-2 output is stored only outside
  // the window path (the backward pass and lbn_read_buffer read it)
  const int b1 = conv_bands(batch, 1);
  if (u_out)
    hipLaunchKernelGGL((k_conv23<3>), dim3(batch * b1), dim3(NBC), 0, st, ctx->a1, ctx->w2f, ctx->p + OFF_B2,
                       ctx->w3f, ctx->p + OFF_B3, nullptr, (void*)u_out, b1, ctx->base, ctx->scale, loss);
  else if (loss.truth)
    hipLaunchKernelGGL((k_conv23<2>), dim3(batch * b1), dim3(NBC), 0, st, ctx->a1, ctx->w2f, ctx->p + OFF_B2,
                       ctx->w3f, ctx->p + OFF_B3, ctx->a2, (void*)ctx->r, b1, ctx->base, ctx->scale, loss);
  else
    hipLaunchKernelGGL((k_conv23<1>), dim3(batch * b1), dim3(NBC), 0, st, ctx->a1, ctx->w2f, ctx->p + OFF_B2,
                       ctx->w3f, ctx->p + OFF_B3, ctx->a2, (void*)ctx->r, b1, ctx->base, ctx->scale, loss);
  HIPCHK(hipGetLastError());
  ctx->last_batch = batch;
  return LB_OK;
}

// partial weight and bias gradients of one layer: workgroup g writes its
// partial into row g of ctx->part (NDEV values per row, each layer at its
// parameter offset, the biases after the weights as in the parameters)
template <int CI, int CO>
lb_status wgrad(lbn_ctx* ctx, const __bf16* x, const __bf16* dz, int batch, size_t off_w, size_t off_b) {
  const int rows = batch * IMG;
  (void)off_b;  // == off_w + 9 CO CI
  // the last layer's padded output channels have zero gradients: not stored
  hipLaunchKernelGGL((k_wgrad<CI, CO>), dim3(wgrad_grid(batch)), dim3(NBW), 0, ctx->stream, x, dz,
                     ctx->part + off_w, (int)NDEV, rows, CO == COUT ? OUT_USED : CO);
  HIPCHK(hipGetLastError());
  return LB_OK;
}

// The partials of the last layer's padded output channels are neither
// stored nor read (zero gradients).
PadRows last_layer_pad() { return PadRows{(int)OFF_W3, (int)OFF_B3, COUT, CH, OUT_USED}; }

// The gradient into ctx->g, when it is read: every layer's partials summed in
// two fixed-order stages, RSEG ranges of partials in parallel into
// ctx->part_seg, then their sum in increasing range order (each parameter's
// sum the same sequence as a reduction of its layer alone; the Adam step
// forms the same sums itself, k_adam_parts).  The padded entries' range sums
// stay at the zero they start with.
lb_status finish_grads(lbn_ctx* ctx) {
  const int n = (int)NDEV;
  hipStream_t st = ctx->stream;
  hipLaunchKernelGGL(k_reduce_parts, dim3((n + 255) / 256, RSEG), dim3(256), 0, st, ctx->part, ctx->grad_parts,
                     n, ctx->part_seg, last_layer_pad());
  const PadRows none{n, n, 1, 1, 1};
  hipLaunchKernelGGL(k_reduce_parts, dim3((n + 255) / 256), dim3(256), 0, st, ctx->part_seg, RSEG, n, ctx->g,
                     none);
  HIPCHK(hipGetLastError());
  return LB_OK;
}

lb_status check_batch(lbn_ctx* ctx, int batch) {
  if (!ctx) return LB_ERR_ARG;
  if (batch < 1 || batch > ctx->cfg.max_batch) return fail(ctx, LB_ERR_ARG, "batch outside 1..max_batch");
  return LB_OK;
}

}  // namespace

extern "C" {

lb_status lbn_init(const lbn_config* cfg, lbn_ctx** out) {
  if (!cfg || !out) return LB_ERR_ARG;
  *out = nullptr;
  if (cfg->coarse < 2 || cfg->coarse > 32 || cfg->max_batch < 1 || cfg->max_batch > (1 << 16))
    return LB_ERR_ARG;
  lbn_ctx* ctx = new lbn_ctx();
  ctx->cfg = *cfg;
  // NULL is HIP's null stream (ordered with PyTorch's default stream)
  ctx->stream = (hipStream_t)cfg->stream;
  const size_t B = (size_t)cfg->max_batch, px = B * IMG * IMG;
  bool ok = true;
  ctx->p = dalloc_t<float>(ctx, NDEV, &ok);
  ctx->m = dalloc_t<float>(ctx, NDEV, &ok);
  ctx->v = dalloc_t<float>(ctx, NDEV, &ok);
  ctx->g = dalloc_t<float>(ctx, NDEV, &ok);
  ctx->w1f = dalloc_t<__bf16>(ctx, W1N, &ok);
  ctx->w1t = dalloc_t<__bf16>(ctx, W1N, &ok);
  ctx->w2f = dalloc_t<__bf16>(ctx, W2N, &ok);
  ctx->w2t = dalloc_t<__bf16>(ctx, W2N, &ok);
  ctx->w3f = dalloc_t<__bf16>(ctx, W3N, &ok);
  ctx->w3t = dalloc_t<__bf16>(ctx, W3N, &ok);
  ctx->x0 = dalloc_t<__bf16>(ctx, px * CIN, &ok);
  ctx->a1 = dalloc_t<__bf16>(ctx, px * CH, &ok);
  ctx->a2 = dalloc_t<__bf16>(ctx, px * CH, &ok);
  ctx->dy = dalloc_t<__bf16>(ctx, px * COUT, &ok);
  ctx->dz1 = dalloc_t<__bf16>(ctx, px * CH, &ok);
  ctx->dz2 = dalloc_t<__bf16>(ctx, px * CH, &ok);
  ctx->r = dalloc_t<float>(ctx, px * COUT, &ok);
  ctx->base = dalloc_t<float>(ctx, px * 3, &ok);
  ctx->scale = dalloc_t<float>(ctx, B, &ok);
  ctx->part = dalloc_t<float>(ctx, (size_t)MAX_PART * NDEV, &ok);
  ctx->part_seg = dalloc_t<float>(ctx, (size_t)RSEG * NDEV, &ok);
  // one loss partial per workgroup of the last layer: batch x bands <= max(480, batch)
  ctx->loss_part = dalloc_t<double>(ctx, std::max(1024, ctx->cfg.max_batch), &ok);
  if (!ok) {
    lbn_free(ctx);
    return LB_ERR_OOM;
  }
  std::vector<float> zero(NDEV, 0.0f);
  for (float* d : {ctx->p, ctx->m, ctx->v, ctx->g})
    if (hipMemcpyAsync(d, zero.data(), NDEV * sizeof(float), hipMemcpyHostToDevice, ctx->stream) != hipSuccess) {
      lbn_free(ctx);
      return LB_ERR_HIP;
    }
  // the range sums of the partial reduction: zero where it never writes
  if (hipMemsetAsync(ctx->part_seg, 0, (size_t)RSEG * NDEV * sizeof(float), ctx->stream) != hipSuccess ||
      hipStreamSynchronize(ctx->stream) != hipSuccess) {
    lbn_free(ctx);
    return LB_ERR_HIP;
  }
  *out = ctx;
  return LB_OK;
}

lb_status lbn_set_params(lbn_ctx* ctx, const float* params, size_t n) {
  if (!ctx || !params) return LB_ERR_ARG;
  if (n != LBN_PARAM_COUNT) return fail(ctx, LB_ERR_BUFSIZE, "parameter vector length");
  std::vector<float> dev;
  params_to_dev(params, dev);
  std::vector<float> zero(NDEV, 0.0f);
  HIPCHK(hipMemcpyAsync(ctx->p, dev.data(), NDEV * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->m, zero.data(), NDEV * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->v, zero.data(), NDEV * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->weights_dirty = true;
  ctx->has_grad = false;
  ctx->adam_t = 0;
  return LB_OK;
}

lb_status lbn_get_params(lbn_ctx* ctx, float* params, size_t n) {
  if (!ctx || !params) return LB_ERR_ARG;
  if (n != LBN_PARAM_COUNT) return fail(ctx, LB_ERR_BUFSIZE, "parameter vector length");
  std::vector<float> dev(NDEV);
  HIPCHK(hipMemcpyAsync(dev.data(), ctx->p, NDEV * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  dev_to_params(dev, params);
  return LB_OK;
}

lb_status lbn_forward(lbn_ctx* ctx, const float* coarse_dev, const float* theta_dev, int32_t batch,
                      float* out_dev) {
  lb_status s = check_batch(ctx, batch);
  if (s) return s;
  if (!coarse_dev || !theta_dev || !out_dev) return fail(ctx, LB_ERR_ARG, "null pointer");
  s = forward(ctx, coarse_dev, theta_dev, batch);
  if (s) return s;
  const int n_px = batch * IMG * IMG;
  hipLaunchKernelGGL(k_combine, dim3((n_px + 255) / 256), dim3(256), 0, ctx->stream, ctx->r, ctx->base,
                     ctx->scale, n_px, out_dev);
  HIPCHK(hipGetLastError());
  return LB_OK;
}

lb_status lbn_window_forward(lbn_ctx* ctx, const float* samples_dev, int32_t n_samples, int32_t k,
                             int32_t dt, float* ring_dev) {
  if (!ctx) return LB_ERR_ARG;
  if (!samples_dev || !ring_dev) return fail(ctx, LB_ERR_ARG, "null pointer");
  if (dt < 1 || 6 * dt > ctx->cfg.max_batch) return fail(ctx, LB_ERR_ARG, "6 dt must not exceed max_batch");
  if (n_samples < 2 || k < 0 || k >= n_samples - 1) return fail(ctx, LB_ERR_ARG, "window outside the history");
  return forward(ctx, nullptr, nullptr, 6 * dt, LiftWindow{samples_dev, n_samples, k, dt}, ring_dev);
}

lb_status lbn_loss_grad(lbn_ctx* ctx, const float* coarse_dev, const float* theta_dev,
                        const float* truth_dev, int32_t batch, double* loss, float* grad) {
  lb_status s = check_batch(ctx, batch);
  if (s) return s;
  if (!coarse_dev || !theta_dev || !truth_dev) return fail(ctx, LB_ERR_ARG, "null pointer");
  const int n_px = batch * IMG * IMG;
  const double inv_count = 1.0 / (3.0 * n_px);
  // the loss and dy = dL/dr come out of the forward's last layer
  s = forward(ctx, coarse_dev, theta_dev, batch, LiftWindow{nullptr, 0, 0, 1}, nullptr,
              LossOut{truth_dev, (float)(2.0 * inv_count), ctx->dy, ctx->loss_part});
  if (s) return s;
  hipStream_t st = ctx->stream;
  const int b1 = conv_bands(batch, 1);
  const int lgrid = batch * b1;  // loss partials: one per workgroup of the last layer
  // layer 3: weights from (a2, dy)
  if ((s = wgrad<CH, COUT>(ctx, ctx->a2, ctx->dy, batch, OFF_W3, OFF_B3))) return s;
  // data gradients through ReLU(a2) and ReLU(a1) in one pass
  hipLaunchKernelGGL(k_back32, dim3(batch * b1), dim3(NBC), 0, st, ctx->dy, ctx->w3t, ctx->w2t, ctx->a2, ctx->a1,
                     ctx->dz2, ctx->dz1, b1);
  // layer 2
  if ((s = wgrad<CH, CH>(ctx, ctx->a1, ctx->dz2, batch, OFF_W2, OFF_B2))) return s;
  // layer 1
  if ((s = wgrad<CIN, CH>(ctx, ctx->x0, ctx->dz1, batch, OFF_W1, OFF_B1))) return s;
  ctx->grad_parts = wgrad_grid(batch);  // summed by the Adam step or finish_grads
  ctx->has_grad = true;
  if (loss) {
    std::vector<double> part(lgrid);
    HIPCHK(hipMemcpyAsync(part.data(), ctx->loss_part, lgrid * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double sum = 0.0;
    for (double v : part) sum += v;
    *loss = sum * inv_count;
  }
  if (grad) {
    if ((s = finish_grads(ctx))) return s;
    std::vector<float> dev(NDEV);
    HIPCHK(hipMemcpyAsync(dev.data(), ctx->g, NDEV * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    dev_to_params(dev, grad);
  }
  return LB_OK;
}

lb_status lbn_adam_step(lbn_ctx* ctx, float lr, float beta1, float beta2, float eps) {
  if (!ctx) return LB_ERR_ARG;
  if (!ctx->has_grad) return fail(ctx, LB_ERR_STATE, "no gradient since the parameters were set");
  if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return fail(ctx, LB_ERR_ARG, "Adam hyper-parameters");
  ctx->adam_t++;
  const float c1 = 1.0f - (float)std::pow((double)beta1, ctx->adam_t);
  const float c2 = 1.0f - (float)std::pow((double)beta2, ctx->adam_t);
  // the gradient summed from the partials in the same pass; the step also
  // writes the bf16 copies of the updated weights
  hipLaunchKernelGGL(k_adam_parts, dim3((NDEV + ADAM_PARAMS - 1) / ADAM_PARAMS), dim3(ADAM_RANGES * ADAM_PARAMS), 0,
                     ctx->stream, ctx->part, ctx->grad_parts,
                     (int)NDEV, last_layer_pad(), ctx->p, ctx->m, ctx->v, lr, beta1, beta2, eps, c1, c2,
                     prep_layers(ctx));
  HIPCHK(hipGetLastError());
  ctx->weights_dirty = false;
  return LB_OK;
}

lb_status lbn_read_buffer(lbn_ctx* ctx, int32_t which, int32_t batch, float* out, size_t n) {
  lb_status s = check_batch(ctx, batch);
  if (s) return s;
  if (!out) return fail(ctx, LB_ERR_ARG, "null pointer");
  const size_t px = (size_t)batch * IMG * IMG;
  const void* src = nullptr;
  size_t count = 0;
  bool bf = false;
  switch (which) {
    case 0: src = ctx->x0; count = px * CIN; bf = true; break;
    case 1: src = ctx->a1; count = px * CH; bf = true; break;
    case 2: src = ctx->a2; count = px * CH; bf = true; break;
    case 3: src = ctx->r; count = px * COUT; break;
    case 4: src = ctx->base; count = px * 3; break;
    case 5: src = ctx->scale; count = (size_t)batch; break;
    default: return fail(ctx, LB_ERR_ARG, "unknown buffer");
  }
  if (n != count) return fail(ctx, LB_ERR_BUFSIZE, "buffer length");
  if (bf) {
    std::vector<uint16_t> raw(count);
    HIPCHK(hipMemcpyAsync(raw.data(), src, count * 2, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    for (size_t i = 0; i < count; i++) {
      const uint32_t u = (uint32_t)raw[i] << 16;
      std::memcpy(&out[i], &u, 4);
    }
  } else {
    HIPCHK(hipMemcpyAsync(out, src, count * 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  return LB_OK;
}

lb_status lbn_sync(lbn_ctx* ctx) {
  if (!ctx) return LB_ERR_ARG;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return LB_OK;
}

const char* lbn_last_error(const lbn_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void lbn_free(lbn_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (void* ptr : ctx->owned) {
    if (ctx->cfg.dev_free) ctx->cfg.dev_free(ptr, ctx->cfg.alloc_user);
    else (void)hipFree(ptr);
  }
  delete ctx;
}

}  // extern "C"
