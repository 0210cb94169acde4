/*
 * libdqo, learned initialization of per-pixel Gaussians (gfx950).
 *
 * Gaussians are spawned from RGB-D observations, one per valid pixel of an
 * object crop (Sec. III-C, Eq. (7)-(8): new geometry is added where the
 * rendered masks say the object is incomplete; opaque Gaussians start at
 * opacity 0.9, Sec. IV).  The plain initialization back-projects each pixel;
 * the learned one adds a small convolutional network's per-pixel prediction
 * of the log-scale offset, opacity logit and colour offset that the plain
 * optimizer would converge to.  The network is this library's extension, not
 * part of the paper.
 *
 * Conventions are those of dqo.h: device pointers are caller-owned, every
 * compute call only enqueues work on `stream`, returns DQO_OK or a negative
 * DQO_E* code after host-side validation (message in dqo_last_error()).
 *
 * Crops: rgbdm[B][5][H][W] float32 (device), channels r, g, b, depth (camera
 * z, metres), mask.  A pixel is VALID when mask > 0.5 and depth > 0.  H and W
 * must be multiples of 16 (at most 4096), 1 <= B.
 *
 * Network: four 3x3 zero-padded convolutions 5 -> 32 -> 64 -> 64 -> 6 with
 * ReLU after the first three.  Weights and activations are BF16, products
 * are accumulated in FP32 on the matrix cores (MFMA), biases are FP32.
 * Input channels: r, g, b, 4 (d - d_min) / d_min at valid pixels (0
 * elsewhere; d_min = the crop's smallest valid depth; FP32 arithmetic),
 * valid mask.  Output channels: log-scale offset, opacity logit, colour
 * offset (3), predicted log-error.
 */
#ifndef DQO_LEARNED_H
#define DQO_LEARNED_H

#include "dqo.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DQO_NET_LAYERS 4
#define DQO_NET_IN 5
#define DQO_NET_OUT 6

/* Parameter layout (host query).  All parameters live in one flat FP32
 * vector theta[n_params]: for layer l, weights at w_offset[l] in the order
 * [cout_pad][9][cin_pad] (tap = 3 * dy + dx of the 3x3 window, entry
 * w[co][ci][dy][dx] of the usual [cout][cin][3][3] form), then the bias at
 * b_offset[l] [cout_pad].  Entries of padded channels must be zero (they
 * receive zero gradient and stay zero under Adam).  Two BF16 copies are
 * derived from theta by dqo_net_pack: the forward copy (w_elems values, same
 * order, layer l at wk_offset[l]) and the transposed copy used for input
 * gradients ([cin_pad][9][cout_pad] with the taps mirrored). */
typedef struct dqo_net_layout {
    int32_t cin[DQO_NET_LAYERS], cout[DQO_NET_LAYERS];         /* 5,32,64,64 -> 32,64,64,6 */
    int32_t cin_pad[DQO_NET_LAYERS], cout_pad[DQO_NET_LAYERS]; /* 16,32,64,64 -> 32,64,64,16 */
    int64_t w_offset[DQO_NET_LAYERS], b_offset[DQO_NET_LAYERS];
    int64_t wk_offset[DQO_NET_LAYERS];
    int64_t n_params; /* FP32 entries of theta (and of its gradient) */
    int64_t w_elems;  /* BF16 entries of each packed weight copy */
} dqo_net_layout;

int dqo_net_layout_get(dqo_net_layout* out /* host */);

/* Bytes of the caller-allocated workspace of a batch of B crops of H x W:
 * input and hidden activations, activation gradients, per-split partial
 * weight gradients.  The forward leaves the activations there for the loss
 * and the backward of the same batch. */
int dqo_net_workspace_size(int32_t B, int32_t H, int32_t W, int64_t* bytes /* host, out */);

/* theta -> BF16 forward copy wf[w_elems] and transposed copy wt[w_elems]
 * (uint16 storage).  Round to nearest even. */
int dqo_net_pack(const dqo_ctx* ctx, const float* theta, uint16_t* wf, uint16_t* wt, void* stream);

/* Network forward of B crops: out[B][6][H][W] float32.  workspace as sized
 * by dqo_net_workspace_size(B, H, W). */
int dqo_net_forward(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm, const uint16_t* wf,
                    const float* theta, void* workspace, float* out, void* stream);

/* Training loss of the last forward (same B, H, W, workspace):
 *   e_c = out_c - label_c (c < 5), s = sum_c chan_w[c] e_c^2,
 *   r = log(s + 1e-4) (the realised log-error, held constant),
 *   L = (1/M) sum over the M valid pixels of [ s + (out_5 - r)^2 ].
 * labels[B][5][H][W] float32.  loss (device, double[2]) receives L and the
 * fit part (1/M) sum s.  The gradient dL/dout, rounded to BF16, is left in
 * the workspace for dqo_net_backward.  chan_w: host double[5]. */
int dqo_net_loss(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm, const float* out,
                 const float* labels, const double* chan_w, double* loss, void* workspace, void* stream);

/* Backward of the last forward + loss: grad[n_params] float32 (overwritten)
 * = dL/dtheta.  Activation gradients are rounded to BF16 between layers;
 * weight gradients are summed in FP32 over fixed pixel splits and then over
 * the splits in a fixed order (deterministic). */
int dqo_net_backward(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const uint16_t* wt, void* workspace,
                     float* grad, void* stream);

/* Adam over a flat FP32 vector (PyTorch's update, one learning rate), with
 * the step count in device memory as in dqo_adam_step_counted (graph-
 * capturable): uses step = *d_step + 1 and stores it back. */
int dqo_adam_flat(const dqo_ctx* ctx, float* params, const float* grads, float* m, float* v, int64_t n, double lr,
                  double beta1, double beta2, double eps, int64_t* d_step, void* stream);

/* Gaussians of B crops (B <= DQO_MAX_VIEWS), one per valid pixel, crop by
 * crop in raster order: crop b fills params columns [offsets[b],
 * offsets[b+1]) of params[14][n] (float32), where offsets (device, int64,
 * B + 1 entries, offsets[0] = 0, offsets[B] <= n) is the exclusive prefix sum
 * of the crops' valid-pixel counts, which the caller counts with the same
 * rule.  Mean = back-projection of the pixel centre at its depth through
 * cams[b] (host), log-scales log(d / fx), identity quaternion, opacity logit
 * log 9, the pixel's colour; ids[n] = obj_id.  When pred (device
 * [B][6][H][W] float32) is given and use_pred (device int32[B]) is NULL or
 * nonzero for the crop: log-scales += pred_0, opacity logit = pred_1, colour
 * += pred_2..4.  Columns beyond a crop's valid pixels are not written. */
int dqo_init_gaussians(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm,
                       const dqo_camera* cams, const int64_t* offsets, const float* pred, const int32_t* use_pred,
                       int64_t n, float* params, int32_t* ids, int32_t obj_id, void* stream);

/* Training labels labels[B][5][H][W] float32 from converged Gaussians laid out
 * as by dqo_init_gaussians: at valid pixels, mean log-scale - log(d / fx),
 * opacity logit, colour - pixel colour; zero elsewhere. */
int dqo_init_labels(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm,
                    const dqo_camera* cams, const int64_t* offsets, const float* params, int64_t n, float* labels,
                    void* stream);

/* Per-crop fallback decision: use_pred[b] = 1 when the mean of the predicted
 * log-error (out channel 5) over the crop's valid pixels is <= threshold,
 * else 0 (plain initialization).  mean_logerr (device, float[B], may be NULL)
 * receives the means. */
int dqo_net_fallback(const dqo_ctx* ctx, int32_t B, int32_t H, int32_t W, const float* rgbdm, const float* out,
                     double threshold, int32_t* use_pred, float* mean_logerr, void* stream);

/* Masked PSNR (peak 1) of rendered colour color[V][3][H][W] against the
 * crops' colour over their valid pixels: psnr[V] (device, double). */
int dqo_masked_psnr(const dqo_ctx* ctx, int32_t V, int32_t H, int32_t W, const float* color, const float* rgbdm,
                    double* psnr, void* stream);

#ifdef __cplusplus
}
#endif

#endif
