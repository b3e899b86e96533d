/* libashrt: learned warm start for the robust inversion.
 *
 * A 2-D U-Net with four 2x down-samplings maps a blended receiver gather to
 * an initial Radon model m0 (one channel per velocity panel) and initial
 * residual weights w0, which robust_invert (ashrt.h) takes as its warm start
 * (thesis Chapter 4: the IRLS outer loop starts from a model and a residual
 * weighting; a good start shortens it).  The network is not in the thesis.
 *
 * Architecture (c = base * (1, 2, 4, 8, 8); every 3x3 convolution has zero
 * padding, a bias and a ReLU):
 *   enc1a Cin->c1, enc1b c1->c1 | 2x2 mean pool | enc2a c1->c2, enc2b |
 *   pool | enc3a c2->c3, enc3b | pool | enc4a c3->c4, enc4b |
 *   pool | bota c4->c5, botb |
 *   dec4a [nearest 2x upsample(botb), enc4b] -> c4, dec4b |
 *   dec3a [up(dec4b), enc3b] -> c3, dec3b |
 *   dec2a [up(dec3b), enc2b] -> c2, dec2b | dec1a [up(dec2b), enc1b] -> c1,
 *   dec1b | head_m 1x1 c1 -> P (linear) | head_w 1x1 c1 -> 1, sigmoid.
 * With base 16 and P = 32 that is 1,225,345 parameters.
 * Parameters: one flat FP32 vector, conv by conv in that order, weight
 * [co][ci][kh][kw] then bias [co].
 *
 * Numerics: 3x3 convolutions run on BF16 matrix cores (v_mfma bf16) with
 * BF16 weights and activations and FP32 accumulation; the 1x1 heads, the
 * loss, gradients and the optimiser are FP32 (loss sums FP64).  Master
 * weights are FP32; their BF16 copies are refreshed after every update.
 *
 * Layouts (device memory, caller-owned, contiguous):
 *   x        [B][H][W]     FP32  network input (the caller scales the gather)
 *   y_model  [B][P][H][W]  FP32  predicted model / scale
 *   y_w      [B][H][W]     FP32  predicted weights in (0, 1)
 * H and W must be multiples of 16.  Every call is stream-ordered on `stream`;
 * none allocates device memory after unet_create (the caller passes a
 * workspace of unet_workspace_bytes).  Return codes are the ASHRT_* status
 * codes of ashrt.h; ashrt_last_error() describes the last failure.
 */
#ifndef UNET_H
#define UNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct unet_desc {
  int32_t cin;    /* input channels: 1                                         */
  int32_t pout;   /* model channels P (velocity panels), 1..128                */
  int32_t base;   /* channels of the first level c1: 16 (c1..c4 = 16..128)     */
} unet_desc;

typedef struct unet_train_params {
  double lr;            /* AdamW step size                                     */
  double beta1, beta2;  /* moment decay rates (0.9, 0.999)                     */
  double eps;           /* 1e-8                                                */
  double weight_decay;  /* decoupled decay (0 = Adam)                          */
  double lam_w;         /* weight of the w0 term in the loss (1)               */
} unet_train_params;

typedef struct unet_net unet_net;

/* Create a network on `device` with zero parameters (set them with
 * unet_set_params).  Allocates the FP32 parameters, gradients, AdamW moments
 * and BF16 copies once. */
int unet_create(const unet_desc *desc, int device, unet_net **out);
void unet_destroy(unet_net *net);
int64_t unet_param_count(const unet_net *net);

/* Copy FP32 parameters in the flat layout above from / to host memory.
 * unet_set_params also resets the AdamW moments and step count. */
int unet_set_params(unet_net *net, const float *host, int64_t n);
int unet_get_params(const unet_net *net, float *host, int64_t n);

/* Workspace for a batch of B inputs of H x W; train != 0 adds what the
 * backward pass needs. */
int unet_workspace_bytes(const unet_net *net, int32_t B, int32_t H, int32_t W, int32_t train,
                         size_t *bytes);

/* Inference: y_model and y_w from x. */
int unet_forward(const unet_net *net, const float *x, int32_t B, int32_t H, int32_t W, float *y_model,
                 float *y_w, void *ws, size_t ws_bytes, void *stream);

/* Loss mean(y_m - t_m)^2 + lam_w mean(y_w - t_w)^2 (FP64, written to the
 * device double *loss) and its gradient w.r.t. the flat parameters (FP32,
 * device [n], overwritten).  Parameters are not changed. */
int unet_loss_grad(unet_net *net, const float *x, const float *t_model, const float *t_w, int32_t B,
                   int32_t H, int32_t W, double lam_w, double *loss, float *grad, void *ws,
                   size_t ws_bytes, void *stream);

/* One training step: loss and gradient as above, then one AdamW update of
 * the parameters and a refresh of their BF16 copies. */
int unet_train_step(unet_net *net, const unet_train_params *tp, const float *x, const float *t_model,
                    const float *t_w, int32_t B, int32_t H, int32_t W, double *loss, void *ws,
                    size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif
