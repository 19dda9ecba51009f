/*
 * dfb_denoise.h -- learned denoiser for low-sample accumulation tiles, an
 * addition to the compositor of dfb.h (the paper has no denoiser; it keeps
 * progressive refinement, Listing 1 accumulationID, as the way to converge).
 *
 * The network is a 3-level U-Net with 32 base channels (conv3x3 + ReLU
 * pairs at 32/64/128 channels, 2x2 average pooling, nearest upsampling,
 * skip concatenation, a 1x1 output conv whose RGB is added to the mean).
 * Input, per pixel: [mean R, G, B, A, log(tile variance), 1/n] (log variance
 * 0 while n < 2).  Output: denoised RGB.  Weights, activations and the
 * operands of every conv3x3 product are bfloat16 on gfx950 MFMA units with
 * FP32 accumulation; master weights, gradients and Adam state are FP32.
 * Parameters are ordered as: for each of the 12 conv3x3 layers (enc1a,
 * enc1b, enc2a, enc2b, enc3a, enc3b, up2, dec2a, dec2b, up1, dec1a, dec1b)
 * its weights [3][3][c_in][c_out] then its bias [c_out]; then the 1x1 output
 * weights [32][3] and bias [3].
 *
 * Conventions as in dfb.h (status codes, stream ordering, sticky HIP errors,
 * one host thread per handle).  Tensors are device pointers, NHWC float32:
 * inputs [n][h][w][6], outputs and targets [n][h][w][3]; h and w must be
 * multiples of 4 and n*h*w at most the configured maximum.
 */
#ifndef DFB_DENOISE_H
#define DFB_DENOISE_H

#include <stdint.h>

#include "dfb.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dfb_denoiser_ctx* dfb_denoiser;

typedef struct {
  int64_t max_pixels;  /* largest n*h*w of any call (sizes the activation buffers) */
  uint32_t seed;       /* He-normal initialisation of the conv3x3 weights */
  float beta1, beta2, eps;  /* Adam (0 -> 0.9, 0.999, 1e-8) */
} dfb_unet_config;

/* Number of float parameters (the layout above). */
int64_t dfb_denoiser_param_count(void);

dfb_status dfb_denoiser_create(const dfb_unet_config* cfg, void* hip_stream, dfb_denoiser* out);
dfb_status dfb_denoiser_destroy(dfb_denoiser net);

/* Replace the FP32 master parameters (host array of param_count floats);
 * resets Adam's moments and step count. */
dfb_status dfb_denoiser_set_params(dfb_denoiser net, const float* host, int64_t n);

/* Copy out, to host: what = 0 master parameters, 1 gradients of the last
 * train step, 2 Adam first moments, 3 Adam second moments. */
dfb_status dfb_denoiser_get_params(dfb_denoiser net, int32_t what, float* host, int64_t n);

/* Forward pass: out = mean RGB + network residual. */
dfb_status dfb_denoiser_forward(dfb_denoiser net, const float* in_dev, float* out_dev, int32_t n,
                                int32_t h, int32_t w);

/* One training step on a batch: forward, MSE loss against target, backward
 * (data and weight gradients), then (if apply_update) one Adam step with
 * learning rate lr.  loss_out: nullable host float (synchronises). */
dfb_status dfb_denoiser_train_step(dfb_denoiser net, const float* in_dev, const float* target_dev,
                                   int32_t n, int32_t h, int32_t w, float lr, int32_t apply_update,
                                   float* loss_out);

/* bfloat16 output (NHWC, uint16 bit patterns) of conv3x3 layer `layer`
 * (0..11, order above) from the last forward, copied to host: bytes must be
 * n*h_l*w_l*c_out*2 for that layer's resolution.  After dfb_denoise the last
 * layer (11) is not available (DFB_ERR_STATE): that call computes the output
 * conv in the last layer's epilogue and does not store its activation. */
dfb_status dfb_denoiser_read_activation(dfb_denoiser net, int32_t layer, void* host, int64_t bytes);

/* The network input of the compositor's current accumulation (its mean,
 * per-tile variance and n) as NHWC [height][width][6] float32 on device. */
dfb_status dfb_denoiser_frame_input(dfb_handle h, float* in_dev);

/* Denoise the compositor's current accumulation in place of its display:
 * runs the network on the whole frame, then per tile keeps the plain mean
 * where the measured variance exceeds var_threshold (n >= 2 and v_t > tau)
 * and the denoised RGB elsewhere (alpha stays the mean's), stores the result
 * as DFB_BUF_DENOISED_F32 and converts it to the display format. */
dfb_status dfb_denoise(dfb_handle h, dfb_denoiser net, float var_threshold);

const char* dfb_denoiser_last_error(dfb_denoiser net);

#ifdef __cplusplus
}
#endif
#endif /* DFB_DENOISE_H */
