/*
 * ncs_cnn.h -- C ABI of the learned warm start for the NCS solver (gfx950).
 *
 * The paper starts NCS from x = 0 (Section 4).  This part adds a learned
 * initial point: the sinogram b is backprojected and filtered with the
 * method's own circulant inverse, z = alpha M^+ E^T b (ncs_prefilter in
 * ncs.h, the multiplier of Section 4.1.1), and a small residual network maps
 * z to x0 = z + N(z).  NCS then starts from x0 with duals taken from the
 * fixed-point relations (ncs_set_init with dual_from_x0 = 1, Section 3.2),
 * and runs to the same objective target as a cold start, so the result is
 * still decided by NCS.
 *
 * Network N: six 3x3 convolutions with zero padding ("same" size), channels
 * 1 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after the first five.
 * Activations and weights are bfloat16; products are accumulated in float on
 * the matrix cores; biases, the residual sum and the output are float.
 *
 * Parameters: one float vector of NCS_CNN_N_PARAMS values.  For each layer
 * in order it holds the weights w[t][c_out][c_in] (row-major; tap
 * t = 3 (dy + 1) + (dx + 1) reads the input pixel (row + dy, col + dx)) and
 * then the bias[c_out].
 *
 * Training: mean squared error L = mean over the batch's pixels of
 * (x0 - target)^2, gradients by backpropagation (bfloat16 activation
 * gradients, float accumulation), Adam on float master parameters (Kingma
 * and Ba, with bias correction).
 *
 * Layouts: images are float [batch][height][width] row-major; activations
 * for the layer-level calls are bfloat16 (uint16 storage) NHWC
 * [batch][height][width][channels].  Any height and width >= 1.
 *
 * Memory, streams and errors follow ncs.h: pointers named *_dev are device
 * pointers owned by the caller; work is queued on the stream given at
 * creation (or per call for the layer-level calls); calls that return host
 * values synchronise; a failing call returns a negative status and leaves a
 * message for ncs_last_error().
 */
#ifndef NCS_CNN_H
#define NCS_CNN_H

#include "ncs.h"

#ifdef __cplusplus
extern "C" {
#endif

#define NCS_CNN_N_PARAMS 37601
#define NCS_CNN_CHANNELS 32
#define NCS_CNN_LAYERS 6

typedef struct ncs_cnn ncs_cnn;

/* Workspace for batches of up to max_batch images of up to
 * max_height x max_width pixels (activations of the six layers and their
 * gradients, about 2 x 6 x 64 bytes per pixel).  Parameters start at zero;
 * set them with ncs_cnn_set_params. */
ncs_status ncs_cnn_create(int32_t max_batch, int32_t max_height, int32_t max_width, void* stream,
                          ncs_cnn** out);

/* Copy the parameter vector from / to the host.  Setting the parameters
 * resets the Adam moments and step count. */
ncs_status ncs_cnn_set_params(ncs_cnn* net, const float* params_host);
ncs_status ncs_cnn_get_params(ncs_cnn* net, float* params_host);

/* x0 = z + N(z) for a batch of images (z_dev and x0_dev may not alias). */
ncs_status ncs_cnn_forward(ncs_cnn* net, const float* z_dev, float* x0_dev, int32_t batch, int32_t height,
                           int32_t width);

/* Loss and gradient of the mean squared error of x0 = z + N(z) against
 * target_dev over the batch.  The gradient stays on the device for
 * ncs_cnn_adam_step; grad_host (NCS_CNN_N_PARAMS floats) and loss_host may
 * be NULL, and when either is non-NULL the call synchronises. */
ncs_status ncs_cnn_gradient(ncs_cnn* net, const float* z_dev, const float* target_dev, int32_t batch,
                            int32_t height, int32_t width, double* loss_host, float* grad_host);

/* One Adam step with the last gradient (step count t incremented first). */
ncs_status ncs_cnn_adam_step(ncs_cnn* net, float lr, float beta1, float beta2, float eps);

/* ncs_cnn_gradient followed by ncs_cnn_adam_step(lr, 0.9, 0.999, 1e-8).
 * loss_host may be NULL (no synchronisation). */
ncs_status ncs_cnn_train_step(ncs_cnn* net, const float* z_dev, const float* target_dev, int32_t batch,
                              int32_t height, int32_t width, float lr, double* loss_host);

/* Loss of the last gradient evaluation (synchronises). */
ncs_status ncs_cnn_last_loss(ncs_cnn* net, double* loss_host);

void ncs_cnn_destroy(ncs_cnn* net);

/* ---- Layer-level operations (the building blocks of the network) ---- */

typedef enum {
    NCS_CONV_RELU_BF16 = 0,   /* out (bf16 NHWC) = max(conv + bias, 0)                  */
    NCS_CONV_RESID_F32 = 1,   /* out (float image) = resid + conv + bias; c_out = 1      */
    NCS_CONV_MASK_BF16 = 2,   /* out (bf16 NHWC) = mask > 0 ? conv : 0 (no bias)         */
    NCS_CONV_F32 = 3          /* out (float NHWC) = conv + bias                          */
} ncs_conv_epilogue;

/* One 3x3 convolution of bfloat16 NHWC input in_dev [batch][h][w][c_in] with
 * weights w_dev (bfloat16 [9][c_out][c_in]) and bias_dev (float [c_out], may
 * be NULL for NCS_CONV_MASK_BF16).  (c_in, c_out) is one of (1, 32),
 * (32, 32), (32, 1).  mask_dev: bfloat16 NHWC [.., c_out] for
 * NCS_CONV_MASK_BF16; resid_dev: float [batch][h][w] for NCS_CONV_RESID_F32.
 * in_dev, w_dev, out_dev and mask_dev must be 16-byte aligned (channels are
 * read and written in groups of 8); NCS_ERR_INVALID_ARG otherwise. */
ncs_status ncs_conv3x3_bf16(const void* in_dev, const void* w_dev, const float* bias_dev, const void* mask_dev,
                            const float* resid_dev, void* out_dev, int32_t batch, int32_t height, int32_t width,
                            int32_t c_in, int32_t c_out, int32_t epilogue, void* stream);

/* Weight and bias gradient of one 3x3 convolution: with input x_dev
 * (bfloat16 NHWC, c_in channels) and output gradient dz_dev (bfloat16 NHWC,
 * c_out channels), grad_dev (float, 9 c_out c_in + c_out values) receives
 * dw[t][o][i] = sum_p dz[p][o] x[p + offset_t][i] and then dbias[o] =
 * sum_p dz[p][o].  x_dev and dz_dev must be 16-byte aligned.  Allocates and
 * frees a partial-sum buffer; synchronises. */
ncs_status ncs_conv3x3_wgrad_bf16(const void* x_dev, const void* dz_dev, int32_t batch, int32_t height,
                                  int32_t width, int32_t c_in, int32_t c_out, float* grad_dev, void* stream);

/* out_dev (bfloat16) = in_dev (float) rounded to nearest, ties to even. */
ncs_status ncs_to_bf16(const float* in_dev, void* out_dev, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NCS_CNN_H */
