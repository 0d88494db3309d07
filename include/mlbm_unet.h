/*
 * mlbm_unet.h - C ABI of the warm-start network (libmlbm.so).
 *
 * The warm start maps a rasterised periodic porous geometry to an initial
 * velocity and density field for the meshless LBM (the project's learned
 * initialisation; the paper starts every run from rest, Sec. 3.1).  The
 * network is an encoder-decoder with skip connections (5 levels in use).
 *
 * The whole network runs through mlbm_unet_forward / _loss / _backward /
 * _adam on one descriptor (below); the layer entry points further down are
 * what those call, exposed for tests of single layers.
 *
 * Conventions: as in mlbm.h (return codes, mlbm_last_error, caller-owned
 * device memory, asynchronous on the given stream, no device allocation).
 * Activations are NHWC bfloat16.  A tensor view is a device pointer plus a
 * channel stride (channels per pixel of the buffer) and a channel offset, so
 * the decoder's concatenations are written in place.  Convolutions are
 * periodic (circular padding) and accumulate in FP32.
 */
#ifndef MLBM_UNET_H
#define MLBM_UNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- the network -------------------------------------------------------------------------
 * Levels l = 0 .. L-1 at resolution res / 2^l with c_l channels: per encoder
 * level two 3x3 convolutions with ReLU (2x2 average pooling between levels),
 * per decoder level a nearest upsampling, the concatenation [upsampled, skip]
 * and two 3x3 convolutions with ReLU, then a 1x1 head.  Input and output are
 * padded to 32 channels: the input image is bf16 [batch][res][res][32] with
 * the c_in real channels first (the rest zero), the output FP32
 * [batch][res][res][32] of which the first c_out channels are the prediction.
 * Layers, in execution order (mlbm_unet_layer): enc0a, enc0b, enc1a, ...,
 * enc{L-1}b, dec{L-2}a, dec{L-2}b, ..., dec0b, head.  Parameters: one FP32
 * array holding, layer after layer, the weights [c_out][k*k][c_in] (tap =
 * dy * k + dx) and the bias [c_out].  All buffers are caller-allocated device
 * memory sized by mlbm_unet_sizes; every call is asynchronous on hip_stream.
 */
#define MLBM_UNET_MAX_LEVELS 6

typedef struct mlbm_unet {
    int32_t levels;                          /* L, 2 .. MLBM_UNET_MAX_LEVELS            */
    int32_t channels[MLBM_UNET_MAX_LEVELS];  /* c_l: multiples of 32, <= 256            */
    int32_t batch;                           /* images per pass                         */
    int32_t res;                             /* square resolution; res / 2^(L-1) must be
                                                8 or a multiple of 16                   */
    int32_t c_in, c_out;                     /* real input / output channels, 1 .. 32   */
    float *params;      /* FP32 [n_params]                                               */
    float *grads;       /* FP32 [n_params]: written by mlbm_unet_backward                 */
    float *adam_m, *adam_v; /* FP32 [n_params] Adam moments (zero before the first step) */
    void *w_bf16;       /* w_bf16_bytes: bf16 copies of the weights (mlbm_unet_refresh)  */
    void *act;          /* act_bytes: activations of the last forward pass               */
    void *act_grad;     /* act_bytes: activation gradients (the loss's output gradient
                           included)                                                     */
    void *work;         /* work_bytes: weight-gradient partials, loss partials           */
} mlbm_unet;

typedef struct mlbm_unet_buffers {
    int64_t n_params;       /* FP32 values of params, grads, adam_m, adam_v             */
    int64_t w_bf16_bytes, act_bytes, work_bytes;
    int32_t n_layers;
} mlbm_unet_buffers;

typedef struct mlbm_unet_layer_info {
    char name[8];            /* "enc0a" .. "head"                                        */
    int32_t ksize, c_in, c_out, res;
    int64_t w_offset, b_offset;  /* float offsets of the weights and bias in params   */
} mlbm_unet_layer_info;

/* Sizes of the buffers for net's shape (its pointers are not read).
 * Errors: MLBM_ERR_ARG (levels, channels, batch or resolution out of range). */
int mlbm_unet_sizes(const mlbm_unet *net, mlbm_unet_buffers *out);

/* Shape and parameter offsets of layer `index` (0 .. n_layers - 1). */
int mlbm_unet_layer(const mlbm_unet *net, int32_t index, mlbm_unet_layer_info *out);

/* bf16 copies of params (forward and data-gradient layouts) into w_bf16. */
int mlbm_unet_refresh(const mlbm_unet *net, void *hip_stream);

/* Forward pass of x (bf16 [batch][res][res][32]) into out (FP32
 * [batch][res][res][c_out]); keeps the activations in act. */
int mlbm_unet_forward(const mlbm_unet *net, const void *x, float *out, void *hip_stream);

/* loss = sum_p mask[p] sum_{c < c_out} (out[p, c] - target[p, c])^2 / (c_out
 * sum_p mask[p]) (device FP32 scalar), with out FP32 [P][c_out], target FP32
 * [P][c_out], mask FP32 [P] (P = batch res^2); the gradient with respect to
 * out is left in act_grad for mlbm_unet_backward.  The normalisation is
 * formed on the device. */
int mlbm_unet_loss(const mlbm_unet *net, const float *out, const float *target, const float *mask, float *loss,
                   void *hip_stream);

/* Gradients of the loss with respect to every parameter (grads), for the
 * input x of the last forward pass: the layers' backward products in reverse
 * order, through the pooling, upsampling, skip concatenations and ReLUs.
 * Weight gradients sum pixel splits in a fixed order (deterministic). */
int mlbm_unet_backward(const mlbm_unet *net, const void *x, void *hip_stream);

/* One bias-corrected Adam step (step t >= 1) on every parameter, after zeroing
 * the gradients of the padded input channels of enc0a and of the padded head
 * outputs (so they stay zero), then mlbm_unet_refresh. */
int mlbm_unet_adam(const mlbm_unet *net, float lr, float beta1, float beta2, float eps, int32_t t,
                   void *hip_stream);

/* ---- layers ---------------------------------------------------------------------------------- */
typedef struct mlbm_conv_desc {
    int32_t n, h, w;          /* images, height (a multiple of 8), width (8 or a
                                 multiple of 16)                                    */
    int32_t c_in, c_out;      /* multiples of 32 (c_out <= 256 for a bias gradient) */
    int32_t ksize;            /* 1 or 3                                             */
    int32_t x_stride, x_offset; /* input view (channels, multiples of 8)           */
    int32_t y_stride, y_offset; /* output view, or the output-gradient view        */
    int32_t c_store;          /* forward: output channels stored (<= c_out)         */
} mlbm_conv_desc;

/*
 * y[p, o] = bias[o] + sum_{tap, i} x[p + tap, i] w[o][tap][i], optional ReLU;
 * w bf16 [c_out][ksize^2][c_in] (tap = dy * ksize + dx, offsets dy - r, dx - r);
 * bias FP32 [c_out] or NULL; y bf16 or (y_f32) FP32.  The data gradient of a
 * convolution is this call on the output gradient with the weights from
 * mlbm_conv_weights' w_dgrad (c_in and c_out exchanged).
 * Errors: MLBM_ERR_ARG (layout), MLBM_ERR_HIP.
 */
int mlbm_conv_forward(const mlbm_conv_desc *desc, const void *x, const void *w, const float *bias, void *y,
                      int32_t relu, int32_t y_f32, void *hip_stream);

/* Workspace bytes of mlbm_conv_wgrad for `splits` pixel splits. */
int64_t mlbm_conv_wgrad_workspace(const mlbm_conv_desc *desc, int32_t splits);

/*
 * dw[o][tap][i] = sum_p dy[p, o] x[p + tap, i] (FP32, written) and, if db is
 * non-NULL, db[o] = sum_p dy[p, o]; the pixel sum is split into `splits`
 * parts whose partials are added in a fixed order (deterministic).  x and dy
 * must be 16-byte aligned (MLBM_ERR_ARG otherwise).
 */
int mlbm_conv_wgrad(const mlbm_conv_desc *desc, const void *x, const void *dy, float *dw, float *db, int32_t splits,
                    void *workspace, void *hip_stream);

/* bf16 copies of FP32 master weights [c_out][k*k][c_in]: w_fwd in the same
 * layout, w_dgrad as [c_in][k*k][c_out] with mirrored taps.  Either may be NULL. */
int mlbm_conv_weights(const float *w_master, int32_t c_out, int32_t ksize, int32_t c_in, void *w_fwd, void *w_dgrad,
                      void *hip_stream);

/* dy[p, c] = 0 where y[p, c] <= 0 (gradient through ReLU given its output). */
int mlbm_relu_backward(int64_t pixels, int32_t channels, const void *y, int32_t y_stride, int32_t y_offset, void *dy,
                       int32_t dy_stride, int32_t dy_offset, void *hip_stream);

/* 2x2 average pooling: x (n, 2h, 2w, c) -> y (n, h, w, c). */
int mlbm_pool_forward(int32_t n, int32_t h, int32_t w, int32_t c, const void *x, int32_t xs, int32_t xo, void *y,
                      int32_t ys, int32_t yo, void *hip_stream);

/* dx (n, 2h, 2w, c) = dy / 4 on each 2x2 block, plus `add` (same shape as dx) if non-NULL. */
int mlbm_pool_backward(int32_t n, int32_t h, int32_t w, int32_t c, const void *dy, int32_t dys, int32_t dyo, void *dx,
                       int32_t dxs, int32_t dxo, const void *add, int32_t as, int32_t ao, void *hip_stream);

/* nearest doubling: x (n, h, w, c) -> y (n, 2h, 2w, c). */
int mlbm_upsample_forward(int32_t n, int32_t h, int32_t w, int32_t c, const void *x, int32_t xs, int32_t xo, void *y,
                          int32_t ys, int32_t yo, void *hip_stream);

/* dx (n, h, w, c) = sum over each 2x2 block of dy (n, 2h, 2w, c). */
int mlbm_upsample_backward(int32_t n, int32_t h, int32_t w, int32_t c, const void *dy, int32_t dys, int32_t dyo,
                           void *dx, int32_t dxs, int32_t dxo, void *hip_stream);

/* Workspace bytes of mlbm_masked_mse. */
int64_t mlbm_mse_workspace(int64_t pixels);

/*
 * loss = inv_count * sum_p mask[p] sum_{c < C} (pred[p, c] - target[p, c])^2 (device FP32
 * scalar), pred FP32 [p][pred_stride], target FP32 [p][C], mask FP32 [p]; dpred (bf16
 * [p][pred_stride], zero past C) = 2 mask (pred - target) inv_count if non-NULL.
 */
int mlbm_masked_mse(int64_t pixels, int32_t c, const float *pred, int32_t pred_stride, const float *target,
                    const float *mask, float inv_count, void *dpred, void *workspace, float *loss, void *hip_stream);

/* One bias-corrected Adam step on m FP32 parameters (step t >= 1). */
int mlbm_adam(int64_t m, float *param, const float *grad, float *m1, float *m2, float lr, float beta1, float beta2,
              float eps, int32_t t, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* MLBM_UNET_H */
