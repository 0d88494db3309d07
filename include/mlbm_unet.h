/*
 * mlbm_unet.h - C ABI of the warm-start network's layer kernels (libmlbm.so).
 *
 * The warm start maps a rasterised periodic porous geometry to an initial
 * velocity and density field for the meshless LBM (the project's learned
 * initialisation; the paper starts every run from rest, Sec. 3.1).  The
 * network is a 5-level encoder-decoder with skip connections; these entry
 * points are its layers, composed by the caller.
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

typedef struct mlbm_conv_desc {
    int32_t n, h, w;          /* images, height, width; n*h*w a multiple of 128     */
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
