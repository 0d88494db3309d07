// Layer kernels of the warm-start network (gfx950): 3x3 / 1x1 periodic
// convolutions as implicit GEMMs on bf16 MFMA (forward, data gradient through
// flipped weights, weight gradient with a deterministic split over pixels),
// average pooling, nearest upsampling, ReLU gradient, masked MSE loss and Adam.
//
// Activations are NHWC bf16; a tensor view is (pointer, channel stride,
// channel offset), so concatenations are written in place.  Channel counts of
// every convolution are multiples of 32.  Accumulation is FP32 everywhere.
//
// MFMA operand layout of v_mfma_f32_32x32x16_bf16 (one wavefront): lane l
// holds 8 consecutive k of row (A) / column (B) l % 32 starting at k = 8 (l / 32);
// result register r of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "mlbm_internal.h"
#include "mlbm.h"
#include "mlbm_unet.h"

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }
__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ bf16x8 load_bf8(const unsigned short *p) {
    u4 v = *(const u4 *)p;
    return __builtin_bit_cast(bf16x8, v);
}

// pixel index -> (n, y, x) and the periodic neighbour at offset (oy, ox)
__device__ __forceinline__ int64_t shifted(int64_t p, int H, int W, int oy, int ox) {
    const int64_t hw = (int64_t)H * W;
    const int64_t n = p / hw;
    const int rem = (int)(p - n * hw);
    int y = rem / W + oy, x = rem % W + ox;
    y = y < 0 ? y + H : (y >= H ? y - H : y);
    x = x < 0 ? x + W : (x >= W ? x - W : x);
    return n * hw + (int64_t)y * W + x;
}

// ---- forward convolution ----------------------------------------------------------
// Block: 4 waves.  BN = 64: waves in a 2x2 grid over 64 pixels x 64 output
// channels; BN = 32: 4 waves over 128 pixels x 32 channels.
template <int BN>
__global__ void __launch_bounds__(256) k_conv_fwd(mlbm_conv_desc d, const unsigned short *x,
                                                 const unsigned short *w, const float *bias, void *y, int relu,
                                                 int y_f32) {
    constexpr int WAVES_PX = BN == 64 ? 2 : 4;
    constexpr int BM = 32 * WAVES_PX;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wr = wave % WAVES_PX, wc = wave / WAVES_PX;
    const int64_t p0 = (int64_t)blockIdx.x * BM + wr * 32;
    const int co0 = blockIdx.y * BN + wc * 32;
    const int row = lane & 31, khalf = (lane >> 5) * 8;
    const int64_t p = p0 + row;
    const int co = co0 + row;
    const int ks = d.ksize, r = ks / 2, taps = ks * ks;
    f32x16 acc = {};
    for (int t = 0; t < taps; ++t) {
        const int64_t ps = shifted(p, d.h, d.w, t / ks - r, t % ks - r);
        const unsigned short *xa = x + ps * d.x_stride + d.x_offset + khalf;
        const unsigned short *wb = w + ((int64_t)co * taps + t) * d.c_in + khalf;
        for (int c = 0; c < d.c_in; c += 16) {
            const bf16x8 a = load_bf8(xa + c);
            const bf16x8 b = load_bf8(wb + c);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
    }
    const int col = co0 + row;  // output channel of this lane
    const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int64_t pp = p0 + (q / 4) * 8 + (lane >> 5) * 4 + (q % 4);
        float v = acc[q] + bv;
        if (relu) v = fmaxf(v, 0.0f);
        if (col < d.c_store) {
            const int64_t o = pp * d.y_stride + d.y_offset + col;
            if (y_f32) ((float *)y)[o] = v;
            else ((unsigned short *)y)[o] = f2bf(v);
        }
    }
}

// Register-blocked forward convolution for c_out a multiple of 64: each wave
// computes 2 x 2 MFMA tiles (64 pixels x 64 output channels), so every operand
// fragment it loads feeds two MFMAs (half the loads per MFMA of k_conv_fwd);
// 2 waves per block over 128 pixels.
__global__ void __launch_bounds__(128) k_conv_fwd_rb(mlbm_conv_desc d, const unsigned short *x,
                                                    const unsigned short *w, const float *bias, void *y, int relu,
                                                    int y_f32) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t p0 = (int64_t)blockIdx.x * 128 + wave * 64;
    const int co0 = blockIdx.y * 64;
    const int row = lane & 31, khalf = (lane >> 5) * 8;
    const int ks = d.ksize, r = ks / 2, taps = ks * ks;
    f32x16 acc[2][2] = {};
    for (int t = 0; t < taps; ++t) {
        const unsigned short *xa[2], *wb[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int64_t ps = shifted(p0 + 32 * i + row, d.h, d.w, t / ks - r, t % ks - r);
            xa[i] = x + ps * d.x_stride + d.x_offset + khalf;
            wb[i] = w + ((int64_t)(co0 + 32 * i + row) * taps + t) * d.c_in + khalf;
        }
        for (int c = 0; c < d.c_in; c += 16) {
            const bf16x8 a0 = load_bf8(xa[0] + c), a1 = load_bf8(xa[1] + c);
            const bf16x8 b0 = load_bf8(wb[0] + c), b1 = load_bf8(wb[1] + c);
            acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1, acc[1][1], 0, 0, 0);
        }
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = co0 + 32 * j + row;  // output channel of this lane
        const float bv = bias ? bias[col] : 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int64_t pp = p0 + 32 * i + (q / 4) * 8 + (lane >> 5) * 4 + (q % 4);
                float v = acc[i][j][q] + bv;
                if (relu) v = fmaxf(v, 0.0f);
                if (col < d.c_store) {
                    const int64_t o = pp * d.y_stride + d.y_offset + col;
                    if (y_f32) ((float *)y)[o] = v;
                    else ((unsigned short *)y)[o] = f2bf(v);
                }
            }
        }
    }
}

// ---- weight gradient ----------------------------------------------------------------
// One wave per (32 output channels) x (32 input channels) x tap tile and pixel
// split; 64-pixel chunks of dy and of the shifted x are transposed through LDS
// so every lane reads 8 consecutive pixels.  Partial sums go to ws[split].
__global__ void __launch_bounds__(64) k_conv_wgrad(mlbm_conv_desc d, const unsigned short *x,
                                                  const unsigned short *dy, float *ws, int64_t px_per_split) {
    __shared__ __align__(16) unsigned short sa[32][64 + 8];  // [co][pixel]
    __shared__ __align__(16) unsigned short sb[32][64 + 8];  // [ci][pixel]
    const int lane = threadIdx.x;
    const int co0 = blockIdx.x * 32, ci0 = blockIdx.y * 32;
    const int taps = d.ksize * d.ksize, r = d.ksize / 2;
    const int t = blockIdx.z % taps, split = blockIdx.z / taps;
    const int oy = t / d.ksize - r, ox = t % d.ksize - r;
    const int64_t P = (int64_t)d.n * d.h * d.w;
    const int64_t pa = split * px_per_split, pb = min(P, pa + px_per_split);
    f32x16 acc = {};
    for (int64_t c0 = pa; c0 < pb; c0 += 64) {
        // stage: lane handles pixel c0 + lane (zero past the end)
        const int64_t p = c0 + lane;
        const bool in = p < pb;
        const int64_t ps = in ? shifted(p, d.h, d.w, oy, ox) : 0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            u4 va = in ? *(const u4 *)(dy + p * d.y_stride + d.y_offset + co0 + 8 * g) : u4{0, 0, 0, 0};
            u4 vb = in ? *(const u4 *)(x + ps * d.x_stride + d.x_offset + ci0 + 8 * g) : u4{0, 0, 0, 0};
            const unsigned a8[4] = {va.x, va.y, va.z, va.w}, b8[4] = {vb.x, vb.y, vb.z, vb.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                sa[8 * g + 2 * h][lane] = (unsigned short)(a8[h] & 0xffff);
                sa[8 * g + 2 * h + 1][lane] = (unsigned short)(a8[h] >> 16);
                sb[8 * g + 2 * h][lane] = (unsigned short)(b8[h] & 0xffff);
                sb[8 * g + 2 * h + 1][lane] = (unsigned short)(b8[h] >> 16);
            }
        }
        __syncthreads();
        const int row = lane & 31, kh = (lane >> 5) * 8;
#pragma unroll
        for (int kk = 0; kk < 64; kk += 16) {
            const bf16x8 a = load_bf8(&sa[row][kk + kh]);
            const bf16x8 b = load_bf8(&sb[row][kk + kh]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // ws layout [split][c_out][taps][c_in]
    const int ci = ci0 + (lane & 31);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int co = co0 + (q / 4) * 8 + (lane >> 5) * 4 + (q % 4);
        ws[(((int64_t)split * d.c_out + co) * taps + t) * d.c_in + ci] = acc[q];
    }
}

// sum of the split partials in a fixed order; dw[c_out][taps][c_in]
__global__ void k_sum_splits(const float *ws, int splits, int64_t m, float *dw, int accumulate) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    float s = 0.0f;
    for (int k = 0; k < splits; ++k) s += ws[(int64_t)k * m + i];
    dw[i] = accumulate ? dw[i] + s : s;
}

// bias gradient: per-channel sums of dy in a fixed order (partials per block)
// Partial bias gradient of px_per_block pixels: thread t reads channels
// 8 (t % G) .. 8 (t % G) + 7 (one 16-byte load) of every (256 / G)-th pixel,
// G = c_out / 8 channel groups; the rows of the block are then summed per
// channel through LDS in a fixed order (deterministic).  c_out <= 256.
__global__ void __launch_bounds__(256) k_bias_partial(mlbm_conv_desc d, const unsigned short *dy, float *ws,
                                                     int64_t px_per_block) {
    __shared__ float red[256][9];
    const int G = d.c_out >> 3, rows = (int)blockDim.x / G;
    const int g = (int)threadIdx.x % G, r = (int)threadIdx.x / G;
    const int64_t P = (int64_t)d.n * d.h * d.w;
    const int64_t a = blockIdx.x * px_per_block, b = min(P, a + px_per_block);
    float s[8] = {};
    if (r < rows) {
#pragma unroll 4
        for (int64_t p = a + r; p < b; p += rows) {
            const u4 v = *(const u4 *)(dy + p * d.y_stride + d.y_offset + 8 * g);
            const unsigned h[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[2 * k] += __uint_as_float(h[k] << 16);
                s[2 * k + 1] += __uint_as_float(h[k] & 0xffff0000u);
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) red[threadIdx.x][k] = s[k];
    __syncthreads();
    const int c = threadIdx.x;
    if (c < d.c_out) {
        float acc = 0.0f;
        for (int rr = 0; rr < rows; ++rr) acc += red[rr * G + (c >> 3)][c & 7];
        ws[(int64_t)blockIdx.x * d.c_out + c] = acc;
    }
}

__global__ void k_bias_sum(const float *ws, int blocks, int c_out, float *db) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c_out) return;
    float s = 0.0f;
    for (int k = 0; k < blocks; ++k) s += ws[(int64_t)k * c_out + c];
    db[c] = s;
}

// ---- weights: FP32 master -> bf16 forward layout and flipped data-gradient layout ------
// master [c_out][taps][c_in]; fwd (same layout) bf16; dgrad [c_in][taps][c_out] with the tap
// mirrored (the adjoint of a periodic convolution is the convolution with mirrored taps).
__global__ void k_weights_bf16(const float *wm, int c_out, int taps, int c_in, unsigned short *wf,
                               unsigned short *wd) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m = (int64_t)c_out * taps * c_in;
    if (i >= m) return;
    const int ci = (int)(i % c_in), t = (int)((i / c_in) % taps), co = (int)(i / ((int64_t)c_in * taps));
    const unsigned short v = f2bf(wm[i]);
    if (wf) wf[i] = v;
    if (wd) wd[((int64_t)ci * taps + (taps - 1 - t)) * c_out + co] = v;
}

// ---- elementwise layers -------------------------------------------------------------------
__global__ void k_relu_bwd(int64_t P, int C, const unsigned short *y, int y_stride, int y_offset,
                           unsigned short *dy, int dy_stride, int dy_offset) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * C) return;
    const int64_t p = i / C;
    const int c = (int)(i - p * C);
    if (!(bf2f(y[p * y_stride + y_offset + c]) > 0.0f)) dy[p * dy_stride + dy_offset + c] = 0;
}

// 2x2 average pooling of x (n, 2h, 2w) into y (n, h, w)
__global__ void k_pool_fwd(int n, int h, int w, int C, const unsigned short *x, int xs, int xo, unsigned short *y,
                           int ys, int yo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)n * h * w * C;
    if (i >= tot) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int xx = (int)(q % w), yy = (int)((q / w) % h);
    const int64_t nn = q / ((int64_t)w * h);
    const int W2 = 2 * w;
    const int64_t b = (nn * 2 * h + 2 * yy) * W2 + 2 * xx;
    const float s = bf2f(x[b * xs + xo + c]) + bf2f(x[(b + 1) * xs + xo + c]) + bf2f(x[(b + W2) * xs + xo + c]) +
                    bf2f(x[(b + W2 + 1) * xs + xo + c]);
    y[q * ys + yo + c] = f2bf(0.25f * s);
}

// dx (n, 2h, 2w) = dy / 4 spread over each 2x2 block, plus add (same shape as dx) if given
__global__ void k_pool_bwd(int n, int h, int w, int C, const unsigned short *dy, int dys, int dyo, unsigned short *dx,
                           int dxs, int dxo, const unsigned short *add, int as, int ao) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)n * 4 * h * w * C;
    if (i >= tot) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int W2 = 2 * w;
    const int xx = (int)(q % W2), yy = (int)((q / W2) % (2 * h));
    const int64_t nn = q / ((int64_t)W2 * 2 * h);
    const int64_t src = (nn * h + yy / 2) * w + xx / 2;
    float v = 0.25f * bf2f(dy[src * dys + dyo + c]);
    if (add) v += bf2f(add[q * as + ao + c]);
    dx[q * dxs + dxo + c] = f2bf(v);
}

// nearest doubling of x (n, h, w) into y (n, 2h, 2w)
__global__ void k_up_fwd(int n, int h, int w, int C, const unsigned short *x, int xs, int xo, unsigned short *y, int ys,
                         int yo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)n * 4 * h * w * C;
    if (i >= tot) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int W2 = 2 * w;
    const int xx = (int)(q % W2), yy = (int)((q / W2) % (2 * h));
    const int64_t nn = q / ((int64_t)W2 * 2 * h);
    const int64_t src = (nn * h + yy / 2) * w + xx / 2;
    y[q * ys + yo + c] = x[src * xs + xo + c];
}

// dx (n, h, w) = sum of dy over each 2x2 block of (n, 2h, 2w)
__global__ void k_up_bwd(int n, int h, int w, int C, const unsigned short *dy, int dys, int dyo, unsigned short *dx,
                         int dxs, int dxo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)n * h * w * C;
    if (i >= tot) return;
    const int c = (int)(i % C);
    const int64_t q = i / C;
    const int xx = (int)(q % w), yy = (int)((q / w) % h);
    const int64_t nn = q / ((int64_t)w * h);
    const int W2 = 2 * w;
    const int64_t b = (nn * 2 * h + 2 * yy) * W2 + 2 * xx;
    const float s = bf2f(dy[b * dys + dyo + c]) + bf2f(dy[(b + 1) * dys + dyo + c]) +
                    bf2f(dy[(b + W2) * dys + dyo + c]) + bf2f(dy[(b + W2 + 1) * dys + dyo + c]);
    dx[q * dxs + dxo + c] = f2bf(s);
}

// masked MSE over the first C channels of pred (fp32 [P][ps]): per-block partial
// sums of the squared error and of the mask, and dpred (bf16 [P][ps], zero past C)
__global__ void __launch_bounds__(256) k_mse(int64_t P, int C, const float *pred, int ps, const float *target,
                                            const float *mask, float inv_count, unsigned short *dpred,
                                            double *partial) {
    __shared__ double s1[256];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (p < P) {
        const float m = mask[p];
        for (int c = 0; c < ps; ++c) {
            float g = 0.0f;
            if (c < C) {
                const float d = (pred[p * ps + c] - target[p * C + c]) * m;
                e += (double)d * d;
                g = 2.0f * d * inv_count;
            }
            if (dpred) dpred[p * ps + c] = f2bf(g);
        }
    }
    s1[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s1[threadIdx.x] += s1[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s1[0];
}

__global__ void k_sum_partials(const double *partial, int64_t m, double scale, float *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int64_t i = 0; i < m; ++i) s += partial[i];
    out[0] = (float)(s * scale);
}

__global__ void k_adam(int64_t m, float *p, const float *g, float *mo, float *vo, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float gi = g[i];
    const float mi = b1 * mo[i] + (1.0f - b1) * gi;
    const float vi = b2 * vo[i] + (1.0f - b2) * gi * gi;
    mo[i] = mi;
    vo[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

int check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mlbm::fail(MLBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return MLBM_OK;
}

unsigned blocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

int check_desc(const mlbm_conv_desc *d) {
    using mlbm::fail;
    if (!d) return fail(MLBM_ERR_ARG, "null descriptor");
    if (d->ksize != 1 && d->ksize != 3) return fail(MLBM_ERR_ARG, "ksize must be 1 or 3");
    if (d->n < 1 || d->h < 1 || d->w < 1) return fail(MLBM_ERR_ARG, "empty tensor");
    if (d->c_in < 32 || d->c_in % 32 || d->c_out < 32 || d->c_out % 32)
        return fail(MLBM_ERR_ARG, "channel counts must be multiples of 32");
    if (((int64_t)d->n * d->h * d->w) % 128) return fail(MLBM_ERR_ARG, "pixel count must be a multiple of 128");
    if (d->x_stride % 8 || d->x_offset % 8 || d->y_stride % 8 || d->y_offset % 8)
        return fail(MLBM_ERR_ARG, "strides and offsets must be multiples of 8 channels");
    if (d->x_offset + d->c_in > d->x_stride) return fail(MLBM_ERR_ARG, "input view exceeds its stride");
    if (d->c_store < 1 || d->c_store > d->c_out) return fail(MLBM_ERR_ARG, "c_store outside [1, c_out]");
    return MLBM_OK;
}

}  // namespace

extern "C" int mlbm_conv_forward(const mlbm_conv_desc *d, const void *x, const void *w, const float *bias, void *y,
                                 int32_t relu, int32_t y_f32, void *stream) {
    mlbm::clear_error();
    int rc = check_desc(d);
    if (rc) return rc;
    if (!x || !w || !y) return mlbm::fail(MLBM_ERR_ARG, "null pointer");
    if (d->y_offset + d->c_store > d->y_stride) return mlbm::fail(MLBM_ERR_ARG, "output view exceeds its stride");
    const int64_t P = (int64_t)d->n * d->h * d->w;
    hipStream_t s = (hipStream_t)stream;
    if (d->c_out % 64 == 0)  // (the pixel count is a multiple of 128: check_desc)
        hipLaunchKernelGGL(k_conv_fwd_rb, dim3((unsigned)(P / 128), d->c_out / 64), dim3(128), 0, s, *d,
                           (const unsigned short *)x, (const unsigned short *)w, bias, y, relu, y_f32);
    else
        hipLaunchKernelGGL(k_conv_fwd<32>, dim3((unsigned)(P / 128), d->c_out / 32), dim3(256), 0, s, *d,
                           (const unsigned short *)x, (const unsigned short *)w, bias, y, relu, y_f32);
    return check("mlbm_conv_forward");
}

extern "C" int64_t mlbm_conv_wgrad_workspace(const mlbm_conv_desc *d, int32_t splits) {
    if (!d || splits < 1) return 0;
    const int64_t m = (int64_t)d->c_out * d->ksize * d->ksize * d->c_in;
    const int64_t P = (int64_t)d->n * d->h * d->w;
    const int64_t bias_blocks = (P + 4095) / 4096;
    return (m * splits + bias_blocks * d->c_out) * (int64_t)sizeof(float);
}

extern "C" int mlbm_conv_wgrad(const mlbm_conv_desc *d, const void *x, const void *dy, float *dw, float *db,
                               int32_t splits, void *workspace, void *stream) {
    mlbm::clear_error();
    int rc = check_desc(d);
    if (rc) return rc;
    if (!x || !dy || !dw || !workspace || splits < 1) return mlbm::fail(MLBM_ERR_ARG, "null pointer or splits < 1");
    if (db && d->c_out > 256) return mlbm::fail(MLBM_ERR_ARG, "bias gradient needs c_out <= 256");
    if (((uintptr_t)x | (uintptr_t)dy) & 15) return mlbm::fail(MLBM_ERR_ARG, "x and dy must be 16-byte aligned");
    if (d->y_offset + d->c_out > d->y_stride) return mlbm::fail(MLBM_ERR_ARG, "gradient view exceeds its stride");
    const int64_t P = (int64_t)d->n * d->h * d->w;
    const int taps = d->ksize * d->ksize;
    const int64_t m = (int64_t)d->c_out * taps * d->c_in;
    int64_t per = (P + splits - 1) / splits;
    per = (per + 63) / 64 * 64;
    const int sp = (int)((P + per - 1) / per);
    float *ws = (float *)workspace;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_conv_wgrad, dim3(d->c_out / 32, d->c_in / 32, taps * sp), dim3(64), 0, s, *d,
                       (const unsigned short *)x, (const unsigned short *)dy, ws, per);
    hipLaunchKernelGGL(k_sum_splits, dim3(blocks(m)), dim3(256), 0, s, (const float *)ws, sp, m, dw, 0);
    if (db) {
        const int64_t pb = 4096;
        const int nb = (int)((P + pb - 1) / pb);
        float *wsb = ws + m * splits;
        hipLaunchKernelGGL(k_bias_partial, dim3(nb), dim3(256), 0, s, *d, (const unsigned short *)dy, wsb, pb);
        hipLaunchKernelGGL(k_bias_sum, dim3(1), dim3(256), 0, s, (const float *)wsb, nb, d->c_out, db);
    }
    return check("mlbm_conv_wgrad");
}

extern "C" int mlbm_conv_weights(const float *w_master, int32_t c_out, int32_t ksize, int32_t c_in, void *w_fwd,
                                 void *w_dgrad, void *stream) {
    mlbm::clear_error();
    if (!w_master || (!w_fwd && !w_dgrad) || c_out < 1 || c_in < 1 || (ksize != 1 && ksize != 3))
        return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    const int64_t m = (int64_t)c_out * ksize * ksize * c_in;
    hipLaunchKernelGGL(k_weights_bf16, dim3(blocks(m)), dim3(256), 0, (hipStream_t)stream, w_master, c_out,
                       ksize * ksize, c_in, (unsigned short *)w_fwd, (unsigned short *)w_dgrad);
    return check("mlbm_conv_weights");
}

extern "C" int mlbm_relu_backward(int64_t pixels, int32_t channels, const void *y, int32_t y_stride, int32_t y_offset,
                                  void *dy, int32_t dy_stride, int32_t dy_offset, void *stream) {
    mlbm::clear_error();
    if (!y || !dy || pixels < 1 || channels < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    hipLaunchKernelGGL(k_relu_bwd, dim3(blocks(pixels * channels)), dim3(256), 0, (hipStream_t)stream, pixels,
                       channels, (const unsigned short *)y, y_stride, y_offset, (unsigned short *)dy, dy_stride,
                       dy_offset);
    return check("mlbm_relu_backward");
}

extern "C" int mlbm_pool_forward(int32_t n, int32_t h, int32_t w, int32_t c, const void *x, int32_t xs, int32_t xo,
                                 void *y, int32_t ys, int32_t yo, void *stream) {
    mlbm::clear_error();
    if (!x || !y || n < 1 || h < 1 || w < 1 || c < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    hipLaunchKernelGGL(k_pool_fwd, dim3(blocks((int64_t)n * h * w * c)), dim3(256), 0, (hipStream_t)stream, n, h, w, c,
                       (const unsigned short *)x, xs, xo, (unsigned short *)y, ys, yo);
    return check("mlbm_pool_forward");
}

extern "C" int mlbm_pool_backward(int32_t n, int32_t h, int32_t w, int32_t c, const void *dy, int32_t dys,
                                  int32_t dyo, void *dx, int32_t dxs, int32_t dxo, const void *add, int32_t as,
                                  int32_t ao, void *stream) {
    mlbm::clear_error();
    if (!dy || !dx || n < 1 || h < 1 || w < 1 || c < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    hipLaunchKernelGGL(k_pool_bwd, dim3(blocks((int64_t)n * 4 * h * w * c)), dim3(256), 0, (hipStream_t)stream, n, h,
                       w, c, (const unsigned short *)dy, dys, dyo, (unsigned short *)dx, dxs, dxo,
                       (const unsigned short *)add, as, ao);
    return check("mlbm_pool_backward");
}

extern "C" int mlbm_upsample_forward(int32_t n, int32_t h, int32_t w, int32_t c, const void *x, int32_t xs,
                                     int32_t xo, void *y, int32_t ys, int32_t yo, void *stream) {
    mlbm::clear_error();
    if (!x || !y || n < 1 || h < 1 || w < 1 || c < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    hipLaunchKernelGGL(k_up_fwd, dim3(blocks((int64_t)n * 4 * h * w * c)), dim3(256), 0, (hipStream_t)stream, n, h, w,
                       c, (const unsigned short *)x, xs, xo, (unsigned short *)y, ys, yo);
    return check("mlbm_upsample_forward");
}

extern "C" int mlbm_upsample_backward(int32_t n, int32_t h, int32_t w, int32_t c, const void *dy, int32_t dys,
                                      int32_t dyo, void *dx, int32_t dxs, int32_t dxo, void *stream) {
    mlbm::clear_error();
    if (!dy || !dx || n < 1 || h < 1 || w < 1 || c < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    hipLaunchKernelGGL(k_up_bwd, dim3(blocks((int64_t)n * h * w * c)), dim3(256), 0, (hipStream_t)stream, n, h, w, c,
                       (const unsigned short *)dy, dys, dyo, (unsigned short *)dx, dxs, dxo);
    return check("mlbm_upsample_backward");
}

extern "C" int64_t mlbm_mse_workspace(int64_t pixels) { return blocks(pixels) * (int64_t)sizeof(double); }

extern "C" int mlbm_masked_mse(int64_t pixels, int32_t c, const float *pred, int32_t pred_stride, const float *target,
                               const float *mask, float inv_count, void *dpred, void *workspace, float *loss,
                               void *stream) {
    mlbm::clear_error();
    if (!pred || !target || !mask || !workspace || !loss || pixels < 1 || c < 1 || pred_stride < c)
        return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const unsigned nb = blocks(pixels);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, pixels, c, pred, pred_stride, target, mask, inv_count,
                       (unsigned short *)dpred, (double *)workspace);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(64), 0, s, (const double *)workspace, (int64_t)nb,
                       (double)inv_count, loss);
    return check("mlbm_masked_mse");
}

extern "C" int mlbm_adam(int64_t m, float *param, const float *grad, float *m1, float *m2, float lr, float beta1,
                         float beta2, float eps, int32_t t, void *stream) {
    mlbm::clear_error();
    if (!param || !grad || !m1 || !m2 || m < 1 || t < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    const float c1 = 1.0f - std::pow(beta1, (float)t), c2 = 1.0f - std::pow(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(blocks(m)), dim3(256), 0, (hipStream_t)stream, m, param, grad, m1, m2, lr, beta1,
                       beta2, eps, c1, c2);
    return check("mlbm_adam");
}
