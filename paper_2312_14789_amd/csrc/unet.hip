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

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

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

// ---- convolution tiles (forward and data gradient) ----------------------------------------
// One workgroup computes a TH x TW pixel tile of one image for BN output
// channels, as an implicit GEMM on v_mfma_f32_32x32x16_bf16: each wave owns
// PM x 32 pixels x PN x 32 channels (PM x PN accumulator tiles, so each
// operand fragment read from LDS feeds PN or PM products).  Per 32-channel
// slice of the input, the tile's input halo ((TH + 2) x (TW + 2) pixels,
// periodic) and the slice of the weights for every tap are staged in LDS with
// 16-byte copies, so each staged input value feeds all taps and every MFMA
// operand is one 16-byte LDS read; the next slice's pieces are loaded into
// registers while the current slice is multiplied.  LDS rows are padded to 40
// halves (80 B) to spread consecutive rows over the banks.  k_conv_tile serves images 8
// pixels wide; 16-wide tiles with more than one input slice go to k_conv_dma
// (the same product, staged by direct global-to-LDS loads), and single-slice
// layers to k_conv_tile_s1.
// Epilogue: bias, ReLU, and optionally a gate (the ReLU gradient of the layer
// whose output gradient this is: zero where that layer's output is <= 0).
constexpr int KC = 32, XP = KC + 8;

// A layer input whose first `split` channels are the nearest 2x upsampling of
// a half-resolution tensor: channel c < split of pixel (y, x) of image n is
// lo[((n * h / 2 + y / 2) * w / 2 + x / 2) * stride + c]; channels from split on
// come from the layer's own input view.  lo = null: no such channels.
struct UpIn {
    const unsigned short *lo;
    int stride, split;
};

// 2 x 2 average pooling of a layer's stored (bf16) output, written by its
// epilogue: pooled pixel (y, x) of channel c at p[(n, y, x) * stride + offset + c]
struct PoolOut {
    unsigned short *p;
    int stride, offset;
};

// Gradient of a nearest 2x upsampling, formed by the epilogue of the product
// that yields the gradient of the upsampled channels (those below split): the
// 2 x 2 sum of each block, zeroed where gate (the half-resolution layer output
// that was upsampled) is not positive, goes to g[(n, y, x) * stride + c]; the
// full-resolution values of those channels are not stored.
struct UpGrad {
    unsigned short *g;
    int stride, split;
    const unsigned short *gate;
};

// Epilogue of one 32 x 32 MFMA result of a forward tile: bias, ReLU, the
// gate (zero where the gate value is not positive) and the store of channel
// col at the lane's 16 pixels pt0 + (q / 4) * 8 + (lane >> 5) * 4 + q % 4 of the
// TW-wide tile at (y0, x0) of image n.  The gate values are all loaded before
// any is used, so their loads overlap.  With po.p set (bf16 output, 16-wide
// tiles), the lane also writes the 2 x 2 averages of its pixels: q, q + 1,
// q + 8 and q + 9 (q = 0, 2, 4, 6) are the corners of one block.
template <int TW, bool GATE = true>
__device__ __forceinline__ void store_tile(const mlbm_conv_desc &d, const f32x16 &acc, int n, int y0, int x0, int pt0,
                                           int col, float bv, int relu, int y_f32, void *__restrict__ y,
                                           const unsigned short *__restrict__ gate, int gate_stride, int gate_offset,
                                           int lane, const PoolOut &po, const UpGrad &ug) {
    if (col >= d.c_store) return;
    const int64_t g0 = ((int64_t)n * d.h + y0) * d.w + x0;
    int off[16];  // pixels from the tile's origin
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int pt = pt0 + (q / 4) * 8 + (lane >> 5) * 4 + (q % 4);
        off[q] = (pt / TW) * d.w + pt % TW;
    }
    float gv[16];
    if (GATE && gate) {
        const unsigned short *gb = gate + g0 * gate_stride + gate_offset + col;
#pragma unroll
        for (int q = 0; q < 16; ++q) gv[q] = bf2f(gb[off[q] * gate_stride]);
    }
    float v[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        v[q] = acc[q] + bv;
        if (relu) v[q] = fmaxf(v[q], 0.0f);
        if (GATE && gate && !(gv[q] > 0.0f)) v[q] = 0.0f;
    }
    if constexpr (TW == 16) {
        if (ug.g && col < ug.split) {  // the same for the whole wave: split is a multiple of 32
            // the same sum order as the upsampling gradient: ((x00 + x01) + x10) + x11
            const int w2 = d.w / 2;
            const int64_t pb = ((int64_t)n * (d.h / 2) + y0 / 2) * w2 + x0 / 2;
            int64_t gi[4];
            float gt[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int pt = pt0 + (k / 2) * 8 + (lane >> 5) * 4 + (k % 2) * 2;
                gi[k] = (pb + (int64_t)(pt / 32) * w2 + (pt % 16) / 2) * ug.stride + col;
                gt[k] = bf2f(ug.gate[gi[k]]);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int q = 2 * k;
                float a = bf2f(f2bf(v[q])) + bf2f(f2bf(v[q + 1]));
                a += bf2f(f2bf(v[q + 8]));
                a += bf2f(f2bf(v[q + 9]));
                ug.g[gi[k]] = gt[k] > 0.0f ? f2bf(a) : (unsigned short)0;
            }
            return;
        }
    }
    const int64_t o0 = g0 * d.y_stride + d.y_offset + col;
    if (y_f32) {
        float *yb = (float *)y + o0;
#pragma unroll
        for (int q = 0; q < 16; ++q) yb[off[q] * d.y_stride] = v[q];
    } else {
        unsigned short *yb = (unsigned short *)y + o0;
#pragma unroll
        for (int q = 0; q < 16; ++q) yb[off[q] * d.y_stride] = f2bf(v[q]);
        if constexpr (TW == 16) {
            if (po.p) {
                // the same sum order as the pooling layer: (x00 + x01) + x10, then + x11
                const int w2 = d.w / 2;
                const int64_t pb = ((int64_t)n * (d.h / 2) + y0 / 2) * w2 + x0 / 2;
#pragma unroll
                for (int q = 0; q < 8; q += 2) {
                    const int pt = pt0 + (q / 4) * 8 + (lane >> 5) * 4 + (q % 4);
                    float a = bf2f(f2bf(v[q])) + bf2f(f2bf(v[q + 1]));
                    a += bf2f(f2bf(v[q + 8]));
                    a = 0.25f * (a + bf2f(f2bf(v[q + 9])));
                    po.p[(pb + (int64_t)(pt / 32) * w2 + (pt % 16) / 2) * po.stride + po.offset + col] = f2bf(a);
                }
            }
        }
    }
}

template <int TH, int TW, int BN, int PM, int PN>
constexpr int conv_threads() { return 64 * (TH * TW / (32 * PM)) * (BN / (32 * PN)); }

template <int TH, int TW, int BN, int KS, int PM = 1, int PN = 1>
__global__ void __launch_bounds__((conv_threads<TH, TW, BN, PM, PN>()))
    k_conv_tile(const mlbm_conv_desc d, const unsigned short *__restrict__ x, const unsigned short *__restrict__ w,
                const float *__restrict__ bias, void *__restrict__ y, int relu, int y_f32,
                const unsigned short *__restrict__ gate, int gate_stride, int gate_offset, const PoolOut po,
                const UpIn up, const UpGrad ug) {
    constexpr int BM = TH * TW, HH = TH + 2, HWD = TW + 2, WPX = BM / (32 * PM);
    constexpr int NT = conv_threads<TH, TW, BN, PM, PN>();
    static_assert(BM % (32 * PM) == 0 && BN % (32 * PN) == 0, "wave tiles must divide the block");
    __shared__ __align__(16) unsigned short xs[HH * HWD * XP];
    __shared__ __align__(16) unsigned short wsm[KS * KS * BN * XP];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wp = wave % WPX, wc = wave / WPX;
    const int tiles_x = d.w / TW, tiles_img = tiles_x * (d.h / TH);
    const int n = blockIdx.x / tiles_img, rem = blockIdx.x % tiles_img;
    const int y0 = (rem / tiles_x) * TH, x0 = (rem % tiles_x) * TW;
    const int co0 = blockIdx.y * BN;
    constexpr int ks = KS, r = KS >> 1, taps = KS * KS;
    const int row = lane & 31, kh = (lane >> 5) * 8;
    // LDS offsets of this lane's A rows (pixels) at tap offset (0, 0) and B rows (channels)
    int aoff[PM], boff[PN];
#pragma unroll
    for (int pm = 0; pm < PM; ++pm) {
        const int pb = (wp * PM + pm) * 32 + row;
        aoff[pm] = ((pb / TW + 1) * HWD + (pb % TW + 1)) * XP + kh;
    }
#pragma unroll
    for (int pn = 0; pn < PN; ++pn) boff[pn] = ((wc * PN + pn) * 32 + row) * XP + kh;
    f32x16 acc[PM][PN];
#pragma unroll
    for (int pm = 0; pm < PM; ++pm)
#pragma unroll
        for (int pn = 0; pn < PN; ++pn) acc[pm][pn] = f32x16{};
    // This thread's share of a slice's staging: global offsets (without the
    // slice's first channel c0) and LDS destinations of its 16-byte pieces of
    // the halo and of the weights of every tap.  Threads past the last piece
    // repeat it (the same bytes to the same place), so loads and stores need no
    // branches: a load under a branch waits for every load before it.
    constexpr int XN = HH * HWD * 4, XR = (XN + NT - 1) / NT, WN = taps * BN * 4, WR = (WN + NT - 1) / NT;
    // (xl: the same pieces in the half-resolution part of the input, if any)
    int64_t xo[XR], xl[XR], wo[WR];
    int xd[XR], wd[WR];
#pragma unroll
    for (int j = 0; j < XR; ++j) {
        const int it = min((int)threadIdx.x + j * NT, XN - 1);
        const int hp = it >> 2, q = it & 3;
        const int hy = hp / HWD, hx = hp - hy * HWD;
        int gy = y0 + hy - 1, gx = x0 + hx - 1;
        gy += gy < 0 ? d.h : 0;
        gy -= gy >= d.h ? d.h : 0;
        gx += gx < 0 ? d.w : 0;
        gx -= gx >= d.w ? d.w : 0;
        const int64_t gp = ((int64_t)n * d.h + gy) * d.w + gx;
        xo[j] = gp * d.x_stride + d.x_offset + 8 * q;
        xl[j] = (((int64_t)n * (d.h / 2) + gy / 2) * (d.w / 2) + gx / 2) * up.stride + 8 * q;
        xd[j] = hp * XP + 8 * q;
    }
#pragma unroll
    for (int j = 0; j < WR; ++j) {
        const int it = min((int)threadIdx.x + j * NT, WN - 1);
        const int q = it & 3, rest = it >> 2;
        const int t = rest % taps, co = rest / taps;
        wo[j] = ((int64_t)(co0 + co) * taps + t) * d.c_in + 8 * q;
        wd[j] = (t * BN + co) * XP + 8 * q;
    }
    // the next slice is read into registers while the current one is multiplied
    u4 xr[XR], wr[WR];
    auto fetch = [&](int c0) __attribute__((always_inline)) {
        if (c0 < up.split) {
#pragma unroll
            for (int j = 0; j < XR; ++j) xr[j] = *(const u4 *)(up.lo + xl[j] + c0);
        } else {
#pragma unroll
            for (int j = 0; j < XR; ++j) xr[j] = *(const u4 *)(x + xo[j] + c0);
        }
#pragma unroll
        for (int j = 0; j < WR; ++j) wr[j] = *(const u4 *)(w + wo[j] + c0);
    };
    fetch(0);
    for (int c0 = 0; c0 < d.c_in; c0 += KC) {
        __syncthreads();  // the previous slice's products are done with the LDS
#pragma unroll
        for (int j = 0; j < XR; ++j) *(u4 *)&xs[xd[j]] = xr[j];
#pragma unroll
        for (int j = 0; j < WR; ++j) *(u4 *)&wsm[wd[j]] = wr[j];
        __syncthreads();
        if (c0 + KC < d.c_in) fetch(c0 + KC);
#pragma unroll
        for (int t = 0; t < taps; ++t) {
            const int toff = ((t / ks - r) * HWD + (t % ks - r)) * XP;
            const unsigned short *wt = &wsm[t * BN * XP];
#pragma unroll
            for (int kk = 0; kk < KC; kk += 16) {
                bf16x8 a[PM], b[PN];
#pragma unroll
                for (int pm = 0; pm < PM; ++pm) a[pm] = load_bf8(&xs[aoff[pm] + toff + kk]);
#pragma unroll
                for (int pn = 0; pn < PN; ++pn) b[pn] = load_bf8(wt + boff[pn] + kk);
#pragma unroll
                for (int pm = 0; pm < PM; ++pm)
#pragma unroll
                    for (int pn = 0; pn < PN; ++pn)
                        acc[pm][pn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[pm], b[pn], acc[pm][pn], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int pn = 0; pn < PN; ++pn) {
        const int col = co0 + (wc * PN + pn) * 32 + row;
        const float bv = bias && col < d.c_store ? bias[col] : 0.0f;
#pragma unroll
        for (int pm = 0; pm < PM; ++pm)
            store_tile<TW>(d, acc[pm][pn], n, y0, x0, (wp * PM + pm) * 32, col, bv, relu, y_f32, y, gate, gate_stride,
                           gate_offset, lane, po, ug);
    }
}

// The forward product of k_conv_tile with each slice staged by direct global
// to LDS loads (16 bytes per lane, written at consecutive LDS slots of the
// issuing wave): no staging registers and no LDS stores, so more waves fit.
// Rows are 64 bytes (one pixel's or one output channel's 32 halves), and a
// lane loads the global chunk that belongs at its slot.  A 16-byte LDS read
// serves 16 lanes per cycle from 64 four-byte banks, the lanes grouped by bit
// 5 of the lane index and the parity of bits 2 - 4; the chunk permutations
// below give every such group 16 distinct bank quads.  Weight row r (32
// consecutive rows per wave) holds chunk c at c ^ ((r >> 2) & 3); halo pixel
// hp in halo row hy holds it at c ^ ((hy + 2 (hp >> 2)) & 3), which keeps the
// operand reads of every tap free of conflicts for 16-pixel-wide tiles
// (18-pixel halo rows).
__device__ __forceinline__ int dma_pos(int r, int c) { return r * KC + 8 * (c ^ ((r >> 2) & 3)); }
__device__ __forceinline__ int halo_pos(int hp, int hy, int c) { return hp * KC + 8 * (c ^ ((hy + 2 * (hp >> 2)) & 3)); }

template <int TH, int TW, int BN, int KS>
__global__ void __launch_bounds__((conv_threads<TH, TW, BN, 1, 1>()))
    k_conv_dma(const mlbm_conv_desc d, const unsigned short *__restrict__ x, const unsigned short *__restrict__ w,
               const float *__restrict__ bias, void *__restrict__ y, int relu, int y_f32,
               const unsigned short *__restrict__ gate, int gate_stride, int gate_offset, const PoolOut po,
               const UpIn up, const UpGrad ug) {
    constexpr int BM = TH * TW, HH = TH + 2, HWD = TW + 2, WPX = BM / 32, NT = conv_threads<TH, TW, BN, 1, 1>();
    constexpr int NW = NT / 64, taps = KS * KS, r = KS >> 1;
    // slots (16 bytes each): the halo rounded up to whole waves, then the weights
    constexpr int XN = HH * HWD * 4, XS = (XN + 63) / 64 * 64, WN = taps * BN * 4;
    static_assert(WN % 64 == 0, "weight slots fill whole waves");
    __shared__ __align__(16) unsigned short lds[(XS + WN) * 8];
    unsigned short *xs = lds, *wsm = lds + XS * 8;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int wp = wave % WPX, wc = wave / WPX;
    const int tiles_x = d.w / TW, tiles_img = tiles_x * (d.h / TH);
    const int n = blockIdx.x / tiles_img, rem = blockIdx.x % tiles_img;
    const int y0 = (rem / tiles_x) * TH, x0 = (rem % tiles_x) * TW;
    const int co0 = blockIdx.y * BN;
    const int row = lane & 31, kc = lane >> 5;
    const int pb = wp * 32 + row;
    const int ay = pb / TW + 1, arow = ay * HWD + (pb % TW + 1), brow = wc * 32 + row;
    // this lane's global offsets (without the slice's first channel) for each of
    // its wave's halo and weight instructions
    constexpr int XI = (XS / 64 + NW - 1) / NW, WI = (WN / 64 + NW - 1) / NW;
    int64_t xo[XI], xl[XI], wo[WI];
#pragma unroll
    for (int i = 0; i < XI; ++i) {
        const int slot = min((i * NW + wave) * 64 + lane, XN - 1);  // slots past the halo repeat its last piece
        const int hp = slot >> 2, hy = hp / HWD, hx = hp - hy * HWD;
        const int c = (slot & 3) ^ ((hy + 2 * (hp >> 2)) & 3);
        int gy = y0 + hy - 1, gx = x0 + hx - 1;
        gy += gy < 0 ? d.h : 0;
        gy -= gy >= d.h ? d.h : 0;
        gx += gx < 0 ? d.w : 0;
        gx -= gx >= d.w ? d.w : 0;
        xo[i] = (((int64_t)n * d.h + gy) * d.w + gx) * d.x_stride + d.x_offset + 8 * c;
        xl[i] = (((int64_t)n * (d.h / 2) + gy / 2) * (d.w / 2) + gx / 2) * up.stride + 8 * c;
    }
#pragma unroll
    for (int i = 0; i < WI; ++i) {
        const int slot = min((i * NW + wave) * 64 + lane, WN - 1);
        const int wr = slot >> 2, c = (slot & 3) ^ ((wr >> 2) & 3);
        const int t = wr / BN, co = wr % BN;
        wo[i] = ((int64_t)(co0 + co) * taps + t) * d.c_in + 8 * c;
    }
    f32x16 acc = {};
    for (int c0 = 0; c0 < d.c_in; c0 += KC) {
        __syncthreads();  // the previous slice's products are done with the LDS
        const bool lo = c0 < up.split;
#pragma unroll
        for (int i = 0; i < XI; ++i) {
            const int base = (i * NW + wave) * 64;
            if (base < XS) {
                const unsigned short *src = lo ? up.lo + xl[i] + c0 : x + xo[i] + c0;
                __builtin_amdgcn_global_load_lds((const void *)src, (__attribute__((address_space(3))) void *)(xs + base * 8),
                                                 16, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < WI; ++i) {
            const int base = (i * NW + wave) * 64;
            if (base < WN)
                __builtin_amdgcn_global_load_lds((const void *)(w + wo[i] + c0),
                                                 (__attribute__((address_space(3))) void *)(wsm + base * 8), 16, 0, 0);
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        // product k (tap k / 2, 16-channel half k % 2) is multiplied while the
        // operands of product k + 1 are read; the scheduling barriers keep those
        // reads ahead of the product (left alone, the compiler moves every read to
        // just before its own product and waits for it there)
        bf16x8 ca, cb, na, nb;
        auto operands = [&](int k, bf16x8 &a, bf16x8 &b) __attribute__((always_inline)) {
            const int t = k >> 1, h = k & 1;
            const int ty = ay + t / KS - r, trow = arow + (t / KS - r) * HWD + (t % KS - r), wrow = t * BN + brow;
            a = load_bf8(&xs[halo_pos(trow, ty, kc + 2 * h)]);
            b = load_bf8(&wsm[dma_pos(wrow, kc + 2 * h)]);
        };
        operands(0, ca, cb);
#pragma unroll
        for (int k = 0; k < 2 * taps; ++k) {
            if (k + 1 < 2 * taps) operands(k + 1, na, nb);
            __builtin_amdgcn_sched_barrier(0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ca, cb, acc, 0, 0, 0);
            __builtin_amdgcn_sched_barrier(0);
            ca = na;
            cb = nb;
        }
    }
    const int col = co0 + wc * 32 + row;
    const float bv = bias && col < d.c_store ? bias[col] : 0.0f;
    store_tile<TW>(d, acc, n, y0, x0, wp * 32, col, bv, relu, y_f32, y, gate, gate_stride, gate_offset, lane, po, ug);
}

// Layers with a single 32-channel input slice (c_in = 32): the weights of
// every tap are staged once per workgroup and serve TPW consecutive pixel
// tiles; each tile's input halo is loaded into registers while the previous
// tile is multiplied.  Same tiles, operand layout and epilogue as k_conv_tile;
// only the halo rows are padded (below).
template <int TH, int TW, int BN, int KS, int TPW, bool GATE>
__global__ void __launch_bounds__(64 * (TH * TW / 32) * (BN / 32))
    k_conv_tile_s1(const mlbm_conv_desc d, const unsigned short *__restrict__ x, const unsigned short *__restrict__ w,
                   const float *__restrict__ bias, void *__restrict__ y, int relu, int y_f32,
                   const unsigned short *__restrict__ gate, int gate_stride, int gate_offset, const PoolOut po,
                   const UpGrad ug) {
    constexpr int BM = TH * TW, HH = TH + 2, HWD = TW + 2, WPX = BM / 32, NT = 64 * WPX * (BN / 32);
    constexpr int XN = HH * HWD * 4, XR = (XN + NT - 1) / NT;
    // halo rows of HWD pixels at an 80-byte pitch, each padded by 48 halves:
    // with the 16-lane groups of a 16-byte LDS read (lanes of equal bit 5 and
    // equal parity of bits 2 - 4) no operand read of any tap meets a bank
    // conflict for 16-pixel-wide tiles, and the tap offsets stay constants
    constexpr int XRS = HWD * XP + 48;
    __shared__ __align__(16) unsigned short xs[HH * XRS];
    __shared__ __align__(16) unsigned short wsm[KS * KS * BN * XP];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int wp = wave % WPX, wc = wave / WPX;
    const int tiles_x = d.w / TW, tiles_img = tiles_x * (d.h / TH), n_tiles = d.n * tiles_img;
    const int ta = blockIdx.x * TPW, tb = min(n_tiles, ta + TPW);
    const int co0 = blockIdx.y * BN;
    constexpr int ks = KS, r = KS >> 1, taps = KS * KS;
    const int row = lane & 31, kh = (lane >> 5) * 8;
    const int pb = wp * 32 + row;
    const int aoff = (pb / TW + 1) * XRS + (pb % TW + 1) * XP + kh;
    const int boff = (wc * 32 + row) * XP + kh;
    {
        // every piece loaded before any is stored, so the loads overlap; threads
        // past the last piece repeat it
        constexpr int WN = taps * BN * 4, WR = (WN + NT - 1) / NT;
        u4 wr[WR];
#pragma unroll
        for (int j = 0; j < WR; ++j) {
            const int it = min((int)threadIdx.x + j * NT, WN - 1);
            const int q = it & 3, rest = it >> 2;
            wr[j] = *(const u4 *)(w + ((int64_t)(co0 + rest / taps) * taps + rest % taps) * d.c_in + 8 * q);
        }
#pragma unroll
        for (int j = 0; j < WR; ++j) {
            const int it = min((int)threadIdx.x + j * NT, WN - 1);
            const int q = it & 3, rest = it >> 2;
            *(u4 *)&wsm[((rest % taps) * BN + rest / taps) * XP + 8 * q] = wr[j];
        }
    }
    u4 xr[XR];
    auto fetch = [&](int tile) __attribute__((always_inline)) {
        const int n = tile / tiles_img, rem = tile % tiles_img;
        const int y0 = (rem / tiles_x) * TH, x0 = (rem % tiles_x) * TW;
#pragma unroll
        for (int j = 0; j < XR; ++j) {
            // threads past the last piece repeat it: no branch around the loads
            const int it = min((int)threadIdx.x + j * NT, XN - 1);
            const int hp = it >> 2, q = it & 3;
            const int hy = hp / HWD, hx = hp - hy * HWD;
            int gy = y0 + hy - 1, gx = x0 + hx - 1;
            gy += gy < 0 ? d.h : 0;
            gy -= gy >= d.h ? d.h : 0;
            gx += gx < 0 ? d.w : 0;
            gx -= gx >= d.w ? d.w : 0;
            const int64_t gp = ((int64_t)n * d.h + gy) * d.w + gx;
            xr[j] = *(const u4 *)(x + gp * d.x_stride + d.x_offset + 8 * q);
        }
    };
    if (ta < tb) fetch(ta);
    const int col = co0 + wc * 32 + row;
    const float bv = bias ? bias[col] : 0.0f;
    for (int tile = ta; tile < tb; ++tile) {
        __syncthreads();  // the previous tile's products are done with the halo
#pragma unroll
        for (int j = 0; j < XR; ++j) {
            const int it = min((int)threadIdx.x + j * NT, XN - 1);
            const int hp = it >> 2, hy = hp / HWD;
            *(u4 *)&xs[hy * XRS + (hp - hy * HWD) * XP + 8 * (it & 3)] = xr[j];
        }
        __syncthreads();
        if (tile + 1 < tb) fetch(tile + 1);
        f32x16 acc = {};
#pragma unroll
        for (int t = 0; t < taps; ++t) {
            const int toff = (t / ks - r) * XRS + (t % ks - r) * XP;
            const unsigned short *wt = &wsm[t * BN * XP];
#pragma unroll
            for (int kk = 0; kk < KC; kk += 16)
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_bf8(&xs[aoff + toff + kk]), load_bf8(wt + boff + kk),
                                                              acc, 0, 0, 0);
        }
        const int n = tile / tiles_img, rem = tile % tiles_img;
        store_tile<TW, GATE>(d, acc, n, (rem / tiles_x) * TH, (rem % tiles_x) * TW, wp * 32, col, bv, relu, y_f32, y, gate,
                       gate_stride, gate_offset, lane, po, ug);
    }
}

// ---- weight gradient -------------------------------------------------------------------------
// dw[o][tap][i] = sum_p dy[p, o] x[p + tap, i]: an MFMA product whose summed
// index is the pixel, so both operands need 8 consecutive pixels of one
// channel per lane.  One workgroup takes BCO output x 32 input channels and
// every tap, over a range of TH x TW pixel tiles.  Wave (co group h, tap row j)
// sums the KS taps of its row for CB blocks of 32 output channels, so each
// output-gradient fragment feeds KS products.  Split k's partials go to
// ws + k * row_stride as [c_out][taps][c_in], its bias sums to
// wsb + k * row_stride.

// The weight gradient without transposes: the output-gradient tile and the
// input halo are staged in their natural pixel-major layout by direct
// global-to-LDS loads, and the MFMA operands (8 consecutive pixels of one
// channel per lane) are read with gfx950's transposing LDS read
// (ds_read_b64_tr_b16): within each group of 16 lanes, lane i receives, as its
// element j, half i % 4 of the 8 bytes that lane 4 j + i / 4 addressed.  So
// lane 4 j + q of a group reads pixel P + j, channels C + 4 q .. C + 4 q + 3,
// and lane 4 q + h gets pixels P .. P + 3 of channel C + 4 q + h; two such
// reads give the 8 pixels of an operand.  The tap column is a pixel offset
// into the natural halo, so no shifted copies are needed.  A transposing read
// serves 32 consecutive lanes per cycle from 64 four-byte banks: 4 pixels x 4
// chunks x 2 eight-byte halves.  16-byte chunks of an LDS row (one pixel p)
// are permuted as c -> c ^ s(p), s(p) = p % 4 for rows of 4 chunks, 2 p % 8
// for rows of 8 and 4 (p % 4) for rows of 16, so those 32 words fall on
// distinct banks.  The bias gradient
// comes from the same operand fragments,
// multiplied by a column of ones.
typedef short v4i16 __attribute__((ext_vector_type(4)));

template <int NCH>
__device__ __forceinline__ int tr_swz(int row) { return NCH >= 16 ? 4 * (row & 3) : (NCH >= 8 ? 2 * row : row) % NCH; }
template <int NCH>
__device__ __forceinline__ int tr_pos(int row, int c) { return (row * NCH + (c ^ tr_swz<NCH>(row))) * 8; }

// bf16x8 operand: pixels rbase + 0..7 (rows of an LDS buffer of NCH 16-byte
// chunks per row), channel block cb (16 lanes: channels cb .. cb + 15)
template <int NCH>
__device__ __forceinline__ bf16x8 tr_operand(const unsigned short *buf, int rbase, int cbase, int lane) {
    const int s = lane & 15, rr = rbase + (s >> 2), ch = cbase + 4 * (s & 3);
    typedef __attribute__((address_space(3))) v4i16 lds_v4;
    const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4 *)(buf + tr_pos<NCH>(rr, ch >> 3) + (ch & 7)));
    const v4i16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4 *)(buf + tr_pos<NCH>(rr + 4, ch >> 3) + (ch & 7)));
    typedef short v8i16 __attribute__((ext_vector_type(8)));
    const v8i16 v = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
    return __builtin_bit_cast(bf16x8, v);
}

template <int TH, int TW, int BCO, int KS, int CB = 1>
__global__ void __launch_bounds__(64 * (BCO / (32 * CB)) * KS)
    k_wgrad_tr(const mlbm_conv_desc d, const unsigned short *__restrict__ x, const unsigned short *__restrict__ dy,
               float *__restrict__ ws, float *__restrict__ wsb, int64_t row_stride, int tiles_per_split, const UpIn up) {
    constexpr int BM = TH * TW, HH = TH + 2, HWD = TW + 2, NT = 64 * (BCO / (32 * CB)) * KS, NW = NT / 64;
    constexpr int DCH = BCO / 8, XCH = 4;                        // 16-byte chunks per LDS row
    constexpr int DN = BM * DCH, XN = HH * HWD * XCH, XS = (XN + 63) / 64 * 64;
    static_assert(DN % 64 == 0 && BCO % (32 * CB) == 0, "whole waves of slots, wave groups divide the block");
    static_assert(TW % 8 == 0, "8 consecutive pixels of an operand lie in one tile row");
    __shared__ __align__(16) unsigned short lds[(DN + XS) * 8];
    unsigned short *dyN = lds, *xN = lds + DN * 8;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    const int ch = wave / KS, trow = wave % KS;
    const int co0 = blockIdx.x * BCO, ci0 = blockIdx.y * 32, split = blockIdx.z;
    const int r = KS >> 1, taps = KS * KS;
    const int tiles_x = d.w / TW, tiles_img = tiles_x * (d.h / TH);
    const int n_tiles = d.n * tiles_img;
    const int ta = split * tiles_per_split, tb = min(n_tiles, ta + tiles_per_split);
    const int kh = (lane >> 5) * 8, cl = (lane & 16);  // this lane's first pixel and 16-channel half of its block
    f32x16 acc[CB][KS], accb[CB];
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
        accb[cb] = f32x16{};
#pragma unroll
        for (int s = 0; s < KS; ++s) acc[cb][s] = f32x16{};
    }
    // the bias gradient: waves of tap row 0 in the first input-channel block's workgroups
    const bool bias_sum = wsb && blockIdx.y == 0 && trow == 0;
    typedef short v8i16 __attribute__((ext_vector_type(8)));
    const v8i16 ones8 = {0x3f80, 0x3f80, 0x3f80, 0x3f80, 0x3f80, 0x3f80, 0x3f80, 0x3f80};  // bf16 1.0
    const bf16x8 ones = __builtin_bit_cast(bf16x8, ones8);
    constexpr int DI = (DN / 64 + NW - 1) / NW, XI = (XS / 64 + NW - 1) / NW;
    for (int tile = ta; tile < tb; ++tile) {
        const int n = tile / tiles_img, rem = tile % tiles_img;
        const int y0 = (rem / tiles_x) * TH, x0 = (rem % tiles_x) * TW;
        __syncthreads();  // the previous tile's products are done with the LDS
#pragma unroll
        for (int i = 0; i < DI; ++i) {
            const int base = (i * NW + wave) * 64;
            if (base < DN) {
                const int slot = base + lane, p = slot / DCH, c = (slot % DCH) ^ tr_swz<DCH>(p);
                const int64_t gp = ((int64_t)n * d.h + y0 + p / TW) * d.w + x0 + p % TW;
                __builtin_amdgcn_global_load_lds((const void *)(dy + gp * d.y_stride + d.y_offset + co0 + 8 * c),
                                                 (__attribute__((address_space(3))) void *)(dyN + base * 8), 16, 0, 0);
            }
        }
#pragma unroll
        for (int i = 0; i < XI; ++i) {
            const int base = (i * NW + wave) * 64;
            if (base < XS) {
                const int slot = min(base + lane, XN - 1);  // slots past the halo repeat its last piece
                const int hp = slot / XCH, c = (slot % XCH) ^ tr_swz<XCH>(hp);
                const int hy = hp / HWD, hx = hp - hy * HWD;
                int gy = y0 + hy - 1, gx = x0 + hx - 1;
                gy += gy < 0 ? d.h : 0;
                gy -= gy >= d.h ? d.h : 0;
                gx += gx < 0 ? d.w : 0;
                gx -= gx >= d.w ? d.w : 0;
                const unsigned short *src;
                if (ci0 < up.split)
                    src = up.lo + (((int64_t)n * (d.h / 2) + gy / 2) * (d.w / 2) + gx / 2) * up.stride + ci0 + 8 * c;
                else
                    src = x + (((int64_t)n * d.h + gy) * d.w + gx) * d.x_stride + d.x_offset + ci0 + 8 * c;
                __builtin_amdgcn_global_load_lds((const void *)src,
                                                 (__attribute__((address_space(3))) void *)(xN + base * 8), 16, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        const int oy = trow - r;
        if constexpr (BCO == 32 && CB == 1 && TW == 16) {
            // one output block per wave and registers to spare: each product's
            // operands are read while the previous product runs (the scheduling
            // barriers keep the compiler from moving the reads down to their use)
            auto opa = [&](int kb) __attribute__((always_inline)) {
                return tr_operand<DCH>(dyN, kb * 16 + kh, ch * 32 + cl, lane);
            };
            auto opb = [&](int kb, int s) __attribute__((always_inline)) {
                const int p0 = kb * 16 + kh;
                return tr_operand<XCH>(xN, (p0 / TW + 1 + oy) * HWD + p0 % TW + s + 1 - r, cl, lane);
            };
            bf16x8 a0 = opa(0), b0 = opb(0, 0), a1 = a0, b1 = b0;
#pragma unroll
            for (int kb = 0; kb < BM / 16; ++kb) {
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    if (s + 1 < KS) b1 = opb(kb, s + 1);
                    else if (kb + 1 < BM / 16) {
                        a1 = opa(kb + 1);
                        b1 = opb(kb + 1, 0);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    if (s == 0 && bias_sum) accb[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, ones, accb[0], 0, 0, 0);
                    acc[0][s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc[0][s], 0, 0, 0);
                    __builtin_amdgcn_sched_barrier(0);
                    b0 = b1;
                    if (s + 1 == KS) a0 = a1;
                }
            }
        } else {
#pragma unroll
            for (int kb = 0; kb < BM / 16; ++kb) {
                const int p0 = kb * 16 + kh, ty = p0 / TW, tx = p0 % TW;
                bf16x8 a[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) a[cb] = tr_operand<DCH>(dyN, p0, (ch * CB + cb) * 32 + cl, lane);
                if (bias_sum) {
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        accb[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[cb], ones, accb[cb], 0, 0, 0);
                }
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    const int hx = tx + s + 1 - r;  // halo column of the tap's first pixel
                    const bf16x8 b = tr_operand<XCH>(xN, (ty + 1 + oy) * HWD + hx, cl, lane);
#pragma unroll
                    for (int cb = 0; cb < CB; ++cb)
                        acc[cb][s] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[cb], b, acc[cb][s], 0, 0, 0);
                }
            }
        }
    }
    // bias: column 0 of the product with ones holds every row's sum (lanes 0 and 32)
    if (bias_sum && (lane & 31) == 0) {
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
#pragma unroll
            for (int q = 0; q < 16; ++q)
                wsb[split * row_stride + co0 + (ch * CB + cb) * 32 + (q / 4) * 8 + (lane >> 5) * 4 + (q % 4)] = accb[cb][q];
    }
    const int ci = ci0 + (lane & 31);
#pragma unroll
    for (int cb = 0; cb < CB; ++cb) {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int t = trow * KS + s;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const int co = co0 + (ch * CB + cb) * 32 + (q / 4) * 8 + (lane >> 5) * 4 + (q % 4);
                ws[split * row_stride + ((int64_t)co * taps + t) * d.c_in + ci] = acc[cb][s][q];
            }
        }
    }
}

// sum of the split partials (split k's m values at ws + k * stride): G lanes
// per element, lane group g sums splits g, g + G, ..., then the G sums are
// added in a fixed tree order (deterministic)
template <int G>
__global__ void __launch_bounds__(64 * G) k_sum_splits_g(const float *__restrict__ ws, int splits, int64_t m,
                                                        int64_t stride, float *__restrict__ dw) {
    __shared__ float part[G][64];
    const int e = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + e;
    float s = 0.0f;
    if (i < m) {
#pragma unroll 8
        for (int k = g; k < splits; k += G) s += ws[(int64_t)k * stride + i];
    }
    part[g][e] = s;
    __syncthreads();
#pragma unroll
    for (int h = G / 2; h > 0; h >>= 1) {
        if (g < h) part[g][e] += part[g + h][e];
        __syncthreads();
    }
    if (g == 0 && i < m) dw[i] = part[0][e];
}

void sum_splits(const float *ws, int splits, int64_t m, int64_t stride, float *dw, hipStream_t s) {
    const dim3 grid((unsigned)((m + 63) / 64));
    if (splits >= 64) hipLaunchKernelGGL(k_sum_splits_g<16>, grid, dim3(1024), 0, s, ws, splits, m, stride, dw);
    else if (splits >= 8) hipLaunchKernelGGL(k_sum_splits_g<4>, grid, dim3(256), 0, s, ws, splits, m, stride, dw);
    else hipLaunchKernelGGL(k_sum_splits_g<1>, grid, dim3(64), 0, s, ws, splits, m, stride, dw);
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

// every layer's conversion in one launch: layer j covers elements [start[j], start[j + 1])
constexpr int MAX_WJOBS = 4 * MLBM_UNET_MAX_LEVELS;
struct WeightJobs {
    int n;
    int64_t start[MAX_WJOBS + 1];
    int64_t w_off[MAX_WJOBS], wf_off[MAX_WJOBS], wd_off[MAX_WJOBS];
    int c_out[MAX_WJOBS], taps[MAX_WJOBS], c_in[MAX_WJOBS];
};

__global__ void k_weights_all(const float *__restrict__ params, unsigned short *__restrict__ wbf, const WeightJobs jb) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= jb.start[jb.n]) return;
    int j = 0;
    while (i >= jb.start[j + 1]) ++j;
    const int k = (int)(i - jb.start[j]), c_in = jb.c_in[j], taps = jb.taps[j];
    const int ci = k % c_in, t = (k / c_in) % taps, co = k / (c_in * taps);
    const unsigned short v = f2bf(params[jb.w_off[j] + k]);
    wbf[jb.wf_off[j] + k] = v;
    wbf[jb.wd_off[j] + ((int64_t)ci * taps + (taps - 1 - t)) * jb.c_out[j] + co] = v;
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

// ---- the same layers on 8 channels per thread (16-byte loads and stores) -----------------
// Used when the channel count, strides and offsets are multiples of 8.
__device__ __forceinline__ void unpack8(u4 v, float f[8]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[2 * k] = __uint_as_float(v[k] << 16);
        f[2 * k + 1] = __uint_as_float(v[k] & 0xffff0000u);
    }
}
__device__ __forceinline__ u4 pack8(const float f[8]) {
    u4 v;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (unsigned)f2bf(f[2 * k]) | ((unsigned)f2bf(f[2 * k + 1]) << 16);
    return v;
}

__global__ void k_relu_bwd_v8(int64_t P, int C8, const unsigned short *y, int y_stride, int y_offset,
                              unsigned short *dy, int dy_stride, int dy_offset) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= P * C8) return;
    const int64_t p = i / C8;
    const int c = (int)(i - p * C8) * 8;
    const u4 yv = *(const u4 *)(y + p * y_stride + y_offset + c);
    u4 *dp = (u4 *)(dy + p * dy_stride + dy_offset + c);
    u4 g = *dp;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const unsigned keep_lo = __uint_as_float(yv[k] << 16) > 0.0f ? 0x0000ffffu : 0u;
        const unsigned keep_hi = __uint_as_float(yv[k] & 0xffff0000u) > 0.0f ? 0xffff0000u : 0u;
        g[k] &= keep_lo | keep_hi;
    }
    *dp = g;
}

// 8 bf16 gradients zeroed where the layer's output (8 bf16 values) is not positive
__device__ __forceinline__ u4 relu_gate8(u4 g, const u4 yv) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const unsigned keep_lo = __uint_as_float(yv[k] << 16) > 0.0f ? 0x0000ffffu : 0u;
        const unsigned keep_hi = __uint_as_float(yv[k] & 0xffff0000u) > 0.0f ? 0xffff0000u : 0u;
        g[k] &= keep_lo | keep_hi;
    }
    return g;
}

__global__ void k_pool_fwd_v8(int n, int h, int w, int C8, const unsigned short *x, int xs, int xo, unsigned short *y,
                              int ys, int yo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)n * h * w * C8;
    if (i >= tot) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int xx = (int)(q % w), yy = (int)((q / w) % h);
    const int64_t nn = q / ((int64_t)w * h);
    const int W2 = 2 * w;
    const int64_t b = (nn * 2 * h + 2 * yy) * W2 + 2 * xx;
    float a[8], t[8];
    unpack8(*(const u4 *)(x + b * xs + xo + c), a);
    unpack8(*(const u4 *)(x + (b + 1) * xs + xo + c), t);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += t[k];
    unpack8(*(const u4 *)(x + (b + W2) * xs + xo + c), t);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += t[k];
    unpack8(*(const u4 *)(x + (b + W2 + 1) * xs + xo + c), t);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = 0.25f * (a[k] + t[k]);
    *(u4 *)(y + q * ys + yo + c) = pack8(a);
}

__global__ void k_pool_bwd_v8(int n, int h, int w, int C8, const unsigned short *dy, int dys, int dyo, unsigned short *dx,
                              int dxs, int dxo, const unsigned short *add, int as, int ao, const unsigned short *gate,
                              int gs, int go) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)n * 4 * h * w * C8;
    if (i >= tot) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int W2 = 2 * w;
    const int xx = (int)(q % W2), yy = (int)((q / W2) % (2 * h));
    const int64_t nn = q / ((int64_t)W2 * 2 * h);
    const int64_t src = (nn * h + yy / 2) * w + xx / 2;
    float v[8], a[8];
    const u4 dv = *(const u4 *)(dy + src * dys + dyo + c);
    const u4 av = add ? *(const u4 *)(add + q * as + ao + c) : u4{0u, 0u, 0u, 0u};
    const u4 gv = gate ? *(const u4 *)(gate + q * gs + go + c) : u4{0u, 0u, 0u, 0u};
    unpack8(dv, v);
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] *= 0.25f;
    if (add) {
        unpack8(av, a);
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] += a[k];
    }
    u4 r = pack8(v);
    if (gate) r = relu_gate8(r, gv);
    *(u4 *)(dx + q * dxs + dxo + c) = r;
}

__global__ void k_up_fwd_v8(int n, int h, int w, int C8, const unsigned short *x, int xs, int xo, unsigned short *y,
                            int ys, int yo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)n * 4 * h * w * C8;
    if (i >= tot) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int W2 = 2 * w;
    const int xx = (int)(q % W2), yy = (int)((q / W2) % (2 * h));
    const int64_t nn = q / ((int64_t)W2 * 2 * h);
    const int64_t src = (nn * h + yy / 2) * w + xx / 2;
    *(u4 *)(y + q * ys + yo + c) = *(const u4 *)(x + src * xs + xo + c);
}

__global__ void k_up_bwd_v8(int n, int h, int w, int C8, const unsigned short *dy, int dys, int dyo, unsigned short *dx,
                            int dxs, int dxo, const unsigned short *gate, int gs, int go) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = (int64_t)n * h * w * C8;
    if (i >= tot) return;
    const int c = (int)(i % C8) * 8;
    const int64_t q = i / C8;
    const int xx = (int)(q % w), yy = (int)((q / w) % h);
    const int64_t nn = q / ((int64_t)w * h);
    const int W2 = 2 * w;
    const int64_t b = (nn * 2 * h + 2 * yy) * W2 + 2 * xx;
    float a[8], t[8];
    unpack8(*(const u4 *)(dy + b * dys + dyo + c), a);
    unpack8(*(const u4 *)(dy + (b + 1) * dys + dyo + c), t);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += t[k];
    unpack8(*(const u4 *)(dy + (b + W2) * dys + dyo + c), t);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += t[k];
    unpack8(*(const u4 *)(dy + (b + W2 + 1) * dys + dyo + c), t);
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] += t[k];
    u4 r = pack8(a);
    if (gate) r = relu_gate8(r, *(const u4 *)(gate + q * gs + go + c));
    *(u4 *)(dx + q * dxs + dxo + c) = r;
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
        if ((int)threadIdx.x < o) s1[threadIdx.x] += s1[threadIdx.x + o];
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

// masked MSE with the normalisation 1 / (C sum mask) read from the device;
// pred FP32 [P][pred_stride], dpred bf16 [P][ps] (ps a multiple of 8, zero past C)
__global__ void __launch_bounds__(256) k_mse_dev(int64_t P, int C, const float *pred, int pred_stride, int ps,
                                                const float *target,
                                                const float *mask, const float *inv_count, unsigned short *dpred,
                                                double *partial) {
    __shared__ double s1[256];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float ic = *inv_count;
    double e = 0.0;
    if (p < P) {
        const float m = mask[p];
        for (int c8 = 0; c8 < ps; c8 += 8) {
            unsigned w[4] = {0u, 0u, 0u, 0u};
            if (c8 < C) {
                // all 8 loads issued before use (past C: the last channel again, weighted 0)
                float pv[8], tv[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int c = min(c8 + j, C - 1);
                    pv[j] = pred[p * pred_stride + c];
                    tv[j] = target[p * C + c];
                }
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    if (c8 + j >= C) break;
                    const float d = (pv[j] - tv[j]) * m;
                    e += (double)d * d;
                    w[j >> 1] |= (unsigned)f2bf(2.0f * d * ic) << (16 * (j & 1));
                }
            }
            *(u4 *)(dpred + p * ps + c8) = u4{w[0], w[1], w[2], w[3]};
        }
    }
    s1[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s1[threadIdx.x] += s1[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s1[0];
}

// per-block sums of the mask (fixed order)
__global__ void __launch_bounds__(256) k_mask_partial(int64_t P, const float *mask, double *partial) {
    __shared__ double s1[256];
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    s1[threadIdx.x] = p < P ? (double)mask[p] : 0.0;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s1[threadIdx.x] += s1[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s1[0];
}

// sum of m partials by one block of 256 threads in a fixed order
__device__ double block_sum_partials(const double *partial, int64_t m) {
    __shared__ double t[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += 256) s += partial[i];
    t[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) t[threadIdx.x] += t[threadIdx.x + o];
        __syncthreads();
    }
    return t[0];
}

// inv = 1 / (C sum of the partials), 1 when the mask is empty
__global__ void __launch_bounds__(256) k_inv_count(const double *partial, int64_t m, int C, float *inv) {
    const double s = block_sum_partials(partial, m);
    if (threadIdx.x == 0) inv[0] = s > 0.0 ? (float)(1.0 / (s * C)) : 1.0f;
}

// loss = inv * sum of the partials
__global__ void __launch_bounds__(256) k_loss_final(const double *partial, int64_t m, const float *inv, float *out) {
    const double s = block_sum_partials(partial, m);
    if (threadIdx.x == 0) out[0] = (float)(s * (double)inv[0]);
}

// zero the gradients of padded channels: enc0a input channels >= c_real_in,
// head rows >= c_real_out (weights and bias)
__global__ void k_mask_pad_grads(float *g_enc0a, int co0, int taps0, int ci0, int c_real_in, float *g_head_w,
                                 float *g_head_b, int co_h, int ci_h, int c_real_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t m0 = (int64_t)co0 * taps0 * ci0, mh = (int64_t)co_h * ci_h;
    if (i < m0) {
        if ((int)(i % ci0) >= c_real_in) g_enc0a[i] = 0.0f;
    } else if (i < m0 + mh) {
        const int64_t j = i - m0;
        if ((int)(j / ci_h) >= c_real_out) g_head_w[j] = 0.0f;
    } else if (i < m0 + mh + co_h) {
        const int64_t j = i - m0 - mh;
        if ((int)j >= c_real_out) g_head_b[j] = 0.0f;
    }
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
    if (d->h % 8 || (d->w != 8 && d->w % 16))
        return fail(MLBM_ERR_ARG, "height must be a multiple of 8, width 8 or a multiple of 16");
    if (d->x_stride % 8 || d->x_offset % 8 || d->y_stride % 8 || d->y_offset % 8)
        return fail(MLBM_ERR_ARG, "strides and offsets must be multiples of 8 channels");
    if (d->x_offset + d->c_in > d->x_stride) return fail(MLBM_ERR_ARG, "input view exceeds its stride");
    if (d->c_store < 1 || d->c_store > d->c_out) return fail(MLBM_ERR_ARG, "c_store outside [1, c_out]");
    return MLBM_OK;
}

}  // namespace

namespace {

void pool_fwd_launch(int n, int h, int w, int c, const unsigned short *x, int xs, int xo, unsigned short *y, int ys,
                     int yo, hipStream_t s);

// tile shape: 8 x 16 pixels, or 8 x 8 for images 8 pixels wide; with pool.p
// set (bf16 output only) the 2 x 2 averages of the stored output are written
// too, by the epilogue of 16-wide tiles or by the pooling layer after 8-wide ones
// up.lo set: the first up.split input channels are upsampled from up.lo (16-wide
// tiles with more than one input slice only)
int conv_launch(const mlbm_conv_desc &d, const void *x, const void *w, const float *bias, void *y, int relu, int y_f32,
                const void *gate, int gate_stride, int gate_offset, hipStream_t s, PoolOut pool = PoolOut{nullptr, 0, 0},
                UpIn up = UpIn{nullptr, 0, 0}, UpGrad ug = UpGrad{nullptr, 0, 0, nullptr}) {
    const auto *xx = (const unsigned short *)x, *ww = (const unsigned short *)w, *gg = (const unsigned short *)gate;
    const PoolOut po = (y_f32 || d.w == 8) ? PoolOut{nullptr, 0, 0} : pool;
    if (up.lo && (d.w == 8 || d.c_in == KC || up.split % KC || up.split > d.c_in))
        return mlbm::fail(MLBM_ERR_ARG, "upsampled input channels need 16-wide tiles and whole 32-channel slices");
    if (ug.g && (d.w == 8 || y_f32 || ug.split % 32 || ug.split > d.c_store))
        return mlbm::fail(MLBM_ERR_ARG, "an upsampling gradient needs 16-wide tiles, bf16 output and 32-channel blocks");
#define MLBM_CONV_K(TH, TW, BN, KS, PM, PN)                                                                         \
    hipLaunchKernelGGL((k_conv_tile<TH, TW, BN, KS, PM, PN>),                                                       \
                       dim3((unsigned)((int64_t)d.n * (d.h / TH) * (d.w / TW)), d.c_out / BN),                     \
                       dim3(conv_threads<TH, TW, BN, PM, PN>()), 0, s, d, xx, ww, bias, y, relu, y_f32, gg,        \
                       gate_stride, gate_offset, po, up, ug)
#define MLBM_CONV(TH, TW, BN, PM, PN)                                                                               \
    do {                                                                                                            \
        if (d.ksize == 3) MLBM_CONV_K(TH, TW, BN, 3, PM, PN);                                                       \
        else MLBM_CONV_K(TH, TW, BN, 1, PM, PN);                                                                    \
    } while (0)
#define MLBM_CONV_S1_G(BN, KS, TPW, G)                                                                              \
    hipLaunchKernelGGL((k_conv_tile_s1<8, 16, BN, KS, TPW, G>), dim3(wgs, d.c_out / BN), dim3(8 * BN), 0, s, d, xx, ww, \
                       bias, y, relu, y_f32, gg, gate_stride, gate_offset, po, ug)
    // (the gate's registers are only allocated where a gate is applied)
#define MLBM_CONV_S1(BN, TPW)                                                                                       \
    do {                                                                                                            \
        if (d.ksize == 3) {                                                                                         \
            if (gg) MLBM_CONV_S1_G(BN, 3, TPW, true);                                                               \
            else MLBM_CONV_S1_G(BN, 3, TPW, false);                                                                 \
        } else {                                                                                                    \
            if (gg) MLBM_CONV_S1_G(BN, 1, TPW, true);                                                               \
            else MLBM_CONV_S1_G(BN, 1, TPW, false);                                                                 \
        }                                                                                                           \
    } while (0)
#define MLBM_DMA(BN)                                                                                                \
    do {                                                                                                            \
        const dim3 g((unsigned)((int64_t)d.n * (d.h / 8) * (d.w / 16)), d.c_out / BN);                               \
        if (d.ksize == 3)                                                                                           \
            hipLaunchKernelGGL((k_conv_dma<8, 16, BN, 3>), g, dim3(8 * BN), 0, s, d, xx, ww, bias, y, relu, y_f32, gg, \
                               gate_stride, gate_offset, po, up, ug);                                              \
        else                                                                                                        \
            hipLaunchKernelGGL((k_conv_dma<8, 16, BN, 1>), g, dim3(8 * BN), 0, s, d, xx, ww, bias, y, relu, y_f32, gg, \
                               gate_stride, gate_offset, po, up, ug);                                              \
    } while (0)
    if (d.c_in == KC && d.w % 16 == 0) {
        // one input slice: weights staged once per workgroup for 4 consecutive tiles
        constexpr int TPW = 4;
        const unsigned wgs = (unsigned)(((int64_t)d.n * (d.h / 8) * (d.w / 16) + TPW - 1) / TPW);
        if (d.c_out % 64 == 0) MLBM_CONV_S1(64, TPW);
        else MLBM_CONV_S1(32, TPW);
    } else if (d.w == 8) {
        if (d.c_out % 64 == 0) MLBM_CONV(8, 8, 64, 1, 1);
        else MLBM_CONV(8, 8, 32, 1, 1);
    } else {
        if (d.c_out % 64 == 0) MLBM_DMA(64);
        else MLBM_DMA(32);
    }
#undef MLBM_CONV_S1
#undef MLBM_CONV_S1_G
#undef MLBM_DMA
#undef MLBM_CONV
#undef MLBM_CONV_K
    if (pool.p && !po.p)
        pool_fwd_launch(d.n, d.h / 2, d.w / 2, d.c_store, (const unsigned short *)y, d.y_stride, d.y_offset, pool.p,
                        pool.stride, pool.offset, s);
    return check("mlbm_conv_forward");
}

int64_t conv_tiles(const mlbm_conv_desc &d) { return (int64_t)d.n * (d.h / 8) * (d.w / (d.w == 8 ? 8 : 16)); }

// tiles per split for `splits` requested splits, and the resulting split count
int wgrad_split(const mlbm_conv_desc &d, int splits, int *per) {
    const int64_t tiles = conv_tiles(d);
    const int64_t sp = std::max<int64_t>(1, std::min<int64_t>(splits, tiles));
    *per = (int)((tiles + sp - 1) / sp);
    return (int)((tiles + *per - 1) / *per);
}

// up.lo set: the first up.split input channels are upsampled from up.lo
int wgrad_launch(const mlbm_conv_desc &d, const void *x, const void *dy, float *dw, float *db, int splits, float *ws,
                 hipStream_t s, UpIn up = UpIn{nullptr, 0, 0}) {
    if (up.lo && (up.split % 32 || up.split > d.c_in))
        return mlbm::fail(MLBM_ERR_ARG, "upsampled input channels must be whole 32-channel blocks");
    int per = 0;
    const int sp = wgrad_split(d, splits, &per);
    const int taps = d.ksize * d.ksize;
    const int64_t m = (int64_t)d.c_out * taps * d.c_in;
    const bool narrow = d.w == 8, wide = d.c_out % 64 == 0;
    const auto *xx = (const unsigned short *)x, *yy = (const unsigned short *)dy;
    // split k's partials: ws[k * row][0, m) weights, [m, m + c_out) bias
    const int64_t row = m + d.c_out;
    float *wsb = db ? ws + m : nullptr;
#define MLBM_WG(TH, TW, BCO, KS, CB)                                                                              \
    hipLaunchKernelGGL((k_wgrad_tr<TH, TW, BCO, KS, CB>), dim3(d.c_out / BCO, d.c_in / 32, sp),                   \
                       dim3(64 * (BCO / (32 * CB)) * KS), 0, s, d, xx, yy, ws, wsb, row, per, up)
    if (d.ksize == 3) {
        if (narrow) {
            if (wide) MLBM_WG(8, 8, 64, 3, 1);
            else MLBM_WG(8, 8, 32, 3, 1);
        } else {
            // 128 (or 64) output channels per workgroup, one 32-channel block per wave
            if (d.c_out % 128 == 0) MLBM_WG(8, 16, 128, 3, 1);
            else if (wide) MLBM_WG(8, 16, 64, 3, 1);
            else MLBM_WG(8, 16, 32, 3, 1);
        }
    } else {
        if (narrow) {
            if (wide) MLBM_WG(8, 8, 64, 1, 1);
            else MLBM_WG(8, 8, 32, 1, 1);
        } else {
            if (wide) MLBM_WG(8, 16, 64, 1, 1);
            else MLBM_WG(8, 16, 32, 1, 1);
        }
    }
#undef MLBM_WG
    int rc = check("mlbm_conv_wgrad");
    if (rc) return rc;
    if (db == dw + m) {
        sum_splits(ws, sp, row, row, dw, s);  // weights and bias in one pass
    } else {
        sum_splits(ws, sp, m, row, dw, s);
        if (db) sum_splits(wsb, sp, d.c_out, row, db, s);
    }
    return check("mlbm_conv_wgrad");
}

int64_t wgrad_workspace(const mlbm_conv_desc &d, int splits) {
    int per = 0;
    const int sp = wgrad_split(d, splits, &per);
    const int64_t m = (int64_t)d.c_out * d.ksize * d.ksize * d.c_in;
    return (m + d.c_out) * sp * (int64_t)sizeof(float);
}

// Pixel splits of a weight gradient: one round of workgroups (as many as the
// GPU holds at once for the configuration wgrad_launch picks, set by the LDS
// each takes) spread over the output blocks, and further whole rounds while a
// workgroup would sweep more than 24 pixel tiles.  One round keeps the split
// partials, which are written and read back once more to be summed, smallest;
// a part of a round leaves some compute units a workgroup more than others.
int wgrad_splits(const mlbm_conv_desc &d) {
    const bool wide = d.c_out % 64 == 0;
    int bco = wide ? 64 : 32, round = 512;
    if (d.ksize == 3 && d.w != 8 && d.c_out % 128 == 0) bco = 128, round = 256;
    else if (d.ksize == 1) round = 1024;
    const int64_t tiles = conv_tiles(d), blocks = (int64_t)(d.c_out / bco) * (d.c_in / 32);
    const int64_t per_round = std::max<int64_t>(1, (round + blocks - 1) / blocks);
    int64_t sp = per_round;
    while ((tiles + sp - 1) / sp > 24 && sp < tiles) sp += per_round;
    return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, sp));
}

// 8-channel paths when every channel count, stride and offset is a multiple of 8
bool v8(int c, int a, int b, int e, int f) { return ((c | a | b | e | f) & 7) == 0; }

void relu_bwd_launch(int64_t P, int C, const unsigned short *y, int ys, int yo, unsigned short *dy, int dys, int dyo,
                     hipStream_t s) {
    if (v8(C, ys, yo, dys, dyo))
        hipLaunchKernelGGL(k_relu_bwd_v8, dim3(blocks(P * (C / 8))), dim3(256), 0, s, P, C / 8, y, ys, yo, dy, dys, dyo);
    else
        hipLaunchKernelGGL(k_relu_bwd, dim3(blocks(P * C)), dim3(256), 0, s, P, C, y, ys, yo, dy, dys, dyo);
}

void pool_fwd_launch(int n, int h, int w, int c, const unsigned short *x, int xs, int xo, unsigned short *y, int ys,
                     int yo, hipStream_t s) {
    if (v8(c, xs, xo, ys, yo))
        hipLaunchKernelGGL(k_pool_fwd_v8, dim3(blocks((int64_t)n * h * w * (c / 8))), dim3(256), 0, s, n, h, w, c / 8, x,
                           xs, xo, y, ys, yo);
    else
        hipLaunchKernelGGL(k_pool_fwd, dim3(blocks((int64_t)n * h * w * c)), dim3(256), 0, s, n, h, w, c, x, xs, xo, y,
                           ys, yo);
}

// gate (optional): the ReLU gradient of the layer whose output dx is, applied to dx
void pool_bwd_launch(int n, int h, int w, int c, const unsigned short *dy, int dys, int dyo, unsigned short *dx, int dxs,
                     int dxo, const unsigned short *add, int as, int ao, hipStream_t s, const unsigned short *gate = nullptr,
                     int gs = 0, int go = 0) {
    if (v8(c, dys, dyo, dxs, dxo) && (!add || v8(as, ao, 0, 0, 0)) && (!gate || v8(gs, go, 0, 0, 0))) {
        hipLaunchKernelGGL(k_pool_bwd_v8, dim3(blocks((int64_t)n * 4 * h * w * (c / 8))), dim3(256), 0, s, n, h, w,
                           c / 8, dy, dys, dyo, dx, dxs, dxo, add, as, ao, gate, gs, go);
    } else {
        hipLaunchKernelGGL(k_pool_bwd, dim3(blocks((int64_t)n * 4 * h * w * c)), dim3(256), 0, s, n, h, w, c, dy, dys,
                           dyo, dx, dxs, dxo, add, as, ao);
        if (gate) relu_bwd_launch((int64_t)n * 4 * h * w, c, gate, gs, go, dx, dxs, dxo, s);
    }
}

void up_fwd_launch(int n, int h, int w, int c, const unsigned short *x, int xs, int xo, unsigned short *y, int ys,
                   int yo, hipStream_t s) {
    if (v8(c, xs, xo, ys, yo))
        hipLaunchKernelGGL(k_up_fwd_v8, dim3(blocks((int64_t)n * 4 * h * w * (c / 8))), dim3(256), 0, s, n, h, w, c / 8,
                           x, xs, xo, y, ys, yo);
    else
        hipLaunchKernelGGL(k_up_fwd, dim3(blocks((int64_t)n * 4 * h * w * c)), dim3(256), 0, s, n, h, w, c, x, xs, xo,
                           y, ys, yo);
}

// gate (optional): the ReLU gradient of the layer whose output dx is, applied to dx
void up_bwd_launch(int n, int h, int w, int c, const unsigned short *dy, int dys, int dyo, unsigned short *dx, int dxs,
                   int dxo, hipStream_t s, const unsigned short *gate = nullptr, int gs = 0, int go = 0) {
    if (v8(c, dys, dyo, dxs, dxo) && (!gate || v8(gs, go, 0, 0, 0))) {
        hipLaunchKernelGGL(k_up_bwd_v8, dim3(blocks((int64_t)n * h * w * (c / 8))), dim3(256), 0, s, n, h, w, c / 8, dy,
                           dys, dyo, dx, dxs, dxo, gate, gs, go);
    } else {
        hipLaunchKernelGGL(k_up_bwd, dim3(blocks((int64_t)n * h * w * c)), dim3(256), 0, s, n, h, w, c, dy, dys, dyo, dx,
                           dxs, dxo);
        if (gate) relu_bwd_launch((int64_t)n * h * w, c, gate, gs, go, dx, dxs, dxo, s);
    }
}

}  // namespace

extern "C" int mlbm_conv_forward(const mlbm_conv_desc *d, const void *x, const void *w, const float *bias, void *y,
                                 int32_t relu, int32_t y_f32, void *stream) {
    mlbm::clear_error();
    int rc = check_desc(d);
    if (rc) return rc;
    if (!x || !w || !y) return mlbm::fail(MLBM_ERR_ARG, "null pointer");
    if (d->y_offset + d->c_store > d->y_stride) return mlbm::fail(MLBM_ERR_ARG, "output view exceeds its stride");
    return conv_launch(*d, x, w, bias, y, relu, y_f32, nullptr, 0, 0, (hipStream_t)stream);
}

extern "C" int64_t mlbm_conv_wgrad_workspace(const mlbm_conv_desc *d, int32_t splits) {
    if (!d || splits < 1 || check_desc(d)) return 0;
    return wgrad_workspace(*d, splits);
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
    return wgrad_launch(*d, x, dy, dw, db, splits, (float *)workspace, (hipStream_t)stream);
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
    relu_bwd_launch(pixels, channels, (const unsigned short *)y, y_stride, y_offset, (unsigned short *)dy, dy_stride,
                    dy_offset, (hipStream_t)stream);
    return check("mlbm_relu_backward");
}

extern "C" int mlbm_pool_forward(int32_t n, int32_t h, int32_t w, int32_t c, const void *x, int32_t xs, int32_t xo,
                                 void *y, int32_t ys, int32_t yo, void *stream) {
    mlbm::clear_error();
    if (!x || !y || n < 1 || h < 1 || w < 1 || c < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    pool_fwd_launch(n, h, w, c, (const unsigned short *)x, xs, xo, (unsigned short *)y, ys, yo, (hipStream_t)stream);
    return check("mlbm_pool_forward");
}

extern "C" int mlbm_pool_backward(int32_t n, int32_t h, int32_t w, int32_t c, const void *dy, int32_t dys,
                                  int32_t dyo, void *dx, int32_t dxs, int32_t dxo, const void *add, int32_t as,
                                  int32_t ao, void *stream) {
    mlbm::clear_error();
    if (!dy || !dx || n < 1 || h < 1 || w < 1 || c < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    pool_bwd_launch(n, h, w, c, (const unsigned short *)dy, dys, dyo, (unsigned short *)dx, dxs, dxo,
                    (const unsigned short *)add, as, ao, (hipStream_t)stream);
    return check("mlbm_pool_backward");
}

extern "C" int mlbm_upsample_forward(int32_t n, int32_t h, int32_t w, int32_t c, const void *x, int32_t xs,
                                     int32_t xo, void *y, int32_t ys, int32_t yo, void *stream) {
    mlbm::clear_error();
    if (!x || !y || n < 1 || h < 1 || w < 1 || c < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    up_fwd_launch(n, h, w, c, (const unsigned short *)x, xs, xo, (unsigned short *)y, ys, yo, (hipStream_t)stream);
    return check("mlbm_upsample_forward");
}

extern "C" int mlbm_upsample_backward(int32_t n, int32_t h, int32_t w, int32_t c, const void *dy, int32_t dys,
                                      int32_t dyo, void *dx, int32_t dxs, int32_t dxo, void *stream) {
    mlbm::clear_error();
    if (!dy || !dx || n < 1 || h < 1 || w < 1 || c < 1) return mlbm::fail(MLBM_ERR_ARG, "bad arguments");
    up_bwd_launch(n, h, w, c, (const unsigned short *)dy, dys, dyo, (unsigned short *)dx, dxs, dxo, (hipStream_t)stream);
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

// ---- the network ------------------------------------------------------------------------------

namespace {

struct Layer {
    char name[8];
    int ksize, c_in, c_out, level;
    int64_t w_off, b_off;     // floats, in params / grads / moments
    int64_t wf_off, wd_off;   // halves, in w_bf16
    int splits;               // pixel splits of the weight gradient
};

// activation buffers (halves, offsets in act and act_grad)
struct Acts {
    int64_t enc_a[MLBM_UNET_MAX_LEVELS], cat[MLBM_UNET_MAX_LEVELS], pool[MLBM_UNET_MAX_LEVELS];
    int64_t dec_a[MLBM_UNET_MAX_LEVELS], dec_b[MLBM_UNET_MAX_LEVELS], bottom, dout, total;
};

struct Net {
    int L, B, R, c_real_in, c_real_out;
    int c[MLBM_UNET_MAX_LEVELS];
    std::vector<Layer> layers;
    Acts a;
    int64_t n_params, n_wbf, ws_floats, work_bytes, loss_blocks;
};

constexpr int PADC = 32;

int net_plan(const mlbm_unet *u, Net &n) {
    using mlbm::fail;
    if (!u) return fail(MLBM_ERR_ARG, "null network");
    n.L = u->levels;
    n.B = u->batch;
    n.R = u->res;
    n.c_real_in = u->c_in;
    n.c_real_out = u->c_out;
    if (n.L < 2 || n.L > MLBM_UNET_MAX_LEVELS) return fail(MLBM_ERR_ARG, "levels must be 2..%d", MLBM_UNET_MAX_LEVELS);
    if (n.B < 1) return fail(MLBM_ERR_ARG, "batch must be positive");
    if (n.c_real_in < 1 || n.c_real_in > PADC || n.c_real_out < 1 || n.c_real_out > PADC)
        return fail(MLBM_ERR_ARG, "input and output channels must be 1..32");
    for (int l = 0; l < n.L; ++l) {
        n.c[l] = u->channels[l];
        if (n.c[l] < 32 || n.c[l] > 256 || n.c[l] % 32) return fail(MLBM_ERR_ARG, "channels must be multiples of 32 up to 256");
    }
    if (n.R < 8 || n.R % (1 << (n.L - 1))) return fail(MLBM_ERR_ARG, "res must be a multiple of 2^(levels-1)");
    const int rmin = n.R >> (n.L - 1);
    if (rmin % 8 || (rmin != 8 && rmin % 16)) return fail(MLBM_ERR_ARG, "the coarsest level must be 8 or a multiple of 16 wide");
    if ((int64_t)n.B * n.R * n.R > (int64_t)1 << 30) return fail(MLBM_ERR_ARG, "batch x res^2 too large");
    // layers in execution order
    n.layers.clear();
    auto add = [&](const char *nm, int lvl, int k, int ci, int co) {
        Layer ly;
        std::snprintf(ly.name, sizeof(ly.name), "%s", nm);
        ly.ksize = k;
        ly.c_in = ci;
        ly.c_out = co;
        ly.level = lvl;
        n.layers.push_back(ly);
    };
    char nm[8];
    int prev = PADC;
    for (int l = 0; l < n.L; ++l) {
        std::snprintf(nm, sizeof(nm), "enc%da", l);
        add(nm, l, 3, prev, n.c[l]);
        std::snprintf(nm, sizeof(nm), "enc%db", l);
        add(nm, l, 3, n.c[l], n.c[l]);
        prev = n.c[l];
    }
    for (int l = n.L - 2; l >= 0; --l) {
        std::snprintf(nm, sizeof(nm), "dec%da", l);
        add(nm, l, 3, prev + n.c[l], n.c[l]);
        std::snprintf(nm, sizeof(nm), "dec%db", l);
        add(nm, l, 3, n.c[l], n.c[l]);
        prev = n.c[l];
    }
    add("head", 0, 1, prev, PADC);
    int64_t pf = 0, ph = 0, ws = 0;
    for (Layer &ly : n.layers) {
        const int64_t m = (int64_t)ly.c_out * ly.ksize * ly.ksize * ly.c_in;
        ly.w_off = pf;
        ly.b_off = pf + m;
        pf += m + ly.c_out;
        ly.wf_off = ph;
        ly.wd_off = ph + m;
        ph += 2 * m;
        mlbm_conv_desc d{};
        const int Rl = n.R >> ly.level;
        d.n = n.B;
        d.h = d.w = Rl;
        d.c_in = ly.c_in;
        d.c_out = ly.c_out;
        d.ksize = ly.ksize;
        ly.splits = wgrad_splits(d);
        ws = std::max(ws, wgrad_workspace(d, ly.splits));
    }
    n.n_params = pf;
    n.n_wbf = ph;
    n.ws_floats = (ws + 3) / 4;
    // activations
    int64_t off = 0;
    auto take = [&](int64_t halves) {
        const int64_t o = off;
        off += (halves + 7) / 8 * 8;  // 16-byte aligned views
        return o;
    };
    for (int l = 0; l < n.L; ++l) {
        const int64_t P = (int64_t)n.B * (n.R >> l) * (n.R >> l);
        n.a.enc_a[l] = take(P * n.c[l]);
        if (l < n.L - 1) {
            n.a.cat[l] = take(P * (n.c[l + 1] + n.c[l]));
            n.a.pool[l] = take(P / 4 * n.c[l]);
            n.a.dec_a[l] = take(P * n.c[l]);
            n.a.dec_b[l] = take(P * n.c[l]);
        } else {
            n.a.bottom = take(P * n.c[l]);
        }
    }
    n.a.dout = take((int64_t)n.B * n.R * n.R * PADC);
    n.a.total = off;
    n.loss_blocks = ((int64_t)n.B * n.R * n.R + 255) / 256;
    // work: weight-gradient partials, then loss partials, mask partials, 1/count
    n.work_bytes = n.ws_floats * 4 + 2 * n.loss_blocks * 8 + 16;
    return MLBM_OK;
}

struct Ptrs {
    unsigned short *act, *grad, *wbf;
    float *ws;
    double *loss_part, *mask_part;
    float *inv;
};

Ptrs net_ptrs(const mlbm_unet *u, const Net &n) {
    Ptrs q;
    q.act = (unsigned short *)u->act;
    q.grad = (unsigned short *)u->act_grad;
    q.wbf = (unsigned short *)u->w_bf16;
    q.ws = (float *)u->work;
    q.loss_part = (double *)(q.ws + n.ws_floats + (n.ws_floats & 1));
    q.mask_part = q.loss_part + n.loss_blocks;
    q.inv = (float *)(q.mask_part + n.loss_blocks);
    return q;
}

mlbm_conv_desc desc_of(const Net &n, const Layer &ly, int xs, int xo, int ys, int yo) {
    mlbm_conv_desc d{};
    const int Rl = n.R >> ly.level;
    d.n = n.B;
    d.h = d.w = Rl;
    d.c_in = ly.c_in;
    d.c_out = ly.c_out;
    d.ksize = ly.ksize;
    d.x_stride = xs;
    d.x_offset = xo;
    d.y_stride = ys;
    d.y_offset = yo;
    d.c_store = ly.c_out;
    return d;
}

const Layer &layer(const Net &n, const char *name) {
    for (const Layer &ly : n.layers)
        if (std::strcmp(ly.name, name) == 0) return ly;
    return n.layers.back();  // not reached: every name is planned
}

int need_buffers(const mlbm_unet *u, bool grads) {
    if (!u->params || !u->w_bf16 || !u->act || !u->work || (grads && (!u->grads || !u->act_grad)))
        return mlbm::fail(MLBM_ERR_ARG, "null network buffer");
    return MLBM_OK;
}

}  // namespace

extern "C" int mlbm_unet_sizes(const mlbm_unet *u, mlbm_unet_buffers *out) {
    mlbm::clear_error();
    if (!out) return mlbm::fail(MLBM_ERR_ARG, "null output");
    Net n;
    int rc = net_plan(u, n);
    if (rc) return rc;
    out->n_params = n.n_params;
    out->w_bf16_bytes = n.n_wbf * 2;
    out->act_bytes = n.a.total * 2;
    out->work_bytes = n.work_bytes;
    out->n_layers = (int32_t)n.layers.size();
    return MLBM_OK;
}

extern "C" int mlbm_unet_layer(const mlbm_unet *u, int32_t index, mlbm_unet_layer_info *out) {
    mlbm::clear_error();
    Net n;
    int rc = net_plan(u, n);
    if (rc) return rc;
    if (!out || index < 0 || index >= (int)n.layers.size()) return mlbm::fail(MLBM_ERR_ARG, "bad layer index");
    const Layer &ly = n.layers[index];
    std::memcpy(out->name, ly.name, sizeof(out->name));
    out->ksize = ly.ksize;
    out->c_in = ly.c_in;
    out->c_out = ly.c_out;
    out->res = n.R >> ly.level;
    out->w_offset = ly.w_off;
    out->b_offset = ly.b_off;
    return MLBM_OK;
}

extern "C" int mlbm_unet_refresh(const mlbm_unet *u, void *stream) {
    mlbm::clear_error();
    Net n;
    int rc = net_plan(u, n);
    if (rc) return rc;
    if (!u->params || !u->w_bf16) return mlbm::fail(MLBM_ERR_ARG, "null params or w_bf16");
    WeightJobs jb{};
    if ((int)n.layers.size() > MAX_WJOBS) return mlbm::fail(MLBM_ERR_ARG, "too many layers");
    jb.n = (int)n.layers.size();
    for (int j = 0; j < jb.n; ++j) {
        const Layer &ly = n.layers[j];
        jb.w_off[j] = ly.w_off;
        jb.wf_off[j] = ly.wf_off;
        jb.wd_off[j] = ly.wd_off;
        jb.c_out[j] = ly.c_out;
        jb.taps[j] = ly.ksize * ly.ksize;
        jb.c_in[j] = ly.c_in;
        jb.start[j + 1] = jb.start[j] + (int64_t)ly.c_out * jb.taps[j] * ly.c_in;
    }
    hipLaunchKernelGGL(k_weights_all, dim3(blocks(jb.start[jb.n])), dim3(256), 0, (hipStream_t)stream, u->params,
                       (unsigned short *)u->w_bf16, jb);
    return check("mlbm_unet_refresh");
}

extern "C" int mlbm_unet_forward(const mlbm_unet *u, const void *x, float *out, void *stream) {
    mlbm::clear_error();
    Net n;
    int rc = net_plan(u, n);
    if (rc) return rc;
    if ((rc = need_buffers(u, false))) return rc;
    if (!x || !out) return mlbm::fail(MLBM_ERR_ARG, "null input or output");
    hipStream_t s = (hipStream_t)stream;
    const Ptrs q = net_ptrs(u, n);
    const float *prm = u->params;
    auto conv = [&](const char *name, const void *xin, int xs, int xo, void *y, int ys, int yo, int relu, int f32,
                    int c_store = 0, PoolOut pool = PoolOut{nullptr, 0, 0}, UpIn up = UpIn{nullptr, 0, 0}) {
        const Layer &ly = layer(n, name);
        mlbm_conv_desc d = desc_of(n, ly, xs, xo, ys, yo);
        if (c_store) d.c_store = c_store;
        return conv_launch(d, xin, q.wbf + ly.wf_off, prm + ly.b_off, y, relu, f32, nullptr, 0, 0, s, pool, up);
    };
    char nm[8];
    const void *h = x;
    int hs = PADC;
    for (int l = 0; l < n.L; ++l) {
        const int c = n.c[l];
        std::snprintf(nm, sizeof(nm), "enc%da", l);
        if ((rc = conv(nm, h, hs, 0, q.act + n.a.enc_a[l], c, 0, 1, 0))) return rc;
        std::snprintf(nm, sizeof(nm), "enc%db", l);
        if (l < n.L - 1) {
            const int cu = n.c[l + 1], cc = cu + c;
            // the skip copy, and its 2 x 2 average as the next level's input
            const PoolOut pool{q.act + n.a.pool[l], c, 0};
            if ((rc = conv(nm, q.act + n.a.enc_a[l], c, 0, q.act + n.a.cat[l], cc, cu, 1, 0, 0, pool))) return rc;
            h = q.act + n.a.pool[l];
        } else {
            if ((rc = conv(nm, q.act + n.a.enc_a[l], c, 0, q.act + n.a.bottom, c, 0, 1, 0))) return rc;
            h = q.act + n.a.bottom;
        }
        hs = c;
    }
    for (int l = n.L - 2; l >= 0; --l) {
        const int c = n.c[l], cu = n.c[l + 1], cc = cu + c;
        // input: the level below upsampled (read from there by the staging) and the skip copy
        std::snprintf(nm, sizeof(nm), "dec%da", l);
        const UpIn up{(const unsigned short *)h, hs, cu};
        if ((rc = conv(nm, q.act + n.a.cat[l], cc, 0, q.act + n.a.dec_a[l], c, 0, 1, 0, 0, PoolOut{nullptr, 0, 0}, up)))
            return rc;
        std::snprintf(nm, sizeof(nm), "dec%db", l);
        if ((rc = conv(nm, q.act + n.a.dec_a[l], c, 0, q.act + n.a.dec_b[l], c, 0, 1, 0))) return rc;
        h = q.act + n.a.dec_b[l];
        hs = c;
    }
    // only the real output channels are stored, packed (the padded ones have zero weights)
    if ((rc = conv("head", h, hs, 0, out, n.c_real_out, 0, 0, 1, n.c_real_out))) return rc;
    return check("mlbm_unet_forward");
}

extern "C" int mlbm_unet_loss(const mlbm_unet *u, const float *out, const float *target, const float *mask,
                              float *loss, void *stream) {
    mlbm::clear_error();
    Net n;
    int rc = net_plan(u, n);
    if (rc) return rc;
    if (!u->act_grad || !u->work || !out || !target || !mask || !loss) return mlbm::fail(MLBM_ERR_ARG, "null pointer");
    hipStream_t s = (hipStream_t)stream;
    const Ptrs q = net_ptrs(u, n);
    const int64_t P = (int64_t)n.B * n.R * n.R;
    hipLaunchKernelGGL(k_mask_partial, dim3((unsigned)n.loss_blocks), dim3(256), 0, s, P, mask, q.mask_part);
    hipLaunchKernelGGL(k_inv_count, dim3(1), dim3(256), 0, s, (const double *)q.mask_part, n.loss_blocks, n.c_real_out,
                       q.inv);
    hipLaunchKernelGGL(k_mse_dev, dim3((unsigned)n.loss_blocks), dim3(256), 0, s, P, n.c_real_out, out, n.c_real_out, PADC,
                       target,
                       mask, (const float *)q.inv, q.grad + n.a.dout, q.loss_part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, (const double *)q.loss_part, n.loss_blocks,
                       (const float *)q.inv, loss);
    return check("mlbm_unet_loss");
}

extern "C" int mlbm_unet_backward(const mlbm_unet *u, const void *x, void *stream) {
    mlbm::clear_error();
    Net n;
    int rc = net_plan(u, n);
    if (rc) return rc;
    if ((rc = need_buffers(u, true))) return rc;
    if (!x) return mlbm::fail(MLBM_ERR_ARG, "null input");
    hipStream_t s = (hipStream_t)stream;
    const Ptrs q = net_ptrs(u, n);
    unsigned short *A = q.act, *G = q.grad;
    float *gp = u->grads;
    auto wgrad = [&](const char *name, const void *xin, int xs, int xo, const void *dy, int ys, int yo,
                     UpIn up = UpIn{nullptr, 0, 0}) {
        const Layer &ly = layer(n, name);
        const mlbm_conv_desc d = desc_of(n, ly, xs, xo, ys, yo);
        return wgrad_launch(d, xin, dy, gp + ly.w_off, gp + ly.b_off, ly.splits, q.ws, s, up);
    };
    // data gradient: the forward product with the mirrored weights, c_in and c_out exchanged;
    // gate = the output of the layer below (its ReLU gradient), or NULL
    auto dgrad = [&](const char *name, const void *dy, int ys, int yo, void *dx, int xs, int xo, const void *gate,
                     int gs, int go, UpGrad ug = UpGrad{nullptr, 0, 0, nullptr}) {
        const Layer &ly = layer(n, name);
        mlbm_conv_desc d = desc_of(n, ly, ys, yo, xs, xo);
        d.c_in = ly.c_out;
        d.c_out = ly.c_in;
        d.c_store = ly.c_in;
        return conv_launch(d, dy, q.wbf + ly.wd_off, nullptr, dx, 0, 0, gate, gs, go, s, PoolOut{nullptr, 0, 0},
                           UpIn{nullptr, 0, 0}, ug);
    };
    char nm[8];
    const int c0 = n.c[0];
    if ((rc = wgrad("head", A + n.a.dec_b[0], c0, 0, G + n.a.dout, PADC, 0))) return rc;
    if ((rc = dgrad("head", G + n.a.dout, PADC, 0, G + n.a.dec_b[0], c0, 0, A + n.a.dec_b[0], c0, 0))) return rc;
    for (int l = 0; l < n.L - 1; ++l) {
        const int c = n.c[l], cu = n.c[l + 1], cc = cu + c;
        std::snprintf(nm, sizeof(nm), "dec%db", l);
        if ((rc = wgrad(nm, A + n.a.dec_a[l], c, 0, G + n.a.dec_b[l], c, 0))) return rc;
        if ((rc = dgrad(nm, G + n.a.dec_b[l], c, 0, G + n.a.dec_a[l], c, 0, A + n.a.dec_a[l], c, 0))) return rc;
        std::snprintf(nm, sizeof(nm), "dec%da", l);
        // this level's input, the decoder output of the level below or the
        // bottleneck: its upsampling is read from there (the concatenation holds
        // only the skip copy), and its gradient goes back there through its ReLU
        const int64_t bl = l + 1 <= n.L - 2 ? n.a.dec_b[l + 1] : n.a.bottom;
        if ((rc = wgrad(nm, A + n.a.cat[l], cc, 0, G + n.a.dec_a[l], c, 0, UpIn{A + bl, cu, cu}))) return rc;
        // (the upsampled channels' gradient is summed into G + bl by the epilogue)
        if ((rc = dgrad(nm, G + n.a.dec_a[l], c, 0, G + n.a.cat[l], cc, 0, nullptr, 0, 0, UpGrad{G + bl, cu, cu, A + bl})))
            return rc;
    }
    for (int l = n.L - 1; l >= 0; --l) {
        const int R = n.R >> l, c = n.c[l];
        unsigned short *gb;
        int bs, bo;
        if (l < n.L - 1) {
            const int cu = n.c[l + 1], cc = cu + c;
            // d(enc_b output) = the pooled path's gradient + the skip gradient, which
            // sits in the skip channels of the concatenation's gradient, through the ReLU
            pool_bwd_launch(n.B, R / 2, R / 2, c, (const unsigned short *)(G + n.a.pool[l]), c, 0, G + n.a.cat[l], cc, cu,
                            (const unsigned short *)(G + n.a.cat[l]), cc, cu, s, A + n.a.cat[l], cc, cu);
            gb = G + n.a.cat[l];
            bs = cc;
            bo = cu;
        } else {
            gb = G + n.a.bottom;
            bs = c;
            bo = 0;
        }
        // (the ReLU gradient was applied by the pooling or upsampling gradient above)
        std::snprintf(nm, sizeof(nm), "enc%db", l);
        if ((rc = wgrad(nm, A + n.a.enc_a[l], c, 0, gb, bs, bo))) return rc;
        if ((rc = dgrad(nm, gb, bs, bo, G + n.a.enc_a[l], c, 0, A + n.a.enc_a[l], c, 0))) return rc;
        std::snprintf(nm, sizeof(nm), "enc%da", l);
        if (l == 0) {
            if ((rc = wgrad(nm, x, PADC, 0, G + n.a.enc_a[0], c, 0))) return rc;
        } else {
            const int cb = n.c[l - 1];
            if ((rc = wgrad(nm, A + n.a.pool[l - 1], cb, 0, G + n.a.enc_a[l], c, 0))) return rc;
            if ((rc = dgrad(nm, G + n.a.enc_a[l], c, 0, G + n.a.pool[l - 1], cb, 0, nullptr, 0, 0))) return rc;
        }
    }
    return check("mlbm_unet_backward");
}

extern "C" int mlbm_unet_adam(const mlbm_unet *u, float lr, float beta1, float beta2, float eps, int32_t t,
                              void *stream) {
    mlbm::clear_error();
    Net n;
    int rc = net_plan(u, n);
    if (rc) return rc;
    if (!u->params || !u->grads || !u->adam_m || !u->adam_v || !u->w_bf16) return mlbm::fail(MLBM_ERR_ARG, "null buffer");
    if (t < 1) return mlbm::fail(MLBM_ERR_ARG, "step t must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const Layer &e0 = n.layers.front(), &hd = n.layers.back();
    const int64_t mm = (int64_t)e0.c_out * 9 * e0.c_in + (int64_t)hd.c_out * hd.c_in + hd.c_out;
    hipLaunchKernelGGL(k_mask_pad_grads, dim3(blocks(mm)), dim3(256), 0, s, u->grads + e0.w_off, e0.c_out, 9, e0.c_in,
                       n.c_real_in, u->grads + hd.w_off, u->grads + hd.b_off, hd.c_out, hd.c_in, n.c_real_out);
    const float c1 = 1.0f - std::pow(beta1, (float)t), c2 = 1.0f - std::pow(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(blocks(n.n_params)), dim3(256), 0, s, n.n_params, u->params, u->grads, u->adam_m,
                       u->adam_v, lr, beta1, beta2, eps, c1, c2);
    rc = check("mlbm_unet_adam");
    if (rc) return rc;
    return mlbm_unet_refresh(u, stream);
}
