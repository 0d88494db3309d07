// Device helpers of the step kernels shared by the translation units of
// libmlbm.so: storage formats, the lattice arithmetic in offset form, the
// step's kernel arguments, tile traversal and LDS staging.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "mlbm.h"

namespace mlbm_dev {


typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef int i4 __attribute__((ext_vector_type(4)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

// D2Q9 velocity set in the order of Sec. 2.1, Eq. 2.
__device__ constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
__device__ constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
// opposite of population k+1, minus one (populations 1..8 stored at 0..7)
__device__ constexpr int OPP8[8] = {2, 3, 0, 1, 6, 7, 4, 5};

template <class C>
__device__ __forceinline__ C omega(int k) {
    return k == 0 ? C(4) / C(9) : (k < 5 ? C(1) / C(9) : C(1) / C(36));
}

// node kind from the packed flags (bits 8-9)
__device__ __forceinline__ unsigned kind_of(unsigned fl) { return (fl >> 8) & 3u; }

// ---- storage formats -------------------------------------------------------

__device__ __forceinline__ float half_to_float(unsigned short h) {
    return __half2float(__ushort_as_half(h));
}
__device__ __forceinline__ unsigned short float_to_half(float f) {
    return __half_as_ushort(__float2half_rn(f));
}
__device__ __forceinline__ float bf16_to_float(unsigned short b) {
    return __uint_as_float(((unsigned)b) << 16);
}
// round to nearest even (finite inputs; NaN stays NaN)
__device__ __forceinline__ unsigned short float_to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)((u >> 16) | ((u & 0xffff) ? 0x40 : 0));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

template <int S> struct Fmt;
template <> struct Fmt<MLBM_F64> { using C = double; static constexpr int TB = 8; };
template <> struct Fmt<MLBM_F32> { using C = float; static constexpr int TB = 4; };
template <> struct Fmt<MLBM_F16S> { using C = float; static constexpr int TB = 2; };
template <> struct Fmt<MLBM_BF16> { using C = float; static constexpr int TB = 2; };

template <int S>
__device__ __forceinline__ float dec16(unsigned short v, float inv_scale) {
    if constexpr (S == MLBM_F16S) return half_to_float(v) * inv_scale;
    else return bf16_to_float(v);
}
// murmur3's 32-bit finaliser (a bijective integer mixer)
__host__ __device__ __forceinline__ unsigned mix32(unsigned x) {
    x ^= x >> 16;
    x *= 0x85ebca6bu;
    x ^= x >> 13;
    x *= 0xc2b2ae35u;
    x ^= x >> 16;
    return x;
}

// Random bits for stochastic rounding of 16-bit stores, counter based: one key
// per (node, step), mixed with the component index.  on == 0: round to nearest.
struct Rnd {
    unsigned key = 0;
    int on = 0;
    __device__ __forceinline__ unsigned bits(int c) const { return mix32(key ^ (0x9e3779b9u * (unsigned)(c + 1))); }
};

// 16-bit encodings.  Stochastic rounding adds uniform random bits below the
// kept mantissa bits of the FP32 value and truncates, so a value is rounded up
// with probability equal to its distance from the lower neighbour: the stored
// value is unbiased (exact for normal results; FP16 subnormals, below 2^-14
// after scaling, are rounded to nearest from the 13-bit step and keep a small bias).
template <int S>
__device__ __forceinline__ unsigned short enc16(float v, float scale, unsigned r = 0, int sr = 0) {
    if constexpr (S == MLBM_F16S) {
        const float x = v * scale;
        if (sr) {
            // with its 13 low bits cleared the value is exact in FP16 (normal range)
            unsigned u = __float_as_uint(x);
            if ((u & 0x7f800000u) != 0x7f800000u) u = (u + (r & 0x1fffu)) & ~0x1fffu;
            return float_to_half(__uint_as_float(u));
        }
        return float_to_half(x);
    } else {
        if (sr) {
            const unsigned u = __float_as_uint(v);
            if ((u & 0x7f800000u) != 0x7f800000u) return (unsigned short)((u + (r & 0xffffu)) >> 16);
        }
        return float_to_bf16(v);
    }
}

// eight population offsets (k = 1..8) of node j
template <int S, class C>
__device__ __forceinline__ void load8(const void *base, int64_t j, C *o, float inv_scale) {
    if constexpr (S == MLBM_F64) {
        const d2 *p = (const d2 *)base + 4 * j;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            d2 v = p[t];
            o[2 * t] = v.x;
            o[2 * t + 1] = v.y;
        }
    } else if constexpr (S == MLBM_F32) {
        const f4 *p = (const f4 *)base + 2 * j;
        f4 a = p[0], b = p[1];
        o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
        o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
    } else {
        u4 v = ((const u4 *)base)[j];
        unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            o[2 * t] = dec16<S>((unsigned short)(w[t] & 0xffff), inv_scale);
            o[2 * t + 1] = dec16<S>((unsigned short)(w[t] >> 16), inv_scale);
        }
    }
}

template <int S, class C>
__device__ __forceinline__ void store8(void *base, int64_t j, const C *o, float scale, Rnd rnd = {}) {
    if constexpr (S == MLBM_F64) {
        d2 *p = (d2 *)base + 4 * j;
#pragma unroll
        for (int t = 0; t < 4; ++t) p[t] = d2{(double)o[2 * t], (double)o[2 * t + 1]};
    } else if constexpr (S == MLBM_F32) {
        f4 *p = (f4 *)base + 2 * j;
        p[0] = f4{(float)o[0], (float)o[1], (float)o[2], (float)o[3]};
        p[1] = f4{(float)o[4], (float)o[5], (float)o[6], (float)o[7]};
    } else {
        unsigned w[4];
#pragma unroll
        for (int t = 0; t < 4; ++t)
            w[t] = (unsigned)enc16<S>((float)o[2 * t], scale, rnd.bits(2 * t), rnd.on) |
                   ((unsigned)enc16<S>((float)o[2 * t + 1], scale, rnd.bits(2 * t + 1), rnd.on) << 16);
        ((u4 *)base)[j] = u4{w[0], w[1], w[2], w[3]};
    }
}

// rest-population offset of node j, stored after the [n][8] block
template <int S, class C>
__device__ __forceinline__ C load1(const void *base, int64_t n, int64_t j, float inv_scale) {
    if constexpr (S == MLBM_F64) return ((const double *)base)[8 * n + j];
    else if constexpr (S == MLBM_F32) return ((const float *)base)[8 * n + j];
    else return dec16<S>(((const unsigned short *)base)[8 * n + j], inv_scale);
}
template <int S, class C>
__device__ __forceinline__ void store1(void *base, int64_t n, int64_t j, C v, float scale, Rnd rnd = {}) {
    if constexpr (S == MLBM_F64) ((double *)base)[8 * n + j] = v;
    else if constexpr (S == MLBM_F32) ((float *)base)[8 * n + j] = v;
    else ((unsigned short *)base)[8 * n + j] = enc16<S>((float)v, scale, rnd.bits(8), rnd.on);
}

// fields (rho - 1, u_x, u_y) of node j
template <int S, class C>
__device__ __forceinline__ void load3(const void *base, int64_t j, C *o, float inv_scale) {
    if constexpr (S == MLBM_F64) {
        const d2 *p = (const d2 *)base + 2 * j;
        d2 a = p[0], b = p[1];
        o[0] = a.x; o[1] = a.y; o[2] = b.x;
    } else if constexpr (S == MLBM_F32) {
        f4 a = ((const f4 *)base)[j];
        o[0] = a.x; o[1] = a.y; o[2] = a.z;
    } else {
        u2 v = ((const u2 *)base)[j];
        o[0] = dec16<S>((unsigned short)(v.x & 0xffff), inv_scale);
        o[1] = dec16<S>((unsigned short)(v.x >> 16), inv_scale);
        o[2] = dec16<S>((unsigned short)(v.y & 0xffff), inv_scale);
    }
}
template <int S, class C>
__device__ __forceinline__ void store3(void *base, int64_t j, const C *o, float scale, Rnd rnd = {}) {
    if constexpr (S == MLBM_F64) {
        d2 *p = (d2 *)base + 2 * j;
        p[0] = d2{(double)o[0], (double)o[1]};
        p[1] = d2{(double)o[2], 0.0};
    } else if constexpr (S == MLBM_F32) {
        ((f4 *)base)[j] = f4{(float)o[0], (float)o[1], (float)o[2], 0.0f};
    } else {
        unsigned a = (unsigned)enc16<S>((float)o[0], scale, rnd.bits(0), rnd.on) |
                     ((unsigned)enc16<S>((float)o[1], scale, rnd.bits(1), rnd.on) << 16);
        unsigned b = (unsigned)enc16<S>((float)o[2], scale, rnd.bits(2), rnd.on);
        ((u2 *)base)[j] = u2{a, b};
    }
}

// streamed (read-once-per-step) data: non-temporal unless cached is set
template <class T>
__device__ __forceinline__ T stream_load(const T *p, int cached) {
    return cached ? *p : __builtin_nontemporal_load(p);
}

// four weights (stencil members 4q..4q+3) of arriving population k+1; W16
// (16-bit states only): the weights are FP16 in the same layout
template <int S, int KQ, bool W16 = false, class C>
__device__ __forceinline__ void load_w4(const void *w, int64_t n, int64_t i, int k, int q, C *o,
                                        int cached = 0) {
    if constexpr (S == MLBM_F64) {
        const d2 *p = (const d2 *)w;
        d2 a = stream_load(p + ((int64_t)(k * 2 * KQ + 2 * q) * n + i), cached);
        d2 b = stream_load(p + ((int64_t)(k * 2 * KQ + 2 * q + 1) * n + i), cached);
        o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
    } else if constexpr (S == MLBM_F16S || S == MLBM_BF16) {
        if constexpr (W16) {
            const u2 *p = (const u2 *)w;
            u2 a = stream_load(p + ((int64_t)(k * KQ + q) * n + i), cached);
            o[0] = half_to_float((unsigned short)(a.x & 0xffffu));
            o[1] = half_to_float((unsigned short)(a.x >> 16));
            o[2] = half_to_float((unsigned short)(a.y & 0xffffu));
            o[3] = half_to_float((unsigned short)(a.y >> 16));
        } else {
            const f4 *p = (const f4 *)w;
            f4 a = stream_load(p + ((int64_t)(k * KQ + q) * n + i), cached);
            o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
        }
    } else {
        const f4 *p = (const f4 *)w;
        f4 a = stream_load(p + ((int64_t)(k * KQ + q) * n + i), cached);
        o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    }
}

__device__ __forceinline__ i4 load_idx4(const int *idx, int64_t n, int64_t i, int q, int cached = 0) {
    return stream_load((const i4 *)idx + ((int64_t)q * n + i), cached);
}

// ---- lattice arithmetic in offset form ---------------------------------------

// equilibrium offset f^eq_k - omega_k of (rho, u) (Sec. 2.1, Eq. 7); sgn = -1
// evaluates the opposite direction k'
template <class C>
__device__ __forceinline__ C feq_off(int k, C sgn, C drho, C rho, C ux, C uy) {
    const C eu = sgn * (C(EX[k]) * ux + C(EY[k]) * uy);
    const C usq = ux * ux + uy * uy;
    return omega<C>(k) * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * usq));
}

// Guo force term F_k (k' for sgn = -1)
template <class C>
__device__ __forceinline__ C force_k(int k, C sgn, C rho, C ux, C uy, C gx, C gy) {
    const C ex = sgn * C(EX[k]), ey = sgn * C(EY[k]);
    const C eu = ex * ux + ey * uy;
    const C eg = ex * gx + ey * gy;
    const C ug = ux * gx + uy * gy;
    return omega<C>(k) * rho * (C(3) * (eg - ug) + C(9) * eu * eg);
}

// TRT collision with Guo forcing on offsets f[0..8] (Sec. 2.1, Eqs. 3-4)
template <class C>
__device__ __forceinline__ void collide(C *f, C omp, C omm, C gx, C gy) {
    const C drho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    const C rho = C(1) + drho;
    const C jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const C jy = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
    const C inv = C(1) / rho;
    const C ux = (jx + C(0.5) * rho * gx) * inv;
    const C uy = (jy + C(0.5) * rho * gy) * inv;
    const C cp = C(1) - C(0.5) * omp, cm = C(1) - C(0.5) * omm;
    {
        const C e0 = feq_off<C>(0, C(1), drho, rho, ux, uy);
        const C F0 = force_k<C>(0, C(1), rho, ux, uy, gx, gy);
        f[0] = f[0] - omp * (f[0] - e0) + cp * F0;
    }
    constexpr int A[4] = {1, 2, 5, 6};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int a = A[t], b = a + 2;  // b = opposite of a for these four
        const C ea = feq_off<C>(a, C(1), drho, rho, ux, uy), eb = feq_off<C>(b, C(1), drho, rho, ux, uy);
        const C Fa = force_k<C>(a, C(1), rho, ux, uy, gx, gy), Fb = force_k<C>(b, C(1), rho, ux, uy, gx, gy);
        const C fp = C(0.5) * (f[a] + f[b]), fm = C(0.5) * (f[a] - f[b]);
        const C ep = C(0.5) * (ea + eb), em = C(0.5) * (ea - eb);
        const C Fp = C(0.5) * (Fa + Fb), Fm = C(0.5) * (Fa - Fb);
        const C sym = -omp * (fp - ep) + cp * Fp;
        const C asy = -omm * (fm - em) + cm * Fm;
        f[a] = f[a] + sym + asy;
        f[b] = f[b] + sym - asy;
    }
}

struct StepArgs {
    int64_t n;
    const int *idx;
    const void *w;
    const uint16_t *flags;
    const double *bc;
    const void *in;
    void *out;
    double omp, omm, gx, gy;
    float scale, inv_scale;
    int64_t grid8;
    int xcd;
    int reverse;   // sweep the tiles in reverse order (alternating sweeps)
    int cached;    // plain loads for weights and indices instead of non-temporal
    const int *halo_off;       // LDS staging: per-tile CSR offsets into halo
    const int *halo;           // LDS staging: halo node lists
    const unsigned short *lidx;  // LDS staging: tile-local member positions [K8/8][n][8]
    const void *wl;            // block weights [8][9] (FP64 storage: double, else float)
    int64_t tile0, tile1;      // tiles [tile0, tile1) of this launch (non-batched)
    int64_t split;             // hybrid sets in one launch: workgroups [split, ...) walk the
    int64_t tile0b, tile1b;    //   block-centre tiles [tile0b, tile1b) over grid8b workgroups
    int64_t grid8b;
    int64_t lag0;              // first node of the trailing run of block centres (n: none);
                               // the tile holding it is visited by both launches, each
                               // updating its own nodes
    int sr;                    // stochastic rounding of 16-bit stores
    unsigned seed;             // this step's random key
    const int *queue;          // batched launches: list of active tiles (NULL: every tile)
    const int *queue_range;    // batched launches: device offsets; this launch walks
    int group;                 //   queue[queue_range[group] .. queue_range[group + 1])
};

// random key of node i in this step (stochastic rounding of 16-bit states)
__device__ __forceinline__ Rnd step_rnd(const StepArgs &a, int64_t i) {
    Rnd r;
    r.on = a.sr;
    r.key = a.sr ? mix32((unsigned)i * 0x9e3779b9u + a.seed) : 0u;
    return r;
}

// Workgroups are dispatched to the 8 XCDs round-robin; with xcd each XCD gets
// a contiguous range of tiles.  With reverse the tiles are visited in the
// opposite order, so alternating sweeps start where the previous one ended and
// meet its most recently cached data first.
__device__ __forceinline__ int64_t tile_at(const StepArgs &a, int64_t b, int64_t grid8) {
    if (a.xcd) {
        const int64_t per = grid8 >> 3;
        const int64_t r = b >> 3;
        b = (b & 7) * per + (a.reverse ? per - 1 - r : r);
    } else if (a.reverse) {
        b = grid8 - 1 - b;
    }
    return b;
}
__device__ __forceinline__ int64_t tile_of(const StepArgs &a) { return tile_at(a, blockIdx.x, a.grid8); }

// Copies the state of every halo node of `tile` into LDS (NB bytes per node,
// same layout as the global state), coalesced over 16-byte (or 8-byte) units.
// The halo is sorted and holds every node of the tile, so the tile's own nodes
// sit at consecutive positions; *self0 receives the first of them.
template <int NB, bool SELF>
__device__ __forceinline__ void stage_halo(const StepArgs &a, int64_t tile, void *smem, int *self0) {
    __syncthreads();  // the previous tile of a persistent workgroup is done with the LDS
    const int h0 = a.halo_off[tile], hn = a.halo_off[tile + 1] - h0;
    const int64_t first = tile * blockDim.x;
    if constexpr (NB >= 16) {
        constexpr int U = NB / 16;
        const u4 *src = (const u4 *)a.in;
        u4 *dst = (u4 *)smem;
        for (int e = threadIdx.x; e < hn * U; e += blockDim.x) {
            const int h = e / U, c = e - h * U;
            const int node = a.halo[h0 + h];
            if (SELF && c == 0 && node == first) *self0 = h;
            dst[e] = src[(int64_t)node * U + c];
        }
    } else {
        const u2 *src = (const u2 *)a.in;
        u2 *dst = (u2 *)smem;
        for (int h = threadIdx.x; h < hn; h += blockDim.x) {
            const int node = a.halo[h0 + h];
            if (SELF && node == first) *self0 = h;
            dst[h] = src[node];
        }
    }
    __syncthreads();
}

// Calls f(tile) for the tiles of this workgroup: one tile per workgroup over
// the whole node range, or (batched launches) a contiguous chunk of the active
// tile list per persistent workgroup.  With xcd the active entries are split
// evenly over the 8 XCDs (the grid is a multiple of 8), each XCD's contiguous
// share over its own workgroups: the grid is sized for a group's full tile
// count, so splitting by workgroup alone would leave the last XCDs idle once
// samples of the group have retired.
template <class F>
__device__ __forceinline__ void for_tiles(const StepArgs &a, F &&f) {
    if (a.queue) {
        const int q0 = a.queue_range[a.group], na = a.queue_range[a.group + 1] - q0;
        int b = blockIdx.x, nw = gridDim.x, lo = 0, cnt = na;
        if (a.xcd) {
            const int x = b & 7;
            nw >>= 3;
            b >>= 3;
            if (b >= nw) return;  // (a grid that is not a multiple of 8)
            lo = (int)(((int64_t)na * x) >> 3);
            cnt = (int)(((int64_t)na * (x + 1)) >> 3) - lo;
        }
        if (a.reverse) b = nw - 1 - b;
        const int chunk = (cnt + nw - 1) / nw;
        const int c1 = lo + min(cnt, (b + 1) * chunk);
        for (int c = lo + b * chunk; c < c1; ++c) f((int64_t)a.queue[q0 + c]);
    } else {
        const int64_t tile = a.tile0 + tile_of(a);
        if (tile < a.tile1) f(tile);
    }
}

// bytes per node of the [n][8] population block / the [n][4] field block
template <int S> constexpr int pop_bytes() { return 8 * Fmt<S>::TB; }
template <int S> constexpr int field_bytes() { return 4 * Fmt<S>::TB; }

// four stencil members of quad q: global node indices, or halo positions when staged
template <bool LDS, int Q>
__device__ __forceinline__ void members(const StepArgs &a, int64_t n, int64_t i, u4 &lv, int *m) {
    if constexpr (LDS) {
        if constexpr ((Q & 1) == 0) lv = stream_load((const u4 *)a.lidx + ((int64_t)(Q >> 1) * n + i), a.cached);
        const unsigned lo = (Q & 1) ? lv.z : lv.x, hi = (Q & 1) ? lv.w : lv.y;
        m[0] = (int)(lo & 0xffffu);
        m[1] = (int)(lo >> 16);
        m[2] = (int)(hi & 0xffffu);
        m[3] = (int)(hi >> 16);
    } else {
        const i4 id = load_idx4(a.idx, n, i, Q, a.cached);
        m[0] = id.x;
        m[1] = id.y;
        m[2] = id.z;
        m[3] = id.w;
    }
}

// Block centres of a hybrid set: members 0..7 are the lattice neighbours
// x + h e_1 .. x + h e_8 (first index plane), member 8 the node itself, at
// position self (its halo position, or i).
template <bool LDS>
__device__ __forceinline__ void block_members(const StepArgs &a, int64_t n, int64_t i, int self, int *m) {
    if constexpr (LDS) {
        const u4 lv = stream_load((const u4 *)a.lidx + i, a.cached);
        const unsigned v[4] = {lv.x, lv.y, lv.z, lv.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            m[2 * t] = (int)(v[t] & 0xffffu);
            m[2 * t + 1] = (int)(v[t] >> 16);
        }
    } else {
        const i4 q0 = load_idx4(a.idx, n, i, 0, a.cached), q1 = load_idx4(a.idx, n, i, 1, a.cached);
        m[0] = q0.x; m[1] = q0.y; m[2] = q0.z; m[3] = q0.w;
        m[4] = q1.x; m[5] = q1.y; m[6] = q1.z; m[7] = q1.w;
    }
    m[8] = self;
}

// one block weight; the address is the same for every lane (a scalar load)
template <int S, class CG>
__device__ __forceinline__ CG block_weight(const StepArgs &a, int t) {
    if constexpr (S == MLBM_F64) return (CG)((const double *)a.wl)[t];
    else return (CG)((const float *)a.wl)[t];
}

// compile-time loop over the stencil quads
template <int Q, int KQ, class F>
__device__ __forceinline__ void for_quads(F &&f) {
    if constexpr (Q < KQ) {
        f(std::integral_constant<int, Q>{});
        for_quads<Q + 1, KQ>(f);
    }
}

// population c of the staged node m
template <int S, class CG>
__device__ __forceinline__ CG load_comp(const void *src, int m, int c, float inv_scale) {
    if constexpr (S == MLBM_F64) return ((const double *)src)[8 * m + c];
    else if constexpr (S == MLBM_F32) return ((const float *)src)[8 * m + c];
    else return dec16<S>(((const unsigned short *)src)[8 * m + c], inv_scale);
}

using StepFn = void (*)(const StepArgs);

// Kernels with eight lanes per node (mlbm_lanes.hip): population or fields
// form, any storage, per-node stencils of kq member quads (3, 4, 7 or 8),
// LDS-staged tiles or global gathers; nullptr if there is none.
StepFn pick_step_lanes_any(int storage, int variant, int kq, bool lds, int w16);
// The same for a hybrid set in one launch per step (per-node tiles first,
// then the block-centre tiles; LDS-staged tiles).
StepFn pick_step_lanes_hyb_any(int storage, int variant, int kq, int w16);

}  // namespace mlbm_dev
