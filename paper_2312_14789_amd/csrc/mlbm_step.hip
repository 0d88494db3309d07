// Fused meshless LBM step kernels for gfx950 (MI355X) and their C ABI entry
// points: initial state, time step (population MLBM and MLBM1), macroscopic
// fields with FP64 reductions.
//
// One thread owns one Eulerian node.  Per step it gathers the post-collision
// state of its K stencil members (Sec. 2.2, Eq. 12), weights them with the
// node's eight weight sets streamed from HBM (non-temporal, so the L2 keeps
// the gathered state), then collides in registers (Sec. 2.1, Eqs. 3-4, Guo
// forcing) and writes its post-collision state to the other buffer.  The
// state holds offsets from the rest equilibrium (f_k - omega_k, or rho - 1),
// so rounding in FP32 and 16-bit storage acts on O(u) quantities and the
// small deviation of FP32 weights from a partition of unity does not act as
// a mass source.  Node order is Morton order, so stencil members of a
// wavefront are near each other in memory; with xcd_remap each XCD receives
// a contiguous range of tiles and its L2 sees the spatial neighbourhood.

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <algorithm>
#include <mutex>
#include <vector>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>

#include "mlbm.h"
#include "mlbm_device.h"
#include "mlbm_internal.h"

using namespace mlbm_dev;

namespace {

// ---- population MLBM step ------------------------------------------------------

// CG: gather (interpolation) arithmetic; C: collision arithmetic.  KQ = 0
// instantiates the block-centre kernel of a hybrid set: it updates the nodes
// from lag0 on, every one a block centre with the shared weights (a node
// without the flag gets a NaN state, so a wrong node range shows up at once);
// the per-node kernels update the nodes before lag0.
template <int S, class CG, class C, int KQ, bool LDS, bool W16 = false>
__device__ __forceinline__ void pop_node(const StepArgs &a, const void *src, int64_t i, int self) {
    if ((KQ == 0) != (i >= a.lag0)) return;  // the other launch's node
    const int64_t n = a.n;
    const unsigned fl = a.flags[i];
    const unsigned bb = fl & 0xffu;
    C f[9];
    // FP64 keeps the weight sum: sum_j w_j f_j = sum_j w_j (f_j - omega) + omega sum_j w_j,
    // exactly the interpolation of the populations; reduced precision drops
    // the (sum_j w_j - 1) omega term, which is weight rounding there.
    constexpr bool kWsum = S == MLBM_F64;
    CG acc[8], sw[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = sw[k] = CG(0);
    if (kind_of(fl) == MLBM_DIRICHLET) {
        const C rb = (C)a.bc[3 * i], ub = (C)a.bc[3 * i + 1], vb = (C)a.bc[3 * i + 2];
#pragma unroll
        for (int k = 0; k < 9; ++k) f[k] = feq_off<C>(k, C(1), rb - C(1), rb, ub, vb);
        store8<S>(a.out, i, f + 1, a.scale);
        store1<S, C>(a.out, n, i, f[0], a.scale);
        return;
    }
    if constexpr (KQ == 0) {
        // block centre: the shared biquadratic weights (no bounce-back here)
        if (!(fl & MLBM_FLAG_LAGRANGE)) {
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[k] = CG(NAN);
        }
        int m[9];
        block_members<LDS>(a, n, i, self, m);
        for_quads<0, 3>([&](auto gc) __attribute__((always_inline)) {
            constexpr int j0 = 4 * decltype(gc)::value, nj = j0 < 8 ? 4 : 1;
            CG v[4][8];
#pragma unroll
            for (int j = 0; j < nj; ++j) load8<S>(src, m[j0 + j], v[j], a.inv_scale);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
#pragma unroll
                for (int j = 0; j < nj; ++j) {
                    const CG wv = block_weight<S, CG>(a, k * 9 + j0 + j);
                    acc[k] = fma(wv, v[j][k], acc[k]);
                    if constexpr (kWsum) sw[k] += wv;
                }
            }
            __builtin_amdgcn_sched_barrier(0);  // keep the groups' loads apart (registers)
        });
    } else {
        u4 lv;
        for_quads<0, KQ>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value;
            int m[4];
            members<LDS, q>(a, n, i, lv, m);
            CG s[4][8];
#pragma unroll
            for (int j = 0; j < 4; ++j) load8<S>(src, m[j], s[j], a.inv_scale);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                CG wv[4];
                load_w4<S, KQ, W16>(a.w, n, i, k, q, wv, a.cached);
                const bool flip = (bb >> k) & 1u;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const CG v = flip ? s[j][OPP8[k]] : s[j][k];
                    acc[k] = fma(wv[j], v, acc[k]);
                    if constexpr (kWsum) sw[k] += wv[j];
                }
            }
        });
    }
    f[0] = load1<S, C>(a.in, n, i, a.inv_scale);
#pragma unroll
    for (int k = 0; k < 8; ++k)
        f[k + 1] = kWsum ? (C)acc[k] + omega<C>(k + 1) * ((C)sw[k] - C(1)) : (C)acc[k];
    collide<C>(f, (C)a.omp, (C)a.omm, (C)a.gx, (C)a.gy);
    if (a.sr) {
        const Rnd rnd = step_rnd(a, i);
        store8<S>(a.out, i, f + 1, a.scale, rnd);
        store1<S, C>(a.out, n, i, f[0], a.scale, rnd);
    } else {
        store8<S>(a.out, i, f + 1, a.scale);
        store1<S, C>(a.out, n, i, f[0], a.scale);
    }
}

// The block-centre kernels (KQ = 0) are short and latency bound: they are
// compiled for at least six waves per SIMD with 32-bit arithmetic (the others
// are left to the compiler, 1 = no constraint).
template <int S, int KQ> constexpr int block_waves() { return KQ != 0 ? 1 : (S == MLBM_F64 ? 3 : 6); }

template <int S, class CG, class C, int KQ, bool LDS, bool W16 = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(block_waves<S, KQ>()))) k_step_pop(const StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int self0;
    for_tiles(a, [&](int64_t tile) __attribute__((always_inline)) {
        if constexpr (LDS) stage_halo<pop_bytes<S>(), KQ == 0>(a, tile, smem, &self0);
        const int64_t i = tile * blockDim.x + threadIdx.x;
        if (i < a.n)
            pop_node<S, CG, C, KQ, LDS, W16>(a, LDS ? (const void *)smem : a.in, i,
                                        KQ == 0 && LDS ? self0 + (int)threadIdx.x : (int)i);
    });
}

// Block-centre tiles of a one-launch hybrid step: 16-bit states stage the
// tile's halo in LDS as the per-node tiles do; 32- and 64-bit states gather
// the eight lattice neighbours straight from global memory (they sit in the
// same or an adjacent Morton tile, so most of them hit in L2), which spares
// the staging pass and its barriers.  Measured on the hybrid Karman set: FP32
// 29.6 -> 28.1 us per step with global gathers; FP16 17.5 us staged against
// 18.9 us with global gathers.
template <int S> constexpr bool block_tiles_staged() { return Fmt<S>::TB == 2; }

// A hybrid set in one launch: workgroups [0, split) take the tiles of the nodes
// with per-node weights, the later ones the block-centre tiles.  The two kinds
// write disjoint nodes and read only the previous state, so nothing orders
// them; in one launch the short block-centre tiles fill the tail of the
// per-node ones instead of waiting for it (two launches leave the chip to drain
// in between, and the block-centre launch alone is too short to hide its
// latency).  The tile holding both kinds is visited from both sides.
template <int S, class CG, class C, int KQ, bool W16>
__global__ void __launch_bounds__(256) k_step_pop_hyb(const StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int self0;
    const int64_t b = blockIdx.x;
    if (b < a.split) {
        const int64_t tile = a.tile0 + tile_at(a, b, a.grid8);
        if (tile >= a.tile1) return;
        stage_halo<pop_bytes<S>(), false>(a, tile, smem, &self0);
        const int64_t i = tile * blockDim.x + threadIdx.x;
        if (i < a.n) pop_node<S, CG, C, KQ, true, W16>(a, (const void *)smem, i, (int)i);
    } else {
        const int64_t tile = a.tile0b + tile_at(a, b - a.split, a.grid8b);
        if (tile >= a.tile1b) return;
        const int64_t i = tile * blockDim.x + threadIdx.x;
        if constexpr (block_tiles_staged<S>()) {
            stage_halo<pop_bytes<S>(), true>(a, tile, smem, &self0);
            if (i < a.n) pop_node<S, CG, C, 0, true, false>(a, (const void *)smem, i, self0 + (int)threadIdx.x);
        } else {
            if (i < a.n) pop_node<S, CG, C, 0, false, false>(a, a.in, i, (int)i);
        }
    }
}

// ---- MLBM1 step (tau = 1, fields only) -------------------------------------------

template <int S, class CG, class C, int KQ, bool LDS, bool W16 = false>
__device__ __forceinline__ void fields_node(const StepArgs &a, const void *src, int64_t i, int self) {
    if ((KQ == 0) != (i >= a.lag0)) return;  // the other launch's node
    const int64_t n = a.n;
    const unsigned fl = a.flags[i];
    const unsigned bb = fl & 0xffu;
    C out[3];
    if (kind_of(fl) == MLBM_DIRICHLET) {
        out[0] = (C)a.bc[3 * i] - C(1);
        out[1] = (C)a.bc[3 * i + 1];
        out[2] = (C)a.bc[3 * i + 2];
    } else {
        constexpr bool kWsum = S == MLBM_F64;  // interpolate rho itself, not rho - 1
        CG ar[8], au[8], av[8], sw[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) ar[k] = au[k] = av[k] = sw[k] = CG(0);
        if constexpr (KQ == 0) {
            // block centre: the shared biquadratic weights (no bounce-back here)
            if (!(fl & MLBM_FLAG_LAGRANGE)) {
#pragma unroll
                for (int k = 0; k < 8; ++k) ar[k] = CG(NAN);
            }
            int mi[9];
            block_members<LDS>(a, n, i, self, mi);
            for_quads<0, 3>([&](auto gc) __attribute__((always_inline)) {
                constexpr int j0 = 4 * decltype(gc)::value, nj = j0 < 8 ? 4 : 1;
                CG m[4][3];
#pragma unroll
                for (int j = 0; j < nj; ++j) load3<S>(src, mi[j0 + j], m[j], a.inv_scale);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
#pragma unroll
                    for (int j = 0; j < nj; ++j) {
                        const CG wv = block_weight<S, CG>(a, k * 9 + j0 + j);
                        ar[k] = fma(wv, m[j][0], ar[k]);
                        au[k] = fma(wv, m[j][1], au[k]);
                        av[k] = fma(wv, m[j][2], av[k]);
                        if constexpr (kWsum) sw[k] += wv;
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
            });
        } else {
        u4 lv;
        for_quads<0, KQ>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value;
            int mi[4];
            members<LDS, q>(a, n, i, lv, mi);
            CG m[4][3];
#pragma unroll
            for (int j = 0; j < 4; ++j) load3<S>(src, mi[j], m[j], a.inv_scale);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                CG wv[4];
                load_w4<S, KQ, W16>(a.w, n, i, k, q, wv, a.cached);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    ar[k] = fma(wv[j], m[j][0], ar[k]);
                    au[k] = fma(wv[j], m[j][1], au[k]);
                    av[k] = fma(wv[j], m[j][2], av[k]);
                    if constexpr (kWsum) sw[k] += wv[j];
                }
            }
        });
        }
        if constexpr (kWsum) {
#pragma unroll
            for (int k = 0; k < 8; ++k) ar[k] += sw[k] - CG(1);
        }
        const C gx = (C)a.gx, gy = (C)a.gy;
        C own[3];
        load3<S>(a.in, i, own, a.inv_scale);
        // rest population from the node's own fields (not interpolated, Sec. 2.2)
        C sum = feq_off<C>(0, C(1), own[0], C(1) + own[0], own[1], own[2]) +
                C(0.5) * force_k<C>(0, C(1), C(1) + own[0], own[1], own[2], gx, gy);
        C jx = C(0), jy = C(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const C sg = ((bb >> k) & 1u) ? C(-1) : C(1);  // source k' on bounce-back
            const C dr = (C)ar[k], uk = (C)au[k], vk = (C)av[k];
            const C rho = C(1) + dr;
            const C fk = feq_off<C>(k + 1, sg, dr, rho, uk, vk) +
                         C(0.5) * force_k<C>(k + 1, sg, rho, uk, vk, gx, gy);
            sum += fk;
            jx += C(EX[k + 1]) * fk;
            jy += C(EY[k + 1]) * fk;
        }
        const C rho = C(1) + sum;
        out[0] = sum;
        out[1] = (jx + C(0.5) * rho * gx) / rho;
        out[2] = (jy + C(0.5) * rho * gy) / rho;
    }
    store3<S>(a.out, i, out, a.scale, step_rnd(a, i));
}

template <int S, class CG, class C, int KQ, bool LDS, bool W16 = false>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(block_waves<S, KQ>()))) k_step_fields(const StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int self0;
    for_tiles(a, [&](int64_t tile) __attribute__((always_inline)) {
        if constexpr (LDS) stage_halo<field_bytes<S>(), KQ == 0>(a, tile, smem, &self0);
        const int64_t i = tile * blockDim.x + threadIdx.x;
        if (i < a.n)
            fields_node<S, CG, C, KQ, LDS, W16>(a, LDS ? (const void *)smem : a.in, i,
                                           KQ == 0 && LDS ? self0 + (int)threadIdx.x : (int)i);
    });
}

// the MLBM1 step of a hybrid set in one launch (as k_step_pop_hyb)
template <int S, class CG, class C, int KQ, bool W16>
__global__ void __launch_bounds__(256) k_step_fields_hyb(const StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int self0;
    const int64_t b = blockIdx.x;
    if (b < a.split) {
        const int64_t tile = a.tile0 + tile_at(a, b, a.grid8);
        if (tile >= a.tile1) return;
        stage_halo<field_bytes<S>(), false>(a, tile, smem, &self0);
        const int64_t i = tile * blockDim.x + threadIdx.x;
        if (i < a.n) fields_node<S, CG, C, KQ, true, W16>(a, (const void *)smem, i, (int)i);
    } else {
        const int64_t tile = a.tile0b + tile_at(a, b - a.split, a.grid8b);
        if (tile >= a.tile1b) return;
        const int64_t i = tile * blockDim.x + threadIdx.x;
        if constexpr (block_tiles_staged<S>()) {
            stage_halo<field_bytes<S>(), true>(a, tile, smem, &self0);
            if (i < a.n) fields_node<S, CG, C, 0, true, false>(a, (const void *)smem, i, self0 + (int)threadIdx.x);
        } else {
            if (i < a.n) fields_node<S, CG, C, 0, false, false>(a, a.in, i, (int)i);
        }
    }
}

// ---- one stencil per departure point (the paper's stencils) ----------------------------
//
// Arriving population k has its own K members (its departure point's nearest
// nodes), in index planes k * K8/8 .. (k + 1) * K8/8 - 1 of the tile-local
// indices; from each member only one population (k, or k' on bounce-back) or
// the fields are read.  LDS-staged tiles only.


// four members of quad q of departure point k (plane k * k8q + q / 2)
__device__ __forceinline__ void members_pd(const StepArgs &a, int64_t n, int64_t i, int plane, int half, u4 &lv,
                                           int *m) {
    if (half == 0) lv = stream_load((const u4 *)a.lidx + ((int64_t)plane * n + i), a.cached);
    const unsigned lo = half ? lv.z : lv.x, hi = half ? lv.w : lv.y;
    m[0] = (int)(lo & 0xffffu);
    m[1] = (int)(lo >> 16);
    m[2] = (int)(hi & 0xffffu);
    m[3] = (int)(hi >> 16);
}

template <int S, class CG, class C, int KQ, bool W16 = false>
__device__ __forceinline__ void pop_node_pd(const StepArgs &a, const void *src, int64_t i) {
    constexpr int K8Q = (KQ + 1) / 2;  // index planes per departure point
    const int64_t n = a.n;
    const unsigned fl = a.flags[i];
    const unsigned bb = fl & 0xffu;
    C f[9];
    if (kind_of(fl) == MLBM_DIRICHLET) {
        const C rb = (C)a.bc[3 * i], ub = (C)a.bc[3 * i + 1], vb = (C)a.bc[3 * i + 2];
#pragma unroll
        for (int k = 0; k < 9; ++k) f[k] = feq_off<C>(k, C(1), rb - C(1), rb, ub, vb);
    } else {
        constexpr bool kWsum = S == MLBM_F64;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = ((bb >> k) & 1u) ? OPP8[k] : k;
            CG acc = CG(0), sw = CG(0);
            u4 lv;
            for_quads<0, KQ>([&](auto qc) __attribute__((always_inline)) {
                constexpr int q = decltype(qc)::value;
                int m[4];
                members_pd(a, n, i, k * K8Q + (q >> 1), q & 1, lv, m);
                CG wv[4];
                load_w4<S, KQ, W16>(a.w, n, i, k, q, wv, a.cached);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    acc = fma(wv[j], load_comp<S, CG>(src, m[j], c, a.inv_scale), acc);
                    if constexpr (kWsum) sw += wv[j];
                }
            });
            f[k + 1] = kWsum ? (C)acc + omega<C>(k + 1) * ((C)sw - C(1)) : (C)acc;
        }
        f[0] = load1<S, C>(a.in, n, i, a.inv_scale);
        collide<C>(f, (C)a.omp, (C)a.omm, (C)a.gx, (C)a.gy);
    }
    if (a.sr) {
        const Rnd rnd = step_rnd(a, i);
        store8<S>(a.out, i, f + 1, a.scale, rnd);
        store1<S, C>(a.out, n, i, f[0], a.scale, rnd);
    } else {
        store8<S>(a.out, i, f + 1, a.scale);
        store1<S, C>(a.out, n, i, f[0], a.scale);
    }
}

template <int S, class CG, class C, int KQ, bool W16 = false>
__global__ void __launch_bounds__(256) k_step_pop_pd(const StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int self0;
    for_tiles(a, [&](int64_t tile) __attribute__((always_inline)) {
        stage_halo<pop_bytes<S>(), false>(a, tile, smem, &self0);
        const int64_t i = tile * blockDim.x + threadIdx.x;
        if (i < a.n) pop_node_pd<S, CG, C, KQ, W16>(a, (const void *)smem, i);
    });
}

template <int S, class CG, class C, int KQ, bool W16 = false>
__device__ __forceinline__ void fields_node_pd(const StepArgs &a, const void *src, int64_t i) {
    constexpr int K8Q = (KQ + 1) / 2;
    const int64_t n = a.n;
    const unsigned fl = a.flags[i];
    const unsigned bb = fl & 0xffu;
    C out[3];
    if (kind_of(fl) == MLBM_DIRICHLET) {
        out[0] = (C)a.bc[3 * i] - C(1);
        out[1] = (C)a.bc[3 * i + 1];
        out[2] = (C)a.bc[3 * i + 2];
    } else {
        constexpr bool kWsum = S == MLBM_F64;
        const C gx = (C)a.gx, gy = (C)a.gy;
        C own[3];
        load3<S>(a.in, i, own, a.inv_scale);
        C sum = feq_off<C>(0, C(1), own[0], C(1) + own[0], own[1], own[2]) +
                C(0.5) * force_k<C>(0, C(1), C(1) + own[0], own[1], own[2], gx, gy);
        C jx = C(0), jy = C(0);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            CG ar = CG(0), au = CG(0), av = CG(0), sw = CG(0);
            u4 lv;
            for_quads<0, KQ>([&](auto qc) __attribute__((always_inline)) {
                constexpr int q = decltype(qc)::value;
                int mi[4];
                members_pd(a, n, i, k * K8Q + (q >> 1), q & 1, lv, mi);
                CG wv[4];
                load_w4<S, KQ, W16>(a.w, n, i, k, q, wv, a.cached);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    CG m[3];
                    load3<S>(src, mi[j], m, a.inv_scale);
                    ar = fma(wv[j], m[0], ar);
                    au = fma(wv[j], m[1], au);
                    av = fma(wv[j], m[2], av);
                    if constexpr (kWsum) sw += wv[j];
                }
            });
            if constexpr (kWsum) ar += sw - CG(1);
            const C sg = ((bb >> k) & 1u) ? C(-1) : C(1);
            const C dr = (C)ar, uk = (C)au, vk = (C)av;
            const C rho = C(1) + dr;
            const C fk = feq_off<C>(k + 1, sg, dr, rho, uk, vk) + C(0.5) * force_k<C>(k + 1, sg, rho, uk, vk, gx, gy);
            sum += fk;
            jx += C(EX[k + 1]) * fk;
            jy += C(EY[k + 1]) * fk;
        }
        const C rho = C(1) + sum;
        out[0] = sum;
        out[1] = (jx + C(0.5) * rho * gx) / rho;
        out[2] = (jy + C(0.5) * rho * gy) / rho;
    }
    store3<S>(a.out, i, out, a.scale, step_rnd(a, i));
}

template <int S, class CG, class C, int KQ, bool W16 = false>
__global__ void __launch_bounds__(256) k_step_fields_pd(const StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int self0;
    for_tiles(a, [&](int64_t tile) __attribute__((always_inline)) {
        stage_halo<field_bytes<S>(), false>(a, tile, smem, &self0);
        const int64_t i = tile * blockDim.x + threadIdx.x;
        if (i < a.n) fields_node_pd<S, CG, C, KQ, W16>(a, (const void *)smem, i);
    });
}

// ---- initial state -----------------------------------------------------------------

struct InitArgs {
    int64_t n;
    const uint16_t *flags;
    const double *bc;
    const double *rho, *u;
    void *out;
    double omp, omm, gx, gy;
    float scale;
    int variant;
};

template <int S>
__global__ void __launch_bounds__(256) k_init(const InitArgs a) {
    using C = double;  // one-off: computed in FP64 and rounded once on store
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const bool dir = kind_of(a.flags[i]) == MLBM_DIRICHLET;
    const double r = dir ? a.bc[3 * i] : a.rho[i];
    const double ux = dir ? a.bc[3 * i + 1] : a.u[2 * i];
    const double uy = dir ? a.bc[3 * i + 2] : a.u[2 * i + 1];
    if (a.variant == MLBM_FIELDS) {
        C o[3] = {(C)(r - 1.0), (C)ux, (C)uy};
        store3<S>(a.out, i, o, a.scale);
        return;
    }
    C f[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = feq_off<C>(k, C(1), (C)(r - 1.0), (C)r, (C)ux, (C)uy);
    if (!dir) collide<C>(f, (C)a.omp, (C)a.omm, (C)a.gx, (C)a.gy);
    store8<S>(a.out, i, f + 1, a.scale);
    store1<S, C>(a.out, a.n, i, f[0], a.scale);
}

// ---- macroscopic fields and reductions ------------------------------------------------

constexpr int RED_BLOCK = 256;

struct MacroArgs {
    int64_t n;
    const int *idx;
    const void *w;
    const uint16_t *flags;
    const double *bc;
    const void *state;
    const double *area;
    double *rho_out, *u_out, *u_prev;
    double *ws;
    double gx, gy, inv_dx2;
    float inv_scale;
    int pd;  // idx holds one stencil per departure point: [8][Kp/4][n][4]
    int w16; // FP16 weights; their sum is then taken as 1, as the step does
};

// wave64 then workgroup tree sum in a fixed order; lane 0 of wave 0 holds the result
__device__ __forceinline__ double block_sum(double v, double *lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int t = 0; t < (int)(blockDim.x >> 6); ++t) s += lds[t];
    return s;
}
__device__ __forceinline__ double block_min(double v, double *lds) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    double s = v;
    if (threadIdx.x == 0)
        for (int t = 0; t < (int)(blockDim.x >> 6); ++t) s = fmin(s, lds[t]);
    return s;
}

template <int S, int V, int KQ>
__global__ void __launch_bounds__(RED_BLOCK) k_macro(const MacroArgs a) {
    using C = typename Fmt<S>::C;
    __shared__ double lds[RED_BLOCK / 64];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[MLBM_RED_FIRST_BAD + 1] = {0, 0, 0, 0, 0, 0, 0, 0, 0, (double)a.n};
    if (i < a.n) {
        const int64_t n = a.n;
        const unsigned fl = a.flags[i];
        const unsigned bb = fl & 0xffu;
        const bool dir = kind_of(fl) == MLBM_DIRICHLET;
        double rho, ux, uy;
        C f[9];
        C m[3];
        if constexpr (V == MLBM_POPULATIONS) {
            load8<S>(a.state, i, f + 1, a.inv_scale);
            f[0] = load1<S, C>(a.state, n, i, a.inv_scale);
            double dr = 0, jx = 0, jy = 0;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                dr += (double)f[k];
                jx += EX[k] * (double)f[k];
                jy += EY[k] * (double)f[k];
            }
            rho = 1.0 + dr;
            ux = jx / rho - 0.5 * a.gx;
            uy = jy / rho - 0.5 * a.gy;
        } else {
            load3<S>(a.state, i, m, a.inv_scale);
            rho = 1.0 + (double)m[0];
            ux = (double)m[1];
            uy = (double)m[2];
        }
        if (dir) {
            rho = a.bc[3 * i];
            ux = a.bc[3 * i + 1];
            uy = a.bc[3 * i + 2];
        }
        if (a.rho_out) a.rho_out[i] = rho;
        if (a.u_out) {
            a.u_out[2 * i] = ux;
            a.u_out[2 * i + 1] = uy;
        }
        if (a.u_prev) {
            const double dx = ux - a.u_prev[2 * i], dy = uy - a.u_prev[2 * i + 1];
            v[MLBM_RED_NORM_DU2] = dx * dx + dy * dy;
            a.u_prev[2 * i] = ux;
            a.u_prev[2 * i + 1] = uy;
        }
        const double A = a.area[i];
        const double sp = sqrt(ux * ux + uy * uy);
        v[MLBM_RED_MASS] = A * rho;
        v[MLBM_RED_INT_UX] = A * ux;
        v[MLBM_RED_INT_UY] = A * uy;
        v[MLBM_RED_INT_SPEED] = A * sp;
        v[MLBM_RED_NORM_U2] = ux * ux + uy * uy;
        if (!(isfinite(rho) && isfinite(ux) && isfinite(uy) && rho > 0.0)) {
            v[MLBM_RED_N_BAD] = 1.0;
            v[MLBM_RED_FIRST_BAD] = (double)i;
        }
        if (bb && !dir) {
            // momentum exchange of every bounced pair (i, k): e_k' (f_k'^post + f_k^new) A / dx^2,
            // populations relative to the rest state (a uniform pressure exerts no net force)
            double Fx = 0, Fy = 0;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (!((bb >> k) & 1u)) continue;
                const int kp = OPP8[k];  // stored index of k'
                double fout, fback = 0;
                if constexpr (V == MLBM_POPULATIONS) {
                    fout = (double)f[kp + 1];
                    double s = 0, sw = 0;
                    for (int q = 0; q < KQ; ++q) {
                        const i4 id = load_idx4(a.idx, n, i, a.pd ? k * KQ + q : q);
                        C wv[4];
                        if (a.w16) load_w4<S, KQ, true>(a.w, n, i, k, q, wv);
                        else load_w4<S, KQ, false>(a.w, n, i, k, q, wv);
                        const int ids[4] = {id.x, id.y, id.z, id.w};
                        for (int j = 0; j < 4; ++j) {
                            C sj[8];
                            load8<S>(a.state, ids[j], sj, a.inv_scale);
                            s += (double)wv[j] * (double)sj[kp];
                            sw += (double)wv[j];
                        }
                    }
                    fback = s + (a.w16 ? 0.0 : (sw - 1.0) * (double)omega<double>(kp + 1));
                } else {
                    const double r0 = 1.0 + (double)m[0];
                    fout = feq_off<double>(kp + 1, 1.0, (double)m[0], r0, (double)m[1], (double)m[2]) +
                           0.5 * force_k<double>(kp + 1, 1.0, r0, (double)m[1], (double)m[2], a.gx, a.gy);
                    double ir = 0, iu = 0, iv = 0, sw = 0;
                    for (int q = 0; q < KQ; ++q) {
                        const i4 id = load_idx4(a.idx, n, i, a.pd ? k * KQ + q : q);
                        C wv[4];
                        if (a.w16) load_w4<S, KQ, true>(a.w, n, i, k, q, wv);
                        else load_w4<S, KQ, false>(a.w, n, i, k, q, wv);
                        const int ids[4] = {id.x, id.y, id.z, id.w};
                        for (int j = 0; j < 4; ++j) {
                            C mj[3];
                            load3<S>(a.state, ids[j], mj, a.inv_scale);
                            ir += (double)wv[j] * (double)mj[0];
                            iu += (double)wv[j] * (double)mj[1];
                            iv += (double)wv[j] * (double)mj[2];
                            sw += (double)wv[j];
                        }
                    }
                    const double rh = 1.0 + ir + (a.w16 ? 0.0 : sw - 1.0);
                    fback = feq_off<double>(kp + 1, 1.0, rh - 1.0, rh, iu, iv) +
                            0.5 * force_k<double>(kp + 1, 1.0, rh, iu, iv, a.gx, a.gy);
                }
                Fx += EX[kp + 1] * (fout + fback);
                Fy += EY[kp + 1] * (fout + fback);
            }
            v[MLBM_RED_FORCE_X] = A * a.inv_dx2 * Fx;
            v[MLBM_RED_FORCE_Y] = A * a.inv_dx2 * Fy;
        }
    }
    double *dst = a.ws + (int64_t)blockIdx.x * (MLBM_RED_FIRST_BAD + 1);
#pragma unroll
    for (int r = 0; r < MLBM_RED_FIRST_BAD; ++r) {
        const double s = block_sum(v[r], lds);
        if (threadIdx.x == 0) dst[r] = s;
    }
    const double mn = block_min(v[MLBM_RED_FIRST_BAD], lds);
    if (threadIdx.x == 0) dst[MLBM_RED_FIRST_BAD] = mn;
}

struct FinalArgs {
    const double *ws;   // per-block partials [nblocks][10]
    int64_t nblocks;
    double *out;        // [MLBM_RED_COUNT], read (previous INT_UX) and written
    double nu, gx, dx, box_area;
};

// sums the per-block partials in a fixed order, then the derived quantities
__global__ void __launch_bounds__(RED_BLOCK) k_reduce_final(const FinalArgs a) {
    __shared__ double lds[RED_BLOCK / 64];
    double r_[MLBM_RED_FIRST_BAD + 1];
    const double prev_ux = threadIdx.x == 0 ? a.out[MLBM_RED_INT_UX] : 0.0;
    for (int r = 0; r <= MLBM_RED_FIRST_BAD; ++r) {
        double s = r == MLBM_RED_FIRST_BAD ? INFINITY : 0.0;
        for (int64_t b = threadIdx.x; b < a.nblocks; b += blockDim.x) {
            const double x = a.ws[b * (MLBM_RED_FIRST_BAD + 1) + r];
            s = r == MLBM_RED_FIRST_BAD ? fmin(s, x) : s + x;
        }
        r_[r] = r == MLBM_RED_FIRST_BAD ? block_min(s, lds) : block_sum(s, lds);
    }
    if (threadIdx.x == 0) {
        for (int r = 0; r <= MLBM_RED_FIRST_BAD; ++r) a.out[r] = r_[r];
        const double u2 = r_[MLBM_RED_NORM_U2], ux = r_[MLBM_RED_INT_UX];
        a.out[MLBM_RED_RESIDUAL] = u2 > 0.0 ? sqrt(r_[MLBM_RED_NORM_DU2] / u2) : 0.0;
        a.out[MLBM_RED_PREV_INT_UX] = prev_ux;
        a.out[MLBM_RED_MEAN_CHANGE] = fabs(ux - prev_ux) / fabs(ux);
        a.out[MLBM_RED_PERMEABILITY] =
            (a.gx != 0.0 && a.box_area > 0.0) ? a.nu * (ux / a.box_area) / a.gx * a.dx * a.dx : NAN;
    }
}

__global__ void k_fill_nan(double *out, int count) {
    const int i = threadIdx.x;
    if (i < count) out[i] = NAN;
}

// ---- dispatch ---------------------------------------------------------------------------

int check_common(const mlbm_step_params *p, const mlbm_device_state *st) {
    using mlbm::fail;
    if (!p || !st) return fail(MLBM_ERR_ARG, "null pointer argument");
    if (st->n < 1 || st->n > (int64_t)INT32_MAX) return fail(MLBM_ERR_ARG, "node count %lld outside [1, 2^31)", (long long)st->n);
    if (st->K < 1 || st->K > 32) return fail(MLBM_ERR_ARG, "K=%d outside [1, 32]", st->K);
    if (p->variant != MLBM_POPULATIONS && p->variant != MLBM_FIELDS) return fail(MLBM_ERR_ARG, "bad variant %d", p->variant);
    if (p->storage < MLBM_F64 || p->storage > MLBM_BF16) return fail(MLBM_ERR_ARG, "bad storage %d", p->storage);
    if (!st->flags || !st->state[0] || !st->state[1]) return fail(MLBM_ERR_ARG, "null device buffer");
    if (st->cur != 0 && st->cur != 1) return fail(MLBM_ERR_ARG, "cur must be 0 or 1");
    if (p->variant == MLBM_POPULATIONS && !(p->tau_plus > 0.5 && p->tau_minus > 0.5))
        return fail(MLBM_ERR_ARG, "relaxation times must exceed 1/2");
    if (p->storage == MLBM_F16S && (p->scale_exp < -30 || p->scale_exp > 30)) return fail(MLBM_ERR_ARG, "scale_exp out of range");
    if (st->w_lagrange && st->K < 10) return fail(MLBM_ERR_ARG, "block weights need stencils of K >= 10");
    if (p->weights16 != 0 && p->weights16 != 1) return fail(MLBM_ERR_ARG, "weights16 must be 0 or 1");
    if (p->weights16 && p->storage != MLBM_F16S && p->storage != MLBM_BF16)
        return fail(MLBM_ERR_UNSUPPORTED, "FP16 weights go with 16-bit states only");
    if (p->fp32_arith)
        return fail(MLBM_ERR_UNSUPPORTED, "FP32 collision arithmetic is not offered (it drifts above the FP32 "
                                          "bar over long runs); FP32 states collide in FP64 registers");
    return MLBM_OK;
}

int storage_bytes(int storage) { return storage == MLBM_F64 ? 8 : storage == MLBM_F32 ? 4 : 2; }

int block_of(const mlbm_step_params *p) {
    const int b = p->block == 0 ? 256 : p->block;
    return b;
}

template <int S, class CG, class C, bool W16 = false>
StepFn pick_step(int variant, int kq, bool lds) {
#define MLBM_CASE(Q)                                                                            \
    case Q:                                                                                     \
        if (lds)                                                                                \
            return variant == MLBM_POPULATIONS ? (StepFn)k_step_pop<S, CG, C, Q, true, W16>     \
                                               : (StepFn)k_step_fields<S, CG, C, Q, true, W16>; \
        return variant == MLBM_POPULATIONS ? (StepFn)k_step_pop<S, CG, C, Q, false, W16>        \
                                           : (StepFn)k_step_fields<S, CG, C, Q, false, W16>;
    switch (kq) {
        MLBM_CASE(0)
        MLBM_CASE(2)
        MLBM_CASE(3)
        MLBM_CASE(4)
        MLBM_CASE(5)
        MLBM_CASE(6)
        MLBM_CASE(7)
        MLBM_CASE(8)
        default:
            return nullptr;
    }
#undef MLBM_CASE
}

// FP32 state: the interpolation sums run in FP32 and the collision in FP64.
// The FP32 rounding drift of a long run comes from the collision (the
// interpolation in FP32 adds nothing measurable), and the FP64 collision costs
// little in a kernel bound by memory traffic.  16-bit states use FP32
// throughout.
template <int S, class CG, class C, bool W16 = false>
StepFn pick_step_pd(int variant, int kq) {
#define MLBM_CASE(Q)                                                                              \
    case Q:                                                                                       \
        return variant == MLBM_POPULATIONS ? (StepFn)k_step_pop_pd<S, CG, C, Q, W16>              \
                                           : (StepFn)k_step_fields_pd<S, CG, C, Q, W16>;
    switch (kq) {
        MLBM_CASE(2)
        MLBM_CASE(3)
        MLBM_CASE(4)
        MLBM_CASE(5)
        MLBM_CASE(6)
        MLBM_CASE(7)
        MLBM_CASE(8)
        default:
            return nullptr;
    }
#undef MLBM_CASE
}

// per-departure stencils: the same arithmetic choices as pick_step_any
StepFn pick_step_pd_any(int storage, int variant, int kq, int w16) {
    switch (storage) {
        case MLBM_F64: return pick_step_pd<MLBM_F64, double, double>(variant, kq);
        case MLBM_F32: return pick_step_pd<MLBM_F32, float, double>(variant, kq);
        case MLBM_F16S:
            return w16 ? pick_step_pd<MLBM_F16S, float, float, true>(variant, kq)
                       : pick_step_pd<MLBM_F16S, float, float>(variant, kq);
        case MLBM_BF16:
            return w16 ? pick_step_pd<MLBM_BF16, float, float, true>(variant, kq)
                       : pick_step_pd<MLBM_BF16, float, float>(variant, kq);
    }
    return nullptr;
}

// w16: FP16 weights (16-bit states; block-centre launches, kq = 0, read no
// per-node weights and take w16 = 0)
StepFn pick_step_any(int storage, int variant, int kq, bool lds, int w16) {
    switch (storage) {
        case MLBM_F64: return pick_step<MLBM_F64, double, double>(variant, kq, lds);
        case MLBM_F32: return pick_step<MLBM_F32, float, double>(variant, kq, lds);
        case MLBM_F16S:
            return w16 && kq ? pick_step<MLBM_F16S, float, float, true>(variant, kq, lds)
                             : pick_step<MLBM_F16S, float, float>(variant, kq, lds);
        case MLBM_BF16:
            return w16 && kq ? pick_step<MLBM_BF16, float, float, true>(variant, kq, lds)
                             : pick_step<MLBM_BF16, float, float>(variant, kq, lds);
    }
    return nullptr;
}

// hybrid sets with tiles in one launch (kq >= 2: the per-node part)
template <int S, class CG, class C, bool W16 = false>
StepFn pick_step_hyb(int variant, int kq) {
#define MLBM_CASE(Q)                                                                              \
    case Q:                                                                                       \
        return variant == MLBM_POPULATIONS ? (StepFn)k_step_pop_hyb<S, CG, C, Q, W16>             \
                                           : (StepFn)k_step_fields_hyb<S, CG, C, Q, W16>;
    switch (kq) {
        MLBM_CASE(2)
        MLBM_CASE(3)
        MLBM_CASE(4)
        MLBM_CASE(5)
        MLBM_CASE(6)
        MLBM_CASE(7)
        MLBM_CASE(8)
        default:
            return nullptr;
    }
#undef MLBM_CASE
}

StepFn pick_step_hyb_any(int storage, int variant, int kq, int w16) {
    switch (storage) {
        case MLBM_F64: return pick_step_hyb<MLBM_F64, double, double>(variant, kq);
        case MLBM_F32: return pick_step_hyb<MLBM_F32, float, double>(variant, kq);
        case MLBM_F16S:
            return w16 ? pick_step_hyb<MLBM_F16S, float, float, true>(variant, kq)
                       : pick_step_hyb<MLBM_F16S, float, float>(variant, kq);
        case MLBM_BF16:
            return w16 ? pick_step_hyb<MLBM_BF16, float, float, true>(variant, kq)
                       : pick_step_hyb<MLBM_BF16, float, float>(variant, kq);
    }
    return nullptr;
}

using MacroFn = void (*)(const MacroArgs);

template <int S>
MacroFn pick_macro(int variant, int kq) {
#define MLBM_CASE(Q)                                                        \
    case Q:                                                                 \
        return variant == MLBM_POPULATIONS ? (MacroFn)k_macro<S, MLBM_POPULATIONS, Q> : (MacroFn)k_macro<S, MLBM_FIELDS, Q>;
    switch (kq) {
        MLBM_CASE(2)
        MLBM_CASE(3)
        MLBM_CASE(4)
        MLBM_CASE(5)
        MLBM_CASE(6)
        MLBM_CASE(7)
        MLBM_CASE(8)
        default:
            return nullptr;
    }
#undef MLBM_CASE
}

MacroFn pick_macro_any(int storage, int variant, int kq) {
    switch (storage) {
        case MLBM_F64: return pick_macro<MLBM_F64>(variant, kq);
        case MLBM_F32: return pick_macro<MLBM_F32>(variant, kq);
        case MLBM_F16S: return pick_macro<MLBM_F16S>(variant, kq);
        case MLBM_BF16: return pick_macro<MLBM_BF16>(variant, kq);
    }
    return nullptr;
}

int hip_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mlbm::fail(MLBM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
    return MLBM_OK;
}

// ---- graph cache of mlbm_step -----------------------------------------------------------
// Every argument a replay depends on; the bytes of StepArgs are zeroed before
// they are filled, so equal launches give equal keys.
struct GraphKey {
    unsigned char args[sizeof(StepArgs)];
    const void *fn0, *fn1;
    int64_t ranges[2][2];
    int64_t shmem;
    int32_t blk, gsteps, cur, device;
    void *stream;
};

constexpr int kGraphCacheSize = 16;
std::mutex g_graph_mutex;
struct GraphEntry {
    GraphKey key;
    hipGraphExec_t exec;
    uint64_t used;
};
GraphEntry g_graphs[kGraphCacheSize];
int g_graph_count = 0;
uint64_t g_graph_clock = 0;

hipGraphExec_t graph_cache_find(const GraphKey &k) {
    std::lock_guard<std::mutex> lock(g_graph_mutex);
    for (int i = 0; i < g_graph_count; ++i)
        if (std::memcmp(&g_graphs[i].key, &k, sizeof(k)) == 0) {
            g_graphs[i].used = ++g_graph_clock;
            return g_graphs[i].exec;
        }
    return nullptr;
}

// keeps exec; the least recently used entry is destroyed when the cache is full
void graph_cache_put(const GraphKey &k, hipGraphExec_t exec) {
    std::lock_guard<std::mutex> lock(g_graph_mutex);
    int slot = g_graph_count;
    if (g_graph_count == kGraphCacheSize) {
        slot = 0;
        for (int i = 1; i < kGraphCacheSize; ++i)
            if (g_graphs[i].used < g_graphs[slot].used) slot = i;
        (void)hipGraphExecDestroy(g_graphs[slot].exec);  // eviction: a failure here changes nothing for the caller
    } else {
        ++g_graph_count;
    }
    g_graphs[slot].key = k;
    g_graphs[slot].exec = exec;
    g_graphs[slot].used = ++g_graph_clock;
}

}  // namespace

extern "C" int mlbm_init_state(const mlbm_step_params *p, mlbm_device_state *st, const double *rho,
                               const double *u, void *stream) {
    using mlbm::fail;
    mlbm::clear_error();
    int rc = check_common(p, st);
    if (rc) return rc;
    if (!rho || !u) return fail(MLBM_ERR_ARG, "null field pointer");
    InitArgs a;
    a.n = st->n;
    a.flags = st->flags;
    a.bc = st->bc;
    a.rho = rho;
    a.u = u;
    a.out = st->state[st->cur];
    a.omp = 1.0 / p->tau_plus;
    a.omm = 1.0 / p->tau_minus;
    a.gx = p->g[0];
    a.gy = p->g[1];
    a.scale = std::ldexp(1.0f, p->scale_exp);
    a.variant = p->variant;
    const int blk = 256;
    const dim3 grid((unsigned)((st->n + blk - 1) / blk));
    hipStream_t s = (hipStream_t)stream;
    switch (p->storage) {
        case MLBM_F64: hipLaunchKernelGGL(k_init<MLBM_F64>, grid, dim3(blk), 0, s, a); break;
        case MLBM_F32: hipLaunchKernelGGL(k_init<MLBM_F32>, grid, dim3(blk), 0, s, a); break;
        case MLBM_F16S: hipLaunchKernelGGL(k_init<MLBM_F16S>, grid, dim3(blk), 0, s, a); break;
        case MLBM_BF16: hipLaunchKernelGGL(k_init<MLBM_BF16>, grid, dim3(blk), 0, s, a); break;
    }
    return hip_check("mlbm_init_state launch");
}

extern "C" int mlbm_step(const mlbm_step_params *p, mlbm_device_state *st, int32_t nsteps, void *stream) {
    using mlbm::fail;
    mlbm::clear_error();
    int rc = check_common(p, st);
    if (rc) return rc;
    if (nsteps < 0) return fail(MLBM_ERR_ARG, "nsteps must be >= 0");
    if (!st->idx || !st->w) return fail(MLBM_ERR_ARG, "null stencil buffer");
    const bool lds = st->tile != 0;
    const int blk0 = lds ? st->tile : block_of(p);
    if (blk0 != 64 && blk0 != 128 && blk0 != 256) return fail(MLBM_ERR_ARG, "block / tile must be 64, 128 or 256");
    const int lanes = p->lanes_per_node == 0 ? 1 : p->lanes_per_node;
    if (lanes != 1 && lanes != 8) return fail(MLBM_ERR_ARG, "lanes_per_node must be 0, 1 or 8");
    if (lanes == 8) {
        if (st->w_lagrange && (!lds || p->hybrid_launches != 0))
            return fail(MLBM_ERR_UNSUPPORTED, "eight lanes per node on a hybrid set: one launch per step with tiles only");
        if (st->per_departure) return fail(MLBM_ERR_UNSUPPORTED, "eight lanes per node: not for per-departure stencils");
        if (lds && st->tile > 128)
            return fail(MLBM_ERR_UNSUPPORTED, "eight lanes per node need tiles of 64 or 128 nodes (8 x tile <= 1024 lanes)");
    }
    // blk: nodes per workgroup; threads: lanes per workgroup
    const int blk = lanes == 8 && !lds ? blk0 / 8 : blk0;
    const int threads = lanes == 8 && lds ? 8 * blk0 : blk0;
    const int kq = (st->K + 3) / 4;
    size_t shmem = 0;
    if (lds) {
        if (!st->halo_off || !st->halo || !st->lidx) return fail(MLBM_ERR_ARG, "null tile buffer");
        const int ts = storage_bytes(p->storage);
        const int nb = p->variant == MLBM_POPULATIONS ? 8 * ts : 4 * ts;
        if (st->max_halo < 1) return fail(MLBM_ERR_ARG, "max_halo must be positive");
        shmem = (size_t)st->max_halo * nb;
        if (shmem > 65536)
            return fail(MLBM_ERR_UNSUPPORTED, "halo of %d nodes needs %zu bytes of LDS (> 64 KiB); use tile 0 or a smaller tile",
                        st->max_halo, shmem);
    }
    if (st->per_departure && !lds) return fail(MLBM_ERR_UNSUPPORTED, "per-departure stencils need tiles");
    if (st->per_departure && st->w_lagrange) return fail(MLBM_ERR_ARG, "per-departure stencils take no block weights");
    StepFn fn = lanes == 8          ? pick_step_lanes_any(p->storage, p->variant, kq, lds, p->weights16)
                : st->per_departure ? pick_step_pd_any(p->storage, p->variant, kq, p->weights16)
                                    : pick_step_any(p->storage, p->variant, kq, lds, p->weights16);
    if (!fn) return fail(MLBM_ERR_UNSUPPORTED, "no kernel for storage %d, variant %d, K=%d", p->storage, p->variant, st->K);
    if (p->variant == MLBM_FIELDS && (p->tau_plus != 1.0 || p->tau_minus != 1.0))
        return fail(MLBM_ERR_ARG, "the fields variant fixes tau = 1");
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n = st->n;
    a.idx = (const int *)st->idx;
    a.w = st->w;
    a.flags = st->flags;
    a.bc = st->bc;
    a.omp = 1.0 / p->tau_plus;
    a.omm = 1.0 / p->tau_minus;
    a.gx = p->g[0];
    a.gy = p->g[1];
    a.scale = std::ldexp(1.0f, p->scale_exp);
    a.inv_scale = std::ldexp(1.0f, -p->scale_exp);
    a.xcd = p->xcd_remap ? 1 : 0;
    a.cached = p->cached_weights ? 1 : 0;
    a.halo_off = st->halo_off;
    a.halo = st->halo;
    a.lidx = st->lidx;
    a.wl = st->w_lagrange;
    a.queue = nullptr;
    a.queue_range = nullptr;
    a.group = 0;
    // nodes [0, lag0) run the per-node weights; in a hybrid set the trailing
    // block centres [lag0, n) run the block-centre kernel.  Each launch covers
    // the tiles holding its nodes, so a tile holding both kinds is visited by
    // both launches, each updating only its own nodes
    const int64_t nb = (st->n + blk - 1) / blk;
    int64_t lag0 = st->n;
    StepFn fb = nullptr;
    if (st->w_lagrange && st->lagrange_begin < st->n) {
        if (st->lagrange_begin < 0) return fail(MLBM_ERR_ARG, "lagrange_begin must be >= 0");
        lag0 = st->lagrange_begin;
        fb = pick_step_any(p->storage, p->variant, 0, lds, 0);
        if (!fb) return fail(MLBM_ERR_UNSUPPORTED, "no block-centre kernel for storage %d", p->storage);
    }
    a.lag0 = lag0;
    const int64_t ranges[2][2] = {{0, (lag0 + blk - 1) / blk}, {lag0 / blk, fb ? nb : 0}};
    StepFn fns[2] = {fn, fb};
    if (p->hybrid_launches != 0 && p->hybrid_launches != 2) return fail(MLBM_ERR_ARG, "hybrid_launches must be 0 or 2");
    // one launch for both node kinds: the per-node tiles' workgroups first (the
    // longer ones), then the block-centre tiles'
    const bool fuse = fb && lds && p->hybrid_launches == 0 && ranges[0][1] > 0;
    a.split = 0;
    a.tile0b = a.tile1b = a.grid8b = 0;
    if (lanes == 8 && fb && !fuse)
        return fail(MLBM_ERR_UNSUPPORTED, "eight lanes per node on a hybrid set needs nodes with per-node weights");
    if (fuse) {
        fns[0] = lanes == 8 ? pick_step_lanes_hyb_any(p->storage, p->variant, kq, p->weights16)
                            : pick_step_hyb_any(p->storage, p->variant, kq, p->weights16);
        if (!fns[0]) return fail(MLBM_ERR_UNSUPPORTED, "no hybrid kernel for storage %d, K=%d", p->storage, st->K);
        fns[1] = nullptr;
        const int64_t cb = ranges[1][1] - ranges[1][0];
        a.tile0b = ranges[1][0];
        a.tile1b = ranges[1][1];
        a.grid8b = p->xcd_remap ? (cb + 7) / 8 * 8 : cb;
    }
    hipStream_t s = (hipStream_t)stream;
    a.sr = (p->stochastic_rounding && (p->storage == MLBM_F16S || p->storage == MLBM_BF16)) ? 1 : 0;
    const int gsteps = p->graph_steps;
    if (gsteps != 0 && (gsteps < 2 || gsteps > 4096 || (gsteps & 1)))
        return fail(MLBM_ERR_ARG, "graph_steps must be 0 or an even number in [2, 4096]");
    if (gsteps && a.sr)
        return fail(MLBM_ERR_UNSUPPORTED, "graph replay with stochastic rounding (its random bits change every step)");
    if (gsteps && !stream) return fail(MLBM_ERR_ARG, "graph replay needs a stream other than the default stream");
    // one step: the launches of its tile ranges (direct, or recorded while capturing)
    auto launch_step = [&]() -> int {
        a.in = st->state[st->cur];
        a.out = st->state[st->cur ^ 1];
        a.reverse = p->alternate_sweeps && st->cur == 1;
        const uint64_t step = st->step_count++;
        a.seed = a.sr ? mix32((unsigned)step ^ mix32((unsigned)(step >> 32) + 0x6a09e667u)) : 0u;
        for (int r = 0; r < 2; ++r) {
            const int64_t cnt = ranges[r][1] - ranges[r][0];
            if (cnt <= 0) continue;
            if (!fns[r]) continue;
            a.tile0 = ranges[r][0];
            a.tile1 = ranges[r][1];
            a.grid8 = a.xcd ? (cnt + 7) / 8 * 8 : cnt;
            if (fuse) a.split = a.grid8;
            hipLaunchKernelGGL(fns[r], dim3((unsigned)(a.grid8 + a.grid8b)), dim3(threads), shmem, s, a);
        }
        const int rc_ = hip_check("mlbm_step launch");
        if (rc_) return rc_;
        st->cur ^= 1;
        return MLBM_OK;
    };
    int32_t left = nsteps;
    if (gsteps && nsteps >= gsteps) {
        // gsteps steps (even: cur comes back to its value) as one graph, captured on
        // first use and kept for later calls that would launch the same kernels
        // with the same arguments; replays cover whole multiples of gsteps
        GraphKey key;
        std::memset(&key, 0, sizeof(key));
        a.in = st->state[st->cur];
        a.out = st->state[st->cur ^ 1];
        a.reverse = p->alternate_sweeps && st->cur == 1;
        a.seed = 0;
        std::memcpy(key.args, &a, sizeof(a));
        key.fn0 = (const void *)fns[0];
        key.fn1 = (const void *)fns[1];
        std::memcpy(key.ranges, ranges, sizeof(ranges));
        key.blk = threads;
        key.shmem = (int64_t)shmem;
        key.gsteps = gsteps;
        key.stream = stream;
        key.cur = st->cur;
        if (hipGetDevice(&key.device) != hipSuccess) return hip_check("hipGetDevice");
        hipGraphExec_t exec = graph_cache_find(key);
        if (!exec) {
            const int cur0 = st->cur;
            const uint64_t count0 = st->step_count;
            if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return hip_check("mlbm_step: hipStreamBeginCapture");
            int rcc = MLBM_OK;
            for (int t = 0; t < gsteps && rcc == MLBM_OK; ++t) rcc = launch_step();
            hipGraph_t graph = nullptr;
            const hipError_t ec = hipStreamEndCapture(s, &graph);
            st->cur = cur0;
            st->step_count = count0;
            if (rcc) {
                if (graph) (void)hipGraphDestroy(graph);  // the launch error is the one reported
                return rcc;
            }
            if (ec != hipSuccess || !graph) return fail(MLBM_ERR_HIP, "mlbm_step: hipStreamEndCapture: %s", hipGetErrorString(ec));
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);  // the executable graph does not need it
            if (ei != hipSuccess) return fail(MLBM_ERR_HIP, "mlbm_step: hipGraphInstantiate: %s", hipGetErrorString(ei));
            graph_cache_put(key, exec);
        }
        const int32_t reps = nsteps / gsteps;
        for (int32_t r = 0; r < reps; ++r)
            if (hipGraphLaunch(exec, s) != hipSuccess) return hip_check("mlbm_step: hipGraphLaunch");
        st->step_count += (uint64_t)reps * (uint64_t)gsteps;
        left = nsteps - reps * gsteps;
    }
    for (int32_t t = 0; t < left; ++t) {
        rc = launch_step();
        if (rc) return rc;
    }
    return MLBM_OK;
}

constexpr int RED_PARTIALS = MLBM_RED_FIRST_BAD + 1;  // per-block partial sums

extern "C" int64_t mlbm_reduction_workspace_bytes(int64_t n) {
    if (n < 1) return 0;
    return ((n + RED_BLOCK - 1) / RED_BLOCK) * RED_PARTIALS * (int64_t)sizeof(double);
}

extern "C" int mlbm_reductions_reset(double *red_out, void *stream) {
    mlbm::clear_error();
    if (!red_out) return mlbm::fail(MLBM_ERR_ARG, "null red_out");
    hipLaunchKernelGGL(k_fill_nan, dim3(1), dim3(64), 0, (hipStream_t)stream, red_out, (int)MLBM_RED_COUNT);
    return hip_check("mlbm_reductions_reset launch");
}

namespace {

// the launches of mlbm_macroscopic with the per-block partials in ws
int macro_launch(const mlbm_step_params *p, const mlbm_device_state *st, const double *area, double dx,
                 double box_area, double *rho_out, double *u_out, double *u_prev, double *ws, double *red_out,
                 hipStream_t s) {
    using mlbm::fail;
    const int kq = (st->K + 3) / 4;
    MacroFn fn = pick_macro_any(p->storage, p->variant, kq);
    if (!fn) return fail(MLBM_ERR_UNSUPPORTED, "no macroscopic kernel for storage %d, K=%d", p->storage, st->K);
    MacroArgs a;
    a.n = st->n;
    a.idx = (const int *)st->idx;
    a.pd = st->per_departure ? 1 : 0;
    a.w = st->w;
    a.flags = st->flags;
    a.bc = st->bc;
    a.state = st->state[st->cur];
    a.area = area;
    a.rho_out = rho_out;
    a.u_out = u_out;
    a.u_prev = u_prev;
    a.ws = ws;
    a.gx = p->g[0];
    a.gy = p->g[1];
    a.inv_dx2 = 1.0 / (dx * dx);
    a.inv_scale = std::ldexp(1.0f, -p->scale_exp);
    a.w16 = p->weights16 ? 1 : 0;
    const int64_t nb = (st->n + RED_BLOCK - 1) / RED_BLOCK;
    hipLaunchKernelGGL(fn, dim3((unsigned)nb), dim3(RED_BLOCK), 0, s, a);
    int rc = hip_check("mlbm_macroscopic launch");
    if (rc) return rc;
    FinalArgs fa;
    fa.ws = ws;
    fa.nblocks = nb;
    fa.out = red_out;
    fa.nu = (p->tau_plus - 0.5) / 3.0;
    fa.gx = p->g[0];
    fa.dx = dx;
    fa.box_area = box_area;
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(RED_BLOCK), 0, s, fa);
    return hip_check("mlbm_macroscopic reduction launch");
}

int macro_check(const mlbm_step_params *p, const mlbm_device_state *st, const double *area, double dx,
                const double *red_out) {
    using mlbm::fail;
    int rc = check_common(p, st);
    if (rc) return rc;
    if (!area || !red_out) return fail(MLBM_ERR_ARG, "null area or output");
    if (!st->idx || !st->w) return fail(MLBM_ERR_ARG, "null stencil buffer");
    if (!(dx > 0.0)) return fail(MLBM_ERR_ARG, "dx must be positive");
    return MLBM_OK;
}

}  // namespace

extern "C" int mlbm_macroscopic(const mlbm_step_params *p, const mlbm_device_state *st, const double *area,
                                double dx, double box_area, double *rho_out, double *u_out, double *u_prev,
                                void *workspace, double *red_out, void *stream) {
    mlbm::clear_error();
    int rc = macro_check(p, st, area, dx, red_out);
    if (rc) return rc;
    if (!workspace) return mlbm::fail(MLBM_ERR_ARG, "null workspace");
    return macro_launch(p, st, area, dx, box_area, rho_out, u_out, u_prev, (double *)workspace, red_out,
                        (hipStream_t)stream);
}

// ---- allocation-free reductions ----------------------------------------------------------
// The per-block partial sums of mlbm_macroscopic_static live in this
// file-scope device array (one copy per GPU, held until the process ends).
// Host code never passes its name to a kernel: the name is a host-side
// stand-in, so each device's address is looked up once with
// hipGetSymbolAddress and kept per device.  Every block writes all of its
// partials before the final sum reads them, so nothing needs clearing.

static __device__ __align__(256) double scratch[(MLBM_STATIC_MAX_NODES / RED_BLOCK) * RED_PARTIALS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

// the current device's address of `scratch`, looked up on its first use
int scratch_ptr(double **out) {
    using mlbm::fail;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return hip_check("hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MLBM_ERR_ARG, "device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(MLBM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = (double *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return MLBM_OK;
}

}  // namespace

extern "C" int mlbm_macroscopic_static(const mlbm_step_params *p, const mlbm_device_state *st, const double *area,
                                       double dx, double box_area, double *rho_out, double *u_out, double *u_prev,
                                       double *red_out, void *stream) {
    mlbm::clear_error();
    int rc = macro_check(p, st, area, dx, red_out);
    if (rc) return rc;
    if (st->n > MLBM_STATIC_MAX_NODES)
        return mlbm::fail(MLBM_ERR_ARG, "n = %lld exceeds the %lld nodes of the static reduction buffer; "
                                        "use mlbm_macroscopic with a workspace", (long long)st->n,
                          (long long)MLBM_STATIC_MAX_NODES);
    double *ws = nullptr;
    rc = scratch_ptr(&ws);
    if (rc) return rc;
    return macro_launch(p, st, area, dx, box_area, rho_out, u_out, u_prev, ws, red_out, (hipStream_t)stream);
}

extern "C" int mlbm_run_to_steady(const mlbm_step_params *p, mlbm_device_state *st, const mlbm_steady *sp,
                                  const double *area, double dx, double box_area, double *u_prev, void *workspace,
                                  double *red_out, double *red_host, int64_t *steps_done, void *stream) {
    using mlbm::fail;
    mlbm::clear_error();
    if (!sp || !red_host || !steps_done || !u_prev) return fail(MLBM_ERR_ARG, "null steady, red_host, steps_done or u_prev");
    if (sp->criterion != MLBM_STEADY_FIELD && sp->criterion != MLBM_STEADY_MEAN)
        return fail(MLBM_ERR_ARG, "bad criterion %d", sp->criterion);
    if (sp->check_every < 1 || sp->hold < 1 || sp->max_steps < 0 || !(sp->tol > 0.0))
        return fail(MLBM_ERR_ARG, "check_every and hold must be >= 1, max_steps >= 0, tol > 0");
    *steps_done = 0;
    hipStream_t s = (hipStream_t)stream;
    int rc = mlbm_reductions_reset(red_out, stream);
    if (rc) return rc;
    rc = mlbm_macroscopic(p, st, area, dx, box_area, nullptr, nullptr, u_prev, workspace, red_out, stream);
    if (rc) return rc;
    const int slot = sp->criterion == MLBM_STEADY_FIELD ? MLBM_RED_RESIDUAL : MLBM_RED_MEAN_CHANGE;
    int64_t steps = 0;
    int below = 0;
    while (steps < sp->max_steps) {
        const int32_t chunk = (int32_t)std::min<int64_t>(sp->check_every, sp->max_steps - steps);
        rc = mlbm_step(p, st, chunk, stream);
        if (rc) return rc;
        steps += chunk;
        *steps_done = steps;
        rc = mlbm_macroscopic(p, st, area, dx, box_area, nullptr, nullptr, u_prev, workspace, red_out, stream);
        if (rc) return rc;
        if (hipMemcpyAsync(red_host, red_out, MLBM_RED_COUNT * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return hip_check("mlbm_run_to_steady: reading the reductions");
        if (red_host[MLBM_RED_N_BAD] > 0.0)
            return fail(MLBM_ERR_UNSTABLE, "unstable after %lld steps: %.0f nodes with non-finite fields or rho <= 0, "
                                           "first node %.0f", (long long)steps, red_host[MLBM_RED_N_BAD],
                        red_host[MLBM_RED_FIRST_BAD]);
        below = red_host[slot] < sp->tol ? below + 1 : 0;
        if (below >= sp->hold) break;
    }
    return MLBM_OK;
}

// ---- batched runs: many samples in one node range ------------------------------------
//
// Samples are concatenated so that every tile (workgroup of `tile` nodes) lies
// in one sample.  A device list of active tiles drives persistent step
// kernels; every check_every steps a per-tile pass accumulates the velocity
// change since the last check, and one workgroup retires converged samples and
// rebuilds the list.  check_every is even, so every check sees the same state
// buffer and a retired sample's final state stays there.

namespace {

struct BatchArgs {
    int64_t n;
    const uint16_t *flags;
    const double *bc;
    const void *state;
    const double *area;
    double *u_prev;
    double *tile_red;
    const int *queue;
    int *counters;
    const int *tile_off;
    int n_samples;
    int n_groups;                // sample groups run one after another within a check
    const int *group_sample_off; // [n_groups + 1] samples of each group
    int *group_queue_off;        // [n_groups + 1] queue range of each group (device)
    int *sample_steps;
    double *sample_res;
    double *sample_ux;
    double gx, gy, tol;
    float inv_scale;
    int check_every;
    int64_t ntiles;
};

constexpr int BATCH_RED = 4;  // du2, u2, sum A u_x, bad nodes

template <int S, int V>
__global__ void __launch_bounds__(256) k_batch_tile_red(const BatchArgs a) {
    __shared__ double lds[256 / 64];
    const int na = a.counters[0];
    for (int c = blockIdx.x; c < na; c += gridDim.x) {
        const int64_t tile = a.queue[c];
        const int64_t i = tile * blockDim.x + threadIdx.x;
        double v[BATCH_RED] = {0, 0, 0, 0};
        if (i < a.n) {
            double rho, ux, uy;
            if constexpr (V == MLBM_POPULATIONS) {
                double f[9];
                load8<S>(a.state, i, f + 1, a.inv_scale);
                f[0] = load1<S, double>(a.state, a.n, i, a.inv_scale);
                double dr = 0, jx = 0, jy = 0;
                for (int k = 0; k < 9; ++k) {
                    dr += (double)f[k];
                    jx += EX[k] * (double)f[k];
                    jy += EY[k] * (double)f[k];
                }
                rho = 1.0 + dr;
                ux = jx / rho - 0.5 * a.gx;
                uy = jy / rho - 0.5 * a.gy;
            } else {
                double m[3];
                load3<S>(a.state, i, m, a.inv_scale);
                rho = 1.0 + m[0];
                ux = m[1];
                uy = m[2];
            }
            if (kind_of(a.flags[i]) == MLBM_DIRICHLET) {
                rho = a.bc[3 * i];
                ux = a.bc[3 * i + 1];
                uy = a.bc[3 * i + 2];
            }
            const double dx = ux - a.u_prev[2 * i], dy = uy - a.u_prev[2 * i + 1];
            a.u_prev[2 * i] = ux;
            a.u_prev[2 * i + 1] = uy;
            v[0] = dx * dx + dy * dy;
            v[1] = ux * ux + uy * uy;
            v[2] = a.area[i] * ux;
            v[3] = (isfinite(rho) && isfinite(ux) && isfinite(uy) && rho > 0.0) ? 0.0 : 1.0;
        }
        for (int r = 0; r < BATCH_RED; ++r) {
            const double s = block_sum(v[r], lds);
            if (threadIdx.x == 0) a.tile_red[tile * BATCH_RED + r] = s;
        }
    }
}

constexpr int MAX_SAMPLES = 4096;

// one workgroup: per-sample residual, retirement, new active tile list
// One workgroup per sample: the sample's residual from its tiles' partial
// sums, added in a fixed order (strided per thread, then a tree), and its
// retirement.
__global__ void __launch_bounds__(256) k_batch_sample_red(const BatchArgs a, int mark) {
    __shared__ double part[BATCH_RED][256];
    const int s = blockIdx.x;
    if (a.sample_steps[s] != 0) return;  // uniform over the workgroup
    double r[BATCH_RED] = {0, 0, 0, 0};
    for (int t = a.tile_off[s] + (int)threadIdx.x; t < a.tile_off[s + 1]; t += blockDim.x)
        for (int q = 0; q < BATCH_RED; ++q) r[q] += a.tile_red[(int64_t)t * BATCH_RED + q];
    for (int q = 0; q < BATCH_RED; ++q) part[q][threadIdx.x] = r[q];
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < BATCH_RED; ++q) part[q][threadIdx.x] += part[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double du2 = part[0][0], u2 = part[1][0];
    const double res = u2 > 0.0 ? sqrt(du2 / u2) : (du2 > 0.0 ? INFINITY : 0.0);
    a.sample_res[s] = res;
    a.sample_ux[s] = part[2][0];
    if (!mark) return;
    const int steps = a.counters[1] + a.check_every;
    if (part[3][0] > 0.0 || !isfinite(res)) a.sample_steps[s] = -steps;
    else if (res < a.tol) a.sample_steps[s] = steps;
}

// Rebuilds the list of active tiles and the groups' queue ranges.
__global__ void __launch_bounds__(256) k_batch_retire(const BatchArgs a, int mark) {
    __shared__ int start[MAX_SAMPLES];
    __shared__ int total, active;
    const int steps = a.counters[1] + a.check_every;
    if (threadIdx.x == 0) {
        int pos = 0, act = 0;
        for (int s = 0; s < a.n_samples; ++s) {
            if (a.sample_steps[s] == 0) {
                start[s] = pos;
                pos += a.tile_off[s + 1] - a.tile_off[s];
                ++act;
            } else {
                start[s] = -1;
            }
        }
        total = pos;
        active = act;
        // queue range of every group: its samples are consecutive, so their
        // active tiles are consecutive in the queue
        int q = 0;
        for (int gi = 0; gi < a.n_groups; ++gi) {
            a.group_queue_off[gi] = q;
            for (int s = a.group_sample_off[gi]; s < a.group_sample_off[gi + 1]; ++s)
                if (start[s] >= 0) q += a.tile_off[s + 1] - a.tile_off[s];
        }
        a.group_queue_off[a.n_groups] = q;
    }
    __syncthreads();
    for (int s = 0; s < a.n_samples; ++s) {
        if (start[s] < 0) continue;
        const int cnt = a.tile_off[s + 1] - a.tile_off[s];
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) ((int *)a.queue)[start[s] + t] = a.tile_off[s] + t;
    }
    if (threadIdx.x == 0) {
        a.counters[0] = total;
        a.counters[1] = mark ? steps : 0;
        a.counters[2] = active;
        a.counters[3] += mark;
    }
}

__global__ void k_batch_reset(const BatchArgs a) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < a.ntiles) ((int *)a.queue)[t] = (int)t;
    if (t < a.n_samples) {
        a.sample_steps[t] = 0;
        a.sample_res[t] = INFINITY;
        a.sample_ux[t] = 0.0;
    }
    if (t == 0) {
        a.counters[0] = (int)a.ntiles;
        a.counters[1] = 0;
        a.counters[2] = a.n_samples;
        a.counters[3] = 0;
    }
}

using RedFn = void (*)(const BatchArgs);

RedFn pick_red(int storage, int variant) {
#define MLBM_RED(S)                                                                          \
    case S:                                                                                  \
        return variant == MLBM_POPULATIONS ? (RedFn)k_batch_tile_red<S, MLBM_POPULATIONS>    \
                                           : (RedFn)k_batch_tile_red<S, MLBM_FIELDS>;
    switch (storage) {
        MLBM_RED(MLBM_F64)
        MLBM_RED(MLBM_F32)
        MLBM_RED(MLBM_F16S)
        MLBM_RED(MLBM_BF16)
    }
#undef MLBM_RED
    return nullptr;
}

int batch_args(const mlbm_step_params *p, const mlbm_device_state *st, const mlbm_batch *b, BatchArgs &ba) {
    using mlbm::fail;
    int rc = check_common(p, st);
    if (rc) return rc;
    if (!b) return fail(MLBM_ERR_ARG, "null batch");
    if (st->tile == 0) return fail(MLBM_ERR_ARG, "batched runs need tiles (state->tile = 64, 128 or 256)");
    if (b->n_samples < 1 || b->n_samples > MAX_SAMPLES) return fail(MLBM_ERR_ARG, "n_samples outside [1, %d]", MAX_SAMPLES);
    if (!b->sample_tile_off || !b->sample_tile_off_host || !b->area || !b->u_prev || !b->tile_red || !b->queue ||
        !b->counters || !b->sample_steps || !b->sample_residual || !b->sample_int_ux)
        return fail(MLBM_ERR_ARG, "null batch buffer");
    const int64_t ntiles = (st->n + st->tile - 1) / st->tile;
    const int32_t *off = b->sample_tile_off_host;
    if (off[0] != 0 || off[b->n_samples] != ntiles)
        return fail(MLBM_ERR_ARG, "sample tiles must cover [0, %lld)", (long long)ntiles);
    for (int s = 0; s < b->n_samples; ++s)
        if (off[s + 1] <= off[s]) return fail(MLBM_ERR_ARG, "sample %d has no tiles", s);
    if (b->check_every < 2 || (b->check_every & 1)) return fail(MLBM_ERR_ARG, "check_every must be even and >= 2");
    if (b->n_groups < 1 || !b->group_sample_off || !b->group_sample_off_host || !b->group_queue_off)
        return fail(MLBM_ERR_ARG, "batch needs at least one sample group");
    const int32_t *go = b->group_sample_off_host;
    if (go[0] != 0 || go[b->n_groups] != b->n_samples) return fail(MLBM_ERR_ARG, "groups must cover the samples");
    for (int gi = 0; gi < b->n_groups; ++gi)
        if (go[gi + 1] <= go[gi]) return fail(MLBM_ERR_ARG, "group %d is empty", gi);
    ba.n = st->n;
    ba.flags = st->flags;
    ba.bc = st->bc;
    ba.state = st->state[st->cur];
    ba.area = b->area;
    ba.u_prev = b->u_prev;
    ba.tile_red = b->tile_red;
    ba.queue = b->queue;
    ba.counters = b->counters;
    ba.tile_off = b->sample_tile_off;
    ba.n_samples = b->n_samples;
    ba.sample_steps = b->sample_steps;
    ba.sample_res = b->sample_residual;
    ba.sample_ux = b->sample_int_ux;
    ba.gx = p->g[0];
    ba.gy = p->g[1];
    ba.tol = 0.0;
    ba.inv_scale = std::ldexp(1.0f, -p->scale_exp);
    ba.check_every = b->check_every;
    ba.ntiles = ntiles;
    ba.n_groups = b->n_groups;
    ba.group_sample_off = b->group_sample_off;
    ba.group_queue_off = b->group_queue_off;
    return MLBM_OK;
}

int batch_grid(const mlbm_batch *b) {
    int g = b->grid > 0 ? b->grid : 1024;
    return (g + 7) / 8 * 8;
}

}  // namespace

extern "C" int mlbm_batch_init(const mlbm_step_params *p, mlbm_device_state *st, mlbm_batch *b, void *stream) {
    using mlbm::fail;
    mlbm::clear_error();
    BatchArgs ba;
    int rc = batch_args(p, st, b, ba);
    if (rc) return rc;
    RedFn red = pick_red(p->storage, p->variant);
    hipStream_t s = (hipStream_t)stream;
    const int64_t cover = std::max<int64_t>(ba.ntiles, b->n_samples);
    hipLaunchKernelGGL(k_batch_reset, dim3((unsigned)((cover + 255) / 256)), dim3(256), 0, s, ba);
    hipLaunchKernelGGL(red, dim3((unsigned)batch_grid(b)), dim3(st->tile), 0, s, ba);
    hipLaunchKernelGGL(k_batch_sample_red, dim3(b->n_samples), dim3(256), 0, s, ba, 0);
    hipLaunchKernelGGL(k_batch_retire, dim3(1), dim3(256), 0, s, ba, 0);
    return hip_check("mlbm_batch_init launch");
}

extern "C" int mlbm_step_batched(const mlbm_step_params *p, mlbm_device_state *st, mlbm_batch *b,
                                 int32_t max_steps, double tol, int32_t use_graph, int32_t *steps_done,
                                 void *stream) {
    using mlbm::fail;
    mlbm::clear_error();
    BatchArgs ba;
    int rc = batch_args(p, st, b, ba);
    if (rc) return rc;
    if (max_steps < 0) return fail(MLBM_ERR_ARG, "max_steps must be >= 0");
    if (!(tol >= 0.0)) return fail(MLBM_ERR_ARG, "tol must be >= 0");
    if (use_graph && !stream) return fail(MLBM_ERR_ARG, "graph capture needs a non-default stream");
    const int kq = (st->K + 3) / 4;
    if (st->per_departure) return fail(MLBM_ERR_UNSUPPORTED, "batched runs take one stencil per node");
    StepFn fn = pick_step_any(p->storage, p->variant, kq, true, p->weights16);
    RedFn red = pick_red(p->storage, p->variant);
    if (!fn || !red) return fail(MLBM_ERR_UNSUPPORTED, "no kernel for storage %d, variant %d, K=%d", p->storage, p->variant, st->K);
    if (p->variant == MLBM_FIELDS && (p->tau_plus != 1.0 || p->tau_minus != 1.0))
        return fail(MLBM_ERR_ARG, "the fields variant fixes tau = 1");
    if (!st->halo_off || !st->halo || !st->lidx || st->max_halo < 1) return fail(MLBM_ERR_ARG, "null tile buffer");
    const int ts = storage_bytes(p->storage);
    const size_t shmem = (size_t)st->max_halo * (p->variant == MLBM_POPULATIONS ? 8 * ts : 4 * ts);
    if (shmem > 65536) return fail(MLBM_ERR_UNSUPPORTED, "halo needs %zu bytes of LDS (> 64 KiB)", shmem);
    ba.tol = tol;
    StepArgs a;
    a.n = st->n;
    a.idx = (const int *)st->idx;
    a.w = st->w;
    a.flags = st->flags;
    a.bc = st->bc;
    a.omp = 1.0 / p->tau_plus;
    a.omm = 1.0 / p->tau_minus;
    a.gx = p->g[0];
    a.gy = p->g[1];
    a.scale = std::ldexp(1.0f, p->scale_exp);
    a.inv_scale = std::ldexp(1.0f, -p->scale_exp);
    a.xcd = p->xcd_remap ? 1 : 0;
    a.cached = p->cached_weights ? 1 : 0;
    a.reverse = 0;
    a.halo_off = st->halo_off;
    a.halo = st->halo;
    a.lidx = st->lidx;
    a.wl = nullptr;  // batched runs use every node's own weights
    a.lag0 = st->n;  // (no block-centre launch)
    a.tile0 = a.tile1 = 0;
    a.split = a.tile0b = a.tile1b = a.grid8b = 0;
    a.sr = 0;        // and round to nearest (a captured graph replays fixed keys)
    a.seed = 0;
    a.queue = b->queue;
    a.queue_range = b->group_queue_off;
    a.grid8 = batch_grid(b);
    const int G = (int)a.grid8;
    hipStream_t s = (hipStream_t)stream;
    const int cur0 = st->cur;
    // one check: check_every steps of every sample group in turn (a group's
    // nodes stay cache-resident across its steps), the per-tile pass, retirement
    // groups whose samples have all retired are left out of the launches
    std::vector<int32_t> qoff(b->n_groups + 1);
    std::vector<char> live(b->n_groups, 1);
    // a group's launches need no more workgroups than it has tiles; while all
    // of its samples are active its tiles are one contiguous range, walked
    // directly (one workgroup per tile, no queue lookup on the critical path)
    std::vector<int> group_grid(b->n_groups), group_tiles(b->n_groups), group_tile0(b->n_groups);
    std::vector<char> full(b->n_groups, 0);
    for (int gi = 0; gi < b->n_groups; ++gi) {
        const int32_t *so = b->sample_tile_off_host, *go = b->group_sample_off_host;
        group_tile0[gi] = so[go[gi]];
        group_tiles[gi] = so[go[gi + 1]] - so[go[gi]];
        group_grid[gi] = std::min(G, (group_tiles[gi] + 7) / 8 * 8);
    }
    // the check_every steps of one group
    auto enqueue_group = [&](int gi) {
        int cur = cur0;
        a.group = gi;
        int grid = group_grid[gi];
        if (full[gi]) {
            a.queue = nullptr;
            a.tile0 = group_tile0[gi];
            a.tile1 = group_tile0[gi] + group_tiles[gi];
            grid = a.xcd ? (group_tiles[gi] + 7) / 8 * 8 : group_tiles[gi];
            a.grid8 = grid;
        } else {
            a.queue = b->queue;
            a.grid8 = G;
        }
        for (int t = 0; t < b->check_every; ++t) {
            a.in = st->state[cur];
            a.out = st->state[cur ^ 1];
            a.reverse = p->alternate_sweeps ? (t & 1) : 0;
            hipLaunchKernelGGL(fn, dim3(grid), dim3(st->tile), shmem, s, a);
            cur ^= 1;
        }
    };
    // the per-tile sums, the per-sample residuals, retirement
    auto enqueue_check = [&]() {
        ba.state = st->state[cur0];
        hipLaunchKernelGGL(red, dim3(G), dim3(st->tile), 0, s, ba);
        hipLaunchKernelGGL(k_batch_sample_red, dim3(b->n_samples), dim3(256), 0, s, ba, 1);
        hipLaunchKernelGGL(k_batch_retire, dim3(1), dim3(256), 0, s, ba, 1);
    };
    // With graphs, each group's steps are one graph and the check another, so
    // a group that retires or loses a sample costs one small capture.
    std::vector<hipGraph_t> graphs(b->n_groups + 1, nullptr);
    std::vector<hipGraphExec_t> execs(b->n_groups + 1, nullptr);
    std::vector<char> graph_full(b->n_groups, 0);
    auto release = [&](int k) {
        if (execs[k]) (void)hipGraphExecDestroy(execs[k]);
        if (graphs[k]) (void)hipGraphDestroy(graphs[k]);
        execs[k] = nullptr;
        graphs[k] = nullptr;
    };
    auto capture = [&](int k) -> int {  // k < n_groups: group k; k == n_groups: the check
        release(k);
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return fail(MLBM_ERR_HIP, "hipStreamBeginCapture failed");
        if (k < b->n_groups) enqueue_group(k);
        else enqueue_check();
        const int r = hip_check("mlbm_step_batched launch");
        hipError_t e = hipStreamEndCapture(s, &graphs[k]);
        if (r) return r;
        if (e != hipSuccess) return fail(MLBM_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&execs[k], graphs[k], nullptr, nullptr, 0);
        if (e != hipSuccess) return fail(MLBM_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        if (k < b->n_groups) graph_full[k] = full[k];
        return MLBM_OK;
    };
    auto run_check = [&]() -> int {
        for (int gi = 0; gi < b->n_groups; ++gi) {
            if (!live[gi]) continue;
            if (!use_graph) {
                enqueue_group(gi);
                continue;
            }
            if (!execs[gi] || graph_full[gi] != full[gi]) {
                const int r = capture(gi);
                if (r) return r;
            }
            if (hipGraphLaunch(execs[gi], s) != hipSuccess) return fail(MLBM_ERR_HIP, "hipGraphLaunch failed");
        }
        if (!use_graph) {
            enqueue_check();
            return hip_check("mlbm_step_batched launch");
        }
        if (!execs[b->n_groups]) {
            const int r = capture(b->n_groups);
            if (r) return r;
        }
        if (hipGraphLaunch(execs[b->n_groups], s) != hipSuccess) return fail(MLBM_ERR_HIP, "hipGraphLaunch failed");
        return MLBM_OK;
    };
    // the queue ranges left by the last retirement decide which groups run
    if (hipMemcpyAsync(qoff.data(), b->group_queue_off, qoff.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MLBM_ERR_HIP, "reading the group queue ranges failed");
    for (int gi = 0; gi < b->n_groups; ++gi) {
        live[gi] = qoff[gi + 1] > qoff[gi];
        full[gi] = qoff[gi + 1] - qoff[gi] == group_tiles[gi];
    }
    int steps = 0;
    int counters[4] = {1, 0, 1, 0};
    rc = MLBM_OK;
    while (steps < max_steps) {
        rc = run_check();
        if (rc) break;
        steps += b->check_every;
        if (hipMemcpyAsync(counters, b->counters, sizeof(counters), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(qoff.data(), b->group_queue_off, qoff.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            rc = fail(MLBM_ERR_HIP, "reading the batch counters failed");
            break;
        }
        if (counters[2] == 0) break;
        for (int gi = 0; gi < b->n_groups; ++gi) {
            live[gi] = qoff[gi + 1] > qoff[gi];
            full[gi] = qoff[gi + 1] - qoff[gi] == group_tiles[gi];
        }
    }
    for (int k = 0; k <= b->n_groups; ++k) release(k);
    if (steps_done) *steps_done = steps;
    return rc;
}
