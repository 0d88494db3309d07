// Step kernels with eight lanes per node (gfx950).
//
// The one-lane-per-node kernels (mlbm_step.hip) give a node set of N nodes N
// lanes: a set of a few thousand nodes fills a few dozen of the 256 compute
// units and the step is bound by the latency of each lane's dependent loads.
// Here lane k (0..7) of a node's group of eight takes arriving population
// k + 1 (population form, Sec. 2.2, Eq. 12) or departure point k + 1 (fields
// form, Sec. 2.2, Eqs. 14-15): its weight set, its K stencil values and its
// interpolation sum, in the same order of operations as the node's own lane
// would.  The group then exchanges its eight sums through wavefront shuffles
// (the groups are aligned to eight lanes of one wavefront), every lane of the
// group forms the node's moments and collision with the same arithmetic as
// the one-lane kernels, and each lane stores its own population (lane 0 also
// the rest population, or the fields).  The results equal those of the
// one-lane kernels to rounding (same sums in the same order; the compiler may
// fuse multiply-adds differently); the mapping trades eight times the lanes
// (and eight copies of the moment arithmetic) for one eighth of the loads
// per lane.
//
// Workgroups: with LDS-staged tiles of T nodes (64 or 128), 8 T lanes per
// workgroup staging the tile's halo exactly as the one-lane kernels do;
// with global gathers, `block` lanes for block / 8 nodes.  Per-node stencils,
// and hybrid sets in one launch per step (the block centres gather their
// eight lattice neighbours and themselves with the shared biquadratic
// weights, Sec. 2.2); not one stencil per departure point.

#include <hip/hip_runtime.h>

#include "mlbm_device.h"

namespace mlbm_dev {

namespace {

// one population (component c of the [n][8] block) of node j
template <int S, class C>
__device__ __forceinline__ void store_comp(void *base, int64_t j, int c, C v, float scale, Rnd rnd = {}) {
    if constexpr (S == MLBM_F64) ((double *)base)[8 * j + c] = (double)v;
    else if constexpr (S == MLBM_F32) ((float *)base)[8 * j + c] = (float)v;
    else ((unsigned short *)base)[8 * j + c] = enc16<S>((float)v, scale, rnd.bits(c), rnd.on);
}

// direction vector of population k + 1 (k = 0..7, Sec. 2.1, Eq. 2) from the
// lane's k by integer selects (no lane-varying table lookups)
__device__ __forceinline__ int ex_of(int k) { return k < 4 ? (k == 0) - (k == 2) : ((k == 4 || k == 7) ? 1 : -1); }
__device__ __forceinline__ int ey_of(int k) { return k < 4 ? (k == 1) - (k == 3) : ((k == 4 || k == 5) ? 1 : -1); }

// The collision of one lane's population: the node's moments from all nine
// offsets f[0..8] (the expressions of collide()), then the TRT update of the
// pair (a, a') holding population k + 1 with a = 1, 2, 5 or 6, evaluated as
// collide() evaluates it, from the lane's own offset and its opposite's.
// Returns the lane's post-collision offset; post0 receives the rest
// population's.
template <class C>
__device__ __forceinline__ C collide_lane(const C *f, int k, C mine, C opp, C omp, C omm, C gx, C gy, C &post0) {
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
        post0 = f[0] - omp * (f[0] - e0) + cp * F0;
    }
    const bool first = (k & 2) == 0;  // population k + 1 is a (1, 2, 5, 6), else a'
    const int ka = first ? k : (k ^ 2), kb = ka ^ 2;
    const C w = ka < 4 ? C(1) / C(9) : C(1) / C(36);
    const C usq = ux * ux + uy * uy;
    auto feq = [&](int kk) __attribute__((always_inline)) {
        const C eu = C(ex_of(kk)) * ux + C(ey_of(kk)) * uy;
        return w * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * usq));
    };
    auto force = [&](int kk) __attribute__((always_inline)) {
        const C ex = C(ex_of(kk)), ey = C(ey_of(kk));
        const C eu = ex * ux + ey * uy;
        const C eg = ex * gx + ey * gy;
        const C ug = ux * gx + uy * gy;
        return w * rho * (C(3) * (eg - ug) + C(9) * eu * eg);
    };
    const C fa = first ? mine : opp, fb = first ? opp : mine;
    const C ea = feq(ka), eb = feq(kb);
    const C Fa = force(ka), Fb = force(kb);
    const C fp = C(0.5) * (fa + fb), fm = C(0.5) * (fa - fb);
    const C ep = C(0.5) * (ea + eb), em = C(0.5) * (ea - eb);
    const C Fp = C(0.5) * (Fa + Fb), Fm = C(0.5) * (Fa - Fb);
    const C sym = -omp * (fp - ep) + cp * Fp;
    const C asy = -omm * (fm - em) + cm * Fm;
    return first ? fa + sym + asy : fb + sym - asy;
}

// The tile's halo into LDS as the one-lane kernels stage it; the tile holds
// T = blockDim.x / 8 nodes and *self0 receives the halo position of its first
// node (its nodes sit at consecutive positions of the sorted halo).
template <int NB>
__device__ __forceinline__ void stage_halo_self(const StepArgs &a, int64_t tile, void *smem, int *self0) {
    __syncthreads();
    const int h0 = a.halo_off[tile], hn = a.halo_off[tile + 1] - h0;
    const int64_t first = tile * (int64_t)(blockDim.x >> 3);
    if constexpr (NB >= 16) {
        constexpr int U = NB / 16;
        const u4 *src = (const u4 *)a.in;
        u4 *dst = (u4 *)smem;
        for (int e = threadIdx.x; e < hn * U; e += blockDim.x) {
            const int h = e / U, c = e - h * U;
            const int node = a.halo[h0 + h];
            if (c == 0 && node == first) *self0 = h;
            dst[e] = src[(int64_t)node * U + c];
        }
    } else {
        const u2 *src = (const u2 *)a.in;
        u2 *dst = (u2 *)smem;
        for (int h = threadIdx.x; h < hn; h += blockDim.x) {
            const int node = a.halo[h0 + h];
            if (node == first) *self0 = h;
            dst[h] = src[node];
        }
    }
    __syncthreads();
}

// first lane of this lane's group of eight in the wavefront
__device__ __forceinline__ int group_base() { return (int)(threadIdx.x & 63u) & ~7; }

// KQ = 0: a block centre of a hybrid set (members: its eight lattice
// neighbours, then itself at position self); the node ranges split at lag0 as
// in the one-lane kernels.
template <int S, class CG, class C, int KQ, bool LDS, bool W16>
__device__ __forceinline__ void pop_lanes(const StepArgs &a, const void *src, int64_t i, int k, int self) {
    if ((KQ == 0) != (i >= a.lag0)) return;  // the other part's node (the whole group)
    const int64_t n = a.n;
    const unsigned fl = a.flags[i];
    if (kind_of(fl) == MLBM_DIRICHLET) {
        // the whole group takes this branch (one node)
        const C rb = (C)a.bc[3 * i], ub = (C)a.bc[3 * i + 1], vb = (C)a.bc[3 * i + 2];
        store_comp<S, C>(a.out, i, k, feq_off<C>(k + 1, C(1), rb - C(1), rb, ub, vb), a.scale);
        if (k == 0) store1<S, C>(a.out, n, i, feq_off<C>(0, C(1), rb - C(1), rb, ub, vb), a.scale);
        return;
    }
    const unsigned bb = fl & 0xffu;
    // source population: k, or its opposite k xor 2 on bounce-back
    const int c = ((bb >> k) & 1u) ? (k ^ 2) : k;
    constexpr bool kWsum = S == MLBM_F64;  // as the one-lane kernels (interpolated weight sum)
    CG acc = CG(0), sw = CG(0);
    if constexpr (KQ == 0) {
        // the shared biquadratic weights of population k + 1 (no bounce-back here)
        if (!(fl & MLBM_FLAG_LAGRANGE)) acc = CG(NAN);
        int m[9];
        block_members<LDS>(a, n, i, self, m);
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            const CG wv = block_weight<S, CG>(a, k * 9 + j);
            acc = fma(wv, load_comp<S, CG>(src, m[j], k, a.inv_scale), acc);
            if constexpr (kWsum) sw += wv;
        }
    } else {
        u4 lv;
        for_quads<0, KQ>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value;
            int m[4];
            members<LDS, q>(a, n, i, lv, m);
            CG wv[4];
            load_w4<S, KQ, W16>(a.w, n, i, k, q, wv, a.cached);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                acc = fma(wv[j], load_comp<S, CG>(src, m[j], c, a.inv_scale), acc);
                if constexpr (kWsum) sw += wv[j];
            }
        });
    }
    const int base = group_base();
    C f[9];
    f[0] = load1<S, C>(a.in, n, i, a.inv_scale);
    C mine;
    if constexpr (kWsum) {
        mine = (C)acc + omega<C>(k + 1) * ((C)sw - C(1));
#pragma unroll
        for (int t = 0; t < 8; ++t) f[t + 1] = __shfl(mine, base + t, 64);
    } else {
        mine = (C)acc;
#pragma unroll
        for (int t = 0; t < 8; ++t) f[t + 1] = (C)__shfl(acc, base + t, 64);
    }
    // the opposite population sits two lanes away (k' = k xor 2)
    const C opp = __shfl_xor(mine, 2, 64);
    C post0;
    const C post = collide_lane<C>(f, k, mine, opp, (C)a.omp, (C)a.omm, (C)a.gx, (C)a.gy, post0);
    if (a.sr) {
        const Rnd rnd = step_rnd(a, i);
        store_comp<S, C>(a.out, i, k, post, a.scale, rnd);
        if (k == 0) store1<S, C>(a.out, n, i, post0, a.scale, rnd);
    } else {
        store_comp<S, C>(a.out, i, k, post, a.scale);
        if (k == 0) store1<S, C>(a.out, n, i, post0, a.scale);
    }
}

template <int S, class CG, class C, int KQ, bool LDS, bool W16>
__device__ __forceinline__ void fields_lanes(const StepArgs &a, const void *src, int64_t i, int k, int self) {
    if ((KQ == 0) != (i >= a.lag0)) return;  // the other part's node (the whole group)
    const int64_t n = a.n;
    const unsigned fl = a.flags[i];
    if (kind_of(fl) == MLBM_DIRICHLET) {
        if (k != 0) return;
        C out[3];
        out[0] = (C)a.bc[3 * i] - C(1);
        out[1] = (C)a.bc[3 * i + 1];
        out[2] = (C)a.bc[3 * i + 2];
        store3<S>(a.out, i, out, a.scale, step_rnd(a, i));
        return;
    }
    const unsigned bb = fl & 0xffu;
    constexpr bool kWsum = S == MLBM_F64;  // interpolate rho itself, not rho - 1
    CG ar = CG(0), au = CG(0), av = CG(0), sw = CG(0);
    if constexpr (KQ == 0) {
        // the shared biquadratic weights of departure point k + 1
        if (!(fl & MLBM_FLAG_LAGRANGE)) ar = CG(NAN);
        int mi[9];
        block_members<LDS>(a, n, i, self, mi);
#pragma unroll
        for (int j = 0; j < 9; ++j) {
            CG m[3];
            load3<S>(src, mi[j], m, a.inv_scale);
            const CG wv = block_weight<S, CG>(a, k * 9 + j);
            ar = fma(wv, m[0], ar);
            au = fma(wv, m[1], au);
            av = fma(wv, m[2], av);
            if constexpr (kWsum) sw += wv;
        }
    } else {
        u4 lv;
        for_quads<0, KQ>([&](auto qc) __attribute__((always_inline)) {
            constexpr int q = decltype(qc)::value;
            int mi[4];
            members<LDS, q>(a, n, i, lv, mi);
            CG m[4][3];
#pragma unroll
            for (int j = 0; j < 4; ++j) load3<S>(src, mi[j], m[j], a.inv_scale);
            CG wv[4];
            load_w4<S, KQ, W16>(a.w, n, i, k, q, wv, a.cached);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                ar = fma(wv[j], m[j][0], ar);
                au = fma(wv[j], m[j][1], au);
                av = fma(wv[j], m[j][2], av);
                if constexpr (kWsum) sw += wv[j];
            }
        });
    }
    if constexpr (kWsum) ar += sw - CG(1);
    const C gx = (C)a.gx, gy = (C)a.gy;
    // equilibrium (plus half the force) of the interpolated fields for the
    // population leaving towards this node (source k' on bounce-back)
    const C sg = ((bb >> k) & 1u) ? C(-1) : C(1);
    const C dr = (C)ar, uk = (C)au, vk = (C)av;
    const C rk = C(1) + dr;
    const C fk = feq_off<C>(k + 1, sg, dr, rk, uk, vk) + C(0.5) * force_k<C>(k + 1, sg, rk, uk, vk, gx, gy);
    const int base = group_base();
    C fs[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) fs[t] = __shfl(fk, base + t, 64);
    if (k != 0) return;
    C own[3];
    load3<S>(a.in, i, own, a.inv_scale);
    // rest population from the node's own fields, then the eight in the
    // order of the one-lane kernels
    C sum = feq_off<C>(0, C(1), own[0], C(1) + own[0], own[1], own[2]) +
            C(0.5) * force_k<C>(0, C(1), C(1) + own[0], own[1], own[2], gx, gy);
    C jx = C(0), jy = C(0);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        sum += fs[t];
        jx += C(EX[t + 1]) * fs[t];
        jy += C(EY[t + 1]) * fs[t];
    }
    const C rho = C(1) + sum;
    C out[3];
    out[0] = sum;
    out[1] = (jx + C(0.5) * rho * gx) / rho;
    out[2] = (jy + C(0.5) * rho * gy) / rho;
    store3<S>(a.out, i, out, a.scale, step_rnd(a, i));
}

// one tile (LDS) or one run of blockDim.x / 8 nodes (global gathers) per
// workgroup; a node's group never straddles a wavefront (blockDim.x is a
// multiple of 64)
template <int S, class CG, class C, int KQ, bool LDS, bool W16>
__global__ void __launch_bounds__(1024) k_step_pop_l8(const StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int unused;
    const int64_t tile = a.tile0 + tile_of(a);
    if (tile >= a.tile1) return;
    if constexpr (LDS) stage_halo<pop_bytes<S>(), false>(a, tile, smem, &unused);
    const int64_t i = tile * (int64_t)(blockDim.x >> 3) + (threadIdx.x >> 3);
    if (i < a.n) pop_lanes<S, CG, C, KQ, LDS, W16>(a, LDS ? (const void *)smem : a.in, i, (int)(threadIdx.x & 7u), (int)i);
}

template <int S, class CG, class C, int KQ, bool LDS, bool W16>
__global__ void __launch_bounds__(1024) k_step_fields_l8(const StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int unused;
    const int64_t tile = a.tile0 + tile_of(a);
    if (tile >= a.tile1) return;
    if constexpr (LDS) stage_halo<field_bytes<S>(), false>(a, tile, smem, &unused);
    const int64_t i = tile * (int64_t)(blockDim.x >> 3) + (threadIdx.x >> 3);
    if (i < a.n) fields_lanes<S, CG, C, KQ, LDS, W16>(a, LDS ? (const void *)smem : a.in, i, (int)(threadIdx.x & 7u), (int)i);
}

// Hybrid sets in one launch (as the one-lane k_step_pop_hyb): workgroups
// [0, split) take the tiles of the nodes with per-node weights (LDS staged),
// the later ones the block-centre tiles, which 16-bit states stage in LDS and
// 32- and 64-bit states gather from global memory.
template <int S> constexpr bool block_tiles_staged_l8() { return Fmt<S>::TB == 2; }

template <bool POP, int S, class CG, class C, int KQ, bool W16>
__device__ __forceinline__ void hyb_lanes(const StepArgs &a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int self0;
    constexpr int NB = POP ? pop_bytes<S>() : field_bytes<S>();
    const int64_t b = blockIdx.x;
    const int64_t tn = blockDim.x >> 3;
    const int k = (int)(threadIdx.x & 7u), loc = (int)(threadIdx.x >> 3);
    auto node = [&](auto kq, bool lds, const void *src, int64_t i, int self) __attribute__((always_inline)) {
        constexpr int Q = decltype(kq)::value;
        if (lds) {
            if constexpr (POP) pop_lanes<S, CG, C, Q, true, Q == 0 ? false : W16>(a, src, i, k, self);
            else fields_lanes<S, CG, C, Q, true, Q == 0 ? false : W16>(a, src, i, k, self);
        } else {
            if constexpr (POP) pop_lanes<S, CG, C, Q, false, false>(a, src, i, k, self);
            else fields_lanes<S, CG, C, Q, false, false>(a, src, i, k, self);
        }
    };
    if (b < a.split) {
        const int64_t tile = a.tile0 + tile_at(a, b, a.grid8);
        if (tile >= a.tile1) return;
        stage_halo<NB, false>(a, tile, smem, &self0);
        const int64_t i = tile * tn + loc;
        if (i < a.n) node(std::integral_constant<int, KQ>{}, true, (const void *)smem, i, (int)i);
    } else {
        const int64_t tile = a.tile0b + tile_at(a, b - a.split, a.grid8b);
        if (tile >= a.tile1b) return;
        const int64_t i = tile * tn + loc;
        if constexpr (block_tiles_staged_l8<S>()) {
            stage_halo_self<NB>(a, tile, smem, &self0);
            if (i < a.n) node(std::integral_constant<int, 0>{}, true, (const void *)smem, i, self0 + loc);
        } else {
            if (i < a.n) node(std::integral_constant<int, 0>{}, false, a.in, i, (int)i);
        }
    }
}

template <int S, class CG, class C, int KQ, bool W16>
__global__ void __launch_bounds__(1024) k_step_pop_hyb_l8(const StepArgs a) {
    hyb_lanes<true, S, CG, C, KQ, W16>(a);
}

template <int S, class CG, class C, int KQ, bool W16>
__global__ void __launch_bounds__(1024) k_step_fields_hyb_l8(const StepArgs a) {
    hyb_lanes<false, S, CG, C, KQ, W16>(a);
}

template <int S, class CG, class C, bool W16 = false>
StepFn pick_lanes_hyb(int variant, int kq) {
#define MLBM_CASE(Q)                                                                              \
    case Q:                                                                                       \
        return variant == MLBM_POPULATIONS ? (StepFn)k_step_pop_hyb_l8<S, CG, C, Q, W16>          \
                                           : (StepFn)k_step_fields_hyb_l8<S, CG, C, Q, W16>;
    switch (kq) {
        MLBM_CASE(3)
        MLBM_CASE(4)
        MLBM_CASE(7)
        MLBM_CASE(8)
        default:
            return nullptr;
    }
#undef MLBM_CASE
}

template <int S, class CG, class C, bool W16 = false>
StepFn pick_lanes(int variant, int kq, bool lds) {
#define MLBM_CASE(Q)                                                                                \
    case Q:                                                                                         \
        if (lds)                                                                                    \
            return variant == MLBM_POPULATIONS ? (StepFn)k_step_pop_l8<S, CG, C, Q, true, W16>      \
                                               : (StepFn)k_step_fields_l8<S, CG, C, Q, true, W16>;  \
        return variant == MLBM_POPULATIONS ? (StepFn)k_step_pop_l8<S, CG, C, Q, false, W16>         \
                                           : (StepFn)k_step_fields_l8<S, CG, C, Q, false, W16>;
    switch (kq) {
        MLBM_CASE(3)
        MLBM_CASE(4)
        MLBM_CASE(7)
        MLBM_CASE(8)
        default:
            return nullptr;
    }
#undef MLBM_CASE
}

}  // namespace

// the arithmetic choices of the one-lane kernels: FP32 states gather in FP32
// and collide in FP64, 16-bit states use FP32 throughout
StepFn pick_step_lanes_any(int storage, int variant, int kq, bool lds, int w16) {
    switch (storage) {
        case MLBM_F64: return pick_lanes<MLBM_F64, double, double>(variant, kq, lds);
        case MLBM_F32: return pick_lanes<MLBM_F32, float, double>(variant, kq, lds);
        case MLBM_F16S:
            return w16 ? pick_lanes<MLBM_F16S, float, float, true>(variant, kq, lds)
                       : pick_lanes<MLBM_F16S, float, float>(variant, kq, lds);
        case MLBM_BF16:
            return w16 ? pick_lanes<MLBM_BF16, float, float, true>(variant, kq, lds)
                       : pick_lanes<MLBM_BF16, float, float>(variant, kq, lds);
    }
    return nullptr;
}

StepFn pick_step_lanes_hyb_any(int storage, int variant, int kq, int w16) {
    switch (storage) {
        case MLBM_F64: return pick_lanes_hyb<MLBM_F64, double, double>(variant, kq);
        case MLBM_F32: return pick_lanes_hyb<MLBM_F32, float, double>(variant, kq);
        case MLBM_F16S:
            return w16 ? pick_lanes_hyb<MLBM_F16S, float, float, true>(variant, kq)
                       : pick_lanes_hyb<MLBM_F16S, float, float>(variant, kq);
        case MLBM_BF16:
            return w16 ? pick_lanes_hyb<MLBM_BF16, float, float, true>(variant, kq)
                       : pick_lanes_hyb<MLBM_BF16, float, float>(variant, kq);
    }
    return nullptr;
}

}  // namespace mlbm_dev
