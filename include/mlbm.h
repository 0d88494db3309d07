/*
 * mlbm.h - C ABI of the meshless lattice Boltzmann library (libmlbm.so).
 *
 * The library implements the time step of the meshless LBM of Strzelczyk &
 * Matyka, "Modeling inertial flows with meshless Lattice Boltzmann Method"
 * (arXiv 2312.14789) on one AMD Instinct MI355X (gfx950):
 *
 *   - population MLBM: collision (TRT, Sec. 2.1 Eqs. 3-5; BGK when
 *     tau- = tau+) fused with the semi-Lagrangian streaming of Sec. 2.2
 *     Eq. 12, in which every population arriving at node x is the weighted
 *     sum of the post-collision population over the node's stencil, taken at
 *     the departure point x - dx e_k;
 *   - MLBM1, the fixed tau = 1 variant (Sec. 2.2, Eqs. 14-15): only density
 *     and velocity are stored, interpolated to the departure points and
 *     turned into the next fields through the equilibria;
 *   - a constant body acceleration g with Guo's second-order forcing, no-slip
 *     surfaces by (interpolated) bounce-back (Sec. 3.1, Sec. 3.2 Eq. 22) and
 *     Dirichlet nodes overwritten by an equilibrium (Sec. 3.1).
 *
 * Conventions (all entry points):
 *   - Every function returns MLBM_OK (0) or a negative MLBM_ERR_* code; the
 *     message of the last failure on the calling thread is returned by
 *     mlbm_last_error() and stays valid until the next call on that thread.
 *   - Host pointers are read or written only during the call.  Device
 *     pointers and the HIP stream are owned by the caller; device work is
 *     enqueued on the given stream (NULL = the default stream) and is
 *     asynchronous; only mlbm_step_batched and mlbm_run_to_steady wait on
 *     their stream.  The library never allocates device memory.
 *   - Node order in every array is the order chosen by mlbm_build_stencils
 *     (perm[new] = old maps back to the caller's order).
 *   - Nothing here is thread safe with respect to the same output buffers.
 */
#ifndef MLBM_H
#define MLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes -------------------------------------------------------- */
#define MLBM_OK               0
#define MLBM_ERR_ARG         -1  /* null pointer, bad size, unsupported value  */
#define MLBM_ERR_GEOMETRY    -2  /* node inside a solid, K > n, degenerate box */
#define MLBM_ERR_SINGULAR    -3  /* a local interpolation system is singular   */
#define MLBM_ERR_HIP         -4  /* a HIP launch or runtime call failed        */
#define MLBM_ERR_UNSUPPORTED -5  /* variant x storage x K combination missing  */
#define MLBM_ERR_UNSTABLE    -6  /* non-finite fields or rho <= 0 seen by a check */

/* ---- node kinds (geometry) ------------------------------------------------ */
#define MLBM_FLUID     0  /* ordinary fluid node                                */
#define MLBM_WALL      1  /* node lying on a no-slip surface (Sec. 3.2)         */
#define MLBM_DIRICHLET 2  /* populations overwritten by f^eq(rho_b, u_b) (Sec. 3.1) */

/* ---- step variants and state storage -------------------------------------- */
#define MLBM_POPULATIONS 0  /* population MLBM (Sec. 2.2, Eq. 12)               */
#define MLBM_FIELDS      1  /* MLBM1, tau = 1, fields only (Sec. 2.2, Eqs. 14-15) */

#define MLBM_F64  0  /* FP64 state, FP64 weights, FP64 arithmetic                 */
#define MLBM_F32  1  /* FP32 state and weights, FP32 interpolation, FP64 collision */
#define MLBM_F16S 2  /* FP16 state scaled by 2^scale_exp, FP32 weights/arithmetic */
#define MLBM_BF16 3  /* BF16 state, FP32 weights and arithmetic                   */

/* ---- geometry and stencil construction (host, FP64) ----------------------- */
typedef struct mlbm_geometry {
    int64_t n;               /* number of nodes                                   */
    const double *xy;        /* host [n][2] node coordinates                      */
    const uint8_t *kind;     /* host [n] MLBM_FLUID / MLBM_WALL / MLBM_DIRICHLET  */
    double lo[2], hi[2];     /* box; nodes must lie in [lo, hi]                   */
    int32_t periodic[2];     /* 1 = periodic along x / y (minimum-image offsets)  */
    int32_t wall_lo_y;       /* 1 = no-slip wall on the line y = lo[1]            */
    int32_t wall_hi_y;       /* 1 = no-slip wall on the line y = hi[1]            */
    int64_t n_disks;         /* number of solid disks                             */
    const double *disks;     /* host [n_disks][3] (cx, cy, r), periodic images used */
    double fluid_area;       /* area the quadrature weights sum to (<= 0: box area
                                minus the disk areas)                             */
} mlbm_geometry;

typedef struct mlbm_stencil_params {
    int32_t K;               /* stencil size, 7 <= K <= 32 (nearest nodes, self included) */
    int32_t reorder;         /* 0 keep the caller's order, 1 Morton (Z) order,
                                2 reverse Cuthill-McKee order of the graph linking
                                each node to its K nearest nodes                  */
    double dx;               /* streaming distance dx > 0, units of xy             */
    int32_t n_threads;       /* host threads; 0 = all hardware threads            */
    double lattice_h;        /* > 0: hybrid set whose regular part is a square
                                lattice of this spacing (K >= 10); 0: RBF-FD at
                                every node                                         */
    int32_t per_departure;   /* 1: one stencil per departure point, its K nearest
                                nodes (the paper's stencils, Sec. 2.2); idx is then
                                [n][8][K].  0: one stencil per node               */
    int32_t simple_bounce_back; /* 1: a departure point inside a solid is replaced
                                by the node itself (simple bounce-back, Sec. 3.1);
                                0: by the mirrored point x + dx e_k              */
} mlbm_stencil_params;

/* Caller-allocated host outputs of mlbm_build_stencils. */
typedef struct mlbm_stencils {
    int64_t *perm;           /* [n]       perm[new] = old                          */
    int32_t *idx;            /* [n][K]    stencil members (new order), idx[i][0] = i;
                                [n][8][K] with per_departure (the K nearest nodes of
                                each departure point, nearest first)              */
    double *w;               /* [n][8][K] weights of arriving populations k = 1..8 */
    uint8_t *bb;             /* [n]       bit k-1 set: population k is rebuilt from
                                          source population k' (bounce-back)      */
    double *area;            /* [n]       quadrature weight of each node           */
    uint8_t *lagrange;       /* [n] or NULL: 1 where the block weights are used    */
    double *w_lagrange;      /* [8][9] or NULL: the block weights of arriving
                                populations k = 1..8 over members 0..8           */
    int64_t n_lagrange;      /* written: number of block centres                  */
} mlbm_stencils;

/*
 * Builds, for every node x_i, the stencil of its K nearest nodes (ties broken
 * by the offset vector x_j - x_i: dx, then dy; minimum image on periodic
 * axes) and, for each k = 1..8, the interpolation weights of the cubic
 * polyharmonic spline with quadratic polynomial augmentation (Sec. 2.2,
 * Eq. 13) at the departure point x_i - dx e_k (Sec. 2.2, Eq. 12).  When that
 * point lies inside a solid (a disk, or beyond a no-slip wall), the point
 * x_i + dx e_k with source population k' is used instead (Sec. 3.2, Eq. 22);
 * if both are inside, the node itself with source k' (simple bounce-back).
 * The stencil is shared by the eight departure points of a node (each has
 * its own weights).  Quadrature weights: squared mean distance to the four
 * nearest other nodes, halved for MLBM_WALL / MLBM_DIRICHLET nodes, scaled to
 * sum to geometry->fluid_area.
 * Hybrid sets (lattice_h > 0, Sec. 2.2): a fluid node whose nine nearest nodes
 * are the 3 x 3 lattice block x + lattice_h e_j around it (the tenth lies
 * farther than the block corners), whose departure points all lie in the
 * fluid and with dx <= lattice_h, is a block centre: its members 0..7 are the
 * lattice neighbours x + lattice_h e_1 .. e_8, member 8 is the node itself,
 * any further members the node itself with weight 0, and its weights are the
 * tensor-product quadratic Lagrange weights through the block, the same for
 * every block centre (w_lagrange).  With reorder = 1 or 2 the block centres
 * follow every other node.
 * Errors: MLBM_ERR_ARG (null pointers, K out of range, dx <= 0),
 * MLBM_ERR_GEOMETRY (K > n, node inside a solid, empty box, node outside the
 * box), MLBM_ERR_SINGULAR (a local system is singular or fails to reproduce
 * quadratics to 1e-9; the message names the node and k).
 */
int mlbm_build_stencils(const mlbm_geometry *geometry, const mlbm_stencil_params *params,
                        mlbm_stencils *out);

/* ---- packed device layout ------------------------------------------------- */
/*
 * Kp = K rounded up to a multiple of 4 (padding members point at the node
 * itself with weight 0).  Packed arrays (all little-endian, node index i fast):
 *   idx    int32  [Kp/4][n][4]
 *   w      F64 storage: double [8][Kp/2][n][2]; otherwise float [8][Kp/4][n][4]
 *   flags  uint16 [n]: bits 0-7 = bb, bits 8-9 = kind, bit 10 = MLBM_FLAG_LAGRANGE
 *   state  (MLBM_POPULATIONS) offsets f_k - omega_k of the post-collision
 *          populations: T [n][8] for k = 1..8, then T [n] for k = 0;
 *          (MLBM_FIELDS) T [n][4] = (rho - 1, u_x, u_y, 0);
 *          T = double / float / half (x 2^scale_exp) / bfloat16 by storage.
 */
typedef struct mlbm_sizes {
    int64_t idx_bytes, w_bytes, flags_bytes, state_bytes;
    int32_t k_padded;
} mlbm_sizes;

int mlbm_packed_sizes(int64_t n, int32_t K, int32_t variant, int32_t storage, mlbm_sizes *out);

/*
 * Host-side packing of the builder's output into the device layout above
 * (host buffers in and out, sized by mlbm_packed_sizes).  Weights are
 * rounded to FP32 for every storage except MLBM_F64.
 * Errors: MLBM_ERR_ARG.
 */
int mlbm_pack_stencils(int64_t n, int32_t K, int32_t storage, const int32_t *idx, const double *w,
                       const uint8_t *bb, const uint8_t *kind, void *idx_packed, void *w_packed,
                       uint16_t *flags);

/*
 * The same for nodes [offset, offset + n) of packed arrays sized for n_total
 * nodes (idx, w, bb, kind hold the n rows; idx already counts from 0 of the
 * whole set), so several node sets can be packed into one (batched runs).
 */
int mlbm_pack_stencils_range(int64_t n_total, int64_t offset, int64_t n, int32_t K, int32_t storage,
                             const int32_t *idx, const double *w, const uint8_t *bb, const uint8_t *kind,
                             void *idx_packed, void *w_packed, uint16_t *flags);

/*
 * FP16 copy of packed FP32 weights for mlbm_step_params.weights16 (16-bit
 * states; not in the paper, whose weights are doubles, Sec. 3.2 Eq. 27), in
 * the same layout [8][k_padded/4][n][4].  Every weight becomes one of its two
 * neighbouring FP16 values: first the nearest (ties to even), then, row by
 * row (one row = the k_padded weights of one direction of one node), single
 * weights move to their other neighbour while that brings the row's summed
 * rounding error closer to zero, so each row keeps its FP32 sum as closely as
 * FP16 allows (an interpolation that keeps reproducing constants).  Zero
 * (padding) weights stay zero.  Host buffers, caller owned.
 * Errors: MLBM_ERR_ARG (null pointers, n < 0, k_padded not a positive
 * multiple of 4 within the stencil limit, a weight that is not finite or
 * whose magnitude reaches 65504).
 */
int mlbm_weights_to_f16(int64_t n, int32_t k_padded, const float *in, uint16_t *out);

/*
 * Sets MLBM_FLAG_LAGRANGE in packed flags[i] where lagrange[i] != 0 (the
 * builder's lagrange output), so that mlbm_step takes those nodes' weights
 * from mlbm_device_state.w_lagrange.  Errors: MLBM_ERR_ARG.
 */
#define MLBM_FLAG_LAGRANGE 0x400u  /* flags bit 10: node interpolated on its lattice block */
int mlbm_mark_lagrange(int64_t n, const uint8_t *lagrange, uint16_t *flags);

/*
 * Tile-local indices for LDS staging.  A tile is `tile` (64, 128 or 256)
 * consecutive nodes, processed by one workgroup of that size.  Its halo is the
 * sorted list of distinct nodes referenced by its stencils (its own nodes
 * included).  Outputs (host, caller-allocated):
 *   halo_off int32 [ntiles + 1]   CSR offsets into halo, ntiles = ceil(n / tile)
 *   halo     int32 [total_halo]   node indices
 *   lidx     uint16 [K8/8][n][8]  position of stencil member j of node i in its
 *                                 tile's halo (K8 = K rounded up to 8; padding
 *                                 members point at the node itself)
 * mlbm_tile_sizes returns total_halo and the largest halo.  idx is the
 * builder's [n][K] array (K <= 256 members per row).  For per-departure
 * stencils pass the rows [n][8][K8] (each departure point's K members padded
 * to K8 with the node itself) as K = 8 * K8: the planes of departure point k
 * are then k * K8/8 .. (k + 1) * K8/8 - 1, the layout mlbm_step reads.
 * Errors: MLBM_ERR_ARG.
 */
int mlbm_tile_sizes(int64_t n, int32_t K, int32_t tile, const int32_t *idx, int64_t *total_halo,
                    int32_t *max_halo);
int mlbm_pack_tiles(int64_t n, int32_t K, int32_t tile, const int32_t *idx, int32_t *halo_off,
                    int32_t *halo, uint16_t *lidx);

/* ---- time stepping (device) ------------------------------------------------ */
typedef struct mlbm_step_params {
    int32_t variant;         /* MLBM_POPULATIONS or MLBM_FIELDS                    */
    int32_t storage;         /* MLBM_F64 / MLBM_F32 / MLBM_F16S / MLBM_BF16         */
    double tau_plus;         /* symmetric relaxation time (> 0.5); MLBM_FIELDS: 1 */
    double tau_minus;        /* antisymmetric relaxation time; = tau_plus for BGK */
    double g[2];             /* body acceleration, lattice units                   */
    int32_t scale_exp;       /* MLBM_F16S: stored value = offset * 2^scale_exp     */
    int32_t block;           /* threads per workgroup, multiple of 64 in [64, 1024];
                                0 = 256                                             */
    int32_t xcd_remap;       /* 1 = give each XCD a contiguous range of node tiles */
    int32_t fp32_arith;      /* must be 0: FP32 states collide in FP64 registers (their
                                interpolation sums are FP32).  1 (FP32 collision) is
                                refused with MLBM_ERR_UNSUPPORTED: over 1000 Taylor-Green
                                steps it drifts 2.3e-5 from the FP64 oracle, above the
                                1e-5 bar of FP32 states, for ~1 % of speed          */
    int32_t alternate_sweeps;/* 1 = visit the node tiles in reverse order on every
                                other step (the step reading state[1])             */
    int32_t cached_weights;  /* 1 = ordinary loads for weights and indices; 0 =
                                non-temporal loads                                  */
    int32_t stochastic_rounding; /* MLBM_F16S / MLBM_BF16 in mlbm_step: 1 = round each
                                stored value up or down at random with the
                                probabilities that make it unbiased (random bits
                                from a counter-based hash of node, component and
                                mlbm_device_state.step_count); 0 = to nearest even.
                                Batched runs always round to nearest.              */
    int32_t weights16;       /* MLBM_F16S / MLBM_BF16 only: 1 = the packed weights are
                                FP16 (mlbm_weights_to_f16), half the weight bytes;
                                their sum is then taken as exactly 1 by the step and
                                by the momentum exchange of mlbm_macroscopic, as
                                for FP32 weights.  0 = FP32 weights               */
    int32_t hybrid_launches; /* hybrid sets (w_lagrange set) with tiles: 0 = one launch
                                per step for both node kinds (workgroups of the
                                per-node tiles first, then the block-centre tiles);
                                2 = one launch per kind.  The results are identical */
    int32_t graph_steps;     /* 0: mlbm_step launches every step from the host.  An even
                                G in [2, 4096]: the launches of G steps are captured once
                                into a HIP graph on the caller's stream (not the default
                                stream), kept by the library for later calls with the
                                same arguments (16 graphs, least recently used dropped),
                                and replayed nsteps / G times; the remaining steps are
                                launched directly.  Same results as direct launches;
                                saves launch overhead on node sets too small to fill
                                the GPU.  Not with stochastic rounding (its random bits
                                change every step): MLBM_ERR_UNSUPPORTED.           */
    int32_t lanes_per_node;  /* mlbm_step only.  0 or 1: one lane per node.  8: a group of
                                eight lanes per node, lane k taking arriving population
                                (or departure point) k + 1 and the group exchanging its
                                sums for the collision; the same sums in the same order
                                (equal to rounding: the kernels may fuse multiply-adds
                                differently), eight times the lanes, for node sets too
                                small to fill the GPU.
                                With tile 64 or 128 a workgroup holds 8 x tile lanes;
                                with tile 0, block lanes for block / 8 nodes.  Per-node
                                stencils with K padded to 12, 16, 28 or 32 members, and
                                hybrid sets (w_lagrange) in one launch per step with
                                tile 64 or 128; per-departure stencils, tile 256, and
                                hybrid sets without tiles or with hybrid_launches = 2
                                give MLBM_ERR_UNSUPPORTED                            */
} mlbm_step_params;

typedef struct mlbm_device_state {
    int64_t n;
    int32_t K;               /* stencil size before padding                        */
    const void *idx;         /* device, packed                                     */
    const void *w;           /* device, packed                                     */
    const uint16_t *flags;   /* device [n]                                         */
    const double *bc;        /* device [n][3] (rho_b, ux_b, uy_b), read on Dirichlet
                                nodes only; may be NULL if there are none          */
    void *state[2];          /* device ping-pong state buffers (state_bytes each)  */
    int32_t cur;             /* index (0/1) of the buffer holding the current state;
                                mlbm_step updates it                                */
    int32_t tile;            /* 0: gather stencil members from global memory; 64, 128
                                or 256: stage each tile's halo in LDS (workgroup =
                                tile nodes) using the three arrays below            */
    int32_t max_halo;        /* largest halo (from mlbm_tile_sizes)                 */
    const int32_t *halo_off; /* device copies of mlbm_pack_tiles' outputs           */
    const int32_t *halo;
    const uint16_t *lidx;
    const void *w_lagrange;  /* device [8][9] block weights (double for MLBM_F64
                                storage, float otherwise) or NULL                 */
    int64_t lagrange_begin;  /* with w_lagrange: nodes [lagrange_begin, n) are all
                                block centres flagged MLBM_FLAG_LAGRANGE (the
                                builder's order puts them last); they are updated
                                by a kernel that reads the shared weights and
                                eight neighbour indices per node, every other
                                node by its own packed weights (which the builder
                                also fills for block centres).  lagrange_begin
                                need not fall on a tile boundary: the tile holding
                                it is visited by both kernels, each updating its
                                own nodes.  A node of that range without the flag
                                gets a NaN state.  Batched runs use the packed
                                weights throughout.                                */
    uint64_t step_count;     /* steps taken (key of the stochastic rounding);
                                mlbm_step adds nsteps                              */
    int32_t per_departure;   /* 1: one stencil per departure point (builder's
                                per_departure); needs tiles, lidx as described at
                                mlbm_pack_tiles, weights packed as usual, idx the
                                eight packed stencils one after another
                                ([8][Kp/4][n][4], read by mlbm_macroscopic's
                                wall force); not with w_lagrange or batched runs  */
} mlbm_device_state;

/*
 * Initial state from fields (device FP64 rho [n], u [n][2]): populations are
 * the equilibrium of (rho, u), collided once (state = post-collision, so the
 * first step starts with streaming) with Dirichlet nodes overwritten; MLBM1
 * stores (rho - 1, u) and (rho_b - 1, u_b) on Dirichlet nodes.  Writes
 * state[cur].  Errors: MLBM_ERR_ARG, MLBM_ERR_UNSUPPORTED, MLBM_ERR_HIP.
 */
int mlbm_init_state(const mlbm_step_params *params, mlbm_device_state *state, const double *rho,
                    const double *u, void *hip_stream);

/*
 * Advances nsteps >= 0 time steps.  Each step reads state[cur], writes
 * state[cur ^ 1] (never in place), then flips cur: for every node, stream
 * (Sec. 2.2, Eq. 12; MLBM1: Eqs. 14-15) and collide (Sec. 2.1, Eq. 3) in one
 * kernel pass.  Errors: MLBM_ERR_ARG, MLBM_ERR_UNSUPPORTED, MLBM_ERR_HIP.
 */
int mlbm_step(const mlbm_step_params *params, mlbm_device_state *state, int32_t nsteps,
              void *hip_stream);

/* ---- batched runs (device) ----------------------------------------------------- */
/*
 * Many independent samples (e.g. porous media of uneven size) run as one
 * concatenated node set whose tiles never straddle two samples (pad each
 * sample to a multiple of `tile` nodes with Dirichlet nodes of zero area and
 * no stencil).  mlbm_device_state must use tiles.  Samples are taken in
 * groups (see n_groups): a group whose samples are all active is stepped with
 * one workgroup per tile; once some of its samples have retired, persistent
 * workgroups (at most `grid`) walk the group's part of a device list of active
 * tiles.  Every check_every steps each sample's residual
 * ||u - u_prev|| / ||u|| is formed, samples below tol retire and the list is
 * rebuilt on the device, so captured graphs can be replayed: one per group
 * (captured again when the group loses a sample) and one for the check.
 */
typedef struct mlbm_batch {
    int32_t n_samples;               /* 1 .. 4096                                     */
    int32_t check_every;             /* steps per check, even, >= 2                   */
    int32_t grid;                    /* persistent workgroups (rounded up to 8); 0 = 1024 */
    const int32_t *sample_tile_off;  /* device [n_samples + 1] tiles of sample s are
                                        [off[s], off[s+1]); off[n_samples] = tile count */
    const int32_t *sample_tile_off_host; /* the same offsets on the host (validation)  */
    const double *area;              /* device [n] quadrature weights (0 on padding)  */
    double *u_prev;                  /* device [n][2] workspace                       */
    double *tile_red;                /* device [tiles][4] workspace                   */
    int32_t *queue;                  /* device [tiles] workspace: active tile list     */
    int32_t *counters;               /* device [4]: active tiles, steps, active samples,
                                        checks                                        */
    int32_t *sample_steps;           /* device [n_samples] out: steps to convergence; 0 =
                                        not converged; -steps = unstable (non-finite) */
    double *sample_residual;         /* device [n_samples] out: last residual          */
    double *sample_int_ux;           /* device [n_samples] out: sum A u_x at last check */
    int32_t n_groups;                /* sample groups (>= 1): within a check each group
                                        runs its check_every steps before the next one,
                                        so a group sized to the memory-side cache stays
                                        resident across its steps                      */
    const int32_t *group_sample_off; /* device [n_groups + 1]: samples of group g are
                                        [off[g], off[g+1]); off[n_groups] = n_samples  */
    const int32_t *group_sample_off_host; /* the same on the host (validation)         */
    int32_t *group_queue_off;        /* device [n_groups + 1] workspace                 */
} mlbm_batch;

/*
 * Resets the batch (every sample active) and records the current velocity as
 * u_prev.  Asynchronous.  Errors: MLBM_ERR_ARG, MLBM_ERR_HIP.
 */
int mlbm_batch_init(const mlbm_step_params *params, mlbm_device_state *state, mlbm_batch *batch,
                    void *hip_stream);

/*
 * Runs checks of check_every steps until every sample has retired (residual
 * below tol, or non-finite fields) or max_steps is reached.  With use_graph
 * the steps of each group and the check are captured into HIP graphs on
 * hip_stream (which must not be the default stream) and replayed; a group
 * whose samples have all retired is no longer launched.  Synchronous:
 * waits on hip_stream after each check to read the counters and the group
 * queue ranges.  state->cur is unchanged on return (an
 * even number of steps per check).  *steps_done receives the steps run.
 * Errors: MLBM_ERR_ARG, MLBM_ERR_UNSUPPORTED, MLBM_ERR_HIP.
 */
int mlbm_step_batched(const mlbm_step_params *params, mlbm_device_state *state, mlbm_batch *batch,
                      int32_t max_steps, double tol, int32_t use_graph, int32_t *steps_done,
                      void *hip_stream);

/* ---- macroscopic fields and reductions (device) ------------------------------ */
#define MLBM_RED_MASS      0   /* sum A rho                                         */
#define MLBM_RED_INT_UX    1   /* sum A u_x   (Sec. 3.2, Eq. 23 without 1/phi)      */
#define MLBM_RED_INT_UY    2   /* sum A u_y                                         */
#define MLBM_RED_INT_SPEED 3   /* sum A |u|   (Sec. 3.2, Eq. 25 numerator)           */
#define MLBM_RED_NORM_U2   4   /* sum |u|^2                                         */
#define MLBM_RED_NORM_DU2  5   /* sum |u - u_prev|^2 (0 if u_prev is NULL)          */
#define MLBM_RED_FORCE_X   6   /* momentum exchange on no-slip surfaces, lattice units */
#define MLBM_RED_FORCE_Y   7
#define MLBM_RED_N_BAD     8   /* number of nodes with non-finite fields or rho <= 0 */
#define MLBM_RED_FIRST_BAD 9   /* smallest such node index, or n                    */
#define MLBM_RED_RESIDUAL  10  /* field residual sqrt(NORM_DU2 / NORM_U2) (0 when
                                  NORM_U2 = 0): ||u - u_prev|| / ||u|| over nodes  */
#define MLBM_RED_PREV_INT_UX 11 /* INT_UX that red_out held before this call (NaN
                                  after mlbm_reductions_reset)                     */
#define MLBM_RED_MEAN_CHANGE 12 /* |INT_UX - PREV_INT_UX| / |INT_UX|: the relative
                                  change of the mean velocity between two calls on
                                  the same red_out (Sec. 3.2, Eq. 24's quantity);
                                  NaN when there is no previous value              */
#define MLBM_RED_PERMEABILITY 13 /* Darcy permeability k = nu U_s / g_x dx^2 in the
                                  units of xy squared: nu = (tau+ - 1/2) / 3 in
                                  lattice units, U_s = INT_UX / box_area the
                                  superficial velocity; NaN when g_x = 0 or
                                  box_area <= 0                                     */
#define MLBM_RED_COUNT     14

/* Bytes of the device workspace mlbm_macroscopic needs for n nodes. */
int64_t mlbm_reduction_workspace_bytes(int64_t n);

/*
 * Fills the device array red_out [MLBM_RED_COUNT] with NaN (a kernel, so it
 * may be captured in a graph), so that the next mlbm_macroscopic on it has no
 * previous mean velocity.  Errors: MLBM_ERR_ARG, MLBM_ERR_HIP.
 */
int mlbm_reductions_reset(double *red_out, void *hip_stream);

/*
 * Macroscopic fields of state[cur]: rho and u (populations: u = sum e f / rho
 * - g/2, the half-force-shifted velocity of the pre-collision populations;
 * Dirichlet nodes report (rho_b, u_b)), written as FP64 to rho_out [n] and
 * u_out [n][2] when these are non-NULL.  If u_prev (device FP64 [n][2]) is
 * non-NULL the squared change against it is accumulated and u is then copied
 * into it.  Reductions over nodes with the quadrature weights area (device
 * FP64 [n]) are summed in FP64 in a fixed order (bitwise reproducible) and
 * written to red_out (device FP64 [MLBM_RED_COUNT]); red_out is also read:
 * its MLBM_RED_INT_UX before the call becomes MLBM_RED_PREV_INT_UX.  The
 * force sums, over every bounced (node, k), e_k' (f_k'^post + f_k^new) A / dx^2
 * relative to the rest state.  dx: the streaming distance in the units of xy;
 * box_area: |D| of the superficial velocity (<= 0: no permeability).
 * workspace: device, mlbm_reduction_workspace_bytes(n) bytes.
 * Errors: MLBM_ERR_ARG, MLBM_ERR_UNSUPPORTED, MLBM_ERR_HIP.
 */
int mlbm_macroscopic(const mlbm_step_params *params, const mlbm_device_state *state,
                     const double *area, double dx, double box_area, double *rho_out, double *u_out,
                     double *u_prev, void *workspace, double *red_out, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * fields and reductions as mlbm_macroscopic, with the same kernels, but the
 * per-block partial sums are kept in a static device array inside the
 * library (MLBM_STATIC_MAX_NODES / 256 * 10 doubles = 5 MiB per GPU, held
 * until the process ends) instead of a caller workspace.  The call allocates
 * nothing.  All calls on one GPU share that array: calls that overlap on one
 * GPU (different streams, or threads) race, so serialise them.  Its address
 * is looked up once per device, on the first call with that device current.
 * Errors: as mlbm_macroscopic, plus MLBM_ERR_ARG when n exceeds
 * MLBM_STATIC_MAX_NODES.
 */
#define MLBM_STATIC_MAX_NODES 16777216LL   /* 2^24 nodes */
int mlbm_macroscopic_static(const mlbm_step_params *params, const mlbm_device_state *state,
                            const double *area, double dx, double box_area, double *rho_out, double *u_out,
                            double *u_prev, double *red_out, void *hip_stream);

/* ---- running to a steady state (device, synchronous) --------------------------- */
#define MLBM_STEADY_FIELD 0    /* stop on MLBM_RED_RESIDUAL < tol                   */
#define MLBM_STEADY_MEAN  1    /* stop on MLBM_RED_MEAN_CHANGE < tol (Sec. 3.2, Eq. 24) */

typedef struct mlbm_steady {
    int32_t criterion;       /* MLBM_STEADY_FIELD or MLBM_STEADY_MEAN              */
    int32_t check_every;     /* steps between checks, >= 1                         */
    int32_t hold;            /* consecutive checks below tol needed, >= 1           */
    int64_t max_steps;       /* step cap, >= 0                                      */
    double tol;              /* > 0                                                 */
} mlbm_steady;

/*
 * Steps the state of `state` until it is steady (Sec. 3.2, Eq. 24; the field
 * residual or the relative change of the mean velocity between checks
 * check_every steps apart stays below tol for `hold` checks) or max_steps are
 * taken: mlbm_step and mlbm_macroscopic (with u_prev) alternate, and after
 * each check the reductions are copied to red_host [MLBM_RED_COUNT] (host)
 * and the stream is synchronised.  Before the first step red_out is reset and
 * u_prev (device FP64 [n][2], caller workspace) takes the current velocity.
 * *steps_done receives the steps taken; red_host holds the last check.
 * Returns MLBM_OK whether or not the state settled (compare red_host with
 * tol), MLBM_ERR_UNSTABLE as soon as a check sees a node with non-finite
 * fields or rho <= 0 (the message names the count, the first node and the
 * step), MLBM_ERR_ARG, MLBM_ERR_UNSUPPORTED or MLBM_ERR_HIP otherwise.
 */
int mlbm_run_to_steady(const mlbm_step_params *params, mlbm_device_state *state, const mlbm_steady *steady,
                       const double *area, double dx, double box_area, double *u_prev, void *workspace,
                       double *red_out, double *red_host, int64_t *steps_done, void *hip_stream);

/* Message of the last failure on this thread ("" if none). */
const char *mlbm_last_error(void);

/* Library version string. */
const char *mlbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MLBM_H */
