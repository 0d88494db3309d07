// Host FP64 construction of the meshless stencils and interpolation weights,
// and host packing into the device layout (see include/mlbm.h).
//
// Per node x_i: the K nearest nodes (cell-list search, minimum image on
// periodic axes, ties broken by the offset vector), the departure point of
// each arriving population k = 1..8 at x_i - dx e_k (Sec. 2.2, Eq. 12), moved
// to the mirrored point x_i + dx e_k with source population k' when it falls
// inside a solid (Sec. 3.2, Eq. 22), and the weights of the cubic
// polyharmonic spline interpolant with quadratic augmentation (Sec. 2.2,
// Eq. 13) evaluated there.  The (K+6)x(K+6) interpolation matrix depends only
// on the stencil, so it is factorised once per node (LU with partial
// pivoting) and solved for the eight departure points.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <functional>
#include <limits>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mlbm.h"
#include "mlbm_internal.h"

namespace {

constexpr int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPPOSITE[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
constexpr int MAXK = 32;
constexpr int NPOLY = 6;

struct Box {
    double lo[2], hi[2], len[2];
    bool per[2];
    bool wall_lo, wall_hi;
    double tol;
};

inline void min_image(const Box &b, double &dx, double &dy) {
    if (b.per[0]) {
        if (dx > 0.5 * b.len[0]) dx -= b.len[0];
        else if (dx < -0.5 * b.len[0]) dx += b.len[0];
    }
    if (b.per[1]) {
        if (dy > 0.5 * b.len[1]) dy -= b.len[1];
        else if (dy < -0.5 * b.len[1]) dy += b.len[1];
    }
}

// Uniform grid of cells over the box holding point ids (CSR layout).
struct CellGrid {
    int nx = 1, ny = 1;
    double cx = 1, cy = 1;
    std::vector<int64_t> start, items;

    int cell_x(const Box &b, double x) const {
        int i = (int)std::floor((x - b.lo[0]) / cx);
        return std::min(std::max(i, 0), nx - 1);
    }
    int cell_y(const Box &b, double y) const {
        int j = (int)std::floor((y - b.lo[1]) / cy);
        return std::min(std::max(j, 0), ny - 1);
    }
    void build(const Box &b, const double *pts, int64_t stride, int64_t m, double cell) {
        nx = std::max(1, (int)std::floor(b.len[0] / cell));
        ny = std::max(1, (int)std::floor(b.len[1] / cell));
        nx = std::min(nx, 1 << 14);
        ny = std::min(ny, 1 << 14);
        cx = b.len[0] / nx;
        cy = b.len[1] / ny;
        std::vector<int64_t> count((size_t)nx * ny + 1, 0);
        std::vector<int32_t> cid(m);
        for (int64_t p = 0; p < m; ++p) {
            int c = cell_y(b, pts[p * stride + 1]) * nx + cell_x(b, pts[p * stride]);
            cid[p] = c;
            count[c + 1]++;
        }
        for (size_t c = 0; c < (size_t)nx * ny; ++c) count[c + 1] += count[c];
        start = count;
        items.assign(m, 0);
        std::vector<int64_t> fill(count.begin(), count.end() - 1);
        for (int64_t p = 0; p < m; ++p) items[fill[cid[p]]++] = p;
    }
};

struct Cand {
    double r2, dx, dy;
    int64_t j;
};

inline bool cand_less(const Cand &a, const Cand &b) {
    if (a.r2 != b.r2) return a.r2 < b.r2;
    if (a.dx != b.dx) return a.dx < b.dx;
    return a.dy < b.dy;
}

struct Builder {
    const mlbm_geometry *g;
    Box box;
    int K;
    double dx;
    CellGrid nodes, disks;
    double rmax = 0;
    double lat_h = 0;          // lattice spacing of the regular part (0: none)
    bool per_departure = false;  // one stencil per departure point (else one per node)
    bool simple_bb = false;      // bounce-back at the node itself (else the mirrored point)
    double wlag[8][9] = {};    // biquadratic Lagrange weights shared by block centres

    // ---- regular blocks of a hybrid set (Sec. 2.2) -------------------------
    // quadratic Lagrange basis through -1, 0, 1, the one that is 1 at a
    static double lag1(int a, double t) {
        switch (a) {
            case -1: return 0.5 * t * (t - 1.0);
            case 0: return (1.0 - t) * (1.0 + t);
            default: return 0.5 * t * (t + 1.0);
        }
    }

    // member slot of the lattice node x + h e_d: the neighbours d = 1..8 take
    // slots 0..7 (one index plane on the device), the node itself slot 8
    static int slot_of(int d) { return d == 0 ? 8 : d - 1; }

    void lagrange_table() {
        for (int k = 1; k <= 8; ++k) {
            const double tx = -dx * EX[k] / lat_h, ty = -dx * EY[k] / lat_h;
            for (int d = 0; d < 9; ++d) wlag[k - 1][slot_of(d)] = lag1(EX[d], tx) * lag1(EY[d], ty);
        }
    }

    // True if the nine nearest nodes of i are x_i + h e_d (d = 0..8, each within
    // 1e-9 h) and the tenth lies beyond the block corners; mem[slot_of(d)]
    // receives the node at x_i + h e_d.
    bool lattice_block(int64_t i, std::vector<Cand> &cand, int64_t *mem) const {
        Cand st[10];
        nearest_n(i, 10, cand, st);
        const double h = lat_h, tol = 1e-9 * h;
        const double corner = std::sqrt(2.0) * h * (1.0 + 1e-9);
        if (!(st[9].r2 > corner * corner)) return false;
        unsigned seen = 0;
        for (int t = 0; t < 9; ++t) {
            const long a = std::lround(st[t].dx / h), b = std::lround(st[t].dy / h);
            if (a < -1 || a > 1 || b < -1 || b > 1) return false;
            if (std::hypot(st[t].dx - (double)a * h, st[t].dy - (double)b * h) > tol) return false;
            int d = 0;
            while (EX[d] != a || EY[d] != b) ++d;
            if (seen & (1u << d)) return false;
            seen |= 1u << d;
            mem[slot_of(d)] = st[t].j;
        }
        return seen == 0x1ffu;
    }

    // A fluid node is interpolated on its block when the streaming distance
    // fits in the block and no departure point needs the bounce-back rule.
    bool is_block_centre(int64_t i, std::vector<Cand> &cand, int64_t *mem) const {
        if (!(lat_h > 0.0) || g->kind[i] != MLBM_FLUID || dx > lat_h) return false;
        const double xi = g->xy[2 * i], yi = g->xy[2 * i + 1];
        for (int k = 1; k <= 8; ++k)
            if (inside_solid(xi - dx * EX[k], yi - dx * EY[k])) return false;
        return lattice_block(i, cand, mem);
    }

    // ---- K nearest neighbours --------------------------------------------
    void nearest(int64_t i, std::vector<Cand> &cand, Cand *out) const { nearest_n(i, K, cand, out); }

    // The K nearest nodes of the point x_i + (ox, oy); offsets are formed as
    // (x_j - x_i) - o, so on a lattice every node's point sees the same
    // offsets and ties.
    void nearest_n(int64_t i, int K, std::vector<Cand> &cand, Cand *out, double ox = 0.0, double oy = 0.0) const {
        const double xi = g->xy[2 * i], yi = g->xy[2 * i + 1];
        cand.clear();
        double px = xi + ox, py = yi + oy, slack2 = 0.0;
        for (int a = 0; a < 2; ++a) {
            double &v = a ? py : px;
            if (box.per[a]) {
                v = box.lo[a] + std::fmod(v - box.lo[a], box.len[a]);
                if (v < box.lo[a]) v += box.len[a];
            } else {
                // a point outside a non-periodic box: the ring search counts
                // its radius from the box edge
                const double out_d = std::max({box.lo[a] - v, 0.0, v - box.hi[a]});
                slack2 += out_d * out_d;
            }
        }
        const double slack = std::sqrt(slack2);
        const int ci = nodes.cell_x(box, px), cj = nodes.cell_y(box, py);
        const double cmin = std::min(nodes.cx, nodes.cy);
        const int rmax_ring = std::max(nodes.nx, nodes.ny);
        bool brute = false;
        for (int r = 0;; ++r) {
            if ((box.per[0] && 2 * r + 1 > nodes.nx) || (box.per[1] && 2 * r + 1 > nodes.ny) ||
                r > rmax_ring) {
                brute = true;
                break;
            }
            for (int dj = -r; dj <= r; ++dj) {
                for (int di = -r; di <= r; ++di) {
                    if (std::max(std::abs(di), std::abs(dj)) != r) continue;
                    int a = ci + di, b = cj + dj;
                    if (box.per[0]) a = (a % nodes.nx + nodes.nx) % nodes.nx;
                    else if (a < 0 || a >= nodes.nx) continue;
                    if (box.per[1]) b = (b % nodes.ny + nodes.ny) % nodes.ny;
                    else if (b < 0 || b >= nodes.ny) continue;
                    const int c = b * nodes.nx + a;
                    for (int64_t q = nodes.start[c]; q < nodes.start[c + 1]; ++q) {
                        const int64_t j = nodes.items[q];
                        double ddx = g->xy[2 * j] - xi, ddy = g->xy[2 * j + 1] - yi;
                        min_image(box, ddx, ddy);
                        ddx -= ox;
                        ddy -= oy;
                        cand.push_back({ddx * ddx + ddy * ddy, ddx, ddy, j});
                    }
                }
            }
            if ((int)cand.size() >= K) {
                std::nth_element(cand.begin(), cand.begin() + (K - 1), cand.end(), cand_less);
                const double kth = cand[K - 1].r2;
                const double reach = r * cmin - slack;
                if (reach > 0.0 && kth < reach * reach) break;
            }
        }
        if (brute) {
            cand.clear();
            for (int64_t j = 0; j < g->n; ++j) {
                double ddx = g->xy[2 * j] - xi, ddy = g->xy[2 * j + 1] - yi;
                min_image(box, ddx, ddy);
                ddx -= ox;
                ddy -= oy;
                cand.push_back({ddx * ddx + ddy * ddy, ddx, ddy, j});
            }
        }
        std::partial_sort(cand.begin(), cand.begin() + K, cand.end(), cand_less);
        std::copy(cand.begin(), cand.begin() + K, out);
    }

    // ---- solids ------------------------------------------------------------
    bool inside_solid(double px, double py) const {
        if (box.wall_lo && py < box.lo[1] - box.tol) return true;
        if (box.wall_hi && py > box.hi[1] + box.tol) return true;
        if (g->n_disks == 0) return false;
        const int ci = disks.cell_x(box, px), cj = disks.cell_y(box, py);
        for (int dj = -1; dj <= 1; ++dj) {
            for (int di = -1; di <= 1; ++di) {
                int a = ci + di, b = cj + dj;
                if (box.per[0]) a = (a % disks.nx + disks.nx) % disks.nx;
                else if (a < 0 || a >= disks.nx) continue;
                if (box.per[1]) b = (b % disks.ny + disks.ny) % disks.ny;
                else if (b < 0 || b >= disks.ny) continue;
                const int c = b * disks.nx + a;
                for (int64_t q = disks.start[c]; q < disks.start[c + 1]; ++q) {
                    const double *d = g->disks + 3 * disks.items[q];
                    double ddx = px - d[0], ddy = py - d[1];
                    min_image(box, ddx, ddy);
                    const double r = d[2] - box.tol;
                    if (ddx * ddx + ddy * ddy < r * r) return true;
                }
            }
        }
        return false;
    }

    // ---- local interpolation -----------------------------------------------
    static void poly2(double x, double y, double *p) {
        p[0] = 1.0;
        p[1] = x;
        p[2] = y;
        p[3] = x * x;
        p[4] = x * y;
        p[5] = y * y;
    }

    // LU factorisation with partial pivoting of the m x m row-major matrix a.
    // Returns false if a pivot vanishes relative to the largest entry.
    static bool lu(double *a, int *piv, int m) {
        double amax = 0;
        for (int t = 0; t < m * m; ++t) amax = std::max(amax, std::fabs(a[t]));
        for (int c = 0; c < m; ++c) {
            int p = c;
            double best = std::fabs(a[c * m + c]);
            for (int r = c + 1; r < m; ++r) {
                const double v = std::fabs(a[r * m + c]);
                if (v > best) { best = v; p = r; }
            }
            if (!(best > 1e-13 * amax)) return false;
            piv[c] = p;
            if (p != c)
                for (int t = 0; t < m; ++t) std::swap(a[c * m + t], a[p * m + t]);
            const double inv = 1.0 / a[c * m + c];
            for (int r = c + 1; r < m; ++r) {
                const double l = a[r * m + c] * inv;
                a[r * m + c] = l;
                if (l != 0.0)
                    for (int t = c + 1; t < m; ++t) a[r * m + t] -= l * a[c * m + t];
            }
        }
        return true;
    }

    // Solves with the factors of lu(): row interchanges first (the stored
    // multipliers were swapped with their rows), then L, then U.
    static void lu_solve(const double *a, const int *piv, int m, double *b) {
        for (int c = 0; c < m; ++c)
            if (piv[c] != c) std::swap(b[c], b[piv[c]]);
        for (int c = 0; c < m; ++c)
            for (int r = c + 1; r < m; ++r) b[r] -= a[r * m + c] * b[c];
        for (int r = m - 1; r >= 0; --r) {
            double s = b[r];
            for (int t = r + 1; t < m; ++t) s -= a[r * m + t] * b[t];
            b[r] = s / a[r * m + r];
        }
    }

    // Local PHS3 + P2 fit (Sec. 2.2, Eq. 13) through K stencil members whose
    // offsets from a common origin are given: coordinates scaled by the stencil
    // radius, the saddle-point matrix factored on first use, then the weights
    // of any evaluation point.
    struct Fit {
        int K = 0, m = 0;
        double R = 0;
        double A[(MAXK + NPOLY) * (MAXK + NPOLY)];
        int piv[MAXK + NPOLY];
        double xs[MAXK], ys[MAXK];
        bool factored = false;

        void setup(const Cand *st, int k_members) {
            K = k_members;
            m = K + NPOLY;
            R = 0;
            for (int j = 0; j < K; ++j) R = std::max(R, std::hypot(st[j].dx, st[j].dy));
            for (int j = 0; j < K; ++j) {
                xs[j] = st[j].dx / R;
                ys[j] = st[j].dy / R;
            }
            for (int r = 0; r < m; ++r)
                for (int c = 0; c < m; ++c) A[r * m + c] = 0.0;
            for (int r = 0; r < K; ++r) {
                for (int c = 0; c < K; ++c) {
                    const double rr = std::hypot(xs[r] - xs[c], ys[r] - ys[c]);
                    A[r * m + c] = rr * rr * rr;
                }
                double p[NPOLY];
                poly2(xs[r], ys[r], p);
                for (int t = 0; t < NPOLY; ++t) {
                    A[r * m + K + t] = p[t];
                    A[(K + t) * m + r] = p[t];
                }
            }
            factored = false;
        }

        // weights wk[K] of the point (ox, oy) (offset from the origin); returns
        // MLBM_OK, MLBM_ERR_SINGULAR (system singular) or -100 (the quadratics
        // are not reproduced)
        int weights(double ox, double oy, double *wk) {
            const double px = ox / R, py = oy / R;
            int jn = 0;
            double dn = std::numeric_limits<double>::infinity();
            double rp[MAXK];
            for (int j = 0; j < K; ++j) {
                rp[j] = std::hypot(xs[j] - px, ys[j] - py);
                if (rp[j] < dn) { dn = rp[j]; jn = j; }
            }
            if (dn < 1e-12) {  // evaluation point on a node: the value there
                for (int j = 0; j < K; ++j) wk[j] = 0.0;
                wk[jn] = 1.0;
                return MLBM_OK;
            }
            if (!factored) {
                if (!lu(A, piv, m)) return MLBM_ERR_SINGULAR;
                factored = true;
            }
            double b[MAXK + NPOLY];
            for (int j = 0; j < K; ++j) b[j] = rp[j] * rp[j] * rp[j];
            poly2(px, py, b + K);
            lu_solve(A, piv, m, b);
            for (int j = 0; j < K; ++j) wk[j] = b[j];
            double pe[NPOLY], acc[NPOLY] = {0, 0, 0, 0, 0, 0};
            poly2(px, py, pe);
            for (int j = 0; j < K; ++j) {
                double pj[NPOLY];
                poly2(xs[j], ys[j], pj);
                for (int t = 0; t < NPOLY; ++t) acc[t] += wk[j] * pj[t];
            }
            for (int t = 0; t < NPOLY; ++t)
                if (!(std::fabs(acc[t] - pe[t]) <= 1e-9)) return -100;
            return MLBM_OK;
        }
    };

    // Stencil(s), weights, bounce-back bits and unnormalised area of node i.
    // st receives the members: K of them (shared stencil), or 8 x MAXK (one
    // stencil per departure point, k-th at st + k * MAXK).  Returns MLBM_OK
    // or an error code with the message in err.
    int node(int64_t i, bool lag, std::vector<Cand> &cand, Cand *st, double *w, uint8_t *bbits,
             double *area, std::string &err) const {
        nearest(i, cand, st);
        if (st[0].j != i || (K > 1 && st[1].r2 == 0.0)) {
            err = "duplicate node coordinates at node " + std::to_string(i);
            return MLBM_ERR_GEOMETRY;
        }
        // quadrature weight: squared mean distance to the 4 nearest other nodes
        double s = 0;
        for (int t = 1; t <= 4; ++t) s += std::hypot(st[t].dx, st[t].dy);
        const double mean = s / 4.0;
        *area = mean * mean * (g->kind[i] != MLBM_FLUID ? 0.5 : 1.0);
        *bbits = 0;
        if (lag) {
            int64_t mem[9];
            if (!is_block_centre(i, cand, mem)) {
                err = "node " + std::to_string(i) + " lost its lattice block";
                return MLBM_ERR_GEOMETRY;
            }
            for (int j = 0; j < K; ++j) {
                st[j].j = j < 9 ? mem[j] : i;
                for (int k = 0; k < 8; ++k) w[(int64_t)k * K + j] = j < 9 ? wlag[k][j] : 0.0;
            }
            if (per_departure)
                for (int k = 1; k < 8; ++k) std::copy(st, st + K, st + k * MAXK);
            return MLBM_OK;
        }
        // departure points and source populations (Sec. 2.2 Eq. 12; Sec. 3.2
        // Eq. 22, or simple bounce-back at the node, Sec. 3.1)
        const double xi = g->xy[2 * i], yi = g->xy[2 * i + 1];
        double ox[8], oy[8];
        for (int k = 1; k <= 8; ++k) {
            double a = -dx * EX[k], b = -dx * EY[k];
            if (inside_solid(xi + a, yi + b)) {
                *bbits |= (uint8_t)(1u << (k - 1));
                if (!simple_bb && !inside_solid(xi - a, yi - b)) {
                    a = -a;
                    b = -b;
                } else {
                    a = 0.0;
                    b = 0.0;
                }
            }
            ox[k - 1] = a;
            oy[k - 1] = b;
        }
        Fit fit;
        if (!per_departure) fit.setup(st, K);
        for (int k = 1; k <= 8; ++k) {
            double *wk = w + (int64_t)(k - 1) * K;
            int rc;
            if (per_departure) {
                // the K nearest nodes of the departure point, weights at that point
                Cand *stk = st + (k - 1) * MAXK;
                nearest_n(i, K, cand, stk, ox[k - 1], oy[k - 1]);
                fit.setup(stk, K);
                rc = fit.weights(0.0, 0.0, wk);
            } else {
                rc = fit.weights(ox[k - 1], oy[k - 1], wk);
            }
            if (rc == MLBM_ERR_SINGULAR) {
                err = "singular interpolation system at node " + std::to_string(i);
                return MLBM_ERR_SINGULAR;
            }
            if (rc != MLBM_OK) {
                err = "interpolation at node " + std::to_string(i) + ", k=" + std::to_string(k) +
                      " does not reproduce quadratics";
                return MLBM_ERR_SINGULAR;
            }
        }
        return MLBM_OK;
    }
};

uint64_t spread_bits(uint32_t v) {
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

}  // namespace

extern "C" int mlbm_build_stencils(const mlbm_geometry *g, const mlbm_stencil_params *p,
                                   mlbm_stencils *out) {
    using mlbm::fail;
    mlbm::clear_error();
    if (!g || !p || !out || !g->xy || !g->kind || !out->perm || !out->idx || !out->w || !out->bb ||
        !out->area)
        return fail(MLBM_ERR_ARG, "null pointer argument");
    if (g->n_disks < 0 || (g->n_disks > 0 && !g->disks)) return fail(MLBM_ERR_ARG, "bad disk list");
    if (p->K < 7 || p->K > MAXK) return fail(MLBM_ERR_ARG, "K=%d outside [7, %d]", p->K, MAXK);
    if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return fail(MLBM_ERR_ARG, "dx must be positive");
    if (p->reorder < 0 || p->reorder > 2) return fail(MLBM_ERR_ARG, "reorder must be 0, 1 or 2");
    if (!(p->lattice_h >= 0.0) || !std::isfinite(p->lattice_h)) return fail(MLBM_ERR_ARG, "lattice_h must be >= 0");
    if (p->lattice_h > 0.0 && p->K < 10) return fail(MLBM_ERR_ARG, "hybrid stencils need K >= 10");
    const int64_t n = g->n;
    if (n < p->K) return fail(MLBM_ERR_GEOMETRY, "K=%d exceeds the node count %lld", p->K, (long long)n);

    Builder B;
    B.g = g;
    B.K = p->K;
    B.dx = p->dx;
    B.lat_h = p->lattice_h;
    B.per_departure = p->per_departure != 0;
    B.simple_bb = p->simple_bounce_back != 0;
    if (B.lat_h > 0.0) B.lagrange_table();
    for (int a = 0; a < 2; ++a) {
        B.box.lo[a] = g->lo[a];
        B.box.hi[a] = g->hi[a];
        B.box.len[a] = g->hi[a] - g->lo[a];
        B.box.per[a] = g->periodic[a] != 0;
        if (!(B.box.len[a] > 0.0)) return fail(MLBM_ERR_GEOMETRY, "empty box");
    }
    B.box.wall_lo = g->wall_lo_y != 0;
    B.box.wall_hi = g->wall_hi_y != 0;
    B.box.tol = 1e-12 * std::max(B.box.len[0], B.box.len[1]);
    for (int64_t i = 0; i < n; ++i) {
        const double x = g->xy[2 * i], y = g->xy[2 * i + 1];
        if (!std::isfinite(x) || !std::isfinite(y) || x < g->lo[0] - B.box.tol ||
            x > g->hi[0] + B.box.tol || y < g->lo[1] - B.box.tol || y > g->hi[1] + B.box.tol)
            return fail(MLBM_ERR_GEOMETRY, "node %lld outside the box", (long long)i);
        if (g->kind[i] > MLBM_DIRICHLET) return fail(MLBM_ERR_ARG, "node %lld has kind %d", (long long)i, g->kind[i]);
    }
    for (int64_t d = 0; d < g->n_disks; ++d) {
        if (!(g->disks[3 * d + 2] > 0.0)) return fail(MLBM_ERR_GEOMETRY, "disk %lld has no radius", (long long)d);
        B.rmax = std::max(B.rmax, g->disks[3 * d + 2]);
    }
    const double cell = std::sqrt(B.box.len[0] * B.box.len[1] / (double)n) * 1.5;
    B.nodes.build(B.box, g->xy, 2, n, cell);
    if (g->n_disks > 0) B.disks.build(B.box, g->disks, 3, g->n_disks, B.rmax);
    for (int64_t i = 0; i < n; ++i)
        if (B.inside_solid(g->xy[2 * i], g->xy[2 * i + 1]))
            return fail(MLBM_ERR_GEOMETRY, "node %lld lies inside a solid", (long long)i);

    int nthreads = p->n_threads > 0 ? p->n_threads : (int)std::thread::hardware_concurrency();
    nthreads = std::max(1, std::min(nthreads, 256));
    auto parallel = [&](const std::function<void(int64_t, int64_t, std::vector<Cand> &)> &body) {
        std::atomic<int64_t> next(0);
        const int64_t chunk = 512;
        auto run = [&]() {
            std::vector<Cand> cand;
            cand.reserve(256);
            for (;;) {
                const int64_t a = next.fetch_add(chunk);
                if (a >= n) break;
                body(a, std::min(n, a + chunk), cand);
            }
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nthreads; ++t) pool.emplace_back(run);
        run();
        for (auto &t : pool) t.join();
    };

    // block centres of the regular part (caller's order)
    std::vector<uint8_t> lag(n, 0);
    if (B.lat_h > 0.0)
        parallel([&](int64_t a, int64_t b, std::vector<Cand> &cand) {
            int64_t mem[9];
            for (int64_t i = a; i < b; ++i) lag[i] = B.is_block_centre(i, cand, mem) ? 1 : 0;
        });

    // node order: Morton (Z) order of the coordinates quantised to 2^20 cells;
    // in a hybrid set the block centres come after every other node
    std::vector<int64_t> perm(n), inv(n);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    if (p->reorder == 1) {
        std::vector<uint64_t> key(n);
        const double q = (double)(1u << 20);
        for (int64_t i = 0; i < n; ++i) {
            double fx = (g->xy[2 * i] - g->lo[0]) / B.box.len[0];
            double fy = (g->xy[2 * i + 1] - g->lo[1]) / B.box.len[1];
            uint32_t ix = (uint32_t)std::min(std::max(fx * q, 0.0), q - 1);
            uint32_t iy = (uint32_t)std::min(std::max(fy * q, 0.0), q - 1);
            key[i] = spread_bits(ix) | (spread_bits(iy) << 1);
        }
        std::stable_sort(perm.begin(), perm.end(), [&](int64_t a, int64_t b) {
            return lag[a] != lag[b] ? lag[a] < lag[b] : key[a] < key[b];
        });
    } else if (p->reorder == 2) {
        // reverse Cuthill-McKee order of the undirected graph that links every
        // node with its K nearest nodes: breadth-first from a far node of each
        // connected part, unvisited neighbours in order of increasing degree
        // (ties: nearer first), the whole sequence reversed
        const int Kg = p->K;
        std::vector<int32_t> out_nb((size_t)n * Kg);
        parallel([&](int64_t a, int64_t b, std::vector<Cand> &cand) {
            Cand nb[8 * MAXK];
            for (int64_t i = a; i < b; ++i) {
                B.nearest_n(i, Kg, cand, nb);
                for (int j = 0; j < Kg; ++j) out_nb[(size_t)i * Kg + j] = (int32_t)nb[j].j;
            }
        });
        std::vector<int64_t> start(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) start[i + 1] += Kg;
        for (size_t e = 0; e < out_nb.size(); ++e) start[out_nb[e] + 1] += 1;
        for (int64_t i = 0; i < n; ++i) start[i + 1] += start[i];
        std::vector<int32_t> nbr(start[n]);
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int j = 0; j < Kg; ++j) nbr[fill[i]++] = out_nb[(size_t)i * Kg + j];
        for (int64_t i = 0; i < n; ++i)
            for (int j = 0; j < Kg; ++j) {
                const int32_t w = out_nb[(size_t)i * Kg + j];
                nbr[fill[w]++] = (int32_t)i;
            }
        auto degree = [&](int64_t v) { return start[v + 1] - start[v]; };
        for (int64_t i = 0; i < n; ++i)
            std::stable_sort(nbr.begin() + start[i], nbr.begin() + start[i + 1],
                             [&](int32_t x, int32_t y) { return degree(x) < degree(y); });
        // visit stamps: 0 unvisited, 1 placed, 2 + c reached by the trial search of part c
        std::vector<int64_t> mark(n, 0), trial;
        std::vector<int64_t> order;
        order.reserve(n);
        auto bfs = [&](int64_t s0, std::vector<int64_t> &seq, int64_t stamp) {
            size_t head = seq.size();
            seq.push_back(s0);
            mark[s0] = stamp;
            while (head < seq.size()) {
                const int64_t v = seq[head++];
                for (int64_t e = start[v]; e < start[v + 1]; ++e) {
                    const int64_t w = nbr[e];
                    if (mark[w] != stamp && mark[w] != 1) { mark[w] = stamp; seq.push_back(w); }
                }
            }
        };
        int64_t part = 0;
        for (int64_t s0 = 0; s0 < n; ++s0) {
            if (mark[s0] == 1) continue;
            trial.clear();
            bfs(s0, trial, 2 + part++);   // the last node reached lies far from s0
            bfs(trial.back(), order, 1);
        }
        std::reverse(order.begin(), order.end());
        perm = order;
        std::stable_partition(perm.begin(), perm.end(), [&](int64_t v) { return lag[v] == 0; });
    }
    for (int64_t i = 0; i < n; ++i) inv[perm[i]] = i;

    std::mutex emu;
    int64_t err_node = n;
    int err_code = MLBM_OK;
    std::string err_msg;
    const int K = p->K;
    const int P = B.per_departure ? 8 : 1;
    parallel([&](int64_t a, int64_t b, std::vector<Cand> &cand) {
        Cand st[8 * MAXK];
        for (int64_t inew = a; inew < b; ++inew) {
            const int64_t i = perm[inew];
            std::string msg;
            double area = 0;
            uint8_t bits = 0;
            const int rc = B.node(i, lag[i] != 0, cand, st, out->w + inew * 8 * K, &bits, &area, msg);
            if (rc != MLBM_OK) {
                std::lock_guard<std::mutex> lk(emu);
                if (i < err_node) { err_node = i; err_code = rc; err_msg = msg; }
                continue;
            }
            for (int k = 0; k < P; ++k)
                for (int j = 0; j < K; ++j) out->idx[(inew * P + k) * K + j] = (int32_t)inv[st[k * MAXK + j].j];
            out->bb[inew] = bits;
            out->area[inew] = area;
            out->perm[inew] = i;
            if (out->lagrange) out->lagrange[inew] = lag[i];
        }
    });
    if (err_code != MLBM_OK) return fail(err_code, "%s", err_msg.c_str());
    out->n_lagrange = 0;
    for (int64_t i = 0; i < n; ++i) out->n_lagrange += lag[i];
    if (out->w_lagrange)
        for (int k = 0; k < 8; ++k)
            for (int j = 0; j < 9; ++j) out->w_lagrange[k * 9 + j] = B.lat_h > 0.0 ? B.wlag[k][j] : 0.0;

    double fluid = g->fluid_area;
    if (!(fluid > 0.0)) {
        fluid = B.box.len[0] * B.box.len[1];
        for (int64_t d = 0; d < g->n_disks; ++d) fluid -= M_PI * g->disks[3 * d + 2] * g->disks[3 * d + 2];
    }
    // normalisation sums in the caller's node order
    double total = 0;
    for (int64_t i = 0; i < n; ++i) total += out->area[inv[i]];
    const double scale = fluid / total;
    for (int64_t i = 0; i < n; ++i) out->area[i] *= scale;
    return MLBM_OK;
}

extern "C" int mlbm_packed_sizes(int64_t n, int32_t K, int32_t variant, int32_t storage, mlbm_sizes *out) {
    using mlbm::fail;
    mlbm::clear_error();
    if (!out) return fail(MLBM_ERR_ARG, "null output");
    if (n < 1 || K < 1 || K > MAXK) return fail(MLBM_ERR_ARG, "bad n or K");
    if (storage < MLBM_F64 || storage > MLBM_BF16) return fail(MLBM_ERR_ARG, "bad storage %d", storage);
    if (variant != MLBM_POPULATIONS && variant != MLBM_FIELDS) return fail(MLBM_ERR_ARG, "bad variant %d", variant);
    const int kp = (K + 3) / 4 * 4;
    const int64_t ts = storage == MLBM_F64 ? 8 : storage == MLBM_F32 ? 4 : 2;
    out->k_padded = kp;
    out->idx_bytes = (int64_t)kp * n * 4;
    out->w_bytes = (int64_t)8 * kp * n * (storage == MLBM_F64 ? 8 : 4);
    out->flags_bytes = n * 2;
    out->state_bytes = variant == MLBM_POPULATIONS ? 9 * n * ts : 4 * n * ts;
    return MLBM_OK;
}

extern "C" int mlbm_pack_stencils_range(int64_t n_total, int64_t offset, int64_t n, int32_t K, int32_t storage,
                                        const int32_t *idx, const double *w, const uint8_t *bb, const uint8_t *kind,
                                        void *idx_packed, void *w_packed, uint16_t *flags) {
    using mlbm::fail;
    mlbm::clear_error();
    if (!idx || !w || !bb || !kind || !idx_packed || !w_packed || !flags) return fail(MLBM_ERR_ARG, "null pointer argument");
    if (n < 1 || K < 1 || K > MAXK || offset < 0 || offset + n > n_total) return fail(MLBM_ERR_ARG, "bad n, offset or K");
    if (storage < MLBM_F64 || storage > MLBM_BF16) return fail(MLBM_ERR_ARG, "bad storage %d", storage);
    const int kp = (K + 3) / 4 * 4;
    const int64_t N = n_total;
    int32_t *ip = (int32_t *)idx_packed;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t i = offset + r;
        for (int j = 0; j < kp; ++j) {
            const int32_t v = j < K ? idx[r * K + j] : (int32_t)i;
            if (v < 0 || v >= N) return fail(MLBM_ERR_ARG, "stencil index out of range at node %lld", (long long)i);
            ip[((int64_t)(j / 4) * N + i) * 4 + (j % 4)] = v;
        }
        flags[i] = (uint16_t)(bb[r] | ((uint16_t)(kind[r] & 3) << 8));
    }
    if (storage == MLBM_F64) {
        double *wp = (double *)w_packed;
        const int kh = kp / 2;
        for (int64_t r = 0; r < n; ++r)
            for (int k = 0; k < 8; ++k)
                for (int j = 0; j < kp; ++j)
                    wp[(((int64_t)k * kh + j / 2) * N + offset + r) * 2 + (j % 2)] = j < K ? w[(r * 8 + k) * K + j] : 0.0;
    } else {
        float *wp = (float *)w_packed;
        const int kq = kp / 4;
        for (int64_t r = 0; r < n; ++r)
            for (int k = 0; k < 8; ++k)
                for (int j = 0; j < kp; ++j)
                    wp[(((int64_t)k * kq + j / 4) * N + offset + r) * 4 + (j % 4)] =
                        j < K ? (float)w[(r * 8 + k) * K + j] : 0.0f;
    }
    return MLBM_OK;
}

// IEEE binary32 -> binary16, round to nearest with ties to even (finite
// inputs below 65520 in magnitude, checked by the caller)
static uint16_t f32_to_f16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t sign = (u >> 16) & 0x8000u;
    const int32_t e = (int32_t)((u >> 23) & 0xffu) - 127;  // unbiased exponent
    uint32_t m = u & 0x7fffffu;
    if (e < -25) return (uint16_t)sign;  // below half the smallest subnormal: 0
    if (e < -14) {
        // subnormal result: value = m' * 2^-24 with m' = (1.m) * 2^(e + 24)
        m |= 0x800000u;
        const int shift = -e - 1;  // 14 .. 24: bits dropped from the 24-bit significand
        const uint32_t q = m >> shift, rem = m & ((1u << shift) - 1u), half = 1u << (shift - 1);
        const uint32_t r = q + ((rem > half || (rem == half && (q & 1u))) ? 1u : 0u);
        return (uint16_t)(sign | r);  // r = 0x400 is the smallest normal: still right
    }
    // normal result: keep 10 of the 23 fraction bits
    uint32_t h = ((uint32_t)(e + 15) << 10) | (m >> 13);
    const uint32_t rem = m & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) h += 1;  // may carry into the exponent
    return (uint16_t)(sign | h);
}

static double f16_value(uint16_t h) {
    const int e = (h >> 10) & 0x1f;
    const double m = (double)(h & 0x3ff);
    const double v = e == 0 ? std::ldexp(m, -24) : std::ldexp(1024.0 + m, e - 25);
    return (h & 0x8000u) ? -v : v;
}

// the FP16 value next to h towards +infinity (up) or -infinity
static uint16_t f16_step(uint16_t h, bool up) {
    const bool neg = (h & 0x8000u) != 0, zero = (h & 0x7fffu) == 0;
    if (zero) return up ? 0x0001u : 0x8001u;
    return (uint16_t)(up != neg ? h + 1 : h - 1);
}

extern "C" int mlbm_weights_to_f16(int64_t n, int32_t k_padded, const float *in, uint16_t *out) {
    using mlbm::fail;
    mlbm::clear_error();
    if (n < 0 || k_padded < 4 || k_padded % 4 != 0 || k_padded > MAXK + 3 || (n > 0 && (!in || !out)))
        return fail(MLBM_ERR_ARG, "bad n, k_padded or null buffer");
    const int64_t count = 8 * (int64_t)k_padded * n;
    for (int64_t t = 0; t < count; ++t)
        if (!std::isfinite(in[t]) || std::fabs(in[t]) >= 65504.0f)
            return fail(MLBM_ERR_ARG, "weight %lld (%g) outside the FP16 range", (long long)t, (double)in[t]);
    const int kq = k_padded / 4;
    // every (direction, node) row: round each weight to nearest, then move
    // single weights to their other FP16 neighbour while that brings the
    // row's sum of rounding errors closer to zero (rows are independent:
    // node ranges on all host threads)
    auto rows = [&](int64_t i0, int64_t i1) {
    for (int k = 0; k < 8; ++k)
        for (int64_t i = i0; i < i1; ++i) {
            int64_t at[4 * (MAXK + 3)];
            double d[4 * (MAXK + 3)];
            uint16_t alt[4 * (MAXK + 3)];
            double err = 0.0;
            int m = 0;
            for (int q = 0; q < kq; ++q)
                for (int j = 0; j < 4; ++j) {
                    const int64_t t = (((int64_t)k * kq + q) * n + i) * 4 + j;
                    const uint16_t h = f32_to_f16_rne(in[t]);
                    out[t] = h;
                    const double r = f16_value(h) - (double)in[t];
                    err += r;
                    if (r != 0.0) {
                        alt[m] = f16_step(h, r < 0.0);
                        d[m] = f16_value(alt[m]) - f16_value(h);
                        at[m++] = t;
                    }
                }
            for (;;) {
                int best = -1;
                double best_err = std::fabs(err);
                for (int c = 0; c < m; ++c)
                    if (at[c] >= 0 && std::fabs(err + d[c]) < best_err) { best = c; best_err = std::fabs(err + d[c]); }
                if (best < 0) break;
                out[at[best]] = alt[best];
                err += d[best];
                at[best] = -1;
            }
        }
    };
    const int nt = (int)std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    const int64_t chunk = (n + nt - 1) / nt;
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t)
        if (t * chunk < n) pool.emplace_back(rows, t * chunk, std::min(n, (t + 1) * chunk));
    rows(0, std::min(n, chunk));
    for (auto &th : pool) th.join();
    return MLBM_OK;
}

extern "C" int mlbm_pack_stencils(int64_t n, int32_t K, int32_t storage, const int32_t *idx, const double *w,
                                  const uint8_t *bb, const uint8_t *kind, void *idx_packed, void *w_packed,
                                  uint16_t *flags) {
    return mlbm_pack_stencils_range(n, 0, n, K, storage, idx, w, bb, kind, idx_packed, w_packed, flags);
}

extern "C" int mlbm_mark_lagrange(int64_t n, const uint8_t *lagrange, uint16_t *flags) {
    using mlbm::fail;
    mlbm::clear_error();
    if (n < 0 || (n > 0 && (!lagrange || !flags))) return fail(MLBM_ERR_ARG, "null pointer or negative n");
    for (int64_t i = 0; i < n; ++i)
        if (lagrange[i]) flags[i] = (uint16_t)(flags[i] | MLBM_FLAG_LAGRANGE);
    return MLBM_OK;
}

// ---- tile-local stencil indices (LDS staging) --------------------------------
//
// A tile is `tile` consecutive nodes (one workgroup).  Its halo is the sorted
// set of distinct nodes its stencils reference (the tile's own nodes
// included); each stencil member is re-addressed as a 16-bit position in that
// halo, so a workgroup can stage the halo state in LDS once and gather from it.

namespace {

int tile_halo(const int32_t *idx, int64_t n, int K, int64_t tile, int64_t t, std::vector<int32_t> &h) {
    const int64_t a = t * tile, b = std::min(n, a + tile);
    h.assign(idx + a * K, idx + b * K);
    std::sort(h.begin(), h.end());
    h.erase(std::unique(h.begin(), h.end()), h.end());
    return (int)h.size();
}

}  // namespace

extern "C" int mlbm_tile_sizes(int64_t n, int32_t K, int32_t tile, const int32_t *idx, int64_t *total_halo,
                               int32_t *max_halo) {
    using mlbm::fail;
    mlbm::clear_error();
    if (!idx || !total_halo || !max_halo) return fail(MLBM_ERR_ARG, "null pointer argument");
    if (n < 1 || K < 1 || K > 8 * MAXK) return fail(MLBM_ERR_ARG, "bad n or K");
    if (tile != 64 && tile != 128 && tile != 256) return fail(MLBM_ERR_ARG, "tile must be 64, 128 or 256");
    const int64_t nt = (n + tile - 1) / tile;
    int64_t tot = 0;
    int32_t mx = 0;
    std::vector<int32_t> h;
    for (int64_t t = 0; t < nt; ++t) {
        const int c = tile_halo(idx, n, K, tile, t, h);
        tot += c;
        mx = std::max(mx, c);
    }
    *total_halo = tot;
    *max_halo = mx;
    return MLBM_OK;
}

extern "C" int mlbm_pack_tiles(int64_t n, int32_t K, int32_t tile, const int32_t *idx, int32_t *halo_off,
                               int32_t *halo, uint16_t *lidx) {
    using mlbm::fail;
    mlbm::clear_error();
    if (!idx || !halo_off || !halo || !lidx) return fail(MLBM_ERR_ARG, "null pointer argument");
    if (n < 1 || K < 1 || K > 8 * MAXK) return fail(MLBM_ERR_ARG, "bad n or K");
    if (tile != 64 && tile != 128 && tile != 256) return fail(MLBM_ERR_ARG, "tile must be 64, 128 or 256");
    const int64_t nt = (n + tile - 1) / tile;
    const int k8 = (K + 7) / 8 * 8;
    std::vector<int32_t> h;
    int64_t off = 0;
    for (int64_t t = 0; t < nt; ++t) {
        const int c = tile_halo(idx, n, K, tile, t, h);
        if (off > INT32_MAX - c) return fail(MLBM_ERR_ARG, "halo lists exceed 2^31 entries");
        halo_off[t] = (int32_t)off;
        std::copy(h.begin(), h.end(), halo + off);
        const int64_t a = t * tile, b = std::min(n, a + tile);
        for (int64_t i = a; i < b; ++i) {
            for (int j = 0; j < k8; ++j) {
                int32_t g = j < K ? idx[i * K + j] : (int32_t)i;
                const int32_t pos = (int32_t)(std::lower_bound(h.begin(), h.end(), g) - h.begin());
                lidx[((int64_t)(j / 8) * n + i) * 8 + (j % 8)] = (uint16_t)pos;
            }
        }
        off += c;
    }
    halo_off[nt] = (int32_t)off;
    return MLBM_OK;
}
