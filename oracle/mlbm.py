"""Meshless LBM (MLBM) and meshless LBM1 (MLBM1) on scattered nodes.

Population MLBM (Sec. 2.2): every step first collides at all Eulerian nodes
(Sec. 2.1, Eq. 3), then streams: the population f_k arriving at x is the
post-collision f_k at the departure point x + dx_k' = x - dx e_k,
approximated by the weighted sum over the stencil (Sec. 2.2, Eq. 12).  The
rest population f_0 is not interpolated.

MLBM1 (Sec. 2.2, Eqs. 14-15): only rho and u are stored; they are
interpolated to the eight departure points, the equilibria (plus half the
force term) are evaluated there and summed into the new fields.

No-slip surfaces (Sec. 3.1 and 3.2): when the departure point of population
k lies inside a solid, the population is taken instead as the post-collision
f_k' at the mirrored point x + dx e_k (the simplified interpolated bounce-back
of Sec. 3.2, used here for every no-slip surface); if that point is inside a
solid too (a throat narrower than dx), the simple bounce-back value f_k' at
the node itself is used.

Straight Dirichlet boundaries (Sec. 3.1): after collision, every population
of a Dirichlet node is overwritten by the equilibrium of the prescribed
density and velocity.

Stencils: one stencil of the K nearest nodes per Eulerian node, shared by its
eight departure points, with separate weights per departure point; or, as in
the paper (Sec. 2.2), one stencil per departure point: the K nearest Eulerian
nodes of that point.  No-slip: the mirrored departure point described above,
or the simple bounce-back f_k = f_k'^post at the node itself, which the paper
uses on its cylinder (Sec. 3.1).  In a
hybrid node set (Sec. 2.2) a fluid node whose nine nearest nodes form a square
block of the lattice spacing h, and none of whose departure points needs the
bounce-back rule, uses the block (nine members) with biquadratic Lagrange
weights instead (oracle.lagrange).
"""
import dataclasses

import numpy as np

from . import lattice as lt
from .lagrange import biquadratic_weights, lattice_block
from .rbf import interpolation_weights, min_image, nearest, nearest_to_point

FLUID, WALL, DIRICHLET = 0, 1, 2


@dataclasses.dataclass
class Stencils:
    idx: np.ndarray     # (n, K) stencil node indices, or (n, 8, K) one stencil per departure point
    w: np.ndarray       # (n, 8, K) weights for k = 1..8
    src: np.ndarray     # (n, 8) source population of each arriving k (k or k')
    point: np.ndarray   # (n, 8, 2) departure point offsets from the node
    area: np.ndarray    # (n,) quadrature weight of each node
    lagrange: np.ndarray = None  # (n,) True where the biquadratic Lagrange block is used


def inside_solid(p, ns, eps=1e-12):
    """True if the point p lies strictly inside a solid: beyond a straight
    no-slip wall or inside an obstacle disk (periodic images included)."""
    box = ns.hi - ns.lo
    tol = eps * float(np.max(box))
    if ns.walls_y[0] and p[1] < ns.lo[1] - tol:
        return True
    if ns.walls_y[1] and p[1] > ns.hi[1] + tol:
        return True
    if len(ns.disks):
        d = min_image(p[None, :] - ns.disks[:, :2], box, ns.periodic)
        r = ns.disks[:, 2] - tol
        return bool(np.any(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] < r * r))
    return False


def departure(ns, i, k, dx, simple_bb=False):
    """Departure point (offset from x_i) and source population of the
    population k arriving at node i (Sec. 2.2, Eq. 12; Sec. 3.2, Eq. 22;
    simple_bb: the node itself, Sec. 3.1)."""
    x = ns.xy[i]
    e = lt.E[k]
    p = x - dx * e
    if not inside_solid(p, ns):
        return -dx * e, k
    q = x + dx * e
    if not simple_bb and not inside_solid(q, ns):
        return dx * e, int(lt.OPP[k])
    return np.zeros(2), int(lt.OPP[k])


def members(st, k):
    """Stencil indices (n, K) used for the arriving population k (1..8)."""
    return st.idx if st.idx.ndim == 2 else st.idx[:, k - 1, :]


def node_area(ns, i, m=4):
    """Unnormalised quadrature weight of node i: the square of the mean distance
    to its m nearest other nodes (h^2 on a regular lattice), halved for nodes
    on a boundary (no-slip surface or Dirichlet), half of whose neighbourhood
    lies outside the fluid."""
    _, off = nearest(ns.xy, i, m + 1, ns.hi - ns.lo, ns.periodic)
    a = float(np.mean(np.hypot(off[1:, 0], off[1:, 1]))) ** 2
    return 0.5 * a if ns.kind[i] != FLUID else a


def stencil_at(ns, i, K, dx, lattice_h=None, per_departure=False, simple_bb=False):
    """Stencil indices (K,) (per_departure: (8, K)), weights (8, K), sources
    (8,), departure offsets (8, 2) of node i, and whether the Lagrange block
    was used (lattice_h: the spacing of the regular part of a hybrid set, None
    for RBF-FD everywhere)."""
    src = np.zeros(8, dtype=np.int64)
    pts = np.zeros((8, 2))
    for k in range(1, 9):
        pts[k - 1], src[k - 1] = departure(ns, i, k, dx, simple_bb)
    if lattice_h is not None and ns.kind[i] == FLUID and dx <= lattice_h and np.all(src == np.arange(1, 9)):
        block = lattice_block(ns, i, lattice_h)
        if block is not None:
            # members: the eight lattice neighbours, then the node itself
            order = [1, 2, 3, 4, 5, 6, 7, 8, 0]
            idx = np.full(K, i, dtype=np.int64)
            idx[:9] = block[order]
            w = np.zeros((8, K))
            w[:, :9] = biquadratic_weights(pts, lattice_h)[:, order]
            if per_departure:
                idx = np.tile(idx, (8, 1))
            return idx, w, src, pts, True
    if per_departure:
        # the K nearest nodes of each departure point, weights at that point
        idx = np.zeros((8, K), dtype=np.int64)
        w = np.zeros((8, K))
        for k in range(8):
            idx[k], X = nearest_to_point(ns.xy, i, pts[k], K, ns.hi - ns.lo, ns.periodic)
            w[k] = interpolation_weights(X, np.zeros((1, 2)))[0]
        return idx, w, src, pts, False
    idx, X = nearest(ns.xy, i, K, ns.hi - ns.lo, ns.periodic)
    w = interpolation_weights(X, pts)
    return idx, w, src, pts, False


def build_stencils(ns, K, dx, lattice_h=None, per_departure=False, simple_bb=False):
    """Stencils of every node, plus quadrature weights normalised so that they
    sum to the analytic fluid area."""
    n = ns.n
    if lattice_h is not None and K < 10:
        raise ValueError("hybrid stencils need K >= 10")
    idx = np.zeros((n, 8, K) if per_departure else (n, K), dtype=np.int64)
    w = np.zeros((n, 8, K))
    src = np.zeros((n, 8), dtype=np.int64)
    pts = np.zeros((n, 8, 2))
    area = np.zeros(n)
    lag = np.zeros(n, dtype=bool)
    for i in range(n):
        idx[i], w[i], src[i], pts[i], lag[i] = stencil_at(ns, i, K, dx, lattice_h, per_departure, simple_bb)
        area[i] = node_area(ns, i)
    area *= ns.fluid_area() / area.sum()
    return Stencils(idx=idx, w=w, src=src, point=pts, area=area, lagrange=lag)


# --------------------------------------------------------------------------
# Population MLBM
# --------------------------------------------------------------------------

def dirichlet_overwrite(fpost, ns):
    """Overwrite all populations of Dirichlet nodes with the equilibrium of the
    prescribed density and velocity (Sec. 3.1).  Pinned by plane Couette flow
    between two Dirichlet lines (exact on the lattice at s = 1, tau = 1) and
    by the convergence of flows between such lines to their closed forms."""
    d = ns.kind == DIRICHLET
    if np.any(d):
        bc = ns.boundary_values()
        fpost[:, d] = lt.equilibrium(bc[d, 0], bc[d, 1:3])
    return fpost


def post_collision(f, ns, tau_plus, tau_minus, g):
    """Collision at every node followed by the Dirichlet overwrite."""
    return dirichlet_overwrite(lt.collide(f, tau_plus, tau_minus, g), ns)


def stream(fpost, st):
    """Semi-Lagrangian streaming (Sec. 2.2, Eq. 12): f_0 stays, every other
    population is the weighted sum of the source population over the stencil."""
    n = fpost.shape[1]
    fnew = np.empty_like(fpost)
    fnew[0] = fpost[0]
    rows = np.arange(n)[:, None]
    for k in range(1, 9):
        s = st.src[:, k - 1][:, None] + 0 * rows
        vals = fpost[s, members(st, k)]
        fnew[k] = np.sum(st.w[:, k - 1, :] * vals, axis=1)
    return fnew


def step(f, ns, st, tau_plus, tau_minus, g=(0.0, 0.0)):
    """One MLBM time step on pre-collision populations f (9, n): collide all,
    then stream all (Sec. 2.1 order of operations, Sec. 2.2 streaming)."""
    return stream(post_collision(f, ns, tau_plus, tau_minus, g), st)


def init_populations(rho, u):
    """Initial populations: the equilibrium of the initial fields (Sec. 3.1)."""
    return lt.equilibrium(rho, u)


def macroscopic(f, ns, g=(0.0, 0.0)):
    """Density and velocity (with the half-force shift) of pre-collision
    populations; Dirichlet nodes report their prescribed values."""
    rho = lt.density(f)
    u = lt.velocity(f, g)
    d = ns.kind == DIRICHLET
    if np.any(d):
        bc = ns.boundary_values()
        rho = rho.copy()
        u = u.copy()
        rho[d] = bc[d, 0]
        u[d] = bc[d, 1:3]
    return rho, u


def bounce_back_force(f, ns, st, tau_plus, tau_minus, g, dx, area=None):
    """Momentum-exchange force on all no-slip surfaces during one step: for
    each bounced pair (node i, arriving k) the population k' that leaves i
    towards the solid is lost to the fluid and the population k that arrives
    instead is gained, so the solid receives e_k' (f_k'^post + f_k^new); each
    node counts with A_i / dx^2 lattice cells (area defaults to the stencil
    quadrature weights).  Populations are taken relative to the rest state
    (f - omega): a uniform pressure exerts no net force on a closed surface,
    but its discretised surface sum on scattered nodes does not vanish, so
    the reference pressure is removed before summing.  The paper reports no
    forces on scattered nodes; the formula is pinned by the steady momentum
    balance of a channel."""
    area = st.area if area is None else area
    fpost = post_collision(f, ns, tau_plus, tau_minus, g)
    fnew = stream(fpost, st)
    F = np.zeros(2)
    for i in range(ns.n):
        for k in range(1, 9):
            kp = int(lt.OPP[k])
            if st.src[i, k - 1] == kp:
                F += (area[i] / dx ** 2) * lt.E[kp] * ((fpost[kp, i] - lt.W[kp]) + (fnew[k, i] - lt.W[k]))
    return F


# --------------------------------------------------------------------------
# MLBM1 (tau = 1, fields only)
# --------------------------------------------------------------------------

def mlbm1_step(rho, u, ns, st, g=(0.0, 0.0)):
    """One MLBM1 step (Sec. 2.2, Eqs. 14-15).  For k >= 1 the fields are
    interpolated to the departure point, the (bounce-back aware) source
    population's equilibrium plus half its force term is evaluated there; the
    rest population uses the node's own fields; the new density is their sum
    and the new velocity their first moment plus half the force, over the new
    density.  Dirichlet nodes keep their prescribed fields."""
    n = ns.n
    g = np.asarray(g, dtype=np.float64)
    fhat = np.empty((9, n))
    cols = np.arange(n)
    own = lt.equilibrium(rho, u) + 0.5 * lt.guo_force(rho, u, g)
    fhat[0] = own[0]
    for k in range(1, 9):
        wk = st.w[:, k - 1, :]
        mk = members(st, k)
        rho_h = np.sum(wk * rho[mk], axis=1)
        u_h = np.stack([np.sum(wk * u[mk, 0], axis=1),
                        np.sum(wk * u[mk, 1], axis=1)], axis=1)
        at_p = lt.equilibrium(rho_h, u_h) + 0.5 * lt.guo_force(rho_h, u_h, g)
        fhat[k] = at_p[st.src[:, k - 1], cols]
    rho_new = lt.density(fhat)
    u_new = (lt.momentum(fhat) + 0.5 * rho_new[:, None] * g[None, :]) / rho_new[:, None]
    d = ns.kind == DIRICHLET
    if np.any(d):
        bc = ns.boundary_values()
        rho_new[d] = bc[d, 0]
        u_new[d] = bc[d, 1:3]
    return rho_new, u_new


def mlbm1_bounce_back_force(rho, u, ns, st, g, dx, area=None):
    """Momentum-exchange force of MLBM1 (same bookkeeping as
    bounce_back_force): the post-collision population k' at the node is its
    equilibrium plus half the force term (tau = 1), the returning population
    k the same at the interpolated fields of the mirrored point; both
    relative to the rest state.  Pinned, like bounce_back_force, by the
    one-step momentum budget of a periodic sample with disks."""
    area = st.area if area is None else area
    g = np.asarray(g, dtype=np.float64)
    own = lt.equilibrium(rho, u) + 0.5 * lt.guo_force(rho, u, g)
    F = np.zeros(2)
    for i in range(ns.n):
        for k in range(1, 9):
            kp = int(lt.OPP[k])
            if st.src[i, k - 1] != kp:
                continue
            w = st.w[i, k - 1]
            nb = members(st, k)[i]
            rh = np.array([np.sum(w * rho[nb])])
            uh = np.array([[np.sum(w * u[nb, 0]), np.sum(w * u[nb, 1])]])
            back = lt.equilibrium(rh, uh) + 0.5 * lt.guo_force(rh, uh, g)
            F += (area[i] / dx ** 2) * lt.E[kp] * ((own[kp, i] - lt.W[kp]) + (back[kp, 0] - lt.W[k]))
    return F


# --------------------------------------------------------------------------
# Reductions (Sec. 3.2, Eqs. 23-25) and the steady-state residual
# --------------------------------------------------------------------------

def reductions(rho, u, area, u_prev=None):
    """FP64 sums over nodes with quadrature weights A_i: mass sum A rho, the
    velocity integral sum A u, the speed integral sum A |u|, and the relative
    change ||u - u_prev|| / ||u|| (node-wise 2-norms)."""
    speed = np.hypot(u[:, 0], u[:, 1])
    out = {
        "mass": float(np.sum(area * rho)),
        "int_ux": float(np.sum(area * u[:, 0])),
        "int_uy": float(np.sum(area * u[:, 1])),
        "int_speed": float(np.sum(area * speed)),
        "norm_u": float(np.sqrt(np.sum(u * u))),
    }
    if u_prev is not None:
        du = u - u_prev
        out["norm_du"] = float(np.sqrt(np.sum(du * du)))
        out["residual"] = out["norm_du"] / out["norm_u"] if out["norm_u"] > 0 else 0.0
    return out


def mean_velocity(red, fluid_area):
    """<u> = (1/phi) int_D u dOmega (Sec. 3.2, Eq. 23): the velocity integral
    over the fluid area."""
    return red["int_ux"] / fluid_area


def tortuosity(red):
    """T_V = <|u|> / <u> (Sec. 3.2, Eq. 25)."""
    return red["int_speed"] / red["int_ux"]


def permeability(red, box_area, nu_lb, g_lb, dx):
    """Darcy permeability k = nu U_s / g with the superficial velocity
    U_s = int_D u dOmega / |D|, converted from lattice units (dx = 1) to the
    node coordinates' units.  Pinned by a plane channel, whose permeability
    is H^2 / 12 (the paper reports none on scattered nodes)."""
    U_s = red["int_ux"] / box_area
    return nu_lb * U_s / g_lb * dx * dx
