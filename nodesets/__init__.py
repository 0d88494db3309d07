"""Seeded, synthetic node sets and geometries for the meshless LBM workloads.

This module is the only code shared by the CPU oracle and the GPU library
tests: it produces *inputs* (node coordinates, node kinds, obstacle lists,
boundary values, smooth initial fields and noise), and it holds none of the
method's arithmetic (no equilibria, no collision, no interpolation weights).

The paper's own point clouds (the hybrid Karman set of Sec. 3.1 and the
porous sample of Sec. 3.2) were never published, so every workload here is a
synthetic stand-in with the same structure: scattered nodes, local refinement
near obstacles, boundary nodes placed exactly on no-slip surfaces (Sec. 3.2),
periodic boxes, and straight Dirichlet boundaries (Sec. 3.1).

Node kinds: 0 = fluid, 1 = node lying on a no-slip surface, 2 = Dirichlet
node whose populations are overwritten by an equilibrium (Sec. 3.1).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FLUID, WALL, DIRICHLET = 0, 1, 2


@dataclasses.dataclass
class NodeSet:
    """A scattered node set with its geometry description (all float64)."""

    xy: np.ndarray            # (n, 2) node coordinates
    kind: np.ndarray          # (n,) uint8 node kind
    lo: np.ndarray            # (2,) box lower corner
    hi: np.ndarray            # (2,) box upper corner
    periodic: tuple           # (bool, bool) periodic along x / y
    walls_y: tuple = (False, False)   # no-slip straight walls at y=lo[1] / y=hi[1]
    disks: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))
    bc: np.ndarray | None = None      # (n, 3) (rho_b, ux_b, uy_b), used on kind-2 nodes
    h: float = 0.0            # reference (bulk) node spacing
    name: str = ""
    h_min: float = 0.0        # finest node spacing (refined regions); 0 means h

    @property
    def n(self) -> int:
        return int(self.xy.shape[0])

    def fluid_area(self) -> float:
        """Analytic area of the fluid region: box minus the obstacle disks."""
        box = float(np.prod(self.hi - self.lo))
        return box - float(np.sum(np.pi * self.disks[:, 2] ** 2)) if len(self.disks) else box

    def boundary_values(self) -> np.ndarray:
        if self.bc is None:
            bc = np.zeros((self.n, 3))
            bc[:, 0] = 1.0
            return bc
        return self.bc


def _grid(lo, hi, h, cell_centred=True):
    """Points of a square grid of spacing h covering [lo, hi)."""
    nx = max(1, int(round((hi[0] - lo[0]) / h)))
    ny = max(1, int(round((hi[1] - lo[1]) / h)))
    off = 0.5 if cell_centred else 0.0
    gx = lo[0] + (np.arange(nx) + off) * (hi[0] - lo[0]) / nx
    gy = lo[1] + (np.arange(ny) + off) * (hi[1] - lo[1]) / ny
    X, Y = np.meshgrid(gx, gy, indexing="xy")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def _wrap(xy, lo, hi, periodic):
    out = xy.copy()
    for d in range(2):
        if periodic[d]:
            L = hi[d] - lo[d]
            out[:, d] = lo[d] + np.mod(out[:, d] - lo[d], L)
    return out


def _in_box(xy, L):
    """Map coordinates into [0, L) for periodic KD-tree queries."""
    out = np.mod(xy, L)
    out[out >= L] = 0.0
    return out


def _min_image(d, L, periodic):
    d = d.copy()
    for a in range(2):
        if periodic[a]:
            d[..., a] -= L[a] * np.round(d[..., a] / L[a])
    return d


# --------------------------------------------------------------------------
# Regular and jittered periodic grids
# --------------------------------------------------------------------------

def regular_grid(n: int, L: float = 1.0) -> NodeSet:
    """Cell-centred n x n grid on the periodic box [0, L)^2, ordered row-major
    (node id = iy * n + ix).  With the streaming distance equal to the spacing
    this is the standard lattice of Sec. 2.1."""
    lo, hi = np.zeros(2), np.full(2, L)
    xy = _grid(lo, hi, L / n)
    return NodeSet(xy=xy, kind=np.zeros(len(xy), np.uint8), lo=lo, hi=hi,
                   periodic=(True, True), h=L / n, name=f"regular{n}")


def jittered_grid(n: int, jitter: float = 0.3, seed: int = 231214789, L: float = 1.0) -> NodeSet:
    """Cell-centred n x n grid on the periodic box [0, L)^2 with every coordinate
    moved by an independent uniform offset in [-jitter*h, jitter*h], then
    wrapped into the box."""
    ns = regular_grid(n, L)
    rng = np.random.default_rng(seed)
    h = L / n
    xy = ns.xy + rng.uniform(-jitter * h, jitter * h, size=ns.xy.shape)
    ns.xy = _wrap(xy, ns.lo, ns.hi, ns.periodic)
    ns.name = f"jittered{n}"
    return ns


def patch_jittered_grid(n: int, radius: float, centre=(0.5, 0.5), jitter: float = 0.3,
                        seed: int = 231214789, L: float = 1.0) -> NodeSet:
    """Hybrid periodic set: the cell-centred n x n grid with only the nodes
    within `radius` (minimum image) of `centre` jittered as in jittered_grid;
    the rest stay on the lattice."""
    ns = regular_grid(n, L)
    rng = np.random.default_rng(seed)
    h = L / n
    d = _min_image(ns.xy - np.asarray(centre, dtype=np.float64), ns.hi - ns.lo, ns.periodic)
    sel = np.hypot(d[:, 0], d[:, 1]) < radius
    off = rng.uniform(-jitter * h, jitter * h, size=ns.xy.shape)
    xy = ns.xy + np.where(sel[:, None], off, 0.0)
    ns.xy = _wrap(xy, ns.lo, ns.hi, ns.periodic)
    ns.name = f"patch{n}"
    return ns


def channel(nx: int, ny: int, jitter: float = 0.0, seed: int = 231214789,
            Lx: float = 1.0, H: float = 1.0) -> NodeSet:
    """Plane channel [0, Lx) x [0, H], periodic along x, no-slip walls at y=0
    and y=H with nodes placed exactly on the walls (the arrangement of
    Sec. 3.2).  Interior rows sit at y = j*H/(ny-1), j = 1..ny-2; interior
    nodes are optionally jittered."""
    lo, hi = np.zeros(2), np.array([Lx, H])
    hx = Lx / nx
    gx = (np.arange(nx) + 0.5) * hx
    gy = np.arange(ny) * H / (ny - 1)
    X, Y = np.meshgrid(gx, gy, indexing="xy")
    xy = np.stack([X.ravel(), Y.ravel()], axis=1)
    kind = np.zeros(len(xy), np.uint8)
    on_wall = (np.isclose(xy[:, 1], 0.0)) | (np.isclose(xy[:, 1], H))
    kind[on_wall] = WALL
    if jitter > 0:
        rng = np.random.default_rng(seed)
        hy = H / (ny - 1)
        dj = rng.uniform(-jitter, jitter, size=xy.shape) * np.array([hx, hy])
        dj[on_wall, 1] = 0.0
        xy = xy + dj
        xy = _wrap(xy, lo, hi, (True, False))
    return NodeSet(xy=xy, kind=kind, lo=lo, hi=hi, periodic=(True, False),
                   walls_y=(True, True), h=H / (ny - 1), name=f"channel{nx}x{ny}")


def dirichlet_channel(nx: int, ny: int, u_top: float = 0.0, jitter: float = 0.0,
                      seed: int = 231214789, H: float = 1.0) -> NodeSet:
    """The plane channel of `channel` (square cells: Lx = nx H / (ny - 1)),
    but its bottom and top rows are Dirichlet lines instead of no-slip walls
    (the straight-boundary arrangement of Sec. 3.1): prescribed rho = 1 and
    velocity (0, 0) at y = 0 and (u_top, 0) at y = H.  No solid lies beyond
    the lines, so departure points below y = 0 or above y = H stay where
    they are."""
    ns = channel(nx, ny, jitter=jitter, seed=seed, Lx=nx * H / (ny - 1), H=H)
    top = np.isclose(ns.xy[:, 1], H)
    bottom = np.isclose(ns.xy[:, 1], 0.0)
    kind = np.zeros(ns.n, np.uint8)
    kind[top | bottom] = DIRICHLET
    bc = np.zeros((ns.n, 3))
    bc[:, 0] = 1.0
    bc[top, 1] = u_top
    return NodeSet(xy=ns.xy, kind=kind, lo=ns.lo, hi=ns.hi, periodic=(True, False),
                   walls_y=(False, False), bc=bc, h=ns.h, name=f"dirichlet_channel{nx}x{ny}")


# --------------------------------------------------------------------------
# Scattered node sets with refinement and obstacles
# --------------------------------------------------------------------------

def _cleanup(xy, hloc, fixed, lo, hi, periodic, frac=0.45):
    """Remove non-fixed nodes that sit closer than frac*max(h_i, h_j) to another
    node (a blue-noise clean-up of the seams between jittered patches).
    Among a conflicting pair the non-fixed node with the larger index goes."""
    from scipy.spatial import cKDTree

    L = hi - lo
    box = [L[0] if periodic[0] else 0, L[1] if periodic[1] else 0]
    keep = np.ones(len(xy), bool)
    for _ in range(4):
        pts = xy[keep]
        ids = np.nonzero(keep)[0]
        if any(box):
            # cKDTree supports periodic boxes only with all positive sizes.
            bs = np.array([b if b else 1e30 for b in box])
            q = pts - lo
            for a in range(2):
                if box[a]:
                    q[:, a] = _in_box(q[:, a], box[a])
            tree = cKDTree(q, boxsize=bs)
            pairs = tree.query_pairs(r=frac * hloc.max(), output_type="ndarray")
            dvec = _min_image(pts[pairs[:, 0]] - pts[pairs[:, 1]], L, periodic)
        else:
            tree = cKDTree(pts)
            pairs = tree.query_pairs(r=frac * hloc.max(), output_type="ndarray")
            dvec = pts[pairs[:, 0]] - pts[pairs[:, 1]]
        if len(pairs) == 0:
            break
        a, b = ids[pairs[:, 0]], ids[pairs[:, 1]]
        dist = np.hypot(dvec[:, 0], dvec[:, 1])
        bad = dist < frac * np.maximum(hloc[a], hloc[b])
        a, b = a[bad], b[bad]
        if len(a) == 0:
            break
        drop = np.where(fixed[b], a, np.where(fixed[a], b, np.maximum(a, b)))
        drop = drop[~fixed[drop]]
        if len(drop) == 0:
            break
        keep[drop] = False
    return keep


def _circle_nodes(cx, cy, r, h):
    m = max(8, int(round(2 * np.pi * r / h)))
    t = 2 * np.pi * np.arange(m) / m
    return np.stack([cx + r * np.cos(t), cy + r * np.sin(t)], axis=1)


def karman(n_target: int = 500_000, seed: int = 231214789, D: float = 1.0,
           u_max: float = 0.05, jitter: float | None = None, hybrid: bool = False,
           wake: float = 6.0, poisson: bool = False) -> NodeSet:
    """Channel 22D x 4.1D with a cylinder of diameter D centred at (2D, 2D).

    Scattered nodes: stratified samples (jittered by jitter h, default 0.35;
    0.2 in the hybrid zone) at spacing h_b in the bulk
    and h_f = h_b / 2 (4x the node density) within 1D of the cylinder surface,
    cleaned of close pairs; nodes exactly on the cylinder surface (spacing h_f,
    no-slip); Dirichlet nodes on the four straight boundaries (spacing h_b):
    parabolic inflow/outflow profile with maximum u_max on x=0 and x=22D,
    zero velocity on y=0 and y=4.1D, unit density (the boundary treatment of
    Sec. 3.1).  h_b is chosen so that the set holds about n_target nodes.

    hybrid: the arrangement of Sec. 3.1 (scattered near the cylinder and in
    its wake, a square lattice elsewhere): bulk nodes are jittered only within
    2D of the cylinder centre and in the wake box [2D, 2D + wake D] x
    [0.5D, 3.5D]; elsewhere they stay on the lattice of spacing h_b, which is
    then D/(10 m) for an integer m so that it divides both channel sides.

    poisson: Poisson-disk nodes instead of the stratified samples: advancing
    fronts grown from the cylinder surface, spacing h_f within 1D of the
    cylinder surface rising linearly to h_b over the next 4 h_f; over the whole
    channel (h_b sized so that the set holds about n_target nodes), or with
    hybrid over the scattered zone only, up to the fixed lattice."""
    if poisson:
        return _karman_poisson(n_target, seed, D, u_max, hybrid, wake)
    if jitter is None:
        # the hybrid zone's jitter: 0.35 h_b diverges at s = 4 on the seam with
        # the lattice, 0.2 h_b does not
        jitter = 0.2 if hybrid else 0.35
    rng = np.random.default_rng(seed)
    Lx, Ly = 22.0 * D, 4.1 * D
    cx, cy, r = 2.0 * D, 2.0 * D, 0.5 * D
    ring = 1.0 * D
    a_fine = np.pi * ((r + ring) ** 2 - r ** 2)
    a_bulk = Lx * Ly - np.pi * (r + ring) ** 2
    hb = math.sqrt((a_bulk + 4.0 * a_fine) / n_target)
    if hybrid:
        hb = 0.1 * D / max(1, round(0.1 * D / hb))
    hf = 0.5 * hb
    lo, hi = np.zeros(2), np.array([Lx, Ly])

    # Bulk: jittered grid away from the boundaries.  The hybrid set's lattice
    # sits on the vertices i h_b, j h_b, so that it continues into the
    # Dirichlet nodes of the sides (a cell-centred lattice leaves a
    # half-spacing layer of irregular stencils along every side)
    if hybrid:
        gx = np.arange(1, int(round(Lx / hb))) * hb
        gy = np.arange(1, int(round(Ly / hb))) * hb
        GX, GY = np.meshgrid(gx, gy, indexing="xy")
        bulk = np.stack([GX.ravel(), GY.ravel()], axis=1)
    else:
        bulk = _grid(lo, hi, hb)
    off = rng.uniform(-jitter * hb, jitter * hb, size=bulk.shape)
    if hybrid:
        near = np.hypot(bulk[:, 0] - cx, bulk[:, 1] - cy) < 2.0 * D
        in_wake = (bulk[:, 0] >= cx) & (bulk[:, 0] <= cx + wake * D) & (np.abs(bulk[:, 1] - cy) <= 1.5 * D)
        off[~(near | in_wake)] = 0.0
    bulk = bulk + off
    rb = np.hypot(bulk[:, 0] - cx, bulk[:, 1] - cy)
    inside = (bulk[:, 0] > 0.5 * hb) & (bulk[:, 0] < Lx - 0.5 * hb) & \
             (bulk[:, 1] > 0.5 * hb) & (bulk[:, 1] < Ly - 0.5 * hb)
    bulk = bulk[inside & (rb > r + ring)]
    # Fine ring around the cylinder.
    flo = np.array([cx - r - ring, cy - r - ring])
    fhi = np.array([cx + r + ring, cy + r + ring])
    fine = _grid(flo, fhi, hf)
    fine = fine + rng.uniform(-jitter * hf, jitter * hf, size=fine.shape)
    rf = np.hypot(fine[:, 0] - cx, fine[:, 1] - cy)
    fine = fine[(rf > r + 0.5 * hf) & (rf <= r + ring)]
    # Surface nodes.
    surf = _circle_nodes(cx, cy, r, hf)
    # Straight-boundary Dirichlet nodes (corners once).
    nbx = int(round(Lx / hb))
    nby = int(round(Ly / hb))
    xs = np.linspace(0.0, Lx, nbx + 1)
    ys = np.linspace(0.0, Ly, nby + 1)[1:-1]
    bnd = np.concatenate([
        np.stack([xs, np.zeros_like(xs)], 1), np.stack([xs, np.full_like(xs, Ly)], 1),
        np.stack([np.zeros_like(ys), ys], 1), np.stack([np.full_like(ys, Lx), ys], 1)])

    xy = np.concatenate([bulk, fine, surf, bnd])
    kind = np.concatenate([np.zeros(len(bulk) + len(fine), np.uint8),
                           np.full(len(surf), WALL, np.uint8),
                           np.full(len(bnd), DIRICHLET, np.uint8)])
    hloc = np.concatenate([np.full(len(bulk), hb), np.full(len(fine), hf),
                           np.full(len(surf), hf), np.full(len(bnd), hb)])
    keep = _cleanup(xy, hloc, kind != FLUID, lo, hi, (False, False))
    xy, kind = xy[keep], kind[keep]
    bc = np.zeros((len(xy), 3))
    bc[:, 0] = 1.0
    d = kind == DIRICHLET
    inout = d & ((np.isclose(xy[:, 0], 0.0)) | (np.isclose(xy[:, 0], Lx)))
    y = xy[:, 1]
    bc[inout, 1] = 4.0 * u_max * y[inout] * (Ly - y[inout]) / Ly ** 2
    return NodeSet(xy=xy, kind=kind, lo=lo, hi=hi, periodic=(False, False),
                   disks=np.array([[cx, cy, r]]), bc=bc, h=hb, name="karman-hybrid" if hybrid else "karman",
                   h_min=hf)


# number of nodes per unit area of an advancing-front Poisson-disk fill of
# spacing h, times h^2 (measured on open regions with the defaults of _front_fill)
_FRONT_DENSITY = 0.89


def _karman_poisson(n_target, seed, D, u_max, hybrid=False, wake=6.0):
    rng = np.random.default_rng(seed)
    Lx, Ly = 22.0 * D, 4.1 * D
    cx, cy, r = 2.0 * D, 2.0 * D, 0.5 * D
    ring = 1.0 * D
    a_fine = np.pi * ((r + ring) ** 2 - r ** 2)
    a_bulk = Lx * Ly - np.pi * (r + ring) ** 2
    hb = math.sqrt(_FRONT_DENSITY * (a_bulk + 4.0 * a_fine) / n_target)
    if hybrid:
        hb = 0.1 * D / max(1, round(0.1 * D / hb))
    hf = 0.5 * hb
    lo, hi = np.zeros(2), np.array([Lx, Ly])

    def spacing(p):
        t = np.clip((np.hypot(p[:, 0] - cx, p[:, 1] - cy) - r - ring) / (4.0 * hf), 0.0, 1.0)
        return hf + (hb - hf) * t

    def in_zone(p, margin=0.0):
        # the scattered zone of the hybrid set: within 2D of the cylinder centre
        # and the wake box [2D, 2D + wake D] x [0.5D, 3.5D]
        near = np.hypot(p[:, 0] - cx, p[:, 1] - cy) < 2.0 * D + margin
        box = ((p[:, 0] >= cx - margin) & (p[:, 0] <= cx + wake * D + margin)
               & (np.abs(p[:, 1] - cy) <= 1.5 * D + margin))
        return near | box

    def admit(c):
        ok = ((c[:, 0] > 0.5 * hb) & (c[:, 0] < Lx - 0.5 * hb) & (c[:, 1] > 0.5 * hb) & (c[:, 1] < Ly - 0.5 * hb)
              & (np.hypot(c[:, 0] - cx, c[:, 1] - cy) > r + 0.5 * hf))
        return ok & in_zone(c, 0.5 * hb) if hybrid else ok

    surf = _circle_nodes(cx, cy, r, hf)
    nbx, nby = int(round(Lx / hb)), int(round(Ly / hb))
    xs = np.linspace(0.0, Lx, nbx + 1)
    ys = np.linspace(0.0, Ly, nby + 1)[1:-1]
    bnd = np.concatenate([
        np.stack([xs, np.zeros_like(xs)], 1), np.stack([xs, np.full_like(xs, Ly)], 1),
        np.stack([np.zeros_like(ys), ys], 1), np.stack([np.full_like(ys, Lx), ys], 1)])
    lat = np.zeros((0, 2))
    if hybrid:
        lat = _grid(lo, hi, hb)
        lat = lat[~in_zone(lat)]
    fluid = _front_fill(np.concatenate([bnd, lat]), surf, spacing, admit, rng, window=6)
    xy = np.concatenate([lat, fluid, surf, bnd])
    kind = np.concatenate([np.zeros(len(lat) + len(fluid), np.uint8), np.full(len(surf), WALL, np.uint8),
                           np.full(len(bnd), DIRICHLET, np.uint8)])
    hloc = np.concatenate([np.full(len(lat), hb), spacing(fluid), np.full(len(surf), hf), np.full(len(bnd), hb)])
    fixed = np.concatenate([np.ones(len(lat), bool), np.zeros(len(fluid), bool), np.ones(len(surf) + len(bnd), bool)])
    keep = _cleanup(xy, hloc, fixed, lo, hi, (False, False))
    xy, kind = xy[keep], kind[keep]
    bc = np.zeros((len(xy), 3))
    bc[:, 0] = 1.0
    inout = (kind == DIRICHLET) & ((np.isclose(xy[:, 0], 0.0)) | (np.isclose(xy[:, 0], Lx)))
    y = xy[:, 1]
    bc[inout, 1] = 4.0 * u_max * y[inout] * (Ly - y[inout]) / Ly ** 2
    return NodeSet(xy=xy, kind=kind, lo=lo, hi=hi, periodic=(False, False), disks=np.array([[cx, cy, r]]), bc=bc,
                   h=hb, name="karman-hybrid-poisson" if hybrid else "karman-poisson", h_min=hf)


def _front_fill(fixed: np.ndarray, seeds: np.ndarray, spacing, admit, rng, n_cand: int = 12,
                period_x: float = 0.0, window: int = 0) -> np.ndarray:
    """Poisson-disk node placement by advancing fronts (after Slak & Kosec,
    2019): every node of the current front proposes n_cand candidates on the
    circle of radius h(p) around itself (random rotation); a candidate is kept
    if admit() accepts it and no node, old or newly kept, lies closer than
    0.99 h(p).  The kept candidates form the next front.  Returns the new
    nodes only (fixed and seeds are taken as already placed).  period_x > 0:
    periodic along x on [0, period_x) (candidates wrapped, distances by
    minimum image).  window > 0: candidates are checked against the fixed
    nodes, the seeds and the nodes of the last `window` fronts only (for large
    sets; a front moves about one spacing per generation, so older nodes lie
    behind it; callers clean up the rare close pair this misses)."""
    from scipy.spatial import cKDTree

    def tree(pts):
        if period_x:
            return cKDTree(pts, boxsize=[period_x, 1e30])
        return cKDTree(pts)

    base_tree = tree(np.concatenate([fixed, seeds]))
    front = seeds
    out = []
    ang0 = 2.0 * np.pi * np.arange(n_cand) / n_cand
    while len(front):
        hp = spacing(front)
        rot = rng.uniform(0.0, 2.0 * np.pi, size=len(front))
        a = rot[:, None] + ang0[None, :]
        cand = (front[:, None, :] + hp[:, None, None] * np.stack([np.cos(a), np.sin(a)], -1)).reshape(-1, 2)
        if period_x:
            cand[:, 0] = np.mod(cand[:, 0], period_x)
            cand[cand[:, 0] >= period_x, 0] = 0.0
        hc = np.repeat(hp, n_cand)
        ok = admit(cand)
        cand, hc = cand[ok], hc[ok]
        if len(cand) == 0:
            break
        dist, _ = base_tree.query(cand)
        recent = out[-window:] if window else out
        if recent:
            dist = np.minimum(dist, tree(np.concatenate(recent)).query(cand)[0])
        ok = dist >= 0.99 * hc
        cand, hc = cand[ok], hc[ok]
        if len(cand) == 0:
            break
        # greedy among the candidates themselves, in proposal order
        nbrs = tree(cand).query_ball_point(cand, r=0.99 * hc)
        taken = np.zeros(len(cand), bool)
        for i in range(len(cand)):
            if not any(taken[j] for j in nbrs[i] if j != i):
                taken[i] = True
        front = cand[taken]
        out.append(front)
    return np.concatenate(out) if out else np.zeros((0, 2))


def karman_paper(h_min: float = 1.0 / 200, h_max: float = 1.0 / 25, grade: float = 0.3,
                 wake_stretch: float = 0.1, d: float = 0.14, u0: float = 1e-2,
                 seed: int = 231214789) -> NodeSet:
    """The cylinder channel of Sec. 3.1: a 3 x 1 channel with a cylinder of
    diameter d on the axis, 0.5 from the inlet; parabolic inflow/outflow with
    maximum u0 and zero velocity on the top and bottom, all four sides by
    equilibrium overwrite (Dirichlet nodes), the cylinder no-slip.  Hybrid
    nodes, symmetric about the channel axis (built in the upper half and
    mirrored): scattered around the cylinder and in its wake, their spacing
    growing from h_min on the cylinder surface to h_max at a distance `grade`
    (the wake distance counted wake_stretch times shorter), and a square
    lattice of spacing h_max elsewhere (aligned with the channel sides, which
    carry the Dirichlet nodes)."""
    rng = np.random.default_rng(seed)
    Lx, Ly = 3.0, 1.0
    cx, cy, R = 0.5, 0.5, 0.5 * d
    lo, hi = np.zeros(2), np.array([Lx, Ly])

    def reach(pts):
        dxw = pts[:, 0] - cx
        dxw = np.where(dxw > 0, dxw * wake_stretch, dxw)
        return np.hypot(dxw, pts[:, 1] - cy) - R

    def spacing(pts):
        return h_min + (h_max - h_min) * np.clip(reach(pts) / grade, 0.0, 1.0)

    # lattice at h_max (cell vertices, upper half including the axis row)
    nx, ny = int(round(Lx / h_max)), int(round(Ly / h_max))
    X, Y = np.meshgrid(np.arange(nx + 1) * (Lx / nx), np.arange(ny + 1) * (Ly / ny), indexing="xy")
    lat = np.stack([X.ravel(), Y.ravel()], axis=1)
    lat = lat[lat[:, 1] >= cy - 1e-12]
    edge = (lat[:, 0] == 0.0) | (lat[:, 0] == Lx) | (lat[:, 1] == Ly)
    bnd = lat[edge]
    lat = lat[~edge]
    lat = lat[reach(lat) > grade]
    # the cylinder surface (upper half) and the axis, each at the local spacing
    m = int(np.ceil(np.pi * d / h_min / 2.0))
    ang = np.linspace(0.0, np.pi, m + 1)
    surf = np.stack([cx + R * np.cos(ang), cy + R * np.sin(ang)], 1)
    axis = []
    for x0, x1 in ((cx - R - grade, cx - R), (cx + R, min(Lx, cx + (R + grade) / wake_stretch))):
        x = x0 if x0 < cx else x0 + h_min
        while x < x1 - 0.5 * h_min:
            if 0.5 * h_max < x < Lx - 0.5 * h_max and (x < cx - R - 0.5 * h_min or x > cx + R + 0.5 * h_min):
                axis.append(x)
            x += float(spacing(np.array([[x, cy]]))[0])
    axis = np.stack([np.asarray(axis), np.full(len(axis), cy)], 1)
    # graded zone: Poisson-disk fronts grown from the surface and the axis up
    # to the lattice (half a lattice step beyond the zone, where the spacing
    # test against the lattice nodes decides)

    def admit(c):
        return ((c[:, 0] > 0.5 * h_max) & (c[:, 0] < Lx - 0.5 * h_max) & (c[:, 1] < Ly - 0.5 * h_max)
                & (c[:, 1] - cy > 0.4 * spacing(c)) & (reach(c) <= grade + 0.5 * h_max)
                & (np.hypot(c[:, 0] - cx, c[:, 1] - cy) > R + 0.5 * h_min))

    cand = _front_fill(np.concatenate([lat, bnd]), np.concatenate([surf, axis]), spacing, admit, rng)
    xy = np.concatenate([lat, cand, axis, surf, bnd])
    kind = np.concatenate([np.zeros(len(lat) + len(cand) + len(axis), np.uint8), np.full(len(surf), WALL, np.uint8),
                           np.full(len(bnd), DIRICHLET, np.uint8)])
    hloc = np.concatenate([np.full(len(lat), h_max), spacing(cand), spacing(axis), np.full(len(surf), h_min),
                           np.full(len(bnd), h_max)])
    fixed = np.concatenate([np.ones(len(lat), bool), np.zeros(len(cand) + len(axis), bool),
                            np.ones(len(surf) + len(bnd), bool)])
    keep = _cleanup(xy, hloc, fixed, lo, hi, (False, False), frac=0.45)
    xy, kind = xy[keep], kind[keep]
    # mirror everything off the axis
    off = xy[:, 1] > cy + 1e-12
    xy = np.concatenate([xy, xy[off] * [1.0, -1.0] + [0.0, 2.0 * cy]])
    kind = np.concatenate([kind, kind[off]])
    bc = np.zeros((len(xy), 3))
    bc[:, 0] = 1.0
    inout = (kind == DIRICHLET) & (np.isclose(xy[:, 0], 0.0) | np.isclose(xy[:, 0], Lx))
    y = xy[:, 1]
    bc[inout, 1] = 4.0 * u0 * y[inout] * (Ly - y[inout]) / Ly ** 2
    return NodeSet(xy=xy, kind=kind, lo=lo, hi=hi, periodic=(False, False), disks=np.array([[cx, cy, R]]), bc=bc,
                   h=h_max, name="karman-paper", h_min=h_min)


def random_disks(phi_target: float, r_min: float, r_max: float, gap: float,
                 rng, L: float = 1.0, max_tries: int = 200_000) -> np.ndarray:
    """Random sequential addition of non-overlapping disks in the periodic box
    [0, L)^2: radii uniform in [r_min, r_max], centres uniform, a candidate is
    rejected if it comes closer than `gap` to a placed disk (periodic images
    included).  Stops once the solid fraction reaches 1 - phi_target."""
    D = np.zeros((64, 3))
    m = 0
    solid = 0.0
    target = (1.0 - phi_target) * L * L
    tries = 0
    while solid < target and tries < max_tries:
        tries += 1
        rr = rng.uniform(r_min, r_max)
        c = rng.uniform(0.0, L, size=2)
        if m:
            d = D[:m, :2] - c
            d -= L * np.round(d / L)
            if not np.all(np.hypot(d[:, 0], d[:, 1]) >= D[:m, 2] + rr + gap):
                continue
        if m == len(D):
            D = np.concatenate([D, np.zeros_like(D)])
        D[m] = (c[0], c[1], rr)
        m += 1
        solid += np.pi * rr * rr
    return D[:m].copy()


def porous(n_target: int = 1_000_000, phi: float = 0.7, seed: int = 231214789,
           r_range=(0.01, 0.03), jitter: float = 0.25, L: float = 1.0,
           disks: np.ndarray | None = None, h: float | None = None) -> NodeSet:
    """Periodic box [0, L)^2 with random non-overlapping disks (porosity phi),
    fluid nodes on a jittered grid of spacing h ~ sqrt(phi L^2 / n_target) (or
    the given h; with jitter 0 and h = L / res the fluid nodes are the centres
    of the fluid pixels of a res^2 raster), and nodes exactly on every disk
    surface (no-slip, Sec. 3.2).  Disks keep a gap of at least 2h so every
    throat holds fluid nodes."""
    rng = np.random.default_rng(seed)
    if h is None:
        h = math.sqrt(phi * L * L / n_target)
    if disks is None:
        disks = random_disks(phi, r_range[0], r_range[1], 2.0 * h, rng, L)
    lo, hi = np.zeros(2), np.full(2, L)
    pts = _grid(lo, hi, h)
    if jitter > 0:
        pts = pts + rng.uniform(-jitter * h, jitter * h, size=pts.shape)
        pts = _wrap(pts, lo, hi, (True, True))
    # drop grid points inside a disk or closer than h/2 to its surface (periodic)
    from scipy.spatial import cKDTree

    keep = np.ones(len(pts), bool)
    if len(disks):
        tree = cKDTree(_in_box(pts, L), boxsize=L)
        for lst in tree.query_ball_point(_in_box(disks[:, :2], L), r=disks[:, 2] + 0.5 * h):
            keep[lst] = False
    fluid = pts[keep]
    surf = [_circle_nodes(c[0], c[1], c[2], h) for c in disks]
    surf = _wrap(np.concatenate(surf), lo, hi, (True, True)) if surf else np.zeros((0, 2))
    xy = np.concatenate([fluid, surf])
    kind = np.concatenate([np.zeros(len(fluid), np.uint8), np.full(len(surf), WALL, np.uint8)])
    hloc = np.full(len(xy), h)
    keep2 = _cleanup(xy, hloc, kind != FLUID, lo, hi, (True, True), frac=0.35)
    xy, kind = xy[keep2], kind[keep2]
    return NodeSet(xy=xy, kind=kind, lo=lo, hi=hi, periodic=(True, True),
                   disks=disks, h=h, name="porous")


def porous_channel(phi: float = 0.64, h: float = 5e-3, h_surf: float = 2.5e-3, band: float = 0.04,
                   r_range=(0.06, 0.1), seed: int = 231214789, L: float = 1.0, gap: float | None = None,
                   seam: float = 0.01, seam_jitter: float = 0.25) -> NodeSet:
    """The porous sample of Sec. 3.2: the box [0, L]^2, periodic along x,
    no-slip walls on y = 0 and y = L (nodes on them), random non-overlapping
    disks (radii uniform in r_range, porosity phi, clear of the walls), and a
    hybrid node set: a square lattice of spacing h farther than `band` from
    every disk, scattered nodes within the band whose spacing grows linearly
    from h_surf on the disk surfaces to h at the band's edge (placed by
    advancing Poisson-disk fronts from the surfaces), and nodes on every disk
    surface at spacing h_surf.  Disks keep `gap` (default 2 h_surf) from each
    other and from the walls.  seam > 0: the outer `seam` of the band holds
    lattice positions moved by U(-seam_jitter h, seam_jitter h) instead of
    front-filled nodes, so the fronts meet a jittered lattice and the exact
    lattice starts behind it."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    # disks: random sequential addition, periodic along x only
    disks = []
    solid, target, tries = 0.0, (1.0 - phi) * L * L, 0
    gap = 2.0 * h_surf if gap is None else gap
    while solid < target and tries < 200_000:
        tries += 1
        rr = rng.uniform(*r_range)
        c = np.array([rng.uniform(0.0, L), rng.uniform(rr + gap, L - rr - gap)])
        if disks:
            D = np.asarray(disks)
            d = D[:, :2] - c
            d[:, 0] -= L * np.round(d[:, 0] / L)
            if not np.all(np.hypot(d[:, 0], d[:, 1]) >= D[:, 2] + rr + gap):
                continue
        disks.append((c[0], c[1], rr))
        solid += np.pi * rr * rr
    disks = np.asarray(disks, dtype=np.float64).reshape(-1, 3)
    lo, hi = np.zeros(2), np.full(2, L)

    def surface_distance(pts):
        d = np.full(len(pts), np.inf)
        for cx, cy, r in disks:
            dx = pts[:, 0] - cx
            dx -= L * np.round(dx / L)
            d = np.minimum(d, np.hypot(dx, pts[:, 1] - cy) - r)
        return d

    # lattice: x = i h (periodic), y = j h (rows on both walls)
    nx, ny = int(round(L / h)), int(round(L / h))
    X, Y = np.meshgrid(np.arange(nx) * (L / nx), np.arange(ny + 1) * (L / ny), indexing="xy")
    lat = np.stack([X.ravel(), Y.ravel()], axis=1)
    dl = surface_distance(lat)
    jit = np.zeros((0, 2))
    if seam > 0.0:
        jit = lat[(dl > band - seam) & (dl <= band)]
        jit = jit[(jit[:, 1] > 0.5 * h) & (jit[:, 1] < L - 0.5 * h)]
        jit = jit + rng.uniform(-seam_jitter * h, seam_jitter * h, size=jit.shape)
        jit[:, 0] = np.mod(jit[:, 0], L)
    lat = lat[dl > band]
    surf = np.concatenate([_circle_nodes(c[0], c[1], c[2], h_surf) for c in disks]) if len(disks) else np.zeros((0, 2))
    surf[:, 0] = np.mod(surf[:, 0], L)
    walls = np.concatenate([np.stack([np.arange(nx) * (L / nx), np.zeros(nx)], 1),
                            np.stack([np.arange(nx) * (L / nx), np.full(nx, L)], 1)])
    on_wall_lat = (np.isclose(lat[:, 1], 0.0)) | (np.isclose(lat[:, 1], L))
    lat_in = lat[~on_wall_lat]

    # band: Poisson-disk fronts grown from the disk surfaces up to the lattice
    # (half a lattice step beyond the band, where the spacing test against the
    # lattice nodes decides)
    def spacing(pts):
        return h_surf + (h - h_surf) * np.clip(surface_distance(pts) / band, 0.0, 1.0)

    def admit(c):
        dc = surface_distance(c)
        return ((c[:, 1] > 0.5 * h_surf) & (c[:, 1] < L - 0.5 * h_surf) & (dc > 0.5 * h_surf)
                & (dc <= band - seam + 0.5 * h))

    cand = _front_fill(np.concatenate([lat_in, walls, jit]), surf, spacing, admit, rng, period_x=L)
    cand = np.concatenate([jit, cand])
    hloc_c = spacing(cand)
    xy = np.concatenate([lat_in, cand, surf, walls])
    kind = np.concatenate([np.zeros(len(lat_in) + len(cand), np.uint8), np.full(len(surf) + len(walls), WALL, np.uint8)])
    hloc = np.concatenate([np.full(len(lat_in), h), hloc_c, np.full(len(surf), h_surf), np.full(len(walls), h)])
    # lattice nodes are fixed too, so the clean-up removes band nodes only
    fixed = np.concatenate([np.ones(len(lat_in), bool), np.zeros(len(cand), bool), np.ones(len(surf) + len(walls), bool)])
    keep = _cleanup(xy, hloc, fixed, lo, hi, (True, False), frac=0.45)
    xy, kind = xy[keep], kind[keep]
    return NodeSet(xy=xy, kind=kind, lo=lo, hi=hi, periodic=(True, False), walls_y=(True, True),
                   disks=disks, h=h, name="porous-channel", h_min=h_surf)


def porous_batch(n_samples: int = 64, seed: int = 231214789, n_range=(50_000, 400_000),
                 phi_range=(0.55, 0.85), r_range=(0.01, 0.03), log=None) -> list:
    """n_samples porous media with node counts and porosities drawn uniformly
    from the given ranges (sample s uses seed + s); log(message) every 32
    samples if given."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=n_samples)
    phis = rng.uniform(phi_range[0], phi_range[1], size=n_samples)
    out = []
    for s in range(n_samples):
        out.append(porous(int(ns[s]), float(phis[s]), seed=seed + 1 + s, r_range=r_range))
        if log is not None and s % 32 == 31:
            log(f"{s + 1}/{n_samples} samples")
    return out


# --------------------------------------------------------------------------
# Fields and masks
# --------------------------------------------------------------------------

def raster_mask(disks: np.ndarray, res: int = 256, L: float = 1.0) -> np.ndarray:
    """Solid mask (1 = solid) of periodic disks at pixel centres of a res^2 raster."""
    c = (np.arange(res) + 0.5) * L / res
    X, Y = np.meshgrid(c, c, indexing="xy")
    m = np.zeros((res, res), np.float32)
    for cx, cy, r in disks:
        dx = X - cx
        dy = Y - cy
        dx -= L * np.round(dx / L)
        dy -= L * np.round(dy / L)
        m[(dx * dx + dy * dy) < r * r] = 1.0
    return m


def smooth_fields(xy: np.ndarray, seed: int, amp_u: float = 0.01, amp_rho: float = 1e-3,
                  L: float = 1.0, modes: int = 3):
    """Smooth periodic random fields (rho, ux, uy) at the given points: sums of a
    few low Fourier modes with seeded amplitudes and phases."""
    rng = np.random.default_rng(seed)
    out = []
    for amp, base in ((amp_rho, 1.0), (amp_u, 0.0), (amp_u, 0.0)):
        f = np.full(len(xy), base)
        for _ in range(modes):
            kx, ky = rng.integers(1, 4, size=2)
            ph = rng.uniform(0, 2 * np.pi)
            a = rng.uniform(0.3, 1.0) * amp / modes
            f = f + a * np.sin(2 * np.pi * (kx * xy[:, 0] + ky * xy[:, 1]) / L + ph)
        out.append(f)
    return out[0], np.stack([out[1], out[2]], axis=1)


def noise(shape, seed: int, amp: float) -> np.ndarray:
    """Seeded uniform noise in [-amp, amp]."""
    return np.random.default_rng(seed).uniform(-amp, amp, size=shape)
