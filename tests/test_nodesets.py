"""Input generators: the node sets have the structure their docstrings state
(symmetry, nodes in the box and outside the solids, boundary nodes where the
boundary conditions need them, the lattice part of hybrid sets)."""
import numpy as np
from scipy.spatial import cKDTree

import nodesets


def _inside_disks(xy, disks, L=None):
    out = np.zeros(len(xy), bool)
    for cx, cy, r in disks:
        dx = xy[:, 0] - cx
        if L is not None:
            dx -= L * np.round(dx / L)
        out |= np.hypot(dx, xy[:, 1] - cy) < r - 1e-12
    return out


def test_paper_cylinder_channel():
    ns = nodesets.karman_paper()
    assert np.all((ns.xy >= ns.lo - 1e-12) & (ns.xy <= ns.hi + 1e-12))
    mirror = ns.xy * [1.0, -1.0] + [0.0, 1.0]
    d, j = cKDTree(ns.xy).query(mirror)
    assert d.max() < 1e-12 and np.array_equal(ns.kind[j], ns.kind)
    assert not np.any(_inside_disks(ns.xy, ns.disks))
    wall = ns.kind == nodesets.WALL
    np.testing.assert_allclose(np.hypot(ns.xy[wall, 0] - 0.5, ns.xy[wall, 1] - 0.5), 0.07, atol=1e-12)
    dirich = ns.kind == nodesets.DIRICHLET
    on_side = (np.isclose(ns.xy[:, 0], 0) | np.isclose(ns.xy[:, 0], 3) | np.isclose(ns.xy[:, 1], 0)
               | np.isclose(ns.xy[:, 1], 1))
    assert np.array_equal(dirich, on_side)
    bc = ns.boundary_values()
    inlet = dirich & np.isclose(ns.xy[:, 0], 0)
    y = ns.xy[inlet, 1]
    np.testing.assert_allclose(bc[inlet, 1], 0.04 * y * (1 - y), atol=1e-15)
    nn, _ = cKDTree(ns.xy).query(ns.xy, k=2)
    assert nn[:, 1].min() > 0.4 * ns.h_min


def test_porous_channel():
    ns = nodesets.porous_channel()
    assert ns.periodic == (True, False) and ns.walls_y == (True, True)
    assert abs(ns.fluid_area() - 0.64) < 0.01
    assert not np.any(_inside_disks(ns.xy, ns.disks, L=1.0))
    # disks clear of the walls and of each other
    r = ns.disks[:, 2]
    assert np.all(ns.disks[:, 1] - r > 0) and np.all(ns.disks[:, 1] + r < 1)
    wall_rows = np.isclose(ns.xy[:, 1], 0) | np.isclose(ns.xy[:, 1], 1)
    assert np.all(ns.kind[wall_rows] == nodesets.WALL)
    # the lattice part: nodes farther than the band (plus the half lattice step
    # the band's fronts may reach beyond it) from every disk sit on the h lattice
    far = np.ones(ns.n, bool)
    for cx, cy, rr in ns.disks:
        dx = ns.xy[:, 0] - cx
        dx -= np.round(dx)
        far &= np.hypot(dx, ns.xy[:, 1] - cy) - rr > 0.04 + 0.5 * ns.h + 1e-9
    grid = ns.xy[far] / ns.h
    np.testing.assert_allclose(grid, np.round(grid), atol=1e-9)
    assert far.sum() > 0.15 * ns.n
    # band nodes keep their spacing: no pair closer than 0.99 of the finer spacing
    d, _ = cKDTree(ns.xy, boxsize=[1.0, 1e30]).query(ns.xy, k=2)
    assert d[:, 1].min() > 0.95 * ns.h_min


def test_hybrid_karman_lattice():
    ns = nodesets.karman(n_target=20000, hybrid=True)
    assert abs(22.0 / ns.h - round(22.0 / ns.h)) < 1e-9 and abs(4.1 / ns.h - round(4.1 / ns.h)) < 1e-9
    fluid = ns.kind == nodesets.FLUID
    # the lattice part sits on the vertices i h, j h, continuing into the
    # Dirichlet nodes of the sides
    g = ns.xy[fluid] / ns.h
    on_lattice = np.all(np.abs(g - np.round(g)) < 1e-9, axis=1)
    assert on_lattice.mean() > 0.4
    dirich = ns.kind == nodesets.DIRICHLET
    gd = ns.xy[dirich] / ns.h
    assert np.all(np.abs(gd - np.round(gd)) < 1e-9)


def test_poisson_karman():
    ns = nodesets.karman(n_target=20000, poisson=True)
    assert abs(ns.n - 20000) < 0.1 * 20000
    assert np.all((ns.xy >= ns.lo - 1e-12) & (ns.xy <= ns.hi + 1e-12))
    assert not np.any(_inside_disks(ns.xy, ns.disks))
    d, _ = cKDTree(ns.xy).query(ns.xy, k=2)
    # no pair closer than (about) the local spacing; the fine ring keeps h_f
    assert d[:, 1].min() > 0.95 * ns.h_min
    fluid = ns.kind == nodesets.FLUID
    r = np.hypot(ns.xy[:, 0] - 2.0, ns.xy[:, 1] - 2.0)
    ring = fluid & (r > 0.6) & (r < 1.4)
    far = fluid & (ns.xy[:, 0] > 6.0) & (ns.xy[:, 0] < 20.0) & (ns.xy[:, 1] > 0.3) & (ns.xy[:, 1] < 3.8)
    # 4x the node density within 1D of the cylinder
    dens_ring = ring.sum() / (np.pi * (1.4 ** 2 - 0.6 ** 2))
    dens_far = far.sum() / (14.0 * 3.5)
    assert 3.4 < dens_ring / dens_far < 4.6
    # nearest-neighbour distances sit between h and 1.6 h: no holes, no clusters
    nn_far = d[far, 1] / ns.h
    assert np.percentile(nn_far, 1) > 0.98 and np.percentile(nn_far, 99) < 1.6
