"""Pins of the oracle's per-departure-point stencils (the paper's: the K
nearest Eulerian nodes of each departure point, Sec. 2.2) and of the simple
bounce-back option (Sec. 3.1): the lattice limit s = 1 equals lattice LBM,
mass on periodic lattices, uniform flow, second-order Taylor-Green decay with
the paper's 25-node stencils, and the simple bounce-back's exact mass balance
in a walled lattice channel."""
import numpy as np
import pytest

import nodesets
from oracle import lattice as lt
from oracle import lbm, mlbm
from oracle.rbf import nearest, nearest_to_point


def test_nearest_to_point_at_a_node_is_the_node_stencil():
    ns = nodesets.jittered_grid(12, seed=2)
    for i in (0, 37, 143):
        a, da = nearest(ns.xy, i, 13, ns.hi - ns.lo, ns.periodic)
        b, db = nearest_to_point(ns.xy, i, np.zeros(2), 13, ns.hi - ns.lo, ns.periodic)
        np.testing.assert_array_equal(a, b)
        np.testing.assert_array_equal(da, db)


def test_per_departure_stencils_surround_their_departure_points():
    ns = nodesets.jittered_grid(16, seed=3)
    dx = 1.0 / 16 / 1.7
    st = mlbm.build_stencils(ns, 12, dx, per_departure=True)
    assert st.idx.shape == (ns.n, 8, 12)
    for i in (5, 100):
        for k in range(8):
            p = ns.xy[i] + st.point[i, k]
            X = nodesets._min_image(ns.xy[st.idx[i, k]] - p, ns.hi - ns.lo, ns.periodic)
            d = np.hypot(ns.xy[:, 0] - p[0], ns.xy[:, 1] - p[1])
            # the K nearest of p, and the weights interpolate linears at p
            assert np.max(np.hypot(X[:, 0], X[:, 1])) <= np.sort(d)[11] + 1e-12
            np.testing.assert_allclose(st.w[i, k].sum(), 1.0, atol=1e-12)
            np.testing.assert_allclose(st.w[i, k] @ X, 0.0, atol=1e-13)


@pytest.mark.parametrize("taus,g", [((0.8, 0.8), (0.0, 0.0)), ((0.53, 0.5 + 0.1875 / 0.03), (2e-5, -1e-5))])
def test_per_departure_at_s1_is_lbm(taus, g):
    n = 16
    ns = nodesets.regular_grid(n)
    st = mlbm.build_stencils(ns, 25, 1.0 / n, per_departure=True)
    rho, u = nodesets.smooth_fields(ns.xy, 1, amp_u=0.03, amp_rho=0.01)
    f = mlbm.init_populations(rho, u)
    fl = f.reshape(9, n, n).copy()
    for _ in range(20):
        f = mlbm.step(f, ns, st, *taus, g)
        fl = lbm.step(fl, *taus, g)
    np.testing.assert_allclose(f, fl.reshape(9, -1), atol=1e-14, rtol=0)


@pytest.mark.parametrize("s", [1.5, 2.7])
def test_per_departure_mass_is_conserved_on_periodic_lattices(s):
    n = 16
    ns = nodesets.regular_grid(n)
    st = mlbm.build_stencils(ns, 25, 1.0 / n / s, per_departure=True)
    rho, u = nodesets.smooth_fields(ns.xy, 3, amp_u=0.03, amp_rho=0.01)
    f = mlbm.init_populations(rho, u)
    m0 = f.sum()
    for _ in range(30):
        f = mlbm.step(f, ns, st, 0.8, 0.8, (1e-5, 0.0))
    assert abs(f.sum() - m0) < 1e-13 * m0


def test_per_departure_uniform_flow_is_a_fixed_point():
    ns = nodesets.jittered_grid(16, seed=6)
    st = mlbm.build_stencils(ns, 25, 1.0 / 16 / 1.7, per_departure=True)
    f = mlbm.init_populations(np.ones(ns.n), np.tile([0.02, -0.01], (ns.n, 1)))
    f0 = f.copy()
    for _ in range(10):
        f = mlbm.step(f, ns, st, 0.8, 0.8)
    np.testing.assert_allclose(f, f0, atol=1e-15, rtol=0)


def _tgv(n, steps, s=1.5, tau=0.8, u0=0.01):
    ns = nodesets.jittered_grid(n, seed=11)
    dx = 1.0 / n / s
    st = mlbm.build_stencils(ns, 25, dx, per_departure=True)
    k = 2 * np.pi
    x, y = ns.xy[:, 0], ns.xy[:, 1]
    u = np.stack([u0 * np.sin(k * x) * np.cos(k * y), -u0 * np.cos(k * x) * np.sin(k * y)], 1)
    rho = 1 - (u0 ** 2 / (4 * lt.CS2)) * (np.cos(2 * k * x) + np.cos(2 * k * y))
    f = mlbm.init_populations(rho, u)
    for _ in range(steps):
        f = mlbm.step(f, ns, st, tau, tau)
    _, uu = mlbm.macroscopic(f, ns)
    ex = u * np.exp(-2 * lt.viscosity(tau) * (k * dx) ** 2 * steps)
    return np.linalg.norm(uu - ex) / np.linalg.norm(ex)


def test_per_departure_taylor_green_decay_converges():
    e16 = _tgv(16, 63)
    e32 = _tgv(32, 250)
    assert e32 < 2e-2
    assert e16 / e32 > 3.0


def test_simple_bounce_back_conserves_mass_in_a_walled_channel():
    # lattice channel with nodes on the walls, dx = h: the population sent
    # into a wall comes back to the same node, so the total is exact
    ns = nodesets.channel(8, 9, Lx=1.0, H=1.0)
    dx = 1.0 / 8
    st = mlbm.build_stencils(ns, 12, dx, simple_bb=True)
    wall = np.nonzero(ns.kind == nodesets.WALL)[0]
    i = wall[0]
    for k in range(1, 9):
        if st.src[i, k - 1] == lt.OPP[k]:
            np.testing.assert_array_equal(st.point[i, k - 1], 0.0)
            j = int(np.argmax(st.w[i, k - 1]))
            assert st.idx[i, j] == i and st.w[i, k - 1, j] == 1.0
    rho, u = nodesets.smooth_fields(ns.xy, 5, amp_u=0.02, amp_rho=0.01)
    u[wall] = 0.0
    f = mlbm.init_populations(rho, u)
    m0 = f.sum()
    for _ in range(50):
        f = mlbm.step(f, ns, st, 0.7, 0.7, (1e-5, 0.0))
    assert abs(f.sum() - m0) < 1e-13 * m0
