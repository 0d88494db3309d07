"""Pins of the oracle's hybrid (regular + scattered) discretisation: the
biquadratic Lagrange weights against what fixes them (the nine biquadratic
monomials, successive one-dimensional quadratic fits by numpy, the lattice
shift at dx = h), the regular-block detection on a lattice with one displaced
node, and whole hybrid steps (s = 1 equals lattice LBM, mass on a periodic
lattice, fixed points, Taylor-Green convergence on a partly jittered set)."""
import numpy as np
import pytest

import nodesets
from oracle import lagrange as lg
from oracle import lattice as lt
from oracle import lbm, mlbm


def _pts(seed, m=40, h=0.3):
    return np.random.default_rng(seed).uniform(-h, h, size=(m, 2))


def test_weights_reproduce_the_biquadratic_space_only():
    h = 0.3
    P = _pts(1, h=h)
    w = lg.biquadratic_weights(P, h)
    X = h * lt.E
    for a in range(3):
        for b in range(3):
            g = X[:, 0] ** a * X[:, 1] ** b
            np.testing.assert_allclose(w @ g, P[:, 0] ** a * P[:, 1] ** b, atol=1e-14, rtol=0)
    # nine conditions fix nine weights; a cubic term is not reproduced
    g3 = X[:, 0] ** 3
    assert np.max(np.abs(w @ g3 - P[:, 0] ** 3)) > 1e-3


def test_weights_equal_successive_one_dimensional_quadratic_fits():
    # tensor-product interpolation = quadratic through each row, evaluated at
    # p_x, then the quadratic through those three values, evaluated at p_y
    h = 0.25
    rng = np.random.default_rng(2)
    vals = rng.normal(size=9)
    grid = np.zeros((3, 3))  # [row y][column x]
    for j in range(9):
        grid[int(lt.E[j, 1]) + 1, int(lt.E[j, 0]) + 1] = vals[j]
    t = np.array([-h, 0.0, h])
    for p in _pts(3, m=10, h=h):
        rows = [np.polyval(np.polyfit(t, grid[r], 2), p[0]) for r in range(3)]
        want = np.polyval(np.polyfit(t, rows, 2), p[1])
        got = lg.biquadratic_weights(p[None], h)[0] @ vals
        assert got == pytest.approx(want, abs=1e-12)


def test_departure_points_at_dx_equal_h_pick_the_lattice_neighbour():
    h = 0.1
    for k in range(1, 9):
        w = lg.biquadratic_weights((-h * lt.E[k])[None], h)[0]
        want = np.zeros(9)
        want[lt.OPP[k]] = 1.0
        np.testing.assert_array_equal(w, want)


def test_block_detection_with_one_displaced_node():
    n = 12
    ns = nodesets.regular_grid(n)
    h = 1.0 / n
    i0 = 5 * n + 6
    ns.xy[i0, 0] += 0.1 * h
    blocks = [lg.lattice_block(ns, i, h) for i in range(ns.n)]
    bad = {i for i, b in enumerate(blocks) if b is None}
    x, y = i0 % n, i0 // n
    want = {((y + dy) % n) * n + (x + dx) % n for dx in (-1, 0, 1) for dy in (-1, 0, 1)}
    assert bad == want
    # members of a detected block are the lattice neighbours in D2Q9 order
    i = 2 * n + 2
    b = blocks[i]
    for j in range(9):
        assert b[j] == (2 + int(lt.E[j, 1])) * n + (2 + int(lt.E[j, 0]))


def test_hybrid_stencils_on_a_partly_jittered_set(oracle_cache):
    ns = nodesets.patch_jittered_grid(16, radius=0.2, seed=4)
    h = 1.0 / 16
    st = mlbm.build_stencils(ns, 12, h / 1.5, lattice_h=h)
    d = nodesets._min_image(ns.xy - 0.5, ns.hi - ns.lo, ns.periodic)
    far = np.hypot(d[:, 0], d[:, 1]) > 0.2 + 2.0 * h
    assert np.all(st.lagrange[far])
    assert not np.any(st.lagrange[np.hypot(d[:, 0], d[:, 1]) < 0.2 - 2.0 * h])
    lag = np.nonzero(st.lagrange)[0]
    assert np.all(st.w[lag][:, :, 9:] == 0.0) and np.all(st.idx[lag][:, 9:] == lag[:, None])
    # every weight row still interpolates constants and linears
    for i in range(ns.n):
        X = nodesets._min_image(ns.xy[st.idx[i]] - ns.xy[i], ns.hi - ns.lo, ns.periodic)
        np.testing.assert_allclose(st.w[i].sum(axis=1), 1.0, atol=1e-12)
        np.testing.assert_allclose(st.w[i] @ X, st.point[i], atol=1e-13)


def test_hybrid_step_at_s1_is_lbm():
    n = 16
    ns = nodesets.regular_grid(n)
    st = mlbm.build_stencils(ns, 10, 1.0 / n, lattice_h=1.0 / n)
    assert np.all(st.lagrange)
    rho, u = nodesets.smooth_fields(ns.xy, 1, amp_u=0.03, amp_rho=0.01)
    f = mlbm.init_populations(rho, u)
    fl = f.reshape(9, n, n).copy()
    for _ in range(20):
        f = mlbm.step(f, ns, st, 0.7, 1.1, (2e-5, -1e-5))
        fl = lbm.step(fl, 0.7, 1.1, (2e-5, -1e-5))
    np.testing.assert_allclose(f, fl.reshape(9, -1), atol=1e-14, rtol=0)


@pytest.mark.parametrize("s", [1.5, 3.0])
def test_hybrid_mass_is_conserved_on_a_periodic_lattice(s):
    n = 16
    ns = nodesets.regular_grid(n)
    st = mlbm.build_stencils(ns, 10, 1.0 / n / s, lattice_h=1.0 / n)
    rho, u = nodesets.smooth_fields(ns.xy, 3, amp_u=0.03, amp_rho=0.01)
    f = mlbm.init_populations(rho, u)
    m0 = f.sum()
    for _ in range(40):
        f = mlbm.step(f, ns, st, 0.8, 0.8, (1e-5, 0.0))
    assert abs(f.sum() - m0) < 1e-13 * m0


def test_hybrid_uniform_flow_is_a_fixed_point():
    ns = nodesets.patch_jittered_grid(20, radius=0.25, seed=6)
    st = mlbm.build_stencils(ns, 12, 1.0 / 20 / 1.7, lattice_h=1.0 / 20)
    assert 0 < st.lagrange.sum() < ns.n
    u = np.tile([0.02, -0.01], (ns.n, 1))
    f = mlbm.init_populations(np.ones(ns.n), u)
    f0 = f.copy()
    for _ in range(10):
        f = mlbm.step(f, ns, st, 0.8, 0.8)
    np.testing.assert_allclose(f, f0, atol=1e-15, rtol=0)


def _tgv_hybrid(n, steps, s=1.5, tau=0.8, u0=0.01):
    ns = nodesets.patch_jittered_grid(n, radius=0.3, seed=7)
    dx = 1.0 / n / s
    st = mlbm.build_stencils(ns, 12, dx, lattice_h=1.0 / n)
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


def test_hybrid_taylor_green_decay_converges():
    e32 = _tgv_hybrid(32, 250)
    e64 = _tgv_hybrid(64, 1000)
    assert e64 < 6e-3
    assert e32 / e64 > 3.0
