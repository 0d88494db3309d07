"""Pins of the oracle's lattice quantities and collision operator against the
moment identities that fix them (Sec. 2.1)."""
import numpy as np
import pytest

from oracle import lattice as lt


def _fields(n=50, seed=0, amp=0.1):
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(-0.05, 0.05, n)
    u = rng.uniform(-amp, amp, (n, 2))
    return rho, u


def test_lattice_constants():
    # e_k of Sec. 2.1, Eq. 2, opposite map, isotropy up to fourth order.
    assert lt.E.shape == (9, 2)
    assert list(lt.OPP) == [0, 3, 4, 1, 2, 7, 8, 5, 6]
    np.testing.assert_allclose(lt.W.sum(), 1.0, atol=1e-15)
    np.testing.assert_allclose(lt.W @ lt.E, 0.0, atol=1e-15)
    M2 = np.einsum("k,ka,kb->ab", lt.W, lt.E, lt.E)
    np.testing.assert_allclose(M2, lt.CS2 * np.eye(2), atol=1e-15)
    M3 = np.einsum("k,ka,kb,kc->abc", lt.W, lt.E, lt.E, lt.E)
    np.testing.assert_allclose(M3, 0.0, atol=1e-15)
    M4 = np.einsum("k,ka,kb,kc,kd->abcd", lt.W, lt.E, lt.E, lt.E, lt.E)
    d = np.eye(2)
    iso = lt.CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                         + np.einsum("ad,bc->abcd", d, d))
    np.testing.assert_allclose(M4, iso, atol=1e-15)


def test_equilibrium_moments():
    # The Hermite equilibrium has exact moments rho, rho u, rho cs2 I + rho u u.
    rho, u = _fields()
    feq = lt.equilibrium(rho, u)
    np.testing.assert_allclose(feq.sum(0), rho, rtol=1e-14)
    np.testing.assert_allclose(lt.momentum(feq), rho[:, None] * u, atol=1e-15)
    P = np.einsum("kn,ka,kb->nab", feq, lt.E, lt.E)
    Pex = rho[:, None, None] * (lt.CS2 * np.eye(2)[None] + u[:, :, None] * u[:, None, :])
    np.testing.assert_allclose(P, Pex, atol=1e-14)


def test_equilibrium_at_rest_is_weights():
    feq = lt.equilibrium(np.array([2.0]), np.zeros((1, 2)))
    np.testing.assert_allclose(feq[:, 0], 2.0 * lt.W, rtol=1e-15)


def test_guo_force_moments():
    # sum F = 0, sum e F = rho g, sum e e F = rho (g u + u g).
    rho, u = _fields()
    g = np.array([3e-4, -2e-4])
    F = lt.guo_force(rho, u, g)
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-17)
    np.testing.assert_allclose(lt.momentum(F), rho[:, None] * g[None], rtol=1e-12)
    S = np.einsum("kn,ka,kb->nab", F, lt.E, lt.E)
    Sex = rho[:, None, None] * (g[None, :, None] * u[:, None, :] + u[:, :, None] * g[None, None, :])
    np.testing.assert_allclose(S, Sex, atol=1e-17)


@pytest.mark.parametrize("taus", [(0.8, 0.8), (0.6, 1.3), (1.0, 1.0)])
def test_collision_conserves_mass_and_shifts_momentum(taus):
    rng = np.random.default_rng(3)
    rho, u = _fields(seed=4)
    f = lt.equilibrium(rho, u) + rng.uniform(-1e-3, 1e-3, (9, len(rho)))
    g = np.array([1e-5, 2e-5])
    fp = lt.collide(f, *taus, g)
    np.testing.assert_allclose(fp.sum(0), f.sum(0), rtol=1e-14)
    rho_f = f.sum(0)
    u_f = lt.velocity(f, g)
    # sum e f^post = rho u + rho g / 2 with u the half-force-shifted velocity
    np.testing.assert_allclose(lt.momentum(fp), rho_f[:, None] * u_f + 0.5 * rho_f[:, None] * g,
                               atol=1e-15)


def test_trt_relaxes_symmetric_and_antisymmetric_parts_separately():
    # A perturbation that is even under k -> k' (zero mass) relaxes with tau+;
    # an odd one (zero momentum) with tau-.  Swapping the two rates fails this.
    rho, u = _fields(n=3, seed=9)
    feq = lt.equilibrium(rho, u)
    tp, tm = 0.7, 1.9
    even = np.zeros((9, 3))
    even[1] = even[3] = 1e-4
    even[2] = even[4] = -1e-4            # zero mass, zero momentum, even
    odd = np.zeros((9, 3))
    odd[5], odd[7] = 1e-4, -1e-4
    odd[6], odd[8] = 1e-4, -1e-4
    odd[2], odd[4] = -2e-4, 2e-4         # odd under k -> k', zero momentum
    np.testing.assert_allclose(lt.momentum(odd), 0.0, atol=1e-18)
    for pert, tau in ((even, tp), (odd, tm)):
        fp = lt.collide(feq + pert, tp, tm)
        np.testing.assert_allclose(fp - feq, (1.0 - 1.0 / tau) * pert, atol=1e-15)


def test_tau_one_collision_is_equilibrium_plus_half_force():
    # BGK with tau = 1 (the LBM1 setting, Sec. 2.1, Eq. 10) returns the
    # equilibrium of the (force-shifted) fields plus half the force term.
    rng = np.random.default_rng(5)
    rho, u = _fields(seed=6)
    g = np.array([1e-4, 0.0])
    f = lt.equilibrium(rho, u) + rng.uniform(-1e-3, 1e-3, (9, len(rho)))
    ue = lt.velocity(f, g)
    re = f.sum(0)
    np.testing.assert_allclose(lt.collide(f, 1.0, 1.0, g),
                               lt.equilibrium(re, ue) + 0.5 * lt.guo_force(re, ue, g), atol=1e-16)


def test_lambda_relation():
    # Lambda = 1/4 with tau+ = 1 gives tau- = 1 (Sec. 2.1, LBM1 setting).
    assert lt.tau_minus_from_lambda(1.0, 0.25) == pytest.approx(1.0, abs=1e-15)
    assert lt.viscosity(0.8) == pytest.approx(0.1, abs=1e-15)
