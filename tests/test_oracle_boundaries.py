"""Pins of the oracle's boundary treatment and wall force against closed forms
and a conservation law, each paired with a planted mistake (in the oracle, on
the CPU) that the pin must catch.

Straight Dirichlet boundaries (Sec. 3.1): after collision every population of
a boundary node is the equilibrium of the prescribed density and velocity.
  - plane Couette flow between two Dirichlet lines, u = U y / H: exact on the
    lattice at s = 1 and tau = 1 (the collision then leaves only equilibria,
    so the overwrite drops nothing); first-order convergence otherwise (the
    overwrite drops the non-equilibrium part of the boundary populations);
  - body-force-driven flow between Dirichlet lines at rest, the parabola
    u = g y (H - y) / (2 nu), on scattered nodes at tau = 1: second order.
  The order of the overwrite (before or after the collision) matters only
  with a body force, and there neither order is exact: each gives the
  boundary populations half the force term's momentum too much or too little.
  No flow singles one out, so the order stays a reading of the text.

Wall force (momentum exchange on no-slip surfaces; not in the paper): over
one step, the fluid's momentum changes by the body force on it minus the
force on the solids.  On scattered nodes the streaming conserves momentum
only approximately, so the balance closes to a few per cent of the body
force; dropping the rest-state subtraction (a uniform pressure on the
discretised surface of a disk) misses it by more than the body force itself.
"""
import types

import numpy as np
import pytest

import nodesets
from oracle import lattice as lt
from oracle import mlbm


def _run_to_steady(ns, st, tau, g, tol, max_steps=60_000, every=200):
    f = mlbm.init_populations(np.ones(ns.n), np.zeros((ns.n, 2)))
    u_old = None
    for it in range(max_steps):
        f = mlbm.step(f, ns, st, tau, tau, g)
        if it % every == every - 1:
            _, u = mlbm.macroscopic(f, ns, g)
            if not np.all(np.isfinite(u)):
                break
            if u_old is not None and np.linalg.norm(u - u_old) <= tol * np.linalg.norm(u):
                break
            u_old = u
    return mlbm.macroscopic(f, ns, g)


def _channel_flow_error(ny, tau, s, jitter, u_top, umax, tol=1e-10, K=12, max_steps=60_000):
    """Relative L2 error of u_x on the fluid nodes of a Dirichlet channel at
    steady state against U y/H + g y (H - y) / (2 nu), lengths in streaming
    distances (the lattice unit is dx = h / s)."""
    ns = nodesets.dirichlet_channel(4, ny, u_top=u_top, jitter=jitter, seed=1)
    dx = ns.h / s
    H = 1.0 / dx
    nu = lt.viscosity(tau)
    g = 8.0 * nu * umax / H ** 2
    st = mlbm.build_stencils(ns, K, dx)
    _, u = _run_to_steady(ns, st, tau, (g, 0.0), tol, max_steps)
    y = ns.xy[:, 1] / dx
    exact = u_top * y / H + g / (2.0 * nu) * y * (H - y)
    fl = ns.kind == nodesets.FLUID
    if not np.all(np.isfinite(u[fl])):
        return np.inf
    return float(np.linalg.norm(u[fl, 0] - exact[fl]) / np.linalg.norm(exact[fl]))


def test_couette_is_exact_on_the_lattice_at_tau_1():
    # s = 1, tau = 1: every post-collision population is an equilibrium, the
    # linear profile is a fixed point of the lattice update, and the
    # Dirichlet lines impose it exactly
    err = _channel_flow_error(9, 1.0, 1.0, 0.0, u_top=0.01, umax=0.0, tol=1e-12)
    assert err < 1e-9


def test_couette_converges_at_first_order_on_scattered_nodes():
    e9 = _channel_flow_error(9, 0.8, 1.3, 0.25, u_top=0.01, umax=0.0)
    e17 = _channel_flow_error(17, 0.8, 1.3, 0.25, u_top=0.01, umax=0.0)
    assert e17 < 1.5e-2
    assert e9 / e17 > 1.7


def test_forced_flow_between_dirichlet_lines_converges_at_second_order():
    e9 = _channel_flow_error(9, 1.0, 1.3, 0.25, u_top=0.0, umax=0.01)
    e17 = _channel_flow_error(17, 1.0, 1.3, 0.25, u_top=0.0, umax=0.01)
    assert e17 < 3e-3
    assert e9 / e17 > 3.5


def test_couette_pin_catches_a_missing_overwrite(monkeypatch):
    # planted mistake: the boundary populations are collided like any other
    monkeypatch.setattr(mlbm, "dirichlet_overwrite", lambda fpost, ns: fpost)
    err = _channel_flow_error(9, 1.0, 1.0, 0.0, u_top=0.01, umax=0.0, tol=1e-12, max_steps=2000)
    assert not err < 1e-3


def test_couette_pin_catches_a_wrong_boundary_velocity(monkeypatch):
    # planted mistake: the boundary equilibrium is taken at the node's own
    # density and velocity instead of the prescribed ones
    def overwrite_local(fpost, ns):
        d = ns.kind == nodesets.DIRICHLET
        fpost[:, d] = lt.equilibrium(lt.density(fpost[:, d]), lt.velocity(fpost[:, d], (0.0, 0.0)))
        return fpost

    monkeypatch.setattr(mlbm, "dirichlet_overwrite", overwrite_local)
    err = _channel_flow_error(9, 1.0, 1.0, 0.0, u_top=0.01, umax=0.0, tol=1e-12, max_steps=2000)
    assert not err < 1e-3


# ---------------------------------------------------------------------------
# wall force: one-step momentum budget on a periodic sample with two disks
# ---------------------------------------------------------------------------

_BUDGET = {}


def _porous_budget(n, variant, tau_plus, tau_minus, steps=(200, 500)):
    """(body force, momentum change, wall force) over one step taken after
    each of `steps` steps from rest, in lattice units, each node counting
    A_i / dx^2 cells.  Populations: the momentum of the pre-collision
    populations; MLBM1: rho u of the stored fields."""
    key = (n, variant, tau_plus, tau_minus, steps)
    if key in _BUDGET:
        return _BUDGET[key]
    disks = np.array([[0.3, 0.35, 0.15], [0.75, 0.7, 0.12]])
    ns = nodesets.porous(n, phi=0.8, seed=3, disks=disks, jitter=0.25)
    dx = ns.h
    st = mlbm.build_stencils(ns, 16, dx)
    g = (0.01 * lt.viscosity(tau_plus) / (0.15 / dx) ** 2, 0.0)
    cells = st.area / dx ** 2
    out = []
    if variant == 0:
        f = mlbm.init_populations(np.ones(ns.n), np.zeros((ns.n, 2)))

        def mom(f_):
            return (cells[None, :, None] * f_[:, :, None] * lt.E[:, None, :]).sum(axis=(0, 1))
    else:
        rho, u = np.ones(ns.n), np.zeros((ns.n, 2))
    for it in range(max(steps) + 1):
        if it in steps:
            if variant == 0:
                F = mlbm.bounce_back_force(f, ns, st, tau_plus, tau_minus, g, dx)
                body = np.sum(cells * lt.density(f)) * np.asarray(g)
                dP = mom(mlbm.step(f, ns, st, tau_plus, tau_minus, g)) - mom(f)
            else:
                F = mlbm.mlbm1_bounce_back_force(rho, u, ns, st, g, dx)
                body = np.sum(cells * rho) * np.asarray(g)
                r2, u2 = mlbm.mlbm1_step(rho, u, ns, st, g)
                dP = (cells[:, None] * (r2[:, None] * u2 - rho[:, None] * u)).sum(axis=0)
            out.append((body, dP, F))
        if variant == 0:
            f = mlbm.step(f, ns, st, tau_plus, tau_minus, g)
        else:
            rho, u = mlbm.mlbm1_step(rho, u, ns, st, g)
    _BUDGET[key] = out
    return out


_CASES = [(700, 0, 1.0, 1.0), (700, 0, 0.8, lt.tau_minus_from_lambda(0.8, 3 / 16)), (700, 1, 1.0, 1.0),
          (2800, 0, 0.8, lt.tau_minus_from_lambda(0.8, 3 / 16)), (2800, 1, 1.0, 1.0)]


@pytest.mark.parametrize("n,variant,tau_plus,tau_minus", _CASES)
def test_wall_force_closes_the_momentum_budget(n, variant, tau_plus, tau_minus):
    for body, dP, F in _porous_budget(n, variant, tau_plus, tau_minus):
        # the walls take a large share of the body force by then
        assert F[0] > 0.3 * body[0]
        miss = (dP - (body - F)) / body[0]
        assert np.all(np.abs(miss) < 0.05), miss


@pytest.mark.parametrize("variant", [0, 1])
def test_budget_pin_catches_a_missing_rest_state_subtraction(monkeypatch, variant):
    # planted mistake: the wall force sums the populations themselves, not
    # their offsets from the rest state (the force functions are the only
    # readers of the lattice weights through this name)
    lt_mut = types.SimpleNamespace(**{k: getattr(lt, k) for k in dir(lt) if not k.startswith("__")})
    lt_mut.W = np.zeros(9)
    monkeypatch.setattr(mlbm, "lt", lt_mut)
    n, v, tp, tm = _CASES[2] if variant else _CASES[0]
    body, dP, F = _porous_budget(n, v, tp, tm, steps=(200,))[0]
    miss = (dP - (body - F)) / body[0]
    assert np.max(np.abs(miss)) > 1.0
