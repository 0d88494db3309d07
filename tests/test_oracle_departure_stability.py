"""Linear stability of the step with the paper's per-departure-point stencils
(Sec. 2.2: the K nearest Eulerian nodes of each departure point) against one
shared stencil per node, on the cylinder channel of Sec. 3.1 (the coarsened
node set, K = 25, TRT with tau+ = 0.53 and Lambda = 3/16, simple bounce-back,
Re = 105).

At rest the step is linear in the populations: the collision's equilibrium
is linear in (rho, j) there, the Dirichlet overwrite fixes the boundary
nodes' perturbation at zero and the streaming is the stencil weights.  The
one-step operator is assembled from the oracle's stencils as a sparse matrix
and its growth rate measured by power iteration from a seeded random
perturbation.  With shared stencils every perturbation decays; with
per-departure stencils one grows by about 6e-4 per step, localised a few
cylinder radii behind the cylinder (0.2 - 0.5 downstream of its centre), just off the axis (the grid-scale noise
the full runs develop there after ~1e4 steps).  Several minutes of CPU: run
with --run-slow."""
import numpy as np
import pytest
import scipy.sparse as sp

import nodesets
from oracle import lattice as lt
from oracle import mlbm


def linear_collision(tau_plus, tau_minus):
    """9 x 9 TRT collision of a perturbation of the rest state: the
    equilibrium's part linear in (rho, j) is w_k (rho + 3 e_k . j)."""
    A = lt.W[:, None] * (1.0 + 3.0 * (lt.E @ lt.E.T))
    P = np.zeros((9, 9))
    P[np.arange(9), lt.OPP] = 1.0
    sym, asym = 0.5 * (np.eye(9) + P), 0.5 * (np.eye(9) - P)
    return np.eye(9) - sym @ (np.eye(9) - A) / tau_plus - asym @ (np.eye(9) - A) / tau_minus


def one_step_operator(ns, st, tau_plus, tau_minus):
    """Sparse (9n x 9n) map of a rest-state perturbation (node-major, nine
    populations per node) over one collide-then-stream step."""
    n = ns.n
    live = (ns.kind != mlbm.DIRICHLET).astype(float)
    C = sp.kron(sp.diags(live), sp.csr_matrix(linear_collision(tau_plus, tau_minus)), format="csr")
    rows, cols, vals = [np.arange(n) * 9], [np.arange(n) * 9], [np.ones(n)]
    for k in range(1, 9):
        m = mlbm.members(st, k)
        rows.append(np.repeat(np.arange(n) * 9 + k, m.shape[1]))
        cols.append((m * 9 + st.src[:, k - 1][:, None]).ravel())
        vals.append(st.w[:, k - 1, :].ravel())
    S = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(9 * n, 9 * n))
    return (S @ C).tocsr()


def growth(L, iters, tail, seed=1):
    """Mean growth factor per step over the last `tail` of `iters` power
    iterations, and the final normalised perturbation."""
    v = np.random.default_rng(seed).normal(size=L.shape[0])
    v /= np.linalg.norm(v)
    logs = []
    for _ in range(iters):
        v = L @ v
        nv = np.linalg.norm(v)
        v /= nv
        logs.append(np.log(nv))
    return float(np.exp(np.mean(logs[-tail:]))), v


def test_rest_operator_with_shared_and_per_departure_stencils():
    # linear consistency of the assembled operator: one application equals
    # one oracle step of a small perturbation of the rest state (exactly
    # linear there, up to the equilibrium's quadratic terms)
    ns = nodesets.karman_paper(h_min=1.0 / 60, h_max=1.0 / 10)
    tp = 0.53
    tm = lt.tau_minus_from_lambda(tp, 3.0 / 16.0)
    dx = 0.14 / 30.0
    st = mlbm.build_stencils(ns, 25, dx, lattice_h=ns.h, per_departure=True, simple_bb=True)
    L = one_step_operator(ns, st, tp, tm)
    # the channel at rest: every Dirichlet node prescribes (1, 0, 0)
    import copy

    rest = copy.copy(ns)
    rest.bc = np.tile([1.0, 0.0, 0.0], (ns.n, 1))
    f0 = mlbm.init_populations(np.ones(ns.n), np.zeros((ns.n, 2)))
    eps = 1e-9
    dv = np.random.default_rng(4).normal(size=(ns.n, 9))
    f1 = mlbm.step(f0 + eps * dv.T, rest, st, tp, tm)
    lin = (L @ dv.ravel()).reshape(ns.n, 9).T * eps
    np.testing.assert_allclose(f1 - f0, lin, atol=1e-15)


@pytest.mark.slow
def test_per_departure_stencils_grow_a_near_wake_mode_shared_stencils_do_not():
    ns = nodesets.karman_paper()
    d, u0, tp = 0.14, 1e-2, 0.53
    tm = lt.tau_minus_from_lambda(tp, 3.0 / 16.0)
    dx = u0 * d / (105.0 * lt.viscosity(tp))
    rates = {}
    for mode in ("shared", "per-departure"):
        st = mlbm.build_stencils(ns, 25, dx, lattice_h=ns.h, per_departure=mode == "per-departure", simple_bb=True)
        rate, v = growth(one_step_operator(ns, st, tp, tm), iters=5000, tail=1000)
        amp = np.abs(v).reshape(ns.n, 9).sum(1)
        peak = ns.xy[np.argmax(amp)]
        rates[mode] = rate
        print(f"[stability] {mode}: growth per step {rate:.6f}, peak at {peak.round(3)}", flush=True)
        if mode == "per-departure":
            assert rate > 1.0003
            # a few radii behind the cylinder (centre 0.5, 0.5; radius 0.07), near the axis
            assert 0.6 < peak[0] < 1.1 and abs(peak[1] - 0.5) < 0.1
        else:
            assert rate < 1.0 + 2e-5
    assert rates["per-departure"] - rates["shared"] > 3e-4
