"""Autotuner for single node sets: it times every launch shape on the node set
itself (one or eight lanes per node, tile, XCD order, sweeps) and applies the
fastest; the shapes it chooses among compute the same sums in the same order
(only the data movement differs), so the tuned run agrees with the default
shape to rounding (kernels built for different shapes may fuse multiply-adds
differently)."""
import numpy as np
import pytest

import nodesets

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_14789_amd import mlbm

    return mlbm


@pytest.mark.parametrize("variant,hybrid", [(0, False), (1, False), (0, True)])
def test_tuned_simulation_matches_default_shape(M, variant, hybrid, tmp_path):
    from paper_2312_14789_amd import autotune

    ns = nodesets.karman(n_target=20000, seed=9, hybrid=hybrid)
    b = M.build_stencils_for(ns, 16, ns.h_min, lattice_h=ns.h if hybrid else 0.0)
    perm = b["perm"]
    tau = 1.0 if variant == 1 else 0.7
    lag = dict(lagrange=b["lagrange"], w_lagrange=b["w_lagrange"]) if hybrid else {}

    def make():
        return M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[perm], b["area"], variant=variant, storage=M.F32,
                            tau_plus=tau, bc=ns.boundary_values()[perm], **lag)

    ref = make()
    ref.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
    ref.step(100)
    sim = make()
    best = autotune.tune_simulation(sim, steps=40, cache_path=str(tmp_path / "tune.json"))
    print(f"[autotune] variant={variant} best lanes={best['lanes']} tile={best['tile']} xcd={best['xcd']} "
          f"sweeps={best['sweeps']} {best['ms_per_step'] * 1e3:.1f} us/step over {len(best['timings'])} shapes",
          flush=True)
    # one lane per node with every tile; eight lanes per node with the tiles
    # it supports (global gathers, 64 and 128 nodes; hybrid sets: 64 and 128)
    per_tile = len(autotune.XCD) * len(autotune.SIM_SWEEPS)
    assert len(best["timings"]) == (len(autotune.SIM_TILES) + (2 if hybrid else 3)) * per_tile
    assert {r["lanes"] for r in best["timings"]} == {1, 8}
    assert sim.ds.tile == best["tile"] and sim.params.lanes_per_node == best["lanes"]
    sim.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
    sim.step(100)
    _, u, _ = sim.macroscopic(ns.h_min)
    _, u_ref, _ = ref.macroscopic(ns.h_min)
    u, u_ref = u.cpu().numpy(), u_ref.cpu().numpy()
    assert np.linalg.norm(u - u_ref) <= 1e-6 * np.linalg.norm(u_ref)
    again = autotune.tune_simulation(make(), steps=40, cache_path=str(tmp_path / "tune.json"))
    assert again["cached"] and again["tile"] == best["tile"] and again["lanes"] == best["lanes"]
