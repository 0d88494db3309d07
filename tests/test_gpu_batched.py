"""Batched runs (many samples in one launch, persistent tile queue, HIP graph
replay, on-device retirement): every sample's state is bitwise the state of
the same sample run alone, with and without graph capture, and samples retire
at the check where their residual first falls below the tolerance."""
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


def _samples(M, sizes=(1500, 2600, 4100), seed=40, variant_pop=False):
    out = []
    for j, n in enumerate(sizes):
        ns = nodesets.porous(n, phi=0.7 + 0.05 * j, seed=seed + j, r_range=(0.04, 0.08))
        b = M.build_stencils_for(ns, 16, ns.h)
        out.append((ns, b))
    return out


def _rows(raw, n_total, a, m, variant, tb):
    """Bytes of node rows [a, a+m) of every state block."""
    if variant == 1:
        blk = raw.reshape(n_total, 4 * tb)
        return blk[a:a + m].tobytes()
    main = raw[: 8 * tb * n_total].reshape(n_total, 8 * tb)
    rest = raw[8 * tb * n_total:].reshape(n_total, tb)
    return main[a:a + m].tobytes() + rest[a:a + m].tobytes()


@pytest.mark.parametrize("variant,storage,group_bytes", [(1, 1, 160e6), (0, 1, 160e6), (1, 2, 160e6), (1, 1, 1),
                                                         (0, 1, 1)])
def test_batched_state_equals_single_runs(M, variant, storage, group_bytes):
    samples = _samples(M)
    g = (3e-6, 0.0)
    tau = 1.0 if variant == 1 else 0.8
    batch = M.BatchSimulation([(b, ns.kind[b["perm"]], None) for ns, b in samples], variant=variant,
                              storage=storage, tau_plus=tau, g=g, tile=256, check_every=100, scale_exp=16,
                              group_bytes=group_bytes)
    assert batch.batch.n_groups == (1 if group_bytes > 1 else len(samples))
    steps_ = 600
    for use_graph in (True, False):
        batch.init_state([np.ones(b["idx"].shape[0]) for _, b in samples],
                         [np.zeros((b["idx"].shape[0], 2)) for _, b in samples])
        ran = batch.run(steps_, tol=0.0, use_graph=use_graph)
        assert ran == steps_
        raw = batch.state_of(0)[0]
        tb = {1: 4, 2: 2}[storage]
        for s_, (ns, b) in enumerate(samples):
            sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[b["perm"]], b["area"], variant=variant,
                               storage=storage, tau_plus=tau, g=g, tile=256, scale_exp=16)
            sim.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
            sim.step(steps_)
            single = sim.state_bytes()
            a, m = int(batch.node_off[s_]), batch.sizes[s_]
            assert _rows(raw, batch.N, a, m, variant, tb) == _rows(single, m, 0, m, variant, tb), (s_, use_graph)


@pytest.mark.parametrize("group_bytes,xcd", [(160e6, 1), (2e6, 1), (160e6, 0)])
def test_batched_retirement(M, group_bytes, xcd):
    # once a sample retires, its group's persistent workgroups walk the
    # shortened active-tile list (split evenly over the XCDs with xcd)
    samples = _samples(M, sizes=(1200, 2000, 3200, 900), seed=50)
    g = (2e-6, 0.0)
    batch = M.BatchSimulation([(b, ns.kind[b["perm"]], None) for ns, b in samples], variant=1, storage=1,
                              g=g, tile=128, check_every=100, group_bytes=group_bytes, xcd_remap=xcd)
    batch.init_state([np.ones(b["idx"].shape[0]) for _, b in samples],
                     [np.zeros((b["idx"].shape[0], 2)) for _, b in samples])
    ran = batch.run(200000, tol=1e-6, use_graph=True)
    steps, res, ux = batch.results()
    print(f"[batched] steps={steps.tolist()} ran={ran}", flush=True)
    assert np.all(steps > 0) and ran == steps.max()
    assert np.all(res < 1e-6)
    raw = batch.state_of(0)[0]
    for s_, (ns, b) in enumerate(samples):
        # the single run of exactly that many steps ends in the same state, with
        # its own residual (FP64 sums in another order) below the tolerance too
        sim = M.Simulation(b["idx"], b["w"], b["bb"], ns.kind[b["perm"]], b["area"], variant=1, storage=1,
                           tau_plus=1.0, g=g, tile=128)
        sim.init_state(np.ones(ns.n), np.zeros((ns.n, 2)))
        n_steps, r1, red = sim.run_to_steady(ns.h, tol=1e-6, check_every=100, max_steps=int(steps[s_]))
        assert n_steps == steps[s_]
        a, m = int(batch.node_off[s_]), batch.sizes[s_]
        assert _rows(raw, batch.N, a, m, 1, 4) == _rows(sim.state_bytes(), m, 0, m, 1, 4)
        assert r1 == pytest.approx(res[s_], rel=1e-6)
        assert ux[s_] == pytest.approx(red[1], rel=1e-9)
