"""Failure detection and checkpoint/resume through the C ABI.

A node whose fields are not finite (or whose density is not positive) must
be counted and named by the device reductions, and a run to steady state
must stop with MLBM_ERR_UNSTABLE instead of stepping on.  The faulty value
is planted in the initial fields on the host: arithmetic on NaN never
faults, so every kernel still runs to its normal end.

A run resumed from a checkpoint continues bitwise as the uninterrupted run
(the paper's porous runs take up to 1.56e6 steps, Sec. 3.2), including the
stochastic rounding of 16-bit states, whose random bits are keyed by the
step count that the checkpoint carries."""
import numpy as np
import pytest

import nodesets
from oracle import mlbm as omlbm

from gpu_util import initial_fields, sim_from_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_14789_amd import mlbm

    return mlbm


_CASE = {}


def _case():
    if not _CASE:
        ns = nodesets.porous(3000, phi=0.7, seed=6, r_range=(0.05, 0.09))
        st = omlbm.build_stencils(ns, 16, ns.h)
        _CASE["c"] = (ns, st)
    return _CASE["c"]


@pytest.mark.parametrize("variant,storage,bad", [(1, 1, "nan"), (0, 1, "nan"), (1, 0, "negative"),
                                                 (0, 2, "nan")])
def test_a_bad_node_is_counted_named_and_stops_the_run(M, variant, storage, bad):
    from paper_2312_14789_amd import _lib

    ns, st = _case()
    tau = 1.0 if variant == 1 else 0.8
    sim = sim_from_oracle(M, ns, st, variant, storage, tau, tau, (1e-6, 0.0), scale_exp=14)
    rho, u = initial_fields(ns, 3, 0.01, 0.001)
    j = 1234
    if bad == "nan":
        u[j, 0] = np.nan
    else:
        rho[j] = -0.5
    print(f"[failure] variant={variant} storage={storage} bad={bad} node={j}", flush=True)
    sim.init_state(rho, u)
    _, _, red = sim.macroscopic(ns.h)
    red = red.cpu().numpy()
    assert red[_lib.RED_N_BAD] == 1
    assert red[_lib.RED_FIRST_BAD] == j
    if bad == "negative":
        # one negative density is no lasting fault: the next MLBM1 update of
        # that node takes only 4/9 of its own fields (the rest population) and
        # the rest from its neighbours, so it comes back positive
        return
    with pytest.raises(M.MlbmError) as e:
        sim.run_to_steady(ns.h, tol=1e-6, check_every=10, max_steps=1000)
    assert e.value.code == _lib.MLBM_ERR_UNSTABLE
    assert "after 10 steps" in str(e.value)


def test_a_healthy_run_reports_no_bad_node(M):
    from paper_2312_14789_amd import _lib

    ns, st = _case()
    sim = sim_from_oracle(M, ns, st, 1, 1, 1.0, 1.0, (1e-6, 0.0))
    sim.init_state(*initial_fields(ns, 3, 0.01, 0.001))
    steps, res, red = sim.run_to_steady(ns.h, tol=1e-6, check_every=100, max_steps=300)
    assert steps == 300 and red[_lib.RED_N_BAD] == 0 and red[_lib.RED_FIRST_BAD] == ns.n


@pytest.mark.parametrize("variant,storage,kw", [(1, 1, {}), (0, 1, {}), (0, 0, {}),
                                                (1, 2, {"stochastic_rounding": 1, "weights16": 1}),
                                                (0, 3, {"stochastic_rounding": 1})])
def test_resumed_run_is_bitwise_the_uninterrupted_one(M, variant, storage, kw, tmp_path):
    ns, st = _case()
    tau = 1.0 if variant == 1 else 0.8
    rho, u = initial_fields(ns, 4, 0.01, 0.001)

    def fresh():
        s_ = sim_from_oracle(M, ns, st, variant, storage, tau, tau, (1e-6, 0.0), scale_exp=14, **kw)
        s_.init_state(rho, u)
        return s_

    print(f"[checkpoint] variant={variant} storage={storage} {kw}", flush=True)
    a = fresh()
    a.step(77)
    path = str(tmp_path / "ck.npz")
    a.save_checkpoint(path)
    a.step(123)
    full = a.state_bytes().copy()
    b = fresh()                      # another simulation of the same set, at its own initial state
    b.load_checkpoint(path)
    assert b.ds.step_count == 77
    b.step(123)
    np.testing.assert_array_equal(b.state_bytes(), full)
    c = sim_from_oracle(M, ns, st, variant, 1 if storage != 1 else 0, tau, tau, (1e-6, 0.0))
    with pytest.raises(ValueError):
        c.load_checkpoint(path)      # another storage
