"""mlbm_macroscopic_static (the allocation-free reductions) against
mlbm_macroscopic with a caller workspace, through the C ABI: two calls in a
row on the same GPU, the second on a smaller node set, must give the same
fields and reductions (the same kernels sum in the same order, so the
results are identical, well inside the FP64 bar of 1e-12)."""
import ctypes

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


def _both(M, sim, dx, box_area):
    """(fields and reductions from mlbm_macroscopic, the same from
    mlbm_macroscopic_static), each with its own u_prev and reductions buffer."""
    import torch

    from paper_2312_14789_amd import _lib

    lib = _lib.lib
    dev = sim.state_d[0].device
    out = []
    for static in (False, True):
        rho = torch.empty(sim.n, dtype=torch.float64, device=dev)
        u = torch.empty((sim.n, 2), dtype=torch.float64, device=dev)
        u_prev = torch.full((sim.n, 2), 1e-3, dtype=torch.float64, device=dev)
        red = torch.full((_lib.RED_COUNT,), float("nan"), dtype=torch.float64, device=dev)
        red[_lib.RED_INT_UX] = 2e-4
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        args = (ctypes.byref(sim.params), ctypes.byref(sim.ds), sim.area_d.data_ptr(), float(dx), float(box_area),
                rho.data_ptr(), u.data_ptr(), u_prev.data_ptr())
        if static:
            _lib.check(lib.mlbm_macroscopic_static(*args, red.data_ptr(), stream))
        else:
            _lib.check(lib.mlbm_macroscopic(*args, sim.ws_d.data_ptr(), red.data_ptr(), stream))
        torch.cuda.synchronize()
        out.append((rho.cpu().numpy(), u.cpu().numpy(), u_prev.cpu().numpy(), red.cpu().numpy()))
    return out


def test_static_reductions_equal_the_workspace_ones_twice_in_a_row(M):
    # first call: a 3000-node porous MLBM1 sample (FP32, body force, walls);
    # second call: a smaller channel of populations (TRT, FP64) on the same
    # static array, which still holds the first call's partials
    ns1 = nodesets.porous(3000, phi=0.7, seed=6, r_range=(0.05, 0.09))
    st1 = omlbm.build_stencils(ns1, 16, ns1.h)
    ns2 = nodesets.channel(12, 25, jitter=0.25, seed=4, Lx=0.5, H=1.0)
    st2 = omlbm.build_stencils(ns2, 16, 1.0 / 24)
    cases = [(ns1, st1, 1, 1, 1.0, 1.0, (2e-6, 0.0), ns1.h),
             (ns2, st2, 0, 0, 0.9, 0.5 + 0.1875 / 0.4, (1e-6, 0.0), 1.0 / 24)]
    assert ns2.n < ns1.n
    for ns, st, variant, storage, tp, tm, g, dx in cases:
        print(f"[no-alloc] n={ns.n} variant={variant} storage={storage}", flush=True)
        sim = sim_from_oracle(M, ns, st, variant, storage, tp, tm, g)
        sim.init_state(*initial_fields(ns, 5, 0.01, 0.001))
        sim.step(40)
        (r0, u0, p0, red0), (r1, u1, p1, red1) = _both(M, sim, dx, float(np.prod(ns.hi - ns.lo)))
        np.testing.assert_array_equal(r1, r0)
        np.testing.assert_array_equal(u1, u0)
        np.testing.assert_array_equal(p1, p0)
        np.testing.assert_array_equal(red1, red0)
        assert red0[8] == 0 and red0[9] == ns.n and np.isfinite(red0[10:]).all()


def test_static_reductions_refuse_more_nodes_than_the_array_holds(M):
    from paper_2312_14789_amd import _lib

    ns = nodesets.channel(12, 25, jitter=0.25, seed=4, Lx=0.5, H=1.0)
    st = omlbm.build_stencils(ns, 16, 1.0 / 24)
    sim = sim_from_oracle(M, ns, st, 0, 1, 0.9, 0.9, (0.0, 0.0))
    sim.ds.n = _lib.STATIC_MAX_NODES + 1        # refused on the host, before any launch
    rc = _lib.lib.mlbm_macroscopic_static(ctypes.byref(sim.params), ctypes.byref(sim.ds), sim.area_d.data_ptr(),
                                          1.0, 1.0, None, None, None, sim.red_d.data_ptr(), None)
    assert rc == _lib.MLBM_ERR_ARG
    assert "static reduction buffer" in _lib.lib.mlbm_last_error().decode()
