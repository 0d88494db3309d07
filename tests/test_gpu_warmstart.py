"""The learned warm start end to end at a small size: steady states from
batched library runs, training with the library's kernels, and what the
trained network gains over starting from rest (the plain run is the
reference: the warm-started run must converge to its permeability within
0.5 %)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def W():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_14789_amd import warmstart

    return warmstart


def test_warm_start_gains_over_rest(W):
    import time

    from paper_2312_14789_amd import unet

    res, g = 64, 1e-5
    # geometries in this process (no workers forked from a process using the GPU)
    geoms = W.make_geometries(104, res=res, seed=77, r_range=(0.04, 0.12), workers=1)
    train_g, test_g = geoms[:96], geoms[96:]
    fields, steps = W.steady_states(train_g, g, batch_size=96)
    train_g, fields, steps, dropped = W.converged_only(train_g, fields, steps)
    print(f"[warm] training steady states: steps {min(steps)}..{max(steps)}, {dropped} not converged", flush=True)
    assert dropped == 0
    data = W.Dataset(train_g, fields, res)
    # four levels: the coarsest is 8 pixels wide at res 64
    net = unet.UNet((32, 64, 128, 256), res=res, batch=8, seed=1)
    hist = W.train(net, data, epochs=60, lr=2e-3)
    print(f"[warm] loss {hist[0]:.4f} -> {hist[-1]:.4f}", flush=True)
    assert hist[-1] < 0.3 * hist[0]
    t0 = time.perf_counter()
    preds = W.predict(net, data, [m for _, m in test_g], data.u_scale, data.r_scale)
    infer = (time.perf_counter() - t0) / len(test_g)
    gains = []
    for (ns, _), f in zip(test_g, preds):
        r = W.compare_runs(ns, f, res, g, infer_s=infer)
        rel = abs(r["warm"]["permeability"] / r["rest"]["permeability"] - 1)
        p = r["prediction"]
        # the prediction against the steady state: a finite error, a flux of the right sign and size
        assert np.isfinite(p["rel_err"]) and p["rel_err"] < 1.0 and 0.5 < p["flux_ratio"] < 1.5
        print(f"[warm] steps rest {r['rest']['steps']} warm {r['warm']['steps']} k err {rel:.2e}", flush=True)
        assert rel <= 5e-3
        gains.append(r["rest"]["steps"] / r["warm"]["steps"])
    print(f"[warm] mean step ratio rest/warm {np.mean(gains):.2f}", flush=True)
    # the residual decays at the rate of the slowest mode, so the steps saved
    # grow with the logarithm of the prediction's accuracy: a few per cent
    # here, at this small training set
    assert np.mean(gains) >= 1.05
