"""Warm-start network kernels (bf16 MFMA convolutions and the other layers)
against the FP64 oracle: single layers, then the forward and backward pass of
a small whole network.  Inputs are rounded to bf16 before both sides see them;
tolerances come from bf16 rounding of the stored activations (2^-9 relative
per rounding, a few roundings deep)."""
import ctypes

import numpy as np
import pytest

from oracle import unet as ou

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def U():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2312_14789_amd import unet

    return unet


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def _bf(U, a):
    return U.from_bf16_bits(U.to_bf16_bits(a)).astype(np.float64)


# widths 8 and 16 run the 8 x 8 and 8 x 16 pixel tiles, multiples of 32 the
# 8 x 32 tiles with 2 x 2 (64 output channels) or 2 x 1 (32) MFMA tiles per wave
@pytest.mark.parametrize("k,ci,co,w", [(3, 32, 64, 8), (3, 96, 32, 8), (1, 32, 32, 8), (3, 64, 128, 32),
                                       (3, 96, 64, 32), (1, 32, 32, 32), (3, 32, 96, 64), (3, 64, 32, 16)])
def test_conv_layer_forward_and_gradients(U, k, ci, co, w):
    import torch

    from paper_2312_14789_amd._lib import ConvDesc, check, lib

    rng = np.random.default_rng(k * 1000 + ci + co + w)
    n, h = 2, 16
    x = _bf(U, rng.normal(size=(n, h, w, ci)))
    wt = _bf(U, rng.normal(scale=0.2, size=(k, k, ci, co)))
    b = rng.normal(size=co).astype(np.float32).astype(np.float64)
    dy = _bf(U, rng.normal(size=(n, h, w, co)))
    ref = ou.conv2d(x, wt, b)
    rdx, rdw, rdb = ou.conv2d_backward(x, wt, dy)
    dev = torch.device("cuda")
    xd = torch.from_numpy(U.to_bf16_bits(x)).to(dev)
    wm = torch.from_numpy(np.ascontiguousarray(np.transpose(wt.reshape(k * k, ci, co), (2, 0, 1)),
                                               dtype=np.float32)).to(dev)
    wf = torch.empty((co, k * k, ci), dtype=torch.int16, device=dev)
    wd = torch.empty((ci, k * k, co), dtype=torch.int16, device=dev)
    bd = torch.from_numpy(b.astype(np.float32)).to(dev)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(lib.mlbm_conv_weights(ctypes.c_void_p(wm.data_ptr()), co, k, ci, ctypes.c_void_p(wf.data_ptr()),
                                ctypes.c_void_p(wd.data_ptr()), s))
    d = ConvDesc(n, h, w, ci, co, k, ci, 0, co, 0, co)
    y = torch.empty((n, h, w, co), dtype=torch.float32, device=dev)
    check(lib.mlbm_conv_forward(ctypes.byref(d), ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(wf.data_ptr()),
                                ctypes.c_void_p(bd.data_ptr()), ctypes.c_void_p(y.data_ptr()), 0, 1, s))
    assert _rel(y.cpu().numpy(), ref) < 1e-5  # FP32 accumulation of exact bf16 products
    dyd = torch.from_numpy(U.to_bf16_bits(dy)).to(dev)
    gw = torch.empty((co, k * k, ci), dtype=torch.float32, device=dev)
    gb = torch.empty(co, dtype=torch.float32, device=dev)
    ws = torch.empty(lib.mlbm_conv_wgrad_workspace(ctypes.byref(d), 3) // 4 + 1, dtype=torch.float32, device=dev)
    check(lib.mlbm_conv_wgrad(ctypes.byref(d), ctypes.c_void_p(xd.data_ptr()), ctypes.c_void_p(dyd.data_ptr()),
                              ctypes.c_void_p(gw.data_ptr()), ctypes.c_void_p(gb.data_ptr()), 3,
                              ctypes.c_void_p(ws.data_ptr()), s))
    gw_ref = np.transpose(rdw.reshape(k * k, ci, co), (2, 0, 1))
    assert _rel(gw.cpu().numpy(), gw_ref) < 1e-5
    assert _rel(gb.cpu().numpy(), rdb) < 1e-5
    dd = ConvDesc(n, h, w, co, ci, k, co, 0, ci, 0, ci)
    dx = torch.empty((n, h, w, ci), dtype=torch.float32, device=dev)
    check(lib.mlbm_conv_forward(ctypes.byref(dd), ctypes.c_void_p(dyd.data_ptr()), ctypes.c_void_p(wd.data_ptr()),
                                None, ctypes.c_void_p(dx.data_ptr()), 0, 1, s))
    assert _rel(dx.cpu().numpy(), rdx) < 1e-5


def _small_net(U, seed=3):
    channels = [32, 64, 64]
    res, batch = 32, 2
    net = U.UNet(channels, res=res, batch=batch, c_out=3, seed=seed)
    params = ou.init_params(channels, 32, 32, seed=seed + 1)
    rng = np.random.default_rng(seed + 2)
    for key in params:
        params[key] = _bf(U, params[key]) if key.endswith(".w") else rng.normal(scale=0.05, size=params[key].shape)
        params[key] = params[key].astype(np.float32).astype(np.float64)
    params["enc0a.w"][:, :, 1:, :] = 0.0
    params["head.w"][..., 3:] = 0.0
    params["head.b"][3:] = 0.0
    net.set_params(params)
    x = np.zeros((batch, res, res, 32))
    x[..., 0] = (rng.uniform(size=(batch, res, res)) > 0.3)
    target = rng.normal(size=(batch, res, res, 3))
    mask = x[..., 0].copy()
    return net, params, channels, x, target, mask


def test_network_forward_backward_matches_oracle(U):
    import torch

    net, params, channels, x, target, mask = _small_net(U)
    dev = torch.device("cuda")
    out = net.forward(torch.from_numpy(U.to_bf16_bits(x)).to(dev)).cpu().numpy()
    ref, acts = ou.forward(params, x, channels)
    err = _rel(out[..., :3], ref[..., :3])
    print(f"[unet] forward rel err {err:.2e}", flush=True)
    assert err < 3e-2
    tg = torch.from_numpy(target.astype(np.float32)).to(dev)
    mk = torch.from_numpy(mask.astype(np.float32)).to(dev)
    loss = float(net.loss_and_grad(tg, mk).item())
    l_ref, d3 = ou.masked_mse(ref[..., :3], target, mask)
    assert loss == pytest.approx(l_ref, rel=3e-2)
    net.backward()
    torch.cuda.synchronize()
    dout = np.zeros(ref.shape)
    dout[..., :3] = d3
    g_ref = ou.backward(params, acts, dout, channels)
    worst = 0.0
    for name, k, ci, co in net.shapes:
        gw = net.gw[name].cpu().numpy()
        ref_w = np.transpose(g_ref[name + ".w"].reshape(k * k, ci, co), (2, 0, 1))
        if name == "enc0a":
            gw, ref_w = gw[:, :, :1], ref_w[:, :, :1]
        if name == "head":
            gw, ref_w = gw[:3], ref_w[:3]
        e = _rel(gw, ref_w)
        worst = max(worst, e)
        print(f"[unet] grad {name}.w rel err {e:.2e}", flush=True)
        # bf16 storage of every activation and activation gradient moves these
        # gradients by up to 6.7 % (largest at the deepest layers) when the same
        # roundings are applied to the FP64 computation of this network; the bar
        # leaves room above that
        assert e < 1e-1, name
    print(f"[unet] worst weight-gradient rel err {worst:.2e}", flush=True)


def test_training_steps_reduce_the_loss(U):
    import torch

    net, params, channels, x, target, mask = _small_net(U, seed=7)
    # a learnable target: smooth functions of the geometry
    blur = ou.upsample2(ou.avgpool2(x[..., :1]))[..., 0]
    target = np.stack([blur, 0.5 * x[..., 0], blur * blur], axis=-1)
    dev = torch.device("cuda")
    xd = torch.from_numpy(U.to_bf16_bits(x)).to(dev)
    tg = torch.from_numpy(target.astype(np.float32)).to(dev)
    mk = torch.from_numpy(mask.astype(np.float32)).to(dev)
    losses = []
    for _ in range(30):
        net.forward(xd)
        losses.append(float(net.loss_and_grad(tg, mk).item()))
        net.backward()
        net.adam_step(3e-3)
    print(f"[unet] loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert losses[-1] < 0.7 * losses[0]
