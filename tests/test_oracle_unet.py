"""Pins of the oracle's network layers: brute-force loops on tiny inputs,
finite-difference gradients of every layer and of a whole small network, and
closed forms (constant fields, the first Adam step)."""
import numpy as np
import pytest

from oracle import unet


def test_conv2d_matches_brute_force_periodic_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 5, 6, 3))
    for k in (1, 3):
        w = rng.normal(size=(k, k, 3, 4))
        b = rng.normal(size=4)
        out = unet.conv2d(x, w, b)
        r = k // 2
        ref = np.zeros_like(out)
        for n in range(2):
            for y in range(5):
                for xx in range(6):
                    for o in range(4):
                        s = b[o]
                        for dy in range(k):
                            for dx in range(k):
                                for i in range(3):
                                    s += x[n, (y + dy - r) % 5, (xx + dx - r) % 6, i] * w[dy, dx, i, o]
                        ref[n, y, xx, o] = s
        np.testing.assert_allclose(out, ref, atol=1e-12)


def test_conv2d_of_constant_field():
    x = np.full((1, 4, 4, 2), 0.5)
    w = np.random.default_rng(1).normal(size=(3, 3, 2, 3))
    out = unet.conv2d(x, w, np.zeros(3))
    np.testing.assert_allclose(out, np.broadcast_to(0.5 * w.sum(axis=(0, 1, 2)), out.shape), atol=1e-12)


def _fd_check(f, params, grads, rng, n=6, eps=1e-6):
    for name, p in params.items():
        flat = p.reshape(-1)
        for j in rng.choice(flat.size, size=min(n, flat.size), replace=False):
            old = flat[j]
            flat[j] = old + eps
            fp = f()
            flat[j] = old - eps
            fm = f()
            flat[j] = old
            fd = (fp - fm) / (2 * eps)
            assert grads[name].reshape(-1)[j] == pytest.approx(fd, rel=1e-5, abs=1e-8), (name, j)


def test_layer_gradients_by_finite_differences():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 4, 6, 3))
    w = rng.normal(size=(3, 3, 3, 2))
    b = rng.normal(size=2)
    t = rng.normal(size=(2, 4, 6, 2))
    loss = lambda: 0.5 * np.sum((unet.conv2d(x, w, b) - t) ** 2)
    dx, dw, db = unet.conv2d_backward(x, w, unet.conv2d(x, w, b) - t)
    _fd_check(loss, {"x": x, "w": w, "b": b}, {"x": dx, "w": dw, "b": db}, rng)
    # pooling and upsampling are adjoint pairs up to their factors
    a = rng.normal(size=(1, 4, 4, 2))
    c = rng.normal(size=(1, 2, 2, 2))
    assert np.sum(unet.avgpool2(a) * c) == pytest.approx(np.sum(a * unet.avgpool2_backward(c)))
    assert np.sum(unet.upsample2(c) * a) == pytest.approx(np.sum(c * unet.upsample2_backward(a)))


def test_network_gradients_by_finite_differences():
    rng = np.random.default_rng(3)
    channels = [3, 4, 5]
    params = unet.init_params(channels, 2, 3, seed=4)
    for k in params:
        if k.endswith(".b"):
            params[k] = rng.normal(scale=0.1, size=params[k].shape)
    x = rng.normal(size=(2, 8, 8, 2))
    t = rng.normal(size=(2, 8, 8, 3))
    mask = (rng.uniform(size=(2, 8, 8)) > 0.3).astype(float)

    def loss():
        out, _ = unet.forward(params, x, channels)
        return unet.masked_mse(out, t, mask)[0]

    out, acts = unet.forward(params, x, channels)
    l, dout = unet.masked_mse(out, t, mask)
    grads = unet.backward(params, acts, dout, channels)
    assert set(grads) == set(params)
    _fd_check(loss, params, grads, rng, n=3)


def test_first_adam_step_moves_by_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -1e-3, 0.2])
    p1, m, v = unet.adam(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    np.testing.assert_allclose(p1, p - 0.01 * np.sign(g), rtol=1e-6)


def test_layer_shapes_of_the_five_level_network():
    shapes = unet.layer_shapes([32, 64, 128, 256, 256], 16, 3)
    assert len(shapes) == 19
    assert shapes[0] == ("enc0a", 3, 16, 32)
    assert ("dec3a", 3, 512, 256) in shapes and ("dec0a", 3, 96, 32) in shapes
    assert shapes[-1] == ("head", 1, 32, 3)
