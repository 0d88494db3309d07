"""Plain FP64 reference of the warm-start network's layers (test
infrastructure only).

The warm start maps a rasterised porous geometry to an initial velocity and
density field.  Periodic samples get periodic (circular) padding.  Tensors
are NHWC: (batch, height, width, channels); convolution weights are
(kh, kw, c_in, c_out).  Every layer comes with its backward pass; the tests
pin them by finite differences and by brute-force loops on tiny inputs.
"""
import numpy as np


def conv2d(x, w, b):
    """out[n, y, x, o] = b[o] + sum_{dy, dx, i} x[n, y+dy-r, x+dx-r, i] w[dy, dx, i, o],
    indices periodic, r = kernel_size // 2."""
    kh, kw = w.shape[:2]
    r = kh // 2
    out = np.zeros(x.shape[:3] + (w.shape[3],))
    for dy in range(kh):
        for dx in range(kw):
            xs = np.roll(x, shift=(r - dy, r - dx), axis=(1, 2))  # xs[y, x] = x[y + dy - r, x + dx - r]
            out += xs @ w[dy, dx]
    return out + b


def conv2d_backward(x, w, dout):
    """Gradients (dx, dw, db) of conv2d for the output gradient dout."""
    kh, kw = w.shape[:2]
    r = kh // 2
    dx_ = np.zeros_like(x)
    dw = np.zeros_like(w)
    for dy in range(kh):
        for dxx in range(kw):
            xs = np.roll(x, shift=(r - dy, r - dxx), axis=(1, 2))
            dw[dy, dxx] = np.einsum("nyxi,nyxo->io", xs, dout)
            dx_ += np.roll(dout @ w[dy, dxx].T, shift=(dy - r, dxx - r), axis=(1, 2))
    db = dout.sum(axis=(0, 1, 2))
    return dx_, dw, db


def relu(x):
    return np.maximum(x, 0.0)


def relu_backward(y, dy):
    """Gradient through relu given its output y."""
    return dy * (y > 0)


def avgpool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def avgpool2_backward(dout):
    return np.repeat(np.repeat(dout, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    """Nearest-neighbour doubling."""
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_backward(dout):
    n, h, w, c = dout.shape
    return dout.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def masked_mse(pred, target, mask):
    """Mean over the masked pixels and all channels of (pred - target)^2, and
    its gradient with respect to pred."""
    m = mask[..., None]
    cnt = m.sum() * pred.shape[-1]
    d = (pred - target) * m
    return float((d * d).sum() / cnt), 2.0 * d / cnt


def adam(param, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba): returns updated (param, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return param - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# The network: an encoder-decoder with skip connections
# ---------------------------------------------------------------------------

def layer_shapes(channels, c_in, c_out):
    """(name, kernel, c_in, c_out) of every convolution, in order: two 3x3
    convolutions per encoder level (average pooling between levels), one
    nearest upsampling, a channel concatenation with the encoder output and
    two 3x3 convolutions per decoder level, a 1x1 head."""
    shapes = []
    prev = c_in
    for lvl, c in enumerate(channels):
        shapes.append((f"enc{lvl}a", 3, prev, c))
        shapes.append((f"enc{lvl}b", 3, c, c))
        prev = c
    for lvl in range(len(channels) - 2, -1, -1):
        c = channels[lvl]
        shapes.append((f"dec{lvl}a", 3, prev + c, c))
        shapes.append((f"dec{lvl}b", 3, c, c))
        prev = c
    shapes.append(("head", 1, prev, c_out))
    return shapes


def init_params(channels, c_in, c_out, seed):
    """He-normal weights, zero biases (FP64)."""
    rng = np.random.default_rng(seed)
    params = {}
    for name, k, ci, co in layer_shapes(channels, c_in, c_out):
        params[name + ".w"] = rng.normal(0.0, np.sqrt(2.0 / (k * k * ci)), size=(k, k, ci, co))
        params[name + ".b"] = np.zeros(co)
    return params


def forward(params, x, channels):
    """Network output and the activations the backward pass needs."""
    acts = {"in": x}
    skips = []
    h = x
    L = len(channels)
    for lvl in range(L):
        h = relu(conv2d(h, params[f"enc{lvl}a.w"], params[f"enc{lvl}a.b"]))
        acts[f"enc{lvl}a"] = h
        h = relu(conv2d(h, params[f"enc{lvl}b.w"], params[f"enc{lvl}b.b"]))
        acts[f"enc{lvl}b"] = h
        skips.append(h)
        if lvl < L - 1:
            h = avgpool2(h)
            acts[f"pool{lvl}"] = h
    for lvl in range(L - 2, -1, -1):
        u = upsample2(h)
        cat = np.concatenate([u, skips[lvl]], axis=-1)
        acts[f"cat{lvl}"] = cat
        h = relu(conv2d(cat, params[f"dec{lvl}a.w"], params[f"dec{lvl}a.b"]))
        acts[f"dec{lvl}a"] = h
        h = relu(conv2d(h, params[f"dec{lvl}b.w"], params[f"dec{lvl}b.b"]))
        acts[f"dec{lvl}b"] = h
    out = conv2d(h, params["head.w"], params["head.b"])
    return out, acts


def backward(params, acts, dout, channels):
    """Gradients of every parameter for the output gradient dout: the head,
    the decoder levels in the reverse of their forward order (0 up to L-2),
    then the encoder levels from the bottleneck down, adding the skip
    gradients where the pooled and the skipped paths meet."""
    g = {}
    L = len(channels)
    dh, g["head.w"], g["head.b"] = conv2d_backward(acts["dec0b"], params["head.w"], dout)
    dskip = [None] * L
    for lvl in range(0, L - 1):
        name_b, name_a = f"dec{lvl}b", f"dec{lvl}a"
        dh = relu_backward(acts[name_b], dh)
        dh, g[name_b + ".w"], g[name_b + ".b"] = conv2d_backward(acts[name_a], params[name_b + ".w"], dh)
        dh = relu_backward(acts[name_a], dh)
        dcat, g[name_a + ".w"], g[name_a + ".b"] = conv2d_backward(acts[f"cat{lvl}"], params[name_a + ".w"], dh)
        cu = dcat.shape[-1] - channels[lvl]
        dskip[lvl] = dcat[..., cu:]
        dh = upsample2_backward(dcat[..., :cu])   # gradient of this level's input
    for lvl in range(L - 1, -1, -1):
        if lvl < L - 1:
            dh = avgpool2_backward(dh) + dskip[lvl]
        name_b, name_a = f"enc{lvl}b", f"enc{lvl}a"
        dh = relu_backward(acts[name_b], dh)
        dh, g[name_b + ".w"], g[name_b + ".b"] = conv2d_backward(acts[name_a], params[name_b + ".w"], dh)
        dh = relu_backward(acts[name_a], dh)
        below = acts["in"] if lvl == 0 else acts[f"pool{lvl - 1}"]
        dh, g[name_a + ".w"], g[name_a + ".b"] = conv2d_backward(below, params[name_a + ".w"], dh)
    return g
