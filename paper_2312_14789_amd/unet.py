"""The warm-start network: an encoder-decoder with skip connections whose
layers are the library's HIP kernels (include/mlbm_unet.h).

This module only allocates device buffers (PyTorch) and calls the layer
entry points in order; every convolution, pooling, upsampling, loss and
optimizer step runs in libmlbm.so.  Layout: NHWC bfloat16 activations, FP32
master weights [c_out][k*k][c_in] with bf16 copies for the forward pass and
for the data gradient, FP32 weight gradients and Adam moments.

Shape: per encoder level two 3x3 convolutions with ReLU (average pooling
between levels), per decoder level a nearest upsampling, a concatenation with
the encoder output of that level and two 3x3 convolutions with ReLU, then a
1x1 head.  The input is padded to 32 channels and the head to 32 output
channels (only the first `c_out` are used), so every convolution works on
multiples of 32 channels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import ConvDesc, check, lib

PAD = 32


def layer_shapes(channels, c_in=PAD, c_out=PAD):
    """(name, ksize, c_in, c_out) of every convolution in execution order."""
    shapes = []
    prev = c_in
    for lvl, c in enumerate(channels):
        shapes += [(f"enc{lvl}a", 3, prev, c), (f"enc{lvl}b", 3, c, c)]
        prev = c
    for lvl in range(len(channels) - 2, -1, -1):
        c = channels[lvl]
        shapes += [(f"dec{lvl}a", 3, prev + c, c), (f"dec{lvl}b", 3, c, c)]
        prev = c
    shapes.append(("head", 1, prev, c_out))
    return shapes


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class UNet:
    def __init__(self, channels=(32, 64, 128, 256, 256), res=256, batch=16, c_out=3, seed=0, device="cuda"):
        import torch

        self.torch = torch
        self.channels = list(channels)
        self.res, self.batch, self.c_out = res, batch, c_out
        self.L = len(channels)
        if res % (1 << (self.L - 1)) or (batch * (res >> (self.L - 1)) ** 2) % 128:
            raise ValueError("resolution / batch incompatible with the pooling levels")
        self.dev = torch.device(device)
        self.shapes = layer_shapes(self.channels)
        rng = np.random.default_rng(seed)
        self.w, self.b, self.wf, self.wd = {}, {}, {}, {}
        self.gw, self.gb, self.m, self.v = {}, {}, {}, {}
        for name, k, ci, co in self.shapes:
            fan = k * k * (1 if name == "enc0a" else ci)  # the input has one real channel
            w = rng.normal(0.0, np.sqrt(2.0 / fan), size=(co, k * k, ci)).astype(np.float32)
            if name == "enc0a":
                w[:, :, 1:] = 0.0
            if name == "head":
                w[c_out:] = 0.0
            self.w[name] = torch.from_numpy(w).to(self.dev)
            self.b[name] = torch.zeros(co, dtype=torch.float32, device=self.dev)
            self.wf[name] = torch.empty((co, k * k, ci), dtype=torch.int16, device=self.dev)
            self.wd[name] = torch.empty((ci, k * k, co), dtype=torch.int16, device=self.dev)
            self.gw[name] = torch.zeros_like(self.w[name])
            self.gb[name] = torch.zeros_like(self.b[name])
            for d in (self.m, self.v):
                d[name + ".w"] = torch.zeros_like(self.w[name])
                d[name + ".b"] = torch.zeros_like(self.b[name])
        self.shape_of = {n: (k, ci, co) for n, k, ci, co in self.shapes}
        self._alloc()
        self.refresh_weights()
        self.t = 0

    # ---- buffers ---------------------------------------------------------------------
    def _alloc(self):
        t, B, L, C = self.torch, self.batch, self.L, self.channels
        bf = t.int16
        self.A, self.G = {}, {}
        for lvl in range(L):
            R = self.res >> lvl
            c = C[lvl]
            self.A[f"enc{lvl}a"] = t.zeros((B, R, R, c), dtype=bf, device=self.dev)
            if lvl < L - 1:
                c_up = C[lvl + 1]
                self.A[f"cat{lvl}"] = t.zeros((B, R, R, c_up + c), dtype=bf, device=self.dev)
                self.A[f"pool{lvl}"] = t.zeros((B, R // 2, R // 2, c), dtype=bf, device=self.dev)
                self.A[f"dec{lvl}a"] = t.zeros((B, R, R, c), dtype=bf, device=self.dev)
                self.A[f"dec{lvl}b"] = t.zeros((B, R, R, c), dtype=bf, device=self.dev)
            else:
                self.A[f"enc{lvl}b"] = t.zeros((B, R, R, c), dtype=bf, device=self.dev)
        self.out = t.zeros((B, self.res, self.res, PAD), dtype=t.float32, device=self.dev)
        for k, v in self.A.items():
            self.G[k] = t.zeros_like(v)
        self.dout = t.zeros((B, self.res, self.res, PAD), dtype=bf, device=self.dev)
        ws = 0
        for name, k, ci, co in self.shapes:
            ws = max(ws, lib.mlbm_conv_wgrad_workspace(ctypes.byref(self._desc(name)), self._splits(name)))
        self.ws = t.zeros(ws // 4 + 1, dtype=t.float32, device=self.dev)
        P = B * self.res * self.res
        self.mse_ws = t.zeros(lib.mlbm_mse_workspace(P) // 8 + 1, dtype=t.float64, device=self.dev)
        self.loss = t.zeros(1, dtype=t.float32, device=self.dev)

    def _res_of(self, name):
        lvl = int(name[3]) if name != "head" else 0
        return self.res >> lvl

    def _desc(self, name, x_view=(None, 0), y_view=(None, 0), c_store=None):
        k, ci, co = self.shape_of[name]
        R = self._res_of(name)
        d = ConvDesc()
        d.n, d.h, d.w = self.batch, R, R
        d.c_in, d.c_out, d.ksize = ci, co, k
        d.x_stride = x_view[0] if x_view[0] else ci
        d.x_offset = x_view[1]
        d.y_stride = y_view[0] if y_view[0] else co
        d.y_offset = y_view[1]
        d.c_store = co if c_store is None else c_store
        return d

    def _splits(self, name):
        k, ci, co = self.shape_of[name]
        R = self._res_of(name)
        tiles = (co // 32) * (ci // 32) * k * k
        P = self.batch * R * R
        return int(max(1, min(P // 256, -(-2048 // tiles))))

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def refresh_weights(self):
        """bf16 forward and data-gradient copies of the FP32 master weights."""
        for name, k, ci, co in self.shapes:
            check(lib.mlbm_conv_weights(_p(self.w[name]), co, k, ci, _p(self.wf[name]), _p(self.wd[name]),
                                        self._stream()))

    def set_params(self, params):
        """Loads weights given as {name.w: (k, k, c_in, c_out), name.b: (c_out,)}
        (unpadded channels are zero-filled) and refreshes the bf16 copies."""
        t = self.torch
        for name, k, ci, co in self.shapes:
            w = np.asarray(params[name + ".w"], dtype=np.float32)
            full = np.zeros((co, k * k, ci), np.float32)
            kk, _, cin, cout = w.shape
            full[:cout, :, :cin] = np.transpose(w.reshape(k * k, cin, cout), (2, 0, 1))
            self.w[name] = t.from_numpy(full).to(self.dev)
            b = np.zeros(co, np.float32)
            b[:cout] = params[name + ".b"]
            self.b[name] = t.from_numpy(b).to(self.dev)
        self.refresh_weights()

    # ---- passes --------------------------------------------------------------------------
    def _conv(self, name, x, x_view, y, y_view, relu=True, y_f32=False, c_store=None):
        d = self._desc(name, x_view, y_view, c_store)
        check(lib.mlbm_conv_forward(ctypes.byref(d), _p(x), _p(self.wf[name]), _p(self.b[name]), _p(y),
                                    int(relu), int(y_f32), self._stream()))

    def forward(self, x):
        """x: int16-viewed bf16 (B, res, res, 32); returns the FP32 head output
        (B, res, res, 32) whose first c_out channels are the prediction."""
        A, C, L, B = self.A, self.channels, self.L, self.batch
        self.x = x
        h, hv = x, (PAD, 0)
        for lvl in range(L):
            R = self.res >> lvl
            c = C[lvl]
            self._conv(f"enc{lvl}a", h, hv, A[f"enc{lvl}a"], (c, 0))
            if lvl < L - 1:
                cat = A[f"cat{lvl}"]
                c_up = C[lvl + 1]
                self._conv(f"enc{lvl}b", A[f"enc{lvl}a"], (c, 0), cat, (c_up + c, c_up))
                check(lib.mlbm_pool_forward(B, R // 2, R // 2, c, _p(cat), c_up + c, c_up, _p(A[f"pool{lvl}"]),
                                            c, 0, self._stream()))
                h, hv = A[f"pool{lvl}"], (c, 0)
            else:
                self._conv(f"enc{lvl}b", A[f"enc{lvl}a"], (c, 0), A[f"enc{lvl}b"], (c, 0))
                h, hv = A[f"enc{lvl}b"], (c, 0)
        for lvl in range(L - 2, -1, -1):
            R = self.res >> lvl
            c = C[lvl]
            c_up = C[lvl + 1]
            cat = A[f"cat{lvl}"]
            check(lib.mlbm_upsample_forward(B, R // 2, R // 2, c_up, _p(h), hv[0], hv[1], _p(cat), c_up + c, 0,
                                            self._stream()))
            self._conv(f"dec{lvl}a", cat, (c_up + c, 0), A[f"dec{lvl}a"], (c, 0))
            self._conv(f"dec{lvl}b", A[f"dec{lvl}a"], (c, 0), A[f"dec{lvl}b"], (c, 0))
            h, hv = A[f"dec{lvl}b"], (c, 0)
        self._conv("head", h, hv, self.out, (PAD, 0), relu=False, y_f32=True)
        return self.out

    def loss_and_grad(self, target, mask):
        """Masked MSE of the first c_out output channels against target (FP32
        (B, res, res, c_out)) on mask (FP32 (B, res, res)); leaves the output
        gradient in self.dout.  Returns the loss as a device tensor."""
        P = self.batch * self.res * self.res
        cnt = float(mask.sum().item()) * self.c_out
        check(lib.mlbm_masked_mse(P, self.c_out, _p(self.out), PAD, _p(target), _p(mask), 1.0 / max(cnt, 1.0),
                                  _p(self.dout), _p(self.mse_ws), _p(self.loss), self._stream()))
        return self.loss

    def _wgrad(self, name, x, x_view, dy, dy_view):
        d = self._desc(name, x_view, dy_view)
        check(lib.mlbm_conv_wgrad(ctypes.byref(d), _p(x), _p(dy), _p(self.gw[name]), _p(self.gb[name]),
                                  self._splits(name), _p(self.ws), self._stream()))

    def _dgrad(self, name, dy, dy_view, dx, dx_view):
        k, ci, co = self.shape_of[name]
        R = self._res_of(name)
        d = ConvDesc()
        d.n, d.h, d.w = self.batch, R, R
        d.c_in, d.c_out, d.ksize = co, ci, k
        d.x_stride, d.x_offset = dy_view
        d.y_stride, d.y_offset = dx_view
        d.c_store = ci
        check(lib.mlbm_conv_forward(ctypes.byref(d), _p(dy), _p(self.wd[name]), None, _p(dx), 0, 0,
                                    self._stream()))

    def _relu_bwd(self, y, yv, dy, dyv, channels, R):
        P = self.batch * R * R
        check(lib.mlbm_relu_backward(P, channels, _p(y), yv[0], yv[1], _p(dy), dyv[0], dyv[1], self._stream()))

    def backward(self):
        """Weight and bias gradients (self.gw, self.gb) of the last forward pass
        for the output gradient in self.dout."""
        A, G, C, L, B = self.A, self.G, self.channels, self.L, self.batch
        c0 = C[0]
        self._wgrad("head", A["dec0b"], (c0, 0), self.dout, (PAD, 0))
        self._dgrad("head", self.dout, (PAD, 0), G["dec0b"], (c0, 0))
        for lvl in range(0, L - 1):
            R = self.res >> lvl
            c, c_up = C[lvl], C[lvl + 1]
            cc = c_up + c
            self._relu_bwd(A[f"dec{lvl}b"], (c, 0), G[f"dec{lvl}b"], (c, 0), c, R)
            self._wgrad(f"dec{lvl}b", A[f"dec{lvl}a"], (c, 0), G[f"dec{lvl}b"], (c, 0))
            self._dgrad(f"dec{lvl}b", G[f"dec{lvl}b"], (c, 0), G[f"dec{lvl}a"], (c, 0))
            self._relu_bwd(A[f"dec{lvl}a"], (c, 0), G[f"dec{lvl}a"], (c, 0), c, R)
            self._wgrad(f"dec{lvl}a", A[f"cat{lvl}"], (cc, 0), G[f"dec{lvl}a"], (c, 0))
            self._dgrad(f"dec{lvl}a", G[f"dec{lvl}a"], (c, 0), G[f"cat{lvl}"], (cc, 0))
            # gradient of this level's input: the decoder output of the level
            # below, or the bottleneck
            below = G[f"dec{lvl + 1}b"] if lvl + 1 <= L - 2 else G[f"enc{L - 1}b"]
            check(lib.mlbm_upsample_backward(B, R // 2, R // 2, c_up, _p(G[f"cat{lvl}"]), cc, 0, _p(below), c_up, 0,
                                             self._stream()))
        for lvl in range(L - 1, -1, -1):
            R = self.res >> lvl
            c = C[lvl]
            if lvl < L - 1:
                c_up = C[lvl + 1]
                cc = c_up + c
                # d(enc_b output) = pooled-path gradient + skip gradient; it lives in
                # the skip channels of the concatenation gradient buffer
                check(lib.mlbm_pool_backward(B, R // 2, R // 2, c, _p(G[f"pool{lvl}"]), c, 0, _p(G[f"cat{lvl}"]), cc,
                                             c_up, _p(G[f"cat{lvl}"]), cc, c_up, self._stream()))
                yb, ybv = A[f"cat{lvl}"], (cc, c_up)
                gb, gbv = G[f"cat{lvl}"], (cc, c_up)
            else:
                yb, ybv = A[f"enc{lvl}b"], (c, 0)
                gb, gbv = G[f"enc{lvl}b"], (c, 0)
            self._relu_bwd(yb, ybv, gb, gbv, c, R)
            self._wgrad(f"enc{lvl}b", A[f"enc{lvl}a"], (c, 0), gb, gbv)
            self._dgrad(f"enc{lvl}b", gb, gbv, G[f"enc{lvl}a"], (c, 0))
            self._relu_bwd(A[f"enc{lvl}a"], (c, 0), G[f"enc{lvl}a"], (c, 0), c, R)
            if lvl == 0:
                self._wgrad("enc0a", self.x, (PAD, 0), G["enc0a"], (c, 0))
            else:
                cb = C[lvl - 1]
                self._wgrad(f"enc{lvl}a", A[f"pool{lvl - 1}"], (cb, 0), G[f"enc{lvl}a"], (c, 0))
                self._dgrad(f"enc{lvl}a", G[f"enc{lvl}a"], (c, 0), G[f"pool{lvl - 1}"], (cb, 0))

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """One Adam step on every weight and bias, then refreshed bf16 copies.
        The padded input channels of the first layer and padded head outputs
        stay zero."""
        self.t += 1
        s = self._stream()
        for name, k, ci, co in self.shapes:
            if name == "enc0a":
                self.gw[name][:, :, 1:] = 0.0
            if name == "head":
                self.gw[name][self.c_out:] = 0.0
                self.gb[name][self.c_out:] = 0.0
            for p, g, key in ((self.w[name], self.gw[name], name + ".w"), (self.b[name], self.gb[name], name + ".b")):
                check(lib.mlbm_adam(p.numel(), _p(p), _p(g), _p(self.m[key]), _p(self.v[key]), float(lr),
                                    float(beta1), float(beta2), float(eps), self.t, s))
        self.refresh_weights()

    def state_dict(self):
        return {**{n + ".w": self.w[n].cpu().numpy() for n in self.w},
                **{n + ".b": self.b[n].cpu().numpy() for n in self.b}}


def to_bf16_bits(a):
    """float array -> int16 array of round-to-nearest-even bfloat16 bits."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16).view(np.int16)


def from_bf16_bits(a):
    u = np.asarray(a).view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)
