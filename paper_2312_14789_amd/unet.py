"""The warm-start network: an encoder-decoder with skip connections run by the
library (include/mlbm_unet.h: mlbm_unet_forward, _loss, _backward, _adam).

This module only allocates the device buffers (PyTorch) that mlbm_unet_sizes
asks for, initialises the parameters and calls the entry points; every
convolution, pooling, upsampling, loss and optimizer step, and the order in
which the backward pass visits them, is the library's.  Layout: NHWC bfloat16
activations, one FP32 parameter array (per layer the weights
[c_out][k*k][c_in], then the bias), bf16 copies of the weights for the forward
pass and the data gradient.

Shape: per encoder level two 3x3 convolutions with ReLU (average pooling
between levels), per decoder level a nearest upsampling, a concatenation with
the encoder output of that level and two 3x3 convolutions with ReLU, then a
1x1 head.  The input is padded to 32 channels and the head to 32 output
channels, of which the first `c_out` are stored.
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import UNetBuffers, UNetDesc, UNetLayerInfo, check, lib

PAD = 32


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class UNet:
    def __init__(self, channels=(32, 64, 128, 256, 256), res=256, batch=16, c_in=1, c_out=3, seed=0, device="cuda"):
        import torch

        self.torch = torch
        self.channels = list(channels)
        self.res, self.batch, self.c_in, self.c_out = res, batch, c_in, c_out
        self.L = len(channels)
        self.dev = torch.device(device)
        self.desc = UNetDesc()
        d = self.desc
        d.levels = self.L
        for i, c in enumerate(self.channels):
            d.channels[i] = c
        d.batch, d.res, d.c_in, d.c_out = batch, res, c_in, c_out
        sz = UNetBuffers()
        check(lib.mlbm_unet_sizes(ctypes.byref(d), ctypes.byref(sz)))
        self.n_params = int(sz.n_params)
        self.layers = []
        for i in range(sz.n_layers):
            li = UNetLayerInfo()
            check(lib.mlbm_unet_layer(ctypes.byref(d), i, ctypes.byref(li)))
            self.layers.append((li.name.decode(), li.ksize, li.c_in, li.c_out, int(li.w_offset), int(li.b_offset)))
        self.shapes = [(nm, k, ci, co) for nm, k, ci, co, _, _ in self.layers]
        f32 = torch.float32
        self.params = torch.zeros(self.n_params, dtype=f32, device=self.dev)
        self.grads = torch.zeros(self.n_params, dtype=f32, device=self.dev)
        self.m = torch.zeros(self.n_params, dtype=f32, device=self.dev)
        self.v = torch.zeros(self.n_params, dtype=f32, device=self.dev)
        u8 = torch.uint8
        self.w_bf16 = torch.zeros(int(sz.w_bf16_bytes), dtype=u8, device=self.dev)
        self.act = torch.zeros(int(sz.act_bytes), dtype=u8, device=self.dev)
        self.act_grad = torch.zeros(int(sz.act_bytes), dtype=u8, device=self.dev)
        self.work = torch.zeros(int(sz.work_bytes), dtype=u8, device=self.dev)
        self.out = torch.zeros((batch, res, res, c_out), dtype=f32, device=self.dev)
        self.loss = torch.zeros(1, dtype=f32, device=self.dev)
        d.params, d.grads, d.adam_m, d.adam_v = (self.params.data_ptr(), self.grads.data_ptr(), self.m.data_ptr(),
                                                 self.v.data_ptr())
        d.w_bf16, d.act, d.act_grad, d.work = (self.w_bf16.data_ptr(), self.act.data_ptr(), self.act_grad.data_ptr(),
                                               self.work.data_ptr())
        # views of the parameter and gradient arrays per layer
        self.w, self.b, self.gw, self.gb = {}, {}, {}, {}
        for nm, k, ci, co, wo, bo in self.layers:
            self.w[nm] = self.params[wo:wo + co * k * k * ci].view(co, k * k, ci)
            self.b[nm] = self.params[bo:bo + co]
            self.gw[nm] = self.grads[wo:wo + co * k * k * ci].view(co, k * k, ci)
            self.gb[nm] = self.grads[bo:bo + co]
        # He initialisation; the padded input channels and head outputs start at zero
        rng = np.random.default_rng(seed)
        host = np.zeros(self.n_params, np.float32)
        for nm, k, ci, co, wo, bo in self.layers:
            fan = k * k * (c_in if nm == "enc0a" else ci)
            w = rng.normal(0.0, np.sqrt(2.0 / fan), size=(co, k * k, ci)).astype(np.float32)
            if nm == "enc0a":
                w[:, :, c_in:] = 0.0
            if nm == "head":
                w[c_out:] = 0.0
            host[wo:wo + w.size] = w.ravel()
        self.params.copy_(torch.from_numpy(host))
        self.refresh_weights()
        self.t = 0
        self.x = None

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream().cuda_stream)

    def refresh_weights(self):
        """mlbm_unet_refresh: bf16 copies of the FP32 parameters."""
        check(lib.mlbm_unet_refresh(ctypes.byref(self.desc), self._stream()))

    def set_params(self, params):
        """Loads weights given as {name.w: (k, k, c_in, c_out), name.b: (c_out,)}
        (unpadded channels are zero-filled) and refreshes the bf16 copies."""
        host = np.zeros(self.n_params, np.float32)
        for nm, k, ci, co, wo, bo in self.layers:
            w = np.asarray(params[nm + ".w"], dtype=np.float32)
            full = np.zeros((co, k * k, ci), np.float32)
            kk, _, cin, cout = w.shape
            full[:cout, :, :cin] = np.transpose(w.reshape(k * k, cin, cout), (2, 0, 1))
            host[wo:wo + full.size] = full.ravel()
            b = np.zeros(co, np.float32)
            b[:cout] = params[nm + ".b"]
            host[bo:bo + co] = b
        self.params.copy_(self.torch.from_numpy(host))
        self.refresh_weights()

    def forward(self, x):
        """mlbm_unet_forward of x (int16-viewed bf16 (B, res, res, 32)); returns
        the FP32 head output (B, res, res, c_out), the prediction."""
        self.x = x.contiguous()
        check(lib.mlbm_unet_forward(ctypes.byref(self.desc), _p(self.x), _p(self.out), self._stream()))
        return self.out

    def loss_and_grad(self, target, mask):
        """mlbm_unet_loss: masked MSE of the first c_out output channels against
        target (FP32 (B, res, res, c_out)) on mask (FP32 (B, res, res)); the
        output gradient stays in the library's buffers.  Returns the loss as a
        device tensor."""
        check(lib.mlbm_unet_loss(ctypes.byref(self.desc), _p(self.out), _p(target.contiguous()),
                                 _p(mask.contiguous()), _p(self.loss), self._stream()))
        return self.loss

    def backward(self):
        """mlbm_unet_backward: every weight and bias gradient (self.gw, self.gb)
        of the last forward pass and loss."""
        check(lib.mlbm_unet_backward(ctypes.byref(self.desc), _p(self.x), self._stream()))

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        """mlbm_unet_adam: one Adam step on every parameter (padded input
        channels and head outputs stay zero), then refreshed bf16 copies."""
        self.t += 1
        check(lib.mlbm_unet_adam(ctypes.byref(self.desc), float(lr), float(beta1), float(beta2), float(eps), self.t,
                                 self._stream()))

    def state_dict(self):
        return {**{n + ".w": self.w[n].cpu().numpy() for n in self.w},
                **{n + ".b": self.b[n].cpu().numpy() for n in self.b}}

    def load_state(self, state):
        """Loads a state_dict (weights [c_out][k*k][c_in], biases)."""
        host = np.zeros(self.n_params, np.float32)
        for nm, k, ci, co, wo, bo in self.layers:
            host[wo:wo + co * k * k * ci] = np.asarray(state[nm + ".w"], np.float32).ravel()
            host[bo:bo + co] = np.asarray(state[nm + ".b"], np.float32)
        self.params.copy_(self.torch.from_numpy(host))
        self.refresh_weights()


def to_bf16_bits(a):
    """float array -> int16 array of round-to-nearest-even bfloat16 bits."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16).view(np.int16)


def from_bf16_bits(a):
    u = np.asarray(a).view(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32)
