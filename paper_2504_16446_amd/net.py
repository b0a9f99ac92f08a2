"""Warm-start network: thin wrappers over the library's layer kernels.

The network maps the normalised backprojection of the data (the ell <= 6
coefficient channels, 28) to initial SH coefficients (28 channels):
six 3x3x3 convolutions 28 -> 32 -> 64 -> 64 -> 64 -> 32 -> 28 with ReLU after
the first five, 'same' zero padding, channels padded to 32 on the device.
Activations are bf16 (stored as int16 bit patterns in torch tensors), the
convolutions run on bf16 MFMA with fp32 accumulation, master weights and Adam
state are fp32.  Every layer operation is a call into libtt_hip.so.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

from ._lib import call, lib

RELU_BF16, BIAS_F32, MASK_BF16 = 0, 1, 2
CHANNELS = [28, 32, 64, 64, 64, 32, 28]  # real channel counts of the layer boundaries


def _pad(c):
    return 32 if c <= 32 else 64


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(dev):
    return C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def bf16_empty(shape, device):
    return torch.empty(shape, dtype=torch.int16, device=device)


def pack_bf16(x: torch.Tensor, cpad: int, shift=None, scale=None, pre=1.0) -> torch.Tensor:
    """float32 [..., cin] -> bf16 bits [..., cpad] of (pre x - shift) * scale."""
    assert x.dtype == torch.float32 and x.is_contiguous()
    cin = x.shape[-1]
    nvox = x.numel() // cin
    out = bf16_empty(x.shape[:-1] + (cpad,), x.device)
    call("tt_pack_bf16", _p(x), nvox, cin, cpad, float(pre), _p(shift), _p(scale), _p(out), _stream(x.device))
    return out


def bf16_to_float(t: torch.Tensor) -> torch.Tensor:
    """Reinterpret bf16 bit patterns as float32 values (for checks and metrics)."""
    return (t.to(torch.int32) << 16).view(torch.float32)


class Conv3d:
    """One 3x3x3 layer with fp32 master weights w[27][ci][co], bias[co], Adam state."""

    def __init__(self, ci, co, device, rng, ci_real=None, co_real=None):
        self.ci, self.co = ci, co
        self.device = device
        ci_real = ci if ci_real is None else ci_real
        co_real = co if co_real is None else co_real
        std = math.sqrt(2.0 / (27 * ci_real))
        w = np.zeros((27, ci, co), np.float32)
        w[:, :ci_real, :co_real] = rng.standard_normal((27, ci_real, co_real)) * std
        self.w = torch.from_numpy(w).to(device)
        self.b = torch.zeros(co, device=device)
        n = call("tt_conv3d_weight_elems", ci, co)
        self.wf = bf16_empty((n,), device)
        self.wd = bf16_empty((n,), device)
        self.gw = torch.zeros_like(self.w)
        self.gb = torch.zeros_like(self.b)
        self.state = [torch.zeros_like(self.w), torch.zeros_like(self.w), torch.zeros_like(self.b),
                      torch.zeros_like(self.b)]
        self.swizzle()

    def swizzle(self):
        call("tt_conv3d_swizzle", _p(self.w), self.ci, self.co, _p(self.wf), _p(self.wd), _stream(self.device))

    def forward(self, x, epi, out=None):
        n, X, Y, Z, ci = x.shape
        assert ci == self.ci and x.dtype == torch.int16 and x.is_contiguous()
        if out is None:
            out = (torch.empty((n, X, Y, Z, self.co), device=self.device) if epi == BIAS_F32
                   else bf16_empty((n, X, Y, Z, self.co), self.device))
        call("tt_conv3d", epi, self.ci, self.co, _p(x), _p(self.wf), _p(self.b), None, _p(out), n, X, Y, Z,
             _stream(self.device))
        return out

    def backward_input(self, gy, mask):
        """Gradient w.r.t. this layer's input, zeroed where the input (a ReLU output) is 0."""
        n, X, Y, Z, co = gy.shape
        out = bf16_empty((n, X, Y, Z, self.ci), self.device)
        call("tt_conv3d", MASK_BF16, self.co, self.ci, _p(gy), _p(self.wd), None, _p(mask), _p(out), n, X, Y, Z,
             _stream(self.device))
        return out

    def backward_weights(self, x, gy, work):
        n, X, Y, Z, _ = x.shape
        need = lib().tt_conv3d_wgrad_work_bytes(self.ci, self.co, n, X, Y, Z)
        assert work.numel() * 4 >= need
        call("tt_conv3d_wgrad", self.ci, self.co, _p(x), _p(gy), n, X, Y, Z, _p(work), work.numel() * 4,
             _p(self.gw), _p(self.gb), _stream(self.device))

    def adam(self, t, lr):
        m, v, mb, vb = self.state
        call("tt_adam", _p(self.w), _p(self.gw), _p(m), _p(v), self.w.numel(), t, lr, 0.9, 0.999, 1e-8,
             _stream(self.device))
        call("tt_adam", _p(self.b), _p(self.gb), _p(mb), _p(vb), self.b.numel(), t, lr, 0.9, 0.999, 1e-8,
             _stream(self.device))
        self.swizzle()


class WarmStartNet:
    """The six-layer network; input/target channel statistics travel with the weights."""

    def __init__(self, device, seed=0):
        self.device = torch.device(device)
        rng = np.random.default_rng(seed)
        self.layers = []
        for i in range(6):
            ci_r, co_r = CHANNELS[i], CHANNELS[i + 1]
            self.layers.append(Conv3d(_pad(ci_r), _pad(co_r), self.device, rng, ci_r, co_r))
        self.in_shift = torch.zeros(CHANNELS[0], device=self.device)
        self.in_scale = torch.ones(CHANNELS[0], device=self.device)
        self.t = 0
        self._work = None
        self._loss_work = torch.empty(1024, dtype=torch.float64, device=self.device)

    def n_params(self):
        return sum(int((l.w != 0).sum()) for l in self.layers) + sum(l.b.numel() for l in self.layers) - 4

    def prepare_input(self, x28: torch.Tensor, pre=1.0) -> torch.Tensor:
        """float32 [..., 28] backprojection (scaled by pre = 1 / kappa) -> standardised bf16 [..., 32]."""
        return pack_bf16(x28.contiguous(), 32, self.in_shift, self.in_scale, pre)

    def set_input_statistics(self, x28: torch.Tensor, pre=1.0):
        """Standardisation from the channel means and standard deviations of pre * x28."""
        nvox = x28.numel() // CHANNELS[0]
        work = torch.empty(int(lib().tt_channel_stats_work_len()), dtype=torch.float64, device=self.device)
        call("tt_channel_stats", _p(x28), nvox, CHANNELS[0], CHANNELS[0], float(pre), _p(self.in_shift),
             _p(self.in_scale), _p(work), work.numel(), _stream(self.device))

    def forward(self, xb: torch.Tensor, keep=False):
        acts = [xb]
        h = xb
        for i, l in enumerate(self.layers):
            h = l.forward(h, BIAS_F32 if i == 5 else RELU_BF16)
            acts.append(h)
        return (h, acts) if keep else h

    def _ensure_work(self, n, X, Y, Z):
        need = max(lib().tt_conv3d_wgrad_work_bytes(l.ci, l.co, n, X, Y, Z) for l in self.layers)
        if self._work is None or self._work.numel() * 4 < need:
            self._work = torch.empty((need + 3) // 4, device=self.device)
        return self._work

    def train_step(self, xb, target28, lr=1e-3):
        """One Adam step on the MSE between the output's 28 channels and target28 (float32)."""
        n, X, Y, Z, _ = xb.shape
        y, acts = self.forward(xb, keep=True)
        nvox = n * X * Y * Z
        gy = bf16_empty((n, X, Y, Z, 32), self.device)
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        scale = 2.0 / (nvox * CHANNELS[-1])
        call("tt_mse", _p(y), _p(target28), nvox, 32, CHANNELS[-1], scale, _p(gy), _p(loss), _p(self._loss_work),
             1024, _stream(self.device))
        work = self._ensure_work(n, X, Y, Z)
        for i in range(5, -1, -1):
            l = self.layers[i]
            l.backward_weights(acts[i], gy, work)
            if i > 0:
                gy = l.backward_input(gy, acts[i])
        self.t += 1
        for l in self.layers:
            l.adam(self.t, lr)
        return loss  # sum of squared errors (device float64)

    def state_dict(self):
        d = {f"w{i}": l.w.cpu() for i, l in enumerate(self.layers)}
        d.update({f"b{i}": l.b.cpu() for i, l in enumerate(self.layers)})
        d["in_shift"], d["in_scale"] = self.in_shift.cpu(), self.in_scale.cpu()
        return d

    def load_state_dict(self, d):
        for i, l in enumerate(self.layers):
            l.w.copy_(d[f"w{i}"].to(self.device))
            l.b.copy_(d[f"b{i}"].to(self.device))
            l.swizzle()
        self.in_shift.copy_(d["in_shift"].to(self.device))
        self.in_scale.copy_(d["in_scale"].to(self.device))


def layer_flops(n_vox):
    """Multiply-add flops of the forward of every layer at the padded channel counts the
    kernels run (2 x 27 x ci x co per voxel)."""
    return [2.0 * 27 * _pad(CHANNELS[i]) * _pad(CHANNELS[i + 1]) * n_vox for i in range(6)]


def bench(device="cuda:0", batch=8, T=48, reps=5):
    """Event-timed forward, input-gradient and weight-gradient launches of every layer and
    the whole training step at batch x T^3 voxels, with the flops of each at the padded
    channel counts (TFLOP/s against the bf16 dense MFMA peak of 2500 TFLOP/s)."""
    dev = torch.device(device)
    model = WarmStartNet(dev, seed=0)
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    x = pack_bf16(torch.randn((batch, T, T, T, CHANNELS[0]), device=dev, generator=g), 32)
    target = torch.randn((batch, T, T, T, CHANNELS[-1]), device=dev, generator=g)
    st = torch.cuda.current_stream(dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        a, b = ev(), ev()
        torch.cuda.synchronize()
        a.record(st)
        for _ in range(reps):
            fn()
        b.record(st)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    y, acts = model.forward(x, keep=True)
    work = model._ensure_work(batch, T, T, T)
    flops = layer_flops(batch * T ** 3)
    rows = []
    for i, l in enumerate(model.layers):
        epi = BIAS_F32 if i == 5 else RELU_BF16
        gy = bf16_empty((batch, T, T, T, l.co), dev)
        gy.copy_(pack_bf16(torch.randn((batch, T, T, T, l.co), device=dev, generator=g), l.co))
        f_ms = timed(lambda: l.forward(acts[i], epi))
        d_ms = timed(lambda: l.backward_input(gy, acts[i])) if i > 0 else None
        w_ms = timed(lambda: l.backward_weights(acts[i], gy, work))
        rows.append({"layer": i, "ci": l.ci, "co": l.co, "forward_ms": f_ms, "forward_TFLOPs": flops[i] / f_ms / 1e9,
                     "dgrad_ms": d_ms, "dgrad_TFLOPs": flops[i] / d_ms / 1e9 if d_ms else None,
                     "wgrad_ms": w_ms, "wgrad_TFLOPs": flops[i] / w_ms / 1e9})
    step_ms = timed(lambda: model.train_step(x, target))
    total = 3 * sum(flops) - flops[0]  # no input gradient for the first layer
    return {"batch": batch, "tile": T, "layers": rows, "train_step_ms": step_ms,
            "train_step_TFLOPs": total / step_ms / 1e9, "peak_TFLOPs": 2500.0,
            "frac": total / step_ms / 1e9 / 2500.0}


if __name__ == "__main__":
    import json
    import sys
    print(json.dumps(bench(reps=int(sys.argv[1]) if len(sys.argv) > 1 else 5)))
