"""Warm-start network layers on the GPU against the float64 oracle.

Inputs and weights are bf16-representable, so every product is exact in fp32
and the kernels differ from the float64 oracle only by fp32 accumulation
order (<= 1e-5 relative) and, for bf16 outputs, by the final rounding
(one bf16 unit, 2^-8 relative).  Volumes are ragged (not multiples of the
4 x 4 x 8 tile) and batched.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import conv as oconv
from paper_2504_16446_amd import net

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
SHAPE = (2, 5, 7, 11)


def _bf16_bits(a):
    """float64 array (bf16-representable) -> int16 torch tensor of bf16 bit patterns."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32) >> 16
    return torch.from_numpy(u.astype(np.uint16).view(np.int16)).to(DEV)


def _from_bits(t):
    return net.bf16_to_float(t).cpu().numpy().astype(np.float64)


def _layer(ci, co, seed):
    rng = np.random.default_rng(seed)
    l = net.Conv3d(ci, co, DEV, rng)
    w = oracle.bf16(rng.standard_normal((27, ci, co)) * 0.2)
    b = rng.standard_normal(co)
    l.w.copy_(torch.tensor(w, dtype=torch.float32))
    l.b.copy_(torch.tensor(b, dtype=torch.float32))
    l.swizzle()
    return l, w.reshape(3, 3, 3, ci, co), b


@pytest.mark.parametrize("ci,co", [(32, 32), (32, 64), (64, 32), (64, 64)])
def test_conv_forward(ci, co):
    l, w, b = _layer(ci, co, ci + co)
    rng = np.random.default_rng(1)
    x = oracle.bf16(rng.standard_normal(SHAPE + (ci,)))
    xb = _bf16_bits(x)
    ref = oconv.conv3d(x, w, b)
    y32 = l.forward(xb, net.BIAS_F32).cpu().numpy()
    assert np.linalg.norm(y32 - ref) / np.linalg.norm(ref) <= 1e-5
    yr = _from_bits(l.forward(xb, net.RELU_BF16))
    refr = np.maximum(ref, 0)
    assert np.all(np.abs(yr - refr) <= 2.0 ** -8 * np.abs(refr) + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("ci,co", [(32, 64), (64, 64), (64, 32)])
def test_conv_input_gradient_with_relu_mask(ci, co):
    l, w, b = _layer(ci, co, 7 * ci + co)
    rng = np.random.default_rng(2)
    gy = oracle.bf16(rng.standard_normal(SHAPE + (co,)))
    mask = oracle.bf16(np.maximum(rng.standard_normal(SHAPE + (ci,)), 0))  # a ReLU output
    got = _from_bits(l.backward_input(_bf16_bits(gy), _bf16_bits(mask)))
    ref = oconv.conv3d_dgrad(gy, w) * (mask > 0)
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("ci,co", [(32, 32), (32, 64), (64, 32), (64, 64)])
def test_conv_weight_and_bias_gradient(ci, co):
    l, _, _ = _layer(ci, co, 3)
    rng = np.random.default_rng(3)
    x = oracle.bf16(rng.standard_normal(SHAPE + (ci,)))
    gy = oracle.bf16(rng.standard_normal(SHAPE + (co,)))
    work = torch.empty(1 << 22, device=DEV)
    l.backward_weights(_bf16_bits(x), _bf16_bits(gy), work)
    gw = l.gw.cpu().numpy().reshape(3, 3, 3, ci, co)
    ref = oconv.conv3d_wgrad(x, gy)
    assert np.linalg.norm(gw - ref) / np.linalg.norm(ref) <= 1e-5
    gb = l.gb.cpu().numpy()
    refb = gy.reshape(-1, co).sum(0)
    assert np.abs(gb - refb).max() <= 1e-5 * np.abs(gy).sum(axis=tuple(range(4))).max()


def test_adam_matches_oracle():
    rng = np.random.default_rng(4)
    l, _, _ = _layer(32, 32, 5)
    w0 = l.w.cpu().numpy().astype(np.float64).ravel()
    m = np.zeros_like(w0)
    v = np.zeros_like(w0)
    w = w0.copy()
    for t in range(1, 4):
        g = rng.standard_normal(w0.shape).astype(np.float32)
        l.gw.copy_(torch.tensor(g.reshape(l.gw.shape)))
        l.gb.zero_()
        l.adam(t, 1e-3)
        w, m, v = oconv.adam_step(w, g, m, v, t)
        got = l.w.cpu().numpy().astype(np.float64).ravel()
        assert np.abs(got - w).max() <= 1e-6


def test_mse_loss_and_gradient():
    rng = np.random.default_rng(6)
    nvox = 1000
    y = rng.standard_normal((nvox, 32)).astype(np.float32)
    t = rng.standard_normal((nvox, 28)).astype(np.float32)
    yt, tt = torch.tensor(y, device=DEV), torch.tensor(t, device=DEV)
    gy = net.bf16_empty((nvox, 32), DEV)
    loss = torch.empty(1, dtype=torch.float64, device=DEV)
    work = torch.empty(1024, dtype=torch.float64, device=DEV)
    from paper_2504_16446_amd._lib import call
    import ctypes as C
    s = torch.cuda.current_stream(DEV).cuda_stream
    call("tt_mse", C.c_void_p(yt.data_ptr()), C.c_void_p(tt.data_ptr()), nvox, 32, 28, 0.5,
         C.c_void_p(gy.data_ptr()), C.c_void_p(loss.data_ptr()), C.c_void_p(work.data_ptr()), 1024, C.c_void_p(s))
    d = y[:, :28].astype(np.float64) - t
    assert abs(loss.item() - (d * d).sum()) <= 1e-9 * (d * d).sum()
    g = _from_bits(gy)
    assert np.all(g[:, 28:] == 0)
    assert np.all(np.abs(g[:, :28] - 0.5 * d) <= 2.0 ** -8 * np.abs(0.5 * d) + 1e-7)


def test_network_training_reduces_loss():
    # composition check (training dynamics are not pinned): a few Adam steps on a fixed batch
    model = net.WarmStartNet(DEV, seed=0)
    rng = np.random.default_rng(8)
    x = torch.tensor(rng.standard_normal((2, 8, 8, 8, 28)).astype(np.float32), device=DEV)
    target = torch.tensor(rng.standard_normal((2, 8, 8, 8, 28)).astype(np.float32), device=DEV) * 0.1
    xb = model.prepare_input(x)
    losses = [float(model.train_step(xb, target, lr=1e-3).item()) for _ in range(30)]
    assert losses[-1] < 0.7 * losses[0], losses[::5]
    assert 380000 <= model.n_params() <= 381000
