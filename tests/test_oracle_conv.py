"""Pins of the network-layer oracle against library special cases (torch CPU, float64)."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import conv


def _torch_conv(x, w, b):
    # channels-last <-> torch's NCDHW; torch computes cross-correlation, as defined
    xt = torch.tensor(x).permute(0, 4, 1, 2, 3)
    wt = torch.tensor(w).permute(4, 3, 0, 1, 2)
    y = F.conv3d(xt, wt, torch.tensor(b), padding=1)
    return y.permute(0, 2, 3, 4, 1).numpy()


@pytest.mark.parametrize("shape,ci,co", [((2, 5, 6, 7), 3, 4), ((1, 4, 4, 4), 8, 5)])
def test_conv_forward_and_gradients_vs_torch(shape, ci, co):
    rng = np.random.default_rng(0)
    x = rng.standard_normal(shape + (ci,))
    w = rng.standard_normal((3, 3, 3, ci, co))
    b = rng.standard_normal(co)
    y = conv.conv3d(x, w, b)
    assert np.abs(y - _torch_conv(x, w, b)).max() < 1e-12
    gy = rng.standard_normal(y.shape)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    yt = F.conv3d(xt.permute(0, 4, 1, 2, 3), wt.permute(4, 3, 0, 1, 2), torch.tensor(b), padding=1)
    yt.permute(0, 2, 3, 4, 1).backward(torch.tensor(gy))
    assert np.abs(conv.conv3d_dgrad(gy, w) - xt.grad.numpy()).max() < 1e-11
    assert np.abs(conv.conv3d_wgrad(x, gy) - wt.grad.numpy()).max() < 1e-10


def test_adam_vs_torch():
    rng = np.random.default_rng(1)
    w0 = rng.standard_normal(50)
    wt = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        wt.grad = torch.tensor(g)
        opt.step()
        w, m, v = conv.adam_step(w, g, m, v, t)
        assert np.abs(w - wt.detach().numpy()).max() < 1e-12
