"""The allocation-free loss/gradient entry point (tt_loss_grad_noalloc) against
tt_loss_grad with an attached workspace, through the C ABI.

Both run the same kernels on the same inputs, so the loss, gradient and
residual must agree exactly; the forward batch differs (the static scratch
holds fewer mapped volumes than the workspace), which changes nothing per
projection.  Two calls in a row, the second on a smaller problem, so that the
second reuses scratch the first left behind; then a problem too large for the
scratch must be refused without touching the device.
"""
import ctypes as C

import pytest
import torch

from geoms import small, workload
from helpers import gpu_projector

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _noalloc(P, c, data, w, mu, want_resid):
    from paper_2504_16446_amd._lib import call
    loss = torch.full((1,), float("nan"), dtype=torch.float64, device=DEV)
    grad = torch.full(P.vol_shape, float("nan"), dtype=torch.float32, device=DEV)
    resid = torch.full(P.data_shape, float("nan"), dtype=torch.float32, device=DEV) if want_resid else None
    P._bind_stream()
    call("tt_loss_grad_noalloc", P._h, _ptr(c), _ptr(data), _ptr(w), float(mu), _ptr(loss), _ptr(grad),
         _ptr(resid))
    return loss, grad, resid


def _inputs(P, seed, weights):
    gen = torch.Generator(device=DEV)
    gen.manual_seed(seed)
    c = torch.randn(P.vol_shape, device=DEV, generator=gen)
    data = torch.randn(P.data_shape, device=DEV, generator=gen)
    w = torch.rand(P.data_shape, device=DEV, generator=gen) + 0.5 if weights else None
    return c, data, w


def _check(P, seed, weights, mu):
    c, data, w = _inputs(P, seed, weights)
    ref_loss, ref_grad, ref_resid = P.loss_grad(c, data, w, mu)
    for want_resid in (True, False):
        loss, grad, resid = _noalloc(P, c, data, w, mu, want_resid)
        torch.cuda.synchronize()
        assert torch.equal(grad, ref_grad), float((grad - ref_grad).abs().max())
        assert float(loss.item()) == float(ref_loss.item()), (loss.item(), ref_loss.item())
        if want_resid:
            assert torch.equal(resid, ref_resid), float((resid - ref_resid).abs().max())


def test_noalloc_matches_workspace_entry_point_twice():
    torch.cuda.set_device(DEV)
    # first call: 100^3 / ell_max 8 / 240 projections of 100x100 x 8 segments,
    # several forward batches in the static scratch (the workspace of the
    # reference is sized for batches of 16 projections)
    og = workload("c2")
    P1 = gpu_projector(og, forward_batch=16)
    _check(P1, 11, weights=True, mu=1e-3)
    del P1
    # second call, smaller problem: the scratch still holds the first call's data
    P2 = gpu_projector(small(ell_max=4))
    _check(P2, 12, weights=False, mu=0.0)


def test_noalloc_rejects_problems_above_the_scratch_limit():
    from paper_2504_16446_amd._lib import TTError
    torch.cuda.set_device(DEV)
    # 128^3 / 300 projections of 128x128 x 16 segments: the folded residual
    # plus the two mapped volumes of the smallest batch exceed
    # TT_NOALLOC_SCRATCH_BYTES
    og = workload("c3")
    P = gpu_projector(og, forward_batch=1)
    c = torch.zeros(P.vol_shape, device=DEV)
    data = torch.zeros(P.data_shape, device=DEV)
    with pytest.raises(TTError) as e:
        _noalloc(P, c, data, None, 0.0, True)
    assert e.value.code == -3 and "static limit" in str(e.value)


def test_noalloc_is_independent_of_the_attached_workspace():
    # the static path never reads the context's workspace: with the smallest
    # valid workspace (one map tile of projections per batch) the results agree
    torch.cuda.set_device(DEV)
    og = small(ell_max=6)
    P = gpu_projector(og, forward_batch=1)
    assert P.batch == 4  # one 16-row map tile: 4 projections x 4 unique segments
    _check(P, 13, weights=True, mu=0.5)


@pytest.mark.parametrize("k", [1, 6])
def test_noalloc_with_the_sparse_fused_forward(k):
    """With a sparse map the scratch holds no mapped volumes, and for k = 1 the
    channel-major copy of c (at most 32 kept channels per projection; k = 6
    keeps 29-41 of the 91 and stages from the coefficient records); the
    results equal the workspace entry point's bit for bit."""
    torch.cuda.set_device(DEV)
    P = gpu_projector(small(ell_max=12, n_seg=16), sparse_k=k)
    assert P.batch == 0
    _check(P, 13 + k, weights=True, mu=1e-3)
