"""GPU parity of the regularisers and the gradient-descent driver against the FP64 oracle.

Laplacian and Huber terms: values and accumulated gradients on seeded
Gaussian fields (ragged sizes and the 100^3 / 45-coefficient volume),
rel-L2 <= 1e-6 (sums of at most 13 float32 products per element).  Gradient
descent with Nesterov momentum on the 32^3 workload with both regularisers:
the iterate after 10 steps and every objective value to 1e-5.
"""
import numpy as np
import pytest
import torch

import oracle
from helpers import gpu_projector, rel_l2
from oracle.regularizers import gradient_descent, huber_reg as o_huber, laplacian, laplacian_reg as o_lap
import tt_inputs as synth
from paper_2504_16446_amd import phantom
from paper_2504_16446_amd.projector import GradientDescent, huber_reg, laplacian_reg, sumsq

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("shape", [(7, 9, 5, 15), (1, 3, 2, 6), (3, 4, 300, 45), (5, 3, 70, 45), (100, 100, 100, 45),
                                   (37, 29, 41, 16), (6, 10, 64, 1)])
def test_laplacian_reg_parity(shape):
    rng = np.random.default_rng(21)
    c = rng.standard_normal(shape).astype(np.float32)
    g0 = rng.standard_normal(shape).astype(np.float32)
    lam = 0.37
    ct, gt = torch.from_numpy(c).to(DEV), torch.from_numpy(g0).to(DEV)
    val = torch.full((1,), 2.5, dtype=torch.float64, device=DEV)
    work = laplacian_reg(ct, lam, gt, val)
    v_ref, g_ref = o_lap(c.astype(np.float64), lam)
    assert rel_l2(work.cpu().numpy(), laplacian(c.astype(np.float64))) <= 1e-6
    assert rel_l2(gt.cpu().numpy() - g0, g_ref) <= 1e-6
    assert abs(float(val.item()) - 2.5 - v_ref) <= 1e-6 * v_ref  # Lap c is formed in float32


def test_huber_reg_parity():
    rng = np.random.default_rng(22)
    c = (0.5 * rng.standard_normal(12345)).astype(np.float32)
    g0 = rng.standard_normal(12345).astype(np.float32)
    ct, gt = torch.from_numpy(c).to(DEV), torch.from_numpy(g0).to(DEV)
    val = torch.zeros(1, dtype=torch.float64, device=DEV)
    huber_reg(ct, 0.3, 1.7, gt, val)
    v_ref, g_ref = o_huber(c.astype(np.float64), 0.3, 1.7)
    assert rel_l2(gt.cpu().numpy() - g0, g_ref) <= 1e-6
    assert abs(float(val.item()) - v_ref) <= 1e-6 * v_ref  # delta enters as float32


def test_gradient_descent_nesterov_parity():
    w = synth.WORKLOADS["c1"]
    og = oracle.Geometry.from_workload(w)
    c_true = phantom.coefficients(w).astype(np.float64)
    data = oracle.project(og, c_true).astype(np.float32).astype(np.float64)
    # step 1 / L with L bounded by power iteration on the oracle's normal operator
    rng = np.random.default_rng(23)
    v = rng.standard_normal(og.vol_shape)
    for _ in range(8):
        v = oracle.adjoint(og, oracle.project(og, v))
        nrm = np.linalg.norm(v)
        v /= nrm
    mu, lam, hub = 1e-3, 1e-2, (0.05, 1e-2)
    L = 2 * (1.05 * nrm + mu + 144 * lam) + hub[1] / hub[0]
    step = 1.0 / L
    c_ref, losses_ref = gradient_descent(og, np.zeros(og.vol_shape), data, step, 10, mu=mu, lam_lap=lam,
                                         huber=hub, nesterov=True)
    P = gpu_projector(og)
    c = torch.zeros(P.vol_shape, device=DEV)
    gd = GradientDescent(P, step, nesterov=True, lam_lap=lam, huber=hub)
    losses = gd.run(c, torch.from_numpy(data.astype(np.float32)).to(DEV), None, mu, 10).cpu().numpy()
    print("gd losses", losses[:3], losses[-1], "ref", losses_ref[-1])
    assert np.all(np.abs(losses - losses_ref) <= 1e-5 * np.abs(losses_ref))
    assert rel_l2(c.cpu().numpy(), c_ref) <= 1e-5
    assert losses[-1] < losses[0]


def test_gradient_descent_huber_loss_parity():
    """Robust data term: fixed-step descent on sum h(Ac - I) + mu |c|^2 with outliers in the data."""
    w = synth.WORKLOADS["c1"]
    og = oracle.Geometry.from_workload(w)
    c_true = phantom.coefficients(w).astype(np.float64)
    data = oracle.project(og, c_true)
    rng = np.random.default_rng(24)
    out = rng.random(data.shape) < 0.01
    data[out] += 50.0 * rng.standard_normal(int(out.sum()))
    data = data.astype(np.float32).astype(np.float64)
    v = rng.standard_normal(og.vol_shape)
    for _ in range(8):
        v = oracle.adjoint(og, oracle.project(og, v))
        nrm = np.linalg.norm(v)
        v /= nrm
    delta, mu = 0.5, 1e-3
    step = 1.0 / (1.05 * nrm / delta + 2 * mu)
    c_ref, losses_ref = gradient_descent(og, np.zeros(og.vol_shape), data, step, 8, mu=mu, loss_delta=delta)
    P = gpu_projector(og)
    c = torch.zeros(P.vol_shape, device=DEV)
    gd = GradientDescent(P, step, loss_delta=delta)
    losses = gd.run(c, torch.from_numpy(data.astype(np.float32)).to(DEV), None, mu, 8).cpu().numpy()
    print("huber-loss gd", losses[0], losses[-1], "ref", losses_ref[-1])
    assert np.all(np.abs(losses - losses_ref) <= 1e-5 * np.abs(losses_ref))
    assert rel_l2(c.cpu().numpy(), c_ref) <= 1e-5
    assert losses[-1] < losses[0]


def test_preconditioned_descent_parity():
    """Diagonal voxel preconditioner 1 / (A^T A u)_{v,0}: the helper against the
    oracle's construction, then 8 preconditioned Nesterov steps."""
    w = synth.WORKLOADS["c1"]
    og = oracle.Geometry.from_workload(w)
    u = np.zeros(og.vol_shape)
    u[..., 0] = 1.0
    dref = oracle.adjoint(og, oracle.project(og, u))[..., :1]
    dref = np.maximum(dref, 1e-6 * dref.max())
    p_ref = np.broadcast_to(1.0 / dref, og.vol_shape).copy()
    P = gpu_projector(og)
    p_gpu = GradientDescent.voxel_preconditioner(P)
    assert rel_l2(p_gpu.cpu().numpy(), p_ref) <= 1e-5
    c_true = phantom.coefficients(w).astype(np.float64)
    data = oracle.project(og, c_true).astype(np.float32).astype(np.float64)
    mu = 1e-3
    step = 0.4  # the preconditioned normal operator has unit scale on the support
    c_ref, losses_ref = gradient_descent(og, np.zeros(og.vol_shape), data, step, 8, mu=mu, nesterov=True,
                                         precond=p_ref.astype(np.float32).astype(np.float64))
    c = torch.zeros(P.vol_shape, device=DEV)
    gd = GradientDescent(P, step, nesterov=True, precond=torch.from_numpy(p_ref.astype(np.float32)).to(DEV))
    losses = gd.run(c, torch.from_numpy(data.astype(np.float32)).to(DEV), None, mu, 8).cpu().numpy()
    print("preconditioned gd", losses[0], losses[-1], "ref", losses_ref[-1])
    assert np.all(np.abs(losses - losses_ref) <= 1e-5 * np.abs(losses_ref))
    assert rel_l2(c.cpu().numpy(), c_ref) <= 1e-5
    assert losses[-1] < losses[0]


def test_regulariser_values_repeat_bit_for_bit():
    # fixed-order float64 partial sums: the same inputs give the same value every time
    rng = np.random.default_rng(31)
    ct = torch.tensor(rng.standard_normal((37, 29, 41, 15)).astype(np.float32), device=DEV)
    vals = []
    for _ in range(3):
        val = torch.zeros(1, dtype=torch.float64, device=DEV)
        g = torch.zeros_like(ct)
        laplacian_reg(ct, 0.3, g, val)
        huber_reg(ct, 0.2, 1.1, g, val)
        sumsq(ct, val, 0.7)
        vals.append(float(val.item()))
    assert vals[0] == vals[1] == vals[2]
