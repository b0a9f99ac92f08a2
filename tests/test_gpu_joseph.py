"""GPU parity of the Joseph-method projector (TT_PROJ_JOSEPH) against the FP64 oracle.

Same bar as the trilinear parity tests: relative L2 <= 1e-5 per output tensor
and the largest element error <= 1e-4 of the largest element, on seeded
Gaussian inputs; at the full workload sizes, sampled rays and voxels and the
adjoint identity over the whole operator.
"""
import numpy as np
import pytest
import torch

import oracle
from geoms import degenerate, small, steep, tilted_angles
from helpers import gpu_projector, rel_l2, rel_max
import tt_inputs as synth
from paper_2504_16446_amd import phantom
from paper_2504_16446_amd.projector import LBFGS, Projector

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


def _t(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device=DEV)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _jos(og):
    """The same geometry with the Joseph model."""
    return oracle.Geometry(og.n, og.ell_max, og.inner, og.outer, og.nj, og.nk, og.n_seg, og.frame,
                           n_sub=og.n_sub, step=og.step, seg_span=og.seg_span, joff=og.joff, koff=og.koff,
                           model="joseph")


def _tiny_offsets():
    inner, outer = tilted_angles(3, (0.0, 33.0))
    return oracle.Geometry((6, 7, 8), 2, inner, outer, 9, 10, 8, synth.lab_frame(),
                           joff=np.linspace(-0.4, 0.3, 6), koff=np.linspace(0.25, -0.35, 6), model="joseph")


def _axis_ties():
    # rotation 0 / 90 / 180 deg at tilt 45: |d_y| = |d_z| or |d_x| = |d_z| (ties go to the lower axis)
    inner = np.deg2rad([0.0, 90.0, 180.0, 270.0, 45.0, 135.0])
    outer = np.deg2rad([45.0, 45.0, 45.0, 45.0, 0.0, 0.0])
    return oracle.Geometry((10, 9, 11), 4, inner, outer, 14, 13, 8, synth.lab_frame(), model="joseph")


CASES = {
    "tiny_offsets": _tiny_offsets,
    "axis_ties": _axis_ties,
    "small_l4": lambda: _jos(small(ell_max=4)),
    "small_l8_seg16": lambda: _jos(small(ell_max=8, n_seg=16)),
    "small_l8_seg32": lambda: _jos(small(ell_max=8, n_seg=32)),   # sixteen unique segments
    "half_circle": lambda: oracle.Geometry((9, 11, 10), 2, *tilted_angles(3, (0.0, 33.0)), 12, 10, 6,
                                           synth.lab_frame(), seg_span=np.pi, model="joseph"),
    "steep_tilts": lambda: steep(model="joseph"),
    "degenerate": lambda: degenerate(model="joseph"),
    "c1": lambda: oracle.Geometry.from_workload(synth.WORKLOADS["c1"], model="joseph"),
}


def _inputs(og, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(og.vol_shape).astype(np.float32).astype(np.float64)
    y = rng.standard_normal(og.data_shape).astype(np.float32).astype(np.float64)
    return c, y


@pytest.mark.parametrize("name", list(CASES))
def test_joseph_forward_adjoint_parity(name):
    og = CASES[name]()
    c, y = _inputs(og, 11)
    P = gpu_projector(og, model="joseph")
    got_f = _np(P.forward(_t(c)))
    got_a = _np(P.adjoint(_t(y)))
    ref_f = oracle.project(og, c)
    ref_a = oracle.adjoint(og, y)
    print(name, "joseph forward", rel_l2(got_f, ref_f), "adjoint", rel_l2(got_a, ref_a))
    assert rel_l2(got_f, ref_f) <= TOL and rel_max(got_f, ref_f) <= 10 * TOL
    assert rel_l2(got_a, ref_a) <= TOL and rel_max(got_a, ref_a) <= 10 * TOL


def test_joseph_loss_grad_and_switch_back():
    og = _jos(small(ell_max=4))
    c, data = _inputs(og, 12)
    mu = 1e-3
    loss, grad, resid = oracle.loss_grad(og, c, data, None, mu)
    P = gpu_projector(og, model="joseph")
    l_g, g_g, r_g = P.loss_grad(_t(c), _t(data), None, mu)
    assert abs(float(l_g.item()) - loss) <= TOL * loss
    assert rel_l2(_np(g_g), grad) <= TOL and rel_l2(_np(r_g), resid) <= TOL
    # a trilinear projector of the same geometry is unaffected
    ot = small(ell_max=4)
    T = gpu_projector(ot)
    assert rel_l2(_np(T.forward(_t(c))), oracle.project(ot, c)) <= TOL


def test_joseph_lbfgs_iterates():
    og = oracle.Geometry.from_workload(synth.WORKLOADS["c1"], model="joseph")
    w = synth.WORKLOADS["c1"]
    c_true = phantom.coefficients(w).astype(np.float64)
    data = oracle.project(og, c_true)
    data += 0.01 * np.abs(data).max() * np.random.default_rng(5).standard_normal(data.shape)
    data = data.astype(np.float32).astype(np.float64)
    c_ref, it, hist, rel = oracle.lbfgs(og, np.zeros(og.vol_shape), data, mu=1e-3, m=10, max_iter=10)
    P = gpu_projector(og, model="joseph")
    c = torch.zeros(P.vol_shape, device=DEV)
    s = LBFGS(P, m=10)
    s.init(c, _t(data), None, 1e-3)
    for _ in range(10):
        s.step()
    err = rel_l2(_np(c), c_ref)
    print("joseph lbfgs c rel-L2 after 10 iterations", err)
    assert err <= 1e-4


@pytest.mark.parametrize("name", ["c2", "c5"])
def test_joseph_full_size_sampled(name):
    w = synth.WORKLOADS[name]
    print(f"[joseph fullsize] {name}: {w.n} ell_max {w.ell_max} S={w.n_proj}", flush=True)
    P = Projector.from_workload(w, device=DEV, model="joseph")
    og = oracle.Geometry.from_workload(w, model="joseph")
    rng = np.random.default_rng(78)
    c = rng.standard_normal(P.vol_shape, dtype=np.float32)
    ct = torch.from_numpy(c).to(DEV)
    I = P.forward(ct).cpu().numpy()
    sjk = np.stack([rng.integers(0, w.n_proj, 192), rng.integers(0, w.nj, 192), rng.integers(0, w.nk, 192)], 1)
    e_f = rel_l2(I[sjk[:, 0], sjk[:, 1], sjk[:, 2]], oracle.project_rays(og, c, sjk))
    y = rng.standard_normal(P.data_shape, dtype=np.float32)
    yt = torch.from_numpy(y).to(DEV)
    g = P.adjoint(yt)
    xyz = np.stack([rng.integers(0, m, 24) for m in w.n], 1)
    e_a = rel_l2(g[xyz[:, 0], xyz[:, 1], xyz[:, 2]].cpu().numpy(), oracle.adjoint_voxels(og, y, xyz))
    lhs = float((torch.from_numpy(I).to(DEV).double() * yt.double()).sum())
    rhs = float((ct.double() * g.double()).sum())
    gap = abs(lhs - rhs) / (float(np.linalg.norm(I)) * float(np.linalg.norm(y)))
    print(f"[joseph fullsize] {name}: forward {e_f:.2e} adjoint {e_a:.2e} identity {gap:.2e}")
    assert e_f <= TOL and e_a <= TOL and gap <= 1e-6
