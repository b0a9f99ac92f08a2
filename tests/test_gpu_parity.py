"""GPU parity: the HIP path against the FP64 oracle, element by element.

Tolerance (float32 path vs float64 oracle): relative L2 error <= 1e-5 per
output tensor, and the largest element error <= 1e-4 of the largest element.
Inputs are seeded Gaussian fields (every coefficient and segment nonzero),
which is harder on the arithmetic than smooth phantoms.
"""
import numpy as np
import pytest
import torch

import oracle
from geoms import degenerate, small, steep, tiny, workload
from helpers import gpu_projector, rel_l2, rel_max
import tt_inputs as synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


def _t(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device=DEV)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _inputs(og, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal(og.vol_shape).astype(np.float32).astype(np.float64)
    y = rng.standard_normal(og.data_shape).astype(np.float32).astype(np.float64)
    return c, y


def _half_circle():
    g = tiny()
    return oracle.Geometry((9, 11, 10), 2, g.inner, g.outer, 12, 10, 6, synth.lab_frame(), seg_span=np.pi)


CASES = {
    "tiny": lambda: tiny(),
    "tiny_offsets_step": lambda: tiny(offsets=True, step=0.8),
    "small_l4": lambda: small(ell_max=4),
    "small_l8_seg16": lambda: small(ell_max=8, n_seg=16),
    "small_l6_seg8": lambda: small(ell_max=6),
    "small_l0": lambda: small(ell_max=0, n_seg=4),
    "small_l10": lambda: small(ell_max=10),                 # C = 66: streamed map (Cp 80), 5 adjoint tiles
    "small_l12_seg16": lambda: small(ell_max=12, n_seg=16),  # C = 91: Cp 96, 6 adjoint tiles, 8 unique segments
    "half_circle_segments": _half_circle,   # no antipodal folding: 6 distinct segments
    "steep_tilts": lambda: steep(),          # forward march gathers these rays from global memory
    "degenerate": lambda: degenerate(),      # 1-voxel-thick volume, one detector row, 2 segments
    "c1": lambda: workload("c1"),
    # the adjoint pairs each voxel with its point inverse (centred detector, even
    # nx, four unique segments): an odd projection count leaves the last pair
    # half empty, and nx / 2 odd leaves the last block with one x-slice pair
    # outside the volume
    "odd_projection_count": lambda: small(ell_max=4, n_rot=5),
    "paired_l8_ragged": lambda: small(ell_max=8, n=(18, 13, 11), n_rot=3),
    # eight unique segments: the adjoint stages each brick's residual window in
    # LDS (detector offsets, a non-unit step, steep tilts)
    "tiny_offsets_step_seg16": lambda: tiny(offsets=True, step=0.8, n_seg=16),
    "steep_seg16": lambda: steep(n_seg=16),
    # sample steps above one voxel (fewer samples than planes along the ray)
    "tiny_step_1p5_seg16": lambda: tiny(offsets=True, step=1.5, n_seg=16),
    "tiny_step_2": lambda: tiny(step=2.0),
    # sixteen unique segments (the widest layout: four float4 per mapped voxel)
    "small_l4_seg32": lambda: small(ell_max=4, n_seg=32),
    "small_l8_seg32": lambda: small(ell_max=8, n_seg=32),
    "steep_seg32": lambda: steep(n_seg=32),
    # twelve distinct segments over a half circle: padded to sixteen channels
    "half_circle_seg12": lambda: oracle.Geometry((9, 11, 10), 2, tiny().inner, tiny().outer, 12, 10, 12,
                                                 synth.lab_frame(), seg_span=np.pi),
}


def _geom(name):
    return CASES[name]()


@pytest.mark.parametrize("name", list(CASES))
def test_forward_parity(name):
    og = _geom(name)
    c, _ = _inputs(og, 1)
    ref = oracle.project(og, c)
    P = gpu_projector(og)
    got = _np(P.forward(_t(c)))
    torch.cuda.synchronize()
    print(name, "forward rel-L2", rel_l2(got, ref), "rel-max", rel_max(got, ref))
    assert rel_l2(got, ref) <= TOL
    assert rel_max(got, ref) <= 10 * TOL


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_parity(name):
    og = _geom(name)
    _, y = _inputs(og, 2)
    ref = oracle.adjoint(og, y)
    P = gpu_projector(og)
    got = _np(P.adjoint(_t(y)))
    print(name, "adjoint rel-L2", rel_l2(got, ref), "rel-max", rel_max(got, ref))
    assert rel_l2(got, ref) <= TOL
    assert rel_max(got, ref) <= 10 * TOL


@pytest.mark.parametrize("name", ["tiny_offsets_step", "small_l8_seg16", "c1", "small_l8_seg32"])
def test_loss_grad_parity(name):
    og = _geom(name)
    c, data = _inputs(og, 3)
    rng = np.random.default_rng(4)
    w = rng.uniform(0.5, 1.5, og.data_shape).astype(np.float32).astype(np.float64)
    mu = 1e-3
    loss, grad, resid = oracle.loss_grad(og, c, data, w, mu)
    P = gpu_projector(og)
    l_g, g_g, r_g = P.loss_grad(_t(c), _t(data), _t(w), mu)
    assert abs(float(l_g.item()) - loss) <= TOL * loss
    assert rel_l2(_np(g_g), grad) <= TOL
    assert rel_l2(_np(r_g), resid) <= TOL
    # without weights and without the residual output
    loss1, grad1, _ = oracle.loss_grad(og, c, data, None, 0.0)
    l1, g1, r1 = P.loss_grad(_t(c), _t(data), None, 0.0, want_resid=False)
    assert r1 is None
    assert abs(float(l1.item()) - loss1) <= TOL * loss1
    assert rel_l2(_np(g1), grad1) <= TOL


def test_adjoint_with_beta_term():
    og = small(ell_max=4)
    c, y = _inputs(og, 5)
    P = gpu_projector(og)
    got = _np(P.adjoint(_t(y), beta=0.37, c=_t(c)))
    ref = oracle.adjoint(og, y) + 0.37 * c
    assert rel_l2(got, ref) <= TOL


def test_adjoint_identity_gpu():
    og = workload("c1")
    c, y = _inputs(og, 6)
    P = gpu_projector(og)
    Ax = P.forward(_t(c)).double()
    ATy = P.adjoint(_t(y)).double()
    lhs = float((Ax * _t(y).double()).sum())
    rhs = float((_t(c).double() * ATy).sum())
    gap = abs(lhs - rhs) / (float(Ax.norm()) * float(np.linalg.norm(y)))
    assert gap < 1e-6


def test_repeat_determinism():
    og = small(ell_max=8, n_seg=16)
    c, y = _inputs(og, 7)
    P = gpu_projector(og)
    a1 = P.forward(_t(c)).clone()
    a2 = P.forward(_t(c))
    b1 = P.adjoint(_t(y)).clone()
    b2 = P.adjoint(_t(y))
    assert torch.equal(a1, a2) and torch.equal(b1, b2)


def test_forward_batches_agree():
    # the same geometry with the smallest forward batch (many batches) gives identical results
    og = small(ell_max=4)
    c, _ = _inputs(og, 8)
    P1 = gpu_projector(og)
    P2 = gpu_projector(og, forward_batch=1)
    assert P2.batch == 4 and P1.batch == og.n_proj
    assert torch.equal(P1.forward(_t(c)), P2.forward(_t(c)))


def test_workspace_is_required_and_sized():
    import ctypes as C
    from paper_2504_16446_amd._lib import TTError, call, lib
    og = small(ell_max=4)
    P = gpu_projector(og)
    h = C.c_void_p()
    with torch.cuda.device(DEV):
        call("tt_create", C.byref(P.geometry), C.byref(h))
    try:
        c = _t(_inputs(og, 9)[0])
        I = torch.empty(og.data_shape, device=DEV)
        with pytest.raises(TTError):  # no workspace attached
            call("tt_project", h, C.c_void_p(c.data_ptr()), C.c_void_p(I.data_ptr()))
        small_ws = int(call("tt_workspace_bytes", h, 1))
        full_ws = int(call("tt_workspace_bytes", h, og.n_proj))
        assert full_ws > small_ws > 0
        ws = torch.empty(small_ws - 256, dtype=torch.uint8, device=DEV)
        with pytest.raises(TTError):  # below the minimum
            call("tt_set_workspace", h, C.c_void_p(ws.data_ptr()), ws.numel())
        ws = torch.empty(full_ws, dtype=torch.uint8, device=DEV)
        call("tt_set_workspace", h, C.c_void_p(ws.data_ptr()), ws.numel())
        call("tt_project", h, C.c_void_p(c.data_ptr()), C.c_void_p(I.data_ptr()))
        assert torch.equal(I, P.forward(c))
    finally:
        lib().tt_destroy(h)

