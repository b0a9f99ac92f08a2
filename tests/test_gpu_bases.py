"""GPU parity of the kernel basis sets (Gaussian kernels, nearest neighbour)
against the FP64 oracle: forward, adjoint and loss gradient, both projector
models, 1e-5 relative L2 (the map and its transpose only change through B)."""
import numpy as np
import pytest
import torch

import oracle
from geoms import tilted_angles
from helpers import gpu_projector, rel_l2, rel_max
import tt_inputs as synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
TOL = 1e-5


def _t(a):
    return torch.tensor(np.asarray(a, dtype=np.float32), device=DEV)


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


CASES = {
    "gk20": dict(basis="gk", dirs=synth.hemisphere_dirs(20), width=0.35),
    "gk64": dict(basis="gk", dirs=synth.hemisphere_dirs(64), width=0.2),
    "gk90_seg16": dict(basis="gk", dirs=synth.hemisphere_dirs(90), width=0.18, n_seg=16),
    "nn16": dict(basis="nn", dirs=synth.truncated_icosahedron_dirs(), width=None),
}


@pytest.mark.parametrize("model", ["trilinear", "joseph"])
@pytest.mark.parametrize("name", list(CASES))
def test_kernel_basis_parity(name, model):
    kw = dict(CASES[name])
    n_seg = kw.pop("n_seg", 8)
    inner, outer = tilted_angles(5, (0.0, 20.0, 45.0), span_deg=360.0)
    og = oracle.Geometry((14, 15, 13), 0, inner, outer, 17, 19, n_seg, synth.lab_frame(), model=model, **kw)
    rng = np.random.default_rng(31)
    c = rng.standard_normal(og.vol_shape).astype(np.float32).astype(np.float64)
    y = rng.standard_normal(og.data_shape).astype(np.float32).astype(np.float64)
    P = gpu_projector(og)
    assert P.n_coeff == og.n_coeff
    f, a = _np(P.forward(_t(c))), _np(P.adjoint(_t(y)))
    rf, ra = oracle.project(og, c), oracle.adjoint(og, y)
    print(name, model, "forward", rel_l2(f, rf), "adjoint", rel_l2(a, ra))
    assert rel_l2(f, rf) <= TOL and rel_max(f, rf) <= 10 * TOL
    assert rel_l2(a, ra) <= TOL and rel_max(a, ra) <= 10 * TOL
    loss, grad, _ = oracle.loss_grad(og, c, y, None, 1e-3)
    lg, gg, _ = P.loss_grad(_t(c), _t(y), None, 1e-3)
    assert abs(float(lg.item()) - loss) <= TOL * loss and rel_l2(_np(gg), grad) <= TOL
