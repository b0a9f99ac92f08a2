"""GPU parity of the derived per-voxel quantities against the FP64 oracle.

The kernel reads float32 coefficients and evaluates in float32 (sums of at
most C terms, a float32 cyclic Jacobi of five sweeps); the oracle gets the
same float32 values and evaluates in float64.  Bounds, with eps = 2^-24:

* mean and tensor entries (one product / six-term sums): 1e-6 relative L2
  per field, every element within 1e-5 of max(|value|, scale);
* variance: a float32 sum of C - 1 squares has relative error <= C eps
  (9.1e-6 for C = 153), so 2e-6 relative L2 and elements within
  max(1e-5, 2 C eps) of their value;
* eigenvalues: 15 plane rotations, each exact up to a few eps of ||M||, move
  an eigenvalue by <= ~45 eps ||M|| (2.7e-6 ||M||): 5e-6 relative L2 and
  1e-5 of max(|value|, mean) per element; the ratios (relative anisotropy,
  FA; scale 1) follow: 1e-5;
* eigenvectors are unique only up to sign and only where the eigenvalue is
  separated from the others: with relative gap g > 1e-3 (gap / max|lambda|),
  Davis-Kahan bounds the angle to the float64 eigenvector by
  45 eps ||M|| / (g max|lambda|) <= 2.7e-6 / g, so |v . v_ref| >= 1 - 1e-5
  and, where the largest component leads the second by 1e-3 (so the sign
  convention decides the same way), every component within 1e-6 + 4e-6 / g.

Fields that vanish are measured against their natural scale: the mean for
the tensor and eigenvalues, its square for the variance, 1 for the ratios
(whose relative L2 error is taken against max(||ratio||, ||1||): for an
isotropic field the float32 eigenvalues differ by a few eps, which leaves an
FA of ~1e-7 where the float64 one is 1e-16).
"""
import numpy as np
import pytest
import torch

import oracle
from oracle.derived import FIELDS, tensor_properties as oracle_props
import tt_inputs as synth
from paper_2504_16446_amd.projector import PROPERTY_FIELDS, tensor_properties

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
F = {n: i for i, n in enumerate(FIELDS)}


def _coeffs(n_vox, ell_max, seed):
    rng = np.random.default_rng(seed)
    c = rng.standard_normal((n_vox, oracle.num_coeffs(ell_max))).astype(np.float32)
    c[:, 0] += 4.0  # positive means
    return c


def _check(got, ref, C):
    assert got.shape == ref.shape
    eps = 2.0 ** -24
    mean = np.abs(ref[:, F["mean"]])
    scales = {"mean": mean, "variance": mean ** 2, "rel_anisotropy": np.ones_like(mean), "fa": np.ones_like(mean)}
    tols = {"variance": (2e-6, max(1e-5, 2 * C * eps)), "lambda1": (5e-6, 1e-5), "lambda2": (5e-6, 1e-5),
            "lambda3": (5e-6, 1e-5), "rel_anisotropy": (1e-5, 1e-5), "fa": (1e-5, 1e-5)}
    for name in ("mean", "variance", "rel_anisotropy", "m_xx", "m_yy", "m_zz", "m_xy", "m_xz", "m_yz",
                 "lambda1", "lambda2", "lambda3", "fa"):
        g, r = got[:, F[name]], ref[:, F[name]]
        sc = scales.get(name, mean)
        t_l2, t_el = tols.get(name, (1e-6, 1e-5))
        # a ratio that vanishes (isotropic voxels) carries an absolute float32
        # error: measured against its scale 1 rather than its own size
        floor = 1.0 if name in ("rel_anisotropy", "fa") else 1e-6
        err = np.linalg.norm(g - r) / max(np.linalg.norm(r), floor * np.linalg.norm(sc))
        assert err <= t_l2, (name, err)
        assert np.all(np.abs(g - r) <= t_el * np.maximum(np.abs(r), sc)), name
    lam = ref[:, [F["lambda1"], F["lambda2"], F["lambda3"]]]
    lmax = np.abs(lam).max(1) + 1e-30
    for i in range(3):
        others = [o for o in range(3) if o != i]
        gap = np.min(np.abs(lam[:, [i]] - lam[:, others]), axis=1) / lmax
        sel = gap > 1e-3
        cols = [F[f"v{i + 1}_{a}"] for a in "xyz"]
        vg, vr = got[sel][:, cols], ref[sel][:, cols]
        assert np.all(np.abs((vg * vr).sum(1)) >= 1 - 1e-5), i
        s = np.sort(np.abs(vr), axis=1)
        lead = (s[:, 2] - s[:, 1]) > 1e-3
        bound = 1e-6 + 4e-6 / gap[sel][lead]
        assert np.all(np.abs(vg[lead] - vr[lead]) <= bound[:, None]), i


@pytest.mark.parametrize("ell_max,n_vox", [(0, 77), (2, 200), (4, 1), (6, 1037), (8, 4160 + 23), (16, 130)])
def test_properties_parity(ell_max, n_vox):
    assert tuple(PROPERTY_FIELDS) == tuple(FIELDS)
    c = _coeffs(n_vox, ell_max, 31 + ell_max)
    got = tensor_properties(torch.from_numpy(c).to(DEV), ell_max).cpu().numpy().astype(np.float64)
    ref = oracle_props(c.astype(np.float64), ell_max)
    _check(got, ref, c.shape[1])


def test_properties_empty_and_shape():
    c = torch.zeros((0, 45), device=DEV)
    out = tensor_properties(c, 8)
    assert tuple(out.shape) == (0, 22)
    c = torch.from_numpy(_coeffs(6 * 5 * 4, 4, 3).reshape(6, 5, 4, 15)).to(DEV)
    assert tuple(tensor_properties(c, 4).shape) == (6, 5, 4, 22)


def test_properties_full_size_sampled():
    """256^3 voxels at ell_max 8 (the largest reconstruction workload) in one launch; sampled voxels checked."""
    w = synth.WORKLOADS["c5"]
    g = torch.Generator(device=DEV)
    g.manual_seed(1234)
    c = torch.randn((w.n_vox, w.n_coeff), device=DEV, generator=g)
    c[:, 0] += 4.0
    got = tensor_properties(c, w.ell_max)
    torch.cuda.synchronize()
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.integers(0, w.n_vox, 4000), [0, w.n_vox - 1]])
    it = torch.from_numpy(idx).to(DEV)
    sub = got[it].cpu().numpy().astype(np.float64)
    ref = oracle_props(c[it].cpu().numpy().astype(np.float64), w.ell_max)
    _check(sub, ref, w.n_coeff)
