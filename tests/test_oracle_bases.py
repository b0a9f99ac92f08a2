"""Pins of the oracle's kernel basis sets (Gaussian kernels, nearest neighbour).

* nearest neighbour: every sub-sample node belongs to exactly one direction,
  so each segment's row of B sums to 1 and holds multiples of 1/n_sub;
* Gaussian kernel, one direction along +z, untilted geometry: the segment
  average of exp(-w^2 / (2 width^2)) with w the angle to +-z written out
  with atan2 (closed form);
* antipodal segments coincide (both bases are antipodally symmetric);
* an isotropic field (every nearest-neighbour coefficient 1) projects like
  the unit isotropic spherical-harmonic field; <Ax, y> = <x, A^T y>.
"""
import math

import numpy as np

import oracle
from geoms import tilted_angles
import tt_inputs as synth


def _geom(basis, dirs, width=None, n=(6, 7, 5), n_seg=8, model="trilinear"):
    inner, outer = tilted_angles(4, (0.0, 25.0, 45.0), span_deg=360.0)
    return oracle.Geometry(n, 0, inner, outer, 9, 8, n_seg, synth.lab_frame(), basis=basis, dirs=dirs,
                           width=width, model=model)


def test_nearest_neighbour_partition_of_unity():
    g = _geom("nn", synth.truncated_icosahedron_dirs())
    B = g.B()
    assert B.shape == (g.n_proj, 8, 16)
    assert np.abs(B.sum(axis=2) - 1.0).max() < 1e-15
    assert np.abs(B * g.n_sub - np.round(B * g.n_sub)).max() < 1e-12


def test_gaussian_kernel_closed_form_and_antipodes():
    width = 0.4
    inner, outer = np.zeros(1), np.zeros(1)
    g = oracle.Geometry((4, 4, 4), 0, inner, outer, 5, 5, 8, synth.lab_frame(), basis="gk",
                        dirs=[[0.0, 0.0, 1.0]], width=width)
    B = g.B()[0, :, 0]
    for c in range(8):
        vals = []
        for m in range(3):
            phi = (c - 0.5 + (m + 0.5) / 3) * 2 * math.pi / 8
            q = (math.cos(phi), 0.0, math.sin(phi))  # lab q0 = +x, q90 = +z, identity rotation
            w = math.atan2(math.hypot(q[0], q[1]), abs(q[2]))
            vals.append(math.exp(-w * w / (2 * width * width)))
        assert abs(B[c] - sum(vals) / 3) < 1e-14
    g2 = _geom("gk", synth.hemisphere_dirs(24), width=0.35)
    B2 = g2.B()
    assert np.abs(B2[:, :4] - B2[:, 4:]).max() < 1e-13


def test_isotropic_field_matches_spherical_harmonics_and_adjoint_identity():
    for model in ("trilinear", "joseph"):
        gn = _geom("nn", synth.truncated_icosahedron_dirs(), model=model)
        gs = oracle.Geometry(gn.n, 0, gn.inner, gn.outer, gn.nj, gn.nk, gn.n_seg, synth.lab_frame(), model=model)
        In = oracle.project(gn, np.ones(gn.vol_shape))
        Is = oracle.project(gs, np.full(gs.vol_shape, math.sqrt(4 * math.pi)))
        assert np.abs(In - Is).max() < 1e-12 * np.abs(Is).max()
    g = _geom("gk", synth.hemisphere_dirs(20), width=0.3)
    rng = np.random.default_rng(12)
    x, y = rng.standard_normal(g.vol_shape), rng.standard_normal(g.data_shape)
    Ax = oracle.project(g, x)
    assert abs(np.vdot(Ax, y) - np.vdot(x, oracle.adjoint(g, y))) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)
