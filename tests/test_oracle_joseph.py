"""Pins of the oracle's Joseph-method projector (the paper's own discretisation).

* axis-aligned rays: identical to the unit-step trilinear projector (both give
  bilinearly interpolated column sums);
* a uniform isotropic field: every ray whose cuts all fall inside the voxel-
  centre hull sums to N_A / |d_A| (closed form);
* a dense system matrix built literally from the definition (loop over rays
  and voxels, bilinear weight of the voxel at the ray's cut with its layer)
  reproduces the forward and adjoint;
* <Ax, y> = <x, A^T y>, and the per-voxel adjoint equals the full one.
"""
import math

import numpy as np
import pytest

import oracle
import tt_inputs as synth


def _geom(n, ell_max, inner_deg, outer_deg, nj, nk, n_seg=8, **kw):
    inner = np.deg2rad(np.asarray(inner_deg, float))
    outer = np.deg2rad(np.asarray(outer_deg, float))
    return oracle.Geometry(n, ell_max, inner, outer, nj, nk, n_seg, synth.lab_frame(), model="joseph", **kw)


def _dominant(d):
    a = 0
    for q in (1, 2):
        if abs(d[q]) > abs(d[a]) + 1e-9:
            a = q
    return a


def _dense_joseph(g):
    """P[s, j, k, voxel] from the definition, voxel-by-voxel."""
    n = np.array(g.n)
    P = np.zeros((g.n_proj, g.nj, g.nk) + g.n)
    for s in range(g.n_proj):
        ej, ek, d, o = oracle.frame(g, s)
        A = _dominant(d)
        others = [q for q in range(3) if q != A]
        for j in range(g.nj):
            for k in range(g.nk):
                base = o + j * ej + k * ek
                for v in np.ndindex(*g.n):
                    xv = np.array(v) - 0.5 * (n - 1)
                    t = (xv[A] - base[A]) / d[A]
                    x = base + t * d
                    w = 1.0 / abs(d[A])
                    for q in others:
                        w *= max(0.0, 1.0 - abs(x[q] - xv[q]))
                    P[(s, j, k) + v] = w
    return P


def test_axis_aligned_rays_equal_trilinear():
    inner = [0.0, 90.0, 180.0, 270.0]
    for n in ((7, 8, 9), (6, 6, 5)):
        gj = _geom(n, 2, inner, [0.0] * 4, 11, 10, joff=np.linspace(-0.4, 0.3, 4), koff=np.linspace(0.2, -0.3, 4))
        gt = oracle.Geometry(n, 2, gj.inner, gj.outer, 11, 10, 8, synth.lab_frame(),
                             joff=gj.joff, koff=gj.koff)
        c = np.random.default_rng(3).standard_normal(gj.vol_shape)
        assert np.abs(oracle.project(gj, c) - oracle.project(gt, c)).max() < 1e-12


def test_uniform_field_interior_rays_closed_form():
    g = _geom((20, 22, 18), 0, [10.0, 33.0, 71.0, 200.0], [0.0, 20.0, 35.0, 10.0], 30, 30, n_seg=4)
    c = np.full(g.vol_shape, math.sqrt(4 * math.pi))   # spherical mean 1 everywhere
    I = oracle.project(g, c)[..., 0]
    n = np.array(g.n)
    checked = 0
    for s in range(g.n_proj):
        ej, ek, d, o = oracle.frame(g, s)
        A = _dominant(d)
        others = [q for q in range(3) if q != A]
        xa = np.arange(n[A]) - 0.5 * (n[A] - 1)
        for j in range(g.nj):
            for k in range(g.nk):
                base = o + j * ej + k * ek
                t = (xa - base[A]) / d[A]
                u = base[None, :] + t[:, None] * d[None, :] + 0.5 * (n - 1)
                if all(np.all((u[:, q] >= 0) & (u[:, q] <= n[q] - 1)) for q in others):
                    assert abs(I[s, j, k] - n[A] / abs(d[A])) < 1e-11
                    checked += 1
    assert checked > 200


def test_dense_definition_and_adjoint_identity():
    g = _geom((5, 6, 4), 2, [7.0, 52.0, 130.0], [0.0, 25.0, 45.0], 8, 7, n_seg=6,
              joff=[0.1, -0.3, 0.25], koff=[-0.2, 0.35, 0.0])
    P = _dense_joseph(g)
    B = g.B()
    rng = np.random.default_rng(8)
    c = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.data_shape)
    ref = np.einsum("sjkxyz,xyzi,sci->sjkc", P, c, B)
    assert np.abs(oracle.project(g, c) - ref).max() < 1e-12
    ref_adj = np.einsum("sjkxyz,sjkc,sci->xyzi", P, y, B)
    assert np.abs(oracle.adjoint(g, y) - ref_adj).max() < 1e-12
    lhs = np.vdot(oracle.project(g, c), y)
    rhs = np.vdot(c, oracle.adjoint(g, y))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(oracle.project(g, c)) * np.linalg.norm(y)


@pytest.mark.parametrize("name", ["c1", "tilted"])
def test_adjoint_identity_and_voxel_subset(name):
    if name == "c1":
        g = oracle.Geometry.from_workload(synth.WORKLOADS["c1"], model="joseph")
    else:
        g = _geom((9, 11, 10), 4, [7.0, 97.0, 187.0, 277.0, 45.0], [0.0, 15.0, 30.0, 45.0, 45.0], 14, 13,
                  joff=np.linspace(-0.4, 0.3, 5), koff=np.linspace(0.25, -0.35, 5))
    rng = np.random.default_rng(9)
    c = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.data_shape)
    Ac, Aty = oracle.project(g, c), oracle.adjoint(g, y)
    assert abs(np.vdot(Ac, y) - np.vdot(c, Aty)) <= 1e-12 * np.linalg.norm(Ac) * np.linalg.norm(y)
    xyz = np.stack([rng.integers(0, m, 25) for m in g.n], 1)
    sub = oracle.adjoint_voxels(g, y, xyz)
    assert np.abs(sub - Aty[xyz[:, 0], xyz[:, 1], xyz[:, 2]]).max() <= 1e-12 * np.abs(Aty).max()
    sjk = np.stack([rng.integers(0, g.n_proj, 30), rng.integers(0, g.nj, 30), rng.integers(0, g.nk, 30)], 1)
    rays = oracle.project_rays(g, c, sjk)
    assert np.abs(rays - Ac[sjk[:, 0], sjk[:, 1], sjk[:, 2]]).max() <= 1e-12 * np.abs(Ac).max()
