"""Pins of the oracle's forward model and adjoint.

Eq. projection_operator / forward_model of the paper, with P_{sjk,xyz}
realised as unit-step trilinear ray sampling with zero padding.  Pinned by
closed-form path lengths of a uniform cube, a separable closed form for affine
fields along oblique rays, chord lengths of a ball, brute force on a tiny
volume (the paper's block-Kronecker form of A built literally), and the
adjoint identity.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import dense
from geoms import small, tiny, workload
import tt_inputs as synth

SQ4PI = math.sqrt(4 * math.pi)


def _iso(n, ell_max, values):
    c = np.zeros(tuple(n) + (oracle.num_coeffs(ell_max),))
    c[..., 0] = values
    return c


def test_uniform_cube_axis_aligned_exact():
    # Rays along a grid axis through voxel-centre columns; samples sit midway
    # between centres, so each voxel receives total weight 1: sum = N.
    N = 32
    g = oracle.Geometry((N, N, N), 4, np.deg2rad([0.0, 90.0, 180.0, 270.0]), np.zeros(4),
                        N, N, 8, synth.lab_frame())
    I = oracle.project(g, _iso(g.n, 4, 1.0))
    assert np.abs(I * SQ4PI - N).max() < 1e-12


def _trapezoid(u, n):
    """sum_i T(u - i) over i = 0..n-1 (tent partition of unity with zero padding)."""
    return np.where((u >= 0) & (u <= n - 1), 1.0,
                    np.where((u > -1) & (u < 0), 1 + u,
                             np.where((u > n - 1) & (u < n), n - u, 0.0)))


def _first_moment(u, n):
    """sum_i T(u - i) x_i with x_i = i - (n-1)/2 (linear precision inside)."""
    h = (n - 1) / 2.0
    return np.where((u >= 0) & (u <= n - 1), u - h,
                    np.where((u > -1) & (u < 0), (1 + u) * (-h),
                             np.where((u > n - 1) & (u < n), (n - u) * h, 0.0)))


@pytest.mark.parametrize("step", [1.0, 0.7])
def test_affine_field_oblique_rays_separable_closed_form(step):
    # Trilinear weights are a tensor product, so for an affine field
    # f_v = h + g . x_v the interpolant at x is
    # h prod_a W_a + sum_a g_a M_a prod_{b != a} W_b with 1-D closed forms.
    g = small(ell_max=2)
    g = oracle.Geometry(g.n, 2, g.inner, g.outer, g.nj, g.nk, g.n_seg, synth.lab_frame(),
                        step=step, joff=np.linspace(-0.3, 0.4, g.n_proj),
                        koff=np.linspace(0.2, -0.1, g.n_proj))
    gvec, h = np.array([0.31, -0.17, 0.23]), 1.7
    xv = dense.voxel_centres(g).reshape(g.n + (3,))
    I = oracle.project(g, _iso(g.n, 2, h + xv @ gvec))
    nl = int(math.ceil((0.5 * math.sqrt(sum(m * m for m in g.n)) + 2) / step)) + 1
    ns = np.arange(-nl, nl + 1)
    for s in range(g.n_proj):
        ej, ek, d, o = oracle.frame(g, s)
        J, K = np.meshgrid(np.arange(g.nj), np.arange(g.nk), indexing="ij")
        X = (o + J[..., None, None] * ej + K[..., None, None] * ek
             + ns[:, None] * step * d)  # (nj, nk, n, 3)
        U = [X[..., a] + (g.n[a] - 1) / 2.0 for a in range(3)]
        W = [_trapezoid(U[a], g.n[a]) for a in range(3)]
        M = [_first_moment(U[a], g.n[a]) for a in range(3)]
        val = h * W[0] * W[1] * W[2]
        val += gvec[0] * M[0] * W[1] * W[2] + gvec[1] * W[0] * M[1] * W[2] + gvec[2] * W[0] * W[1] * M[2]
        ref = step * val.sum(-1)
        got = I[s] * SQ4PI  # every segment: isotropic field
        assert np.abs(got - ref[..., None]).max() < 1e-12 * max(1.0, np.abs(ref).max())


def test_ball_chord_lengths():
    g = workload("c1")
    R = 14.0
    xv = dense.voxel_centres(g).reshape(g.n + (3,))
    I = oracle.project(g, _iso(g.n, 4, (np.linalg.norm(xv, axis=-1) <= R).astype(float)))
    errs = []
    for s in range(g.n_proj):
        ej, ek, d, o = oracle.frame(g, s)
        J, K = np.meshgrid(np.arange(g.nj), np.arange(g.nk), indexing="ij")
        U = o + J[..., None] * ej + K[..., None] * ek
        rho = np.linalg.norm(U, axis=-1)
        sel = rho <= R - 2
        chord = 2 * np.sqrt(R * R - rho[sel] ** 2)
        errs.append(I[s][..., 0][sel] * SQ4PI - chord)
    e = np.concatenate(errs)
    assert np.abs(e).max() <= 1.5
    assert np.sqrt(np.mean(e ** 2)) <= 0.5
    assert abs(e.mean()) <= 0.05


def test_isotropic_field_gives_equal_segments():
    g = small(ell_max=4)
    rng = np.random.default_rng(3)
    I = oracle.project(g, _iso(g.n, 4, rng.uniform(size=g.n)))
    assert np.abs(I - I[..., :1]).max() < 1e-13 * np.abs(I).max()


def test_mass_conservation():
    # Each voxel spreads total weight 1 over an axis-aligned projection.  For
    # oblique ones the tent summed over the rotated sample lattice ripples
    # around 1 by a few percent per voxel (aliasing of the tent's spectrum),
    # which averages to about 1e-3 over this small ball.
    N = 24
    inner = np.deg2rad([0.0, 37.0, 71.0])
    outer = np.deg2rad([0.0, 0.0, 30.0])
    g = oracle.Geometry((N, N, N), 2, inner, outer, 2 * N, 2 * N, 8, synth.lab_frame())
    rng = np.random.default_rng(4)
    xv = dense.voxel_centres(g).reshape(g.n + (3,))
    vals = rng.uniform(size=g.n) * (np.linalg.norm(xv, axis=-1) < 9)
    I = oracle.project(g, _iso(g.n, 2, vals))
    tot = vals.sum()
    mass = I[..., 0].sum(axis=(1, 2)) * SQ4PI
    assert abs(mass[0] - tot) < 1e-11 * tot
    assert np.abs(mass[1:] - tot).max() < 3e-3 * tot


@pytest.mark.parametrize("kw", [dict(), dict(offsets=True, step=0.8), dict(ell_max=4, n=(5, 5, 6))])
def test_brute_force_dense_system_matrix(kw):
    g = tiny(**kw)
    A = dense.dense_A(g)
    rng = np.random.default_rng(7)
    c = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.data_shape)
    Ac = oracle.project(g, c)
    assert np.abs(Ac.reshape(-1) - A @ c.reshape(-1)).max() < 1e-13 * np.abs(Ac).max()
    ATy = oracle.adjoint(g, y)
    ref = A.T @ y.reshape(-1)
    assert np.abs(ATy.reshape(-1) - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["tiny", "c1"])
def test_adjoint_identity(name):
    g = tiny(offsets=True) if name == "tiny" else workload("c1")
    rng = np.random.default_rng(8)
    x = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.data_shape)
    Ax = oracle.project(g, x)
    ATy = oracle.adjoint(g, y)
    gap = abs(np.vdot(Ax, y) - np.vdot(x, ATy)) / (np.linalg.norm(Ax) * np.linalg.norm(y))
    assert gap < 1e-12


def test_ray_and_voxel_subsets_match_full():
    g = small(ell_max=4)
    rng = np.random.default_rng(9)
    c = rng.standard_normal(g.vol_shape)
    y = rng.standard_normal(g.data_shape)
    I = oracle.project(g, c)
    sjk = np.stack([rng.integers(0, g.n_proj, 40), rng.integers(0, g.nj, 40),
                    rng.integers(0, g.nk, 40)], axis=1)
    assert np.abs(oracle.project_rays(g, c, sjk) - I[sjk[:, 0], sjk[:, 1], sjk[:, 2]]).max() < 1e-12
    G = oracle.adjoint(g, y)
    xyz = np.stack([rng.integers(0, m, 40) for m in g.n], axis=1)
    xyz[:3] = [[0, 0, 0], [g.n[0] - 1, g.n[1] - 1, g.n[2] - 1], [0, g.n[1] - 1, 0]]
    got = oracle.adjoint_voxels(g, y, xyz)
    assert np.abs(got - G[xyz[:, 0], xyz[:, 1], xyz[:, 2]]).max() < 1e-12 * np.abs(G).max()


def test_segment_first_adjoint_equals_adjoint():
    # sum_s B_s^T (P_s^T fold(y_s)) equals the adjoint computed ray by ray
    for g in (small(ell_max=4), small(ell_max=8, n_seg=16), tiny(offsets=True, step=0.8)):
        y = np.random.default_rng(31).standard_normal(g.data_shape)
        ref = oracle.adjoint(g, y)
        got = oracle.adjoint_segment_first(g, y)
        assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # without antipodal folding (half-circle segments)
    g = oracle.Geometry((7, 8, 9), 2, [0.3, 1.1], [0.0, 0.5], 9, 10, 6, synth.lab_frame(), seg_span=np.pi)
    assert oracle.unique_segments(g) == 6
    y = np.random.default_rng(32).standard_normal(g.data_shape)
    assert np.abs(oracle.adjoint_segment_first(g, y) - oracle.adjoint(g, y)).max() < 1e-12 * np.abs(oracle.adjoint(g, y)).max()


def test_bf16_rounding_helper():
    x = np.array([1.0, 1.00390625, 1.005859375, -3.1415926, 1e-3, 65504.0])
    r = oracle.bf16(x)
    # 8 significant bits: 1 + 2^-8 is a tie between 1 and 1 + 2^-7 and rounds to even (1.0)
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == 1.0078125
    assert abs(r[3] + 3.140625) < 1e-12
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)
