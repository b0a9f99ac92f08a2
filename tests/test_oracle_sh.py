"""Pins of the oracle's spherical harmonics and goniometer rotation.

Spherical harmonics: section 3.2 of the paper (real, even-order, band limit
ell_max).  Pinned by exact quadrature, a library special case (scipy), the
addition theorem and closed forms of the lowest orders.
"""
import numpy as np
import pytest
import scipy.special as sp
from numpy.polynomial import legendre as npleg
from scipy.spatial.transform import Rotation

import oracle
from geoms import small


def _unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


@pytest.mark.parametrize("ell_max", [0, 2, 4, 6, 8, 12])
def test_counts(ell_max):
    assert oracle.num_coeffs(ell_max) == sum(2 * l + 1 for l in range(0, ell_max + 1, 2))
    assert oracle.sh(ell_max, np.array([0.3, -0.2, 0.9])).shape == (oracle.num_coeffs(ell_max),)


@pytest.mark.parametrize("ell_max", [2, 4, 8, 12])
def test_orthonormal_by_exact_quadrature(ell_max):
    # Gauss-Legendre in cos(theta) (exact to degree 2n-1) x trapezoid in phi
    # (exact for trigonometric degree < n_phi): exact for all products Y_i Y_j.
    x, wx = npleg.leggauss(ell_max + 1)
    n_phi = 2 * ell_max + 1
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    X, PH = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - X ** 2)
    dirs = np.stack([st * np.cos(PH), st * np.sin(PH), X], axis=-1).reshape(-1, 3)
    W = (wx[:, None] * np.full(n_phi, 2 * np.pi / n_phi)[None, :]).reshape(-1)
    Y = oracle.sh(ell_max, dirs)
    G = Y.T @ (W[:, None] * Y)
    assert np.abs(G - np.eye(G.shape[0])).max() < 1e-13


@pytest.mark.parametrize("ell_max", [2, 4, 8])
def test_matches_scipy_after_convention_map(ell_max):
    rng = np.random.default_rng(5)
    d = _unit(rng, 200)
    theta = np.arccos(np.clip(d[:, 2], -1, 1))
    phi = np.mod(np.arctan2(d[:, 1], d[:, 0]), 2 * np.pi)
    Y = oracle.sh(ell_max, d)
    i = 0
    for l in range(0, ell_max + 1, 2):
        for m in range(-l, l + 1):
            z = sp.sph_harm_y(l, abs(m), theta, phi)  # includes (-1)^m
            if m == 0:
                ref = z.real
            elif m > 0:
                ref = np.sqrt(2) * (-1) ** m * z.real
            else:
                ref = np.sqrt(2) * (-1) ** m * z.imag
            assert np.abs(Y[:, i] - ref).max() < 1e-13, (l, m)
            i += 1


@pytest.mark.parametrize("l,m", [(0, 0), (2, 0), (2, 1), (2, 2), (4, 3), (6, 6), (8, 5)])
def test_legendre_vs_scipy(l, m):
    for x in np.linspace(-1, 1, 13):
        ref = (-1) ** m * sp.lpmv(m, l, x)  # scipy carries the Condon-Shortley phase
        assert abs(oracle.legendre(l, m, x) - ref) < 1e-12 * max(1.0, abs(ref))


@pytest.mark.parametrize("l", [0, 2, 4, 6, 8])
def test_addition_theorem(l):
    rng = np.random.default_rng(l)
    a, b = _unit(rng, 50), _unit(rng, 50)
    Ya, Yb = oracle.sh(8, a), oracle.sh(8, b)
    lo = l * (l - 1) // 2
    sl = slice(lo, lo + 2 * l + 1)
    lhs = (Ya[:, sl] * Yb[:, sl]).sum(1)
    coef = np.zeros(l + 1)
    coef[l] = 1
    rhs = (2 * l + 1) / (4 * np.pi) * npleg.legval((a * b).sum(1), coef)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_low_order_closed_forms():
    rng = np.random.default_rng(11)
    d = _unit(rng, 64)
    x, y, z = d.T
    Y = oracle.sh(2, d)
    assert np.allclose(Y[:, 0], 1 / np.sqrt(4 * np.pi), atol=1e-15, rtol=0)
    # i = l(l-1)/2 + l + m for l = 2: m = -2..2 -> 1..5
    ref = {
        1: np.sqrt(15 / (4 * np.pi)) * x * y,            # m = -2
        2: np.sqrt(15 / (4 * np.pi)) * y * z,            # m = -1
        3: np.sqrt(5 / (16 * np.pi)) * (3 * z * z - 1),  # m = 0
        4: np.sqrt(15 / (4 * np.pi)) * x * z,            # m = 1
        5: np.sqrt(15 / (16 * np.pi)) * (x * x - y * y), # m = 2
    }
    for i, r in ref.items():
        assert np.abs(Y[:, i] - r).max() < 1e-14, i


def test_rotation_matches_scipy():
    # R_s = R_beta(beta_s) R_alpha(alpha_s) with right-handed axis rotations.
    g = small()
    fr = g.frame
    for s in range(g.n_proj):
        Ra = Rotation.from_rotvec(g.inner[s] * np.asarray(fr["alpha"]))
        Rb = Rotation.from_rotvec(g.outer[s] * np.asarray(fr["beta"]))
        ref = (Rb * Ra).as_matrix()
        assert np.abs(oracle.rotation(g, s) - ref).max() < 1e-14


def test_frame_is_rotated_lab_vectors():
    g = small()
    fr = g.frame
    for s in range(g.n_proj):
        R = oracle.rotation(g, s)
        ej, ek, d, o = oracle.frame(g, s)
        assert np.allclose(ej, R.T @ fr["j"], atol=1e-15)
        assert np.allclose(ek, R.T @ fr["k"], atol=1e-15)
        assert np.allclose(d, R.T @ fr["p"], atol=1e-15)
        cj, ck = (g.nj - 1) / 2, (g.nk - 1) / 2
        assert np.allclose(o, -cj * ej - ck * ek, atol=1e-13)
