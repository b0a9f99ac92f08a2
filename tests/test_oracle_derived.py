"""Pins of the derived-quantity oracle against closed forms and identities.

* isotropic field: mean c00 / sqrt(4 pi), zero variance, M = mean I / 3, FA 0;
* the lobe (n.q)^2, written in SH through the addition theorem: mean 1/3,
  variance 4/45, M = (I + 2 n n^T) / 15 with eigenvector n for eigenvalue
  1/5, FA = 2 / sqrt(11);
* Parseval: variance = (1 / 4 pi) * sum of squared coefficients above l = 0;
* trace(M) = mean, M blind to l >= 4, and V diag(lambda) V^T = M.
"""
import math

import numpy as np

import oracle
from oracle.derived import FIELDS, sphere_quadrature, tensor_properties

F = {name: i for i, name in enumerate(FIELDS)}


def _M(out):
    M = np.empty(out.shape[:-1] + (3, 3))
    for a, b, key in ((0, 0, "m_xx"), (1, 1, "m_yy"), (2, 2, "m_zz"), (0, 1, "m_xy"), (0, 2, "m_xz"), (1, 2, "m_yz")):
        M[..., a, b] = M[..., b, a] = out[..., F[key]]
    return M


def test_quadrature_integrates_monomials_exactly():
    # <x^a y^b z^c> over the sphere: zero unless all even, else a closed form
    q, w = sphere_quadrature(8)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs((w * q[:, 2] ** 2).sum() - 1.0 / 3.0) < 1e-15
    assert abs((w * q[:, 0] ** 4).sum() - 1.0 / 5.0) < 1e-15
    assert abs((w * q[:, 0] ** 2 * q[:, 1] ** 2).sum() - 1.0 / 15.0) < 1e-15
    assert abs((w * q[:, 0] ** 2 * q[:, 1] ** 2 * q[:, 2] ** 2).sum() - 1.0 / 105.0) < 1e-15
    assert abs((w * q[:, 0] * q[:, 1] ** 3).sum()) < 1e-15


def test_isotropic_field():
    c = np.zeros((2, 15))
    c[0, 0], c[1, 0] = 2.0, -0.5
    out = tensor_properties(c, 4)
    mean = c[:, 0] / math.sqrt(4 * math.pi)
    assert np.allclose(out[:, F["mean"]], mean, rtol=1e-14)
    assert np.allclose(out[:, F["variance"]], 0.0, atol=1e-14)
    assert np.allclose(_M(out), mean[:, None, None] * np.eye(3) / 3.0, atol=1e-14)
    assert np.allclose(out[:, [F["lambda1"], F["lambda2"], F["lambda3"]]], (mean / 3.0)[:, None], atol=1e-14)
    assert np.allclose(out[:, F["fa"]], 0.0, atol=1e-7)


def _lobe_coeffs(n, ell_max):
    """(n.q)^2 = 1/3 + (2/3) P2(n.q), with P2(n.q) = (4 pi / 5) sum_m Y2m(n) Y2m(q)."""
    c = np.zeros(oracle.num_coeffs(ell_max))
    c[0] = math.sqrt(4 * math.pi) / 3.0
    Yn = oracle.sh(ell_max, np.asarray(n, float)[None])[0]
    c[1:6] = (2.0 / 3.0) * (4 * math.pi / 5.0) * Yn[1:6]
    return c


def test_lobe_closed_forms():
    rng = np.random.default_rng(5)
    for _ in range(6):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        out = tensor_properties(_lobe_coeffs(n, 6)[None], 6)[0]
        assert abs(out[F["mean"]] - 1.0 / 3.0) < 1e-14
        assert abs(out[F["variance"]] - 4.0 / 45.0) < 1e-14
        assert abs(out[F["rel_anisotropy"]] - 2.0 / math.sqrt(5.0)) < 1e-13
        assert np.allclose(_M(out), (np.eye(3) + 2.0 * np.outer(n, n)) / 15.0, atol=1e-15)
        lam = out[[F["lambda1"], F["lambda2"], F["lambda3"]]]
        assert np.allclose(lam, [1 / 5, 1 / 15, 1 / 15], atol=1e-15)
        v1 = out[[F["v1_x"], F["v1_y"], F["v1_z"]]]
        assert abs(abs(v1 @ n) - 1.0) < 1e-12
        assert abs(np.abs(v1).max() - v1[np.abs(v1).argmax()]) == 0.0  # sign convention
        assert abs(out[F["fa"]] - 2.0 / math.sqrt(11.0)) < 1e-13


def test_parseval_trace_and_band_limit():
    rng = np.random.default_rng(11)
    ell_max = 8
    c = rng.standard_normal((40, oracle.num_coeffs(ell_max)))
    c[:, 0] += 6.0
    out = tensor_properties(c, ell_max)
    assert np.allclose(out[:, F["variance"]], (c[:, 1:] ** 2).sum(1) / (4 * math.pi), rtol=1e-13)
    M = _M(out)
    assert np.allclose(np.trace(M, axis1=1, axis2=2), out[:, F["mean"]], rtol=1e-13)
    c2 = c.copy()
    c2[:, 6:] = rng.standard_normal((40, c.shape[1] - 6))
    assert np.allclose(_M(tensor_properties(c2, ell_max)), M, atol=1e-14)
    V = np.stack([out[:, [F[f"v{i}_x"], F[f"v{i}_y"], F[f"v{i}_z"]]] for i in (1, 2, 3)], axis=2)
    lam = out[:, [F["lambda1"], F["lambda2"], F["lambda3"]]]
    assert np.allclose(V @ (lam[:, :, None] * V.transpose(0, 2, 1)), M, atol=1e-13)
    assert np.allclose(V.transpose(0, 2, 1) @ V, np.eye(3), atol=1e-13)
    assert np.all(lam[:, 0] >= lam[:, 1]) and np.all(lam[:, 1] >= lam[:, 2])
