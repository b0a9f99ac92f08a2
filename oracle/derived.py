"""FP64 oracle for the per-voxel quantities derived from reconstructed coefficients.

Test infrastructure only (see the package docstring).  Each quantity is the
plain definition from the paper's section on deriving standard quantities
from the output, evaluated by exact spherical quadrature of the expanded
function f(q) = sum_i c_i Y_i(q):

* spherical mean          fbar = <f>                     (the mean-intensity equation)
* spherical variance      var  = <(f - fbar)^2>
* relative anisotropy     sqrt(var) / fbar               (spherical standard deviation over the mean)
* second-moment tensor    M_ab = <q_a q_b f>             (the second-moment equation)
* eigenvalues / vectors   of M, eigenvalues in descending order
* fractional anisotropy   FA from the eigenvalues        (the FA equation)

<g> is the average over the unit sphere, (1 / 4 pi) * integral of g.  The
quadrature is Gauss-Legendre in cos(theta) times the trapezoid rule in phi,
with enough nodes to be exact for the polynomial degrees involved (2 ell_max
for the variance), so each value is the definition up to rounding.
"""
from __future__ import annotations

import numpy as np

from . import sh

__all__ = ["sphere_quadrature", "tensor_properties", "FIELDS"]

# Column order of tensor_properties' output.
FIELDS = ("mean", "variance", "rel_anisotropy",
          "m_xx", "m_yy", "m_zz", "m_xy", "m_xz", "m_yz",
          "lambda1", "lambda2", "lambda3",
          "v1_x", "v1_y", "v1_z", "v2_x", "v2_y", "v2_z", "v3_x", "v3_y", "v3_z",
          "fa")


def sphere_quadrature(degree: int):
    """Nodes (n, 3) and weights (n,) with sum(w g(q)) = <g> for polynomials of the given degree."""
    n_t = degree // 2 + 1                 # Gauss-Legendre exact to degree 2 n_t - 1 >= degree
    n_p = degree + 1                      # trapezoid in phi exact for trig degree < n_p
    x, wx = np.polynomial.legendre.leggauss(n_t)
    phi = 2.0 * np.pi * np.arange(n_p) / n_p
    st = np.sqrt(1.0 - x * x)
    q = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                  np.outer(x, np.ones(n_p))], axis=-1).reshape(-1, 3)
    w = np.outer(wx, np.full(n_p, 1.0 / n_p)).reshape(-1) / 2.0  # (1/4pi) * (2pi/n_p) * wx
    return q, w


def tensor_properties(c, ell_max: int):
    """Derived quantities per voxel: array (..., len(FIELDS)) in FIELDS order.

    Eigenvectors are unit length with their largest-magnitude component made
    positive; for repeated eigenvalues they are not unique (compare spans).
    """
    c = np.asarray(c, dtype=np.float64)
    shape = c.shape[:-1]
    cf = c.reshape(-1, c.shape[-1])
    q, w = sphere_quadrature(2 * max(ell_max, 2))
    Y = sh(ell_max, q)                    # (n_nodes, C)
    f = cf @ Y.T                          # (V, n_nodes)
    mean = f @ w
    var = ((f - mean[:, None]) ** 2) @ w
    qq = q[:, :, None] * q[:, None, :]    # (n_nodes, 3, 3)
    M = np.einsum("vn,n,nab->vab", f, w, qq)
    lam, vec = np.linalg.eigh(M)          # ascending
    lam = lam[:, ::-1]
    vec = vec[:, :, ::-1]
    idx = np.abs(vec).argmax(axis=1)      # per eigenvector, largest component
    sgn = np.sign(np.take_along_axis(vec, idx[:, None, :], axis=1))
    sgn[sgn == 0] = 1.0
    vec = vec * sgn
    l1, l2, l3 = lam[:, 0], lam[:, 1], lam[:, 2]
    num = np.sqrt((l1 - l2) ** 2 + (l2 - l3) ** 2 + (l3 - l1) ** 2)
    den = np.sqrt(2.0 * (l1 ** 2 + l2 ** 2 + l3 ** 2))
    fa = np.divide(num, den, out=np.zeros_like(num), where=den > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        ra = np.sqrt(np.maximum(var, 0.0)) / mean
    out = np.concatenate([
        mean[:, None], var[:, None], ra[:, None],
        M[:, 0, 0, None], M[:, 1, 1, None], M[:, 2, 2, None],
        M[:, 0, 1, None], M[:, 0, 2, None], M[:, 1, 2, None],
        lam,
        vec[:, :, 0], vec[:, :, 1], vec[:, :, 2],
        fa[:, None]], axis=1)
    return out.reshape(shape + (len(FIELDS),))
