"""Seeded synthetic inputs shared by the GPU path, the oracle, the tests and the benchmark.

This module draws random numbers and lays out workload configurations only.
It holds none of the tensor-tomography arithmetic (no rotations of the
goniometer, no spherical harmonics, no projection): every quantity here is a
plain input that either side of a comparison consumes unchanged.

Workloads (all unit voxels, parallel beam, segments over the full circle):

* ``c1`` 32^3, ell_max 4, 15 rotations over [0, 180) deg x tilts {0,15,30,45},
  detector 32x32 x 8 segments, twisted-fibre phantom, radius 14, 1% noise.
* ``c2`` 100^3, ell_max 8, 60 rotations over [0, 360) x 4 tilts, 100x100 x 8,
  twisted-fibre phantom, radius 45, 1% noise, mu = 1e-3.
* ``c3`` 128^3, ell_max 8, 75 rotations over [0, 360) x 4 tilts, 128x128 x 16,
  twisted-fibre phantom, radius 57, 1% noise.
* ``c4`` 48^3, ell_max 6, 30 rotations x 4 tilts, 64x64 x 8, multi-bundle
  phantom, radius 21, 1% noise (training data for the warm-start network).
* ``c5`` 256^3, ell_max 8, 100 rotations x 4 tilts, 256x256 x 16,
  multi-bundle phantom, radius 114, no noise.

The angle grids exclude the end point (n * step for n < count), which gives the
stated projection counts (60/240/300/120/400).  Projection index
s = tilt_index * n_rot + rot_index.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "Workload", "WORKLOADS", "lab_frame", "angles", "gaussian", "uniform",
    "twisted_fibre_field", "multi_bundle_field", "noise", "truncated_icosahedron_dirs", "hemisphere_dirs",
]


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n: tuple            # (nx, ny, nz)
    ell_max: int
    n_rot: int
    rot_span_deg: float
    tilts_deg: tuple
    nj: int
    nk: int
    n_seg: int
    radius: float
    phantom: str        # "twisted" | "bundles"
    noise: float        # relative to max |I_clean|; 0 = none
    mu: float
    seed_phantom: int
    seed_noise: int
    n_sub: int = 3
    step: float = 1.0

    @property
    def n_proj(self) -> int:
        return self.n_rot * len(self.tilts_deg)

    @property
    def n_coeff(self) -> int:
        return (self.ell_max // 2 + 1) * (self.ell_max + 1)

    @property
    def n_vox(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]


_T = (0.0, 15.0, 30.0, 45.0)
WORKLOADS = {
    "c1": Workload("c1", (32, 32, 32), 4, 15, 180.0, _T, 32, 32, 8, 14.0,
                   "twisted", 0.01, 1e-3, 1001, 2001),
    "c2": Workload("c2", (100, 100, 100), 8, 60, 360.0, _T, 100, 100, 8, 45.0,
                   "twisted", 0.01, 1e-3, 1002, 2002),
    "c3": Workload("c3", (128, 128, 128), 8, 75, 360.0, _T, 128, 128, 16, 57.0,
                   "twisted", 0.01, 1e-3, 1003, 2003),
    "c4": Workload("c4", (48, 48, 48), 6, 30, 360.0, _T, 64, 64, 8, 21.0,
                   "bundles", 0.01, 1e-3, 0, 100000),
    "c5": Workload("c5", (256, 256, 256), 8, 100, 360.0, _T, 256, 256, 16, 114.0,
                   "bundles", 0.0, 1e-3, 1005, 2005),
}


def lab_frame():
    """Lab-frame unit vectors (p, j, k, q0, q90, alpha_axis, beta_axis).

    The paper's standard frame (beam +z, rotation axis +y, tilt axis +x) turned
    by +90 deg about x, so that the rotation stage turns about z and the tilt
    stage about x: beam -y, raster j +z, raster k +x, detector origin +x,
    detector +90 deg +z, inner axis +z, outer axis +x.
    """
    return dict(
        p=(0.0, -1.0, 0.0), j=(0.0, 0.0, 1.0), k=(1.0, 0.0, 0.0),
        q0=(1.0, 0.0, 0.0), q90=(0.0, 0.0, 1.0),
        alpha=(0.0, 0.0, 1.0), beta=(1.0, 0.0, 0.0),
    )


def angles(w: Workload):
    """(inner, outer) angle arrays in radians, tilt-major projection order."""
    rot = np.arange(w.n_rot, dtype=np.float64) * (w.rot_span_deg / w.n_rot)
    inner = np.tile(rot, len(w.tilts_deg))
    outer = np.repeat(np.asarray(w.tilts_deg, dtype=np.float64), w.n_rot)
    return np.deg2rad(inner), np.deg2rad(outer)


def gaussian(shape, seed: int, dtype=np.float64):
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


def uniform(shape, seed: int, lo=0.0, hi=1.0, dtype=np.float64):
    return np.random.default_rng(seed).uniform(lo, hi, shape).astype(dtype)


def noise(shape, seed: int):
    """Unit-variance Gaussian noise; the caller scales it by sigma."""
    return np.random.default_rng(seed).standard_normal(shape)


def _centred_grid(n):
    ax = [np.arange(m, dtype=np.float64) - (m - 1) / 2.0 for m in n]
    return np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1)  # (nx,ny,nz,3)


def _unit(rng, k=None):
    v = rng.standard_normal((3,) if k is None else (k, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def twisted_fibre_field(w: Workload, seed: int | None = None):
    """Smoothly twisting fibre field inside a ball.

    Returns ``(direction[nx,ny,nz,3], degree[nx,ny,nz], density[nx,ny,nz])``.
    A twist axis ``a`` and a start direction ``n0`` (perpendicular to ``a``)
    are drawn uniformly; the fibre direction at voxel x turns in the plane
    perpendicular to ``a`` by (a . x) / N radians (1 rad across the volume).
    The degree of orientation is i.i.d. uniform on [0, 1]; density is 1 inside
    the ball of the workload's radius and 0 outside.
    """
    rng = np.random.default_rng(w.seed_phantom if seed is None else seed)
    a = _unit(rng)
    g = _unit(rng)
    n0 = g - (g @ a) * a
    n0 /= np.linalg.norm(n0)
    b = np.cross(a, n0)
    x = _centred_grid(w.n)
    theta = (x @ a) / float(max(w.n))
    direction = np.cos(theta)[..., None] * n0 + np.sin(theta)[..., None] * b
    degree = rng.uniform(0.0, 1.0, w.n)
    density = (np.linalg.norm(x, axis=-1) <= w.radius).astype(np.float64)
    return direction, degree, density


def bundle_params(w: Workload, seed: int | None = None):
    """Random parameters of the multi-bundle phantom.

    Returns a list of ``(axis[3], centre[3], radius, degree)``, one per bundle
    (1 to 3 bundles): axis uniform on the sphere, centre uniform in the ball of
    radius 0.2 N, radius uniform in [0.08 N, 0.2 N], degree of orientation
    uniform in [0, 1].
    """
    rng = np.random.default_rng(w.seed_phantom if seed is None else seed)
    N = float(max(w.n))
    k = int(rng.integers(1, 4))
    out = []
    for _ in range(k):
        axis = _unit(rng)
        u = _unit(rng)
        centre = u * (0.2 * N) * rng.uniform() ** (1.0 / 3.0)
        radius = rng.uniform(0.08 * N, 0.2 * N)
        degree = rng.uniform(0.0, 1.0)
        out.append((axis, centre, float(radius), float(degree)))
    return out


def multi_bundle_field(w: Workload, seed: int | None = None, background=0.1):
    """One to three straight cylindrical fibre bundles inside a ball.

    Returns ``(bundles, background_density)`` where ``bundles`` is a list of
    ``(direction[3], degree, mask[nx,ny,nz])`` and ``background_density`` is an
    isotropic density (``background`` inside the ball, 0 outside).  Bundle
    parameters as in ``bundle_params``; masks are clipped to the ball.
    """
    x = _centred_grid(w.n)
    ball = np.linalg.norm(x, axis=-1) <= w.radius
    bundles = []
    for axis, centre, radius, degree in bundle_params(w, seed):
        rel = x - centre
        along = rel @ axis
        perp = rel - along[..., None] * axis
        mask = (np.linalg.norm(perp, axis=-1) <= radius) & ball
        bundles.append((axis, degree, mask.astype(np.float64)))
    return bundles, background * ball.astype(np.float64)


def zh_lobe_weights(degree):
    """Legendre weights g_l of the fibre lobe (1 - d) + 5 d u^4 for l = 0, 2, 4.

    Plain polynomial bookkeeping of the phantom's shape: 5 u^4 equals
    P0 + (20/7) P2 + (8/7) P4, so the lobe is g0 P0 + g2 P2 + g4 P4 with
    g0 = 1, g2 = 20 d / 7, g4 = 8 d / 7.  Returned as an array of shape
    (..., 3).
    """
    d = np.asarray(degree, dtype=np.float64)
    return np.stack([np.ones_like(d), 20.0 * d / 7.0, 8.0 * d / 7.0], axis=-1)


def truncated_icosahedron_dirs():
    """Face-centre directions of the truncated icosahedron, one of each antipodal
    pair (16 directions): its 12 pentagons sit over the vertices of the regular
    icosahedron with vertices (0, +-1, +-g) and cyclic permutations (g the
    golden ratio), its 20 hexagons over that icosahedron's face centres.  A
    grid for the nearest-neighbour basis."""
    g = (1.0 + math.sqrt(5.0)) / 2.0
    ico = []
    for s1 in (1.0, -1.0):
        for s2 in (1.0, -1.0):
            base = (0.0, s1, s2 * g)
            for k in range(3):
                ico.append(base[k:] + base[:k])
    ico = np.array(ico)
    faces = []
    n = len(ico)
    for a in range(n):
        for b in range(a + 1, n):
            for c in range(b + 1, n):
                if all(abs(np.linalg.norm(ico[p] - ico[q]) - 2.0) < 1e-9 for p, q in ((a, b), (a, c), (b, c))):
                    faces.append(ico[[a, b, c]].mean(axis=0))
    v = np.concatenate([ico, np.array(faces)])
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    keep = []
    for p in v:  # one of each antipodal pair: first nonzero coordinate positive
        if p[np.flatnonzero(np.abs(p) > 1e-12)[0]] > 0:
            keep.append(p)
    return np.array(keep)


def hemisphere_dirs(n: int):
    """n directions spread over the upper hemisphere (golden-angle spiral in
    z = cos(theta) from 1 towards 0); a grid for the Gaussian-kernel basis."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (k + 0.5) / n
    r = np.sqrt(1.0 - z * z)
    phi = k * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)

