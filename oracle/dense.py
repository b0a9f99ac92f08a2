"""Brute-force dense system matrix for tiny volumes (test infrastructure).

Builds P_{sjk,xyz} by visiting every ray (s,j,k), every sample n along it and
every voxel of the grid, and evaluating the trilinear tent weight directly; no
neighbour search.  The system matrix is then assembled literally as the
paper's block-Kronecker form A = [P_s (x) B_s] stacked over s
(Eq. forward_model).  Only sensible for volumes of a few hundred voxels.
"""
from __future__ import annotations

import math

import numpy as np

from . import Geometry, frame


def voxel_centres(g: Geometry):
    ax = [np.arange(m, dtype=np.float64) - (m - 1) / 2.0 for m in g.n]
    X = np.stack(np.meshgrid(*ax, indexing="ij"), axis=-1)
    return X.reshape(-1, 3)


def dense_P(g: Geometry, s: int):
    """P[j*nk + k, voxel] for projection s (step included)."""
    ej, ek, d, o = frame(g, s)
    xv = voxel_centres(g)
    half = 0.5 * math.sqrt(sum(m * m for m in g.n)) + 2.0
    nl = int(math.ceil(half / g.step)) + 1
    P = np.zeros((g.nj * g.nk, xv.shape[0]))
    for j in range(g.nj):
        for k in range(g.nk):
            row = P[j * g.nk + k]
            for n in range(-nl, nl + 1):
                x = o + j * ej + k * ek + n * g.step * d
                t = np.clip(1.0 - np.abs(xv - x), 0.0, None)
                row += g.step * t.prod(axis=1)
    return P


def dense_A(g: Geometry):
    B = g.B()  # the basis constants in use (exact, or their sparse approximation)
    blocks = [np.kron(dense_P(g, s), B[s]) for s in range(g.n_proj)]
    return np.vstack(blocks)
