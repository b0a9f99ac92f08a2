"""Phantom coefficients from the seeded fibre fields, using the library's SH.

The fibre lobe (1 - d) + 5 d (n . q)^4 is zonal about the fibre direction n;
by the spherical-harmonic addition theorem its coefficients are
c_lm = rho g_l 4 pi / (2 l + 1) Y_lm(n), with the Legendre weights g_l of
the lobe (synth.zh_lobe_weights).  Multi-bundle phantoms sum one lobe per
bundle plus an isotropic background.
"""
from __future__ import annotations

import numpy as np

import tt_inputs as synth
from .projector import sh_eval


def _ell_of_index(ell_max):
    return np.concatenate([np.full(2 * l + 1, l) for l in range(0, ell_max + 1, 2)])


def _lobe(ell_max, direction, weights):
    Y = sh_eval(ell_max, direction)
    ells = _ell_of_index(ell_max)
    scale = np.zeros(Y.shape)
    for slot, l in enumerate((0, 2, 4)):
        if l <= ell_max:
            scale[..., ells == l] = (weights[..., slot] * 4.0 * np.pi / (2 * l + 1))[..., None]
    return scale * Y


def coefficients(w: synth.Workload, seed=None, dtype=np.float32):
    """SH coefficients [nx, ny, nz, C] of the workload's phantom."""
    if w.phantom == "twisted":
        direction, degree, density = synth.twisted_fibre_field(w, seed)
        c = _lobe(w.ell_max, direction, synth.zh_lobe_weights(degree)) * density[..., None]
        return c.astype(dtype)
    bundles, background = synth.multi_bundle_field(w, seed)
    c = np.zeros(w.n + (w.n_coeff,), dtype=dtype)
    for axis, degree, mask in bundles:
        lobe = _lobe(w.ell_max, axis[None], synth.zh_lobe_weights(np.array([degree])))[0]
        c += (mask[..., None] * lobe).astype(dtype)
    c[..., 0] += (background * np.sqrt(4.0 * np.pi)).astype(dtype)
    return c
