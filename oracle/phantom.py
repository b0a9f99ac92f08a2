"""Phantom coefficients and noisy data computed with the oracle (test infrastructure).

The fibre lobe (1 - d) + 5 d (n . q)^4 is zonal about the fibre direction n,
so by the spherical-harmonic addition theorem its coefficients are
c_lm = rho g_l 4 pi / (2l + 1) Y_lm(n) with the Legendre weights g_l of the
lobe (g_0 = 1, g_2 = 20 d / 7, g_4 = 8 d / 7, higher orders 0).
"""
from __future__ import annotations

import numpy as np

import tt_inputs as synth

from . import Geometry, project, sh


def _ell_of_index(ell_max):
    return np.concatenate([np.full(2 * l + 1, l) for l in range(0, ell_max + 1, 2)])


def lobe_coeffs(ell_max, direction, weights):
    """Coefficients of sum_l weights[..., l/2] P_l(n . q) for l = 0, 2, 4."""
    Y = sh(ell_max, direction)
    ells = _ell_of_index(ell_max)
    fac = np.zeros(Y.shape)
    for idx, l in enumerate((0, 2, 4)):
        if l > ell_max:
            break
        sel = ells == l
        fac[..., sel] = (weights[..., idx] * 4.0 * np.pi / (2 * l + 1))[..., None]
    return fac * Y


def phantom_coeffs(w: synth.Workload, seed=None):
    if w.phantom == "twisted":
        direction, degree, density = synth.twisted_fibre_field(w, seed)
        c = lobe_coeffs(w.ell_max, direction, synth.zh_lobe_weights(degree))
        return c * density[..., None]
    bundles, bg = synth.multi_bundle_field(w, seed)
    C = w.n_coeff
    c = np.zeros(w.n + (C,))
    for axis, degree, mask in bundles:
        cb = lobe_coeffs(w.ell_max, axis[None], synth.zh_lobe_weights(np.array([degree])))[0]
        c += mask[..., None] * cb
    iso = np.zeros(C)
    iso[0] = np.sqrt(4.0 * np.pi)  # spherical mean 1
    return c + bg[..., None] * iso


def noisy_data(g: Geometry, w: synth.Workload, c):
    clean = project(g, c)
    if w.noise <= 0:
        return clean, clean
    sigma = w.noise * np.abs(clean).max()
    return clean + sigma * synth.noise(clean.shape, w.seed_noise), clean
