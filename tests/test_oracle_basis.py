"""Pins of the oracle's segment-averaged basis constants B_{s,c,i}.

Eq. projection_matrix of the paper: B_{sc,i} is the mean of B_i(R_s^T q(phi))
over detector segment c.  Pinned by the isotropic column, the Funk-Hecke
theorem, the antipodal symmetry of even orders, closed forms at zero angles
and the printed standard geometry (Table tab:geometry_vectors).
"""
import json
import os

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
from geoms import small, workload
import tt_inputs as synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _ell_of_index(ell_max):
    return np.concatenate([np.full(2 * l + 1, l) for l in range(0, ell_max + 1, 2)])


def test_isotropic_column():
    g = small(ell_max=8)
    B = g.B()
    assert np.abs(B[:, :, 0] - 1 / np.sqrt(4 * np.pi)).max() < 1e-15


@pytest.mark.parametrize("ell_max,n_seg", [(4, 8), (8, 8), (8, 16), (6, 8)])
def test_funk_hecke_segment_mean(ell_max, n_seg):
    # The 3*n_seg midpoint nodes are equispaced on the great circle
    # perpendicular to the beam, so their mean integrates the restriction of a
    # band-limited function exactly; Funk-Hecke gives P_l(0) Y_i(d_s).
    g = small(ell_max=ell_max, n_seg=n_seg)
    B = g.B()
    ells = _ell_of_index(ell_max)
    P0 = np.array([npleg.legval(0.0, np.eye(ell_max + 1)[l]) for l in ells])
    for s in range(g.n_proj):
        _, _, d, _ = oracle.frame(g, s)
        ref = P0 * oracle.sh(ell_max, d)
        assert np.abs(B[s].mean(axis=0) - ref).max() < 1e-13


def test_antipodal_segments_coincide():
    g = small(ell_max=8, n_seg=16)
    B = g.B()
    assert np.abs(B[:, 8:, :] - B[:, :8, :]).max() < 1e-13


def test_zero_angle_closed_form():
    # At alpha = beta = 0 the probed direction of sub-sample phi is
    # cos(phi) q0 + sin(phi) q90 = (cos phi, 0, sin phi) in the lab frame used
    # here; Y_20 = sqrt(5/(16 pi)) (3 z^2 - 1), Y_22 = sqrt(15/(16 pi)) (x^2 - y^2).
    g = oracle.Geometry((4, 4, 4), 2, [0.0], [0.0], 4, 4, 8, synth.lab_frame())
    B = g.B()[0]
    for c in range(8):
        phis = (c + (np.arange(3) + 0.5) / 3 - 0.5) * 2 * np.pi / 8
        x, z = np.cos(phis), np.sin(phis)
        assert abs(B[c, 3] - np.mean(np.sqrt(5 / (16 * np.pi)) * (3 * z * z - 1))) < 1e-15
        assert abs(B[c, 5] - np.mean(np.sqrt(15 / (16 * np.pi)) * x * x)) < 1e-15
        assert abs(B[c, 4] - np.mean(np.sqrt(15 / (4 * np.pi)) * x * z)) < 1e-15
        assert abs(B[c, 1]) < 1e-15 and abs(B[c, 2]) < 1e-15


def test_lab_frame_is_standard_table_turned_about_x():
    with open(os.path.join(GOLD, "geometry_vectors.json")) as f:
        table = json.load(f)
    Q = np.array([[1.0, 0, 0], [0, 0, -1], [0, 1, 0]])  # +90 deg about x
    ours = synth.lab_frame()
    for key in ("p", "j", "k", "q0", "q90", "alpha", "beta"):
        assert np.allclose(Q @ np.asarray(table[key], float), ours[key]), key
    # right-handed raster/beam triad in both frames
    assert np.allclose(np.cross(table["j"], table["k"]), -np.asarray(table["p"]))
    assert np.allclose(np.cross(ours["j"], ours["k"]), -np.asarray(ours["p"]))


def test_workload_projection_counts():
    for name, n in (("c1", 60), ("c2", 240), ("c3", 300), ("c4", 120), ("c5", 400)):
        assert synth.WORKLOADS[name].n_proj == n
    g = workload("c1")
    assert g.B().shape == (60, 8, 15)
