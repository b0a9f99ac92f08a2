"""Pins of the oracle's sparse approximation of the basis constants (the
sparse variant of the asynchronous pipelines, sect. "Pipelines").

* k at least the number of basis functions keeps B exactly; the
  nearest-neighbour basis has at most n_sub nonzeros per segment, so
  k = n_sub keeps it exactly;
* selection: a row keeps at most k entries, each equal to B's, and no
  dropped magnitude exceeds a kept one; on rows without near ties the kept
  set is that of a stable sort of -|B| (library special case); exact and
  near ties go to the lower index (hand-made rows);
* the operator: a field with a single nonzero basis channel i projects, in
  segment (s, c), to the exact projection when i is kept for (s, c) and to
  zero when it is dropped; the dense system matrix built literally from the
  approximated constants reproduces forward and adjoint;
  <Ax, y> = <x, A^T y>.
"""
import numpy as np
import pytest

import oracle
from oracle.dense import dense_A
from geoms import tilted_angles
import tt_inputs as synth


def _sh_geom(ell_max=4, n=(5, 6, 4), n_seg=8, sparse_k=0):
    inner, outer = tilted_angles(3, (0.0, 30.0))
    return oracle.Geometry(n, ell_max, inner, outer, 7, 6, n_seg, synth.lab_frame(), sparse_k=sparse_k)


def test_full_k_keeps_everything():
    B = _sh_geom(ell_max=6).B()
    C = B.shape[-1]
    assert np.array_equal(oracle.sparse_basis(B, C), B)
    assert np.array_equal(oracle.sparse_basis(B, C + 5), B)


def test_nearest_neighbour_basis_is_kept_exactly_at_n_sub():
    inner, outer = tilted_angles(4, (0.0, 25.0, 45.0), span_deg=360.0)
    g = oracle.Geometry((4, 5, 3), 0, inner, outer, 6, 5, 8, synth.lab_frame(), basis="nn",
                        dirs=synth.truncated_icosahedron_dirs())
    B = g.B()
    assert (np.count_nonzero(B, axis=-1) <= g.n_sub).all()
    assert np.array_equal(oracle.sparse_basis(B, g.n_sub), B)
    # k = 1 keeps each row's largest share (a multiple of 1 / n_sub)
    B1 = oracle.sparse_basis(B, 1)
    assert np.array_equal(B1.max(axis=-1), B.max(axis=-1))
    assert (np.count_nonzero(B1, axis=-1) == 1).all()


@pytest.mark.parametrize("k", [1, 2, 3, 7, 14])
def test_selection_properties_on_spherical_harmonic_rows(k):
    B = _sh_geom(ell_max=4).B()
    Bt = oracle.sparse_basis(B, k)
    kept = Bt != 0
    assert (kept.sum(axis=-1) <= k).all()
    assert np.array_equal(Bt[kept], B[kept])
    mag = np.abs(B)
    scale = mag.max(axis=-1)
    for r in range(B.shape[0] * B.shape[1]):
        s, c = divmod(r, B.shape[1])
        sel = kept[s, c]
        if sel.all() or not sel.any():
            continue
        assert mag[s, c][sel].min() >= mag[s, c][~sel].max() - oracle.SPARSE_TIE * scale[s, c]


def test_selection_equals_stable_sort_without_ties():
    rng = np.random.default_rng(11)
    B = rng.standard_normal((3, 4, 15))
    for k in range(1, 16):
        Bt = oracle.sparse_basis(B, k)
        ref = np.zeros_like(B)
        for s in range(3):
            for c in range(4):
                idx = np.argsort(-np.abs(B[s, c]), kind="stable")[:k]
                ref[s, c, idx] = B[s, c, idx]
        assert np.array_equal(Bt, ref)


def test_ties_go_to_the_lower_index():
    row = np.array([[[0.5, -0.5, 0.2, 0.5]]])
    assert np.array_equal(oracle.sparse_basis(row, 1), [[[0.5, 0.0, 0.0, 0.0]]])
    assert np.array_equal(oracle.sparse_basis(row, 2), [[[0.5, -0.5, 0.0, 0.0]]])
    assert np.array_equal(oracle.sparse_basis(row, 3), [[[0.5, -0.5, 0.0, 0.5]]])
    near = np.array([[[-0.3, 0.1, 0.3 + 1e-12]]])
    assert np.array_equal(oracle.sparse_basis(near, 1), [[[-0.3, 0.0, 0.0]]])
    apart = np.array([[[-0.3, 0.1, 0.3 + 1e-6]]])
    assert np.array_equal(oracle.sparse_basis(apart, 1), [[[0.0, 0.0, 0.3 + 1e-6]]])


@pytest.mark.parametrize("i", [0, 3, 9, 14])
def test_single_channel_field_routes_kept_entries(i):
    k = 3
    g = _sh_geom(ell_max=4)
    gs = _sh_geom(ell_max=4, sparse_k=k)
    rng = np.random.default_rng(i)
    c = np.zeros(g.vol_shape)
    c[..., i] = rng.standard_normal(g.n)
    I = oracle.project(g, c)
    Is = oracle.project(gs, c)
    kept = gs.B()[:, :, i] != 0  # [S, n_seg]
    assert kept.any() and (~kept).any()
    scale = np.abs(I).max()
    for s in range(g.n_proj):
        for cs in range(g.n_seg):
            ref = I[s, :, :, cs] if kept[s, cs] else 0.0
            assert np.abs(Is[s, :, :, cs] - ref).max() <= 1e-13 * scale


def test_dense_matrix_and_adjoint_identity():
    gs = _sh_geom(ell_max=2, n=(4, 3, 5), sparse_k=2)
    A = dense_A(gs)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(gs.vol_shape)
    y = rng.standard_normal(gs.data_shape)
    Ax = oracle.project(gs, x)
    Aty = oracle.adjoint(gs, y)
    assert np.abs(A @ x.ravel() - Ax.ravel()).max() <= 1e-13 * np.abs(Ax).max()
    assert np.abs(A.T @ y.ravel() - Aty.ravel()).max() <= 1e-13 * np.abs(Aty).max()
    gap = abs(np.dot(Ax.ravel(), y.ravel()) - np.dot(x.ravel(), Aty.ravel()))
    assert gap <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)
