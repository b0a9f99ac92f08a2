"""Host-side checks of the HIP library (no GPU needed).

The library loads and exports every function declared in include/tt.h; its
own float64 spherical harmonics and basis constants (an implementation
independent of the oracle's) agree with the oracle; invalid arguments give
error codes instead of crashes.
"""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle
from geoms import small, tiny
from helpers import geometry_struct

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2504_16446_amd import _lib
    return _lib


def test_exports_every_header_symbol():
    L = _lib()
    lib = L.lib()
    with open(os.path.join(ROOT, "include", "tt.h")) as f:
        text = f.read()
    names = set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(tt_[a-z_0-9]+)\s*\(", text, re.M))
    assert len(names) >= 20, names
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(L.EXPORTED) <= names | {"tt_lbfgs_destroy"}


@pytest.mark.parametrize("ell_max", [0, 2, 4, 8, 12, 16])
def test_sh_matches_oracle(ell_max):
    from paper_2504_16446_amd.projector import sh_eval
    rng = np.random.default_rng(ell_max + 100)
    d = rng.standard_normal((300, 3))
    d[:2] = [[0, 0, 1.0], [0, 0, -2.0]]  # both poles
    assert np.abs(sh_eval(ell_max, d) - oracle.sh(ell_max, d)).max() < 1e-12


@pytest.mark.parametrize("kw", [dict(), dict(n_seg=16, ell_max=8), dict(offsets=True)])
def test_basis_matrix_matches_oracle(kw):
    og = small(**{k: v for k, v in kw.items() if k != "offsets"}) if "offsets" not in kw else tiny(offsets=True)
    g = geometry_struct(og)
    B = np.empty((og.n_proj, og.n_seg, og.n_coeff))
    _lib().call("tt_geometry_basis", C.byref(g), B.ctypes.data_as(C.POINTER(C.c_double)))
    assert np.abs(B - og.B()).max() < 1e-13


def test_error_codes_without_device():
    L = _lib()
    og = tiny()
    B = np.empty((og.n_proj, og.n_seg, og.n_coeff))
    Bp = B.ctypes.data_as(C.POINTER(C.c_double))
    lib = L.lib()
    for field, val, code in (("ell_max", 3, -1), ("ell_max", 18, -6), ("nx", 0, -2), ("n_seg", 0, -1),
                             ("n_sub", 0, -1), ("step", 0.0, -1), ("step", float("nan"), -1),
                             ("map_precision", 7, -1)):
        g = geometry_struct(og)
        setattr(g, field, val)
        assert lib.tt_geometry_basis(C.byref(g), Bp) == code, (field, val)
        assert len(lib.tt_last_error()) > 0
    g = geometry_struct(og)
    g.p[:] = [0.0, 0.0, 1.0]  # not orthogonal to j = +z
    assert lib.tt_geometry_basis(C.byref(g), Bp) == -1
    g = geometry_struct(og)
    g.inner_angle = None
    assert lib.tt_geometry_basis(C.byref(g), Bp) == -1
    assert lib.tt_geometry_basis(None, Bp) == -1
    assert lib.tt_sh_eval(3, 1, None, None) == -1
    assert lib.tt_num_coeffs(8) == 45 and lib.tt_num_coeffs(-2) == -1
    h = C.c_void_p()
    assert lib.tt_create(None, C.byref(h)) == -1 and not h.value
    assert lib.tt_project(None, None, None) == -1
    assert lib.tt_adjoint(None, None, None, C.c_float(0), None) == -1
    assert lib.tt_lbfgs_step(None) == -1
    assert lib.tt_loss_grad_noalloc(None, None, None, None, C.c_double(0.0), None, None, None) == -1
    assert lib.tt_error_string(-5) == b"non-finite value"


def test_product_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_2504_16446_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "tt_oracle" not in text, f


def test_oracle_never_imports_product():
    # the oracle shares only the seeded input generators (tt_inputs) with the product
    for dirpath, _, files in os.walk(os.path.join(ROOT, "oracle")):
        for f in files:
            if f.endswith((".py", ".c", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "paper_2504_16446_amd" not in text and "libtt_hip" not in text, f
    text = open(os.path.join(ROOT, "tt_inputs.py")).read()
    assert "paper_2504_16446_amd" not in text and "import oracle" not in text


def test_tensor_properties_argument_errors_without_device():
    lib = _lib().lib()
    buf = (C.c_float * 64)()
    p = C.cast(buf, C.c_void_p)
    assert lib.tt_tensor_properties(None, 1, 2, p, None) == -1
    assert lib.tt_tensor_properties(None, 0, 2, None, None) == 0
    assert lib.tt_tensor_properties(p, 1, 3, p, None) == -1
    assert lib.tt_tensor_properties(p, 1, 18, p, None) == -6
    assert lib.tt_tensor_properties(p, -1, 2, p, None) == -2
    assert lib.tt_tensor_properties(p, 0, 2, p, None) == 0
    odd = C.c_void_p(C.addressof(buf) + 4)
    assert lib.tt_tensor_properties(odd, 1, 2, p, None) == -1


def test_regulariser_argument_errors_without_device():
    lib = _lib().lib()
    buf = (C.c_float * 64)()
    p = C.cast(buf, C.c_void_p)
    d = (C.c_double * 1)()
    dp = C.cast(d, C.c_void_p)
    assert lib.tt_laplacian_reg(None, 2, 2, 2, 1, 1.0, p, p, None, None, 0, None) == -1
    assert lib.tt_laplacian_reg(p, 0, 2, 2, 1, 1.0, p, p, None, None, 0, None) == -2
    assert lib.tt_laplacian_reg(p, 2, 2, 2, 1, float("nan"), p, p, None, None, 0, None) == -1
    assert lib.tt_laplacian_reg(p, 2, 2, 2, 1025, 1.0, p, p, None, None, 0, None) == -6  # more coefficients than supported
    assert lib.tt_laplacian_reg(p, 2, 2, 2, 1, 1.0, p, p, dp, dp, 4095, None) == -1  # partials too short for a value
    assert lib.tt_huber_reg(p, 4, 0.0, 1.0, p, None, None, 0, None) == -1
    assert lib.tt_huber_reg(p, -1, 0.1, 1.0, p, None, None, 0, None) == -2
    assert lib.tt_huber_reg(None, 0, 0.1, 1.0, None, None, None, 0, None) == 0
    assert lib.tt_huber_reg(p, 4, 0.1, 1.0, p, dp, None, 0, None) == -1  # a value needs partials
    assert lib.tt_gd_step(p, p, None, None, 4, 0.1, 0.0, None) == -1
    assert lib.tt_gd_step(p, p, p, None, 4, float("inf"), 0.0, None) == -1
    assert lib.tt_gd_step(None, None, None, None, 0, 0.1, 0.0, None) == 0


def test_huber_loss_argument_errors_without_device():
    lib = _lib().lib()
    buf = (C.c_float * 64)()
    p = C.cast(buf, C.c_void_p)
    d = (C.c_double * 1)()
    dp = C.cast(d, C.c_void_p)
    assert lib.tt_huber_loss(p, p, None, 4, 0.0, p, dp, dp, 4096, None) == -1
    assert lib.tt_huber_loss(None, p, None, 4, 0.5, p, dp, dp, 4096, None) == -1
    assert lib.tt_huber_loss(None, None, None, 0, 0.5, None, None, None, 0, None) == 0
    assert lib.tt_sumsq(p, 4, 1.0, None, dp, 4096, None) == -1
    assert lib.tt_sumsq(p, -2, 1.0, dp, dp, 4096, None) == -2
    assert lib.tt_sumsq(p, 4, 1.0, dp, None, 0, None) == -1


def test_create_rejects_orders_above_twelve_without_device():
    L = _lib()
    lib = L.lib()
    og = tiny(ell_max=14)
    g = geometry_struct(og)
    h = C.c_void_p()
    assert lib.tt_create(C.byref(g), C.byref(h)) == -6
    assert h.value is None


@pytest.mark.parametrize("basis,width", [("gk", 0.35), ("nn", None)])
def test_kernel_basis_matrix_matches_oracle(basis, width):
    import tt_inputs as _s
    dirs = _s.hemisphere_dirs(20) if basis == "gk" else _s.truncated_icosahedron_dirs()
    og = oracle.Geometry((6, 7, 5), 0, *geoms_tilted(), 9, 8, 8, _s.lab_frame(), basis=basis, dirs=dirs,
                         width=width)
    g = geometry_struct(og)
    B = np.empty((og.n_proj, og.n_seg, og.n_coeff))
    _lib().call("tt_geometry_basis", C.byref(g), B.ctypes.data_as(C.POINTER(C.c_double)))
    ref = og.B()
    if basis == "nn":
        # both sides pick the nearest grid direction; ties cannot occur at these nodes
        assert np.array_equal(B, ref)
    else:
        assert np.abs(B - ref).max() < 1e-13


def geoms_tilted():
    from geoms import tilted_angles
    return tilted_angles(4, (0.0, 25.0, 45.0), span_deg=360.0)


def test_kernel_basis_argument_errors_without_device():
    og = tiny()
    g = geometry_struct(og)
    B = np.empty(4096)
    Bp = B.ctypes.data_as(C.POINTER(C.c_double))
    lib = _lib().lib()
    g.basis = 1
    g.n_dirs = 0
    assert lib.tt_geometry_basis(C.byref(g), Bp) == -1
    d = np.array([[0.0, 0.0, 1.0]] * 3)
    g.n_dirs, g.dirs = 3, d.ctypes.data_as(C.POINTER(C.c_double))
    g.kernel_width = 0.0
    assert lib.tt_geometry_basis(C.byref(g), Bp) == -1
    g.kernel_width = 0.3
    assert lib.tt_geometry_basis(C.byref(g), Bp) == 0
    g.basis = 7
    assert lib.tt_geometry_basis(C.byref(g), Bp) == -1
