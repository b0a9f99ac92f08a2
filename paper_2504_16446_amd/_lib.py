"""ctypes binding of libtt_hip.so (argument marshalling only).

Every computation runs in the HIP library; this module converts Python
arguments to the C ABI of ``include/tt.h`` and raises on error codes.  There
is no fallback: if the library is missing, importing the package's GPU entry
points raises.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtt_hip.so")

TT_MAP_FP32, TT_MAP_BF16 = 0, 1
TT_PROJ_TRILINEAR, TT_PROJ_JOSEPH = 0, 1
TT_BASIS_SH, TT_BASIS_GK, TT_BASIS_NN = 0, 1, 2
REDUCE_WORK = 4096  # TT_REDUCE_WORK: float64 partials of a value reduction
KERNEL_CLASSES = ["map", "march", "fold", "backproject", "residual", "vector", "plan", "fused"]
_ERRORS = {-1: "EINVAL", -2: "ESHAPE", -3: "ENOMEM", -4: "EHIP", -5: "ENONFINITE", -6: "EUNSUPPORTED"}


class TTError(RuntimeError):
    def __init__(self, code, where, msg):
        super().__init__(f"{where}: TT_{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class Geometry(C.Structure):
    """Mirror of ``tt_geometry``."""
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("ell_max", C.c_int32), ("n_proj", C.c_int32),
        ("nj", C.c_int32), ("nk", C.c_int32), ("n_seg", C.c_int32), ("n_sub", C.c_int32),
        ("map_precision", C.c_int32),
        ("step", C.c_double), ("seg_span", C.c_double),
        ("inner_angle", C.POINTER(C.c_double)), ("outer_angle", C.POINTER(C.c_double)),
        ("j_offset", C.POINTER(C.c_double)), ("k_offset", C.POINTER(C.c_double)),
        ("p", C.c_double * 3), ("j", C.c_double * 3), ("k", C.c_double * 3),
        ("q0", C.c_double * 3), ("q90", C.c_double * 3),
        ("alpha_axis", C.c_double * 3), ("beta_axis", C.c_double * 3),
        ("basis", C.c_int32), ("n_dirs", C.c_int32), ("dirs", C.POINTER(C.c_double)),
        ("kernel_width", C.c_double),
    ]


_lib = None
_vp, _fp, _dp = C.c_void_p, C.c_void_p, C.c_void_p

# (name, restype, argtypes)
_SIGS = [
    ("tt_create", C.c_int, [C.POINTER(Geometry), C.POINTER(C.c_void_p)]),
    ("tt_destroy", None, [_vp]),
    ("tt_set_stream", C.c_int, [_vp, _vp]),
    ("tt_set_map_precision", C.c_int, [_vp, C.c_int]),
    ("tt_set_projector", C.c_int, [_vp, C.c_int]),
    ("tt_set_sparse_map", C.c_int, [_vp, C.c_int]),
    ("tt_num_coeffs", C.c_int, [C.c_int]),
    ("tt_sizes", C.c_int, [_vp, C.POINTER(C.c_int64)]),
    ("tt_basis_matrix", C.c_int, [_vp, C.POINTER(C.c_double)]),
    ("tt_ray_samples", C.c_int, [_vp, C.POINTER(C.c_int64)]),
    ("tt_geometry_basis", C.c_int, [C.POINTER(Geometry), C.POINTER(C.c_double)]),
    ("tt_sh_eval", C.c_int, [C.c_int, C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    ("tt_project", C.c_int, [_vp, _fp, _fp]),
    ("tt_adjoint", C.c_int, [_vp, _fp, _fp, C.c_float, _fp]),
    ("tt_loss_grad", C.c_int, [_vp, _fp, _fp, _fp, C.c_double, _dp, _fp, _fp]),
    ("tt_loss_grad_noalloc", C.c_int, [_vp, _fp, _fp, _fp, C.c_double, _dp, _fp, _fp]),
    ("tt_workspace_bytes", C.c_int64, [_vp, C.c_int]),
    ("tt_set_workspace", C.c_int, [_vp, _vp, C.c_size_t]),
    ("tt_lbfgs_workspace_bytes", C.c_int64, [_vp, C.c_int]),
    ("tt_lbfgs_create", C.c_int, [_vp, C.c_int, _vp, C.c_size_t, C.POINTER(C.c_void_p)]),
    ("tt_lbfgs_refresh", C.c_int, [_vp]),
    ("tt_normal_work_bytes", C.c_int64, [_vp]),
    ("tt_kappa", C.c_int, [_vp, C.c_double, _vp, C.c_size_t, C.POINTER(C.c_double)]),
    ("tt_voxel_preconditioner", C.c_int, [_vp, C.c_double, _fp, _vp, C.c_size_t]),
    ("tt_channel_stats_work_len", C.c_int64, []),
    ("tt_channel_stats", C.c_int, [_fp, C.c_int64, C.c_int, C.c_int, C.c_float, _fp, _fp, _dp, C.c_int64, _vp]),
    ("tt_lbfgs_destroy", None, [_vp]),
    ("tt_lbfgs_init", C.c_int, [_vp, _fp, _fp, _fp, C.c_double]),
    ("tt_lbfgs_step", C.c_int, [_vp]),
    ("tt_lbfgs_step_direction", C.c_int, [_vp, _fp]),
    ("tt_lbfgs_query", C.c_int, [_vp, C.POINTER(C.c_double)]),
    ("tt_lbfgs_run", C.c_int, [_vp, C.c_int, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int)]),
    ("tt_timing_enable", C.c_int, [_vp, C.c_int]),
    ("tt_timing_read", C.c_int, [_vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    ("tt_conv3d_weight_elems", C.c_int64, [C.c_int, C.c_int]),
    ("tt_conv3d_swizzle", C.c_int, [_fp, C.c_int, C.c_int, _vp, _vp, _vp]),
    ("tt_conv3d", C.c_int, [C.c_int, C.c_int, C.c_int, _vp, _vp, _fp, _vp, _vp, C.c_int, C.c_int, C.c_int,
                            C.c_int, _vp]),
    ("tt_conv3d_wgrad_work_bytes", C.c_size_t, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int]),
    ("tt_conv3d_wgrad", C.c_int, [C.c_int, C.c_int, _vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, _fp, C.c_size_t,
                                  _fp, _fp, _vp]),
    ("tt_adam", C.c_int, [_fp, _fp, _fp, _fp, C.c_int64, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, _vp]),
    ("tt_mse", C.c_int, [_fp, _fp, C.c_int64, C.c_int, C.c_int, C.c_float, _vp, _dp, _dp, C.c_int64, _vp]),
    ("tt_pack_bf16", C.c_int, [_fp, C.c_int64, C.c_int, C.c_int, C.c_float, _fp, _fp, _vp, _vp]),
    ("tt_tile_gather", C.c_int, [_fp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp, C.c_int, _vp,
                                 C.c_int, _vp, C.c_int, C.c_int, C.c_float, _fp, _fp, C.c_int, C.c_int, _vp, _vp]),
    ("tt_tile_blend", C.c_int, [_fp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, _vp, C.c_int, _vp, C.c_int, _vp,
                                C.c_int, C.c_int, C.c_int, C.c_int, _fp, _vp]),
    ("tt_tensor_properties", C.c_int, [_fp, C.c_int64, C.c_int, _fp, _vp]),
    ("tt_laplacian_reg", C.c_int, [_fp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, _fp, _fp, _dp, _dp,
                                   C.c_int64, _vp]),
    ("tt_huber_reg", C.c_int, [_fp, C.c_int64, C.c_double, C.c_double, _fp, _dp, _dp, C.c_int64, _vp]),
    ("tt_gd_step", C.c_int, [_fp, _fp, _fp, _fp, C.c_int64, C.c_float, C.c_float, _vp]),
    ("tt_huber_loss", C.c_int, [_fp, _fp, _fp, C.c_int64, C.c_double, _fp, _dp, _dp, C.c_int64, _vp]),
    ("tt_sumsq", C.c_int, [_fp, C.c_int64, C.c_double, _dp, _dp, C.c_int64, _vp]),
    ("tt_last_error", C.c_char_p, []),
    ("tt_error_string", C.c_char_p, [C.c_int]),
]
EXPORTED = [s[0] for s in _SIGS]


def lib():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2504_16446_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc, where):
    if rc < 0:
        raise TTError(rc, where, lib().tt_last_error().decode())
    return rc


def call(name, *args):
    return check(getattr(lib(), name)(*args), name)
