"""Shared helpers: oracle geometry <-> GPU projector, error metrics."""
import numpy as np


def rel_l2(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def rel_max(got, ref):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def gpu_projector(og, **kw):
    """Projector with exactly the oracle geometry's parameters."""
    from paper_2504_16446_amd.projector import Projector
    if getattr(og, "basis", "sh") != "sh":
        kw.setdefault("basis", og.basis)
        kw.setdefault("dirs", og.dirs)
        kw.setdefault("width", og.width)
    if getattr(og, "model", "trilinear") != "trilinear":
        kw.setdefault("model", og.model)
    return Projector(og.n, og.ell_max, og.inner, og.outer, og.nj, og.nk, og.n_seg,
                     frame=og.frame, n_sub=og.n_sub, step=og.step, seg_span=og.seg_span,
                     joff=og.joff, koff=og.koff, **kw)


def geometry_struct(og, precision=0):
    """ctypes tt_geometry for an oracle geometry (host-only calls)."""
    import ctypes as C
    from paper_2504_16446_amd._lib import Geometry
    g = Geometry()
    g.nx, g.ny, g.nz = og.n
    g.ell_max, g.n_proj = og.ell_max, og.n_proj
    g.nj, g.nk, g.n_seg, g.n_sub = og.nj, og.nk, og.n_seg, og.n_sub
    g.map_precision = precision
    g.step, g.seg_span = og.step, og.seg_span
    P = C.POINTER(C.c_double)
    g.inner_angle = og.inner.ctypes.data_as(P)
    g.outer_angle = og.outer.ctypes.data_as(P)
    g.j_offset = og.joff.ctypes.data_as(P) if og.joff is not None else None
    g.k_offset = og.koff.ctypes.data_as(P) if og.koff is not None else None
    for field, key in (("p", "p"), ("j", "j"), ("k", "k"), ("q0", "q0"), ("q90", "q90"),
                       ("alpha_axis", "alpha"), ("beta_axis", "beta")):
        getattr(g, field)[:] = og.frame[key]
    if getattr(og, "basis", "sh") != "sh":
        g.basis = {"gk": 1, "nn": 2}[og.basis]
        g.n_dirs = og.dirs.shape[0]
        g.dirs = og.dirs.ctypes.data_as(P)
        g.kernel_width = og.width or 0.0
    return g
