"""FP64 CPU oracle for the tensor-tomography hot path (test infrastructure).

Only the test-suite, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg use this package.  It wraps ``tt_oracle.c`` (plain C, FP64,
written from the paper's equations) through ctypes and shares nothing with the
GPU library.  See ``tt_oracle.c`` for the equations each function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Private volumes of the threaded adjoint are limited to this many bytes.
MEM_BUDGET = float(os.environ.get("TT_ORACLE_MEM", 8e9))


def build(force: bool = True) -> str:
    """Compile the oracle with the host C compiler (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)


class Geom(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("ell_max", C.c_int32), ("n_proj", C.c_int32),
        ("nj", C.c_int32), ("nk", C.c_int32), ("n_seg", C.c_int32), ("n_sub", C.c_int32),
        ("model", C.c_int32),
        ("step", C.c_double), ("seg_span", C.c_double),
        ("inner", _dp), ("outer", _dp), ("joff", _dp), ("koff", _dp),
        ("p", C.c_double * 3), ("j", C.c_double * 3), ("k", C.c_double * 3),
        ("q0", C.c_double * 3), ("q90", C.c_double * 3),
        ("alpha", C.c_double * 3), ("beta", C.c_double * 3),
        ("basis", C.c_int32), ("n_dirs", C.c_int32), ("dirs", _dp), ("width", C.c_double),
    ]


def _declare(L):
    L.og_num_coeffs.argtypes = [C.c_int]
    L.og_num_coeffs.restype = C.c_int
    L.og_legendre.argtypes = [C.c_int, C.c_int, C.c_double]
    L.og_legendre.restype = C.c_double
    L.og_sh_batch.argtypes = [C.c_int, C.c_int64, _dp, _dp]
    L.og_rotation.argtypes = [C.POINTER(Geom), C.c_int, _dp]
    L.og_projection_frame.argtypes = [C.POINTER(Geom), C.c_int, _dp]
    L.og_basis_matrix.argtypes = [C.POINTER(Geom), _dp]
    L.og_project.argtypes = [C.POINTER(Geom), _dp, _dp, _dp]
    L.og_project_rays.argtypes = [C.POINTER(Geom), _dp, _dp, C.c_int64, _ip, _dp]
    L.og_adjoint.argtypes = [C.POINTER(Geom), _dp, _dp, _dp, C.c_double]
    L.og_adjoint_voxels.argtypes = [C.POINTER(Geom), _dp, _dp, C.c_int64, _ip, _dp]
    L.og_loss_grad.argtypes = [C.POINTER(Geom), _dp, _dp, _dp, _dp, C.c_double, _dp, _dp,
                               C.c_double]
    L.og_loss_grad.restype = C.c_double
    L.og_lbfgs.argtypes = [C.POINTER(Geom), _dp, _dp, _dp, _dp, C.c_double, C.c_int, C.c_int,
                           C.c_double, _dp, _dp, C.c_double]
    L.og_lbfgs.restype = C.c_int
    L.og_max_threads.restype = C.c_int
    L.og_splat_projection.argtypes = [C.POINTER(Geom), C.c_int, _dp, C.c_int, _dp]


def _p(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_coeffs(ell_max: int) -> int:
    return (ell_max // 2 + 1) * (ell_max + 1)


def max_threads() -> int:
    return lib().og_max_threads()


class Geometry:
    """Acquisition geometry; keeps the angle arrays alive for the C struct."""

    def __init__(self, n, ell_max, inner, outer, nj, nk, n_seg, frame, n_sub=3, step=1.0,
                 seg_span=2 * np.pi, joff=None, koff=None, model="trilinear", basis="sh", dirs=None,
                 width=None, sparse_k=0):
        self.n = tuple(int(v) for v in n)
        self.ell_max = int(ell_max)
        self.inner = _f64(inner)
        self.outer = _f64(outer)
        self.joff = None if joff is None else _f64(joff)
        self.koff = None if koff is None else _f64(koff)
        self.nj, self.nk, self.n_seg, self.n_sub = int(nj), int(nk), int(n_seg), int(n_sub)
        self.step, self.seg_span = float(step), float(seg_span)
        self.frame = {k: tuple(float(x) for x in v) for k, v in frame.items()}
        if model not in ("trilinear", "joseph"):
            raise ValueError("model must be 'trilinear' or 'joseph'")
        self.model = model
        if basis not in ("sh", "gk", "nn"):
            raise ValueError("basis must be 'sh', 'gk' or 'nn'")
        self.basis = basis
        self.dirs = None if basis == "sh" else _f64(dirs).reshape(-1, 3)
        self.width = None if basis != "gk" else float(width)
        g = Geom()
        g.model = 1 if model == "joseph" else 0
        g.basis = {"sh": 0, "gk": 1, "nn": 2}[basis]
        if basis != "sh":
            g.n_dirs = self.dirs.shape[0]
            g.dirs = _p(self.dirs)
            g.width = self.width if basis == "gk" else 0.0
        g.nx, g.ny, g.nz = self.n
        g.ell_max = self.ell_max
        g.n_proj = len(self.inner)
        g.nj, g.nk, g.n_seg, g.n_sub = self.nj, self.nk, self.n_seg, self.n_sub
        g.step, g.seg_span = self.step, self.seg_span
        g.inner, g.outer = _p(self.inner), _p(self.outer)
        g.joff, g.koff = _p(self.joff), _p(self.koff)
        for name, field in (("p", "p"), ("j", "j"), ("k", "k"), ("q0", "q0"), ("q90", "q90"),
                            ("alpha", "alpha"), ("beta", "beta")):
            getattr(g, field)[:] = self.frame[name]
        self._g = g
        self._B = None
        if sparse_k < 0:
            raise ValueError("sparse_k must be >= 0 (0: the exact basis constants)")
        self.sparse_k = int(sparse_k)

    @classmethod
    def from_workload(cls, w, **kw):
        import tt_inputs as synth
        inner, outer = synth.angles(w)
        args = dict(n=w.n, ell_max=w.ell_max, inner=inner, outer=outer, nj=w.nj, nk=w.nk,
                    n_seg=w.n_seg, frame=synth.lab_frame(), n_sub=w.n_sub, step=w.step)
        args.update(kw)
        return cls(**args)

    @property
    def n_proj(self):
        return len(self.inner)

    @property
    def n_coeff(self):
        return num_coeffs(self.ell_max) if self.basis == "sh" else self.dirs.shape[0]

    @property
    def vol_shape(self):
        return self.n + (self.n_coeff,)

    @property
    def data_shape(self):
        return (self.n_proj, self.nj, self.nk, self.n_seg)

    def ref(self):
        return C.byref(self._g)

    def B(self):
        """Basis constants in use: the exact B, or its sparse approximation
        when ``sparse_k`` > 0 (see ``sparse_basis``)."""
        if self._B is None:
            B = basis_matrix(self)
            self._B = sparse_basis(B, self.sparse_k) if self.sparse_k > 0 else B
        return self._B


def legendre(l, m, x):
    return lib().og_legendre(int(l), int(m), float(x))


def sh(ell_max, dirs):
    d = _f64(dirs).reshape(-1, 3)
    out = np.empty((d.shape[0], num_coeffs(ell_max)))
    lib().og_sh_batch(int(ell_max), d.shape[0], _p(d), _p(out))
    return out.reshape(np.shape(dirs)[:-1] + (num_coeffs(ell_max),))


def rotation(g: Geometry, s: int):
    R = np.empty(9)
    lib().og_rotation(g.ref(), int(s), _p(R))
    return R.reshape(3, 3)


def frame(g: Geometry, s: int):
    """(e_j, e_k, d, o) of projection s in centred sample coordinates."""
    f = np.empty(12)
    lib().og_projection_frame(g.ref(), int(s), _p(f))
    return f[0:3], f[3:6], f[6:9], f[9:12]


def basis_matrix(g: Geometry):
    B = np.empty((g.n_proj, g.n_seg, g.n_coeff))
    lib().og_basis_matrix(g.ref(), _p(B))
    return B


SPARSE_TIE = 1e-9


def sparse_basis(B, k, tie=SPARSE_TIE):
    """Sparse approximation of the basis constants (the sparse variant of the
    asynchronous pipelines, sect. "Pipelines": the reciprocal-space map is
    replaced by a sparse approximation so that it can be applied inside the
    ray sum).  The paper names the approximation without a rule; the reading
    used here: in every row (projection s, segment c) of B, keep the k entries
    of largest magnitude and set the others to zero.  Entries are taken one
    at a time: the largest remaining magnitude m is found, and among the
    remaining entries with |B| >= m - tie * max|row| the lowest index is
    kept (so exact and near ties go to the lower basis index).  k >= the row
    length keeps the whole row."""
    B = np.asarray(B, dtype=np.float64)
    out = np.zeros_like(B)
    C = B.shape[-1]
    rows = B.reshape(-1, C)
    res = out.reshape(-1, C)
    for r in range(rows.shape[0]):
        row = rows[r]
        mag = np.abs(row)
        scale = mag.max()
        left = list(range(C))
        for _ in range(min(int(k), C)):
            m = max(mag[i] for i in left)
            pick = min(i for i in left if mag[i] >= m - tie * scale)
            res[r, pick] = row[pick]
            left.remove(pick)
    return out


def project(g: Geometry, c, B=None):
    """I = A c; B overrides the basis constants (shape n_proj x n_seg x C)."""
    c = _f64(c)
    assert c.shape == g.vol_shape, (c.shape, g.vol_shape)
    B = g.B() if B is None else _f64(B)
    assert B.shape == (g.n_proj, g.n_seg, g.n_coeff)
    out = np.empty(g.data_shape)
    lib().og_project(g.ref(), _p(B), _p(c), _p(out))
    return out


def splat_projection(g: Geometry, s: int, yf):
    """Q[x, y, z, u] = sum over rays and samples of projection s of step * T * yf[j, k, u]."""
    yf = _f64(yf)
    nu = yf.shape[-1]
    assert yf.shape == (g.nj, g.nk, nu)
    Q = np.empty(g.n + (nu,))
    lib().og_splat_projection(g.ref(), int(s), _p(yf), int(nu), _p(Q))
    return Q


def bf16(x):
    """Round to bfloat16 (nearest even) through float32, returned as float64."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unique_segments(g: Geometry):
    """Number of distinct segments: n_seg / 2 when the segments cover the full
    circle (even orders make antipodal segments equal), else n_seg."""
    full = abs(g.seg_span - 2 * np.pi) < 1e-12 and g.n_seg % 2 == 0
    return g.n_seg // 2 if full else g.n_seg


def adjoint_segment_first(g: Geometry, y, round_q=None, round_b=None):
    """Adjoint evaluated as sum_s B_s^T Q_s with Q_s the splat of the folded y.

    ``round_q`` / ``round_b`` (e.g. ``bf16``) are applied to Q_s and to the
    unique-segment basis constants before the contraction, which reproduces
    the rounding points of a reduced-precision map."""
    y = _f64(y)
    U = unique_segments(g)
    yf = np.zeros(g.data_shape[:3] + (U,))
    for cseg in range(g.n_seg):
        yf[..., cseg % U] += y[..., cseg]
    Bu = g.B()[:, :U, :]
    if round_b is not None:
        Bu = round_b(Bu)
    out = np.zeros(g.vol_shape)
    for s in range(g.n_proj):
        Q = splat_projection(g, s, yf[s])
        if round_q is not None:
            Q = round_q(Q)
        out += Q @ Bu[s]
    return out


def project_rays(g: Geometry, c, sjk):
    c = _f64(c)
    idx = np.ascontiguousarray(sjk, dtype=np.int32).reshape(-1, 3)
    out = np.empty((idx.shape[0], g.n_seg))
    lib().og_project_rays(g.ref(), _p(g.B()), _p(c), idx.shape[0],
                          idx.ctypes.data_as(_ip), _p(out))
    return out


def adjoint(g: Geometry, y):
    y = _f64(y)
    assert y.shape == g.data_shape, (y.shape, g.data_shape)
    out = np.empty(g.vol_shape)
    lib().og_adjoint(g.ref(), _p(g.B()), _p(y), _p(out), MEM_BUDGET)
    return out


def adjoint_voxels(g: Geometry, y, xyz):
    y = _f64(y)
    idx = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
    out = np.empty((idx.shape[0], g.n_coeff))
    lib().og_adjoint_voxels(g.ref(), _p(g.B()), _p(y), idx.shape[0],
                            idx.ctypes.data_as(_ip), _p(out))
    return out


def loss_grad(g: Geometry, c, data, w=None, mu=0.0):
    """(loss, grad, resid) of L = sum w (Ac - I)^2 + mu sum c^2."""
    c, data = _f64(c), _f64(data)
    w = None if w is None else _f64(w)
    grad = np.empty(g.vol_shape)
    resid = np.empty(g.data_shape)
    loss = lib().og_loss_grad(g.ref(), _p(g.B()), _p(c), _p(data), _p(w), float(mu),
                              _p(grad), _p(resid), MEM_BUDGET)
    return loss, grad, resid


def lbfgs(g: Geometry, c0, data, w=None, mu=0.0, m=10, max_iter=10, tol=0.0):
    """L-BFGS with exact line search.  Returns (c, iters, hist[iters,2], final_rel)."""
    c = _f64(c0).copy()
    data = _f64(data)
    w = None if w is None else _f64(w)
    hist = np.zeros((max(max_iter, 1), 2))
    fr = C.c_double(0.0)
    it = lib().og_lbfgs(g.ref(), _p(g.B()), _p(c), _p(data), _p(w), float(mu), int(m),
                        int(max_iter), float(tol), _p(hist), C.byref(fr), MEM_BUDGET)
    return c, it, hist[:it], fr.value
