"""Python face of the C ABI: projector, autograd function and L-BFGS solver.

Argument marshalling only.  PyTorch provides device memory and the current
HIP stream; every step of the computation runs in ``libtt_hip.so``.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np
import torch

import tt_inputs as synth

from . import _lib
from ._lib import Geometry, call, lib

__all__ = ["Projector", "ProjectFn", "project", "LBFGS", "sh_eval", "num_coeffs", "tensor_properties",
           "PROPERTY_FIELDS", "laplacian_reg", "huber_reg", "sumsq", "GradientDescent"]


def num_coeffs(ell_max: int) -> int:
    return call("tt_num_coeffs", int(ell_max))


def sh_eval(ell_max: int, dirs) -> np.ndarray:
    """Real even-order spherical harmonics at directions ``dirs[..., 3]`` (host)."""
    d = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
    out = np.empty((d.shape[0], num_coeffs(ell_max)))
    call("tt_sh_eval", int(ell_max), d.shape[0], d.ctypes.data_as(C.POINTER(C.c_double)),
         out.ctypes.data_as(C.POINTER(C.c_double)))
    return out.reshape(np.shape(dirs)[:-1] + (out.shape[1],))


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _f32(t: torch.Tensor, shape, name, device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float32 or t.device != device:
        raise ValueError(f"{name} must be float32 on {device}, got {t.dtype} on {t.device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


class Projector:
    """Forward model I = A c, adjoint and loss gradient for one geometry.

    Shapes: coefficients ``(nx, ny, nz, C)``, data ``(n_proj, nj, nk, n_seg)``.
    ``sparse_k`` >= 1 selects the sparse fused forward (``tt_set_sparse_map``):
    the k largest-magnitude basis constants of every projection and segment are
    kept, and the forward needs no mapped-volume workspace.
    """

    def __init__(self, n, ell_max, inner, outer, nj, nk, n_seg, frame=None, n_sub=3, step=1.0,
                 seg_span=2 * math.pi, joff=None, koff=None, map_precision="fp32", device=None,
                 model="trilinear", basis="sh", dirs=None, width=None, forward_batch=None,
                 workspace_budget=None, sparse_k=0):
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("Projector runs on a HIP device only")
        frame = synth.lab_frame() if frame is None else frame
        self._keep = [np.ascontiguousarray(inner, dtype=np.float64),
                      np.ascontiguousarray(outer, dtype=np.float64),
                      None if joff is None else np.ascontiguousarray(joff, dtype=np.float64),
                      None if koff is None else np.ascontiguousarray(koff, dtype=np.float64)]
        if len(self._keep[0]) != len(self._keep[1]):
            raise ValueError("inner and outer angle arrays differ in length")
        g = Geometry()
        g.nx, g.ny, g.nz = (int(v) for v in n)
        g.ell_max, g.n_proj = int(ell_max), len(self._keep[0])
        g.nj, g.nk, g.n_seg, g.n_sub = int(nj), int(nk), int(n_seg), int(n_sub)
        g.map_precision = _lib.TT_MAP_BF16 if map_precision == "bf16" else _lib.TT_MAP_FP32
        g.step, g.seg_span = float(step), float(seg_span)
        g.inner_angle, g.outer_angle = _dptr(self._keep[0]), _dptr(self._keep[1])
        g.j_offset, g.k_offset = _dptr(self._keep[2]), _dptr(self._keep[3])
        for field, key in (("p", "p"), ("j", "j"), ("k", "k"), ("q0", "q0"), ("q90", "q90"),
                           ("alpha_axis", "alpha"), ("beta_axis", "beta")):
            getattr(g, field)[:] = [float(x) for x in frame[key]]
        if basis not in ("sh", "gk", "nn"):
            raise ValueError("basis must be 'sh', 'gk' or 'nn'")
        if basis != "sh":
            grid = np.ascontiguousarray(dirs, dtype=np.float64).reshape(-1, 3)
            self._keep.append(grid)
            g.basis = _lib.TT_BASIS_GK if basis == "gk" else _lib.TT_BASIS_NN
            g.n_dirs = grid.shape[0]
            g.dirs = _dptr(grid)
            g.kernel_width = float(width) if basis == "gk" else 0.0
        self.basis = basis
        self.geometry = g
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            call("tt_create", C.byref(g), C.byref(handle))
        self._h = handle
        if model not in ("trilinear", "joseph"):
            raise ValueError("model must be 'trilinear' or 'joseph'")
        call("tt_set_projector", self._h,
             _lib.TT_PROJ_JOSEPH if model == "joseph" else _lib.TT_PROJ_TRILINEAR)
        self.model = model
        self.n = tuple(int(v) for v in n)
        self.ell_max, self.n_proj = int(ell_max), g.n_proj
        self.nj, self.nk, self.n_seg = int(nj), int(nk), int(n_seg)
        self.precision = map_precision
        self._ws = None
        self.sparse_k = 0
        self.set_sparse_map(int(sparse_k), forward_batch, workspace_budget)

    def set_sparse_map(self, k: int, forward_batch=None, workspace_budget=None):
        """Select the exact map (k = 0) or the sparse fused forward with k kept
        basis constants per projection and segment, and attach a workspace for
        that mode (device memory owned here, handed to the library).  The
        two-pass forward maps `forward_batch` projections per pass; by default
        as many as fit a budget of 1/8 of the free device memory, clamped to
        [1, 24] GiB.  The fused forward needs no mapped volumes."""
        call("tt_set_sparse_map", self._h, int(k))
        self.sparse_k = int(k)
        sizes = (C.c_int64 * 8)()
        call("tt_sizes", self._h, sizes)
        per_proj = int(sizes[7])
        if self.sparse_k > 0:
            forward_batch = 0
        elif forward_batch is None:
            if workspace_budget is None:
                free, _ = torch.cuda.mem_get_info(self.device)
                workspace_budget = min(24 << 30, max(1 << 30, free // 8))
            forward_batch = max(1, int(workspace_budget) // per_proj)
        nbytes = int(call("tt_workspace_bytes", self._h, int(min(forward_batch, self.n_proj))))
        if self._ws is None or self._ws.numel() < nbytes:
            self._ws = None
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._bind_stream()
        call("tt_set_workspace", self._h, C.c_void_p(self._ws.data_ptr()), nbytes)
        call("tt_sizes", self._h, sizes)
        self.n_coeff, self.n_unique, self.batch, self.work_bytes = (
            int(sizes[2]), int(sizes[3]), int(sizes[4]), int(sizes[5]))

    @classmethod
    def from_workload(cls, w: synth.Workload, **kw):
        inner, outer = synth.angles(w)
        return cls(w.n, w.ell_max, inner, outer, w.nj, w.nk, w.n_seg, n_sub=w.n_sub, step=w.step, **kw)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().tt_destroy(h)
            except Exception:
                pass
            self._h = None

    @property
    def vol_shape(self):
        return self.n + (self.n_coeff,)

    @property
    def data_shape(self):
        return (self.n_proj, self.nj, self.nk, self.n_seg)

    def set_precision(self, precision: str):
        call("tt_set_map_precision", self._h,
             _lib.TT_MAP_BF16 if precision == "bf16" else _lib.TT_MAP_FP32)
        self.precision = precision

    def timing(self, on: bool = True):
        """Start (or stop) per-kernel-class event timing on this projector's stream."""
        call("tt_timing_enable", self._h, int(bool(on)))

    def timing_read(self):
        """{class: (total_ms, launches)} since the last read; synchronises."""
        ms = (C.c_double * len(_lib.KERNEL_CLASSES))()
        n = (C.c_int64 * len(_lib.KERNEL_CLASSES))()
        call("tt_timing_read", self._h, ms, n)
        return {k: (ms[i], int(n[i])) for i, k in enumerate(_lib.KERNEL_CLASSES)}

    def ray_samples(self) -> int:
        """Ray samples (or Joseph cuts) of all projections that touch the volume."""
        out = C.c_int64(0)
        call("tt_ray_samples", self._h, C.byref(out))
        return int(out.value)

    def basis_matrix(self) -> np.ndarray:
        B = np.empty((self.n_proj, self.n_seg, self.n_coeff))
        call("tt_basis_matrix", self._h, _dptr(B))
        return B

    def _bind_stream(self):
        call("tt_set_stream", self._h, C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def forward(self, c: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        pc = _f32(c, self.vol_shape, "c", self.device)
        if out is None:
            out = torch.empty(self.data_shape, dtype=torch.float32, device=self.device)
        po = _f32(out, self.data_shape, "out", self.device)
        self._bind_stream()
        call("tt_project", self._h, pc, po)
        return out

    def adjoint(self, y: torch.Tensor, out: torch.Tensor | None = None, beta: float = 0.0,
                c: torch.Tensor | None = None) -> torch.Tensor:
        py = _f32(y, self.data_shape, "y", self.device)
        if out is None:
            out = torch.empty(self.vol_shape, dtype=torch.float32, device=self.device)
        po = _f32(out, self.vol_shape, "out", self.device)
        pcv = _f32(c, self.vol_shape, "c", self.device) if c is not None else None
        self._bind_stream()
        call("tt_adjoint", self._h, py, po, float(beta), pcv)
        return out

    def _normal_work(self):
        n = int(call("tt_normal_work_bytes", self._h))
        return torch.empty(n, dtype=torch.uint8, device=self.device)

    def kappa(self, radius: float) -> float:
        """Lower median over the voxels within `radius` of the centre of (A^T A u)_{v,0},
        u the unit isotropic field (the network-input scale; synchronises)."""
        work = self._normal_work()
        out = C.c_double(0.0)
        self._bind_stream()
        call("tt_kappa", self._h, float(radius), C.c_void_p(work.data_ptr()), work.numel(), C.byref(out))
        return out.value

    def loss_grad(self, c, data, w=None, mu=0.0, want_resid=True):
        """(loss[1] float64, grad, resid) of sum w (Ac - I)^2 + mu sum c^2."""
        pc = _f32(c, self.vol_shape, "c", self.device)
        pd = _f32(data, self.data_shape, "data", self.device)
        pw = _f32(w, self.data_shape, "w", self.device) if w is not None else None
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        grad = torch.empty(self.vol_shape, dtype=torch.float32, device=self.device)
        resid = torch.empty(self.data_shape, dtype=torch.float32, device=self.device) if want_resid else None
        self._bind_stream()
        call("tt_loss_grad", self._h, pc, pd, pw, float(mu), C.c_void_p(loss.data_ptr()),
             C.c_void_p(grad.data_ptr()), C.c_void_p(resid.data_ptr()) if resid is not None else None)
        return loss, grad, resid


class ProjectFn(torch.autograd.Function):
    """Differentiable I = A c: the backward pass is the library's exact adjoint."""

    @staticmethod
    def forward(ctx, c, projector: Projector):
        ctx.projector = projector
        return projector.forward(c.contiguous())

    @staticmethod
    def backward(ctx, grad_out):
        return ctx.projector.adjoint(grad_out.contiguous()), None


def project(c: torch.Tensor, projector: Projector) -> torch.Tensor:
    return ProjectFn.apply(c, projector)


class LBFGS:
    """Device-resident L-BFGS on sum w (Ac - I)^2 + mu sum c^2 (exact line search)."""

    def __init__(self, projector: Projector, m: int = 10):
        self.projector = projector
        nbytes = int(call("tt_lbfgs_workspace_bytes", projector._h, int(m)))
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=projector.device)
        h = C.c_void_p()
        projector._bind_stream()
        call("tt_lbfgs_create", projector._h, int(m), C.c_void_p(self._ws.data_ptr()), nbytes, C.byref(h))
        self._h = h
        self.m = m
        self._refs = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().tt_lbfgs_destroy(h)
            except Exception:
                pass
            self._h = None

    def init(self, c: torch.Tensor, data: torch.Tensor, w: torch.Tensor | None = None, mu: float = 0.0):
        p = self.projector
        pc = _f32(c, p.vol_shape, "c", p.device)
        pd = _f32(data, p.data_shape, "data", p.device)
        pw = _f32(w, p.data_shape, "w", p.device) if w is not None else None
        self._refs = (c, data, w)  # the solver reads these buffers on every step
        p._bind_stream()
        call("tt_lbfgs_init", self._h, pc, pd, pw, float(mu))

    def step(self):
        self.projector._bind_stream()
        call("tt_lbfgs_step", self._h)

    def step_direction(self, d: torch.Tensor):
        """One iteration along d (exact line search along d; the pair enters the history)."""
        p = self.projector
        pd = _f32(d, p.vol_shape, "d", p.device)
        p._bind_stream()
        call("tt_lbfgs_step_direction", self._h, pd)

    def refresh(self):
        """Recompute the residual A c - I with an explicit forward projection (the
        iterations update it incrementally); query() then reports it."""
        self.projector._bind_stream()
        call("tt_lbfgs_refresh", self._h)

    def query(self):
        """(loss, ||r||, ||I||, accepted pairs); synchronises."""
        out = (C.c_double * 4)()
        self.projector._bind_stream()
        call("tt_lbfgs_query", self._h, out)
        return tuple(out)

    def run(self, max_iter: int, rel_tol: float = 0.0):
        """Iterate; returns (iterations, history[iters, 2] of (loss, ||r||/||I||))."""
        hist = np.zeros((max(max_iter, 1), 2))
        it = C.c_int(0)
        self.projector._bind_stream()
        call("tt_lbfgs_run", self._h, int(max_iter), float(rel_tol),
             hist.ctypes.data_as(C.POINTER(C.c_double)), C.byref(it))
        return it.value, hist[: it.value]


# Column order of tensor_properties (matches TT_PROP_FIELDS in tt.h).
PROPERTY_FIELDS = ("mean", "variance", "rel_anisotropy",
                   "m_xx", "m_yy", "m_zz", "m_xy", "m_xz", "m_yz",
                   "lambda1", "lambda2", "lambda3",
                   "v1_x", "v1_y", "v1_z", "v2_x", "v2_y", "v2_z", "v3_x", "v3_y", "v3_z",
                   "fa")


def tensor_properties(c: torch.Tensor, ell_max: int, out: torch.Tensor | None = None) -> torch.Tensor:
    """Derived per-voxel quantities of coefficients c[..., C]: tensor [..., 22].

    Mean, variance, relative anisotropy, second-moment tensor, its eigenvalues
    (descending) and eigenvectors, and the fractional anisotropy, in the order
    of PROPERTY_FIELDS.  Runs on the current HIP stream.
    """
    C_ = num_coeffs(ell_max)
    if not isinstance(c, torch.Tensor) or c.dtype != torch.float32 or not c.is_cuda or not c.is_contiguous():
        raise ValueError("c must be a contiguous float32 device tensor")
    if c.shape[-1] != C_:
        raise ValueError(f"c has {c.shape[-1]} coefficients, expected {C_} for ell_max {ell_max}")
    n_vox = c.numel() // C_
    shape = tuple(c.shape[:-1]) + (len(PROPERTY_FIELDS),)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=c.device)
    _f32(out, shape, "out", c.device)
    stream = torch.cuda.current_stream(c.device).cuda_stream
    call("tt_tensor_properties", C.c_void_p(c.data_ptr()), n_vox, int(ell_max), C.c_void_p(out.data_ptr()),
         C.c_void_p(stream))
    return out


def _stream(t):
    return C.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


_PARTIALS = {}


def _partials(device):
    """float64 partial-sum buffer (TT_REDUCE_WORK elements) for value reductions on this device."""
    key = torch.device(device)
    buf = _PARTIALS.get(key)
    if buf is None:
        buf = _PARTIALS[key] = torch.empty(_lib.REDUCE_WORK, dtype=torch.float64, device=key)
    return C.c_void_p(buf.data_ptr()), buf.numel()


def sumsq(x: torch.Tensor, value: torch.Tensor, scale: float = 1.0):
    """value[0] += scale * sum x^2 (float64, fixed summation order)."""
    _dev_f32(x, "x")
    pp, pn = _partials(x.device)
    call("tt_sumsq", C.c_void_p(x.data_ptr()), x.numel(), float(scale), C.c_void_p(value.data_ptr()), pp, pn,
         _stream(x))


def _dev_f32(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 device tensor")
    return C.c_void_p(t.data_ptr())


def laplacian_reg(c: torch.Tensor, lam: float, grad: torch.Tensor, value: torch.Tensor | None = None,
                  work: torch.Tensor | None = None) -> torch.Tensor:
    """grad += 2 lam Lap(Lap c); value += lam sum (Lap c)^2 (float64 device scalar).

    c is (nx, ny, nz, C); returns the work tensor holding Lap c."""
    if c.dim() != 4:
        raise ValueError("c must be (nx, ny, nz, C)")
    work = torch.empty_like(c) if work is None else work
    for t, n in ((c, "c"), (grad, "grad"), (work, "work")):
        _dev_f32(t, n)
        if t.shape != c.shape:
            raise ValueError(f"{n} has shape {tuple(t.shape)}, expected {tuple(c.shape)}")
    vp = None
    if value is not None:
        if value.dtype != torch.float64 or not value.is_cuda:
            raise ValueError("value must be a float64 device tensor")
        vp = C.c_void_p(value.data_ptr())
    nx, ny, nz, nc = (int(v) for v in c.shape)
    pp, pn = _partials(c.device)
    call("tt_laplacian_reg", C.c_void_p(c.data_ptr()), nx, ny, nz, nc, float(lam), C.c_void_p(work.data_ptr()),
         C.c_void_p(grad.data_ptr()), vp, pp, pn, _stream(c))
    return work


def huber_reg(c: torch.Tensor, delta: float, lam: float, grad: torch.Tensor, value: torch.Tensor | None = None):
    """grad += lam h'(c); value += lam sum h(c), h the Huber function of width delta."""
    _dev_f32(c, "c")
    _dev_f32(grad, "grad")
    if grad.shape != c.shape:
        raise ValueError("grad and c differ in shape")
    vp = None
    if value is not None:
        if value.dtype != torch.float64 or not value.is_cuda:
            raise ValueError("value must be a float64 device tensor")
        vp = C.c_void_p(value.data_ptr())
    pp, pn = _partials(c.device)
    call("tt_huber_reg", C.c_void_p(c.data_ptr()), c.numel(), float(delta), float(lam), C.c_void_p(grad.data_ptr()),
         vp, pp, pn, _stream(c))


class GradientDescent:
    """Fixed-step gradient descent, optionally with Nesterov momentum (m_k = (k-1)/(k+2)),
    on sum w (Ac - I)^2 (or the Huber loss sum w h_loss_delta(Ac - I)) + mu |c|^2
    + lam_lap sum (Lap c)^2 + huber_lam sum h_delta(c)."""

    def __init__(self, projector: Projector, step: float, nesterov: bool = False, lam_lap: float = 0.0,
                 huber: tuple | None = None, loss_delta: float | None = None,
                 precond: torch.Tensor | None = None):
        self.P, self.step, self.nesterov = projector, float(step), bool(nesterov)
        self.lam_lap, self.huber = float(lam_lap), huber
        self.loss_delta = None if loss_delta is None else float(loss_delta)
        if precond is not None:
            _f32(precond, projector.vol_shape, "precond", projector.device)
        self.precond = precond

    @staticmethod
    def voxel_preconditioner(projector: Projector, floor: float = 1e-6) -> torch.Tensor:
        """Diagonal preconditioner 1 / (A^T A u)_{v,0} per voxel (all coefficients of a
        voxel share it), u the unit isotropic field: the normal operator's scale at
        each voxel, floored at floor times its maximum (computed by the library)."""
        p = torch.empty(projector.vol_shape, device=projector.device)
        work = projector._normal_work()
        projector._bind_stream()
        call("tt_voxel_preconditioner", projector._h, float(floor), C.c_void_p(p.data_ptr()),
             C.c_void_p(work.data_ptr()), work.numel())
        return p

    def objective_grad(self, c, data, w=None, mu=0.0, work=None):
        """(value float64[1], grad) of the whole objective at c."""
        if self.loss_delta is None:
            loss, grad, _ = self.P.loss_grad(c, data, w, mu, want_resid=False)
        else:
            # Huber loss of the residual (+ mu |c|^2): y = w h'(Ac - I), grad = A^T y + 2 mu c
            _f32(data, self.P.data_shape, "data", self.P.device)
            if w is not None:
                _f32(w, self.P.data_shape, "w", self.P.device)
            I = self.P.forward(c)
            loss = torch.zeros(1, dtype=torch.float64, device=c.device)
            y = torch.empty_like(I)
            pp, pn = _partials(c.device)
            call("tt_huber_loss", C.c_void_p(I.data_ptr()), C.c_void_p(data.data_ptr()),
                 C.c_void_p(w.data_ptr()) if w is not None else None, I.numel(), self.loss_delta,
                 C.c_void_p(y.data_ptr()), C.c_void_p(loss.data_ptr()), pp, pn, _stream(c))
            if mu:
                sumsq(c, loss, mu)
            grad = self.P.adjoint(y, beta=2.0 * mu, c=c)
        if self.lam_lap:
            laplacian_reg(c, self.lam_lap, grad, loss, work)
        if self.huber is not None:
            huber_reg(c, self.huber[0], self.huber[1], grad, loss)
        return loss, grad

    def run(self, c: torch.Tensor, data, w=None, mu=0.0, iters=10):
        """Iterates in place on c; returns the objective before each step (float64, length iters)."""
        _f32(c, self.P.vol_shape, "c", self.P.device)
        y = c.clone()
        work = torch.empty_like(c) if self.lam_lap else None
        losses = torch.empty(iters, dtype=torch.float64, device=c.device)
        for k in range(1, iters + 1):
            val, grad = self.objective_grad(y, data, w, mu, work)
            losses[k - 1:k].copy_(val)
            m = (k - 1.0) / (k + 2.0) if self.nesterov else 0.0
            call("tt_gd_step", C.c_void_p(c.data_ptr()), C.c_void_p(y.data_ptr()), C.c_void_p(grad.data_ptr()),
                 C.c_void_p(self.precond.data_ptr()) if self.precond is not None else None,
                 c.numel(), self.step, m, _stream(c))
        return losses

