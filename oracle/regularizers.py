"""FP64 oracle for the other objectives on the same operator (test infrastructure only).

Written from the paper's description of the loss functions, regularisers and
optimisers of sect. 3.5 ("Optimization"):

* Laplacian regulariser: lambda * sum over voxels and coefficients of the
  squared finite-difference Laplacian of each coefficient channel.  Reading:
  the 7-point stencil (sum of the six face neighbours minus six times the
  voxel) with zero outside the volume; its gradient is 2 lambda Lap(Lap c)
  because that stencil matrix is symmetric.
* Huber norm of the tensor field: lambda * sum h(c) with
  h(x) = x^2 / (2 delta) for |x| <= delta and |x| - delta / 2 otherwise
  (quadratic for small, absolute value for large coefficients, continuous
  with a continuous derivative clamp(x / delta, -1, 1)).
* Huber loss (robust regression on the residual, the HuberLoss of sect.
  3.5): sum w h(Ac - I) with the same h; its gradient is A^T (w h'(r)).
* Gradient descent with a fixed step, optionally with Nesterov momentum and a
  diagonal preconditioner p (the paper's loss functions accept one):
  c_{k+1} = y_k - step p grad f(y_k), y_{k+1} = c_{k+1} + m_k (c_{k+1} - c_k),
  m_k = (k - 1) / (k + 2) for k = 1, 2, ... (Nesterov's schedule), m_k = 0
  without momentum; y_0 = c_0.
"""
from __future__ import annotations

import numpy as np

from . import adjoint, loss_grad, project

__all__ = ["laplacian", "laplacian_reg", "huber_reg", "huber_loss", "nesterov_momentum", "gradient_descent"]


def laplacian(c):
    """7-point Laplacian of every channel of c[nx, ny, nz, C], zero outside."""
    c = np.asarray(c, dtype=np.float64)
    p = np.pad(c, ((1, 1), (1, 1), (1, 1), (0, 0)))
    return (p[2:, 1:-1, 1:-1] + p[:-2, 1:-1, 1:-1] + p[1:-1, 2:, 1:-1] + p[1:-1, :-2, 1:-1]
            + p[1:-1, 1:-1, 2:] + p[1:-1, 1:-1, :-2] - 6.0 * p[1:-1, 1:-1, 1:-1])


def laplacian_reg(c, lam):
    """(lambda * sum (Lap c)^2, 2 lambda Lap(Lap c))."""
    L = laplacian(c)
    return lam * float((L * L).sum()), 2.0 * lam * laplacian(L)


def huber_reg(c, delta, lam):
    """(lambda * sum h(c), lambda * h'(c))."""
    c = np.asarray(c, dtype=np.float64)
    a = np.abs(c)
    h = np.where(a <= delta, c * c / (2.0 * delta), a - 0.5 * delta)
    return lam * float(h.sum()), lam * np.clip(c / delta, -1.0, 1.0)


def huber_loss(g, c, data, delta, w=None):
    """(sum w h(r), A^T (w h'(r))) with r = A c - data."""
    r = project(g, c) - np.asarray(data, dtype=np.float64)
    wt = 1.0 if w is None else np.asarray(w, dtype=np.float64)
    a = np.abs(r)
    h = np.where(a <= delta, r * r / (2.0 * delta), a - 0.5 * delta)
    return float((wt * h).sum()), adjoint(g, wt * np.clip(r / delta, -1.0, 1.0))


def nesterov_momentum(k: int) -> float:
    """Momentum of step k >= 1 in Nesterov's schedule."""
    return (k - 1.0) / (k + 2.0)


def gradient_descent(g, c0, data, step, iters, w=None, mu=0.0, lam_lap=0.0, huber=None, nesterov=False,
                     loss_delta=None, precond=None):
    """Fixed-step gradient descent on the data term + mu |c|^2 + Laplacian + Huber terms.

    The data term is sum w (Ac - I)^2, or the Huber loss sum w h(Ac - I) of
    width loss_delta when that is given.  huber = (delta, lambda) or None.
    precond: optional positive diagonal (array of c's shape) multiplying the
    gradient in each step.
    Returns (c, losses) with losses[k] the objective at the point whose
    gradient step k takes (y_k)."""
    c = np.asarray(c0, dtype=np.float64).copy()
    y = c.copy()
    losses = []
    for k in range(1, iters + 1):
        if loss_delta is None:
            f, grad, _ = loss_grad(g, y, data, w, mu)
        else:
            f, grad = huber_loss(g, y, data, loss_delta, w)
            f, grad = f + mu * float((y * y).sum()), grad + 2.0 * mu * y
        if lam_lap:
            fl, gl = laplacian_reg(y, lam_lap)
            f, grad = f + fl, grad + gl
        if huber is not None:
            fh, gh = huber_reg(y, huber[0], huber[1])
            f, grad = f + fh, grad + gh
        losses.append(f)
        c_new = y - step * (grad if precond is None else precond * grad)
        m = nesterov_momentum(k) if nesterov else 0.0
        y = c_new + m * (c_new - c)
        c = c_new
    return c, np.array(losses)
