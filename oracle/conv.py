"""FP64 oracle for the warm-start network's layers (test infrastructure).

3-D convolution with 3x3x3 kernels, stride 1 and zero padding 1 ("same"),
channels-last layout x[n, X, Y, Z, ci], weights w[dx, dy, dz, ci, co]:

  y[n, v, co] = b[co] + sum_{d in {0,1,2}^3} sum_ci x[n, v + d - 1, ci] w[d, ci, co]

with x = 0 outside the volume; its gradients with respect to the input and
the weights written out from that definition, and one Adam step (Kingma & Ba,
2015: m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
w <- w - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)).
"""
from __future__ import annotations

import itertools

import numpy as np

TAPS = list(itertools.product(range(3), repeat=3))


def _pad(x):
    return np.pad(x, ((0, 0), (1, 1), (1, 1), (1, 1), (0, 0)))


def conv3d(x, w, b=None):
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    N, X, Y, Z, _ = x.shape
    xp = _pad(x)
    y = np.zeros((N, X, Y, Z, w.shape[-1]))
    for dx, dy, dz in TAPS:
        y += xp[:, dx:dx + X, dy:dy + Y, dz:dz + Z, :] @ w[dx, dy, dz]
    if b is not None:
        y += np.asarray(b, np.float64)
    return y


def conv3d_dgrad(gy, w):
    """d loss / d x for y = conv3d(x, w): gx[v, ci] = sum_d sum_co gy[v - d + 1, co] w[d, ci, co]."""
    gy = np.asarray(gy, np.float64)
    w = np.asarray(w, np.float64)
    N, X, Y, Z, _ = gy.shape
    gp = _pad(gy)
    gx = np.zeros((N, X, Y, Z, w.shape[3]))
    for dx, dy, dz in TAPS:
        # v - d + 1 in padded coordinates is v + (2 - d)
        sl = gp[:, 2 - dx:2 - dx + X, 2 - dy:2 - dy + Y, 2 - dz:2 - dz + Z, :]
        gx += sl @ w[dx, dy, dz].T
    return gx


def conv3d_wgrad(x, gy):
    """d loss / d w: gw[d, ci, co] = sum_{n, v} x[n, v + d - 1, ci] gy[n, v, co]."""
    x = np.asarray(x, np.float64)
    gy = np.asarray(gy, np.float64)
    N, X, Y, Z, Ci = x.shape
    Co = gy.shape[-1]
    xp = _pad(x)
    gw = np.zeros((3, 3, 3, Ci, Co))
    g2 = gy.reshape(-1, Co)
    for dx, dy, dz in TAPS:
        gw[dx, dy, dz] = xp[:, dx:dx + X, dy:dy + Y, dz:dz + Z, :].reshape(-1, Ci).T @ g2
    return gw


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns (w, m, v) as new float64 arrays (t starts at 1)."""
    w, g, m, v = (np.asarray(a, np.float64) for a in (w, g, m, v))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
