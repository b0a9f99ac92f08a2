"""Pins of the regulariser / gradient-descent oracle.

* Laplacian: discrete sine modes are its eigenvectors with eigenvalue
  -sum_a 2 (1 - cos(pi k_a / (N_a + 1))) (closed form for the zero-boundary
  7-point stencil); quadratic and linear fields in the interior; symmetry;
  the gradient of the regulariser by central differences.
* Huber: the two branches, continuity, gradient by central differences.
* Gradient descent: the first step is c0 - step grad f(c0); without momentum
  it converges to the dense normal-equation solution of the regularised
  problem; with Nesterov momentum it gets there in fewer iterations.
"""
import math

import numpy as np

import oracle
from oracle.dense import dense_A
from oracle.regularizers import gradient_descent, huber_loss, huber_reg, laplacian, laplacian_reg, nesterov_momentum
from geoms import tiny


def test_laplacian_sine_modes_closed_form():
    n = (7, 9, 6)
    grid = np.meshgrid(*[np.arange(1, m + 1) for m in n], indexing="ij")
    for kvec in ((1, 1, 1), (2, 5, 3), (7, 1, 6)):
        mode = np.prod([np.sin(math.pi * k * x / (m + 1)) for k, x, m in zip(kvec, grid, n)], axis=0)
        lam = -sum(2.0 * (1.0 - math.cos(math.pi * k / (m + 1))) for k, m in zip(kvec, n))
        L = laplacian(mode[..., None])[..., 0]
        assert np.abs(L - lam * mode).max() < 1e-13


def test_laplacian_polynomials_interior_and_symmetry():
    n = (8, 7, 9)
    x, y, z = np.meshgrid(*[np.arange(m, dtype=float) for m in n], indexing="ij")
    c = np.stack([x * x + y * y + z * z, 2 * x - 3 * y + z + 4.0], axis=-1)
    L = laplacian(c)[1:-1, 1:-1, 1:-1]
    assert np.abs(L[..., 0] - 6.0).max() < 1e-12
    assert np.abs(L[..., 1]).max() < 1e-12
    rng = np.random.default_rng(2)
    a, b = rng.standard_normal(n + (3,)), rng.standard_normal(n + (3,))
    assert abs(np.vdot(laplacian(a), b) - np.vdot(a, laplacian(b))) < 1e-10


def test_laplacian_reg_gradient_fd():
    rng = np.random.default_rng(3)
    c = rng.standard_normal((5, 6, 4, 2))
    lam = 0.7
    _, grad = laplacian_reg(c, lam)
    h = 1e-5
    for _ in range(12):
        idx = tuple(int(rng.integers(0, m)) for m in c.shape)
        cp, cm = c.copy(), c.copy()
        cp[idx] += h
        cm[idx] -= h
        fd = (laplacian_reg(cp, lam)[0] - laplacian_reg(cm, lam)[0]) / (2 * h)
        assert abs(fd - grad[idx]) < 1e-6 * max(1.0, abs(grad[idx]))


def test_huber_branches_and_gradient():
    delta, lam = 0.3, 2.0
    x = np.array([-2.0, -0.3, -0.1, 0.0, 0.05, 0.3, 1.7])
    v, g = huber_reg(x, delta, lam)
    ref = lam * sum(t * t / (2 * delta) if abs(t) <= delta else abs(t) - delta / 2 for t in x)
    assert abs(v - ref) < 1e-14
    # continuity of value and derivative at |x| = delta
    for s in (-1, 1):
        lo = huber_reg(np.array([s * delta * (1 - 1e-12)]), delta, 1.0)
        hi = huber_reg(np.array([s * delta * (1 + 1e-12)]), delta, 1.0)
        assert abs(lo[0] - hi[0]) < 1e-12 and abs(lo[1][0] - hi[1][0]) < 1e-11
    h = 1e-6
    for t in (-1.1, -0.2, 0.01, 0.25, 0.9):
        fd = (huber_reg(np.array([t + h]), delta, lam)[0] - huber_reg(np.array([t - h]), delta, lam)[0]) / (2 * h)
        assert abs(fd - huber_reg(np.array([t]), delta, lam)[1][0]) < 1e-7


def _small_problem():
    g = tiny(ell_max=2, n=(4, 5, 3), nj=6, nk=5)
    rng = np.random.default_rng(4)
    data = rng.standard_normal(g.data_shape)
    return g, data


def test_gradient_descent_first_step_and_convergence():
    g, data = _small_problem()
    mu, lam = 0.5, 5e-3
    A = dense_A(g).reshape(-1, int(np.prod(g.vol_shape)))
    Lmat = np.stack([laplacian(e.reshape(g.vol_shape)).ravel() for e in np.eye(A.shape[1])], axis=1)
    H = 2 * (A.T @ A + mu * np.eye(A.shape[1]) + lam * Lmat.T @ Lmat)
    c_star = np.linalg.solve(H, 2 * A.T @ data.ravel()).reshape(g.vol_shape)
    ev = np.linalg.eigvalsh(H)
    step = 1.0 / ev.max()
    c0 = np.zeros(g.vol_shape)
    c1, _ = gradient_descent(g, c0, data, step, 1, mu=mu, lam_lap=lam)
    _, grad0, _ = oracle.loss_grad(g, c0, data, None, mu)
    assert np.abs(c1 - (c0 - step * (grad0 + laplacian_reg(c0, lam)[1]))).max() < 1e-14
    assert ev.max() / ev.min() < 100  # well conditioned: the iteration counts below suffice
    c_gd, loss_gd = gradient_descent(g, c0, data, step, 100, mu=mu, lam_lap=lam)
    c_nv, loss_nv = gradient_descent(g, c0, data, step, 100, mu=mu, lam_lap=lam, nesterov=True)
    e_gd = np.linalg.norm(c_gd - c_star) / np.linalg.norm(c_star)
    e_nv = np.linalg.norm(c_nv - c_star) / np.linalg.norm(c_star)
    assert e_nv < 0.2 * e_gd                                 # momentum accelerates
    assert np.all(np.diff(loss_gd) <= 1e-12 * loss_gd[0])   # fixed step 1/L: monotone
    c_long, _ = gradient_descent(g, c0, data, step, 1500, mu=mu, lam_lap=lam)
    assert np.linalg.norm(c_long - c_star) / np.linalg.norm(c_star) < 1e-12
    assert nesterov_momentum(1) == 0.0 and abs(nesterov_momentum(4) - 0.5) < 1e-15


def test_huber_loss_small_residuals_and_fd():
    g, data = _small_problem()
    rng = np.random.default_rng(6)
    c = rng.standard_normal(g.vol_shape)
    # a width above every residual: the Huber loss is the squared loss / (2 delta)
    r = oracle.project(g, c) - data
    delta = 1.01 * np.abs(r).max()
    v, grad = huber_loss(g, c, data, delta)
    l2, g2, _ = oracle.loss_grad(g, c, data, None, 0.0)
    assert abs(v - l2 / (2 * delta)) < 1e-12 * l2 and np.abs(grad - g2 / (2 * delta)).max() < 1e-12 * np.abs(g2).max()
    # a narrow width: central differences (piecewise quadratic; steps small against the kink distances)
    delta = 0.2 * np.abs(r).max()
    w = rng.uniform(0.5, 1.5, g.data_shape)
    v, grad = huber_loss(g, c, data, delta, w)
    h = 1e-7
    for _ in range(8):
        idx = tuple(int(rng.integers(0, m)) for m in c.shape)
        cp, cm = c.copy(), c.copy()
        cp[idx] += h
        cm[idx] -= h
        fd = (huber_loss(g, cp, data, delta, w)[0] - huber_loss(g, cm, data, delta, w)[0]) / (2 * h)
        assert abs(fd - grad[idx]) < 1e-5 * max(1.0, abs(grad[idx]))


def test_preconditioned_descent_first_step_and_minimiser():
    g, data = _small_problem()
    mu = 0.5
    A = dense_A(g).reshape(-1, int(np.prod(g.vol_shape)))
    H = 2 * (A.T @ A + mu * np.eye(A.shape[1]))
    c_star = np.linalg.solve(H, 2 * A.T @ data.ravel()).reshape(g.vol_shape)
    rng = np.random.default_rng(9)
    p = rng.uniform(0.5, 2.0, g.vol_shape)
    Ph = np.sqrt(p.ravel())
    step = 1.0 / np.linalg.eigvalsh(Ph[:, None] * H * Ph[None, :]).max()
    c0 = np.zeros(g.vol_shape)
    c1, _ = gradient_descent(g, c0, data, step, 1, mu=mu, precond=p)
    _, grad0, _ = oracle.loss_grad(g, c0, data, None, mu)
    assert np.abs(c1 - (c0 - step * p * grad0)).max() < 1e-14
    c_long, losses = gradient_descent(g, c0, data, step, 3000, mu=mu, precond=p)
    assert np.linalg.norm(c_long - c_star) / np.linalg.norm(c_star) < 1e-10
    assert np.all(np.diff(losses) <= 1e-12 * losses[0])
