"""Pins of the oracle's loss, gradient and L-BFGS.

Loss: Eq. opt_prob_general_form with squared norms and D = identity,
L(c) = sum w (Ac - I)^2 + mu sum c^2 (Eq. residual for r = Ac - I).
Optimiser: L-BFGS (section 3.5 "Optimization") with the exact line search of
the quadratic loss.  Pinned by central differences (exact for a quadratic up
to rounding), by the theorem that L-BFGS with exact line searches and a scalar
initial matrix reproduces conjugate gradients on a quadratic, and by the dense
normal-equation solution on a tiny volume.
"""
import numpy as np
import pytest

import oracle
from oracle import dense, phantom
from geoms import small, tiny, workload
import tt_inputs as synth


def _problem(g, seed=12):
    rng = np.random.default_rng(seed)
    data = rng.standard_normal(g.data_shape)
    w = rng.uniform(0.5, 1.5, g.data_shape)
    c = 0.1 * rng.standard_normal(g.vol_shape)
    return rng, data, w, c


def test_loss_value_by_definition():
    g = tiny()
    rng, data, w, c = _problem(g)
    A = dense.dense_A(g)
    r = A @ c.reshape(-1) - data.reshape(-1)
    ref = np.sum(w.reshape(-1) * r * r) + 0.3 * np.sum(c * c)
    loss, grad, resid = oracle.loss_grad(g, c, data, w, 0.3)
    assert abs(loss - ref) < 1e-12 * ref
    assert np.abs(resid.reshape(-1) - r).max() < 1e-12


def test_gradient_central_differences():
    g = small(ell_max=2)
    rng, data, w, c = _problem(g)
    mu = 0.05
    loss, grad, resid = oracle.loss_grad(g, c, data, w, mu)
    h = 1e-3
    for t in range(12):
        idx = tuple(int(rng.integers(0, m)) for m in g.vol_shape)
        cp, cm = c.copy(), c.copy()
        cp[idx] += h
        cm[idx] -= h
        _, _, rp = oracle.loss_grad(g, cp, data, w, mu)
        _, _, rm = oracle.loss_grad(g, cm, data, w, mu)
        # cancellation-free numerator of L(c+h e) - L(c-h e)
        num = np.sum(w * (rp - rm) * (rp + rm)) + mu * (cp[idx] ** 2 - cm[idx] ** 2)
        fd = num / (2 * h)
        assert abs(fd - grad[idx]) < 1e-9 * max(1.0, np.abs(grad).max()), (idx, fd, grad[idx])


def _cg(g, data, w, mu, c0, iters):
    """Textbook linear CG on (A^T W A + mu I) c = A^T W I; returns all iterates."""
    def H(v):
        return oracle.adjoint(g, w * oracle.project(g, v)) + mu * v
    b = oracle.adjoint(g, w * data)
    c = c0.copy()
    r = b - H(c)
    p = r.copy()
    rr = np.vdot(r, r)
    out = []
    for _ in range(iters):
        Hp = H(p)
        a = rr / np.vdot(p, Hp)
        c = c + a * p
        r = r - a * Hp
        rr_new = np.vdot(r, r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        out.append(c.copy())
    return out


@pytest.mark.parametrize("m", [1, 3, 10])
def test_lbfgs_equals_cg_on_quadratic(m):
    g = tiny()
    rng, data, w, c0 = _problem(g)
    mu = 1e-2
    ref = _cg(g, data, w, mu, c0, 8)
    for k in (1, 4, 8):
        c, it, hist, _ = oracle.lbfgs(g, c0, data, w, mu, m=m, max_iter=k)
        assert it == k
        err = np.linalg.norm(c - ref[k - 1]) / np.linalg.norm(ref[k - 1])
        assert err < 1e-9, (m, k, err)


def test_lbfgs_converges_to_dense_solution():
    g = tiny()
    rng, data, w, c0 = _problem(g)
    mu = 0.5
    A = dense.dense_A(g)
    H = A.T @ (w.reshape(-1)[:, None] * A) + mu * np.eye(A.shape[1])
    x = np.linalg.solve(H, A.T @ (w.reshape(-1) * data.reshape(-1)))
    c, it, hist, rel = oracle.lbfgs(g, np.zeros(g.vol_shape), data, w, mu, m=10, max_iter=400)
    assert np.linalg.norm(c.reshape(-1) - x) < 1e-8 * np.linalg.norm(x)
    assert np.all(np.diff(hist[:, 0]) <= 1e-12 * hist[0, 0])  # monotone loss


def test_lbfgs_stops_at_tolerance():
    w_ = synth.WORKLOADS["c1"]
    g = small(ell_max=4, n=(16, 16, 16), nj=16, nk=16)
    rng = np.random.default_rng(1)
    c_true = rng.standard_normal(g.vol_shape) * 0.1
    data = oracle.project(g, c_true)
    c, it, hist, rel = oracle.lbfgs(g, np.zeros(g.vol_shape), data, None, 1e-6, m=10,
                                    max_iter=500, tol=5e-2)
    assert it < 500
    assert hist[-1, 1] <= 5e-2 and (it == 1 or hist[-2, 1] > 5e-2)
    assert abs(rel - hist[-1, 1]) < 1e-9


def test_phantom_spherical_mean_is_density():
    # The lobe (1-d) + 5 d u^4 has spherical mean 1, so c_00 Y_00 = density.
    w_ = synth.WORKLOADS["c1"]
    c = phantom.phantom_coeffs(w_)
    _, _, density = synth.twisted_fibre_field(w_)
    assert np.abs(c[..., 0] / np.sqrt(4 * np.pi) - density).max() < 1e-14
    # band limit: orders above 4 are empty
    assert c.shape[-1] == 15
    # pointwise: the SH series reproduces the lobe at random directions
    rng = np.random.default_rng(2)
    direction, degree, _ = synth.twisted_fibre_field(w_)
    v = (16, 16, 16)
    q = rng.standard_normal((20, 3))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    f = oracle.sh(4, q) @ c[v]
    u = q @ direction[v]
    ref = (1 - degree[v]) + 5 * degree[v] * u ** 4
    assert np.abs(f - ref).max() < 1e-12
