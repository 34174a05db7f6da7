"""Pins for oracle.precond: Galerkin targets, MLP backpropagation and Adam."""
import numpy as np

from oracle import gp, precond


def _params(rng, I=4, H=7, O=5):
    return {"W1": rng.standard_normal((I, H)) * 0.5, "b1": rng.standard_normal(H) * 0.1,
            "W2": rng.standard_normal((H, H)) * 0.5, "b2": rng.standard_normal(H) * 0.1,
            "W3": rng.standard_normal((H, O)) * 0.5, "b3": rng.standard_normal(O) * 0.1,
            "in_mu": rng.standard_normal(I), "in_sd": rng.uniform(0.5, 2, I),
            "out_mu": rng.standard_normal(O), "out_sd": rng.uniform(0.5, 2, O)}


def test_mlp_gradient_vs_finite_differences():
    r = np.random.default_rng(0)
    p = _params(r)
    psis = r.standard_normal((9, 4))
    T = r.standard_normal((9, 5))
    loss, g = precond.mlp_grad(p, psis, T)
    np.testing.assert_allclose(loss, precond.mlp_loss(p, psis, T), rtol=1e-14)
    h = 1e-6
    for name in ["W1", "b1", "W2", "b2", "W3", "b3"]:
        fd = np.zeros_like(p[name])
        for idx in np.ndindex(p[name].shape):
            q = {k: v.copy() for k, v in p.items()}
            q[name][idx] += h
            lp = precond.mlp_loss(q, psis, T)
            q[name][idx] -= 2 * h
            lm = precond.mlp_loss(q, psis, T)
            fd[idx] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(g[name], fd, rtol=1e-6, atol=1e-9)


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = precond.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 0.01)
    # bias-corrected first step: m^ = g, v^ = g^2, so the step is -lr g / (|g| + eps)
    np.testing.assert_allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_galerkin_targets_closed_forms():
    r = np.random.default_rng(1)
    n, k = 60, 8
    X = r.uniform(size=(n, 2)).astype(np.float32)
    psi = np.log([1.0, 0.3, 0.3, 0.1])
    y = r.standard_normal(n)
    U, _ = np.linalg.qr(r.standard_normal((n, k)))
    t = precond.galerkin_targets(X, psi, y, U)
    K = gp.kernel_matrix(X, psi)
    # c is the Galerkin solution: U^T (K U c - y) = 0
    np.testing.assert_allclose(U.T @ (K @ (U @ t[:k]) - y), 0, atol=1e-10)
    np.testing.assert_allclose(np.exp(t[k:2 * k]), np.einsum("ik,ij,jk->k", U, K, U), rtol=1e-12)
    # tr K = n (sigma^2 + lambda)
    np.testing.assert_allclose(np.exp(t[-1]) * (n - k) + np.exp(t[k:2 * k]).sum(), n * 1.1, rtol=1e-12)
    # with U = eigenvectors of K the target d are the eigenvalues
    w, Q = np.linalg.eigh(K)
    t2 = precond.galerkin_targets(X, psi, y, Q[:, -k:])
    np.testing.assert_allclose(np.exp(t2[k:2 * k]), w[-k:], rtol=1e-10)


def test_precond_coefficients_spd():
    k = 4
    out = np.array([0.0] * k + [-5, 0.2, 1.0, -9] + [0.5])
    h, tinv, c = precond.precond_coefficients(out, np.zeros(2 * k + 1), np.ones(2 * k + 1), k)
    # d floored at tau -> 1/d - 1/tau <= 0 and tau_inv + h = 1/d > 0
    assert np.all(h <= 0) and np.all(tinv + h > 0)
