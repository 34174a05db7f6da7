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
    h, tinv, c, ok = precond.precond_coefficients(out, np.zeros(2 * k + 1), np.ones(2 * k + 1), k)
    # d floored at tau -> 1/d - 1/tau <= 0 and tau_inv + h = 1/d > 0
    assert ok and np.all(h <= 0) and np.all(tinv + h > 0)


def test_precond_coefficients_hand_computed():
    # k = 2, u = mu + sd * y worked out by hand:
    #   y  = (1, -1,   0, 1,   0.5),  mu = (0, 1, ln 4, 0, 0),  sd = (0.5, 2, 1, ln 2, 2 ln 3)
    #   u  = (0.5, -1, ln 4, ln 2, ln 3)  ->  c = (0.5, -1), d = (4, 2), tau = 3
    #   d floored at tau: (4, 3);  h = (1/4 - 1/3, 1/3 - 1/3) = (-1/12, 0);  tau_inv = 1/3
    y = np.array([1.0, -1.0, 0.0, 1.0, 0.5])
    mu = np.array([0.0, 1.0, np.log(4.0), 0.0, 0.0])
    sd = np.array([0.5, 2.0, 1.0, np.log(2.0), 2 * np.log(3.0)])
    h, tinv, c, ok = precond.precond_coefficients(y, mu, sd, 2)
    assert ok
    np.testing.assert_allclose(c, [0.5, -1.0], rtol=1e-15)
    np.testing.assert_allclose(h, [-1.0 / 12.0, 0.0], atol=1e-15)
    np.testing.assert_allclose(tinv, 1.0 / 3.0, rtol=1e-15)
    # tau_inv + h_kappa = 1 / max(d_kappa, tau): the eigenvalues of P^-1 on span(U)
    np.testing.assert_allclose(tinv + h, [0.25, 1.0 / 3.0], rtol=1e-14)


def test_precond_coefficients_rejects_unusable_outputs():
    k = 2
    mu, sd = np.zeros(2 * k + 1), np.ones(2 * k + 1)
    good = np.array([0.1, 0.2, 1.0, 2.0, 0.5])
    assert precond.precond_coefficients(good, mu, sd, k)[3]
    # exactly at the edge of the range is accepted, past it is not
    edge = good.copy()
    edge[2 * k] = 60.0
    assert precond.precond_coefficients(edge, mu, sd, k)[3]
    for idx, val in [(0, np.nan), (2, np.inf), (3, -60.5), (2 * k, 61.0), (1, -np.inf)]:
        bad = good.copy()
        bad[idx] = val
        h, tinv, c, ok = precond.precond_coefficients(bad, mu, sd, k)
        assert not ok and tinv == -1.0 and np.all(h == 0) and np.all(c == 0), idx


def test_adam_constant_gradient_invariant():
    # with a constant gradient the bias-corrected moments are exact at every step
    # (m^_t = g, v^_t = g^2), so each step moves p by -lr g / (|g| + eps): a check of the
    # moment carry and of both bias corrections past the first step
    g = np.array([0.3, -2.0, 1e-3, 5.0])
    lr, T = 0.01, 25
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, T + 1):
        p, m, v = precond.adam_step(p, g, m, v, t, lr)
        np.testing.assert_allclose(p, -t * lr * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # the moments themselves: m_T = (1 - b1^T) g and v_T = (1 - b2^T) g^2
    np.testing.assert_allclose(m, (1 - 0.9 ** T) * g, rtol=1e-12)
    np.testing.assert_allclose(v, (1 - 0.999 ** T) * g * g, rtol=1e-12)


def test_adam_is_invariant_to_gradient_scale():
    # Adam's step depends on g only through m^ / sqrt(v^): scaling every gradient by the
    # same factor leaves the trajectory unchanged (up to eps)
    r = np.random.default_rng(3)
    G = r.standard_normal((12, 5))
    p1, m1, v1 = np.ones(5), np.zeros(5), np.zeros(5)
    p2, m2, v2 = np.ones(5), np.zeros(5), np.zeros(5)
    for t in range(1, 13):
        p1, m1, v1 = precond.adam_step(p1, G[t - 1], m1, v1, t, 1e-2, eps=0.0)
        p2, m2, v2 = precond.adam_step(p2, 1e3 * G[t - 1], m2, v2, t, 1e-2, eps=0.0)
    np.testing.assert_allclose(p1, p2, rtol=1e-12)
    # a gradient that flips sign every step: the first moment averages it out
    p, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    steps = []
    for t in range(1, 200):
        p_new, m, v = precond.adam_step(p, np.array([(-1.0) ** t]), m, v, t, 1e-3)
        steps.append(abs(p_new - p)[0])
        p = p_new
    assert steps[-1] < 0.1 * steps[0]


def test_warm_start_is_the_basis_combination():
    r = np.random.default_rng(5)
    U = r.standard_normal((30, 4))
    c = np.array([1.0, 0.0, -2.0, 0.5])
    np.testing.assert_allclose(precond.warm_start(U, c), U[:, 0] - 2 * U[:, 2] + 0.5 * U[:, 3], rtol=1e-14)
