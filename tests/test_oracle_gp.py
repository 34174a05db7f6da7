"""Pins for oracle.gp: covariance, derivatives, log marginal likelihood, exact gradient.

Independent references: scikit-learn's GP kernels and log marginal likelihood (its
hyper-parameter vector is exactly psi = (log sigma^2, log ell_1..d, log lambda)),
scipy's multivariate normal, closed forms and central finite differences.
"""
import numpy as np
import pytest
import scipy.stats as st
from sklearn.gaussian_process import GaussianProcessRegressor
from sklearn.gaussian_process.kernels import RBF, ConstantKernel, WhiteKernel

from oracle import gp


def _problem(n=40, d=3, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(size=(n, d)).astype(np.float32)
    psi = np.concatenate([[np.log(1.3)], np.log(rng.uniform(0.2, 0.8, d)), [np.log(0.07)]])
    y = rng.standard_normal(n)
    return X, psi, y


def _sk_kernel(psi, d):
    return (ConstantKernel(np.exp(psi[0])) * RBF(np.exp(psi[1:d + 1]))
            + WhiteKernel(np.exp(psi[d + 1])))


def test_kernel_and_derivatives_match_sklearn():
    X, psi, _ = _problem()
    d = X.shape[1]
    k = _sk_kernel(psi, d)
    np.testing.assert_allclose(k.theta, psi, rtol=0, atol=1e-15)
    K_sk, dK_sk = k(X.astype(np.float64), eval_gradient=True)
    np.testing.assert_allclose(gp.kernel_matrix(X, psi), K_sk, rtol=1e-13, atol=1e-14)
    for j, Dj in enumerate(gp.kernel_derivatives(X, psi)):
        np.testing.assert_allclose(Dj, dK_sk[:, :, j], rtol=1e-12, atol=1e-14)


def test_log_marginal_likelihood_and_gradient_match_sklearn_and_scipy():
    X, psi, y = _problem()
    d = X.shape[1]
    k = _sk_kernel(psi, d)
    reg = GaussianProcessRegressor(kernel=k, alpha=0.0, optimizer=None, normalize_y=False)
    reg.fit(X.astype(np.float64), y)
    lml, grad = reg.log_marginal_likelihood(psi, eval_gradient=True)
    np.testing.assert_allclose(gp.log_marginal_likelihood(X, psi, y), lml, rtol=1e-12)
    np.testing.assert_allclose(gp.exact_gradient(X, psi, y), grad, rtol=1e-9, atol=1e-9)
    K = gp.kernel_matrix(X, psi)
    ref = st.multivariate_normal(mean=np.zeros(len(y)), cov=K).logpdf(y)
    np.testing.assert_allclose(gp.log_marginal_likelihood(X, psi, y), ref, rtol=1e-12)


@pytest.mark.parametrize("n,d", [(5, 1), (60, 2), (200, 3)])
def test_exact_gradient_vs_finite_differences(n, d):
    X, psi, y = _problem(n, d, seed=n)
    g = gp.exact_gradient(X, psi, y)
    h = 1e-5
    for j in range(len(psi)):
        e = np.zeros_like(psi)
        e[j] = h
        fd = (gp.log_marginal_likelihood(X, psi + e, y)
              - gp.log_marginal_likelihood(X, psi - e, y)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])), (j, fd, g[j])


def test_derivatives_vs_finite_differences():
    X, psi, _ = _problem(25, 2, seed=3)
    dK = gp.kernel_derivatives(X, psi)
    h = 1e-6
    for j in range(len(psi)):
        e = np.zeros_like(psi)
        e[j] = h
        fd = (gp.kernel_matrix(X, psi + e) - gp.kernel_matrix(X, psi - e)) / (2 * h)
        np.testing.assert_allclose(dK[j], fd, rtol=1e-7, atol=1e-9)


def test_single_point_closed_form():
    X = np.array([[0.3, -0.2]], dtype=np.float32)
    psi = np.array([np.log(2.0), 0.1, -0.4, np.log(0.3)])
    y = np.array([0.7])
    v = 2.0 + 0.3
    ref = -0.5 * np.log(v) - y[0] ** 2 / (2 * v) - 0.5 * np.log(2 * np.pi)
    np.testing.assert_allclose(gp.log_marginal_likelihood(X, psi, y), ref, rtol=1e-14)
    # d/dlog sigma^2 and d/dlog lambda of the scalar Gaussian; lengthscales do not enter
    g = gp.exact_gradient(X, psi, y)
    dv = np.array([2.0, 0.0, 0.0, 0.3])
    ref_g = -0.5 * dv / v + 0.5 * y[0] ** 2 * dv / v ** 2
    np.testing.assert_allclose(g, ref_g, rtol=1e-13, atol=1e-15)


def test_two_point_closed_form():
    X = np.array([[0.0], [0.5]], dtype=np.float32)
    s2, ell, lam = 1.5, 0.25, 0.1
    psi = np.log([s2, ell, lam])
    y = np.array([0.4, -1.1])
    k12 = s2 * np.exp(-0.5 * 0.25 / ell ** 2)
    a, c = s2 + lam, k12
    det = a * a - c * c
    quad = (a * y[0] ** 2 - 2 * c * y[0] * y[1] + a * y[1] ** 2) / det
    ref = -0.5 * np.log(det) - 0.5 * quad - np.log(2 * np.pi)
    np.testing.assert_allclose(gp.log_marginal_likelihood(X, psi, y), ref, rtol=1e-14)


def test_kernel_entries_closed_forms():
    s2, lam = 1.7, 0.2
    ell = np.array([0.5, 2.0])
    psi = np.log(np.concatenate([[s2], ell, [lam]]))
    # scaled squared distance sum_k (dx_k / ell_k)^2 = 2  ->  sigma^2 e^-1
    X = np.array([[0.0, 0.0], [0.5, 2.0]], dtype=np.float32)
    K = gp.kernel_matrix(X, psi)
    np.testing.assert_allclose(np.diag(K), s2 + lam, rtol=1e-15)
    np.testing.assert_allclose(K[0, 1], s2 * np.exp(-1.0), rtol=1e-15)
    np.testing.assert_allclose(K, K.T, rtol=0, atol=0)


def test_gradient_invariant_sigma_plus_lambda():
    # dK/dpsi_0 + dK/dpsi_{d+1} = K, hence g_0 + g_{d+1} = 1/2 y^T K^-1 y - n/2 exactly
    X, psi, y = _problem(50, 2, seed=7)
    g = gp.exact_gradient(X, psi, y)
    a = gp.solve(X, psi, y)
    np.testing.assert_allclose(g[0] + g[-1], 0.5 * y @ a - 0.5 * len(y), rtol=1e-10)


def test_lengthscale_scale_invariance():
    X, psi, y = _problem(30, 3, seed=9)
    c = 2.0  # a power of two keeps X * c exact in FP32
    psi2 = psi.copy()
    psi2[1:-1] += np.log(c)
    np.testing.assert_allclose(gp.kernel_matrix(X * np.float32(c), psi2),
                               gp.kernel_matrix(X, psi), rtol=1e-13)
    np.testing.assert_allclose(gp.log_marginal_likelihood(X * np.float32(c), psi2, y),
                               gp.log_marginal_likelihood(X, psi, y), rtol=1e-12)


def test_row_blocks_and_products_consistent():
    X, psi, _ = _problem(33, 2, seed=11)
    V = np.random.default_rng(1).standard_normal((33, 4))
    rows = np.array([0, 5, 32])
    K = gp.kernel_matrix(X, psi)
    np.testing.assert_array_equal(gp.kernel_matrix(X, psi, rows=rows), K[rows])
    np.testing.assert_allclose(gp.kmv(X, psi, V, rows=rows), (K @ V)[rows], rtol=1e-14)
    full = gp.dkmv(X, psi, V)
    np.testing.assert_allclose(gp.dkmv(X, psi, V, rows=rows), full[:, rows], rtol=1e-14)
    # the derivative blocks add up to K V for psi_0 and psi_{d+1}
    np.testing.assert_allclose(full[0] + full[-1], K @ V, rtol=1e-13, atol=1e-13)


def test_cholesky_succeeds_and_spd():
    X, psi, _ = _problem(80, 4, seed=5)
    K = gp.kernel_matrix(X, psi)
    np.linalg.cholesky(K)
    assert gp.condition_number(K) >= 1.0
