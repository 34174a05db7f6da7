"""Pins for oracle.diagnostics: PSRF, ESS, the subset MAP and its negative Hessian."""
import numpy as np
import scipy.optimize as so

from oracle import diagnostics as od
from oracle import gp


def test_psrf_identical_chains_and_iid_chains():
    z = np.random.default_rng(0).standard_normal(500)
    # identical chains: B = 0, so PSRF = sqrt((T - 1) / T) exactly
    np.testing.assert_allclose(od.psrf(np.tile(z, (4, 1))), np.sqrt(499 / 500), rtol=1e-14)
    iid = np.random.default_rng(1).standard_normal((10, 4000, 3))
    r = od.psrf(iid)
    assert np.all(np.abs(r - 1.0) < 0.01), r
    # invariant under a common affine map of all chains
    np.testing.assert_allclose(od.psrf(3.0 * iid - 7.0), r, rtol=1e-12)


def test_psrf_detects_separated_chains():
    x = np.random.default_rng(2).standard_normal((4, 1000)) + np.arange(4)[:, None] * 2.0
    assert od.psrf(x)[0] > 2.0


def test_psrf_two_chains_brute_force():
    # two chains of length 3, the definition evaluated by hand-expanded sums
    a = [1.0, 2.0, 4.0]
    b = [0.0, 3.0, 3.0]
    ma, mb = 7.0 / 3.0, 2.0
    va = sum((v - ma) ** 2 for v in a) / 2.0
    vb = sum((v - mb) ** 2 for v in b) / 2.0
    W = (va + vb) / 2.0
    mm = (ma + mb) / 2.0
    B_over_T = ((ma - mm) ** 2 + (mb - mm) ** 2) / 1.0
    V = 2.0 / 3.0 * W + 1.5 * B_over_T
    np.testing.assert_allclose(od.psrf(np.array([a, b]))[0], np.sqrt(V / W), rtol=1e-14)


def test_ess_iid_and_ar1():
    r = np.random.default_rng(3)
    iid = r.standard_normal(20000)
    assert 0.9 < od.ess(iid)[0] / 20000 < 1.1
    # AR(1) x_t = phi x_{t-1} + e_t: integrated autocorrelation time (1 + phi) / (1 - phi)
    phi, T = 0.9, 40000
    e = r.standard_normal(T)
    x = np.empty(T)
    x[0] = e[0] / np.sqrt(1 - phi ** 2)
    for t in range(1, T):
        x[t] = phi * x[t - 1] + e[t]
    ratio = od.ess(x)[0] / (T * (1 - phi) / (1 + phi))
    assert 0.8 < ratio < 1.25, ratio


def _small_gp(n=60, seed=4):
    r = np.random.default_rng(seed)
    X = r.uniform(size=(n, 2)).astype(np.float32)
    psi = np.log([1.0, 0.3, 0.5, 0.1])
    K = gp.kernel_matrix(X, psi)
    y = np.linalg.cholesky(K) @ r.standard_normal(n)
    return X, y, psi


def test_neg_hessian_matches_second_differences_of_log_p():
    X, y, psi = _small_gp()
    A = od.neg_hessian(X, y, psi)
    h = 1e-3
    P = len(psi)
    H2 = np.empty((P, P))
    lp = lambda p: gp.log_marginal_likelihood(X, p, y)
    for j in range(P):
        for k in range(P):
            ej, ek = np.eye(P)[j] * h, np.eye(P)[k] * h
            H2[j, k] = (lp(psi + ej + ek) - lp(psi + ej - ek) - lp(psi - ej + ek) + lp(psi - ej - ek)) / (4 * h * h)
    np.testing.assert_allclose(A, -H2, rtol=2e-4, atol=2e-4 * np.abs(H2).max())
    # a Gaussian prior N(a, b^2) adds 1 / b^2 to the diagonal
    b = np.full(P, 2.0)
    np.testing.assert_allclose(od.neg_hessian(X, y, psi, 1, np.zeros(P), b) - A, np.eye(P) / 4.0,
                               atol=1e-6)


def test_subset_map_matches_a_library_optimiser():
    X, y, psi = _small_gp()
    P = len(psi)
    a, b = np.zeros(P), np.full(P, 3.0)
    psi_map, A = od.subset_map(X, y, psi + 0.2, 1, a, b)
    f = lambda p: -(gp.log_marginal_likelihood(X, p, y) - 0.5 * np.sum(((p - a) / b) ** 2))
    ref = so.minimize(f, psi + 0.2, method="Nelder-Mead",
                      options={"xatol": 1e-10, "fatol": 1e-12, "maxiter": 20000, "maxfev": 40000})
    np.testing.assert_allclose(psi_map, ref.x, atol=1e-4)
    assert np.all(np.linalg.eigvalsh(A) > 0)
