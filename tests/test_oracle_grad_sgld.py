"""Pins for oracle.stoch_grad (eq. gradient:unbiased) and oracle.sgld (Sec. 2.1)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.stats as st

from oracle import gp, rng, sgld, stoch_grad, ulisse


def _gp(n=30, seed=0, lam=0.1):
    r = np.random.default_rng(seed)
    X = r.uniform(size=(n, 2)).astype(np.float32)
    psi = np.log([1.0, 0.3, 0.4, lam])
    K = gp.kernel_matrix(X, psi)
    y = np.linalg.cholesky(K) @ r.standard_normal(n)
    return X, psi, y


def test_assemble_with_exact_solves_and_unit_probes_is_the_exact_gradient():
    # r_c = sqrt(n) e_c for c = 1..n makes the probe average the exact trace
    X, psi, y = _gp(20)
    n = len(y)
    R = np.sqrt(n) * np.eye(n)
    S = gp.solve(X, psi, np.column_stack([y, y, R]))
    g = stoch_grad.assemble(X, psi, R, S)
    np.testing.assert_allclose(g, gp.exact_gradient(X, psi, y), rtol=1e-9, atol=1e-10)


@pytest.mark.parametrize("kind", [0, 1])
def test_hutchinson_mean_and_variance_closed_forms(kind):
    # E[r^T B r] = Tr(B); Var = 2 ||B_s||_F^2 (Gaussian) or 2(||B_s||_F^2 - sum diag^2)
    X, psi, y = _gp(25, seed=1)
    n = len(y)
    K = gp.kernel_matrix(X, psi)
    dK = gp.kernel_derivatives(X, psi)
    a = gp.solve(X, psi, y)
    N = 20000
    R = rng.probes(3, 4, 0, n, N, kind)
    KR = gp.solve(X, psi, R)
    for j in range(len(psi)):
        B = sla.solve(K, dK[j])
        Bs = 0.5 * (B + B.T)
        var = 2 * np.sum(Bs ** 2) - (2 * np.sum(np.diag(Bs) ** 2) if kind == 1 else 0.0)
        samples = np.einsum("ic,ic->c", R, dK[j] @ KR)
        np.testing.assert_allclose(np.mean((samples - samples.mean()) ** 2), var, rtol=0.08)
        assert abs(samples.mean() - np.trace(B)) < 5 * np.sqrt(var / N)
        # the estimator built from the same samples
        g_est = 0.5 * a @ dK[j] @ a - samples.mean() / 2.0
        assert abs(g_est - gp.exact_gradient(X, psi, y)[j]) < 5 * 0.5 * np.sqrt(var / N)


def test_stochastic_gradient_conditional_mean_is_cg_solution_gradient():
    # for fixed probes, E over the u_j draws of g~ = gradient built from the CG solutions
    # (two independent tracks make the quadratic term unbiased)
    X, psi, y = _gp(25, seed=2, lam=0.2)
    n = len(y)
    R = rng.probes(1, 1, 0, n, 3, 0)
    q, rate, eps = 0.05, 0.05, 1e-13
    S_exact = gp.solve(X, psi, np.column_stack([y, y, R]))
    target = stoch_grad.assemble(X, psi, R, S_exact)
    N = 3000
    gs = np.array([stoch_grad.stoch_grad(X, psi, y, R, q, rate, eps, 1000, 9, 9, k)[0]
                   for k in range(N)])
    se = gs.std(axis=0, ddof=1) / np.sqrt(N)
    z = (gs.mean(axis=0) - target) / se
    assert np.all(np.abs(z) < 5.0), z


def test_stochastic_gradient_structure():
    X, psi, y = _gp(30, seed=3)
    n = len(y)
    R = rng.probes(1, 2, 3, n, 4, 1)
    g, St, Scg, stats = stoch_grad.stoch_grad(X, psi, y, R, 1.0, 1.0, 1e-8, 1000, 1, 2, 3)
    assert g.shape == (4,) and St.shape == (n, 6) and Scg.shape == (n, 5)
    assert all(s["l"] >= 1 for s in stats) and len(stats[0]["J"]) == 2
    np.testing.assert_allclose(g, stoch_grad.assemble(X, psi, R, St), rtol=1e-14)


def test_prior_gradients_vs_finite_differences():
    psi = np.array([0.3, -1.2, 0.8])
    a = np.array([2.0, 1.5, 3.0])
    b = np.array([1.0, 0.5, 2.0])
    h = 1e-6

    def logp(kind, p):
        if kind == 1:
            return st.norm(a, b).logpdf(p).sum()
        return (st.gamma(a, scale=1 / b).logpdf(np.exp(p)) + p).sum()  # Jacobian

    for kind in (1, 2):
        g = sgld.prior_grad(psi, kind, a, b)
        for j in range(3):
            e = np.zeros(3)
            e[j] = h
            fd = (logp(kind, psi + e) - logp(kind, psi - e)) / (2 * h)
            assert abs(fd - g[j]) < 1e-6
    np.testing.assert_array_equal(sgld.prior_grad(psi, 0), 0.0)


def test_step_formula_and_drawn_noise():
    psi = np.array([0.1, 0.2])
    g = np.array([1.0, -2.0])
    L = np.array([[2.0, 0.0], [0.5, 1.0]])
    xi = np.array([0.3, -0.7])
    out = sgld.step(psi, g, 0.01, L, xi)
    np.testing.assert_allclose(out, psi + 0.005 * (L @ L.T @ g) + 0.1 * (L @ xi), rtol=1e-15)
    out2 = sgld.step_drawn(psi, g, 0.01, 1, 2, 7, L)
    np.testing.assert_allclose(out2, sgld.step(psi, g, 0.01, L, rng.sgld_normals(1, 2, 7, 2)))


@pytest.mark.parametrize("v", [0.0, 2.0])
def test_stationary_variance_on_gaussian_target(v):
    # 1-D target N(mu, s), M = 1: x' = mu + A (x - mu) + sqrt(eps) xi + (eps/2) noise,
    # A = 1 - eps/(2 s);  C = (eps + eps^2 v / 4) / (1 - A^2)
    mu, s, eps = 0.7, 1.3, 0.5
    A = 1 - eps / (2 * s)
    C = (eps + eps ** 2 * v / 4) / (1 - A ** 2)
    r = np.random.default_rng(0)
    chains = 400
    x = np.full(chains, mu)
    L = np.eye(chains)
    acc = []
    for t in range(3000):
        g = -(x - mu) / s + np.sqrt(v) * r.standard_normal(chains)
        x = sgld.step(x, g, eps, L, r.standard_normal(chains))
        if t >= 200:
            acc.append(x.copy())
    acc = np.array(acc)
    np.testing.assert_allclose(acc.mean(), mu, atol=0.02)
    np.testing.assert_allclose(acc.var(), C, rtol=0.03)
    assert abs(acc.var() - s) > 0.05 * s  # the eps-bias is visible and predicted


def test_sgld_recovers_tiny_gp_posterior():
    # two free log-parameters (log ell_1, log lambda); grid posterior as reference
    r = np.random.default_rng(5)
    n = 30
    X = r.uniform(size=(n, 2)).astype(np.float32)
    truth = np.log([1.0, 0.3, 0.3, 0.1])
    y = np.linalg.cholesky(gp.kernel_matrix(X, truth)) @ r.standard_normal(n)
    free = [1, 3]
    pa, pb = truth[free], np.array([1.0, 1.0])  # N(truth, 1) prior on the free ones

    def logpost(f):
        p = truth.copy()
        p[free] = f
        return gp.log_marginal_likelihood(X, p, y) + st.norm(pa, pb).logpdf(f).sum()

    g1 = np.linspace(truth[1] - 2.5, truth[1] + 2.5, 81)
    g2 = np.linspace(truth[3] - 3.0, truth[3] + 2.0, 81)
    lp = np.array([[logpost(np.array([u, w])) for w in g2] for u in g1])
    w = np.exp(lp - lp.max())
    w /= w.sum()
    G1, G2 = np.meshgrid(g1, g2, indexing="ij")
    mean = np.array([(w * G1).sum(), (w * G2).sum()])
    cov = np.array([[(w * (G1 - mean[0]) ** 2).sum(), (w * (G1 - mean[0]) * (G2 - mean[1])).sum()],
                    [0, (w * (G2 - mean[1]) ** 2).sum()]])
    cov[1, 0] = cov[0, 1]
    Lm = np.linalg.cholesky(cov)
    eps = 0.1
    f = mean.copy()
    draws = []
    nr = np.random.default_rng(6)
    for t in range(12000):
        p = truth.copy()
        p[free] = f
        g = gp.exact_gradient(X, p, y)[free]
        f = sgld.step(f, g, eps, Lm, nr.standard_normal(2), prior_kind=1, a=pa, b=pb)
        draws.append(f.copy())
    draws = np.array(draws[1000:])
    # batch means for the Monte Carlo error of the chain average
    bm = draws.reshape(50, -1, 2).mean(axis=1)
    se = bm.std(axis=0, ddof=1) / np.sqrt(50)
    assert np.all(np.abs(draws.mean(axis=0) - mean) < 4 * se + 0.02 * np.sqrt(np.diag(cov)))
    np.testing.assert_allclose(draws.var(axis=0), np.diag(cov), rtol=0.2)


def test_schedule_endpoints_and_monotone():
    a, b = sgld.schedule_from_endpoints(1e-1, 1e-4, 40000)
    np.testing.assert_allclose(sgld.eps_schedule(a, b, 1.0, 0), 1e-1, rtol=1e-12)
    np.testing.assert_allclose(sgld.eps_schedule(a, b, 1.0, 39999), 1e-4, rtol=1e-12)
    e = sgld.eps_schedule(a, b, 1.0, np.arange(40000))
    assert np.all(np.diff(e) < 0)
    # the conditions of Sec. 2.1: sum eps_t diverges (harmonic), sum eps_t^2 converges
    np.testing.assert_allclose(a, 4.0039, rtol=1e-4)


def test_langevin_ratio_matches_symmetric_square_root_form():
    import scipy.linalg as sla
    r = np.random.default_rng(3)
    G = r.standard_normal((100, 5)) @ r.standard_normal((5, 5))
    A = r.standard_normal((5, 5))
    M = A @ A.T + 5 * np.eye(5)
    L = np.linalg.cholesky(M)
    Mh = np.real(sla.sqrtm(M))
    V = np.cov(G.T)
    ref = 0.25 * 0.01 * np.max(np.linalg.eigvalsh(Mh @ V @ Mh))
    np.testing.assert_allclose(sgld.langevin_ratio(G, L, 0.01), ref, rtol=1e-10)
    np.testing.assert_allclose(sgld.langevin_ratio(G, None, 0.01),
                               0.25 * 0.01 * np.linalg.eigvalsh(V)[-1], rtol=1e-12)
