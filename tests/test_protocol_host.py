"""Host-side statistics of the SGLD protocol against the oracle's definitions (CPU)."""
import numpy as np

from oracle import diagnostics as od
from paper_1501_05427_amd import protocol


def test_psrf_matches_oracle():
    r = np.random.default_rng(0)
    x = r.standard_normal((6, 700, 3)) + r.standard_normal((6, 1, 3)) * 0.3
    np.testing.assert_allclose(protocol.psrf(x), od.psrf(x), rtol=1e-12)
    np.testing.assert_allclose(protocol.psrf(x[:, :, 0]), od.psrf(x[:, :, 0]), rtol=1e-12)


def test_ess_matches_oracle():
    r = np.random.default_rng(1)
    T = 3001
    e = r.standard_normal((T, 2))
    x = np.empty_like(e)
    x[0] = e[0]
    for t in range(1, T):
        x[t] = np.array([0.7, 0.95]) * x[t - 1] + e[t]
    np.testing.assert_allclose(protocol.ess(x), od.ess(x), rtol=1e-9)


def test_init_chains_moments():
    M = np.array([[2.0, 0.3], [0.3, 0.5]])
    Z = protocol.init_chains(np.array([1.0, -2.0]), M, 200000, seed=3)
    np.testing.assert_allclose(Z.mean(0), [1.0, -2.0], atol=0.01)
    np.testing.assert_allclose(np.cov(Z.T), M, atol=0.02)
