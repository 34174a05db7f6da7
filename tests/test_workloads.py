"""The seeded input generators: determinism, shapes, and the random-Fourier-feature draw
against the squared-exponential covariance it samples from (Rahimi & Recht, 2007)."""
import numpy as np

import workloads


def test_generators_are_seeded_and_shaped():
    a, b = workloads.rff_gp(n=512, d=8, seed=3), workloads.rff_gp(n=512, d=8, seed=3)
    for k in ("X", "y", "psi"):
        np.testing.assert_array_equal(a[k], b[k])
    assert a["X"].dtype == np.float32 and a["y"].dtype == np.float32 and a["X"].shape == (512, 8)
    assert a["psi"].shape == (10,) and np.isclose(a["psi"][0], 0.0) and np.isclose(a["psi"][-1], np.log(0.05))
    ell = np.exp(a["psi"][1:-1])
    assert np.all((ell >= 0.5) & (ell <= 2.0))
    m = workloads.mixture(n=4096, d=16, seed=4)
    assert m["X"].shape == (4096, 16) and m["X"].dtype == np.float32 and m["psi"].shape == (18,)
    t = workloads.tiny()
    assert t["X"].shape == (1000, 2) and t["X"].min() >= 0.0 and t["X"].max() <= 1.0


def test_rff_draw_has_the_squared_exponential_covariance():
    # three points at scaled squared distances 0, 1 and 4 from the first: the covariance of
    # f over independent draws is sigma^2 exp(-r^2 / 2)
    ell = np.array([0.7, 1.3])
    X = np.array([[0.0, 0.0], [0.7, 0.0], [0.0, 2.6]], dtype=np.float32)
    draws = np.array([workloads._rff_draw(X, ell, 1.5, np.random.default_rng(s), n_features=512)
                      for s in range(4000)])
    C = np.cov(draws.T)
    r2 = np.array([0.0, 1.0, 4.0])
    np.testing.assert_allclose(C[0], 1.5 * np.exp(-r2 / 2), atol=0.08)
    np.testing.assert_allclose(draws.mean(axis=0), 0.0, atol=0.08)
