"""Seeded synthetic inputs for the GP workloads (shared by the tests and the benchmark).

This module only draws random inputs; it contains none of the method's arithmetic
(no covariance, no solver).  The two public datasets the paper measures on (UCI
Concrete, n = 1030, d = 8; DELVE Census 8L, n = 22784, d = 8) are not available; these
generators stand in for them at the shapes of the workloads below.

Draw order is fixed per workload so that a seed reproduces every array.

  tiny        n = 1000, d = 2, X ~ U[0,1]^2 (FP64 draw, stored FP32), sigma^2 = 1,
              ell = (0.3, 0.3), lambda = 0.1; z ~ N(0, I) for y = chol(K) z (the caller
              forms y because that needs the covariance); seed 0
  rff_gp      X ~ N(0, I) (FP32), ell_k = exp(U[log 0.5, log 2]) drawn first,
              sigma^2 = 1, lambda = 0.05, y = f + sqrt(lambda) N(0, 1) with f a
              2048-feature random-Fourier-feature draw of the SE-ARD GP; n = 16384
              (seed 1) and n = 65536 (seed 2), d = 8
  mixture     X from 8 equal-weight unit-covariance Gaussians with centres ~ N(0, 9 I)
              (the spread is our reading), d = 16, n = 131072, seed 4
"""
import numpy as np


def psi_from(sigma2, ell, lam):
    """Log-parameter vector (log sigma^2, log ell_1..d, log lambda)."""
    ell = np.atleast_1d(np.asarray(ell, dtype=np.float64))
    return np.concatenate([[np.log(sigma2)], np.log(ell), [np.log(lam)]])


def tiny(n=1000, seed=0):
    """X (float32), psi, z (the standard normals that y = chol(K) z is built from)."""
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.0, 1.0, size=(n, 2)).astype(np.float32)
    z = rng.standard_normal(n)
    return dict(X=X, psi=psi_from(1.0, [0.3, 0.3], 0.1), z=z)


def _rff_draw(X, ell, sigma2, rng, n_features=2048, chunk=8192):
    d = X.shape[1]
    omega = rng.standard_normal((n_features, d))
    phase = rng.uniform(0.0, 2.0 * np.pi, n_features)
    w = rng.standard_normal(n_features)
    f = np.empty(X.shape[0])
    scale = np.sqrt(2.0 * sigma2 / n_features)
    for s in range(0, X.shape[0], chunk):
        Xs = X[s:s + chunk].astype(np.float64) / ell
        f[s:s + chunk] = scale * (np.cos(Xs @ omega.T + phase) @ w)
    return f


def rff_gp(n=16384, d=8, seed=1, sigma2=1.0, lam=0.05, n_features=2048):
    """X (float32), psi (truth), y (float32) from a random-Fourier-feature GP draw."""
    rng = np.random.default_rng(seed)
    ell = np.exp(rng.uniform(np.log(0.5), np.log(2.0), d))
    X = rng.standard_normal((n, d)).astype(np.float32)
    f = _rff_draw(X, ell, sigma2, rng, n_features)
    y = (f + np.sqrt(lam) * rng.standard_normal(n)).astype(np.float32)
    return dict(X=X, psi=psi_from(sigma2, ell, lam), y=y)


def mixture(n=131072, d=16, seed=4, n_comp=8, spread=3.0, sigma2=1.0, lam=0.05):
    rng = np.random.default_rng(seed)
    ell = np.exp(rng.uniform(np.log(0.5), np.log(2.0), d)) * np.sqrt(d / 8.0)
    centres = spread * rng.standard_normal((n_comp, d))
    lab = rng.integers(0, n_comp, n)
    X = (centres[lab] + rng.standard_normal((n, d))).astype(np.float32)
    f = _rff_draw(X, ell, sigma2, rng)
    y = (f + np.sqrt(lam) * rng.standard_normal(n)).astype(np.float32)
    return dict(X=X, psi=psi_from(sigma2, ell, lam), y=y)


def gaussian_matrix(n, m, seed):
    """Seeded FP32 N(0, 1) matrix, e.g. right-hand sides or probes supplied by the caller."""
    return np.random.default_rng(seed).standard_normal((n, m)).astype(np.float32)


def rademacher_matrix(n, m, seed):
    return np.where(np.random.default_rng(seed).random((n, m)) < 0.5, -1.0, 1.0).astype(np.float32)


WORKLOADS = {
    "tiny_n1000_d2": dict(n=1000, d=2, m=5, probes=4, probe_kind="rademacher"),
    "rff_n16384_d8_m17": dict(n=16384, d=8, m=17, probes=16, probe_kind="gaussian"),
    "rff_n65536_d8_m32": dict(n=65536, d=8, m=32, probes=31, probe_kind="gaussian"),
}
