"""Preconditioned SGLD update of Sec. 2.1, its step-size schedule and Langevin-phase
monitor, and the priors on psi, FP64 (oracle).

psi_{t+1} = psi_t + eps_t/2 M (g~ + grad log p(psi)) + eta_t,  eta_t ~ N(0, eps_t M),
with M = L L^T given by its lower Cholesky factor L and eta_t = sqrt(eps_t) L xi.

Priors (the paper leaves the prior of its experiments unspecified):
  kind 0  flat                                   grad = 0
  kind 1  psi_j ~ N(a_j, b_j^2)                  grad = -(psi_j - a_j) / b_j^2
  kind 2  theta_j = exp(psi_j) ~ Gamma(a_j, b_j)  (shape a, rate b; Jacobian included)
          log p(psi_j) = a_j psi_j - b_j exp(psi_j) + const,  grad = a_j - b_j exp(psi_j)
"""
import numpy as np

from . import rng as _rng


def prior_grad(psi, kind, a=None, b=None):
    psi = np.asarray(psi, dtype=np.float64)
    if kind == 0:
        return np.zeros_like(psi)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if kind == 1:
        return -(psi - a) / (b * b)
    if kind == 2:
        return a - b * np.exp(psi)
    raise ValueError("prior kind must be 0, 1 or 2")


def step(psi, g, eps, L=None, xi=None, prior_kind=0, a=None, b=None):
    psi = np.asarray(psi, dtype=np.float64)
    P = psi.shape[0]
    L = np.eye(P) if L is None else np.asarray(L, dtype=np.float64)
    xi = np.zeros(P) if xi is None else np.asarray(xi, dtype=np.float64)
    M = L @ L.T
    drift = 0.5 * eps * (M @ (np.asarray(g, dtype=np.float64) + prior_grad(psi, prior_kind, a, b)))
    return psi + drift + np.sqrt(eps) * (L @ xi)


def step_drawn(psi, g, eps, seed, stream, step_index, L=None, prior_kind=0, a=None, b=None):
    """SGLD update with xi drawn from the SGLD Philox stream of this step."""
    xi = _rng.sgld_normals(seed, stream, step_index, len(psi))
    return step(psi, g, eps, L, xi, prior_kind, a, b)


def eps_schedule(a, b, gamma, t):
    """Step size eps_t = a (b + t)^(-gamma) (Sec. 2.1; gamma = 1 in Sec. 5.1)."""
    return a * (b + np.asarray(t, dtype=np.float64)) ** (-gamma)


def schedule_from_endpoints(eps_first, eps_last, T):
    """(a, b) of eps_t = a / (b + t) with eps_0 = eps_first and eps_{T-1} = eps_last, the
    reading of the decreasing schedules of Sec. 5.1 (e.g. 1e-1 to 1e-4 over 40000 steps)."""
    b = (T - 1) * eps_last / (eps_first - eps_last)
    return eps_first * b, b


def langevin_ratio(G, L, eps):
    """(eps / 4) lambda_max(M^(1/2) V M^(1/2)) with V the sample covariance of the rows of G
    (divisor rows - 1) and M = L L^T (Sec. 2.1)."""
    G = np.asarray(G, dtype=np.float64)
    V = np.cov(G, rowvar=False, ddof=1)
    L = np.eye(G.shape[1]) if L is None else np.asarray(L, dtype=np.float64)
    B = L.T @ V @ L
    return 0.25 * eps * np.linalg.eigvalsh(0.5 * (B + B.T))[-1]
