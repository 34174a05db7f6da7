"""Preconditioned SGLD update of Sec. 2.1 and the priors on psi, FP64 (oracle).

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
