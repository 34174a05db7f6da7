"""Chain diagnostics and the SGLD preconditioner of the paper's experiments, FP64 (oracle).

* psrf: the potential scale reduction factor of Gelman & Rubin (1992), used in Sec. 5 to
  assess convergence of parallel SGLD chains.  For m chains of length T and one parameter,
  W is the mean within-chain variance and B / T the variance of the chain means;
  V = (T - 1) / T W + (1 + 1 / m) B / T and PSRF = sqrt(V / W).
* ess: effective sample size T / tau with tau = 1 + 2 sum_k rho_k, the autocorrelations
  summed by Geyer's initial positive sequence (pairs rho_{2k} + rho_{2k+1} while they are
  positive), the estimator behind the paper's "effective sample size" figures.
* subset_map / neg_hessian: the MAP of log p(y | psi) + log p(psi) on a data subset and
  the negative Hessian there; its inverse is the SGLD preconditioner M of Sec. 5, and
  N(psi_MAP, M) is the paper's distribution of chain starting points.  The Hessian is the
  central difference of the exact gradient; the MAP is found by Newton steps on it.
"""
import numpy as np

from . import gp as _gp
from . import sgld as _sgld


def psrf(chains):
    """chains: (m, T) or (m, T, P) -> PSRF per parameter."""
    x = np.asarray(chains, dtype=np.float64)
    if x.ndim == 2:
        x = x[:, :, None]
    m, T, _ = x.shape
    means = x.mean(axis=1)                      # (m, P)
    W = x.var(axis=1, ddof=1).mean(axis=0)      # mean within-chain variance
    B_over_T = means.var(axis=0, ddof=1)        # variance of the chain means
    V = (T - 1) / T * W + (1.0 + 1.0 / m) * B_over_T
    return np.sqrt(V / W)


def autocorrelation(x, k):
    """Sample autocorrelation of x at lag k (biased covariance estimate, divided by T)."""
    x = np.asarray(x, dtype=np.float64)
    T = x.shape[0]
    c = x - x.mean()
    return (c[:T - k] @ c[k:]) / (c @ c)


def ess(x):
    """x: (T,) or (T, P) -> effective sample size per parameter."""
    x = np.asarray(x, dtype=np.float64)
    if x.ndim == 1:
        x = x[:, None]
    T, P = x.shape
    out = np.empty(P)
    for j in range(P):
        tau = -1.0  # tau = -rho_0 + 2 sum of the positive pair sums (rho_0 = 1)
        k = 0
        while 2 * k + 1 < T:
            pair = autocorrelation(x[:, j], 2 * k) + autocorrelation(x[:, j], 2 * k + 1)
            if pair <= 0.0:
                break
            tau += 2.0 * pair
            k += 1
        out[j] = T / max(tau, 1e-300)
    return out


def log_post_grad(X, y, psi, prior_kind=0, a=None, b=None):
    return _gp.exact_gradient(X, psi, y) + _sgld.prior_grad(psi, prior_kind, a, b)


def neg_hessian(X, y, psi, prior_kind=0, a=None, b=None, h=1e-4):
    """-d^2/dpsi^2 [log p(y | psi) + log p(psi)] by central differences of the gradient."""
    psi = np.asarray(psi, dtype=np.float64)
    P = psi.shape[0]
    H = np.empty((P, P))
    for k in range(P):
        e = np.zeros(P)
        e[k] = h
        H[:, k] = (log_post_grad(X, y, psi + e, prior_kind, a, b)
                   - log_post_grad(X, y, psi - e, prior_kind, a, b)) / (2 * h)
    return -0.5 * (H + H.T)


def subset_map(X, y, psi0, prior_kind=0, a=None, b=None, iters=50, tol=1e-8):
    """Newton iterations psi <- psi + (-H)^-1 g from psi0 (halving the step while it does
    not reduce ||g||); returns (psi_MAP, -H at psi_MAP)."""
    psi = np.asarray(psi0, dtype=np.float64).copy()
    g = log_post_grad(X, y, psi, prior_kind, a, b)
    for _ in range(iters):
        A = neg_hessian(X, y, psi, prior_kind, a, b)
        step = np.linalg.solve(A, g)
        t = 1.0
        while True:
            cand = psi + t * step
            gc = log_post_grad(X, y, cand, prior_kind, a, b)
            if np.linalg.norm(gc) < np.linalg.norm(g) or t < 1e-6:
                break
            t *= 0.5
        psi, g = cand, gc
        if np.linalg.norm(g) < tol * max(1.0, len(y)):
            break
    return psi, neg_hessian(X, y, psi, prior_kind, a, b)
