"""Learned preconditioner quantities in FP64 (oracle).

The paper has no learned component; it only notes that ULISSE applies to any CG variant
(Sec. 4) and studies a preconditioned CG (Sec. 3.3).  What is checked here is plain
arithmetic:

  galerkin_targets  T = U^T K U, w = U^T y;  c = T^-1 w, log diag T,
                    log tau with tau = (tr K - tr T) / (n - k)
  MLP               in -> H (tanh) -> H (tanh) -> O on standardised inputs, mean squared
                    error on standardised targets, hand-written backpropagation
  Adam              Kingma & Ba (2015), bias-corrected moments
  coefficients      network output -> (h, tau_inv, c), with the plain solver as fallback
                    when the output is unusable
"""
import numpy as np

from . import gp as _gp


def galerkin_targets(X, psi, y, U):
    U = np.asarray(U, dtype=np.float64)
    n, k = U.shape
    K = _gp.kernel_matrix(X, psi)
    T = U.T @ K @ U
    w = U.T @ np.asarray(y, dtype=np.float64)
    c = np.linalg.solve(T, w)
    tau = (np.trace(K) - np.trace(T)) / (n - k)
    return np.concatenate([c, np.log(np.diag(T)), [np.log(tau)]])


def mlp_forward(params, psis):
    """Returns (outputs, cache); params: dict W1, b1, W2, b2, W3, b3, in_mu, in_sd."""
    x = (np.asarray(psis, dtype=np.float64) - params["in_mu"]) / params["in_sd"]
    a1 = np.tanh(x @ params["W1"] + params["b1"])
    a2 = np.tanh(a1 @ params["W2"] + params["b2"])
    y = a2 @ params["W3"] + params["b3"]
    return y, (x, a1, a2)


def mlp_loss(params, psis, targets):
    y, _ = mlp_forward(params, psis)
    t = (np.asarray(targets, dtype=np.float64) - params["out_mu"]) / params["out_sd"]
    return np.mean((y - t) ** 2)


def mlp_grad(params, psis, targets):
    """Loss and gradients by backpropagation (chain rule through the three layers)."""
    y, (x, a1, a2) = mlp_forward(params, psis)
    t = (np.asarray(targets, dtype=np.float64) - params["out_mu"]) / params["out_sd"]
    B, O = y.shape
    dy = 2.0 * (y - t) / (B * O)
    g = {"W3": a2.T @ dy, "b3": dy.sum(axis=0)}
    d2 = (dy @ params["W3"].T) * (1.0 - a2 ** 2)
    g["W2"] = a1.T @ d2
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ params["W2"].T) * (1.0 - a1 ** 2)
    g["W1"] = x.T @ d1
    g["b1"] = d1.sum(axis=0)
    return np.mean((y - t) ** 2), g


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (returns new p, m, v) at step t >= 1."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def precond_coefficients(outputs, out_mu, out_sd, k):
    """Network output (standardised) -> (h, tau_inv, c, accepted) of
    P^-1 = tau^-1 I + U diag(h) U^T and the warm start s0 = U c, with d floored at tau.

    u = out_mu + out_sd * outputs holds c (k values), log d (k) and log tau.  The output is
    rejected when any u is not finite or a log d or log tau lies outside [-60, 60]: the
    solver then falls back to plain CG, represented as h = 0, tau_inv = -1, c = 0 and
    accepted = False.
    """
    u = np.asarray(out_mu, dtype=np.float64) + np.asarray(out_sd, dtype=np.float64) * np.asarray(outputs, dtype=np.float64)
    logs = u[k:2 * k + 1]
    if not np.all(np.isfinite(u)) or np.any(np.abs(logs) > 60.0):
        return np.zeros(k), -1.0, np.zeros(k), False
    tau = np.exp(u[2 * k])
    d = np.maximum(np.exp(u[k:2 * k]), tau)
    return 1.0 / d - 1.0 / tau, 1.0 / tau, u[:k], True


def warm_start(U, c):
    """s0 = U c, the learned warm start of the y system."""
    return np.asarray(U, dtype=np.float64) @ np.asarray(c, dtype=np.float64)
