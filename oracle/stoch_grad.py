"""Unbiased stochastic gradient of the log marginal likelihood, FP64 (oracle).

eq. gradient:unbiased with probe index c and parameter index j (the paper reuses i for
both), and with the y-term formed from two independent ULISSE estimates of K^-1 y that
share one CG run (Sec. 4.1):
    g~_j = 1/2 s~_a^T dK_j s~_b - 1/(2 N_r) sum_c r_c^T dK_j s~_c,
where s~_c estimates K^-1 r_c.  Every product is dense FP64.
"""
import numpy as np

from . import gp as _gp
from . import rng as _rng
from . import ulisse as _ul


def assemble(X, psi, R, St):
    """Gradient from the solutions: St columns = (s~_a, s~_b, s~_1, ..., s~_Nr)."""
    R = np.asarray(R, dtype=np.float64)
    nr = R.shape[1]
    dK = _gp.kernel_derivatives(X, psi)
    g = np.empty(len(dK))
    for j, Dj in enumerate(dK):
        quad = 0.5 * St[:, 0] @ Dj @ St[:, 1]
        tr = sum(R[:, c] @ Dj @ St[:, 2 + c] for c in range(nr))
        g[j] = quad - tr / (2.0 * nr)
    return g


def stoch_grad(X, psi, y, R, q, rate, eps, max_iter, seed, stream, step,
               S_warm=None, eps_relative=False, apply_pinv=None, refresh=0):
    """One unbiased gradient estimate.  R (n, N_r) holds the probes r_c.

    Returns (g, St, S_cg, stats); S_cg are the last CG iterates (warm starts).
    """
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    K = _gp.kernel_matrix(X, psi)
    B = np.column_stack([y, R])
    St, Scg, stats = _ul.solve_systems(lambda v: K @ v, B, S_warm, q, rate, eps, max_iter,
                                       seed, stream, step, two_track_first=True,
                                       eps_relative=eps_relative, apply_pinv=apply_pinv,
                                       refresh=refresh)
    return assemble(X, psi, R, St), St, Scg, stats


def draw_probes(seed, stream, step, n, n_probes, kind):
    return _rng.probes(seed, stream, step, n, n_probes, kind)
