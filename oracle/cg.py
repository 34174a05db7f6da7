"""The Conjugate Gradient algorithm of Sec. 3.1 (Alg. 1), in FP64 (oracle).

Inputs as in Alg. 1: a product v -> K v (the covariance matrix-vector product), the
right-hand side b, the initial vector s_0, the threshold epsilon and the maximum number
of iterations T.  The residual e is the algorithm's recursively updated one, not
b - K s recomputed.  Reading taken for T: at most T products K d_i inside the loop.

Residual replacement (refresh = k > 0): after an iteration whose recursive residual norm
has fallen below 2^-k times the norm at the last replacement (or at the start), and is
above `floor`, the recursive residual is replaced by b - K s_i.  With inexact products
K d (the low-precision products of the GPU library) the recursive residual drifts from
the true one and the iterates converge to the solution of a perturbed system, which the
replacement prevents (the "reliable updates" of Sleijpen & van der Vorst, 1996, triggered
by the residual reduction as in van der Vorst & Ye, 2000).  The replacement product has
an accuracy floor of its own, and replacing the residual at that floor again and again
stalls the iteration: a replacement whose residual is not at least twice smaller than
the one at the previous replacement ends the replacements of this run.  The iteration
restarts from the replaced residual (the next direction is the residual itself, or its
preconditioned form), so that the recurrences stay consistent with it: after a
replacement at iteration i the run continues as a fresh run of Alg. 1 from s_i, and the
iterates still converge to K^-1 b, which is all the series of Sec. 4 needs.  The paper warns
that single precision hurts CG (Sec. 3.2); this is the remedy for the BF16 products.
`refresh_matvec` is the product used for the replacement (default: matvec).
"""
import numpy as np


class _Replacement:
    """The replacement rule of the module docstring for one CG run."""

    def __init__(self, k, floor, matvec, b, e0):
        self.k, self.floor, self.matvec, self.b = k, floor, matvec, b
        self.ref = np.linalg.norm(e0)
        self.on = bool(k)

    def __call__(self, s, e):
        """(residual, restart): the residual to continue with and whether it was replaced."""
        if not self.on:
            return e, False
        r = np.linalg.norm(e)
        if r < self.ref * 2.0 ** -self.k and r > self.floor:
            e = self.b - self.matvec(s)
            r_new = np.linalg.norm(e)
            if not r_new < 0.5 * self.ref:
                self.on = False
            self.ref = r_new
            return e, True
        return e, False


def cg_iterates(matvec, b, s0, refresh=0, refresh_matvec=None, floor=0.0):
    """Yield (i, s_i, e_i, delta_i) for i = 1, 2, ... following Alg. 1.

    delta_i = s_i - s_{i-1} = alpha_{i-1} d_{i-1} is the increment that the ULISSE
    series of Sec. 4 is written in.
    """
    b = np.asarray(b, dtype=np.float64)
    s = np.array(s0, dtype=np.float64, copy=True)
    e = b - matvec(s)
    replace = _Replacement(refresh, floor, refresh_matvec or matvec, b, e)
    d = e.copy()
    rho = e @ e
    i = 0
    while True:
        q = matvec(d)
        alpha = rho / (d @ q)
        delta = alpha * d
        s = s + delta
        e = e - alpha * q
        i += 1
        e, restart = replace(s, e)
        yield i, s, e, delta
        rho_next = e @ e
        beta = 0.0 if restart else rho_next / rho
        d = e + beta * d
        rho = rho_next


def cg(matvec, b, s0, eps, max_iter):
    """Plain Alg. 1: returns (s, iterations, converged, ||e||)."""
    b = np.asarray(b, dtype=np.float64)
    s = np.array(s0, dtype=np.float64, copy=True)
    e0 = b - matvec(s)
    if np.linalg.norm(e0) < eps:
        return s, 0, True, np.linalg.norm(e0)
    for i, s, e, _ in cg_iterates(matvec, b, s0):
        r = np.linalg.norm(e)
        if r < eps:
            return s, i, True, r
        if i >= max_iter:
            return s, i, False, r


def pcg_iterates(matvec, apply_pinv, b, s0, refresh=0, refresh_matvec=None, floor=0.0):
    """Preconditioned CG (the variant named in Sec. 3.3, with a preconditioner applied as
    z = P^-1 e): yields (i, s_i, e_i, delta_i) like cg_iterates.

    e is the unpreconditioned residual b - K s (recursively updated); the step lengths use
    rho = e^T z.  With P = I this is Alg. 1.
    """
    b = np.asarray(b, dtype=np.float64)
    s = np.array(s0, dtype=np.float64, copy=True)
    e = b - matvec(s)
    replace = _Replacement(refresh, floor, refresh_matvec or matvec, b, e)
    z = apply_pinv(e)
    d = z.copy()
    rho = e @ z
    i = 0
    while True:
        q = matvec(d)
        alpha = rho / (d @ q)
        delta = alpha * d
        s = s + delta
        e = e - alpha * q
        i += 1
        e, restart = replace(s, e)
        yield i, s, e, delta
        z = apply_pinv(e)
        rho_next = e @ z
        beta = 0.0 if restart else rho_next / rho
        d = z + beta * d
        rho = rho_next


def lowrank_pinv(U, h, tau_inv):
    """v -> tau_inv v + U (h * (U^T v)): inverse of the rank-k-plus-identity preconditioner
    P = U diag(dk) U^T + tau (I - U U^T) for orthonormal U, with h_k = 1/dk - 1/tau."""
    U = np.asarray(U, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    return lambda v: tau_inv * v + U @ (h * (U.T @ v))


def shifted_inner_pinv(matvec, delta, eps_inner, max_inner):
    """v -> approximate (K + delta I)^-1 v by an inner run of Alg. 1 from zero: the PCG
    variant of Sec. 3.3 whose preconditioner J = K + delta I (delta > 0) is itself applied
    by CG.

    The inner run stops at the first iterate with ||r|| < eps_inner ||v|| or after
    `max_inner` products, whichever comes first (eps_inner = 0: exactly max_inner
    iterations).  Because CG is not linear in its right-hand side, the preconditioner
    changes from one outer iteration to the next unless the inner solves converge.
    """
    def shifted(v):
        return matvec(v) + delta * v

    def apply(v):
        v = np.asarray(v, dtype=np.float64)
        nv = np.linalg.norm(v)
        if nv == 0.0:
            return np.zeros_like(v)
        for i, s, r, _ in cg_iterates(shifted, v, np.zeros_like(v)):
            if np.linalg.norm(r) < eps_inner * nv or i >= max_inner:
                return s

    return apply
