"""Covariance function and the quantities built from it, in FP64 (oracle).

Parametrisation (log-parameters, fixed order):
    psi = (log sigma^2, log ell_1, ..., log ell_d, log lambda),  P = d + 2.

Covariance (Sec. 2, eq. covariance:rbf, in its ARD form with a decaying exponent):
    k(x_i, x_j) = sigma^2 exp(-1/2 sum_k (x_ik - x_jk)^2 / ell_k^2) + lambda delta_ij.
The paper writes the isotropic form with one decay rate tau = 1/(2 ell^2); equal ell_k
recover it.

Derivatives with respect to psi (derived here; the paper uses them in eq.
gradient:exact without writing them out):
    dK/dpsi_0     = K_f                              (signal part, K - lambda I)
    dK/dpsi_k     = K_f * (x_ik - x_jk)^2 / ell_k^2  (k = 1..d)
    dK/dpsi_{d+1} = lambda I

Log marginal likelihood (Sec. 2): -1/2 log|K| - 1/2 y^T K^-1 y - n/2 log(2 pi), via
Cholesky. Exact gradient (eq. gradient:exact):
    g_j = -1/2 Tr(K^-1 dK_j) + 1/2 y^T K^-1 dK_j K^-1 y.

Every function takes X as an (n, d) array; it is promoted to FP64 exactly.
"""
import numpy as np
import scipy.linalg as sla


def unpack_psi(psi, d):
    """Return (sigma2, ell[d], lam) from the log-parameter vector."""
    psi = np.asarray(psi, dtype=np.float64)
    if psi.shape != (d + 2,):
        raise ValueError(f"psi must have {d + 2} entries, got {psi.shape}")
    return np.exp(psi[0]), np.exp(psi[1:d + 1]), np.exp(psi[d + 1])


def _sq_diffs(X, psi, rows=None, cols=None):
    """Per-dimension scaled squared differences (x_ik - x_jk)^2 / ell_k^2, shape (d, r, c)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    _, ell, _ = unpack_psi(psi, d)
    Xr = X if rows is None else X[rows]
    Xc = X if cols is None else X[cols]
    out = np.empty((d, Xr.shape[0], Xc.shape[0]))
    for k in range(d):
        diff = Xr[:, k][:, None] - Xc[:, k][None, :]   # explicit difference
        out[k] = diff * diff / (ell[k] * ell[k])
    return out


def _diag_mask(n, rows, cols):
    r = np.arange(n) if rows is None else np.asarray(rows)
    c = np.arange(n) if cols is None else np.asarray(cols)
    return (r[:, None] == c[None, :]).astype(np.float64)


def signal_matrix(X, psi, rows=None, cols=None):
    """K_f = sigma^2 exp(-1/2 sum_k D_k), the covariance without the noise term."""
    d = np.asarray(X).shape[1]
    sigma2, _, _ = unpack_psi(psi, d)
    D = _sq_diffs(X, psi, rows, cols)
    return sigma2 * np.exp(-0.5 * D.sum(axis=0))


def kernel_matrix(X, psi, rows=None, cols=None):
    """Dense K (or the block K[rows][:, cols]) including the noise on the diagonal."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    _, _, lam = unpack_psi(psi, d)
    return signal_matrix(X, psi, rows, cols) + lam * _diag_mask(n, rows, cols)


def kernel_derivatives(X, psi, rows=None, cols=None):
    """List of the P matrices dK/dpsi_j (j = 0..d+1), each of shape (rows, cols)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    sigma2, _, lam = unpack_psi(psi, d)
    D = _sq_diffs(X, psi, rows, cols)
    Kf = sigma2 * np.exp(-0.5 * D.sum(axis=0))
    out = [Kf]
    for k in range(d):
        out.append(Kf * D[k])
    out.append(lam * _diag_mask(n, rows, cols))
    return out


def kmv(X, psi, V, rows=None):
    """K V (or rows of it): the covariance matrix-vector product of Sec. 3, dense in FP64."""
    V = np.asarray(V, dtype=np.float64)
    return kernel_matrix(X, psi, rows=rows) @ V


def dkmv(X, psi, V, rows=None):
    """Stack of dK/dpsi_j V for j = 0..d+1, shape (P, rows, m)."""
    V = np.asarray(V, dtype=np.float64)
    return np.stack([Dj @ V for Dj in kernel_derivatives(X, psi, rows=rows)])


def log_marginal_likelihood(X, psi, y):
    """log p(y | psi, X) through the Cholesky factor K = L L^T (Sec. 2)."""
    y = np.asarray(y, dtype=np.float64)
    K = kernel_matrix(X, psi)
    L = np.linalg.cholesky(K)
    a = sla.cho_solve((L, True), y)
    n = y.shape[0]
    return -np.sum(np.log(np.diag(L))) - 0.5 * y @ a - 0.5 * n * np.log(2.0 * np.pi)


def exact_gradient(X, psi, y):
    """Exact gradient of log p(y | psi, X) with respect to psi (eq. gradient:exact)."""
    y = np.asarray(y, dtype=np.float64)
    K = kernel_matrix(X, psi)
    cf = sla.cho_factor(K, lower=True)
    a = sla.cho_solve(cf, y)
    Kinv = sla.cho_solve(cf, np.eye(K.shape[0]))
    g = []
    for Dj in kernel_derivatives(X, psi):
        g.append(-0.5 * np.sum(Kinv * Dj) + 0.5 * a @ Dj @ a)
    return np.array(g)


def solve(X, psi, B):
    """K^-1 B by Cholesky: the paper's ground truth for solver error (Sec. 3.2)."""
    K = kernel_matrix(X, psi)
    return sla.cho_solve(sla.cho_factor(K, lower=True), np.asarray(B, dtype=np.float64))


def condition_number(K):
    """kappa = lambda_max / lambda_min of a symmetric matrix (Sec. 3.1)."""
    ev = np.linalg.eigvalsh(K)
    return ev[-1] / ev[0]
