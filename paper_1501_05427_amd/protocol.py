"""Host-side pieces of the paper's SGLD protocol (Sec. 5) on top of the library.

* exact_gradient: the gradient of log p(y | psi) on a (small) data set from converged
  solves, with the probes r_c = sqrt(n) e_c running over every coordinate, so that the
  probe term of the estimator is exactly 1/2 tr(K^-1 dK/dpsi_j); the solves run through
  gp_stoch_grad in batches of at most 62 probes.
* subset_map / neg_hessian / sgld_preconditioner: the MAP on a random subset of the inputs
  (500 points for Concrete, 1000 for Census in the paper), the negative Hessian of the log
  posterior there (central differences of exact gradients), and M = (-H)^-1 with its
  Cholesky factor, the SGLD preconditioner of Sec. 5.
* init_chains: starting points drawn from N(psi_MAP, M), as for the paper's parallel chains.
* psrf / ess: the potential scale reduction factor (Gelman & Rubin, 1992) and the effective
  sample size (Geyer's initial positive sequence) of the resulting chains.

Every covariance product runs in the library's kernels; the host only does P x P algebra
and the statistics of short traces.
"""
import numpy as np

from . import binding as pb

MAX_PROBES = 62


def _prior_grad(psi, prior):
    kind = prior.get("kind", 0) if prior else 0
    if kind == 0:
        return np.zeros_like(psi)
    a, b = np.asarray(prior["a"], np.float64), np.asarray(prior["b"], np.float64)
    if kind == 1:
        return -(psi - a) / (b * b)
    if kind == 2:
        return a - b * np.exp(psi)
    raise ValueError("prior kind must be 0, 1 or 2")


def exact_gradient(h, X, y, psi, eps=1e-6, max_iter=20000):
    """d/dpsi log p(y | psi, X) (device X (n, d) FP32, y (n,) FP32, psi numpy P) -> numpy P.

    Batch k with b_k unit probes gives g_k = q - (1 / 2 b_k) sum_batch r^T dK s; with the
    same quadratic term q in every batch, sum_k (b_k / n) g_k is the exact gradient.
    """
    import torch
    n = X.shape[0]
    params = pb.make_params(q=0.0, rate=1.0, eps=eps, eps_relative=1, max_iter=max_iter)
    psid = torch.as_tensor(np.asarray(psi, np.float64)).cuda()
    total = np.zeros(len(psi))
    root_n = float(np.sqrt(n))
    for c0 in range(0, n, MAX_PROBES):
        b = min(MAX_PROBES, n - c0)
        R = pb.colmajor(n, b)
        R.zero_()
        idx = torch.arange(b, device=R.device)
        R[c0 + idx, idx] = root_n
        g, stats = pb.gp_stoch_grad(h, X, psid, y, params, R=R)
        flags = [s["flags"] for s in pb.decode_stats(stats)]
        if any(flags):
            raise RuntimeError(f"a subset solve did not converge (flags {flags}); raise max_iter")
        total += (b / n) * g.cpu().numpy()
    return total


def probe_mean_gradient(h, X, y, psi, batches, probes=31, probe_stream=21, eps=1e-6,
                        max_iter=5000, progress=None, prec=None, refresh=0):
    """Reference gradient for large n: the plain estimator with converged solves (q = 0, so
    the series never truncates) averaged over `batches` draws of `probes` Gaussian probes.

    Each batch is an unbiased estimate of d/dpsi log p(y | psi) whose only error is the
    Hutchinson noise of its probes (and the CG tolerance); returns (mean, standard error of
    the mean) as numpy arrays.  Probes come from Philox stream `probe_stream`, one counter
    per batch.  prec / refresh: the products' arithmetic mode (FP32 by default) and the
    residual replacement of the solves (0 = off), to measure what a mode does to the mean.
    """
    import torch
    n = X.shape[0]
    psid = psi if torch.is_tensor(psi) else torch.as_tensor(np.asarray(psi, np.float64)).cuda()
    P = psid.shape[0]
    ref = pb.make_params(q=0.0, rate=1.0, eps=eps, eps_relative=1, max_iter=max_iter, rng_stream=3,
                         refresh=refresh, prec=pb.GP_FP32 if prec is None else prec)
    R = pb.colmajor(n, probes)
    S_warm = torch.zeros((1 + probes, n), dtype=torch.float64, device="cuda").t()
    g = torch.zeros(P, dtype=torch.float64, device="cuda")
    stats = pb.stats_tensor(1 + probes)
    gs = []
    for b in range(batches):
        pb.gp_draw_probes(h, n, probes, pb.PROBE_GAUSSIAN, probe_stream, b, R=R)
        S_warm[:, 1:].zero_()   # the y column keeps its warm start: q = 0 converges anyway
        ref.rng_counter = b
        pb.gp_stoch_grad(h, X, psid, y, ref, R=R, S_warm=S_warm, g=g, stats=stats)
        gs.append(g.cpu().numpy().copy())
        flags = [s["flags"] for s in pb.decode_stats(stats)]
        if any(flags):
            raise RuntimeError(f"a reference solve did not converge (flags {flags}); raise max_iter")
        if progress is not None:
            progress(b + 1, batches)
    gs = np.array(gs)
    se = gs.std(0, ddof=1) / np.sqrt(len(gs)) if len(gs) > 1 else np.full(P, np.inf)
    return gs.mean(0), se


def log_post_grad(h, X, y, psi, prior=None):
    psi = np.asarray(psi, np.float64)
    return exact_gradient(h, X, y, psi) + _prior_grad(psi, prior)


def neg_hessian(h, X, y, psi, prior=None, step=1e-3):
    psi = np.asarray(psi, np.float64)
    P = len(psi)
    H = np.empty((P, P))
    for k in range(P):
        e = np.zeros(P)
        e[k] = step
        H[:, k] = (log_post_grad(h, X, y, psi + e, prior) - log_post_grad(h, X, y, psi - e, prior)) / (2 * step)
    return -0.5 * (H + H.T)


def subset_map(h, X, y, psi0, prior=None, iters=30, tol=1e-5):
    """Damped Newton iterations on the log posterior of (X, y): psi <- psi + t (-H)^-1 g,
    halving t while ||g|| does not drop.  Returns (psi_MAP, -H at psi_MAP)."""
    psi = np.asarray(psi0, np.float64).copy()
    g = log_post_grad(h, X, y, psi, prior)
    n = X.shape[0]
    for _ in range(iters):
        A = neg_hessian(h, X, y, psi, prior)
        direction = np.linalg.solve(A, g)
        t = 1.0
        while True:
            cand = psi + t * direction
            gc = log_post_grad(h, X, y, cand, prior)
            if np.linalg.norm(gc) < np.linalg.norm(g) or t < 1e-6:
                break
            t *= 0.5
        psi, g = cand, gc
        if np.linalg.norm(g) < tol * n:
            break
    return psi, neg_hessian(h, X, y, psi, prior)


def sgld_preconditioner(h, X_host, y_host, psi0, prior=None, n_sub=500, seed=0):
    """MAP and M = (-H)^-1 on a random subset of n_sub points; returns (psi_MAP, M, L) with
    M = L L^T (L lower triangular), ready for sgld_step / sgld_run."""
    import torch
    r = np.random.default_rng(seed)
    n = X_host.shape[0]
    idx = np.sort(r.choice(n, size=min(n_sub, n), replace=False))
    Xs = torch.as_tensor(np.ascontiguousarray(X_host[idx], dtype=np.float32)).cuda()
    ys = torch.as_tensor(np.ascontiguousarray(y_host[idx], dtype=np.float32)).cuda()
    psi_map, A = subset_map(h, Xs, ys, psi0, prior)
    M = np.linalg.inv(A)
    M = 0.5 * (M + M.T)
    return psi_map, M, np.linalg.cholesky(M)


def init_chains(psi_map, M, n_chains, seed=0):
    """n_chains starting points from N(psi_MAP, M) (rows)."""
    L = np.linalg.cholesky(np.asarray(M, np.float64))
    z = np.random.default_rng(seed).standard_normal((n_chains, len(psi_map)))
    return np.asarray(psi_map, np.float64)[None, :] + z @ L.T


def psrf(chains):
    """chains (m, T) or (m, T, P) -> potential scale reduction factor per parameter:
    sqrt(V / W), V = (T - 1) / T W + (1 + 1 / m) B / T."""
    x = np.asarray(chains, np.float64)
    if x.ndim == 2:
        x = x[:, :, None]
    m, T, _ = x.shape
    W = np.mean(np.var(x, axis=1, ddof=1), axis=0)
    B_T = np.var(np.mean(x, axis=1), axis=0, ddof=1)
    return np.sqrt(((T - 1) / T * W + (1 + 1 / m) * B_T) / W)


def ess(x):
    """x (T,) or (T, P) -> effective sample size T / tau per parameter, tau from the
    autocorrelations summed in positive pairs (Geyer's initial positive sequence); the
    autocorrelations come from one FFT per parameter."""
    x = np.asarray(x, np.float64)
    if x.ndim == 1:
        x = x[:, None]
    T, P = x.shape
    c = x - x.mean(axis=0)
    f = np.fft.rfft(c, n=2 * T, axis=0)
    acov = np.fft.irfft(f * np.conj(f), axis=0)[:T]
    rho = acov / acov[0]
    out = np.empty(P)
    for j in range(P):
        npairs = T // 2
        pairs = rho[0:2 * npairs:2, j] + rho[1:2 * npairs:2, j]
        neg = np.nonzero(pairs <= 0.0)[0]
        K = neg[0] if len(neg) else npairs
        tau = -1.0 + 2.0 * np.sum(pairs[:K])
        out[j] = T / max(tau, 1e-300)
    return out


def plain_chain_states(h, X, y, starts, steps, M_chol, eps, probes=4, probe_period=20, q=1.0,
                       prior=None, rng_stream=41, seed=900, progress=None):
    """The log-parameters visited by plain-solver SGLD chains: the (theta, solve) pairs the
    method itself generates, from which the learned preconditioner takes its training
    inputs.  One chain per row of `starts`, all over the same GP (device X, y), stepped
    together through gp_batch_* (gp_stoch_grad + sgld_step per chain, FP32 products, no
    preconditioner): `probes` Gaussian probes redrawn every `probe_period` steps with warm
    starts, threshold q sqrt(n), step size eps, SGLD preconditioner M = L L^T (M_chol: P x P
    numpy lower factor), prior as for sgld_step (dict kind, a, b).  Returns
    (len(starts) * steps, P) numpy, the state after every step of every chain.  progress:
    optional callable(steps done, steps), called every 10 steps."""
    import torch
    starts = np.asarray(starts, np.float64)
    C, P = starts.shape
    Ld = torch.as_tensor(np.ascontiguousarray(np.asarray(M_chol, np.float64).T)).cuda()
    kind = prior.get("kind", 0) if prior else 0
    pa = torch.as_tensor(np.asarray(prior["a"], np.float64)).cuda() if kind else None
    pbb = torch.as_tensor(np.asarray(prior["b"], np.float64)).cuda() if kind else None
    probs = [{"X": X, "y": y, "psi": torch.as_tensor(starts[c].copy()).cuda(), "M_chol": Ld,
              "prior": (kind, pa, pbb)} for c in range(C)]
    params = pb.make_params(q=q, rate=1.0, eps=1e-6, eps_relative=1, max_iter=2000, rng_stream=rng_stream)
    batch = pb.Batch(probs, probes, params, seed=seed, probe_kind=pb.PROBE_GAUSSIAN,
                     probe_period=probe_period, iters_per_graph=8, autotune=False, streams=min(C, 8))
    out = np.empty((steps, C, P))
    for t in range(steps):
        batch.step(t, eps)
        out[t] = torch.stack([p["psi"] for p in probs]).cpu().numpy()
        if progress is not None and (t + 1) % 10 == 0:
            progress(t + 1, steps)
    batch.close()
    if not np.all(np.isfinite(out)):
        raise RuntimeError("a plain-solver chain left the finite range")
    return out.transpose(1, 0, 2).reshape(C * steps, P)
