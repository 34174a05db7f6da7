"""ULISSE: the unbiased, randomly truncated CG series of Sec. 4, in FP64 (oracle).

The CG solution is the telescoping sum s = s_0 + delta_1 + ... + delta_T.  With the
early-stop threshold alpha = q sqrt(n), l is the first iteration whose residual norm is
below alpha.  The estimate keeps s_0 + delta_1 + ... + delta_{l-1} and then, for
j = 0, 1, ..., draws u_j ~ U[0, 1) and, while u_j < 1/w_j, adds (w_0 ... w_j) delta_{l+j};
the first rejection stops both the series and the CG run.  Weights w_r = exp(rate r)
(the paper writes exp(beta r); its experiments use beta = 1, i.e. rate = 1).

Readings where the paper is silent:
  * l >= 1 always (a warm start already below alpha still takes one CG step);
  * residual norms are those of Alg. 1's recursive residual;
  * CG convergence (||e|| < eps) ends the series: every later increment is zero;
  * the iteration cap ends it too and sets NOTCONV (the estimate is then biased);
  * u_j < 1/w_j is a strict comparison in FP64 with 1/w_j = exp(-rate j);
  * several tracks share one CG path and draw their u_j independently (Sec. 4.1);
  * with residual replacement (refresh = k) a residual that has fallen by 2^k since the
    last replacement, and is above 2^k eps, is replaced by b - K s_i (see oracle.cg).
"""
import numpy as np

from . import cg as _cg
from . import rng as _rng

NOTCONV = 1


def weight_product(rate, j):
    """W_j = w_0 w_1 ... w_j = exp(rate j (j + 1) / 2)."""
    return np.exp(rate * j * (j + 1) / 2.0)


def survival(rate, j):
    """P(J >= j) = 1 / W_j: the probability that increment delta_{l+j} is kept."""
    return np.exp(-rate * j * (j + 1) / 2.0)


def expected_tail_terms(rate, jmax=100000):
    """E[J + 1] = sum_j P(J >= j): the mean number of increments kept from l on."""
    j = np.arange(jmax, dtype=np.float64)
    return float(np.sum(survival(rate, j)))


class _LazyCG:
    """One CG run whose increments are produced on demand and shared by all tracks."""

    def __init__(self, matvec, b, s0, apply_pinv=None, refresh=0, floor=0.0, refresh_matvec=None):
        if apply_pinv is None:
            self.it = _cg.cg_iterates(matvec, b, s0, refresh, refresh_matvec, floor)
        else:
            self.it = _cg.pcg_iterates(matvec, apply_pinv, b, s0, refresh, refresh_matvec, floor)
        self.deltas = [None]     # 1-based: deltas[i] = delta_i
        self.norms = [None]
        self.last_s = np.array(s0, dtype=np.float64, copy=True)

    def get(self, i):
        while len(self.deltas) <= i:
            _, s, e, delta = next(self.it)
            self.deltas.append(delta)
            self.norms.append(float(np.linalg.norm(e)))
            self.last_s = s
        return self.deltas[i], self.norms[i]


def solve(matvec, b, s0, alpha, eps, max_iter, rate, uniform, ntracks=1, apply_pinv=None,
          refresh=0, refresh_matvec=None):
    """One ULISSE solve of K s = b (over preconditioned CG when apply_pinv is given: the
    series argument of Sec. 4 holds for any CG variant, as the paper notes).

    uniform(track, j) returns u_j for that track.  Returns a dict with
      s_tilde  list of ntracks FP64 vectors (the unbiased estimates)
      s_cg     the last CG iterate computed (used to warm-start the next solve)
      l, J     threshold iteration and, per track, the last kept tail index
      iters    number of CG iterations run (= number of products K d)
      flags    NOTCONV if the cap was hit before the series ended
    """
    b = np.asarray(b, dtype=np.float64)
    cgrun = _LazyCG(matvec, b, s0, apply_pinv, refresh, eps, refresh_matvec)
    base = np.array(s0, dtype=np.float64, copy=True)
    flags = 0
    i = 0
    l = 0
    # s~ = s_0 + delta_1 + ... + delta_{l-1}
    while True:
        i += 1
        delta, r = cgrun.get(i)
        if r < alpha or r < eps:
            l = i
            break
        base = base + delta
        if i >= max_iter:
            flags |= NOTCONV
            return dict(s_tilde=[base.copy() for _ in range(ntracks)], s_cg=cgrun.last_s,
                        l=0, J=[0] * ntracks, iters=i, flags=flags)
    s_tilde, Js = [], []
    for t in range(ntracks):
        st = base.copy()
        j = 0
        W = 1.0
        while True:
            u = uniform(t, j)
            if not (u < np.exp(-rate * j)):
                j -= 1
                break
            W = W * np.exp(rate * j)
            delta, r = cgrun.get(l + j)
            st = st + W * delta
            if r < eps:
                break
            if l + j >= max_iter:
                flags |= NOTCONV
                break
            j += 1
        s_tilde.append(st)
        Js.append(j)
    iters = l + max(Js)
    s_cg = np.array(s0, dtype=np.float64, copy=True)
    for k in range(1, iters + 1):
        s_cg = s_cg + cgrun.deltas[k]
    return dict(s_tilde=s_tilde, s_cg=s_cg, l=l, J=Js, iters=iters, flags=flags)


def solve_systems(matvec, B, S0, q, rate, eps, max_iter, seed, stream, step,
                  two_track_first=False, eps_relative=False, apply_pinv=None, refresh=0,
                  refresh_matvec=None):
    """ULISSE on every column of B with the library's counter layout for the u_j.

    Column c is system c; with two_track_first, column 0 carries tracks 0 and 1.
    Returns (S_tilde list in the library's column order, S_cg, per-system stats).
    """
    B = np.asarray(B, dtype=np.float64)
    n, m = B.shape
    alpha = q * np.sqrt(n)
    out_cols, scg, stats = [], np.zeros((n, m)), []
    for c in range(m):
        b = B[:, c]
        s0 = np.zeros(n) if S0 is None else np.asarray(S0, dtype=np.float64)[:, c]
        thr = eps * np.linalg.norm(b) if eps_relative else eps
        nt = 2 if (two_track_first and c == 0) else 1

        def uniform(t, j, c=c):
            return _rng.ulisse_uniform(seed, stream, step, c, t, j)

        res = solve(matvec, b, s0, alpha, thr, max_iter, rate, uniform, nt, apply_pinv, refresh,
                    refresh_matvec)
        out_cols.extend(res["s_tilde"])
        scg[:, c] = res["s_cg"]
        stats.append(dict(l=res["l"], J=res["J"], iters=res["iters"], flags=res["flags"]))
    return np.stack(out_cols, axis=1), scg, stats


def exact_mean(base, tail):
    """E[s~] over the draws for a fixed CG path: base + sum_j P(J>=j) W_j delta_{l+j}."""
    m = np.array(base, dtype=np.float64, copy=True)
    for dlt in tail:
        m = m + dlt
    return m


def exact_cov(tail, rate):
    """Cov[s~] = sum_{i,j} (W_min(i,j) - 1) delta_{l+i} delta_{l+j}^T for a fixed path."""
    tail = [np.asarray(t, dtype=np.float64) for t in tail]
    n = tail[0].shape[0]
    C = np.zeros((n, n))
    for a, da in enumerate(tail):
        for b_, db in enumerate(tail):
            C += (weight_product(rate, min(a, b_)) - 1.0) * np.outer(da, db)
    return C
