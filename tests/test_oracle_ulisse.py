"""Pins for oracle.ulisse: the randomly truncated CG series of Sec. 4.

Independent references: the closed-form tail probabilities P(J >= j) = 1 / W_j,
enumeration over every truncation point of a fixed CG path (exact mean and covariance),
Cholesky solutions, the paper's printed tail lengths, and chi-square / Monte Carlo checks
of the draws.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.stats as st

from oracle import cg, gp, rng, ulisse


def _system(n=40, lam=0.05, seed=0):
    r = np.random.default_rng(seed)
    X = r.uniform(size=(n, 2)).astype(np.float32)
    K = gp.kernel_matrix(X, np.log([1.0, 0.3, 0.3, lam]))
    return K, r.standard_normal(n)


def _forced(Jt):
    """u_j that keeps exactly the increments j = 0..Jt."""
    return lambda t, j: 0.0 if j <= Jt else 1.0 - 2.0 ** -53


def test_printed_tail_lengths(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "ulisse_tail_lengths.txt"))
            if l.strip() and not l.startswith("#")]
    for beta, printed in rows:
        beta, printed = float(beta), float(printed)
        # reading w_r = exp(r / beta): rate = 1 / beta
        assert abs(ulisse.expected_tail_terms(1.0 / beta) - printed) < 0.06
    # the literal exp(beta r) gives ~1.0 at beta = 100, which does not match the print
    assert abs(ulisse.expected_tail_terms(100.0) - 12.6) > 10
    np.testing.assert_allclose(ulisse.expected_tail_terms(1.0), 1.4201909683, rtol=1e-9)


def test_weight_product_definition():
    rate = 0.7
    for j in range(6):
        W = np.prod([np.exp(rate * r) for r in range(j + 1)])
        np.testing.assert_allclose(ulisse.weight_product(rate, j), W, rtol=1e-13)
        np.testing.assert_allclose(ulisse.survival(rate, j),
                                   np.prod([np.exp(-rate * r) for r in range(j + 1)]), rtol=1e-13)


def _path(K, b, alpha, eps):
    """Deterministic CG path: base s_{l-1}, tail increments delta_l..delta_T."""
    deltas, norms = [None], [None]
    s = np.zeros_like(b)
    for i, s, e, dl in cg.cg_iterates(lambda v: K @ v, b, np.zeros_like(b)):
        deltas.append(dl)
        norms.append(np.linalg.norm(e))
        if norms[-1] < eps:
            break
    T = len(deltas) - 1
    l = next(i for i in range(1, T + 1) if norms[i] < alpha)
    base = sum(deltas[1:l], np.zeros_like(b))
    return base, deltas[l:], l, T, s


@pytest.mark.parametrize("rate", [1.0, 0.3])
def test_exact_mean_and_covariance_by_enumeration(rate):
    K, b = _system()
    eps = 1e-9
    base, tail, l, T, sT = _path(K, b, alpha=0.5, eps=eps)
    assert len(tail) >= 3
    mv = lambda v: K @ v
    outs, probs = [], []
    for Jt in range(len(tail)):
        res = ulisse.solve(mv, b, np.zeros_like(b), 0.5, eps, 10000, rate, _forced(Jt))
        assert res["l"] == l and res["J"] == [Jt]
        p = ulisse.survival(rate, Jt) - (ulisse.survival(rate, Jt + 1) if Jt < len(tail) - 1 else 0.0)
        outs.append(res["s_tilde"][0])
        probs.append(p)
        # a prefix of the weighted series
        ref = base + sum(ulisse.weight_product(rate, j) * tail[j] for j in range(Jt + 1))
        np.testing.assert_allclose(res["s_tilde"][0], ref, rtol=1e-12, atol=1e-12)
    probs = np.array(probs)
    assert abs(probs.sum() - 1.0) < 1e-12
    mean = sum(p * o for p, o in zip(probs, outs))
    # unbiased for the converged CG solution, hence for K^-1 b up to the CG threshold
    np.testing.assert_allclose(mean, sT, rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(mean, ulisse.exact_mean(base, tail), rtol=1e-10, atol=1e-10)
    exact = sla.cho_solve(sla.cho_factor(K), b)
    assert np.linalg.norm(mean - exact) < 1e-6 * np.linalg.norm(exact)
    cov = sum(p * np.outer(o - mean, o - mean) for p, o in zip(probs, outs))
    ref_cov = ulisse.exact_cov(tail, rate)
    np.testing.assert_allclose(cov, ref_cov, rtol=1e-8, atol=1e-8 * np.abs(ref_cov).max())


def test_monte_carlo_mean_is_the_solution():
    # the mean of many ULISSE draws approaches K^-1 b within Monte Carlo error, in a
    # setting where the whole remaining tail is reached often enough to be sampled
    # (N P(J >= T - l) >= 50) and the CG floor is far below the Monte Carlo error
    K, b = _system(30, lam=0.1, seed=1)
    n = len(b)
    eps, rate, L = 1e-13, 0.02, 20
    norms = []
    for i, s, e, dl in cg.cg_iterates(lambda v: K @ v, b, np.zeros(n)):
        norms.append(np.linalg.norm(e))
        if norms[-1] < eps:
            break
    alpha = 0.5 * (norms[-L] + norms[-L - 1])  # L increments remain from l on
    base, tail, l, T, sT = _path(K, b, alpha, eps)
    assert len(tail) == L
    N = 4000
    assert N * ulisse.survival(rate, L - 1) > 50
    acc = np.zeros(n)
    for k in range(N):
        res = ulisse.solve_systems(lambda v: K @ v, b[:, None], None, alpha / np.sqrt(n), rate,
                                   eps, 1000, seed=5, stream=6, step=k)[0]
        acc += res[:, 0]
    mean = acc / N
    se = np.sqrt(np.diag(ulisse.exact_cov(tail, rate)) / N)
    exact = sla.cho_solve(sla.cho_factor(K), b)
    assert np.all(np.abs(sT - exact) < 0.1 * se)
    z = (mean - exact) / se
    assert np.all(np.abs(z) < 5.0), np.abs(z).max()


def test_tail_length_histogram_chi_square():
    K, b = _system(40, lam=1e-3, seed=2)
    rate = 1.0
    n = len(b)
    counts = np.zeros(4)
    N = 3000
    ext = 0.0
    for k in range(N):
        _, _, stats = ulisse.solve_systems(lambda v: K @ v, b[:, None], None, 10.0 / np.sqrt(n),
                                           rate, 1e-14, 1000, seed=1, stream=2, step=k)
        J = stats[0]["J"][0]
        counts[min(J, 3)] += 1
        ext += J + 1
    p = np.array([ulisse.survival(rate, j) - ulisse.survival(rate, j + 1) for j in range(3)])
    p = np.append(p, ulisse.survival(rate, 3))
    chi2 = np.sum((counts - N * p) ** 2 / (N * p))
    assert st.chi2.sf(chi2, df=3) > 1e-3
    # mean tail length: 1.42 at rate 1
    assert abs(ext / N - ulisse.expected_tail_terms(rate)) < 4 * 0.7 / np.sqrt(N)


def test_two_tracks_share_the_path_and_draw_independently():
    K, b = _system(40, lam=1e-3, seed=3)
    n = len(b)
    same = 0
    for k in range(200):
        St, Scg, stats = ulisse.solve_systems(lambda v: K @ v, b[:, None], None, 10 / np.sqrt(n),
                                              1.0, 1e-14, 1000, seed=3, stream=4, step=k,
                                              two_track_first=True)
        assert St.shape == (n, 2)
        s = stats[0]
        assert s["iters"] == s["l"] + max(s["J"])
        same += s["J"][0] == s["J"][1]
    # P(J_a = J_b) = sum_j P(J = j)^2 ~ 0.53 at rate 1: far from 0 and from 1
    assert 60 < same < 160


def test_warm_start_at_solution_still_takes_a_step():
    K, b = _system()
    s_exact = sla.cho_solve(sla.cho_factor(K), b)
    res = ulisse.solve(lambda v: K @ v, b, s_exact, 1.0, 1e-30, 5, 1.0, _forced(0))
    assert res["l"] == 1 and res["iters"] == 1
    np.testing.assert_allclose(res["s_tilde"][0], s_exact, rtol=1e-8, atol=1e-10)


def test_cap_sets_notconv():
    K, b = _system(40, lam=1e-4)
    res = ulisse.solve(lambda v: K @ v, b, np.zeros_like(b), 1e-12, 1e-14, 3, 1.0, _forced(0))
    assert res["flags"] & ulisse.NOTCONV and res["iters"] == 3


def test_s_cg_is_the_last_cg_iterate():
    K, b = _system(40, lam=1e-3, seed=4)
    res = ulisse.solve(lambda v: K @ v, b, np.zeros_like(b), 5.0, 1e-14, 100, 1.0, _forced(2))
    it = res["iters"]
    for i, s, e, dl in cg.cg_iterates(lambda v: K @ v, b, np.zeros_like(b)):
        if i == it:
            np.testing.assert_allclose(res["s_cg"], s, rtol=1e-13, atol=1e-13)
            break


@pytest.mark.parametrize("kind", ["lowrank", "shifted_inner"])
def test_exact_mean_over_preconditioned_cg_path(kind):
    # unbiasedness does not depend on the CG variant: enumerate J over a PCG path, with the
    # rank-k preconditioner or with J = K + delta I applied by 5 inner CG steps (Sec. 3.3)
    K, b = _system(40, lam=0.05, seed=6)
    if kind == "lowrank":
        w, Q = np.linalg.eigh(K)
        U, dk = Q[:, -6:], w[-6:]
        tau = np.mean(w[:-6])
        pinv = cg.lowrank_pinv(U, 1 / dk - 1 / tau, 1 / tau)
    else:
        pinv = cg.shifted_inner_pinv(lambda v: K @ v, 0.05, 0.0, 5)
    rate, eps = 0.5, 1e-11
    deltas, norms = [None], [None]
    for i, s, e, dl in cg.pcg_iterates(lambda v: K @ v, pinv, b, np.zeros(40)):
        deltas.append(dl)
        norms.append(np.linalg.norm(e))
        if norms[-1] < eps:
            break
    T = len(deltas) - 1
    alpha = 0.5 * (norms[T - 3] + norms[T - 4]) if norms[T - 3] < norms[T - 4] else norms[T - 3] * 1.0001
    mean = np.zeros(40)
    total = 0.0
    for Jt in range(8):
        res = ulisse.solve(lambda v: K @ v, b, np.zeros(40), alpha, eps, 1000, rate, _forced(Jt),
                           apply_pinv=pinv)
        l = res["l"]
        tail = T - l
        if Jt > tail:
            break
        p = ulisse.survival(rate, Jt) - (ulisse.survival(rate, Jt + 1) if Jt < tail else 0.0)
        mean += p * res["s_tilde"][0]
        total += p
    np.testing.assert_allclose(total, 1.0, rtol=1e-12)
    np.testing.assert_allclose(mean, sla.cho_solve(sla.cho_factor(K), b), rtol=1e-7, atol=1e-8)


def test_exact_mean_from_a_warm_start_is_the_solution():
    # a warm start s0 (as the learned part supplies, s0 = U c) changes the CG path but not the
    # expectation: enumerating every truncation point gives the solution again, with or
    # without a preconditioner
    K, b = _system(40, lam=0.05, seed=9)
    sol = sla.cho_solve(sla.cho_factor(K), b)
    s0 = sol + 0.3 * np.random.default_rng(1).standard_normal(40)
    w, Q = np.linalg.eigh(K)
    pinv = cg.lowrank_pinv(Q[:, -6:], 1 / w[-6:] - 1 / np.mean(w[:-6]), 1 / np.mean(w[:-6]))
    rate, eps = 0.5, 1e-11
    for ap in (None, pinv):
        it = cg.cg_iterates(lambda v: K @ v, b, s0) if ap is None else cg.pcg_iterates(lambda v: K @ v, ap, b, s0)
        norms = [np.linalg.norm(b - K @ s0)]
        for i, s_, e, dl in it:
            norms.append(np.linalg.norm(e))
            if norms[-1] < eps:
                break
        T = len(norms) - 1
        alpha = 0.5 * (norms[T - 2] + norms[T - 3]) if norms[T - 2] < norms[T - 3] else norms[T - 2] * 1.0001
        mean, total = np.zeros(40), 0.0
        for Jt in range(8):
            res = ulisse.solve(lambda v: K @ v, b, s0, alpha, eps, 1000, rate, _forced(Jt), apply_pinv=ap)
            tail = T - res["l"]
            if Jt > tail:
                break
            p = ulisse.survival(rate, Jt) - (ulisse.survival(rate, Jt + 1) if Jt < tail else 0.0)
            mean += p * res["s_tilde"][0]
            total += p
        np.testing.assert_allclose(total, 1.0, rtol=1e-12)
        np.testing.assert_allclose(mean, sol, rtol=1e-7, atol=1e-8)


def test_converged_series_with_residual_replacement_is_the_solution():
    # with replacements (and the restarts they bring) the CG iterates still converge to
    # K^-1 b, so a series run to convergence returns the Cholesky solution
    r = np.random.default_rng(11)
    X = r.uniform(size=(120, 2)).astype(np.float32)
    psi = np.log([1.0, 0.25, 0.4, 0.05])
    K = gp.kernel_matrix(X, psi)
    B = r.standard_normal((120, 3))
    St, _, stats = ulisse.solve_systems(lambda v: K @ v, B, None, 1e-12, 1e-9, 1e-10, 2000, 5, 1, 0,
                                        eps_relative=True, refresh=3)
    np.testing.assert_allclose(St, np.linalg.solve(K, B), rtol=1e-6, atol=1e-8)
    assert all(s["flags"] == 0 for s in stats)


def test_residual_replacement_keeps_the_exact_mean_of_the_series():
    # the exact mean over the truncation points of one path (the enumeration pin of the
    # plain series) holds over a path with replacements too: E[s~] = s_T
    r = np.random.default_rng(12)
    X = r.uniform(size=(40, 2)).astype(np.float32)
    psi = np.log([1.0, 0.3, 0.3, 0.2])
    K = gp.kernel_matrix(X, psi)
    b = r.standard_normal(40)
    its = list(zip(range(12), cg.cg_iterates(lambda v: K @ v, b, np.zeros(40), refresh=1)))
    deltas = [dl for _, (i, s, e, dl) in its]
    s_T = its[-1][1][1]
    l = 3
    base = sum(deltas[:l - 1])
    tail = [deltas[l - 1 + j] for j in range(len(deltas) - l + 1)]
    np.testing.assert_allclose(ulisse.exact_mean(base, tail), s_T, rtol=1e-12, atol=1e-12)
