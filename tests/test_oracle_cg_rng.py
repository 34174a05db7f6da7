"""Pins for oracle.cg (Alg. 1) and oracle.rng (Philox4x64-10 and the draw mappings)."""
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as ssl
import scipy.stats as st

from oracle import cg, gp, rng


def _spd(n=30, lam=0.1, seed=0):
    r = np.random.default_rng(seed)
    X = r.uniform(size=(n, 2)).astype(np.float32)
    psi = np.log([1.0, 0.3, 0.3, lam])
    return gp.kernel_matrix(X, psi), r.standard_normal(n)


def test_cg_matches_cholesky_solution():
    # the paper's solver error: ||s_CG - s_Cholesky|| (Sec. 3.2)
    K, b = _spd()
    s, it, ok, res = cg.cg(lambda v: K @ v, b, np.zeros_like(b), 1e-10, 10 * len(b))
    ref = sla.cho_solve(sla.cho_factor(K), b)
    assert ok
    assert np.linalg.norm(s - ref) <= 1e-8 * np.linalg.norm(ref)


def test_cg_exact_in_at_most_n_steps_well_conditioned():
    r = np.random.default_rng(2)
    A = r.standard_normal((8, 8))
    K = A @ A.T + 8 * np.eye(8)
    b = r.standard_normal(8)
    s, it, ok, _ = cg.cg(lambda v: K @ v, b, np.zeros(8), 1e-10, 100)
    assert ok and it <= 8
    np.testing.assert_allclose(K @ s, b, atol=1e-9)


def test_cg_matches_scipy_and_recursive_residual():
    K, b = _spd(40, seed=3)
    s0 = np.random.default_rng(4).standard_normal(40)
    for i, s, e, delta in cg.cg_iterates(lambda v: K @ v, b, s0):
        np.testing.assert_allclose(e, b - K @ s, atol=1e-9)
        if i == 10:
            break
    s, _, ok, _ = cg.cg(lambda v: K @ v, b, s0, 1e-11, 1000)
    ref, info = ssl.cg(K, b, x0=s0, rtol=1e-13, atol=0, maxiter=1000)
    assert ok and info == 0
    np.testing.assert_allclose(s, ref, rtol=1e-8, atol=1e-9)


def test_cg_iterations_grow_with_condition_number():
    # Sec. 3: iterations grow with kappa; here kappa is raised by shrinking the noise
    its = []
    for lam in [1.0, 1e-1, 1e-2, 1e-3]:
        K, b = _spd(60, lam=lam, seed=5)
        _, it, ok, _ = cg.cg(lambda v: K @ v, b, np.zeros(60), 1e-8, 100000)
        assert ok
        its.append(it)
    assert its == sorted(its) and its[-1] > its[0]


def _philox_reference(ctr, key):
    """Philox4x64-10 round function written from its published definition."""
    M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
    W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B
    mask = (1 << 64) - 1
    c, k = list(ctr), list(key)
    for _ in range(10):
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & mask, (p0 >> 64) ^ c[3] ^ k[1], p0 & mask]
        k = [(k[0] + W0) & mask, (k[1] + W1) & mask]
    return c


def test_philox_known_answers(golden_dir):
    rows = [l.split() for l in open(os.path.join(golden_dir, "philox4x64_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 2
    for r in rows:
        v = [int(x, 16) for x in r]
        ctr, key, out = v[0:4], v[4:6], v[6:10]
        got = rng.blocks(key[0], key[1], ctr[1], ctr[2], ctr[3], 1, first_block=ctr[0])
        assert [int(x) for x in got[0]] == out
        assert _philox_reference(ctr, key) == out


@pytest.mark.parametrize("w1,purpose,step,first", [(0, 1, 0, 0), (5, 2, 9, 3), (17, 3, 2**40, 0)])
def test_counter_layout_block_by_block(w1, purpose, step, first):
    got = rng.blocks(123, 456, w1, purpose, step, 5, first_block=first)
    for b in range(5):
        ref = _philox_reference([first + b, w1, purpose, step], [123, 456])
        assert [int(x) for x in got[b]] == ref


def test_mappings_distributions():
    x = rng.words(7, 8, 0, rng.PROBE, 0, 200000)
    u = rng.uniform_co(x)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert st.kstest(u, "uniform").pvalue > 1e-3
    assert rng.uniform_oc(np.array([0], dtype=np.uint64))[0] == 2.0 ** -53
    assert rng.uniform_co(np.array([2**64 - 1], dtype=np.uint64))[0] == 1.0 - 2.0 ** -53
    z = rng.gaussians(7, 8, 1, rng.PROBE, 0, 200000)
    assert st.kstest(z, "norm").pvalue > 1e-3
    s = rng.rademacher(x)
    assert set(np.unique(s)) == {-1.0, 1.0}
    assert abs(s.mean()) < 5 / np.sqrt(len(s))
    # Rademacher = top bit; Box-Muller pairs words (0,1) and (2,3)
    blk = rng.blocks(7, 8, 1, rng.PROBE, 0, 1)[0]
    za, zb = rng.box_muller(blk[0:1], blk[1:2])
    np.testing.assert_array_equal(z[:2], [za[0], zb[0]])


def test_probe_matrix_columns_are_independent_streams():
    R = rng.probes(1, 2, 3, 100, 3, kind=0)
    assert R.shape == (100, 3)
    np.testing.assert_array_equal(R[:, 1], rng.gaussians(1, 2, 1, rng.PROBE, 3, 100))
    Rr = rng.probes(1, 2, 3, 100, 2, kind=1)
    assert set(np.unique(Rr)) == {-1.0, 1.0}


def test_pcg_with_exact_preconditioner_converges_in_one_step():
    K, b = _spd(30, seed=7)
    Kinv = np.linalg.inv(K)
    it = cg.pcg_iterates(lambda v: K @ v, lambda v: Kinv @ v, b, np.zeros(30))
    i, s, e, _ = next(it)
    np.testing.assert_allclose(s, sla.cho_solve(sla.cho_factor(K), b), rtol=1e-9, atol=1e-10)
    assert np.linalg.norm(e) < 1e-9 * np.linalg.norm(b)


def test_pcg_identity_is_cg_and_lowrank_preconditioner_helps():
    K, b = _spd(60, lam=1e-2, seed=8)
    for (i1, s1, e1, _), (i2, s2, e2, _) in zip(cg.cg_iterates(lambda v: K @ v, b, np.zeros(60)),
                                              cg.pcg_iterates(lambda v: K @ v, lambda v: v, b, np.zeros(60))):
        np.testing.assert_allclose(s1, s2, rtol=1e-12, atol=1e-12)
        if i1 == 8:
            break
    # deflating the top 10 eigenvectors: P^-1 = (1/tau) I + U (1/d - 1/tau) U^T
    w, Q = np.linalg.eigh(K)
    U, dk = Q[:, -10:], w[-10:]
    tau = np.mean(w[:-10])
    pinv = cg.lowrank_pinv(U, 1 / dk - 1 / tau, 1 / tau)
    P = U @ np.diag(dk) @ U.T + tau * (np.eye(60) - U @ U.T)
    np.testing.assert_allclose(pinv(b), np.linalg.solve(P, b), rtol=1e-9, atol=1e-12)

    def run(gen, tol):
        for i, s, e, _ in gen:
            if np.linalg.norm(e) < tol * np.linalg.norm(b) or i >= 500:
                return i, s
    n_cg, _ = run(cg.cg_iterates(lambda v: K @ v, b, np.zeros(60)), 1e-8)
    n_pcg, _ = run(cg.pcg_iterates(lambda v: K @ v, pinv, b, np.zeros(60)), 1e-8)
    assert n_pcg < n_cg < 500
    _, s = run(cg.pcg_iterates(lambda v: K @ v, pinv, b, np.zeros(60)), 1e-10)
    np.testing.assert_allclose(s, sla.cho_solve(sla.cho_factor(K), b), rtol=1e-8, atol=1e-9)


# ---- PCG with J = K + delta I applied by an inner CG (Sec. 3.3) ----------------------------

def test_shifted_inner_solve_is_the_shifted_system_solution():
    K, b = _spd(40, seed=11)
    for delta in (1e-3, 0.1, 2.0):
        z = cg.shifted_inner_pinv(lambda v: K @ v, delta, 1e-13, 400)(b)
        ref = sla.cho_solve(sla.cho_factor(K + delta * np.eye(40)), b)
        np.testing.assert_allclose(z, ref, rtol=1e-9, atol=1e-11)
    assert not np.any(cg.shifted_inner_pinv(lambda v: K @ v, 0.1, 0.0, 5)(np.zeros(40)))


def test_shifted_inner_solve_fixed_count_is_that_many_cg_steps():
    # eps_inner = 0: exactly max_inner products; the result is the max_inner-th Krylov iterate
    # of (K + delta I), which minimises the energy error over that Krylov space
    K, b = _spd(40, seed=12)
    delta, k = 0.05, 4
    A = K + delta * np.eye(40)
    calls = []
    z = cg.shifted_inner_pinv(lambda v: (calls.append(1), K @ v)[1], delta, 0.0, k)(b)
    assert len(calls) == k + 1  # k steps plus the initial residual b - K 0
    Kr = np.column_stack([np.linalg.matrix_power(A, j) @ b for j in range(k)])
    Q, _ = np.linalg.qr(Kr)
    c = np.linalg.solve(Q.T @ A @ Q, Q.T @ b)
    np.testing.assert_allclose(z, Q @ c, rtol=1e-8, atol=1e-10)


def test_pcg_shifted_large_delta_is_cg_and_zero_delta_one_step():
    K, b = _spd(50, lam=1e-2, seed=13)
    mv = lambda v: K @ v
    # delta >> ||K||: J^-1 ~ I / delta, a scalar preconditioner, which leaves CG's iterates
    # unchanged (up to O(||K|| / delta))
    pinv = cg.shifted_inner_pinv(mv, 1e9, 1e-14, 200)
    for (i1, s1, _, _), (i2, s2, _, _) in zip(cg.cg_iterates(mv, b, np.zeros(50)),
                                              cg.pcg_iterates(mv, pinv, b, np.zeros(50))):
        np.testing.assert_allclose(s2, s1, rtol=1e-6, atol=1e-8)
        if i1 == 6:
            break
    # delta -> 0 with converged inner solves: J = K, one outer step reaches K^-1 b
    pinv0 = cg.shifted_inner_pinv(mv, 1e-12, 1e-14, 2000)
    _, s, e, _ = next(cg.pcg_iterates(mv, pinv0, b, np.zeros(50)))
    np.testing.assert_allclose(s, sla.cho_solve(sla.cho_factor(K), b), rtol=1e-6, atol=1e-8)


def test_pcg_shifted_converges_to_the_solution_with_inexact_inner_solves():
    K, b = _spd(60, lam=1e-2, seed=14)
    mv = lambda v: K @ v
    pinv = cg.shifted_inner_pinv(mv, 0.1, 0.0, 6)
    for i, s, e, _ in cg.pcg_iterates(mv, pinv, b, np.zeros(60)):
        if np.linalg.norm(e) < 1e-10 * np.linalg.norm(b) or i >= 300:
            break
    assert i < 300
    np.testing.assert_allclose(s, sla.cho_solve(sla.cho_factor(K), b), rtol=1e-7, atol=1e-8)


def _spd_kappa(n, seed, kappa):
    r = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(r.standard_normal((n, n)))
    return (Q * np.geomspace(1.0, kappa, n)) @ Q.T


def _restart_check(make_run, iterates_fresh, K, b, n_first):
    """Up to the first replacement the run is plain (P)CG; after a replacement at
    iteration i the run continues exactly as a fresh run started from s_i."""
    calls = []

    def counted(v):
        calls.append(1)
        return K @ v

    run, at = [], []
    for i, s, e, d in make_run(counted):
        run.append((i, s.copy(), e.copy()))
        if calls and not at:
            at.append(i)
        if len(run) == n_first:
            break
    assert at, "no replacement happened"
    i_rep = at[0]
    ref = list(zip(range(i_rep), iterates_fresh(np.zeros(len(b)))))
    for (_, (i2, s2, e2, _d2)), (i, s, e) in zip(ref, run):
        np.testing.assert_allclose(s, s2, rtol=1e-9, atol=1e-12 * np.abs(s2).max())
    s_i = run[i_rep - 1][1]
    # the replaced residual is the true one ...
    np.testing.assert_allclose(run[i_rep - 1][2], b - K @ s_i, rtol=0, atol=1e-12 * np.linalg.norm(b))
    # ... and the following iterates are those of a fresh run from s_i
    fresh = list(zip(range(3), iterates_fresh(s_i)))
    for j in range(3):
        s_run = run[i_rep + j][1]
        np.testing.assert_allclose(s_run, fresh[j][1][1], rtol=1e-8, atol=1e-10 * np.abs(s_run).max())


def test_residual_replacement_restarts_cg_from_the_current_iterate():
    K = _spd_kappa(60, 0, 1e3)
    b = np.random.default_rng(1).standard_normal(60)
    mv = lambda v: K @ v
    _restart_check(lambda rm: cg.cg_iterates(mv, b, np.zeros(60), refresh=2, refresh_matvec=rm),
                   lambda s0: cg.cg_iterates(mv, b, s0), K, b, 40)


def test_residual_replacement_rule():
    # exact products, so a replaced residual has the norm of the recursive one: the
    # replacements happen exactly where the recursive norm first falls below 2^-k of the
    # norm at the previous replacement, while it is above the floor
    K = _spd_kappa(40, 6, 1e2)
    b = np.random.default_rng(7).standard_normal(40)
    calls = []

    def counted(v):
        calls.append(1)
        return K @ v

    k, floor = 2, 1e-6 * np.linalg.norm(b)
    ref, expect, got = np.linalg.norm(b), [], []
    for i, s, e, _ in cg.cg_iterates(lambda v: K @ v, b, np.zeros(40), refresh=k,
                                     refresh_matvec=counted, floor=floor):
        r = np.linalg.norm(e)
        if r < ref * 2.0 ** -k and r > floor:
            expect.append(i)
            ref = r
        got += [i] * (len(calls) - len(got))
        if r < 1e-3 * floor or i >= 200:
            break
    assert got == expect and len(got) >= 3, (got, expect)
    # the rule stops replacing below the floor
    assert all(np.isfinite(got))


def test_residual_replacement_removes_the_bias_of_inexact_products():
    # products with a fixed relative perturbation (K + E) d, the way low-precision tile
    # products perturb K d: without replacement CG converges to (K + E)^-1 b; with the
    # residual replaced (by b - K s, an accurate product) whenever it has fallen by 2^4,
    # down to 2^4 times the stopping threshold, to K^-1 b within that threshold
    n = 80
    K = _spd_kappa(n, 2, 1e2)
    r = np.random.default_rng(3)
    E = r.standard_normal((n, n))
    E = 0.5 * (E + E.T)
    E *= 3e-3 * np.linalg.norm(K, 2) / np.linalg.norm(E, 2)
    b = r.standard_normal(n)
    x = np.linalg.solve(K, b)
    x_pert = np.linalg.solve(K + E, b)
    inexact = lambda v: (K + E) @ v
    exact = lambda v: K @ v
    thr = 1e-10 * np.linalg.norm(b)
    last = {}
    for name, kw in [("none", {}), ("refresh", dict(refresh=4, refresh_matvec=exact, floor=thr))]:
        for i, s, e, _ in cg.cg_iterates(inexact, b, np.zeros(n), **kw):
            if np.linalg.norm(e) < thr or i == 2000:
                last[name] = s
                break
    err_none = np.linalg.norm(last["none"] - x) / np.linalg.norm(x)
    err_fresh = np.linalg.norm(last["refresh"] - x) / np.linalg.norm(x)
    assert np.linalg.norm(last["none"] - x_pert) < 1e-8 * np.linalg.norm(x)
    assert err_none > 1e-3
    # the last replacement happens above thr; the drift after it is 3e-3 of what is left
    assert err_fresh < 1e-8, (err_none, err_fresh)


def test_pcg_residual_replacement_restarts_pcg_from_the_current_iterate():
    K = _spd_kappa(50, 4, 1e3)
    b = np.random.default_rng(5).standard_normal(50)
    w, Q = np.linalg.eigh(K)
    pinv = cg.lowrank_pinv(Q[:, -8:], 1.0 / w[-8:] - 1.0 / w[:-8].mean(), 1.0 / w[:-8].mean())
    mv = lambda v: K @ v
    _restart_check(lambda rm: cg.pcg_iterates(mv, pinv, b, np.zeros(50), refresh=2, refresh_matvec=rm),
                   lambda s0: cg.pcg_iterates(mv, pinv, b, s0), K, b, 40)
