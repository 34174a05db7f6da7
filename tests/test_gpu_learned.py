"""GPU parity of the learned warm start and preconditioner: the map from the network's
output to the preconditioner, the warm start s0 = U c, ULISSE over PCG from that warm
start, and the fallback to the plain solver, each against the FP64 oracle (or against the
plain GPU solver, which the oracle pins elsewhere) through the C ABI.

The paper has no learned component; what is checked is that the network only changes the
cost of the solves: ULISSE over any CG variant keeps its mean (Sec. 4), and an unusable
network output leaves the plain CG of Alg. 1 in charge.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import cg as ocg
from oracle import gp as ogp
from oracle import precond as opc
from oracle import ulisse as oul

pytestmark = pytest.mark.gpu

pb = pytest.importorskip("paper_1501_05427_amd.binding")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return pb.Handle(0, seed=4321)


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def colm(a, dtype=torch.float32):
    a = np.asarray(a)
    return dev(np.ascontiguousarray(a.T), dtype).t()


def problem(n, d, seed, lam=0.1, ell=(0.3, 0.8)):
    r = np.random.default_rng(seed)
    X = r.uniform(size=(n, d)).astype(np.float32)
    psi = np.concatenate([[np.log(1.2)], np.log(r.uniform(*ell, d)), [np.log(lam)]])
    return X, psi


def colwise_rel(out, ref):
    out = np.asarray(out, dtype=np.float64)
    return np.linalg.norm(out - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)


def random_network(I, H, O, seed, out_mu=None, out_sd=None):
    """FP32 parameter buffer of the library's layout with Xavier-scaled random weights."""
    r = np.random.default_rng(seed)
    p = {"W1": r.standard_normal((I, H)) * (2 / (I + H)) ** 0.5, "b1": r.standard_normal(H) * 0.1,
         "W2": r.standard_normal((H, H)) * (1 / H) ** 0.5, "b2": r.standard_normal(H) * 0.1,
         "W3": r.standard_normal((H, O)) * (2 / (H + O)) ** 0.5, "b3": r.standard_normal(O) * 0.1,
         "in_mu": r.standard_normal(I), "in_sd": r.uniform(0.5, 2, I),
         "out_mu": r.standard_normal(O) if out_mu is None else out_mu,
         "out_sd": r.uniform(0.5, 2, O) if out_sd is None else out_sd}
    lay = pb.mlp_layout(I, H, O)
    buf = np.zeros(lay["total"], np.float32)
    for name, v in p.items():
        v = np.asarray(v, np.float32).ravel()
        buf[lay[name]:lay[name] + v.size] = v
    return buf, lay


@pytest.mark.parametrize("k", [16, 64])
def test_precond_from_mlp_matches_oracle_map(h, k):
    # the device map from the network output to (h, tau_inv, c) against the oracle's
    # precond_coefficients applied to the same (BF16-inference) output
    I, H, O = 10, 256, 2 * k + 1
    # output scales that put log d and log tau around a realistic spectrum (d in e^[2, 8])
    out_mu = np.concatenate([np.zeros(k), np.linspace(8, 2, k), [1.0]])
    out_sd = np.concatenate([np.ones(k), 0.5 * np.ones(k + 1)])
    buf, lay = random_network(I, H, O, seed=k, out_mu=out_mu, out_sd=out_sd)
    bufd = dev(buf)
    r = np.random.default_rng(7)
    for trial in range(4):
        psi = r.standard_normal(I)
        psid = dev(psi)
        coef = torch.zeros(k + 1, dtype=torch.float64, device="cuda")
        cvec = torch.zeros(k, dtype=torch.float64, device="cuda")
        pb.precond_from_mlp(h, bufd, I, H, O, psid, k, coef=coef, c=cvec)
        Y = pb.precond_mlp_forward(h, bufd, I, H, O, psid[None, :], bf16=True)
        torch.cuda.synchronize()
        mu = buf[lay["out_mu"]:lay["out_mu"] + O].astype(np.float64)
        sd = buf[lay["out_sd"]:lay["out_sd"] + O].astype(np.float64)
        hh, tinv, c, ok = opc.precond_coefficients(Y.cpu().numpy()[0].astype(np.float64), mu, sd, k)
        assert ok
        got = coef.cpu().numpy()
        np.testing.assert_allclose(got[:k], hh, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(got[k], tinv, rtol=1e-12)
        np.testing.assert_allclose(cvec.cpu().numpy(), c, rtol=1e-12, atol=1e-15)
        # d floored at tau: the preconditioner is SPD
        assert np.all(got[k] + got[:k] > 0)


def test_precond_from_mlp_rejects_unusable_outputs(h):
    k = 16
    I, H, O = 6, 64, 2 * k + 1
    psid = dev(np.zeros(I))
    # (a) a NaN weight makes every output NaN; (b) a huge output scale pushes log tau out of
    # [-60, 60]: both are rejected with the fallback marker tau_inv = -1, h = 0, c = 0
    buf, lay = random_network(I, H, O, seed=1)
    bad_nan = buf.copy()
    bad_nan[lay["W2"] + 5] = np.nan
    bad_range = buf.copy()
    bad_range[lay["out_sd"] + 2 * k] = 1e4
    bad_range[lay["b3"] + 2 * k] = 1.0
    for bad in (bad_nan, bad_range):
        coef = torch.full((k + 1,), 7.0, dtype=torch.float64, device="cuda")
        cvec = torch.full((k,), 7.0, dtype=torch.float64, device="cuda")
        pb.precond_from_mlp(h, dev(bad), I, H, O, psid, k, coef=coef, c=cvec)
        torch.cuda.synchronize()
        got = coef.cpu().numpy()
        assert got[k] == -1.0 and np.all(got[:k] == 0.0) and np.all(cvec.cpu().numpy() == 0.0)
    coef = torch.zeros(k + 1, dtype=torch.float64, device="cuda")
    pb.precond_from_mlp(h, dev(buf), I, H, O, psid, k, coef=coef)
    torch.cuda.synchronize()
    assert coef.cpu().numpy()[k] > 0


def test_precond_warm_start_is_u_times_c(h):
    n, k = 3001, 64
    r = np.random.default_rng(3)
    U = r.standard_normal((n, k)).astype(np.float32)
    c = r.standard_normal(k)
    s0 = torch.zeros(n, dtype=torch.float64, device="cuda")
    pb.precond_warm_start(h, colm(U), dev(c), s0)
    torch.cuda.synchronize()
    ref = opc.warm_start(U.astype(np.float64), c)
    np.testing.assert_allclose(s0.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


def _deflation(K, k):
    w, Q = np.linalg.eigh(K)
    tau = np.mean(w[:-k])
    return Q[:, -k:], 1.0 / w[-k:] - 1.0 / tau, 1.0 / tau


@pytest.mark.parametrize("m,two_track", [(3, 1), (17, 1)])
def test_ulisse_pcg_from_learned_warm_start_draw_for_draw(h, m, two_track):
    # ULISSE over PCG with system 0 started from U c: decisions and estimates against the
    # oracle's PCG series from the same start (the series of Sec. 4 over any CG variant)
    n, d, k = 400, 2, 16
    X, psi = problem(n, d, seed=50 + m, lam=0.2, ell=(0.2, 0.4))
    K = ogp.kernel_matrix(X, psi)
    U, hh, tinv = _deflation(K, k)
    U32 = U.astype(np.float32)
    Bm = np.random.default_rng(m).standard_normal((n, m)).astype(np.float32)
    # c: the Galerkin warm start of system 0 in span(U), perturbed so that the start is
    # neither zero nor the solution's projection
    c = np.linalg.solve(U.T @ K @ U, U.T @ Bm[:, 0]) * 0.8
    s00 = U32.astype(np.float64) @ c
    pinv = ocg.lowrank_pinv(U32.astype(np.float64), hh, tinv)
    norms = []
    for i, s_, e, dl in ocg.pcg_iterates(lambda v: K @ v, pinv, Bm[:, 0].astype(np.float64), s00):
        norms.append(np.linalg.norm(e))
        if i >= 2 and min(norms[:-1]) > 1.5 * norms[-1]:
            break
    q = np.sqrt(min(norms[:-1]) * norms[-1]) / np.sqrt(n)
    rate, eps = 0.7, 1e-6
    params = pb.make_params(q=q, rate=rate, eps=eps, eps_relative=1, max_iter=200,
                            two_track_first=two_track, rng_stream=6, rng_counter=4)
    pc = pb.make_precond(colm(U32), dev(np.concatenate([hh, [tinv]])), cvec=dev(c))
    St, stats = pb.ulisse_solve_pc(h, dev(X), dev(psi), colm(Bm), params, pc)
    torch.cuda.synchronize()
    S0 = np.zeros((n, m))
    S0[:, 0] = s00
    ref_St, _, ref_stats = oul.solve_systems(lambda v: K @ v, Bm.astype(np.float64), S0, q, rate, eps,
                                             200, h.seed, 6, 4, two_track_first=bool(two_track),
                                             eps_relative=True, apply_pinv=pinv)
    for c_, (g_, r_) in enumerate(zip(pb.decode_stats(stats), ref_stats)):
        assert (g_["l"], g_["iters"], g_["J_a"], g_["flags"]) == (r_["l"], r_["iters"], r_["J"][0], r_["flags"]), c_
    assert colwise_rel(St.cpu().numpy(), ref_St).max() <= 2e-4


def test_fallback_runs_the_plain_solver(h):
    # a network with a NaN weight: precond_from_mlp marks the fallback, the preconditioned
    # gradient then runs plain CG (from the caller's warm start, not U c) with the same draws
    # as gp_stoch_grad, and every system carries ULISSE_FALLBACK
    n, d, k, nr = 900, 3, 32, 16
    X, psi = problem(n, d, seed=12, lam=0.1, ell=(0.3, 0.6))
    y = workloads.gaussian_matrix(n, 1, seed=1)[:, 0]
    R = workloads.gaussian_matrix(n, nr, seed=2)
    U, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((n, k)))
    I, H, O = d + 2, 64, 2 * k + 1
    buf, lay = random_network(I, H, O, seed=5)
    buf[lay["W1"]] = np.nan
    Xd, psid, yd, Rd = dev(X), dev(psi), dev(y), colm(R)
    coef = torch.zeros(k + 1, dtype=torch.float64, device="cuda")
    cvec = torch.zeros(k, dtype=torch.float64, device="cuda")
    pb.precond_from_mlp(h, dev(buf), I, H, O, psid, k, coef=coef, c=cvec)
    pc = pb.make_precond(colm(U.astype(np.float32)), coef, cvec=cvec)
    params = pb.make_params(q=0.5, rate=1.0, eps=1e-6, eps_relative=1, max_iter=500,
                            rng_stream=2, rng_counter=8)
    warm = 0.5 * ogp.solve(X, psi, np.column_stack([y, R]).astype(np.float64))
    Sw_plain = colm(warm, torch.float64)
    Sw_pc = colm(warm, torch.float64)
    g0, st0 = pb.gp_stoch_grad(h, Xd, psid, yd, params, R=Rd, S_warm=Sw_plain)
    g1, st1 = pb.gp_stoch_grad_pc(h, Xd, psid, yd, params, pc, R=Rd, S_warm=Sw_pc)
    torch.cuda.synchronize()
    assert coef.cpu().numpy()[k] == -1.0
    a, b = pb.decode_stats(st0), pb.decode_stats(st1)
    for c_ in range(nr + 1):
        assert b[c_]["flags"] == (a[c_]["flags"] | pb.ULISSE_FALLBACK), c_
        assert (a[c_]["l"], a[c_]["J_a"], a[c_]["J_b"], a[c_]["iters"]) == \
               (b[c_]["l"], b[c_]["J_a"], b[c_]["J_b"], b[c_]["iters"]), c_
    ga, gb = g0.cpu().numpy(), g1.cpu().numpy()
    # z = e exactly; only the order of the sums behind e^T z differs from the plain path
    np.testing.assert_allclose(gb, ga, rtol=1e-9, atol=1e-9 * np.abs(ga).max())
    np.testing.assert_allclose(Sw_pc.cpu().numpy(), Sw_plain.cpu().numpy(), rtol=1e-9,
                               atol=1e-9 * np.abs(warm).max())


def test_learned_warm_start_and_preconditioner_gains(h, capsys):
    # a trained network at new psi: converged solves of the y system need fewer products
    # from s0 = U c than from zero, the preconditioner cuts them further, and the converged
    # gradient is the plain one (the network changes only the cost)
    n, d, k, nr = 4096, 2, 64, 8
    X, psi0 = problem(n, d, seed=21, lam=0.01, ell=(0.15, 0.25))
    y = workloads.gaussian_matrix(n, 1, seed=4)[:, 0]
    Xd, yd = dev(X), dev(y)
    U, ritz = pb.precond_build_basis(h, Xd, dev(psi0), k)
    r = np.random.default_rng(7)
    psis = psi0 + 0.05 * r.standard_normal((64, d + 2))
    T = pb.precond_targets(h, Xd, yd, U, dev(psis))
    I, H, O = d + 2, 128, 2 * k + 1
    prm = torch.zeros(pb.precond_mlp_size(I, H, O), dtype=torch.float32, device="cuda")
    pb.precond_mlp_init(h, prm, I, H, O, dev(psis), T, seed=1)
    adam = torch.zeros(2 * pb.mlp_layout(I, H, O)["trainable"], dtype=torch.float32, device="cuda")
    pb.precond_mlp_train(h, prm, adam, I, H, O, dev(psis), T, 800, 0, 2e-3)
    R = workloads.gaussian_matrix(n, nr, seed=9)
    params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=5000)
    rows = []
    for j in range(3):
        psi_t = dev(psi0 + 0.05 * np.random.default_rng(100 + j).standard_normal(d + 2))
        coef = torch.zeros(k + 1, dtype=torch.float64, device="cuda")
        cvec = torch.zeros(k, dtype=torch.float64, device="cuda")
        pb.precond_from_mlp(h, prm, I, H, O, psi_t, k, coef=coef, c=cvec)
        pc_only = pb.make_precond(U, coef)
        both = pb.make_precond(U, coef, cvec=cvec)
        g0, s0 = pb.gp_stoch_grad(h, Xd, psi_t, yd, params, R=colm(R))
        # the warm start alone: plain CG with the y system started from U c
        s_uc = torch.zeros(n, dtype=torch.float64, device="cuda")
        pb.precond_warm_start(h, U, cvec, s_uc)
        S0 = torch.zeros((1 + nr, n), dtype=torch.float64, device="cuda").t()
        S0[:, 0] = s_uc
        g1, s1 = pb.gp_stoch_grad(h, Xd, psi_t, yd, params, R=colm(R), S_warm=S0)
        g2, s2 = pb.gp_stoch_grad_pc(h, Xd, psi_t, yd, params, pc_only, R=colm(R))
        g3, s3 = pb.gp_stoch_grad_pc(h, Xd, psi_t, yd, params, both, R=colm(R))
        torch.cuda.synchronize()
        its = [pb.decode_stats(s)[0]["iters"] for s in (s0, s1, s2, s3)]
        rows.append(its)
        assert all(not (st["flags"] & pb.ULISSE_FALLBACK) for st in pb.decode_stats(s3))
        a = g0.cpu().numpy()
        for gx in (g1, g2, g3):
            np.testing.assert_allclose(gx.cpu().numpy(), a, rtol=1e-3, atol=1e-4 * np.abs(a).max())
    rows = np.array(rows)
    with capsys.disabled():
        print(f"\n[learned gains] y-system CG iterations per psi (plain, warm start U c, "
              f"preconditioner, both):\n{rows}")
    assert np.all(rows[:, 1] <= rows[:, 0])         # the warm start alone never costs
    # with the preconditioner, the start changes the count by rounding only: PCG from U c and
    # from zero have no ordering theorem, and the FP32 summation order of the products moves
    # a count by one iteration either way
    assert np.all(rows[:, 3] <= rows[:, 2] + 1)
    assert np.all(rows[:, 3] < 0.6 * rows[:, 0])
