"""GPU parity of the unbiased gradient on the paths the other parity tests leave out:
d = 16 inputs, the BF16 split-K+V arithmetic, and the tiny workload run as a 200-step
SGLD chain.  Every comparison is against the FP64 oracle through the C ABI.

Tolerances:
  * FP32, draw for draw: decisions (l, J, iteration counts) exactly; gradient components
    within 2e-4 relative (the FP32 product error, <= 1e-5 per column, amplified by the
    conditioning of the test systems; the bound used by the other draw-for-draw tests).
  * BF16 split K + V, draw for draw: the product terms carry the rounding of the hi + lo
    halves of K and V, <= 3 * 2^-17 relative per term against 2^-24 in FP32.  The
    rounding errors of the halves are independent, so column errors average the same way
    as in FP32: on the 4096-point precision report the per-column K.V error is 4.4e-6
    against 1.9e-7 in FP32, a factor 23.  The FP32 tolerance of the estimates (2e-4)
    scaled by that factor is 4.6e-3; the tests use 2e-3, the bound of the BF16 ULISSE
    draw-for-draw test.  The gradient reduction of the BF16 modes takes its G tiles from
    hi + lo halves (2^-16 relative per entry), far below that.
  * Means over many estimates: within 3 Monte Carlo standard errors.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import cg as ocg
from oracle import diagnostics as odg
from oracle import gp as ogp
from oracle import rng as orng
from oracle import sgld as osgld
from oracle import stoch_grad as osg
from oracle import ulisse as oul

pytestmark = pytest.mark.gpu

pb = pytest.importorskip("paper_1501_05427_amd.binding")

FP32_TOL = 2e-4
BF16_KV_TOL = 2e-3


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def h():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return pb.Handle(0, seed=1234)


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


def safe_q(K, b, target_l):
    """q whose threshold q sqrt(n) sits midway (log scale) between the running minimum of
    the residual norms before some iteration l >= target_l and the norm at l, with a gap
    of at least 1.5, so products with a small relative error take the same l."""
    norms = []
    for i, s, e, dl in ocg.cg_iterates(lambda v: K @ v, b, np.zeros(len(b))):
        norms.append(np.linalg.norm(e))
        if i >= target_l and min(norms[:-1]) > 1.5 * norms[-1]:
            return np.sqrt(min(norms[:-1]) * norms[-1]) / np.sqrt(len(b))
        assert i < 200


# (n, d, probes, lambda, lengthscale range, seed): kappa 88 at d = 16, 31 at d = 8; every
# system stops within four CG iterations
CASES = {"d16": (640, 16, 8, 0.5, (0.5, 0.9), 617),
         "d16_m17": (640, 16, 16, 0.5, (0.5, 0.9), 617),
         "d8_m17": (600, 8, 16, 0.5, (0.2, 0.5), 608)}


def _draw_for_draw(h, case, prec, tol):
    n, d, nr, lam, ell, seed = CASES[case]
    X, psi = problem(n, d, seed=seed, lam=lam, ell=ell)
    K = ogp.kernel_matrix(X, psi)
    assert np.linalg.cond(K) < 100
    y = (np.linalg.cholesky(K) @ np.random.default_rng(1).standard_normal(n)).astype(np.float32)
    R = workloads.gaussian_matrix(n, nr, seed=3)
    q = safe_q(K, y.astype(np.float64), 2)
    stream, counter = 5, 9
    params = pb.make_params(q=q, rate=1.0, eps=1e-6, eps_relative=1, max_iter=300,
                            rng_stream=stream, rng_counter=counter, prec=prec)
    g, stats = pb.gp_stoch_grad(h, dev(X), dev(psi), dev(y), params, R=colm(R))
    torch.cuda.synchronize()
    g_ref, _, _, ref_stats = osg.stoch_grad(X, psi, y, R, q, 1.0, 1e-6, 300, h.seed, stream,
                                            counter, eps_relative=True)
    st = pb.decode_stats(stats)
    for c in range(nr + 1):
        assert ref_stats[c]["iters"] <= 7
        got = (st[c]["l"], st[c]["iters"], st[c]["J_a"], st[c]["flags"])
        assert got == (ref_stats[c]["l"], ref_stats[c]["iters"], ref_stats[c]["J"][0],
                       ref_stats[c]["flags"]), (c, st[c], ref_stats[c])
    assert st[0]["J_b"] == ref_stats[0]["J"][1]
    got = g.cpu().numpy()
    np.testing.assert_allclose(got, g_ref, rtol=tol, atol=tol * np.abs(g_ref).max())
    return got, g_ref


def test_stoch_grad_draw_for_draw_d16(h):
    # P = 18 log-parameters: the d = 16 forms of the product and of the fused gradient
    # reduction, over several row tiles of 256 and a ragged last tile
    _draw_for_draw(h, "d16", pb.GP_FP32, FP32_TOL)


@pytest.mark.parametrize("case", ["d8_m17", "d16_m17"])
def test_stoch_grad_draw_for_draw_bf16_split_kv(h, case):
    # 17 right-hand sides: the BF16 MFMA products and the split-BF16 gradient reduction
    _draw_for_draw(h, case, pb.GP_BF16_SPLIT_KV, BF16_KV_TOL)


@pytest.mark.parametrize("prec", [pb.GP_FP32, pb.GP_BF16_SPLIT_KV])
def test_stoch_grad_converged_mean_matches_exact_gradient_d16(h, prec):
    # converged solves (tiny q and rate): the estimator is Hutchinson's, whose mean over the
    # probe draws is the exact gradient (eq. gradient:unbiased); 31 Gaussian probes per
    # estimate so the products take the MFMA path and, in the BF16 mode, the split-BF16
    # gradient reduction.  The solve error of the mode (split K + V: 2.5e-5 relative on the
    # 4096-point report) is far below the standard error.
    n, d, nr, N = 640, 16, 31, 200
    X, psi = problem(n, d, seed=617, lam=0.5, ell=(0.5, 0.9))
    K = ogp.kernel_matrix(X, psi)
    y = (np.linalg.cholesky(K) @ np.random.default_rng(4).standard_normal(n)).astype(np.float32)
    g_exact = ogp.exact_gradient(X, psi, y.astype(np.float64))
    params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=400, prec=prec)
    Xd, psid, yd = dev(X), dev(psi), dev(y)
    gs = []
    for k in range(N):
        params.rng_counter = k
        g, st = pb.gp_stoch_grad(h, Xd, psid, yd, params, n_probes=nr)
        gs.append(g)
    gs = torch.stack(gs).cpu().numpy()
    assert not any(s["flags"] for s in pb.decode_stats(st))
    se = gs.std(axis=0, ddof=1) / np.sqrt(N)
    z = (gs.mean(axis=0) - g_exact) / se
    assert np.all(np.abs(z) < 3.0), z


# ---------------------------------------------------------------------------------------
# The tiny workload as a chain: n = 1000, d = 2, 4 Rademacher probes, 200 SGLD steps
# ---------------------------------------------------------------------------------------
def test_tiny_workload_200_step_chain_matches_oracle(h, capsys):
    """The tiny workload (X ~ U[0,1]^2, sigma^2 = 1, ell = (0.3, 0.3), lambda = 0.1, y drawn
    from the GP by Cholesky with seed 0) run for 200 SGLD steps with step size 1e-3: fresh
    Rademacher probes every step, q = 1, rate 1, the y system warm-started from its last CG
    iterate, prior N(0, 3^2) on every log-parameter, and the SGLD preconditioner of the
    paper's experiments (Sec. 5): M = the inverse negative Hessian of the log posterior,
    here at the true psi on all 1000 points.  With M = I the constant step 1e-3 is unstable
    for this estimator: one heavy-tailed gradient estimate throws psi out of range (the
    oracle chain overflows after 34 steps), which is what the preconditioner prevents.

    Step by step, the oracle is given the GPU chain's state before the step (psi_t and the
    warm start) and the same Philox counters:
      * the update from the GPU's gradient lands on the GPU's psi_{t+1} to FP64 rounding;
      * the y system (||y|| < alpha = q sqrt(n), so l = 1 and the tail is set by the draws)
        takes the same decisions at every step.
    A Rademacher probe has ||r|| = sqrt(n) = alpha exactly, so its threshold iteration l is
    where CG's non-monotone residual first falls below its initial norm, about ten
    iterations in, on a system with kappa ~ 3500: by then FP32 directions (the vectors the
    covariance product consumes) and FP64 ones follow visibly different CG paths, and
    finite-precision CG converges later than exact CG, so the GPU's probes cross alpha
    later than the FP64 oracle's in about half of the solves (+0.66 iterations on average).
    The test checks that explanation with a test-side run of the same CG with its directions
    and kernel entries rounded to FP32 (FP64 otherwise): it accounts for most of the shift
    (measured: 0.47 of the 0.66; the rest comes from the GPU's other FP32 rounding, of the
    scaled inputs, exp2 and the product's partial sums, which the emulation does not copy),
    and the shift stays below one iteration.  The series is unbiased
    over any convergent CG variant (Sec. 4), so the gradients must match the FP64 oracle in
    distribution: the paired differences of the gradient components have mean zero within 3
    standard errors; a free-running oracle chain driven by the same draws visits the same
    region (means of psi over the last 150 steps within 3 standard errors); and the tail
    index J of every track matches the closed form E[J] = sum_{j>=1} exp(-j(j+1)/2).
    """
    n, nr, T, eps_t = 1000, 4, 200, 1e-3
    q, rate, eps_rel, max_iter = 1.0, 1.0, 1e-6, 500
    stream = 3
    w = workloads.tiny(n=n, seed=0)
    X, psi0 = w["X"], w["psi"]
    K0 = ogp.kernel_matrix(X, psi0)
    y = (np.linalg.cholesky(K0) @ w["z"]).astype(np.float32)
    P = 4
    a, b = np.zeros(P), 3.0 * np.ones(P)
    negH = odg.neg_hessian(X, y.astype(np.float64), psi0, prior_kind=1, a=a, b=b)
    L = np.linalg.cholesky(np.linalg.inv(negH))
    Xd, yd, psid = dev(X), dev(y), dev(psi0)
    Ld = colm(L, torch.float64)
    ad, bd = dev(a), dev(b)
    Sw = torch.zeros((1 + nr, n), dtype=torch.float64, device="cuda").t()
    params = pb.make_params(q=q, rate=rate, eps=eps_rel, eps_relative=1, max_iter=max_iter,
                            rng_stream=stream)
    psis, warms, gs, stats = [], [], [], []
    for t in range(T):
        params.rng_counter = t
        psis.append(psid.clone())
        warms.append(Sw[:, 0].clone())
        g, st = pb.gp_stoch_grad(h, Xd, psid, yd, params, n_probes=nr,
                                 probe_kind=pb.PROBE_RADEMACHER, S_warm=Sw)
        gs.append(g)
        stats.append(st)
        pb.sgld_step(h, psid, g, eps_t, rng_stream=stream, rng_counter=t, prior_kind=1,
                     prior_a=ad, prior_b=bd, M_chol=Ld)
    psis.append(psid.clone())
    torch.cuda.synchronize()
    psis = torch.stack(psis).cpu().numpy()
    warms = torch.stack(warms).cpu().numpy()
    gs = torch.stack(gs).cpu().numpy()
    stats = [pb.decode_stats(s) for s in stats]

    alpha = q * np.sqrt(n)

    def l_fp32_directions(psi_t, b):
        """First CG iteration with ||e|| < alpha when the direction and the kernel entries
        are rounded to FP32 before each product (everything else FP64)."""
        K32 = ogp.signal_matrix(X, psi_t).astype(np.float32).astype(np.float64)
        lam_t = np.exp(psi_t[-1])
        e = b.astype(np.float64).copy()
        dd = e.copy()
        rho = e @ e
        for i in range(1, max_iter):
            d32 = dd.astype(np.float32).astype(np.float64)
            qv = K32 @ d32 + lam_t * d32
            al = rho / (d32 @ qv)
            e = e - al * qv
            if np.linalg.norm(e) < alpha:
                return i
            rn = e @ e
            dd = e + rn / rho * d32
            rho = rn
        return 0

    g_ref, dl, dit, dl32, J_gpu, J_ref = [], [], [], [], [], []
    for t in range(T):
        R = orng.probes(h.seed, stream, t, n, nr, 1)
        S0 = np.zeros((n, 1 + nr))
        S0[:, 0] = warms[t]
        g_o, _, _, st_ref = osg.stoch_grad(X, psis[t], y, R, q, rate, eps_rel, max_iter, h.seed,
                                           stream, t, S_warm=S0, eps_relative=True)
        g_ref.append(g_o)
        own = osgld.step_drawn(psis[t], gs[t], eps_t, h.seed, stream, t, L=L, prior_kind=1, a=a, b=b)
        np.testing.assert_allclose(psis[t + 1], own, rtol=1e-12, atol=1e-12)
        sg = stats[t]
        assert all(s_["flags"] == 0 for s_ in sg) and all(s_["flags"] == 0 for s_ in st_ref), t
        assert (sg[0]["l"], sg[0]["J_a"], sg[0]["J_b"], sg[0]["iters"]) == \
               (st_ref[0]["l"], st_ref[0]["J"][0], st_ref[0]["J"][1], st_ref[0]["iters"]), t
        for c in range(1, 1 + nr):
            dl.append(sg[c]["l"] - st_ref[c]["l"])
            dit.append(sg[c]["iters"] - st_ref[c]["iters"])
            dl32.append(sg[c]["l"] - l_fp32_directions(psis[t], R[:, c - 1]))
        J_gpu += [s_["J_a"] for s_ in sg] + [sg[0]["J_b"]]
        J_ref += [s_["J"][0] for s_ in st_ref] + [st_ref[0]["J"][1]]
    g_ref = np.array(g_ref)

    def zscore(x):
        x = np.asarray(x, dtype=np.float64)
        se = x.std(axis=0, ddof=1) / np.sqrt(len(x))
        return np.where(se > 0, x.mean(axis=0) / np.where(se > 0, se, 1.0), 0.0)

    z_l, z_l32, z_g = zscore(dl), zscore(dl32), zscore(gs - g_ref)
    differ = sum(1 for v in dit if v != 0)
    # free-running oracle chain with the same draws
    psi_o = psi0.copy()
    S_o = np.zeros((n, 1 + nr))
    traj_o = []
    for t in range(T):
        R = orng.probes(h.seed, stream, t, n, nr, 1)
        S0 = np.zeros((n, 1 + nr))
        S0[:, 0] = S_o[:, 0]
        g_o, _, S_o, _ = osg.stoch_grad(X, psi_o, y, R, q, rate, eps_rel, max_iter, h.seed,
                                        stream, t, S_warm=S0, eps_relative=True)
        psi_o = osgld.step_drawn(psi_o, g_o, eps_t, h.seed, stream, t, L=L, prior_kind=1, a=a, b=b)
        traj_o.append(psi_o)
    traj_o = np.array(traj_o)

    def batch_mean_se(x, nb=10):
        m_ = x.reshape(nb, -1, x.shape[1]).mean(axis=1)
        return x.mean(axis=0), m_.std(axis=0, ddof=1) / np.sqrt(nb)

    mg, seg = batch_mean_se(psis[51:])
    mo, seo = batch_mean_se(traj_o[50:])
    z_psi = (mg - mo) / np.sqrt(seg ** 2 + seo ** 2)
    with capsys.disabled():
        print(f"\n[tiny chain] probe solves whose iteration count differs: {differ} of {T * nr}; "
              f"l - l(FP64 oracle): mean {np.mean(dl):.3f} (z {z_l:.1f}); l - l(FP32 directions): "
              f"mean {np.mean(dl32):.3f} (z {z_l32:.2f}); z of gradient differences {np.round(z_g, 2)}; "
              f"psi means (GPU, oracle chain) {np.round(mg, 3)} {np.round(mo, 3)}, z {np.round(z_psi, 2)}")
    assert 0.0 <= np.mean(dl) < 1.0 and abs(np.mean(dl32)) < 0.5 * np.mean(dl)
    assert np.all(np.abs(z_g) < 3)
    assert np.all(np.abs(z_psi) < 3)
    EJ = oul.expected_tail_terms(rate) - 1.0
    for Js in (np.array(J_gpu, float), np.array(J_ref, float)):
        se = Js.std(ddof=1) / np.sqrt(len(Js))
        assert abs(Js.mean() - EJ) < 3 * se, (Js.mean(), EJ, se)


# ---------------------------------------------------------------------------------------
# Residual replacement
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("prec,tol", [(pb.GP_FP32, FP32_TOL), (pb.GP_BF16_SPLIT_KV, BF16_KV_TOL)])
def test_ulisse_with_residual_replacement_draw_for_draw(h, prec, tol):
    # refresh = 1: the residual is replaced by b - K s (FP32 product) and the iteration
    # restarted whenever its norm has halved since the last replacement; decisions and
    # estimates against the oracle's series with the same rule (exact products).  kappa 69,
    # every system runs 12 to 15 iterations with many replacements (the oracle counts them)
    n, d, m = 600, 8, 20
    X, psi = problem(n, d, seed=608, lam=0.5, ell=(0.2, 0.5))
    K = ogp.kernel_matrix(X, psi)
    Bm = np.random.default_rng(m).standard_normal((n, m)).astype(np.float32)
    q = safe_q(K, Bm[:, 0].astype(np.float64), 3)
    eps, rate = 1e-6, 0.7
    params = pb.make_params(q=q, rate=rate, eps=eps, eps_relative=1, max_iter=200,
                            two_track_first=1, rng_stream=8, rng_counter=5, prec=prec, refresh=1)
    St, stats = pb.ulisse_solve(h, dev(X), dev(psi), colm(Bm), params)
    torch.cuda.synchronize()
    calls = []
    ref_St, _, ref_stats = oul.solve_systems(lambda v: K @ v, Bm.astype(np.float64), None, q, rate,
                                             eps, 200, h.seed, 8, 5, two_track_first=True,
                                             eps_relative=True, refresh=1,
                                             refresh_matvec=lambda v: (calls.append(1), K @ v)[1])
    assert len(calls) >= 2 * m
    st = pb.decode_stats(stats)
    for c in range(m):
        assert (st[c]["l"], st[c]["iters"], st[c]["J_a"], st[c]["flags"]) == \
               (ref_stats[c]["l"], ref_stats[c]["iters"], ref_stats[c]["J"][0], ref_stats[c]["flags"]), c
    assert st[0]["J_b"] == ref_stats[0]["J"][1]
    num = np.linalg.norm(St.cpu().numpy() - ref_St, axis=0)
    assert np.all(num <= tol * np.linalg.norm(ref_St, axis=0)), (num / np.linalg.norm(ref_St, axis=0)).max()


@pytest.mark.parametrize("prec,bound", [(pb.GP_BF16_SPLIT_V, 2e-5), (pb.GP_BF16_SPLIT_KV, 1e-5)])
def test_residual_replacement_removes_the_bf16_solve_bias(h, prec, bound, capsys):
    # converged solves on the first 4096 points of the n = 65536, d = 8 workload against the
    # oracle's dense solution: without replacement the BF16 iterates converge to the solution
    # of the perturbed system (split V: about 1.6e-2 away); with it, to within 10x the FP32
    # mode's own error (2e-6 on this report)
    w = workloads.rff_gp(n=65536, d=8, seed=2)
    X, psi, y = w["X"][:4096], w["psi"], w["y"][:4096]
    V = np.column_stack([y, workloads.gaussian_matrix(4096, 31, seed=13)]).astype(np.float32)
    ref = ogp.solve(X, psi, V.astype(np.float64))
    errs = {}
    for rf in (0, 3, 5):
        params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=4000,
                                prec=prec, refresh=rf)
        St, stats = pb.ulisse_solve(h, dev(X), dev(psi), colm(V), params)
        torch.cuda.synchronize()
        sts = pb.decode_stats(stats)
        assert not any(s["flags"] for s in sts), (rf, sts)
        e = colwise_rel(St.cpu().numpy(), ref)
        errs[rf] = (float(np.median(e)), float(e.max()), max(s["iters"] for s in sts))
    with capsys.disabled():
        print(f"\n[residual replacement] mode {prec}: solve rel err (median, max, iterations) "
              f"without {errs[0]}; refresh 3 {errs[3]}; refresh 5 {errs[5]}")
    assert errs[3][1] <= bound and errs[5][1] <= bound


@pytest.mark.parametrize("prec", [pb.GP_BF16_SPLIT_V, pb.GP_BF16_SPLIT_KV])
def test_bf16_gradient_bias_on_subsample_4096(h, prec, capsys):
    # the gradient with converged solves in a BF16 mode, averaged over 24 batches of 31 probes,
    # against the oracle's Cholesky gradient of the first 4096 points of the n = 65536, d = 8
    # workload, per component in units of the mean's standard error.  With residual
    # replacement (k = 3) the solves land within ~2e-6 of K^-1 b and every component lies
    # within 4 SE.  Without it the split-V solves converge 1.6e-2 away from K^-1 b, and the
    # report shows what that does to the gradient.
    from paper_1501_05427_amd import protocol
    w = workloads.rff_gp(n=65536, d=8, seed=2)
    X, psi, y = w["X"][:4096], w["psi"], w["y"][:4096]
    ref = ogp.exact_gradient(X.astype(np.float64), psi, y.astype(np.float64))
    z = {}
    for rf in (0, 3):
        mean, se = protocol.probe_mean_gradient(h, dev(X), dev(y), psi, batches=24, probes=31,
                                                prec=prec, refresh=rf)
        z[rf] = (mean - ref) / se
    with capsys.disabled():
        print(f"\n[bf16 gradient bias] mode {prec}: (mean - exact) / SE per component, "
              f"without replacement {np.round(z[0], 2).tolist()}; refresh 3 {np.round(z[3], 2).tolist()}")
    assert np.all(np.abs(z[3]) < 4.0), z[3]


def colwise_rel(out, ref):
    out = np.asarray(out, dtype=np.float64)
    return np.linalg.norm(out - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)


# ---------------------------------------------------------------------------------------
# BF16 breakdown -> FP32 rerun
# ---------------------------------------------------------------------------------------
def _breakdown_case():
    # two input dimensions, 2048 random features: K is so ill-conditioned that its BF16
    # rounding (V split, K whole: 2^-9 of each entry) is indefinite for some probe systems
    w = workloads.rff_gp(n=2980, d=2, seed=1266371723, n_features=2048)
    return dev(w["X"]), dev(w["y"]), dev(w["psi"])


def _no_rerun(stats):
    return [dict(s, flags=s["flags"] & ~pb.ULISSE_FP32_RERUN) for s in stats]


def test_bf16_breakdown_reruns_gradient_in_fp32(h):
    X, y, psi = _breakdown_case()
    n, nr = X.shape[0], 16
    R = pb.gp_draw_probes(h, n, nr, pb.PROBE_GAUSSIAN, 1, 0)
    out = {}
    for name, prec, refresh in (("v", pb.GP_BF16_SPLIT_V, 3), ("fp32", pb.GP_FP32, 0)):
        params = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=1000, rng_stream=1,
                                prec=prec, refresh=refresh)
        S_warm = torch.zeros((1 + nr, n), dtype=torch.float64, device="cuda").t()
        g, st = pb.gp_stoch_grad(h, X, psi, y, params, R=R, S_warm=S_warm)
        torch.cuda.synchronize()
        out[name] = (g.cpu().numpy(), pb.decode_stats(st), S_warm.cpu().numpy())
    gv, sv, wv = out["v"]
    g32, s32, w32 = out["fp32"]
    # the flag is set only when some BF16 system broke down; the FP32 run has no breakdown
    assert all(s["flags"] & pb.ULISSE_FP32_RERUN for s in sv), sv
    assert not any(s["flags"] & pb.ULISSE_BREAKDOWN for s in s32), s32
    assert _no_rerun(sv) == s32
    np.testing.assert_array_equal(gv, g32)
    np.testing.assert_array_equal(wv, w32)
    assert np.all(np.isfinite(gv))


def test_bf16_breakdown_reruns_solve_in_fp32(h):
    X, _, psi = _breakdown_case()
    n, m = X.shape[0], 16
    B = pb.gp_draw_probes(h, n, m, pb.PROBE_GAUSSIAN, 1, 0)
    out = {}
    for name, prec, refresh in (("v", pb.GP_BF16_SPLIT_V, 3), ("fp32", pb.GP_FP32, 0)):
        params = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=1000, rng_stream=1,
                                prec=prec, refresh=refresh)
        S_cg = torch.zeros((m, n), dtype=torch.float64, device="cuda").t()
        S, st = pb.ulisse_solve(h, X, psi, B, params, S_cg=S_cg)
        torch.cuda.synchronize()
        out[name] = (S.cpu().numpy(), pb.decode_stats(st), S_cg.cpu().numpy())
    Sv, sv, cv = out["v"]
    S32, s32, c32 = out["fp32"]
    assert all(s["flags"] & pb.ULISSE_FP32_RERUN for s in sv), sv
    assert _no_rerun(sv) == s32
    np.testing.assert_array_equal(Sv, S32)
    np.testing.assert_array_equal(cv, c32)


def test_bf16_without_breakdown_does_not_rerun(h):
    # a well-conditioned system in split V: no breakdown, no rerun, a BF16 result
    X, psi = problem(3000, 8, seed=41)
    n, m = X.shape[0], 16
    Xd, psid = dev(X), dev(psi)
    B = pb.gp_draw_probes(h, n, m, pb.PROBE_GAUSSIAN, 1, 0)
    params = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=1000, rng_stream=1,
                            prec=pb.GP_BF16_SPLIT_V, refresh=3)
    S, st = pb.ulisse_solve(h, Xd, psid, B, params)
    params.prec, params.refresh = pb.GP_FP32, 0
    S32, _ = pb.ulisse_solve(h, Xd, psid, B, params)
    torch.cuda.synchronize()
    assert not any(s["flags"] & (pb.ULISSE_FP32_RERUN | pb.ULISSE_BREAKDOWN) for s in pb.decode_stats(st))
    assert not np.array_equal(S.cpu().numpy(), S32.cpu().numpy())
