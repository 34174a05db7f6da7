"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances:
  * covariance products (FP32): per column ||out - ref||_2 / ||ref||_2 <= 1e-5;
  * raw Philox words and Rademacher probes: bit-exact;
  * Gaussian probes: the FP64 Box-Muller values agree to 1e-12 relative before the
    rounding to FP32, so the FP32 probes agree to 1 ulp;
  * ULISSE and the gradient, draw for draw: the discrete decisions (l, J, iteration
    counts) exactly; the FP64 series estimates within 2e-4 normwise, the size of the FP32
    product error (about 1e-6) amplified by the conditioning of the test systems.
"""
import numpy as np
import pytest
import torch

import workloads
from oracle import cg as ocg
from oracle import gp as ogp
from oracle import rng as orng
from oracle import sgld as osgld
from oracle import stoch_grad as osg
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
    return pb.Handle(0, seed=1234)


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def colm(a, dtype=torch.float32):
    """(n, m) numpy -> column-major device tensor."""
    a = np.asarray(a)
    return dev(np.ascontiguousarray(a.T), dtype).t()


def problem(n, d, seed, lam=0.1, ell=(0.3, 0.8)):
    r = np.random.default_rng(seed)
    X = r.uniform(size=(n, d)).astype(np.float32)
    psi = np.concatenate([[np.log(1.2)], np.log(r.uniform(*ell, d)), [np.log(lam)]])
    return X, psi


def colwise_rel(out, ref):
    out = np.asarray(out, dtype=np.float64)
    num = np.linalg.norm(out - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return num / np.maximum(den, 1e-300)


# ---------------------------------------------------------------------------------------
# RNG
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("k0,k1,first,w1,w2,w3", [(0, 0, 0, 0, 0, 0), (1234, 7, 5, 3, 2, 11),
                                                   (2**64 - 1, 2**63, 2**40, 17, 1, 2**33)])
def test_philox_bitexact(k0, k1, first, w1, w2, w3):
    nb = 1000
    out = pb.gp_philox(k0, k1, first, w1, w2, w3, nb)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint64).reshape(nb, 4)
    ref = orng.blocks(k0, k1, w1, w2, w3, nb, first_block=first)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("n", [1, 7, 1001])
def test_probe_draws(h, kind, n):
    R = pb.gp_draw_probes(h, n, 3, kind, 99, 5)
    torch.cuda.synchronize()
    got = R.cpu().numpy()
    ref = orng.probes(h.seed, 99, 5, n, 3, kind).astype(np.float32)
    if kind == 1:
        np.testing.assert_array_equal(got, ref)
    else:
        np.testing.assert_allclose(got, ref, rtol=2.0 ** -23, atol=1e-30)


# ---------------------------------------------------------------------------------------
# Covariance products
# ---------------------------------------------------------------------------------------
KMV_CASES = [
    (1, 1, 1), (17, 2, 5), (300, 3, 15), (1000, 2, 5), (1000, 8, 16), (1000, 8, 17),
    (777, 16, 32), (2049, 8, 64), (513, 5, 33), (1500, 4, 1), (256, 8, 12),
    # right-hand sides past a multiple of 16 that the FP32 path takes on the VALU
    (1000, 8, 18), (700, 16, 20), (513, 5, 35), (600, 8, 51), (300, 16, 49), (1300, 3, 19),
]


@pytest.mark.parametrize("n,d,m", KMV_CASES)
def test_kmv_parity(h, n, d, m):
    X, psi = problem(n, d, seed=n * 31 + d)
    V = np.random.default_rng(m).standard_normal((n, m)).astype(np.float32)
    out = pb.gp_kmv(h, dev(X), dev(psi), colm(V))
    torch.cuda.synchronize()
    ref = ogp.kmv(X, psi, V)
    assert colwise_rel(out.cpu().numpy(), ref).max() <= 1e-5


@pytest.mark.parametrize("case", ["duplicates", "tiny_ell", "huge_ell", "noise_dominated"])
def test_kmv_edge_cases(h, case):
    n, d, m = 600, 3, 17
    r = np.random.default_rng(5)
    X = r.uniform(size=(n, d)).astype(np.float32)
    psi = np.log([1.0, 0.4, 0.4, 0.4, 0.1])
    if case == "duplicates":
        X[1::2] = X[0::2]
    elif case == "tiny_ell":      # K ~ (sigma^2 + lambda) I
        psi[1:4] = np.log(1e-4)
    elif case == "huge_ell":      # K ~ sigma^2 11^T + lambda I
        psi[1:4] = np.log(1e4)
    else:                         # sigma^2 << lambda
        psi[0], psi[-1] = np.log(1e-6), np.log(3.0)
    V = r.standard_normal((n, m)).astype(np.float32)
    out = pb.gp_kmv(h, dev(X), dev(psi), colm(V))
    torch.cuda.synchronize()
    ref = ogp.kmv(X, psi, V)
    assert colwise_rel(out.cpu().numpy(), ref).max() <= 1e-5


def test_kmv_leading_dimensions(h):
    n, d, m = 300, 2, 6
    X, psi = problem(n, d, 3)
    Xp = np.zeros((n, 5), np.float32)
    Xp[:, :d] = X
    V = np.random.default_rng(0).standard_normal((n, m)).astype(np.float32)
    Vbig = torch.zeros((m, n + 13), device="cuda")
    Vbig[:, :n] = dev(V.T)
    Vv = Vbig.t()[:n]
    outbig = torch.full((m, n + 7), 7.0, device="cuda")
    Xt = dev(Xp)[:, :d]
    pb.gp_kmv(h, Xt, dev(psi), Vv, out=outbig.t()[:n])
    torch.cuda.synchronize()
    got = outbig.cpu().numpy()
    assert colwise_rel(got[:, :n].T, ogp.kmv(X, psi, V)).max() <= 1e-5
    assert np.all(got[:, n:] == 7.0)  # nothing written past n


# Error bounds of the BF16 contraction modes, per column, relative to || |K| |V| ||:
# split-V rounds every K entry to BF16 (|delta| <= 2^-9) and V to hi + lo (2^-17);
# split-KV keeps K_hi + K_lo and V_hi + V_lo and drops K_lo V_lo (about 3 * 2^-18 in all).
# Both bounds carry a factor 2 of margin plus the FP32 accumulation term.
BF16_BOUND = {pb.GP_BF16_SPLIT_V: 2.0 ** -8, pb.GP_BF16_SPLIT_KV: 6 * 2.0 ** -18}


def absprod_norm(X, psi, V):
    return np.linalg.norm(np.abs(ogp.kernel_matrix(X, psi)) @ np.abs(V.astype(np.float64)), axis=0)


@pytest.mark.parametrize("prec", [pb.GP_BF16_SPLIT_V, pb.GP_BF16_SPLIT_KV])
@pytest.mark.parametrize("n,d,m", [(1000, 8, 16), (777, 2, 32), (2049, 16, 33), (600, 5, 64)])
def test_kmv_bf16_error_bound(h, prec, n, d, m):
    X, psi = problem(n, d, seed=n + m)
    V = np.random.default_rng(m).standard_normal((n, m)).astype(np.float32)
    out = pb.gp_kmv(h, dev(X), dev(psi), colm(V), prec=prec)
    torch.cuda.synchronize()
    ref = ogp.kmv(X, psi, V)
    err = np.linalg.norm(out.cpu().numpy().astype(np.float64) - ref, axis=0)
    bound = (BF16_BOUND[prec] + 1e-6) * absprod_norm(X, psi, V)
    assert np.all(err <= bound), (err / bound).max()


def test_kmv_bf16_below_16_columns_is_fp32(h):
    # with fewer than 16 right-hand sides the contraction is on the VALU in FP32
    n, d, m = 500, 3, 7
    X, psi = problem(n, d, seed=1)
    V = np.random.default_rng(0).standard_normal((n, m)).astype(np.float32)
    a = pb.gp_kmv(h, dev(X), dev(psi), colm(V), prec=pb.GP_BF16_SPLIT_V)
    b = pb.gp_kmv(h, dev(X), dev(psi), colm(V), prec=pb.GP_FP32)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


@pytest.mark.parametrize("prec", [pb.GP_FP32, pb.GP_BF16_SPLIT_V, pb.GP_BF16_SPLIT_KV])
def test_precision_report_subsample_4096(h, prec, capsys):
    # the n = 65536, d = 8 workload restricted to its first 4096 points, solved densely by
    # the oracle: error of K V and of converged solves for each arithmetic mode
    w = workloads.rff_gp(n=65536, d=8, seed=2)
    X, psi, y = w["X"][:4096], w["psi"], w["y"][:4096]
    V = np.column_stack([y, workloads.gaussian_matrix(4096, 31, seed=13)]).astype(np.float32)
    out = pb.gp_kmv(h, dev(X), dev(psi), colm(V), prec=prec)
    params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=4000, prec=prec)
    St, stats = pb.ulisse_solve(h, dev(X), dev(psi), colm(V), params)
    torch.cuda.synchronize()
    ref_kv = ogp.kmv(X, psi, V)
    ref_s = ogp.solve(X, psi, V.astype(np.float64))
    e_kv = colwise_rel(out.cpu().numpy(), ref_kv).max()
    e_s = colwise_rel(St.cpu().numpy(), ref_s)
    its = [s["iters"] for s in pb.decode_stats(stats)]
    with capsys.disabled():
        print(f"\n[precision report] mode {prec}: K.V max col rel err {e_kv:.2e}; solve rel err "
              f"median {np.median(e_s):.2e} max {e_s.max():.2e}; CG iterations {min(its)}-{max(its)}")
    bound = {pb.GP_FP32: 1e-5, pb.GP_BF16_SPLIT_V: 2e-2, pb.GP_BF16_SPLIT_KV: 1e-4}[prec]
    assert e_kv <= bound


@pytest.mark.parametrize("n,d,m", [(400, 2, 3), (700, 8, 16), (333, 3, 20), (257, 16, 5)])
def test_dkmv_parity(h, n, d, m):
    X, psi = problem(n, d, seed=7 * n)
    V = np.random.default_rng(1).standard_normal((n, m)).astype(np.float32)
    out = pb.gp_dkmv(h, dev(X), dev(psi), colm(V))
    torch.cuda.synchronize()
    got = out.cpu().numpy()            # (P, m, n)
    ref = ogp.dkmv(X, psi, V)          # (P, n, m)
    for j in range(d + 2):
        assert colwise_rel(got[j].T, ref[j]).max() <= 1e-5, j


def test_kmv_full_size_sampled_n16384_m17(h):
    # the n = 16384, d = 8 workload with y + 16 probes (one MFMA block and one VALU
    # column) in the default launch shape; sampled rows from the oracle
    w = workloads.rff_gp(n=16384, d=8, seed=1)
    X, psi = w["X"], w["psi"]
    V = workloads.gaussian_matrix(16384, 17, seed=12)
    out = pb.gp_kmv(h, dev(X), dev(psi), colm(V))
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(3).choice(16384, 64, replace=False))
    rows[0], rows[-1] = 0, 16383
    ref = ogp.kmv(X, psi, V, rows=rows)
    assert colwise_rel(out.cpu().numpy()[rows], ref).max() <= 1e-5


def test_kmv_full_size_sampled_mixture_n131072_d16(h):
    # the largest workload (n = 131072, d = 16, 8-Gaussian mixture inputs, m = 32) in the
    # default launch shape (two row blocks per wave at d = 16); sampled rows from the oracle
    w = workloads.mixture(n=131072, d=16, seed=4)
    X, psi = w["X"], w["psi"]
    V = workloads.gaussian_matrix(131072, 32, seed=14)
    out = pb.gp_kmv(h, dev(X), dev(psi), colm(V))
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(4).choice(131072, 24, replace=False))
    rows[0], rows[-1] = 0, 131071
    ref = ogp.kmv(X, psi, V, rows=rows)
    assert colwise_rel(out.cpu().numpy()[rows], ref).max() <= 1e-5


@pytest.mark.parametrize("rows_seed", [0, 1])
def test_kmv_full_size_sampled(h, rows_seed):
    # the benchmark's workload (n = 65536, d = 8, m = 32) in the benchmark's launch shape;
    # the oracle computes a sample of output rows one by one
    w = workloads.rff_gp(n=65536, d=8, seed=2)
    X, psi = w["X"], w["psi"]
    V = workloads.gaussian_matrix(65536, 32, seed=11)
    out = pb.gp_kmv(h, dev(X), dev(psi), colm(V))
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(rows_seed).choice(65536, 48, replace=False))
    rows[-1] = 65535
    got = out.cpu().numpy()[rows]
    ref = ogp.kmv(X, psi, V, rows=rows)
    assert colwise_rel(got, ref).max() <= 1e-5


# ---------------------------------------------------------------------------------------
# ULISSE, draw for draw
# ---------------------------------------------------------------------------------------
def _safe_q(K, b, s0, target_l):
    """q whose threshold q sqrt(n) sits midway (log scale) between the running minimum of
    the residual norms before some iteration l >= target_l and the norm at l, with a
    clear gap, so FP32 and FP64 runs take the same l."""
    norms = []
    for i, s, e, dl in ocg.cg_iterates(lambda v: K @ v, b, s0):
        norms.append(np.linalg.norm(e))
        if i >= target_l and min(norms[:-1]) > 1.5 * norms[-1]:
            hi, lo = min(norms[:-1]), norms[-1]
            return np.sqrt(hi * lo) / np.sqrt(len(b))
        assert i < 200


@pytest.mark.parametrize("two_track,warm,m,prec", [(0, False, 3, 0), (1, False, 5, 0), (1, True, 4, 0),
                                                   (0, True, 17, 0), (1, False, 20, 2)])
def test_ulisse_draw_for_draw(h, two_track, warm, m, prec):
    n, d = 400, 2
    X, psi = problem(n, d, seed=40 + m, lam=0.2, ell=(0.2, 0.4))
    K = ogp.kernel_matrix(X, psi)
    Bm = np.random.default_rng(m).standard_normal((n, m)).astype(np.float32)
    S0 = None
    if warm:
        S0 = 0.9 * ogp.solve(X, psi, Bm.astype(np.float64))
    q = _safe_q(K, Bm[:, 0].astype(np.float64), np.zeros(n) if S0 is None else S0[:, 0], 3)
    eps, rate = 1e-6, 0.7
    params = pb.make_params(q=q, rate=rate, eps=eps, eps_relative=1, max_iter=200,
                            two_track_first=two_track, rng_stream=77, rng_counter=3, prec=prec)
    Scg = torch.zeros((m, n), dtype=torch.float64, device="cuda").t()
    St, stats = pb.ulisse_solve(h, dev(X), dev(psi), colm(Bm), params,
                                S0=None if S0 is None else colm(S0, torch.float64), S_cg=Scg)
    torch.cuda.synchronize()
    st_gpu = pb.decode_stats(stats)
    ref_St, ref_Scg, ref_stats = oul.solve_systems(
        lambda v: K @ v, Bm.astype(np.float64), S0, q, rate, eps, 200, h.seed, 77, 3,
        two_track_first=bool(two_track), eps_relative=True)
    for c in range(m):
        g, r = st_gpu[c], ref_stats[c]
        assert g["l"] == r["l"] and g["iters"] == r["iters"], (c, g, r)
        assert g["J_a"] == r["J"][0], (c, g, r)
        if two_track and c == 0:
            assert g["J_b"] == r["J"][1]
        assert g["flags"] == r["flags"]
    tol = 2e-4 if prec == pb.GP_FP32 else 2e-3
    assert colwise_rel(St.cpu().numpy(), ref_St).max() <= tol
    assert colwise_rel(Scg.cpu().numpy(), ref_Scg).max() <= tol


def test_ulisse_cap_sets_notconv(h):
    n, d, m = 300, 2, 2
    X, psi = problem(n, d, seed=3, lam=1e-3)
    Bm = np.random.default_rng(0).standard_normal((n, m)).astype(np.float32)
    params = pb.make_params(q=1e-9, rate=1.0, eps=1e-12, eps_relative=1, max_iter=4)
    St, stats = pb.ulisse_solve(h, dev(X), dev(psi), colm(Bm), params)
    torch.cuda.synchronize()
    for s in pb.decode_stats(stats):
        assert s["iters"] == 4 and (s["flags"] & pb.ULISSE_NOTCONV)


def test_ulisse_converged_series_is_the_solution(h):
    # small q and tiny rate: the tail runs to convergence, s~ = s_T ~ K^-1 b
    n, d, m = 500, 3, 4
    X, psi = problem(n, d, seed=9, lam=0.3)
    Bm = np.random.default_rng(2).standard_normal((n, m)).astype(np.float32)
    params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=500)
    St, stats = pb.ulisse_solve(h, dev(X), dev(psi), colm(Bm), params)
    torch.cuda.synchronize()
    ref = ogp.solve(X, psi, Bm.astype(np.float64))
    assert colwise_rel(St.cpu().numpy(), ref).max() <= 1e-4


# ---------------------------------------------------------------------------------------
# Stochastic gradient and SGLD
# ---------------------------------------------------------------------------------------
# Draw-for-draw comparisons need CG paths that FP32 products do not change: CG on these
# kernel matrices turns chaotic in finite precision after some iterations (on badly
# conditioned systems a relative perturbation of 1e-8 already changes residual norms by
# O(1) within ten iterations), so the test systems are well conditioned (kappa < 100)
# and stop within the first few iterations, where a CPU emulation with 1e-5 relative
# product noise changes no residual norm by more than 1e-4.
@pytest.mark.parametrize("given_probes", [True, False])
@pytest.mark.parametrize("n,d,nr,lam,ell,seed", [(300, 2, 4, 1.0, (0.1, 0.3), 302),
                                                 (600, 8, 16, 0.5, (0.2, 0.5), 608)])
def test_stoch_grad_draw_for_draw(h, given_probes, n, d, nr, lam, ell, seed):
    X, psi = problem(n, d, seed=seed, lam=lam, ell=ell)
    K = ogp.kernel_matrix(X, psi)
    y = (np.linalg.cholesky(K) @ np.random.default_rng(1).standard_normal(n)).astype(np.float32)
    stream, counter = 5, 9
    if given_probes:
        R = workloads.gaussian_matrix(n, nr, seed=3)
    else:
        R = orng.probes(h.seed, stream, counter, n, nr, 0).astype(np.float32)
    q = _safe_q(K, y.astype(np.float64), np.zeros(n), 2)
    eps, rate = 1e-6, 1.0
    params = pb.make_params(q=q, rate=rate, eps=eps, eps_relative=1, max_iter=300,
                            rng_stream=stream, rng_counter=counter)
    g, stats = pb.gp_stoch_grad(h, dev(X), dev(psi), dev(y), params,
                                R=colm(R) if given_probes else None, n_probes=nr)
    torch.cuda.synchronize()
    g_ref, St, Scg, ref_stats = osg.stoch_grad(X, psi, y, R, q, rate, eps, 300, h.seed, stream,
                                               counter, eps_relative=True)
    st_gpu = pb.decode_stats(stats)
    for c in range(nr + 1):
        assert ref_stats[c]["iters"] <= 7
        assert (st_gpu[c]["l"], st_gpu[c]["iters"]) == (ref_stats[c]["l"], ref_stats[c]["iters"]), c
    got = g.cpu().numpy()
    scale = np.abs(g_ref).max()
    np.testing.assert_allclose(got, g_ref, rtol=2e-4, atol=2e-4 * scale)


def test_stoch_grad_exact_solve_mean_matches_exact_gradient(h):
    # with converged solves (tiny q and rate) the estimator is Hutchinson's; its mean over
    # many probe draws is the exact gradient, within Monte Carlo error
    n, d, nr = 200, 2, 8
    X, psi = problem(n, d, seed=2, lam=0.3)
    K = ogp.kernel_matrix(X, psi)
    y = (np.linalg.cholesky(K) @ np.random.default_rng(4).standard_normal(n)).astype(np.float32)
    g_exact = ogp.exact_gradient(X, psi, y.astype(np.float64))
    params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=400)
    Xd, psid, yd = dev(X), dev(psi), dev(y)
    N = 400
    gs = []
    for k in range(N):
        params.rng_counter = k
        g, _ = pb.gp_stoch_grad(h, Xd, psid, yd, params, n_probes=nr)
        gs.append(g)
    gs = torch.stack(gs).cpu().numpy()
    se = gs.std(axis=0, ddof=1) / np.sqrt(N)
    z = (gs.mean(axis=0) - g_exact) / se
    assert np.all(np.abs(z) < 3.0), z   # gradient means within 3 Monte Carlo standard errors


def test_stoch_grad_full_size_consistency(h):
    # n = 65536, d = 8, 31 probes, in the benchmark's launch shapes: every component of the
    # fused gradient reduction agrees with derivative products (gp_dkmv, pinned to the
    # oracle above) of the same series estimates, assembled in FP64 on the host
    n, d, nr = 65536, 8, 31
    w = workloads.rff_gp(n=n, d=d, seed=2)
    Xd, psid, yd = dev(w["X"]), dev(w["psi"]), dev(w["y"])
    R = workloads.gaussian_matrix(n, nr, seed=12)
    Rd = colm(R)
    params = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=500,
                            rng_stream=3, rng_counter=1)
    g, stats = pb.gp_stoch_grad(h, Xd, psid, yd, params, R=Rd)
    B = torch.cat([yd[:, None], Rd], dim=1).t().contiguous().t()
    p2 = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=500,
                        two_track_first=1, rng_stream=3, rng_counter=1)
    St, stats2 = pb.ulisse_solve(h, Xd, psid, B, p2)
    dKS = pb.gp_dkmv(h, Xd, psid, St.float().t().contiguous().t())   # (P, m+1, n)
    torch.cuda.synchronize()
    assert pb.decode_stats(stats) == pb.decode_stats(stats2)
    Stn = St.cpu().numpy()
    dKSn = dKS.cpu().numpy().astype(np.float64)
    Rn = R.astype(np.float64)
    ref = np.array([0.5 * Stn[:, 0] @ dKSn[j, 1] - sum(Rn[:, c] @ dKSn[j, c + 2] for c in range(nr)) / (2 * nr)
                    for j in range(d + 2)])
    gn = g.cpu().numpy()
    assert np.all(np.isfinite(gn))
    scale = np.abs(ref).max()
    np.testing.assert_allclose(gn, ref, rtol=1e-4, atol=1e-5 * scale)
    for s in pb.decode_stats(stats):
        assert s["l"] >= 1 and s["iters"] == s["l"] + max(s["J_a"], s["J_b"]) and s["flags"] == 0


@pytest.mark.parametrize("d,nr", [(3, 4), (12, 20), (5, 36), (8, 52), (2, 62)])
def test_stoch_grad_consistency_column_counts(h, d, nr):
    # the fused gradient reduction at every padded width of its A and B operands (1 + nr
    # columns rounded up to 8, 8 to 64) against derivative products of the same series
    # estimates (gp_dkmv), assembled in FP64 on the host; a ragged n over several tiles
    n = 3000
    X, psi = problem(n, d, seed=40 + nr, lam=0.2, ell=(0.3, 0.9))
    y = np.random.default_rng(nr).standard_normal(n).astype(np.float32)
    R = workloads.gaussian_matrix(n, nr, seed=nr + 1)
    Xd, psid, yd, Rd = dev(X), dev(psi), dev(y), colm(R)
    params = pb.make_params(q=0.5, rate=1.0, eps=1e-6, eps_relative=1, max_iter=500,
                            rng_stream=6, rng_counter=2)
    g, stats = pb.gp_stoch_grad(h, Xd, psid, yd, params, R=Rd)
    B = torch.cat([yd[:, None], Rd], dim=1).t().contiguous().t()
    p2 = pb.make_params(q=0.5, rate=1.0, eps=1e-6, eps_relative=1, max_iter=500,
                        two_track_first=1, rng_stream=6, rng_counter=2)
    St, stats2 = pb.ulisse_solve(h, Xd, psid, B, p2)
    dKS = pb.gp_dkmv(h, Xd, psid, St.float().t().contiguous().t())   # (P, m+1, n)
    torch.cuda.synchronize()
    assert pb.decode_stats(stats) == pb.decode_stats(stats2)
    Stn = St.cpu().numpy()
    dKSn = dKS.cpu().numpy().astype(np.float64)
    Rn = R.astype(np.float64)
    ref = np.array([0.5 * Stn[:, 0] @ dKSn[j, 1] - sum(Rn[:, c] @ dKSn[j, c + 2] for c in range(nr)) / (2 * nr)
                    for j in range(d + 2)])
    gn = g.cpu().numpy()
    assert np.all(np.isfinite(gn))
    np.testing.assert_allclose(gn, ref, rtol=1e-4, atol=1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("prior_kind", [0, 1, 2])
def test_sgld_step_parity(h, prior_kind):
    P = 6
    r = np.random.default_rng(prior_kind)
    psi = r.standard_normal(P)
    g = r.standard_normal(P) * 10
    A = r.standard_normal((P, P))
    L = np.linalg.cholesky(A @ A.T + P * np.eye(P))
    a, b = r.uniform(1, 3, P), r.uniform(0.5, 2, P)
    psid = dev(psi)
    pb.sgld_step(h, psid, dev(g), 1e-3, rng_stream=4, rng_counter=8, prior_kind=prior_kind,
                 prior_a=dev(a), prior_b=dev(b), M_chol=dev(L.ravel(order="F")))
    torch.cuda.synchronize()
    ref = osgld.step_drawn(psi, g, 1e-3, h.seed, 4, 8, L, prior_kind, a, b)
    np.testing.assert_allclose(psid.cpu().numpy(), ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("freeze_ratio", [1e-12, 1e12])
def test_sgld_run_protocol(h, freeze_ratio):
    # the paper's protocol on a small chain: probes redrawn every 3 steps, warm starts,
    # decreasing step size, monitor on batches of 4 gradients, freeze rule; converged
    # solves keep both sides on the same path, so the traces must agree
    n, d, nr, T = 300, 2, 4, 10
    X, psi = problem(n, d, seed=302, lam=1.0, ell=(0.1, 0.3))
    K = ogp.kernel_matrix(X, psi)
    y = (np.linalg.cholesky(K) @ np.random.default_rng(1).standard_normal(n)).astype(np.float32)
    q, rate, eps_c, stream = 1e-12, 1e-9, 1e-7, 6
    a, b = osgld.schedule_from_endpoints(2e-3, 1e-3, T)
    L = np.diag(np.full(d + 2, n ** -0.5))
    params = pb.make_params(q=q, rate=rate, eps=eps_c, eps_relative=1, max_iter=500, rng_stream=stream)
    sched = pb.make_schedule(a, b, 1.0, freeze_ratio, batch=4, probe_period=3, n_probes=nr,
                             probe_kind=pb.PROBE_RADEMACHER)
    state = pb.new_state(0)
    psid = dev(psi)
    S_warm = torch.zeros((nr + 1, n), dtype=torch.float64, device="cuda").t()
    R = pb.colmajor(n, nr)
    trace = torch.zeros((T, d + 2), dtype=torch.float64, device="cuda")
    eps_tr = torch.zeros(T, dtype=torch.float64, device="cuda")
    ratio_tr = torch.zeros(T, dtype=torch.float64, device="cuda")
    pa, pbb = np.zeros(d + 2), np.full(d + 2, 3.0)
    Ld = dev(L.ravel(order="F"))
    # two calls (6 + 4 steps) exercise resumption
    pb.sgld_run(h, dev(X), psid, dev(y), params, sched, state, 6, S_warm, R, prior_kind=1,
                prior_a=dev(pa), prior_b=dev(pbb), M_chol=Ld, trace=trace[:6], eps_trace=eps_tr[:6],
                ratio_trace=ratio_tr[:1])
    pb.sgld_run(h, dev(X), psid, dev(y), params, sched, state, 4, S_warm, R, prior_kind=1,
                prior_a=dev(pa), prior_b=dev(pbb), M_chol=Ld, trace=trace[6:], eps_trace=eps_tr[6:],
                ratio_trace=ratio_tr[1:])
    torch.cuda.synchronize()
    # oracle run of the same protocol
    p_o = psi.copy()
    Sw = np.zeros((n, nr + 1))
    R_o = None
    G = []
    ratios, eps_list, tr = [], [], []
    frozen, eps_frozen, frozen_at = False, 0.0, -1
    for t in range(T):
        if t % 3 == 0:
            R_o = orng.probes(h.seed, stream, t // 3, n, nr, 1)
            Sw[:, 1:] = 0.0
        g, St, Scg, _ = osg.stoch_grad(X, p_o, y, R_o, q, rate, eps_c, 500, h.seed, stream, t,
                                       S_warm=Sw, eps_relative=True)
        Sw = Scg
        G.append(g)
        e = eps_frozen if frozen else osgld.eps_schedule(a, b, 1.0, t)
        eps_list.append(e)
        p_o = osgld.step_drawn(p_o, g, e, h.seed, stream, t, L, 1, pa, pbb)
        tr.append(p_o.copy())
        if (t + 1) % 4 == 0:
            rr = osgld.langevin_ratio(np.array(G[-4:]), L, e)
            ratios.append(rr)
            if not frozen and rr < freeze_ratio:
                frozen, eps_frozen, frozen_at = True, e, t
    np.testing.assert_allclose(eps_tr.cpu().numpy(), eps_list, rtol=1e-14)
    np.testing.assert_allclose(trace.cpu().numpy(), np.array(tr), rtol=1e-7, atol=1e-7)
    np.testing.assert_allclose(ratio_tr.cpu().numpy()[:2], ratios, rtol=1e-3)
    assert (state.frozen, state.frozen_at) == (int(frozen), frozen_at) and state.t == T


def _deflation(K, k):
    """Top-k eigenvectors of K and the matching h, tau_inv (test-side construction)."""
    w, Q = np.linalg.eigh(K)
    U, dk = Q[:, -k:], w[-k:]
    tau = np.mean(w[:-k])
    h_ = 1.0 / dk - 1.0 / tau
    return U, h_, 1.0 / tau


@pytest.mark.parametrize("k,m,two_track", [(16, 3, 0), (32, 17, 1), (64, 5, 1)])
def test_ulisse_pcg_draw_for_draw(h, k, m, two_track):
    n, d = 400, 2
    X, psi = problem(n, d, seed=40 + m, lam=0.2, ell=(0.2, 0.4))
    K = ogp.kernel_matrix(X, psi)
    U, hh, tinv = _deflation(K, k)
    pinv = ocg.lowrank_pinv(U, hh, tinv)
    Bm = np.random.default_rng(m).standard_normal((n, m)).astype(np.float32)
    # threshold between two residual norms of the preconditioned run of system 0
    norms = []
    for i, s_, e, dl in ocg.pcg_iterates(lambda v: K @ v, pinv, Bm[:, 0].astype(np.float64), np.zeros(n)):
        norms.append(np.linalg.norm(e))
        if i >= 2 and min(norms[:-1]) > 1.5 * norms[-1]:
            break
    q = np.sqrt(min(norms[:-1]) * norms[-1]) / np.sqrt(n)
    rate, eps = 0.7, 1e-6
    params = pb.make_params(q=q, rate=rate, eps=eps, eps_relative=1, max_iter=200,
                            two_track_first=two_track, rng_stream=5, rng_counter=2)
    Ud = colm(U.astype(np.float32))
    coef = dev(np.concatenate([hh, [tinv]]))
    pc = pb.make_precond(Ud, coef)
    St, stats = pb.ulisse_solve_pc(h, dev(X), dev(psi), colm(Bm), params, pc)
    torch.cuda.synchronize()
    U32 = U.astype(np.float32).astype(np.float64)
    ref_St, _, ref_stats = oul.solve_systems(lambda v: K @ v, Bm.astype(np.float64), None, q, rate, eps,
                                             200, h.seed, 5, 2, two_track_first=bool(two_track),
                                             eps_relative=True, apply_pinv=ocg.lowrank_pinv(U32, hh, tinv))
    for c, (g_, r) in enumerate(zip(pb.decode_stats(stats), ref_stats)):
        assert (g_["l"], g_["iters"], g_["J_a"], g_["flags"]) == (r["l"], r["iters"], r["J"][0], r["flags"]), c
    assert colwise_rel(St.cpu().numpy(), ref_St).max() <= 2e-4


def test_pcg_converged_solution_and_fewer_iterations(h):
    n, d, m, k = 1000, 2, 4, 64
    X, psi = problem(n, d, seed=3, lam=0.02, ell=(0.2, 0.3))
    K = ogp.kernel_matrix(X, psi)
    U, hh, tinv = _deflation(K, k)
    Bm = np.random.default_rng(0).standard_normal((n, m)).astype(np.float32)
    params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=3000)
    pc = pb.make_precond(colm(U.astype(np.float32)), dev(np.concatenate([hh, [tinv]])))
    St_pc, st_pc = pb.ulisse_solve_pc(h, dev(X), dev(psi), colm(Bm), params, pc)
    St, st = pb.ulisse_solve(h, dev(X), dev(psi), colm(Bm), params)
    torch.cuda.synchronize()
    ref = ogp.solve(X, psi, Bm.astype(np.float64))
    assert colwise_rel(St_pc.cpu().numpy(), ref).max() <= 1e-4, (pb.decode_stats(st_pc), pb.decode_stats(st))
    it_pc = max(s["iters"] for s in pb.decode_stats(st_pc))
    it = max(s["iters"] for s in pb.decode_stats(st))
    assert it_pc < 0.7 * it, (it_pc, it)


# ---------------------------------------------------------------------------------------
# PCG with J = K + delta I applied by an inner CG (Sec. 3.3)
# ---------------------------------------------------------------------------------------
def _pcg_q(K, b, pinv, target_l=1):
    """q between two residual norms of a PCG run (same rule as _safe_q)."""
    norms = []
    for i, s_, e, dl in ocg.pcg_iterates(lambda v: K @ v, pinv, b, np.zeros(len(b))):
        norms.append(np.linalg.norm(e))
        if i >= target_l + 1 and min(norms[:-1]) > 1.5 * norms[-1]:
            return np.sqrt(min(norms[:-1]) * norms[-1]) / np.sqrt(len(b))
        assert i < 100


@pytest.mark.parametrize("m,two_track,delta,max_inner", [(3, 0, 0.5, 4), (17, 1, 0.2, 3), (5, 1, 1.0, 6)])
def test_ulisse_shift_pcg_draw_for_draw(h, m, two_track, delta, max_inner):
    # a fixed inner count (eps_inner = 0) leaves no inner decision to rounding
    n, d = 400, 2
    X, psi = problem(n, d, seed=40 + m, lam=0.2, ell=(0.2, 0.4))
    K = ogp.kernel_matrix(X, psi)
    Bm = np.random.default_rng(m).standard_normal((n, m)).astype(np.float32)
    pinv = ocg.shifted_inner_pinv(lambda v: K @ v, delta, 0.0, max_inner)
    q = _pcg_q(K, Bm[:, 0].astype(np.float64), pinv)
    rate, eps = 0.7, 1e-6
    params = pb.make_params(q=q, rate=rate, eps=eps, eps_relative=1, max_iter=200,
                            two_track_first=two_track, rng_stream=5, rng_counter=2)
    sp = pb.make_shift_precond(delta, 0.0, max_inner)
    St, stats = pb.ulisse_solve_shift_pc(h, dev(X), dev(psi), colm(Bm), params, sp)
    torch.cuda.synchronize()
    ref_St, _, ref_stats = oul.solve_systems(lambda v: K @ v, Bm.astype(np.float64), None, q, rate, eps,
                                             200, h.seed, 5, 2, two_track_first=bool(two_track),
                                             eps_relative=True, apply_pinv=pinv)
    for c, (g_, r) in enumerate(zip(pb.decode_stats(stats), ref_stats)):
        assert (g_["l"], g_["iters"], g_["J_a"], g_["flags"]) == (r["l"], r["iters"], r["J"][0], r["flags"]), c
    assert colwise_rel(St.cpu().numpy(), ref_St).max() <= 2e-4


def test_shift_pcg_converged_solution_and_outer_iterations(h):
    n, d, m = 1000, 2, 4
    X, psi = problem(n, d, seed=3, lam=0.02, ell=(0.2, 0.3))
    Bm = np.random.default_rng(0).standard_normal((n, m)).astype(np.float32)
    params = pb.make_params(q=0.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=3000)
    sp = pb.make_shift_precond(0.05, 1e-4, 200)
    St_sp, st_sp = pb.ulisse_solve_shift_pc(h, dev(X), dev(psi), colm(Bm), params, sp)
    St, st = pb.ulisse_solve(h, dev(X), dev(psi), colm(Bm), params)
    torch.cuda.synchronize()
    ref = ogp.solve(X, psi, Bm.astype(np.float64))
    ss, sc = pb.decode_stats(st_sp), pb.decode_stats(st)
    assert not any(s_["flags"] for s_ in ss), ss
    assert colwise_rel(St_sp.cpu().numpy(), ref).max() <= 1e-4
    assert colwise_rel(St.cpu().numpy(), ref).max() <= 1e-4
    # nearly exact inner solves of a close J: far fewer outer iterations than plain CG
    assert max(s_["iters"] for s_ in ss) < 0.5 * max(s_["iters"] for s_ in sc), (ss, sc)


def test_stoch_grad_shift_pcg_draw_for_draw(h):
    n, d, nr, lam, ell, seed = 300, 2, 4, 1.0, (0.1, 0.3), 302
    X, psi = problem(n, d, seed=seed, lam=lam, ell=ell)
    K = ogp.kernel_matrix(X, psi)
    y = (np.linalg.cholesky(K) @ np.random.default_rng(1).standard_normal(n)).astype(np.float32)
    R = workloads.gaussian_matrix(n, nr, seed=3)
    delta, max_inner = 0.5, 3
    pinv = ocg.shifted_inner_pinv(lambda v: K @ v, delta, 0.0, max_inner)
    q = _pcg_q(K, y.astype(np.float64), pinv)
    stream, counter, eps, rate = 5, 9, 1e-6, 1.0
    params = pb.make_params(q=q, rate=rate, eps=eps, eps_relative=1, max_iter=300,
                            rng_stream=stream, rng_counter=counter)
    sp = pb.make_shift_precond(delta, 0.0, max_inner)
    g, stats = pb.gp_stoch_grad_shift_pc(h, dev(X), dev(psi), dev(y), params, sp, R=colm(R))
    torch.cuda.synchronize()
    g_ref, St, Scg, ref_stats = osg.stoch_grad(X, psi, y, R, q, rate, eps, 300, h.seed, stream, counter,
                                               eps_relative=True, apply_pinv=pinv)
    st_gpu = pb.decode_stats(stats)
    for c in range(nr + 1):
        assert ref_stats[c]["iters"] <= 7
        assert (st_gpu[c]["l"], st_gpu[c]["iters"]) == (ref_stats[c]["l"], ref_stats[c]["iters"]), c
    scale = np.abs(g_ref).max()
    np.testing.assert_allclose(g.cpu().numpy(), g_ref, rtol=2e-4, atol=2e-4 * scale)


# ---------------------------------------------------------------------------------------
# Learned warm start and preconditioner
# ---------------------------------------------------------------------------------------
def _host_params(rng, I, H, O):
    return {"W1": rng.standard_normal((I, H)) * (2 / (I + H)) ** 0.5, "b1": rng.standard_normal(H) * 0.1,
            "W2": rng.standard_normal((H, H)) * (2 / (2 * H)) ** 0.5, "b2": rng.standard_normal(H) * 0.1,
            "W3": rng.standard_normal((H, O)) * (2 / (H + O)) ** 0.5, "b3": rng.standard_normal(O) * 0.1,
            "in_mu": rng.standard_normal(I), "in_sd": rng.uniform(0.5, 2, I),
            "out_mu": rng.standard_normal(O), "out_sd": rng.uniform(0.5, 2, O)}


def _pack(p, I, H, O):
    lay = pb.mlp_layout(I, H, O)
    buf = np.zeros(lay["total"], np.float32)
    for name in ["W1", "b1", "W2", "b2", "W3", "b3", "in_mu", "in_sd", "out_mu", "out_sd"]:
        v = np.asarray(p[name], np.float32).ravel()
        buf[lay[name]:lay[name] + v.size] = v
    return buf


def _f32(p):
    return {k: np.asarray(v, np.float32).astype(np.float64) for k, v in p.items()}


def test_mlp_forward_grad_adam_vs_oracle(h):
    from oracle import precond as opc
    I, H, O, B = 10, 256, 129, 64
    r = np.random.default_rng(0)
    p = _host_params(r, I, H, O)
    buf = dev(_pack(p, I, H, O))
    assert pb.precond_mlp_size(I, H, O) == buf.numel()
    psis = r.standard_normal((B, I))
    T = r.standard_normal((B, O)).astype(np.float32)
    Y = pb.precond_mlp_forward(h, buf, I, H, O, dev(psis))
    Yb = pb.precond_mlp_forward(h, buf, I, H, O, dev(psis), bf16=True)
    loss, grad = pb.precond_mlp_grad(h, buf, I, H, O, dev(psis), dev(T))
    torch.cuda.synchronize()
    pf = _f32(p)
    y_ref, _ = opc.mlp_forward(pf, psis)
    np.testing.assert_allclose(Y.cpu().numpy(), y_ref, rtol=1e-4, atol=1e-4)
    # BF16 operands: each product term carries about 2^-8 relative error
    assert np.abs(Yb.cpu().numpy() - y_ref).max() < 0.05 * np.abs(y_ref).max()
    l_ref, g_ref = opc.mlp_grad(pf, psis, T.astype(np.float64))
    np.testing.assert_allclose(loss.item(), l_ref, rtol=1e-4)
    lay = pb.mlp_layout(I, H, O)
    gn = grad.cpu().numpy()
    for name in ["W1", "b1", "W2", "b2", "W3", "b3"]:
        got = gn[lay[name]:lay[name] + g_ref[name].size].reshape(g_ref[name].shape)
        np.testing.assert_allclose(got, g_ref[name], rtol=2e-3, atol=2e-4 * np.abs(g_ref[name]).max())
    # one Adam step from zero moments
    adam = torch.zeros(2 * lay["trainable"], dtype=torch.float32, device="cuda")
    pb.precond_mlp_train(h, buf, adam, I, H, O, dev(psis), dev(T), 1, 0, 1e-3)
    torch.cuda.synchronize()
    after = buf.cpu().numpy()
    for name in ["W3", "b1"]:
        new, _, _ = opc.adam_step(pf[name], g_ref[name], 0 * g_ref[name], 0 * g_ref[name], 1, 1e-3)
        got = after[lay[name]:lay[name] + new.size].reshape(new.shape)
        np.testing.assert_allclose(got, new, rtol=1e-4, atol=2e-6)


def test_mlp_init_constants_and_training_reduces_loss(h):
    I, H, O, N = 4, 64, 9, 256
    r = np.random.default_rng(1)
    psis = r.standard_normal((N, I)) * [1, 2, 3, 4] + [0, 1, 2, 3]
    T = np.column_stack([np.sin(psis @ r.standard_normal(I)) for _ in range(O)]).astype(np.float32)
    buf = torch.zeros(pb.precond_mlp_size(I, H, O), dtype=torch.float32, device="cuda")
    pb.precond_mlp_init(h, buf, I, H, O, dev(psis), dev(T), seed=3)
    torch.cuda.synchronize()
    lay = pb.mlp_layout(I, H, O)
    got = buf.cpu().numpy()
    np.testing.assert_allclose(got[lay["in_mu"]:lay["in_mu"] + I], psis.mean(0), rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(got[lay["in_sd"]:lay["in_sd"] + I], psis.std(0), rtol=1e-4)
    np.testing.assert_allclose(got[lay["out_mu"]:lay["out_mu"] + O], T.mean(0), rtol=1e-4, atol=1e-5)
    w2 = got[lay["W2"]:lay["W2"] + H * H]
    assert abs(w2.std() - (1.0 / H) ** 0.5) < 0.1 * (1.0 / H) ** 0.5
    adam = torch.zeros(2 * lay["trainable"], dtype=torch.float32, device="cuda")
    trace = torch.zeros(400, dtype=torch.float32, device="cuda")
    pb.precond_mlp_train(h, buf, adam, I, H, O, dev(psis), dev(T), 400, 0, 3e-3, loss_trace=trace)
    torch.cuda.synchronize()
    tr = trace.cpu().numpy()
    assert tr[-1] < 0.3 * tr[0] and np.all(np.isfinite(tr))


def test_basis_orthonormal_and_ritz_values_interlace(h):
    n, d, k = 1500, 2, 32
    X, psi = problem(n, d, seed=11, lam=0.05, ell=(0.2, 0.3))
    U, ritz = pb.precond_build_basis(h, dev(X), dev(psi), k)
    torch.cuda.synchronize()
    Un = U.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(Un.T @ Un, np.eye(k), atol=1e-4)
    lam = np.linalg.eigvalsh(ogp.kernel_matrix(X, psi))[::-1]
    rz = ritz.cpu().numpy()
    # Cauchy interlacing: the j-th Ritz value lies below the j-th eigenvalue
    assert np.all(rz <= lam[:k] * (1 + 1e-5))
    np.testing.assert_allclose(rz[:4], lam[:4], rtol=1e-3)
    assert np.all(np.diff(rz) <= 1e-9 * rz[0])


def test_galerkin_targets_vs_oracle(h):
    from oracle import precond as opc
    n, d, k = 700, 3, 16
    X, psi0 = problem(n, d, seed=5, lam=0.1)
    y = np.random.default_rng(2).standard_normal(n).astype(np.float32)
    U, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((n, k)))
    U32 = U.astype(np.float32)
    psis = np.stack([psi0 + 0.1 * np.random.default_rng(i).standard_normal(d + 2) for i in range(3)])
    T = pb.precond_targets(h, dev(X), dev(y), colm(U32), dev(psis))
    torch.cuda.synchronize()
    got = T.cpu().numpy()
    for i in range(3):
        ref = opc.galerkin_targets(X, psis[i], y, U32.astype(np.float64))
        np.testing.assert_allclose(got[i], ref, rtol=2e-4, atol=2e-4 * np.abs(ref[:k]).max())


def test_learned_preconditioner_gains_and_keeps_the_gradient(h):
    # a small end-to-end run: basis at the reference psi, targets for psi's around it, a
    # trained network; at new psi's the preconditioned solves need fewer iterations and the
    # converged gradient is the same as without preconditioning
    n, d, k, nr = 4096, 2, 64, 8
    X, psi0 = problem(n, d, seed=21, lam=0.01, ell=(0.15, 0.25))
    y = workloads.gaussian_matrix(n, 1, seed=4)[:, 0]
    Xd, yd = dev(X), dev(y)
    U, ritz = pb.precond_build_basis(h, Xd, dev(psi0), k)
    r = np.random.default_rng(7)
    psis = psi0 + 0.05 * r.standard_normal((48, d + 2))
    T = pb.precond_targets(h, Xd, yd, U, dev(psis))
    I, H, O = d + 2, 128, 2 * k + 1
    prm = torch.zeros(pb.precond_mlp_size(I, H, O), dtype=torch.float32, device="cuda")
    pb.precond_mlp_init(h, prm, I, H, O, dev(psis), T, seed=1)
    adam = torch.zeros(2 * pb.mlp_layout(I, H, O)["trainable"], dtype=torch.float32, device="cuda")
    pb.precond_mlp_train(h, prm, adam, I, H, O, dev(psis), T, 600, 0, 2e-3)
    R = workloads.gaussian_matrix(n, nr, seed=9)
    params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=5000)
    its_plain, its_pc = [], []
    for j in range(3):
        psi_t = dev(psi0 + 0.05 * np.random.default_rng(100 + j).standard_normal(d + 2))
        coef = pb.precond_from_mlp(h, prm, I, H, O, psi_t, k)
        pc = pb.make_precond(U, coef)
        g0, s0 = pb.gp_stoch_grad(h, Xd, psi_t, yd, params, R=colm(R))
        g1, s1 = pb.gp_stoch_grad_pc(h, Xd, psi_t, yd, params, pc, R=colm(R))
        torch.cuda.synchronize()
        its_plain.append(max(s["iters"] for s in pb.decode_stats(s0)))
        its_pc.append(max(s["iters"] for s in pb.decode_stats(s1)))
        a, b = g0.cpu().numpy(), g1.cpu().numpy()
        np.testing.assert_allclose(b, a, rtol=1e-3, atol=1e-4 * np.abs(a).max())
    assert max(its_pc) < 0.6 * min(its_plain), (its_pc, its_plain)


# ---------------------------------------------------------------------------------------
# SGLD protocol: exact subset gradient, MAP and preconditioner M (Sec. 5)
# ---------------------------------------------------------------------------------------
def test_protocol_exact_gradient_vs_oracle(h):
    from paper_1501_05427_amd import protocol
    n, d = 300, 2
    X, psi = problem(n, d, seed=77, lam=0.1, ell=(0.2, 0.5))
    K = ogp.kernel_matrix(X, psi)
    y = (np.linalg.cholesky(K) @ np.random.default_rng(7).standard_normal(n)).astype(np.float32)
    g = protocol.exact_gradient(h, dev(X), dev(y), psi)
    ref = ogp.exact_gradient(X, psi, y.astype(np.float64))
    np.testing.assert_allclose(g, ref, rtol=1e-4, atol=1e-4 * np.abs(ref).max())


def test_reference_gradient_on_subsample_4096_vs_oracle(h):
    # the reference gradient of the equal-error comparison (converged solves averaged over
    # Gaussian probe batches) on the first 4096 points of the n = 65536, d = 8 workload,
    # against the oracle's Cholesky gradient of the same points: every component within
    # 3 standard errors of the batch mean (plus the 1e-6 CG tolerance scaled by |g|)
    from paper_1501_05427_amd import protocol
    w = workloads.rff_gp(n=65536, d=8, seed=2)
    X, psi, y = w["X"][:4096], w["psi"], w["y"][:4096]
    mean, se = protocol.probe_mean_gradient(h, dev(X), dev(y), psi, batches=16, probes=31)
    ref = ogp.exact_gradient(X.astype(np.float64), psi, y.astype(np.float64))
    assert np.all(np.isfinite(se)) and np.all(se > 0)
    tol = 3.0 * se + 1e-5 * np.abs(ref).max()
    assert np.all(np.abs(mean - ref) <= tol), (mean, ref, se)
    # and the noise is the Hutchinson noise, not a bias: the standard error is a small
    # fraction of the gradient's norm
    assert np.linalg.norm(se) < 0.1 * np.linalg.norm(ref)


def test_protocol_subset_map_and_preconditioner_vs_oracle(h):
    from oracle import diagnostics as od
    from paper_1501_05427_amd import protocol
    n, d = 400, 2
    X, psi = problem(n, d, seed=78, lam=0.1, ell=(0.2, 0.5))
    K = ogp.kernel_matrix(X, psi)
    y = (np.linalg.cholesky(K) @ np.random.default_rng(8).standard_normal(n)).astype(np.float32)
    prior = {"kind": 1, "a": np.zeros(d + 2), "b": np.full(d + 2, 3.0)}
    psi_map, M, L = protocol.sgld_preconditioner(h, X, y, psi + 0.1, prior, n_sub=200, seed=5)
    idx = np.sort(np.random.default_rng(5).choice(n, size=200, replace=False))
    ref_map, ref_A = od.subset_map(X[idx], y[idx].astype(np.float64), psi + 0.1, 1, prior["a"], prior["b"])
    np.testing.assert_allclose(psi_map, ref_map, atol=2e-3)
    ref_M = np.linalg.inv(ref_A)
    np.testing.assert_allclose(M, ref_M, rtol=2e-2, atol=2e-2 * np.abs(ref_M).max())
    np.testing.assert_allclose(L @ L.T, M, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------------------------------
# Batched SGLD (captured graphs) and the autotuner
# ---------------------------------------------------------------------------------------
def _batch_problems(specs, nr):
    out = []
    for i, (n, d) in enumerate(specs):
        w = workloads.rff_gp(n=n, d=d, seed=100 + i, n_features=256)
        out.append({"X": dev(w["X"]), "y": dev(w["y"]), "psi": dev(w["psi"]),
                    "M_chol": dev(np.eye(d + 2) / np.sqrt(n)),
                    "prior": (1, dev(np.zeros(d + 2)), dev(np.full(d + 2, 3.0)))})
    return out


@pytest.mark.parametrize("prec,refresh,ipg,T,period", [(pb.GP_FP32, 0, 4, 5, 2), (pb.GP_BF16_SPLIT_V, 3, 4, 5, 2),
                                                       (pb.GP_FP32, 0, 2, 8, 3)])
def test_batch_reproduces_unbatched_calls(prec, refresh, ipg, T, period):
    # each chain of the batch must follow exactly the trajectory of the unbatched calls with
    # the same Philox keys and counters (autotune off: identical product shapes); also with
    # BF16 products and residual replacement, whose decisions are taken on the device inside
    # the captured iteration graph.  The last case takes two iterations per replay and a
    # redraw every third step, so the steps need different replay counts and the replays
    # queued from the previous step of the same kind are sometimes too many, sometimes too few
    specs = [(300, 2), (700, 4), (1500, 8), (2049, 16), (4000, 3)]
    nr, eps = 16, 1e-3
    probs = _batch_problems(specs, nr)
    params = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=2000, rng_stream=3,
                            prec=prec, refresh=refresh)
    ref = [{k: (v.clone() if torch.is_tensor(v) else v) for k, v in p.items()} for p in probs]
    batch = pb.Batch(probs, nr, params, seed=900, probe_period=period, iters_per_graph=ipg,
                     autotune=False, streams=3)
    for t in range(T):
        batch.step(t, eps)
    torch.cuda.synchronize()
    st = batch.stats()
    assert st["eager_steps"] == 1 and st["graph_steps"] == T - 1 and st["captures"] == 4, st
    assert st["iteration_graphs"] >= T - 1, st
    if prec != pb.GP_FP32:
        # the n = 4000, d = 3 chain's split-V solve breaks down (BF16 rounding leaves its K
        # indefinite): the batch redoes that chain's step in FP32, as the unbatched call does
        assert st["fp32_reruns"] >= 1, st
    for i, ((n, d), p) in enumerate(zip(specs, ref)):
        hi = pb.Handle(0, seed=900 + i)
        S_warm = torch.zeros((1 + nr, n), dtype=torch.float64, device="cuda").t()
        R = pb.colmajor(n, nr)
        g = torch.zeros(d + 2, dtype=torch.float64, device="cuda")
        kind, a, b = p["prior"]
        for t in range(T):
            if t % period == 0:
                pb.gp_draw_probes(hi, n, nr, pb.PROBE_GAUSSIAN, params.rng_stream, t // period, R=R)
                S_warm[:, 1:].zero_()
            params.rng_counter = t
            pb.gp_stoch_grad(hi, p["X"], p["psi"], p["y"], params, R=R, S_warm=S_warm, g=g)
            pb.sgld_step(hi, p["psi"], g, eps, rng_stream=params.rng_stream, rng_counter=t, prior_kind=kind,
                         prior_a=a, prior_b=b, M_chol=p["M_chol"])
        torch.cuda.synchronize()
        ch = batch.chains[i]
        np.testing.assert_array_equal(ch["psi"].cpu().numpy(), p["psi"].cpu().numpy(), err_msg=f"chain {i}")
        np.testing.assert_array_equal(ch["g"].cpu().numpy(), g.cpu().numpy(), err_msg=f"chain {i}")
        np.testing.assert_array_equal(ch["R"].cpu().numpy(), R.cpu().numpy(), err_msg=f"chain {i}")
    batch.close()


def test_autotuned_products_match_oracle():
    h2 = pb.Handle(0, seed=5)
    pb.gp_autotune(h2, 1)
    for n, d, m in [(3000, 8, 32), (2049, 16, 17), (5000, 2, 5)]:
        X, psi = problem(n, d, seed=n + d)
        V = np.random.default_rng(m).standard_normal((n, m)).astype(np.float32)
        out = pb.gp_kmv(h2, dev(X), dev(psi), colm(V))
        out2 = pb.gp_kmv(h2, dev(X), dev(psi), colm(V))  # the cached shape
        torch.cuda.synchronize()
        ref = ogp.kmv(X, psi, V)
        assert colwise_rel(out.cpu().numpy(), ref).max() <= 1e-5
        assert colwise_rel(out2.cpu().numpy(), ref).max() <= 1e-5
        split = pb.gp_autotune_split(h2, n, d, m)
        assert 1 <= split <= 64


@pytest.mark.parametrize("prec,refresh", [(pb.GP_BF16_SPLIT_KV, 0), (pb.GP_BF16_SPLIT_V, 3)])
def test_batch_learned_bf16_reproduces_unbatched_calls(prec, refresh):
    # chains with their own basis and trained network, BF16 products: the batch evaluates
    # the network at each chain's psi inside its captured set-up graph; with V split, the
    # preconditioned solves of a chain that breaks down are redone in FP32 over the same
    # preconditioner
    specs = [(1500, 2), (2500, 4), (3000, 8)]
    nr, T, period, eps, k, H = 16, 4, 2, 1e-3, 16, 64
    probs = _batch_problems(specs, nr)
    hs = pb.Handle(0, seed=1)
    for i, p in enumerate(probs):
        d = p["X"].shape[1]
        U, _ = pb.precond_build_basis(hs, p["X"], p["psi"], k)
        psis = p["psi"][None, :] + 0.03 * torch.from_numpy(
            np.random.default_rng(i).standard_normal((32, d + 2))).cuda()
        Tg = pb.precond_targets(hs, p["X"], p["y"], U, psis)
        I, O = d + 2, 2 * k + 1
        prm = torch.zeros(pb.precond_mlp_size(I, H, O), dtype=torch.float32, device="cuda")
        pb.precond_mlp_init(hs, prm, I, H, O, psis, Tg, seed=3)
        adam = torch.zeros(2 * pb.mlp_layout(I, H, O)["trainable"], dtype=torch.float32, device="cuda")
        pb.precond_mlp_train(hs, prm, adam, I, H, O, psis, Tg, 200, 0, 2e-3)
        p["learned"] = {"mlp": prm, "hidden": H, "U": U,
                        "coef": torch.zeros(k + 1, dtype=torch.float64, device="cuda")}
    torch.cuda.synchronize()
    params = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=2000, rng_stream=3)
    params.prec, params.refresh = prec, refresh
    psi0 = [p["psi"].clone() for p in probs]
    batch = pb.Batch(probs, nr, params, seed=900, probe_period=period, iters_per_graph=4,
                     autotune=False, streams=2)
    for t in range(T):
        batch.step(t, eps)
    torch.cuda.synchronize()
    if prec == pb.GP_BF16_SPLIT_V:
        # some of these preconditioned split-V solves break down (3 chain steps are redone)
        assert batch.stats()["fp32_reruns"] >= 1
    for i, ((n, d), p) in enumerate(zip(specs, probs)):
        hi = pb.Handle(0, seed=900 + i)
        psi = psi0[i]
        S_warm = torch.zeros((1 + nr, n), dtype=torch.float64, device="cuda").t()
        R = pb.colmajor(n, nr)
        g = torch.zeros(d + 2, dtype=torch.float64, device="cuda")
        coef = torch.zeros(k + 1, dtype=torch.float64, device="cuda")
        pc = pb.make_precond(p["learned"]["U"], coef)
        kind, a, b = p["prior"]
        for t in range(T):
            if t % period == 0:
                pb.gp_draw_probes(hi, n, nr, pb.PROBE_GAUSSIAN, params.rng_stream, t // period, R=R)
                S_warm[:, 1:].zero_()
            params.rng_counter = t
            pb.precond_from_mlp(hi, p["learned"]["mlp"], d + 2, H, 2 * k + 1, psi, k, coef=coef)
            pb.gp_stoch_grad_pc(hi, p["X"], psi, p["y"], params, pc, R=R, S_warm=S_warm, g=g)
            pb.sgld_step(hi, psi, g, eps, rng_stream=params.rng_stream, rng_counter=t, prior_kind=kind,
                         prior_a=a, prior_b=b, M_chol=p["M_chol"])
        torch.cuda.synchronize()
        ch = batch.chains[i]
        np.testing.assert_array_equal(ch["psi"].cpu().numpy(), psi.cpu().numpy(), err_msg=f"chain {i}")
        np.testing.assert_array_equal(ch["g"].cpu().numpy(), g.cpu().numpy(), err_msg=f"chain {i}")
    batch.close()


@pytest.mark.parametrize("prec", [pb.GP_BF16_SPLIT_KV])
def test_bf16_gradient_reduction_matches_fp32(h, prec):
    # the BF16 modes also take the gradient's G tiles from split BF16 operands; with
    # converged solves the estimate must agree with the FP32 path to the solve accuracy of
    # the mode (split K+V: ~3e-5 on the 4096-point report) plus the G rounding (~2^-17)
    n, d, nr = 3000, 4, 31
    X, psi = problem(n, d, seed=31, lam=0.1, ell=(0.2, 0.5))
    y = workloads.gaussian_matrix(n, 1, seed=2)[:, 0]
    R = workloads.gaussian_matrix(n, nr, seed=3)
    params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=3000)
    g32, st32 = pb.gp_stoch_grad(h, dev(X), dev(psi), dev(y), params, R=colm(R))
    params.prec = prec
    g16, st16 = pb.gp_stoch_grad(h, dev(X), dev(psi), dev(y), params, R=colm(R))
    torch.cuda.synchronize()
    assert not any(s["flags"] for s in pb.decode_stats(st16))
    a, b = g32.cpu().numpy(), g16.cpu().numpy()
    np.testing.assert_allclose(b, a, rtol=1e-3, atol=1e-3 * np.abs(a).max())


def test_dkmv_matches_finite_differences_of_kmv(h):
    # an independent route to dK/dpsi_j V: central differences of the product itself
    n, d, m, step = 777, 3, 17, 1e-3
    X, psi = problem(n, d, seed=41)
    V = np.random.default_rng(2).standard_normal((n, m)).astype(np.float32)
    dk = pb.gp_dkmv(h, dev(X), dev(psi), colm(V))
    kv = pb.gp_kmv(h, dev(X), dev(psi), colm(V)).cpu().numpy()
    torch.cuda.synchronize()
    dk = dk.cpu().numpy()
    for j in range(d + 2):
        e = np.zeros(d + 2)
        e[j] = step
        up = pb.gp_kmv(h, dev(X), dev(psi + e), colm(V)).cpu().numpy()
        dn = pb.gp_kmv(h, dev(X), dev(psi - e), colm(V)).cpu().numpy()
        fd = (up.astype(np.float64) - dn) / (2 * step)
        err = np.linalg.norm(fd - dk[j].T, axis=0)
        bound = 2e-3 * np.linalg.norm(dk[j].T, axis=0) + 1e-3 * np.linalg.norm(kv, axis=0)
        assert np.all(err <= bound), (j, (err / bound).max())

