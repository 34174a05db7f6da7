"""Product shapes: the symmetric FP32 product against split-K and the oracle, the shape pins,
and the autotuner's cache file, through the C ABI.

Tolerance as for every FP32 covariance product: per column ||out - ref||_2 / ||ref||_2 <= 1e-5
against the FP64 oracle.  The two shapes sum the same products in different orders, so they
agree to FP32 rounding, not bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle import cg as ocg
from oracle import gp as ogp
from oracle import rng as orng
from oracle import stoch_grad as osg
from oracle import ulisse as oul

pytestmark = pytest.mark.gpu

pb = pytest.importorskip("paper_1501_05427_amd.binding")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


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


def _safe_q(K, b, target_l):
    """q whose threshold q sqrt(n) sits midway (log scale) between the running minimum of the
    residual norms before an iteration l >= target_l and the norm at l, with a clear gap, so
    FP32 and FP64 runs of system 0 take the same l."""
    norms = []
    for i, s, e, dl in ocg.cg_iterates(lambda v: K @ v, b, np.zeros_like(b)):
        norms.append(np.linalg.norm(e))
        if i >= target_l and min(norms[:-1]) > 1.5 * norms[-1]:
            return np.sqrt(min(norms[:-1]) * norms[-1]) / np.sqrt(len(b))
        assert i < 200


def colwise_rel(out, ref):
    out = np.asarray(out, dtype=np.float64)
    return np.linalg.norm(out - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)


# n from the smallest the symmetric product takes (n_pad = 2048, 8 row tiles) up, ragged
# tails inside the last row tile and the last column chunk; one and two MFMA blocks, with
# and without the VALU column
SYM_CASES = [(1793, 3, 17), (2049, 8, 16), (3000, 5, 17), (4100, 8, 32), (2300, 2, 33),
             (6000, 8, 32), (9000, 1, 16), (2600, 16, 32), (3100, 12, 17), (2049, 16, 33),
             # under 16 right-hand sides: one zero-padded MFMA block against the VALU contraction
             (2049, 8, 1), (3000, 5, 5), (4100, 3, 12), (2600, 16, 4), (1900, 2, 15)]


@pytest.mark.parametrize("n,d,m", SYM_CASES)
def test_symmetric_and_split_k_products_match_oracle(n, d, m):
    h = pb.Handle(0, seed=7)
    X, psi = problem(n, d, seed=3 * n + d)
    V = np.random.default_rng(m + n).standard_normal((n, m)).astype(np.float32)
    ref = ogp.kmv(X, psi, V)
    outs = {}
    for code in (pb.SHAPE_SYM, 2048):
        pb.gp_tune_set(h, n, d, m, code)
        got_code, split = pb.gp_tune_get(h, n, d, m)
        assert got_code == code and (split == 1 if code == pb.SHAPE_SYM else split >= 1)
        out = pb.gp_kmv(h, dev(X), dev(psi), colm(V))
        torch.cuda.synchronize()
        outs[code] = out.cpu().numpy().astype(np.float64)
        assert colwise_rel(outs[code], ref).max() <= 1e-5, code
    # the two differ by their rounding only: no tighter than the sum of the two bounds
    assert colwise_rel(outs[pb.SHAPE_SYM], outs[2048]).max() <= 2e-5


# the BF16 bound of the covariance products: per column, of || |K| |V| || (the rounding of one
# BF16 value, 2^-9, and of a hi + lo pair, about 2^-17, with margin), plus the FP32 term
BF16_BOUND = {pb.GP_BF16_SPLIT_V: 2.0 ** -8, pb.GP_BF16_SPLIT_KV: 6 * 2.0 ** -18}


@pytest.mark.parametrize("prec", [pb.GP_BF16_SPLIT_V, pb.GP_BF16_SPLIT_KV])
@pytest.mark.parametrize("n,d,m", [(2049, 8, 17), (3000, 5, 32), (4100, 2, 24), (6000, 8, 31), (2600, 16, 32)])
def test_symmetric_bf16_products_match_oracle_and_split_k(prec, n, d, m):
    # BF16 products (two MFMA blocks: 17 to 32 right-hand sides) through both shapes: each within the BF16 bound
    # of the oracle; the two use the same BF16 operands and differ in the order of their FP32
    # and FP64 sums only
    h = pb.Handle(0, seed=7)
    X, psi = problem(n, d, seed=5 * n + d)
    V = np.random.default_rng(m + 2 * n).standard_normal((n, m)).astype(np.float32)
    ref = ogp.kmv(X, psi, V)
    bound = (BF16_BOUND[prec] + 1e-6) * np.linalg.norm(
        np.abs(ogp.kernel_matrix(X, psi)) @ np.abs(V.astype(np.float64)), axis=0)
    outs = {}
    for code in (pb.SHAPE_SYM, 2048):
        pb.gp_tune_set(h, n, d, m, code, prec=prec)
        assert pb.gp_tune_get(h, n, d, m, prec=prec)[0] == code
        out = pb.gp_kmv(h, dev(X), dev(psi), colm(V), prec=prec)
        torch.cuda.synchronize()
        outs[code] = out.cpu().numpy().astype(np.float64)
        err = np.linalg.norm(outs[code] - ref, axis=0)
        assert np.all(err <= bound), (code, (err / bound).max())
    assert colwise_rel(outs[pb.SHAPE_SYM], outs[2048]).max() <= 2e-5


@pytest.mark.parametrize("prec", [pb.GP_FP32, pb.GP_BF16_SPLIT_KV])
def test_converged_solves_through_both_shapes_at_full_size(prec, capsys):
    # n = 33000 (n_pad 33024), 17 systems: the symmetric shape is the default there, in FP32
    # and in the BF16 modes.  Converged solves (CG to 1e-6 relative; BF16 with residual
    # replacement, k = 3) through it and through split-K: each solution's true residual
    # ||b - K s|| / ||b||, taken with an FP32 product of the solution, and the difference of
    # the two solutions are printed.  Both are bounded by 1e-3: far above the solve tolerance
    # times the conditioning and the FP32 evaluation error (1e-7 ||K|| ||s|| / ||b||, with
    # ||s|| / ||b|| ~ 15 here), far below what a wrong partial layout in the solver's product
    # would give.  A dense oracle of this size is out of reach; the oracle comparison of the
    # products is in the cases above.
    import workloads
    n, d, m = 33000, 8, 17
    h = pb.Handle(0, seed=11)
    w = workloads.rff_gp(n=n, d=d, seed=7, n_features=256)
    X, psi = dev(w["X"]), dev(w["psi"])
    B = np.column_stack([w["y"], workloads.gaussian_matrix(n, m - 1, seed=3)]).astype(np.float32)
    assert pb.gp_tune_get(h, n, d, m, prec=prec)[0] == pb.SHAPE_SYM
    params = pb.make_params(q=1e-12, rate=1e-9, eps=1e-6, eps_relative=1, max_iter=3000, prec=prec,
                            refresh=3 if prec != pb.GP_FP32 else 0)
    sol, res = {}, {}
    for code in (pb.SHAPE_SYM, 2048):
        pb.gp_tune_set(h, n, d, m, code, prec=prec)
        St, stats = pb.ulisse_solve(h, X, psi, colm(B), params)
        KS = pb.gp_kmv(h, X, psi, St.to(torch.float32))   # default FP32 product
        torch.cuda.synchronize()
        assert not any(s_["flags"] for s_ in pb.decode_stats(stats)), code
        sol[code] = St.cpu().numpy()
        res[code] = np.linalg.norm(B - KS.cpu().numpy().astype(np.float64), axis=0) / np.linalg.norm(B, axis=0)
    diff = colwise_rel(sol[pb.SHAPE_SYM], sol[2048]).max()
    with capsys.disabled():
        print(f"\n[shapes at n = 33000] mode {prec}: true residual max symmetric {res[pb.SHAPE_SYM].max():.2e}, "
              f"split-K {res[2048].max():.2e}; solutions differ by {diff:.2e}")
    assert res[pb.SHAPE_SYM].max() <= 1e-3 and res[2048].max() <= 1e-3
    assert diff <= 1e-3


def test_symmetric_product_is_refused_where_it_does_not_apply():
    h = pb.Handle(0, seed=7)
    for n, d, m, prec in [(1000, 4, 16, pb.GP_FP32),      # n_pad below 2048
                          (4000, 4, 48, pb.GP_FP32),      # three MFMA blocks
                          (4000, 4, 18, pb.GP_FP32),      # two VALU columns
                          (4000, 4, 16, pb.GP_BF16_SPLIT_KV),   # BF16: one MFMA block
                          (4000, 4, 48, pb.GP_BF16_SPLIT_V),    # BF16: three MFMA blocks
                          (4000, 4, 64, pb.GP_BF16_SPLIT_KV),   # BF16: four MFMA blocks
                          (215000, 8, 32, pb.GP_FP32)]:         # partials above 24 GiB
        with pytest.raises(RuntimeError, match="symmetric"):
            pb.gp_tune_set(h, n, d, m, pb.SHAPE_SYM, prec=prec)
    with pytest.raises(RuntimeError):
        pb.gp_tune_set(h, 4000, 4, 16, 2 ** 21)
    # the memory cap moves the default to split-K (host-only calls: nothing is allocated)
    assert pb.gp_tune_get(h, 212000, 8, 32)[0] == pb.SHAPE_SYM
    code, split = pb.gp_tune_get(h, 215000, 8, 32)
    assert code > 0 and split > 1
    # under 16 right-hand sides the FP32 default takes the padded symmetric product where
    # m + d >= 12 and n >= 16129, the VALU contraction elsewhere; the BF16 modes keep the latter
    for n, d, m, sym in [(16384, 8, 5, True), (16384, 8, 3, False), (16384, 2, 5, False), (16384, 2, 10, True),
                         (16128, 8, 5, False), (65536, 8, 1, False), (131072, 16, 1, True)]:
        assert (pb.gp_tune_get(h, n, d, m)[0] == pb.SHAPE_SYM) == sym, (n, d, m)
    assert pb.gp_tune_get(h, 65536, 8, 5, prec=pb.GP_BF16_SPLIT_KV)[0] != pb.SHAPE_SYM


@pytest.mark.parametrize("m", [17, 5])
def test_ulisse_draw_for_draw_through_the_symmetric_product(m):
    # the solver's products through the pinned symmetric shape (n = 2500: 10 row tiles; 17
    # systems: one MFMA block and the VALU column; 5 systems: one block padded with zero
    # columns), draw for draw against the oracle
    h = pb.Handle(0, seed=1234)
    n, d = 2500, 4
    X, psi = problem(n, d, seed=11, lam=0.3, ell=(0.2, 0.4))
    K = ogp.kernel_matrix(X, psi)
    Bm = np.random.default_rng(5).standard_normal((n, m)).astype(np.float32)
    pb.gp_tune_set(h, n, d, m, pb.SHAPE_SYM)
    q, eps, rate = _safe_q(K, Bm[:, 0].astype(np.float64), 3), 1e-6, 0.7
    params = pb.make_params(q=q, rate=rate, eps=eps, eps_relative=1, max_iter=300, two_track_first=1,
                            rng_stream=9, rng_counter=2)
    Scg = torch.zeros((m, n), dtype=torch.float64, device="cuda").t()
    St, stats = pb.ulisse_solve(h, dev(X), dev(psi), colm(Bm), params, S_cg=Scg)
    torch.cuda.synchronize()
    st_gpu = pb.decode_stats(stats)
    ref_St, ref_Scg, ref_stats = oul.solve_systems(
        lambda v: K @ v, Bm.astype(np.float64), None, q, rate, eps, 300, h.seed, 9, 2,
        two_track_first=True, eps_relative=True)
    for c in range(m):
        g, r = st_gpu[c], ref_stats[c]
        assert g["l"] == r["l"] and g["iters"] == r["iters"] and g["J_a"] == r["J"][0], (c, g, r)
        assert g["flags"] == r["flags"]
    assert colwise_rel(St.cpu().numpy(), ref_St).max() <= 2e-4
    assert colwise_rel(Scg.cpu().numpy(), ref_Scg).max() <= 2e-4


def test_stoch_grad_draw_for_draw_through_the_padded_symmetric_product():
    # y + 4 probes (5 systems) through the symmetric product with one zero-padded MFMA block,
    # the default of such products from n = 16129 at d = 8, pinned here at n = 2100; the
    # gradient draw for draw against the oracle (well-conditioned system, short CG paths, as
    # in the other draw-for-draw tests)
    h = pb.Handle(0, seed=4321)
    n, d, nr = 2100, 8, 4
    X, psi = problem(n, d, seed=2108, lam=1.0, ell=(0.1, 0.3))
    K = ogp.kernel_matrix(X, psi)
    y = (np.linalg.cholesky(K) @ np.random.default_rng(1).standard_normal(n)).astype(np.float32)
    pb.gp_tune_set(h, n, d, 1 + nr, pb.SHAPE_SYM)
    assert pb.gp_tune_get(h, n, d, 1 + nr)[0] == pb.SHAPE_SYM
    stream, counter = 5, 9
    R = orng.probes(h.seed, stream, counter, n, nr, 0).astype(np.float32)
    q, eps, rate = _safe_q(K, y.astype(np.float64), 2), 1e-6, 1.0
    params = pb.make_params(q=q, rate=rate, eps=eps, eps_relative=1, max_iter=300,
                            rng_stream=stream, rng_counter=counter)
    g, stats = pb.gp_stoch_grad(h, dev(X), dev(psi), dev(y), params, n_probes=nr)
    torch.cuda.synchronize()
    g_ref, _, _, ref_stats = osg.stoch_grad(X, psi, y, R, q, rate, eps, 300, h.seed, stream, counter,
                                            eps_relative=True)
    st_gpu = pb.decode_stats(stats)
    for c in range(nr + 1):
        assert ref_stats[c]["iters"] <= 7
        assert (st_gpu[c]["l"], st_gpu[c]["iters"]) == (ref_stats[c]["l"], ref_stats[c]["iters"]), c
    got = g.cpu().numpy()
    np.testing.assert_allclose(got, g_ref, rtol=2e-4, atol=2e-4 * np.abs(g_ref).max())


def test_tuning_cache_round_trip(tmp_path):
    h = pb.Handle(0, seed=3)
    pb.gp_autotune(h, 1)
    shapes = [(3000, 8, 32), (4096, 4, 17), (2000, 2, 5)]
    for n, d, m in shapes:
        assert pb.gp_tune_get(h, n, d, m)[0] == -1  # not timed yet
        X, psi = problem(n, d, seed=n)
        V = np.random.default_rng(1).standard_normal((n, m)).astype(np.float32)
        pb.gp_kmv(h, dev(X), dev(psi), colm(V))
    torch.cuda.synchronize()
    codes = {s: pb.gp_tune_get(h, *s) for s in shapes}
    assert all(c >= 0 for c, _ in codes.values())
    path = tmp_path / "shapes.txt"
    pb.gp_tune_save(h, path)
    lines = path.read_text().splitlines()
    assert lines[0] == "ulisse_gp shape cache v1" and len(lines) == 1 + len(shapes)

    h2 = pb.Handle(0, seed=3)
    pb.gp_autotune(h2, 1)
    pb.gp_tune_load(h2, path)
    for s in shapes:
        assert pb.gp_tune_get(h2, *s) == codes[s]
    # a pin wins over the loaded entry and its removal restores it
    n, d, m = shapes[0]
    pb.gp_tune_set(h2, n, d, m, 256)
    assert pb.gp_tune_get(h2, n, d, m)[0] == 256
    pb.gp_tune_set(h2, n, d, m, -1)
    assert pb.gp_tune_get(h2, n, d, m) == codes[shapes[0]]
    # with the autotuner off the loaded entries are not used: the default is back
    pb.gp_autotune(h2, 0)
    assert pb.gp_tune_get(h2, 2000, 2, 5) == pb.gp_tune_get(pb.Handle(0, seed=3), 2000, 2, 5)

    # a malformed file is refused as a whole and leaves the entries as they were
    bad = tmp_path / "bad.txt"
    bad.write_text("ulisse_gp shape cache v1\n4096 4 20 0 0\n4096 4 20 zero 0\n")
    h3 = pb.Handle(0, seed=3)
    pb.gp_autotune(h3, 1)
    with pytest.raises(RuntimeError, match="line 3"):
        pb.gp_tune_load(h3, bad)
    assert pb.gp_tune_get(h3, 4096, 4, 17)[0] == -1
    (tmp_path / "nohdr.txt").write_text("4096 4 20 0 0\n")
    with pytest.raises(RuntimeError, match="not a tuning cache"):
        pb.gp_tune_load(h3, tmp_path / "nohdr.txt")
