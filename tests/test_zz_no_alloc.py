"""gp_kmv_noalloc (the covariance product for callers that cannot allocate: its buffers
live in the library's fixed device scratch) against gp_kmv, through the C ABI, on two
calls in a row with the second one smaller, and against the FP64 oracle.  Tolerance: the
FP32 product bound of 1e-5 per column against the oracle (Sec. 3, the CMVP) and against
gp_kmv (the two may use different split-K chunkings, so their sums are not bitwise
equal); the split K + V mode against its own rounding bound."""
import numpy as np
import pytest
import torch

from oracle import gp as ogp

pytestmark = pytest.mark.gpu

pb = pytest.importorskip("paper_1501_05427_amd.binding")


@pytest.fixture(autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def colm(a):
    return dev(np.ascontiguousarray(np.asarray(a).T)).t()


def colwise_rel(out, ref):
    out = np.asarray(out, dtype=np.float64)
    return np.linalg.norm(out - ref, axis=0) / np.maximum(np.linalg.norm(ref, axis=0), 1e-300)


def case(n, d, m, seed):
    r = np.random.default_rng(seed)
    X = r.uniform(size=(n, d)).astype(np.float32)
    psi = np.concatenate([[np.log(1.1)], np.log(r.uniform(0.3, 0.8, d)), [np.log(0.1)]])
    V = r.standard_normal((n, m)).astype(np.float32)
    return X, psi, V


@pytest.mark.parametrize("prec", [pb.GP_FP32, pb.GP_BF16_SPLIT_KV])
def test_noalloc_kmv_two_calls_match_gp_kmv_and_oracle(prec):
    h = pb.Handle(0, seed=5)
    # first call larger (several row tiles, ragged n, split-K), second call smaller: the
    # scratch keeps the first call's contents, which the second must not depend on
    for n, d, m, seed in [(5000, 8, 33, 1), (777, 3, 17, 2)]:
        X, psi, V = case(n, d, m, seed)
        Xd, psid, Vd = dev(X), dev(psi), colm(V)
        out = pb.colmajor(n, m)
        pb.gp_kmv_noalloc(h, Xd, psid, Vd, out, prec=prec)
        ref_gpu = pb.gp_kmv(h, Xd, psid, Vd, prec=prec)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.all(np.isfinite(got))
        ref = ogp.kmv(X, psi, V)
        if prec == pb.GP_FP32:
            assert colwise_rel(got, ref).max() <= 1e-5
            assert colwise_rel(got, ref_gpu.cpu().numpy().astype(np.float64)).max() <= 1e-5
        else:
            # split K + V: 6 2^-18 of || |K| |V| || per column (plus the FP32 term), the bound
            # of the BF16 product tests
            absprod = np.linalg.norm(np.abs(ogp.kernel_matrix(X, psi)) @ np.abs(V.astype(np.float64)), axis=0)
            bound = (6 * 2.0 ** -18 + 1e-6) * absprod
            assert np.all(np.linalg.norm(got - ref, axis=0) <= bound)
            assert np.all(np.linalg.norm(got - ref_gpu.cpu().numpy(), axis=0) <= 2 * bound)
    h.close()


def test_noalloc_kmv_full_size_and_rejection():
    # n = 65536, d = 8, m = 32 (the benchmark's product): fits the 32 MiB scratch with a
    # smaller split-K than gp_kmv; sampled rows against the oracle.  m = 64 does not fit.
    import workloads
    h = pb.Handle(0, seed=6)
    w = workloads.rff_gp(n=65536, d=8, seed=2)
    X, psi = w["X"], w["psi"]
    V = workloads.gaussian_matrix(65536, 32, seed=11)
    out = pb.colmajor(65536, 32)
    pb.gp_kmv_noalloc(h, dev(X), dev(psi), colm(V), out)
    torch.cuda.synchronize()
    rows = np.sort(np.random.default_rng(0).choice(65536, 32, replace=False))
    ref = ogp.kmv(X, psi, V, rows=rows)
    assert colwise_rel(out.cpu().numpy()[rows], ref).max() <= 1e-5
    V64 = torch.zeros((64, 65536), dtype=torch.float32, device="cuda").t()
    out64 = pb.colmajor(65536, 64)
    with pytest.raises(pb.GPError) as ei:
        pb.gp_kmv_noalloc(h, dev(X), dev(psi), V64, out64)
    assert ei.value.status == pb.GP_EINVAL and "scratch" in str(ei.value)
    h.close()
