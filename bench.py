"""Benchmark of the hot path: one SGLD step = one unbiased gradient estimate (ULISSE solves
for y and 31 Gaussian probes, fused gradient reduction) + the SGLD update, on the
n = 65536, d = 8 synthetic GP workload (32 right-hand sides).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline] [--no-batched]

Prints one JSON line.  `value` is gradient estimates per second of the plain FP32 path over
the K timed steps, with inputs resident in HBM, under the protocol: fresh probes every
step, psi starting at the truth, the y system warm-started from its last CG iterate,
q = 1, rate 1, step size 1e-3, SGLD preconditioner M from the MAP of a 500-point subset
(the paper's recipe, Sec. 5).  From the same saved state and with the same draws the line
also carries: the paper's protocol (probes redrawn every 20 steps), BF16 products (V split
hi + lo by default, `--bf16-mode kv` splits K too) with residual replacement, the learned preconditioner (trained on the states of
plain-solver SGLD chains) with and without its warm start U c, the Galerkin
preconditioner on the same basis without learning (fixed at the MAP, or recomputed at
every step), an equal-error comparison at a state of the chain (the paper's error measure,
Sec. 4.2), K.V throughput per arithmetic mode, the batched 64-GP form and the CPU oracle.

The roofline object is for the dominant kernel, the covariance product (kmv): algorithmic
flops per launch n^2 (3d + 2m) divided by its average launch time, taken from hipEvents
recorded by the library on the launch stream during the timed steps.  HBM traffic per
launch comes from the committed rocprofv3 counter summary if it was taken on the current
kmv source, else null.

    python bench.py --profile-kmv     a short run for rocprofv3: 5 kmv launches at the
                                      same shape plus a 1 GiB copy (counter calibration)
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N, D, NPROBES = 65536, 8, 31
PROBE_PERIOD = 20
LEARN_JITTER = 0.03   # batched learned leg: spread of each GP's training psi's around its start
M = 1 + NPROBES
WORKLOAD = "rff_n65536_d8_m32"
VALU_FP32_PEAK_TFLOPS = 157.3   # 256 CU x 2.4 GHz x 256 flop/CU/clk (datasheet FP32 vector)
KMV_SRC = os.path.join(ROOT, "paper_1501_05427_amd", "csrc", "kmv.hip")
PMC_SUMMARY = os.path.join(ROOT, "profiles", "kmv_rff_n65536_d8_m32_pmc.txt")


def kmv_flops(n, d, m):
    return float(n) * n * (3 * d + 2 * m)


def kmv_source_hash():
    return hashlib.sha256(open(KMV_SRC, "rb").read()).hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per kmv launch from the committed counter summary (None if stale/absent)."""
    if not os.path.exists(PMC_SUMMARY):
        return None
    vals = {}
    for line in open(PMC_SUMMARY):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kmv_source_sha256_16") != kmv_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(X, psi, passes_per_estimate, budget_rows=(768, 256)):
    """The FP64 oracle on a bounded sample of the same workload, scaled to estimates/s.

    Times oracle.gp.kmv on `budget_rows[0]` rows (all 65536 columns, 32 right-hand sides)
    and the oracle's gradient assembly on `budget_rows[1]` rows (the P = 10 derivative
    blocks times the solutions); both scale linearly in the number of rows.  One estimate
    costs `passes_per_estimate` full products plus one full assembly.
    """
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import gp as ogp
    r = np.random.default_rng(0)
    V = r.standard_normal((N, M))
    rows_k = np.arange(budget_rows[0])
    t0 = time.perf_counter()
    ogp.kmv(X, psi, V, rows=rows_k)
    t_kmv = (time.perf_counter() - t0) * N / len(rows_k)
    rows_a = np.arange(budget_rows[1])
    t0 = time.perf_counter()
    dK = ogp.kernel_derivatives(X, psi, rows=rows_a)
    for Dj in dK:
        _ = Dj @ V
    t_asm = (time.perf_counter() - t0) * N / len(rows_a)
    blas_threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    per_est = passes_per_estimate * t_kmv + t_asm
    # the oracle forms kernel entries with element-wise numpy (one thread), which is most of
    # its time; only its dense products go through BLAS, on up to blas_threads threads
    return dict(value=1.0 / per_est, unit="grad_estimates/s", cores=1, blas_threads=int(blas_threads),
                kind="oracle",
                sample=(f"oracle FP64 K.V on {budget_rows[0]} of {N} rows and gradient assembly on "
                        f"{budget_rows[1]} rows of the n={N}, d={D}, m={M} workload, scaled by rows "
                        f"to {passes_per_estimate:.2f} products + 1 assembly per estimate; kernel "
                        f"entries on one thread, BLAS products on up to {blas_threads}"),
                kmv_s_full=t_kmv, assembly_s_full=t_asm)


def cpu_baseline_report():
    """The oracle's CPU timings in full (no GPU): matrix-free FP64 K.V, FP64 ULISSE gradient
    estimates and the dense Cholesky exact gradient, each on one thread and on every thread
    the process may use.  Every figure is either a full run or a row/system sample scaled
    linearly, as stated in its entry.
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    import workloads
    from oracle import gp as ogp
    from oracle import rng as orng
    from oracle import stoch_grad as osg
    from oracle import ulisse as oul

    cores = len(os.sched_getaffinity(0))
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    t_start = time.perf_counter()

    def say(msg):
        print(f"cpu report: {msg} ({time.perf_counter() - t_start:.0f} s)", file=sys.stderr, flush=True)

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    rows = []
    rff2 = workloads.rff_gp(n=16384, d=8, seed=1)
    rff3 = workloads.rff_gp(n=65536, d=8, seed=2)
    tiny = workloads.tiny(n=1000, seed=0)
    Xt, psit = tiny["X"], tiny["psi"]
    yt = np.linalg.cholesky(ogp.kernel_matrix(Xt, psit)) @ tiny["z"]
    for threads in (1, cores):
        with threadpool_limits(limits=threads):
            # (i) matrix-free K.V: rows of the product, scaled by rows
            for w, n, m, nrows in ((rff2, 16384, 17, 256 * threads), (rff3, 65536, 32, 64 * threads)):
                V = np.random.default_rng(0).standard_normal((n, m))
                rr = np.arange(min(nrows, n))
                t = timed(lambda: ogp.kmv(w["X"], w["psi"], V, rows=rr)) * n / len(rr)
                rows.append(dict(item="kmv_fp64", n=n, d=8, m=m, threads=threads, seconds=t,
                                 gflops=kmv_flops(n, 8, m) / t / 1e9,
                                 sample=f"{len(rr)} of {n} rows, scaled by rows"))
                say(f"K.V n={n} on {threads} threads: {t:.2f} s")
            # (ii) ULISSE gradient estimates, n = 1000 (4 Rademacher probes, q = 1, c = 1)
            R = osg.draw_probes(0, 1, 0, 1000, 4, 1)
            t = timed(lambda: osg.stoch_grad(Xt, psit, yt, R, 1.0, 1.0, 1e-8, 10000, 0, 1, 0))
            rows.append(dict(item="ulisse_gradient", n=1000, d=2, m=5, threads=threads,
                             seconds=t, estimates_per_s=1.0 / t, sample="one full estimate"))
            say(f"ULISSE gradient n=1000 on {threads} threads: {t:.2f} s")
            # ... and n = 16384 (y + 16 Gaussian probes): dense K once, the y system and one
            # probe system solved in full and scaled to 17 systems, the assembly on rows
            X2, psi2, y2 = rff2["X"], rff2["psi"], rff2["y"].astype(np.float64)
            n2, nr2 = 16384, 16
            holder = {}
            t_k = timed(lambda: holder.__setitem__("K", ogp.kernel_matrix(X2, psi2)))
            K = holder.pop("K")
            R2 = orng.probes(0, 1, 0, n2, nr2, 0)
            B = np.column_stack([y2, R2[:, 0]])
            t_s = timed(lambda: oul.solve_systems(lambda v: K @ v, B, None, 1.0, 1.0, 1e-6, 5000,
                                                  0, 1, 0, two_track_first=True, eps_relative=True))
            del K
            ra = np.arange(64 * threads)
            S = np.random.default_rng(1).standard_normal((n2, 2 + nr2))
            t_a = timed(lambda: [Dj @ S for Dj in ogp.kernel_derivatives(X2, psi2, rows=ra)]) * n2 / len(ra)
            t = t_k + t_s * (1 + nr2) / 2 + t_a
            rows.append(dict(item="ulisse_gradient", n=n2, d=8, m=1 + nr2, threads=threads,
                             seconds=t, estimates_per_s=1.0 / t,
                             sample=(f"dense K {t_k:.2f} s; 2 of {1 + nr2} systems solved "
                                     f"({t_s:.2f} s, scaled); assembly on {len(ra)} rows, scaled")))
            say(f"ULISSE gradient n=16384 on {threads} threads: {t:.2f} s")
            # (iii) dense Cholesky exact gradient: n = 1000 and the first 4096 points of n = 65536
            for Xe, pe, ye, tag in ((Xt, psit, yt, "n=1000, d=2"),
                                    (rff3["X"][:4096], rff3["psi"], rff3["y"][:4096].astype(np.float64),
                                     "n=4096 (first rows of n=65536), d=8")):
                t = timed(lambda: ogp.exact_gradient(Xe, pe, ye))
                rows.append(dict(item="exact_gradient_cholesky", n=len(ye), d=Xe.shape[1],
                                 threads=threads, seconds=t, sample=f"one full gradient, {tag}"))
                say(f"exact gradient {tag} on {threads} threads: {t:.2f} s")
    print(json.dumps({"cpu_report": rows, "cores": cores, "cpu_model": model,
                      "kind": "oracle"}), flush=True)


def kmv_report(pb, h):
    """gp_kmv throughput per precision mode on the workload shapes: n = 16384 (m = 17) and
    n = 65536 (m = 32) of the random-Fourier-feature inputs, n = 65536 with m = 4 (the VALU
    contraction) and the n = 131072, d = 16 mixture (m = 32).  Kernel time from the
    library's hipEvents around the product kernel; call time (packing, BF16 split, split-K
    reduction included) from torch events on the same stream."""
    import numpy as np
    import torch

    import workloads
    shapes = (("rff", 16384, 8, 17, 1), ("rff", 16384, 8, 32, 1), ("rff", 65536, 8, 32, 2),
              ("rff", 65536, 8, 4, 2), ("mixture", 131072, 16, 32, 4))
    names = {pb.GP_FP32: "fp32", pb.GP_BF16_SPLIT_V: "bf16_split_v", pb.GP_BF16_SPLIT_KV: "bf16_split_kv"}
    rows = []
    for kind, n, d, m, seed in shapes:
        w = workloads.rff_gp(n=n, d=d, seed=seed) if kind == "rff" else workloads.mixture(n=n, d=d, seed=seed)
        X = torch.from_numpy(w["X"]).cuda()
        psi = torch.from_numpy(w["psi"]).cuda()
        V = pb.colmajor(n, m)
        V.copy_(torch.from_numpy(workloads.gaussian_matrix(n, m, seed=11)).cuda())
        out = pb.colmajor(n, m)
        reps = max(5, int(2e10 // (n * n)))
        for prec in (pb.GP_FP32, pb.GP_BF16_SPLIT_V, pb.GP_BF16_SPLIT_KV):
            # FP32: both product shapes where the symmetric one applies, each pinned
            variants = [("default", -1)]
            if prec == pb.GP_FP32:
                variants = [("split_k", 2048)]
                try:
                    pb.gp_tune_set(h, n, d, m, pb.SHAPE_SYM)
                    variants.append(("symmetric", pb.SHAPE_SYM))
                except pb.GPError:
                    pass
            if prec == pb.GP_FP32:
                variants.append(("autotuned", None))
            for shape, code in variants:
                if code is None:
                    # the autotuner's choice: the first call of this shape with it on times the candidates
                    pb.gp_tune_set(h, n, d, m, -1, prec=prec)
                    pb.gp_autotune(h, 1)
                else:
                    pb.gp_autotune(h, 0)
                    pb.gp_tune_set(h, n, d, m, code, prec=prec)
                for _ in range(3):
                    pb.gp_kmv(h, X, psi, V, out=out, prec=prec)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                pb.gp_profile(h, 1)
                e0.record()
                for _ in range(reps):
                    pb.gp_kmv(h, X, psi, V, out=out, prec=prec)
                e1.record()
                torch.cuda.synchronize()
                pr = pb.gp_profile_read(h)
                pb.gp_profile(h, 0)
                k_ms = pr["kmv_ms"] / max(1, pr["kmv_launches"])
                main_ms = pr["kmv_main_ms"] / max(1, pr["kmv_main_launches"])
                c_ms = e0.elapsed_time(e1) / reps
                fl = kmv_flops(n, d, m)
                tuned = pb.gp_tune_get(h, n, d, m, prec=prec)
                pb.gp_autotune(h, 0)
                rows.append(dict(workload=f"{kind}_n{n}_d{d}", n=n, d=d, m=m, prec=names[prec], shape=shape,
                                 shape_code=tuned[0], split=tuned[1],
                                 kernel_ms=k_ms, main_kernel_ms=main_ms, call_ms=c_ms, tflops=fl / k_ms / 1e9,
                                 frac_fp32_valu_peak=fl / k_ms / 1e9 / VALU_FP32_PEAK_TFLOPS,
                                 exp_per_s=float(n) * n / (k_ms * 1e-3), launches=pr["kmv_launches"]))
                print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            pb.gp_tune_set(h, n, d, m, -1, prec=prec)
    print(json.dumps({"kmv_report": rows, "flops_per_pair": "3d + 2m (algorithmic, m unpadded)",
                      "kernel_ms": "product kernels of one call (the symmetric shape: kernel + reduce)",
                      "main_kernel_ms": "the main product kernel alone"}),
          flush=True)


def pipes_report(pb, h):
    """Issue-rate probe of the compute pipes (gp_pipe_probe): cycles per loop iteration per
    wave, at eight waves per SIMD, of FP32 VALU FMAs, FP32 and BF16 MFMAs, each MFMA kind with
    independent VALU work, and exp2.  hidden_* = the part of the MFMA-alone cycles that the
    VALU work hid when both ran (0: the two pipes run in series)."""
    r = pb.gp_pipe_probe(h, iters=4000)
    cyc = {k: v[1] for k, v in r.items()}
    out = {"pipes": {k: {"ms": v[0], "cycles_per_iter_wave": v[1]} for k, v in r.items()},
           "hidden_fp32_mfma_frac": (cyc["valu_fma128"] + cyc["mfma_f32_x4"] - cyc["mfma_f32_x4+valu_fma128"]) / cyc["mfma_f32_x4"],
           "hidden_bf16_mfma_frac": (cyc["valu_fma128"] + cyc["mfma_bf16_x4"] - cyc["mfma_bf16_x4+valu_fma128"]) / cyc["mfma_bf16_x4"],
           "exp_over_fma_cost": cyc["exp128"] / cyc["valu_fma128"]}
    print(json.dumps(out), flush=True)


def say(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def matched_error_rates(rows_a, rows_b):
    """Speed of method b over method a at equal gradient error: at every point of one
    method whose mean log10 error lies inside the other's measured range, the other's
    estimates/s there by log-linear interpolation between its points, and the ratio
    rate_b / rate_a."""
    import numpy as np

    def curve(rows):
        pts = sorted((r["mean_log10_rel_sq_err"], np.log(r["grad_estimates_per_s"])) for r in rows)
        return [p_[0] for p_ in pts], [p_[1] for p_ in pts]

    xa, ya = curve(rows_a)
    xb, yb = curve(rows_b)
    out = []
    for r in rows_b:
        e = r["mean_log10_rel_sq_err"]
        if xa[0] <= e <= xa[-1]:
            ra = float(np.exp(np.interp(e, xa, ya)))
            out.append({"at": "b", "q": r["q"], "error": e, "rate_a": ra,
                        "rate_b": r["grad_estimates_per_s"], "speedup": r["grad_estimates_per_s"] / ra})
    for r in rows_a:
        e = r["mean_log10_rel_sq_err"]
        if xb[0] <= e <= xb[-1]:
            rb = float(np.exp(np.interp(e, xb, yb)))
            out.append({"at": "a", "q": r["q"], "error": e, "rate_a": r["grad_estimates_per_s"],
                        "rate_b": rb, "speedup": rb / r["grad_estimates_per_s"]})
    return out


def learned_from_chains(pb, h, X, y, psi_map, M_sub, L_full, eps_t, prior, chains, steps, epochs,
                        k=64, H=256, probes=4, seed=1, q=1.0, psi_eval=None):
    """The learned warm start and preconditioner, trained on (psi, solve) pairs that the
    plain solver generates: the states of `chains` plain-solver SGLD chains (started from
    N(psi_MAP, M_subset), `steps` steps each), the basis U of K(psi_MAP), the Galerkin solve
    and spectrum of K(psi) on U at every state as targets, and the MLP trained on them by
    Adam, all in the library's kernels."""
    import numpy as np
    import torch
    from paper_1501_05427_amd import protocol
    t0 = time.perf_counter()
    starts = protocol.init_chains(psi_map, M_sub, chains, seed=seed)
    states = protocol.plain_chain_states(
        h, X, y, starts, steps, L_full, eps_t, probes=probes, prior=prior, q=q,
        progress=lambda t, T: say(f"training chains: {t}/{T} steps, {time.perf_counter() - t0:.0f} s"))
    t_chain = time.perf_counter() - t0
    psis = torch.from_numpy(states).cuda()
    U, ritz = pb.precond_build_basis(h, X, torch.from_numpy(psi_map).cuda(), k)
    # the Galerkin targets of every state, in pieces of 256 states
    parts = []
    for a in range(0, psis.shape[0], 256):
        parts.append(pb.precond_targets(h, X, y, U, psis[a:a + 256]))
        if (a // 256) % 4 == 3:
            torch.cuda.synchronize()
            say(f"training targets: {a + 256}/{psis.shape[0]}, {time.perf_counter() - t0:.0f} s")
    T = torch.cat(parts)
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t0 - t_chain
    I_, O_ = len(psi_map), 2 * k + 1
    prm = torch.zeros(pb.precond_mlp_size(I_, H, O_), dtype=torch.float32, device="cuda")
    pb.precond_mlp_init(h, prm, I_, H, O_, psis, T, seed=5)
    adam = torch.zeros(2 * pb.mlp_layout(I_, H, O_)["trainable"], dtype=torch.float32, device="cuda")
    ltr = torch.zeros(epochs, dtype=torch.float32, device="cuda")
    pb.precond_mlp_train(h, prm, adam, I_, H, O_, psis, T, epochs, 0, 2e-3, loss_trace=ltr)
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    spread = states.std(axis=0)
    # where the network is evaluated, against the training states: per coordinate, the
    # distance from their mean in units of their spread, and the distance to the nearest state
    far = {}
    if psi_eval is not None:
        pe = np.asarray(psi_eval, np.float64)
        z = (pe - states.mean(axis=0)) / np.maximum(spread, 1e-300)
        nearest = np.sqrt((((states - pe) / np.maximum(spread, 1e-300)) ** 2).sum(axis=1)).min()
        far = {"eval_z_from_state_mean": z.tolist(), "eval_max_abs_z": float(np.abs(z).max()),
               "eval_nearest_state_scaled_dist": float(nearest)}
    return {"prm": prm, "U": U, "I": I_, "H": H, "O": O_, "k": k, "ritz": ritz, "psis": psis,
            "info": {"pairs": int(states.shape[0]), "chains": chains, "steps_per_chain": steps,
                     "probes": probes, "epochs": epochs, "rank": k, "hidden": H,
                     "basis_at": "subset MAP",
                     "train_loss_first_last": [float(ltr[0]), float(ltr[-1])],
                     "ritz_top_bottom": [float(ritz[0]), float(ritz[-1])],
                     "state_sd_mean": float(spread.mean()), "chain_q": q, **far,
                     "seconds_chains": t_chain, "seconds_targets": t_targets, "seconds_total": t_total}}


class Chain:
    """One SGLD chain on the benchmark workload and the estimators the legs compare.

    Methods of `estimate`: plain_fp32 (gp_stoch_grad, FP32 products), plain_bf16 (BF16
    products, split V or split K+V, with residual replacement), and, over the rank-k basis U of the
    learned set-up with the same BF16 products: learned_bf16 (coefficients from the network
    at the chain's psi), learned_bf16_uc (the same plus the warm start U c of the y
    system), galerkin_direct_bf16 (coefficients of the Galerkin preconditioner computed at
    the chain's psi: one K U product per estimate) and galerkin_fixed_bf16 (computed once,
    at the subset MAP)."""

    def __init__(self, pb, h, X, y, M_chol, refresh, k=64, bf16_prec=None):
        import torch
        self.pb, self.h, self.X, self.y, self.M_chol, self.refresh, self.k = pb, h, X, y, M_chol, refresh, k
        self.bf16_prec = pb.GP_BF16_SPLIT_V if bf16_prec is None else bf16_prec
        P = D + 2
        self.psi = torch.zeros(P, dtype=torch.float64, device="cuda")
        self.S_warm = torch.zeros((M, N), dtype=torch.float64, device="cuda").t()
        self.R = pb.colmajor(N, NPROBES)
        self.g = torch.zeros(P, dtype=torch.float64, device="cuda")
        self.stats = pb.stats_tensor(M)
        self.flagged = torch.zeros((), dtype=torch.int64, device="cuda")
        self.fallbacks = torch.zeros((), dtype=torch.int64, device="cuda")
        self.reruns = torch.zeros((), dtype=torch.int64, device="cuda")
        self.params = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=1000, rng_stream=1)
        self.coef = torch.zeros(k + 1, dtype=torch.float64, device="cuda")
        self.cvec = torch.zeros(k, dtype=torch.float64, device="cuda")
        self.prior_a = torch.zeros(P, dtype=torch.float64, device="cuda")
        self.prior_b = torch.full((P,), 3.0, dtype=torch.float64, device="cuda")
        self.L = None

    def set_learned(self, L, coef_map):
        import torch
        pb = self.pb
        self.L = L
        self.pc = pb.make_precond(L["U"], self.coef)
        self.pc_uc = pb.make_precond(L["U"], self.coef, cvec=self.cvec)
        self.T1 = torch.zeros((1, 2 * self.k + 1), dtype=torch.float32, device="cuda")
        self.coef_map = coef_map

    def estimate(self, method, t, period=1, new_probes=True):
        """One gradient estimate of `method` at step t into self.g."""
        import torch
        pb, h, prm = self.pb, self.h, self.params
        prm.rng_counter = t
        prm.prec = pb.GP_FP32 if method == "plain_fp32" else self.bf16_prec
        prm.refresh = 0 if method == "plain_fp32" else self.refresh
        if period > 1 and new_probes:
            pb.gp_draw_probes(h, N, NPROBES, pb.PROBE_GAUSSIAN, 7, t // period, R=self.R)
            self.S_warm[:, 1:].zero_()
        kw = dict(R=self.R if period > 1 else None, n_probes=NPROBES, S_warm=self.S_warm, g=self.g,
                  stats=self.stats)
        if method in ("plain_fp32", "plain_bf16"):
            pb.gp_stoch_grad(h, self.X, self.psi, self.y, prm, **kw)
            fl = self.stats.view(M, -1)[:, 24:28].view(torch.int32)
            self.reruns.add_(fl.bitwise_and(pb.ULISSE_FP32_RERUN).ne(0).any().to(torch.int64))
            return
        L = self.L
        if method.startswith("learned"):
            pb.precond_from_mlp(h, L["prm"], L["I"], L["H"], L["O"], self.psi, self.k, coef=self.coef, c=self.cvec)
        elif method == "galerkin_direct_bf16":
            pb.precond_targets(h, self.X, self.y, L["U"], self.psi[None, :], targets=self.T1)
            pb.precond_from_targets(h, self.T1[0], self.k, coef=self.coef, c=self.cvec)
        elif method == "galerkin_fixed_bf16":
            self.coef.copy_(self.coef_map)
        else:
            raise ValueError(method)
        pc = self.pc_uc if method == "learned_bf16_uc" else self.pc
        pb.gp_stoch_grad_pc(h, self.X, self.psi, self.y, prm, pc, **kw)
        fl = self.stats.view(M, -1)[:, 24:28].view(torch.int32)
        self.fallbacks.add_(fl.bitwise_and(pb.ULISSE_FALLBACK).ne(0).any().to(torch.int64))
        self.reruns.add_(fl.bitwise_and(pb.ULISSE_FP32_RERUN).ne(0).any().to(torch.int64))

    def step(self, method, t, period, first, eps_t):
        import torch
        pb = self.pb
        self.estimate(method, t, period, first or t % period == 0)
        pb.sgld_step(self.h, self.psi, self.g, eps_t, rng_stream=1, rng_counter=t, prior_kind=1,
                     prior_a=self.prior_a, prior_b=self.prior_b, M_chol=self.M_chol)
        fl = self.stats.view(M, -1)[:, 24:28].view(torch.int32)
        self.flagged.add_(fl.bitwise_and(pb.ULISSE_NOTCONV | pb.ULISSE_BREAKDOWN).ne(0).any().to(torch.int64))

    def timed(self, method, first, count, period, eps_t):
        import torch
        pb = self.pb
        torch.cuda.synchronize()
        pb.gp_profile(self.h, 1)
        t0 = time.perf_counter()
        for t in range(first, first + count):
            self.step(method, t, period, t == first, eps_t)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        pr = pb.gp_profile_read(self.h)
        pb.gp_profile(self.h, 0)
        return el, pr


def main_line(args, pb, h, X, y, w, psi0):
    """The default benchmark line: one SGLD step = one unbiased gradient estimate + the SGLD
    update on the n = 65536, d = 8 workload (31 Gaussian probes, 32 right-hand sides).

    Headline protocol (`value`): fresh probes every step, psi starting at the truth, the y
    system warm-started from its last CG iterate, q = 1, rate 1, prior N(0, 3^2) on psi, the
    SGLD preconditioner of the paper's experiments (Sec. 5): M = (-H)^-1 at the MAP of a
    random 500-point subset, scaled by 500 / n for the full data, and the step size at which
    the paper's Langevin-phase monitor (eps / 4) lambda_max(L^T V L) meets its freeze
    threshold 0.002 (Sec. 2.1), V the covariance of 16 gradient estimates at the truth: the
    chain in its sampling phase.  Every other leg starts from the same saved state with the
    same draws."""
    import numpy as np
    import torch
    from paper_1501_05427_amd import protocol
    P = D + 2
    prior = {"kind": 1, "a": np.zeros(P), "b": np.full(P, 3.0)}
    eps_train = 1e-3     # the training chains: their transient phase gives the pairs their spread
    t0 = time.perf_counter()
    psi_map, M_sub, _ = protocol.sgld_preconditioner(h, w["X"], w["y"], w["psi"], prior, n_sub=500, seed=0)
    t_map = time.perf_counter() - t0
    M_full = M_sub * (500.0 / N)
    L_full = np.linalg.cholesky(M_full)
    M_chol = torch.from_numpy(np.ascontiguousarray(L_full.T)).cuda()
    say(f"subset MAP and M: {t_map:.1f} s")
    k = 64
    bf16_prec = {"kv": pb.GP_BF16_SPLIT_KV, "v": pb.GP_BF16_SPLIT_V}[args.bf16_mode]
    ch = Chain(pb, h, X, y, M_chol, args.refresh, k=k, bf16_prec=bf16_prec)
    ch.psi.copy_(psi0)
    # the step size at the freeze threshold of the Langevin-phase monitor
    G = []
    for r in range(17):
        ch.estimate("plain_fp32", 90_000 + r)
        if r > 0:           # the first estimate only warms the y system up
            G.append(ch.g.cpu().numpy().copy())
    V = np.cov(np.array(G).T)
    lam_max = float(np.linalg.eigvalsh(L_full.T @ V @ L_full).max())
    eps_t = 4 * 0.002 / lam_max
    ch.S_warm.zero_()
    say(f"step size at the Langevin freeze threshold: {eps_t:.3g} (lambda_max {lam_max:.3g})")

    K_, W_ = args.steps, args.warmup
    for t in range(W_):
        ch.step("plain_fp32", t, 1, t == 0, eps_t)
    saved = (ch.psi.clone(), ch.S_warm.clone())

    def restore():
        ch.psi.copy_(saved[0])
        ch.S_warm.copy_(saved[1])

    def leg(method, period, count):
        restore()
        ch.reruns.zero_()
        el, pr = ch.timed(method, W_, count, period, eps_t)
        out = {"grad_estimates_per_s": count / el, "steps": count, "probe_period": period,
               "kmv_passes_per_estimate": pr["kmv_passes"] / count,
               "kmv_avg_launch_ms": pr["kmv_ms"] / max(1, pr["kmv_launches"]),
               "dquad_avg_ms": pr["dquad_ms"] / max(1, pr["dquad_launches"])}
        if method != "plain_fp32":
            out["steps_with_fp32_rerun"] = int(ch.reruns.item())  # BF16 solves that broke down
        return out

    # the headline: plain FP32, fresh probes every step
    restore()
    ch.flagged.zero_()
    elapsed, prof = ch.timed("plain_fp32", W_, K_, 1, eps_t)
    value = K_ / elapsed
    psi_eval = ch.psi.clone()       # a state of the chain, off the training set, for the error leg
    headline_flagged = int(ch.flagged.item())
    final_stats = pb.decode_stats(ch.stats)
    say(f"plain FP32, fresh probes: {value:.2f} estimates/s")
    # the paper's protocol: probes redrawn every 20 steps, every system warm-started
    paper = leg("plain_fp32", PROBE_PERIOD, K_)
    say(f"plain FP32, paper protocol: {paper['grad_estimates_per_s']:.2f} estimates/s")
    bf16 = leg("plain_bf16", 1, K_)
    say(f"BF16 split {'K+V' if args.bf16_mode == 'kv' else 'V'}: {bf16['grad_estimates_per_s']:.2f} estimates/s")

    # K.V throughput of each arithmetic mode at the same shape (m = 32)
    import workloads
    Vb = pb.colmajor(N, M)
    Vb.copy_(torch.from_numpy(workloads.gaussian_matrix(N, M, seed=11)).cuda())
    outb = pb.colmajor(N, M)
    kv_modes = {}
    for name, prec in (("fp32", pb.GP_FP32), ("bf16_split_v", pb.GP_BF16_SPLIT_V),
                       ("bf16_split_kv", pb.GP_BF16_SPLIT_KV)):
        pb.gp_kmv(h, X, psi0, Vb, out=outb, prec=prec)
        torch.cuda.synchronize()
        pb.gp_profile(h, 1)
        for _ in range(5):
            pb.gp_kmv(h, X, psi0, Vb, out=outb, prec=prec)
        pr = pb.gp_profile_read(h)
        pb.gp_profile(h, 0)
        ms = pr["kmv_ms"] / pr["kmv_launches"]
        kv_modes[name] = {"avg_launch_ms": ms, "tflops": kmv_flops(N, D, M) / (ms * 1e-3) / 1e12}

    learned = None
    equal = None
    if args.learned_steps:
        Lr = learned_from_chains(pb, h, X, y, psi_map, M_sub, L_full, eps_train, prior,
                                 args.learn_chains, args.learn_chain_steps, args.learn_epochs, k=k,
                                 q=args.learn_chain_q, psi_eval=w["psi"])
        Lr["info"]["chain_step_size"] = eps_train
        Tm = pb.precond_targets(h, X, y, Lr["U"], torch.from_numpy(psi_map[None, :].copy()).cuda())
        ch.set_learned(Lr, pb.precond_from_targets(h, Tm[0], k))
        say(f"learned set-up: {Lr['info']['pairs']} pairs, {Lr['info']['seconds_total']:.1f} s")
        legs = {}
        ch.fallbacks.zero_()
        for method in ("learned_bf16", "learned_bf16_uc", "galerkin_fixed_bf16", "galerkin_direct_bf16"):
            legs[method] = leg(method, 1, args.learned_steps)
            say(f"{method}: {legs[method]['grad_estimates_per_s']:.2f} estimates/s")
        legs["paper_protocol"] = leg("learned_bf16", PROBE_PERIOD, args.learned_steps)
        learned = dict(legs["learned_bf16"])
        learned.update({"vs_plain_fp32": learned["grad_estimates_per_s"] / value,
                        "precision": {"kv": "bf16_split_kv", "v": "bf16_split_v"}[args.bf16_mode],
                        "refresh": args.refresh,
                        "with_warm_start_uc": legs["learned_bf16_uc"],
                        "galerkin_fixed_at_map_bf16": legs["galerkin_fixed_bf16"],
                        "galerkin_direct_bf16": legs["galerkin_direct_bf16"],
                        "paper_protocol": legs["paper_protocol"],
                        "steps_with_fallback": int(ch.fallbacks.item()),
                        "training": Lr["info"]})
        if args.equal_error_reps:
            equal = equal_error_leg(args, pb, h, X, y, ch, psi_eval)

    # the dominant kernel: the main product kernel, timed by its own hipEvent pair; the whole
    # product (the symmetric shape adds the FP64 reduce of its partials) is reported beside it
    kmv_avg_s = prof["kmv_ms"] / max(1, prof["kmv_launches"]) / 1e3
    main_avg_s = prof["kmv_main_ms"] / max(1, prof["kmv_main_launches"]) / 1e3
    achieved = kmv_flops(N, D, M) / main_avg_s / 1e12
    pass_achieved = kmv_flops(N, D, M) / kmv_avg_s / 1e12
    sym_shape = pb.gp_tune_get(h, N, D, M)[0] == pb.SHAPE_SYM
    kv_kernel = ("kmv_sym_f32_kernel<8, 2, 0> (K.V, m=32, symmetric shape; its reduce in pass_*)"
                 if sym_shape else "kmv_mfma_f32_kernel<8, 2, 0, 4> (K.V, m=32, split-K)")
    return {
        "metric": "unbiased grad estimates/s and K·V TFLOP/s at n=65536, learned+BF16 vs plain",
        "value": value,
        "unit": "grad_estimates/s",
        "n_gpus": 1,
        "steps": K_,
        "warmup": W_,
        "ms_per_step": 1e3 * elapsed / K_,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": N, "d": D, "rhs": M, "probes": NPROBES,
                   "probe_kind": "gaussian", "probe_period": 1, "q": 1.0, "rate": 1.0,
                   "eps_rel": 1e-6, "psi_start": "truth", "warm_start": "y from its last CG iterate",
                   "sgld_eps": eps_t, "sgld_eps_rule": "(eps/4) lambda_max(L^T V L) = 0.002, V from "
                   "16 estimates at the truth (the freeze threshold of the Langevin-phase monitor)",
                   "sgld_M": "(-H)^-1 at the MAP of a 500-point subset, x 500/n",
                   "precision": "fp32",
                   "value_is": "plain FP32 path; learned+BF16 in learned_bf16, K.V in roofline"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / VALU_FP32_PEAK_TFLOPS,
                     "traffic": traffic_from_profile(), "kernel": kv_kernel,
                     "avg_launch_ms": main_avg_s * 1e3, "launches": prof["kmv_main_launches"],
                     "pass_achieved": pass_achieved, "pass_frac": pass_achieved / VALU_FP32_PEAK_TFLOPS,
                     "pass_avg_ms": kmv_avg_s * 1e3,
                     "pass_is": "the whole product: main kernel + the symmetric shape's FP64 reduce",
                     "traffic_is": "HBM bytes of the whole product (main kernel + reduce)"},
        "kv_tflops": achieved,
        "kmv_passes_per_estimate": prof["kmv_passes"] / K_,
        "dquad_avg_ms": prof["dquad_ms"] / max(1, prof["dquad_launches"]),
        "exp_per_s": N * float(N) / kmv_avg_s,
        "paper_protocol": paper,
        f"bf16_split_{args.bf16_mode}_solver": dict(bf16, refresh=args.refresh),
        "kv_by_precision": kv_modes,
        "learned_bf16": learned,
        "equal_error": equal,
        "sgld_preconditioner": {"subset": 500, "map_seconds": t_map, "psi_map": psi_map.tolist(),
                                "M_diag": np.diag(M_full).tolist()},
        "last_step_stats": {"l": [s_["l"] for s_ in final_stats],
                            "J_max": max(max(s_["J_a"], s_["J_b"]) for s_ in final_stats)},
        "steps_with_flagged_systems": headline_flagged,
        "psi_final": psi_eval.cpu().numpy().tolist(),
    }


def equal_error_leg(args, pb, h, X, y, ch, psi_eval):
    """Gradient error against estimates/s at one state of the headline chain (not in the
    training set): the paper's error measure, the mean over repetitions of
    log10 ||g~ - g_ref||^2 / ||g_ref||^2 (Sec. 4.2), with g_ref the plain estimator with
    converged solves averaged over batches of 31 probes (its standard error reported).
    Every estimate draws fresh probes; the y system keeps its warm start from the previous
    estimate.  Methods: plain FP32, and with the chain's BF16 products plus residual
    replacement: the learned preconditioner, the Galerkin preconditioner on the same basis
    computed directly at the psi of each estimate (its K U product counted in the time),
    and the Galerkin preconditioner fixed at the subset MAP."""
    import numpy as np
    import torch
    from paper_1501_05427_amd import protocol
    t0 = time.perf_counter()
    g_ref, g_se = protocol.probe_mean_gradient(h, X, y, psi_eval, args.equal_error_ref_batches,
                                               probes=NPROBES, probe_stream=21)
    t_ref = time.perf_counter() - t0
    say(f"equal error: reference gradient {t_ref:.1f} s")
    rows = {}
    q_saved = ch.params.q
    for method in ("plain_fp32", "learned_bf16", "galerkin_direct_bf16", "galerkin_fixed_bf16"):
        rows[method] = []
        for q in (args.equal_error_q_plain if method == "plain_fp32" else args.equal_error_q):
            ch.params.q = q
            ch.psi.copy_(psi_eval)
            ch.S_warm.zero_()
            ch.reruns.zero_()
            errs, el = [], 0.0
            for r in range(args.equal_error_reps + 1):   # r = 0 warms the y system up, untimed
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                ch.estimate(method, 50_000 + r)
                torch.cuda.synchronize()
                if r == 0:
                    continue
                el += time.perf_counter() - t1
                e = ch.g.cpu().numpy() - g_ref
                errs.append(float(np.sum(e * e) / np.sum(g_ref * g_ref)))
            lg = np.log10(np.array(errs))
            rows[method].append({"q": q, "reps": len(errs), "mean_log10_rel_sq_err": float(lg.mean()),
                                 "se": float(lg.std(ddof=1) / np.sqrt(len(lg))),
                                 "grad_estimates_per_s": len(errs) / el,
                                 "var_normalised_throughput": len(errs) / el / float(np.mean(errs)),
                                 "fp32_reruns": int(ch.reruns.item())})
            say(f"equal error {method} q={q}: {rows[method][-1]['mean_log10_rel_sq_err']:.2f} "
                f"+- {rows[method][-1]['se']:.2f}, {rows[method][-1]['grad_estimates_per_s']:.2f}/s")
    ch.params.q = q_saved
    base = rows["plain_fp32"]
    return {"psi": "the headline chain's last state", "g_ref_rel_se": float(np.linalg.norm(g_se) / np.linalg.norm(g_ref)),
            "ref_probes": args.equal_error_ref_batches * NPROBES, "ref_seconds": t_ref,
            "methods": rows,
            "learned_bf16_vs_plain_fp32_at_matched_error": matched_error_rates(base, rows["learned_bf16"]),
            "learned_bf16_vs_galerkin_direct_at_matched_error":
                matched_error_rates(rows["galerkin_direct_bf16"], rows["learned_bf16"]),
            "learned_bf16_vs_galerkin_fixed_at_matched_error":
                matched_error_rates(rows["galerkin_fixed_bf16"], rows["learned_bf16"])}


def error_sweep(args, pb, h, X, y, w, psi0):
    """Gradient error against estimates/s, plain FP32 against learned + BF16 split-K+V (and,
    on request, the two halves of that change: BF16 products alone, the learned
    preconditioner alone).

    Error of one estimate: log10 ||g~ - g_ref||^2 / ||g_ref||^2, averaged over `reps`
    independent estimates at the workload's psi (the paper's measure of gradient accuracy,
    Sec. 4.2), which is off the network's training set: the states of plain-solver SGLD
    chains started around the MAP of a 500-point subset, where the basis is built.  g_ref: the plain FP32 estimator with converged solves (q = 0, so the series
    never truncates; CG to 1e-6 relative) averaged over `ref_probes` Gaussian probes; its
    standard error is reported.  Each estimate draws fresh probes; the y system keeps its
    warm start from the previous estimate as it would along a chain.
    """
    import numpy as np
    import torch
    P = D + 2
    g = torch.zeros(P, dtype=torch.float64, device="cuda")
    R = pb.colmajor(N, NPROBES)
    stats = pb.stats_tensor(M)
    S_warm = torch.zeros((M, N), dtype=torch.float64, device="cuda").t()

    # reference gradient
    from paper_1501_05427_amd import protocol
    t0 = time.perf_counter()
    batches = max(1, args.ref_probes // NPROBES)

    def progress(b, total):
        print(f"reference: {b}/{total} probe batches, {time.perf_counter() - t0:.1f} s",
              file=sys.stderr, flush=True)
    g_ref, g_ref_se = protocol.probe_mean_gradient(h, X, y, psi0, batches, probes=NPROBES,
                                                   probe_stream=21, progress=progress)
    t_ref = time.perf_counter() - t0

    # the network: trained on the states of plain-solver SGLD chains (basis at the subset MAP)
    from paper_1501_05427_amd import protocol
    P = D + 2
    prior = {"kind": 1, "a": np.zeros(P), "b": np.full(P, 3.0)}
    t0 = time.perf_counter()
    psi_map, M_sub, _ = protocol.sgld_preconditioner(h, w["X"], w["y"], w["psi"], prior, n_sub=500, seed=0)
    L_full = np.linalg.cholesky(M_sub * (500.0 / N))
    say(f"subset MAP: {time.perf_counter() - t0:.1f} s")
    L = learned_from_chains(pb, h, X, y, psi_map, M_sub, L_full, 1e-3, prior, args.learn_chains,
                            args.learn_chain_steps, args.learn_epochs, probes=args.learn_chain_probes,
                            q=args.learn_chain_q, psi_eval=psi0.cpu().numpy())
    say(f"learned set-up: {L['info']['pairs']} pairs, {L['info']['seconds_total']:.1f} s "
        f"(chains {L['info']['seconds_chains']:.1f} s); evaluation point max |z| "
        f"{L['info']['eval_max_abs_z']:.1f} from the training states")
    L["coef"] = torch.zeros(L["k"] + 1, dtype=torch.float64, device="cuda")
    L["pc"] = pb.make_precond(L["U"], L["coef"])
    psi = psi0.clone()

    def run(method, q):
        params = pb.make_params(q=q, rate=1.0, eps=1e-6, eps_relative=1, max_iter=1000, rng_stream=5)
        learned = method.startswith("learned")
        if method.endswith("bf16"):
            params.prec = pb.GP_BF16_SPLIT_KV
            params.refresh = args.refresh
        if learned:
            pb.precond_from_mlp(h, L["prm"], L["I"], L["H"], L["O"], psi, L["k"], coef=L["coef"])
        S_warm.zero_()
        errs, passes = [], 0.0
        elapsed = 0.0
        for r in range(args.sweep_reps + 1):  # rep 0 warms the y system up, untimed
            torch.cuda.synchronize()
            pb.gp_profile(h, 1)
            t0 = time.perf_counter()
            pb.gp_draw_probes(h, N, NPROBES, pb.PROBE_GAUSSIAN, 23, r, R=R)
            S_warm[:, 1:].zero_()
            params.rng_counter = r
            if learned:
                pb.precond_from_mlp(h, L["prm"], L["I"], L["H"], L["O"], psi, L["k"], coef=L["coef"])
                pb.gp_stoch_grad_pc(h, X, psi, y, params, L["pc"], R=R, S_warm=S_warm, g=g, stats=stats)
            else:
                pb.gp_stoch_grad(h, X, psi, y, params, R=R, S_warm=S_warm, g=g, stats=stats)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            pr = pb.gp_profile_read(h)
            pb.gp_profile(h, 0)
            if r % 10 == 0:
                print(f"{method} q={q}: estimate {r}, {elapsed:.1f} s", file=sys.stderr, flush=True)
            if r == 0:
                continue
            elapsed += dt
            passes += pr["kmv_passes"]
            e = g.cpu().numpy() - g_ref
            errs.append(float(np.sum(e * e) / np.sum(g_ref * g_ref)))
        errs = np.array(errs)
        return {"method": method, "q": q, "reps": len(errs),
                "mean_log10_rel_sq_err": float(np.mean(np.log10(errs))),
                "se_mean_log10": float(np.std(np.log10(errs), ddof=1) / np.sqrt(len(errs))),
                "rel_mse": float(np.mean(errs)),
                "grad_estimates_per_s": len(errs) / elapsed,
                "kmv_passes_per_estimate": passes / len(errs),
                "var_normalised_throughput": len(errs) / elapsed / float(np.mean(errs))}

    rows = []
    for method in args.sweep_methods:
        for q in args.sweep_q:
            rows.append(run(method, q))
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    out = {"error_sweep": rows, "g_ref": g_ref.tolist(), "g_ref_se": g_ref_se.tolist(),
           "ref_probes": batches * NPROBES, "ref_seconds": t_ref, "training": L["info"],
           "matched_error": matched_error_rates([r for r in rows if r["method"] == "plain_fp32"],
                                                [r for r in rows if r["method"] == "learned_bf16"])
           if {"plain_fp32", "learned_bf16"} <= {r["method"] for r in rows} else None,
           "workload": WORKLOAD, "probes": NPROBES, "fresh_probes_every_estimate": True}
    print(json.dumps(out), flush=True)


def solver_study(args, pb, h):
    """The solver study of Sec. 3.2 and Sec. 4.2 on synthetic data, against the condition
    number: CG iterations to convergence; ULISSE products per solve and the per-element
    standard deviation of its estimates (Fig. 3's measure); log10 relative squared error of
    the gradient (Fig. 4's measure) for q in {0.1, 1} and rate c in {1, 0.01}.

    Inputs: the n = 16384, d = 8 random-Fourier-feature workload with lambda varied to set
    kappa = (lambda_max(K_f) + lambda) / lambda.  The ULISSE draws for one kappa share one CG
    path: the right-hand side y is repeated in 32 columns, whose uniforms are independent.
    """
    import numpy as np
    import torch
    import workloads
    n, d, m = 16384, 8, 32
    w = workloads.rff_gp(n=n, d=d, seed=1)
    X = torch.from_numpy(w["X"]).cuda()
    y = torch.from_numpy(w["y"]).cuda()
    Y = pb.colmajor(n, m)
    Y.copy_(y[:, None].expand(n, m))
    R = pb.colmajor(n, NPROBES)
    g = torch.zeros(d + 2, dtype=torch.float64, device="cuda")
    # (q, rate); q = 0 is plain CG run to convergence (the "CG" line of Figs. 3 and 4)
    settings = [(0.0, 1.0), (0.1, 1.0), (1.0, 1.0), (0.1, 0.01), (1.0, 0.01)]
    rows = []
    for lam in args.study_lambdas:
        psi_np = w["psi"].copy()
        psi_np[-1] = np.log(lam)
        psi = torch.from_numpy(psi_np).cuda()
        # lambda_max of K by power iteration
        v = pb.colmajor(n, 1)
        v.copy_(torch.from_numpy(workloads.gaussian_matrix(n, 1, seed=5)).cuda())
        for _ in range(40):
            kv = pb.gp_kmv(h, X, psi, v)
            v.copy_(kv / torch.linalg.vector_norm(kv))
        lmax = float(torch.dot(v[:, 0], pb.gp_kmv(h, X, psi, v)[:, 0]))
        kappa = lmax / lam
        t0 = time.perf_counter()
        conv = pb.make_params(q=0.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=args.study_max_iter)
        St, st = pb.ulisse_solve(h, X, psi, Y[:, :1], conv)
        cg_stats = pb.decode_stats(st)[0]
        s_ref = St[:, 0].clone()
        row = {"lambda": lam, "kappa": kappa, "cg_iters": cg_stats["iters"],
               "cg_flags": cg_stats["flags"], "solution_rms": float(torch.sqrt(torch.mean(s_ref ** 2))),
               "settings": [], "shifted_pcg": []}
        # PCG with J = K + delta I (Sec. 3.3): outer iterations and all products (outer and
        # inner) to the same convergence as CG, for a few shifts and inner tolerances
        for rel_delta in ((1.0, 10.0, 100.0) if kappa < 1e5 else ()):
            for eps_in in (1e-1, 1e-2):
                sp = pb.make_shift_precond(rel_delta * lam, eps_in, 5000)
                pb.gp_profile(h, 1)
                Ssp, stsp = pb.ulisse_solve_shift_pc(h, X, psi, Y[:, :1], conv, sp)
                prs = pb.gp_profile_read(h)
                pb.gp_profile(h, 0)
                ss_ = pb.decode_stats(stsp)[0]
                row["shifted_pcg"].append({"delta_over_lambda": rel_delta, "eps_inner": eps_in,
                                           "outer_iters": ss_["iters"], "flags": ss_["flags"],
                                           "total_products": prs["kmv_passes"],
                                           "rel_diff_to_cg": float(torch.linalg.vector_norm(Ssp[:, 0] - s_ref)
                                                                   / torch.linalg.vector_norm(s_ref))})
                print(f"kappa {kappa:.3g}: shifted PCG delta={rel_delta}*lambda eps_in={eps_in}: "
                      f"{ss_['iters']} outer, {prs['kmv_passes']} products", file=sys.stderr, flush=True)
        # reference gradient: converged solves, averaged over batches of NPROBES probes
        gs = []
        for b in range(args.study_ref_batches):
            conv.rng_counter = 1000 + b
            pb.gp_stoch_grad(h, X, psi, y, conv, n_probes=NPROBES, g=g)
            gs.append(g.cpu().numpy().copy())
        g_ref = np.mean(gs, 0)
        row["g_ref_rel_se"] = float(np.linalg.norm(np.std(gs, 0, ddof=1) / np.sqrt(len(gs)))
                                    / np.linalg.norm(g_ref))
        for q, c in settings:
            par = pb.make_params(q=q, rate=c, eps=1e-6, eps_relative=1, max_iter=args.study_max_iter,
                                 rng_stream=11)
            St, st = pb.ulisse_solve(h, X, psi, Y, par)
            ss = pb.decode_stats(st)
            Sn = St.cpu().numpy()
            per_elem_std = float(np.mean(np.std(Sn, axis=1, ddof=1)))
            errs = []
            for r in range(args.study_reps):
                par.rng_counter = 5000 + r
                pb.gp_stoch_grad(h, X, psi, y, par, n_probes=args.study_probes, g=g)
                e = g.cpu().numpy() - g_ref
                errs.append(float(np.sum(e * e) / np.sum(g_ref * g_ref)))
            print(f"kappa {kappa:.3g}: q={q} rate={c} done, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
            row["settings"].append({
                "q": q, "rate": c,
                "products_mean": float(np.mean([s_["iters"] for s_ in ss])),
                "l_mean": float(np.mean([s_["l"] for s_ in ss])),
                "J_mean": float(np.mean([s_["J_a"] for s_ in ss])),
                "flagged": int(sum(1 for s_ in ss if s_["flags"])),
                "per_element_std": per_elem_std,
                "grad_mean_log10_err": float(np.mean(np.log10(errs))),
                "grad_reps": len(errs)})
        row["seconds"] = time.perf_counter() - t0
        rows.append(row)
        print(json.dumps(row), flush=True)
    print(json.dumps({"solver_study": rows, "workload": "rff_n16384_d8", "probes": args.study_probes,
                      "ref_probes": args.study_ref_batches * NPROBES, "draws_per_path": m}), flush=True)


def batched_bench(args, pb, n_features=2048, learn_pairs=128, learn_epochs=1000, emit=True):
    """64 independent SGLD chains over 64 GPs (n uniform in [2048, 32768], d in {2, 4, 8, 16},
    the random-Fourier-feature generator with a sub-seed per GP, y + 16 probes each),
    stepped together through gp_batch_* (captured graphs, autotuned product shapes), against
    the same chains stepped one after another through gp_stoch_grad + sgld_step.
    Protocol of the main bench: probes redrawn every 20 steps with warm starts, q = 1,
    M = I / n, eps = 1e-3, N(0, 3^2) prior on psi."""
    import numpy as np
    import torch
    import workloads
    B, nr = args.batch_chains, 16
    r = np.random.default_rng(3)
    ns = r.integers(2048, 32768, endpoint=True, size=B)
    ds = r.choice([2, 4, 8, 16], size=B)
    seeds = r.integers(0, 2**31, size=B)
    probs = []
    for i in range(B):
        n, d = int(ns[i]), int(ds[i])
        w = workloads.rff_gp(n=n, d=d, seed=int(seeds[i]), n_features=n_features)
        probs.append({"X": torch.from_numpy(w["X"]).cuda(), "y": torch.from_numpy(w["y"]).cuda(),
                      "psi": torch.from_numpy(w["psi"]).cuda(),
                      "M_chol": torch.diag(torch.full((d + 2,), n ** -0.5, dtype=torch.float64)).cuda(),
                      "prior": (1, torch.zeros(d + 2, dtype=torch.float64, device="cuda"),
                                torch.full((d + 2,), 3.0, dtype=torch.float64, device="cuda"))})
    pairs = float(np.sum(ns.astype(np.float64) ** 2))
    params = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=1000, rng_stream=1)
    eps_t = 1e-3
    psi0 = [p["psi"].clone() for p in probs]
    out = {"workload": f"batch{B}_rff_n2048-32768_d2-16_m17", "chains": B, "pairs_per_product_sweep": pairs,
           "rff_features": n_features}
    if args.batch_only_graphs:
        # the batched FP32 form alone (autotuning off), for a kernel trace of its steps
        batch = pb.Batch(probs, nr, params, seed=7000, probe_period=PROBE_PERIOD, iters_per_graph=8,
                         autotune=False, streams=8)
        for t in range(args.warmup):
            batch.step(t, eps_t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(args.warmup, args.warmup + args.batch_steps):
            batch.step(t, eps_t)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out["batched_graphs"] = {"grad_estimates_per_s": B * args.batch_steps / el,
                                 "ms_per_step": 1e3 * el / args.batch_steps, "stats": batch.stats(),
                                 "first_timed_step": args.warmup, "steps": args.batch_steps}
        batch.close()
        if emit:
            print(json.dumps({"batched": out}), flush=True)
        return out
    # unbatched: the same chains one after another (own handle per chain, eager calls)
    hs = [pb.Handle(0, seed=7000 + i) for i in range(B)]
    st = []
    for i, p in enumerate(probs):
        n, d = p["X"].shape
        st.append({"S_warm": torch.zeros((1 + nr, n), dtype=torch.float64, device="cuda").t(),
                   "R": pb.colmajor(n, nr), "g": torch.zeros(d + 2, dtype=torch.float64, device="cuda")})

    def unbatched_step(t):
        for i, p in enumerate(probs):
            s_ = st[i]
            n = p["X"].shape[0]
            if t % PROBE_PERIOD == 0:
                pb.gp_draw_probes(hs[i], n, nr, pb.PROBE_GAUSSIAN, params.rng_stream, t // PROBE_PERIOD, R=s_["R"])
                s_["S_warm"][:, 1:].zero_()
            params.rng_counter = t
            pb.gp_stoch_grad(hs[i], p["X"], p["psi"], p["y"], params, R=s_["R"], S_warm=s_["S_warm"], g=s_["g"])
            kind, a, b = p["prior"]
            pb.sgld_step(hs[i], p["psi"], s_["g"], eps_t, rng_stream=params.rng_stream, rng_counter=t,
                         prior_kind=kind, prior_a=a, prior_b=b, M_chol=p["M_chol"])

    for t in range(args.warmup):
        unbatched_step(t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.warmup, args.warmup + args.batch_steps):
        unbatched_step(t)
    torch.cuda.synchronize()
    el_u = time.perf_counter() - t0
    out["unbatched"] = {"grad_estimates_per_s": B * args.batch_steps / el_u,
                        "ms_per_step": 1e3 * el_u / args.batch_steps}
    print(json.dumps({"unbatched_done": out["unbatched"]}), file=sys.stderr, flush=True)
    del hs
    # the BF16 forms: V split (with residual replacement) or K and V split (without)
    tag = args.batch_bf16
    bf16_prec = pb.GP_BF16_SPLIT_V if tag == "v" else pb.GP_BF16_SPLIT_KV
    bf16_refresh = args.refresh if tag == "v" else 0
    bf16_mode = f"batched_graphs_autotuned_bf16_split_{tag}"
    for mode, tune, prec in (("batched_graphs", False, pb.GP_FP32), ("batched_graphs_autotuned", True, pb.GP_FP32),
                             (bf16_mode, True, bf16_prec)):
        for i, p in enumerate(probs):
            p["psi"].copy_(psi0[i])
        params.prec = prec
        params.refresh = bf16_refresh if prec != pb.GP_FP32 else 0
        batch = pb.Batch(probs, nr, params, seed=7000, probe_period=PROBE_PERIOD, iters_per_graph=8,
                         autotune=tune, streams=8)
        for t in range(args.warmup):
            batch.step(t, eps_t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(args.warmup, args.warmup + args.batch_steps):
            batch.step(t, eps_t)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[mode] = {"grad_estimates_per_s": B * args.batch_steps / el, "ms_per_step": 1e3 * el / args.batch_steps,
                     "stats": batch.stats(),
                     "psi_finite": bool(all(torch.isfinite(p["psi"]).all().item() for p in probs))}
        batch.close()
        print(json.dumps({mode: out[mode]}), file=sys.stderr, flush=True)
    out["steps"] = args.batch_steps
    # learned preconditioner per GP (basis at the chain's start, 128 Galerkin pairs, 1000 Adam
    # steps, all in the library's kernels; set-up untimed) + BF16 split-K+V products
    t_setup = time.perf_counter()
    hs_setup = pb.Handle(0, seed=11)
    k, H = 64, 256
    for i, p in enumerate(probs):
        p["psi"].copy_(psi0[i])
        d = p["X"].shape[1]
        U, _ = pb.precond_build_basis(hs_setup, p["X"], p["psi"], k)
        rr = np.random.default_rng(1000 + i)
        psis = torch.from_numpy(psi0[i].cpu().numpy() + LEARN_JITTER * rr.standard_normal((learn_pairs, d + 2))).cuda()
        Tg = pb.precond_targets(hs_setup, p["X"], p["y"], U, psis)
        I_, O_ = d + 2, 2 * k + 1
        prm = torch.zeros(pb.precond_mlp_size(I_, H, O_), dtype=torch.float32, device="cuda")
        pb.precond_mlp_init(hs_setup, prm, I_, H, O_, psis, Tg, seed=5)
        adam = torch.zeros(2 * pb.mlp_layout(I_, H, O_)["trainable"], dtype=torch.float32, device="cuda")
        pb.precond_mlp_train(hs_setup, prm, adam, I_, H, O_, psis, Tg, learn_epochs, 0, 2e-3)
        p["learned"] = {"mlp": prm, "hidden": H, "U": U,
                        "coef": torch.zeros(k + 1, dtype=torch.float64, device="cuda")}
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    mode = f"batched_graphs_autotuned_learned_bf16_split_{tag}"
    params.prec = bf16_prec
    params.refresh = bf16_refresh
    batch = pb.Batch(probs, nr, params, seed=7000, probe_period=PROBE_PERIOD, iters_per_graph=8,
                     autotune=True, streams=8)
    for t in range(args.warmup):
        batch.step(t, eps_t)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.warmup, args.warmup + args.batch_steps):
        batch.step(t, eps_t)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out[mode] = {"grad_estimates_per_s": B * args.batch_steps / el, "ms_per_step": 1e3 * el / args.batch_steps,
                 "stats": batch.stats(), "setup_s": t_setup, "rank": k, "hidden": H,
                 "psi_finite": bool(all(torch.isfinite(p["psi"]).all().item() for p in probs))}
    batch.close()
    print(json.dumps({mode: out[mode]}), file=sys.stderr, flush=True)
    params.prec = pb.GP_FP32
    params.refresh = 0
    u = out["unbatched"]["grad_estimates_per_s"]
    out["speedup_vs_unbatched"] = {m_: out[m_]["grad_estimates_per_s"] / u for m_ in
                                   ("batched_graphs", "batched_graphs_autotuned", bf16_mode, mode)}
    out["learn_pairs"], out["learn_epochs"] = learn_pairs, learn_epochs
    if emit:
        print(json.dumps({"batched": out}), flush=True)
    return out


def chains_bench(args, pb):
    """The paper's multi-chain protocol (Sec. 5) on the n = 16384, d = 8 workload: SGLD
    preconditioner M from the MAP on a random 500-point subset, scaled by 500 / n for the
    full data set (the posterior covariance shrinks like 1 / n); chains started from
    N(psi_MAP, M_subset) for dispersion; probes (4 per estimate and q = 1 as in the paper,
    or as given) redrawn every 20 steps with warm starts; all chains stepped together by gp_batch_*.  The step
    size is the one at which the Langevin-phase monitor (eps / 4) lambda_max(L^T V L) meets
    the freeze threshold 0.002, with V the covariance of 32 gradient estimates at psi_MAP:
    the step the paper's schedule freezes at.  Reports the PSRF over the second half of the
    run and the effective sample size of every chain there."""
    import numpy as np
    import torch
    import workloads
    from paper_1501_05427_amd import protocol
    n, d, nr, C, T = 16384, 8, args.chain_probes, args.chain_count, args.chain_steps
    w = workloads.rff_gp(n=n, d=d, seed=1)
    P = d + 2
    h = pb.Handle(0, seed=31)
    prior = {"kind": 1, "a": np.zeros(P), "b": np.full(P, 3.0)}
    t0 = time.perf_counter()
    psi_map, M_sub, _ = protocol.sgld_preconditioner(h, w["X"], w["y"], w["psi"], prior, n_sub=500, seed=0)
    t_map = time.perf_counter() - t0
    M_full = M_sub * (500.0 / n)
    L_full = np.linalg.cholesky(M_full)
    starts = protocol.init_chains(psi_map, M_sub, C, seed=1)
    X = torch.from_numpy(w["X"]).cuda()
    y = torch.from_numpy(w["y"]).cuda()
    Ld = torch.from_numpy(np.ascontiguousarray(L_full.T)).cuda()  # column-major lower factor
    pa = torch.zeros(P, dtype=torch.float64, device="cuda")
    pbb = torch.full((P,), 3.0, dtype=torch.float64, device="cuda")
    probs = [{"X": X, "y": y, "psi": torch.from_numpy(starts[c].copy()).cuda(), "M_chol": Ld,
              "prior": (1, pa, pbb)} for c in range(C)]
    params = pb.make_params(q=args.chain_q, rate=1.0, eps=1e-6, eps_relative=1, max_iter=2000, rng_stream=2)
    batch = pb.Batch(probs, nr, params, seed=500, probe_kind=pb.PROBE_GAUSSIAN, probe_period=PROBE_PERIOD,
                     iters_per_graph=8, autotune=True, streams=min(C, 8))
    # gradient-noise covariance at psi_MAP -> the step at the freeze threshold
    hv = pb.Handle(0, seed=77)
    psi_m = torch.from_numpy(psi_map.copy()).cuda()
    Sw = torch.zeros((1 + nr, n), dtype=torch.float64, device="cuda").t()
    G = []
    for k in range(33):
        params.rng_counter = 10_000 + k
        g_, _ = pb.gp_stoch_grad(hv, X, psi_m, y, params, n_probes=nr, S_warm=Sw)
        if k > 0:  # the first solve only warms the y system up
            G.append(g_.cpu().numpy())
    V = np.cov(np.array(G).T)
    lam_max = float(np.linalg.eigvalsh(L_full.T @ V @ L_full).max())
    eps = 4 * 0.002 / lam_max
    trace = np.empty((C, T, P))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(T):
        batch.step(t, eps)
        trace[:, t, :] = torch.stack([p["psi"] for p in probs]).cpu().numpy()
        if t % 200 == 199:
            print(f"chains: step {t + 1}/{T}, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    el = time.perf_counter() - t0
    half = trace[:, T // 2:, :]
    rhat = protocol.psrf(half)
    ess = np.array([protocol.ess(half[c]) for c in range(C)])
    out = {"chains": {"workload": "rff_n16384_d8", "n_chains": C, "steps": T, "probes": nr, "q": args.chain_q,
                      "subset": 500, "map_seconds": t_map, "psi_map": psi_map.tolist(),
                      "eps": eps, "langevin_lambda_max": lam_max,
                      "psi_truth": w["psi"].tolist(), "M_scale": 500.0 / n,
                      "seconds": el, "grad_estimates_per_s": C * T / el,
                      "psrf_second_half": rhat.tolist(), "psrf_max": float(rhat.max()),
                      "ess_second_half_min_per_chain": ess.min(axis=1).tolist(),
                      "ess_fraction_min": float(ess.min() / (T - T // 2)),
                      "posterior_mean_second_half": half.reshape(-1, P).mean(axis=0).tolist(),
                      "posterior_sd_second_half": half.reshape(-1, P).std(axis=0).tolist(),
                      "batch_stats": batch.stats()}}
    batch.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--learned-steps", type=int, default=None,
                    help="steps of each learned / Galerkin leg (default: --steps; 0 skips them)")
    ap.add_argument("--learn-chains", type=int, default=8,
                    help="plain-solver SGLD chains whose states train the network")
    ap.add_argument("--learn-chain-steps", type=int, default=32)
    ap.add_argument("--learn-chain-probes", type=int, default=4, help="probes of the training chains")
    ap.add_argument("--learn-chain-q", type=float, default=1.0, help="threshold q of the training chains' solver")
    ap.add_argument("--learn-pairs", type=int, default=256, help="error sweep: jittered training pairs")
    ap.add_argument("--learn-epochs", type=int, default=1500)
    ap.add_argument("--bf16-mode", choices=("kv", "v"), default="v",
                    help="BF16 legs: split V only (v, two products; on this workload, with residual "
                         "replacement, as accurate as kv and 7-9%% faster per estimate) or split K and V "
                         "(kv, three)")
    ap.add_argument("--refresh", type=int, default=3,
                    help="residual replacement of the BF16 legs: on a 2^refresh residual drop")
    ap.add_argument("--equal-error-reps", type=int, default=30, help="0 skips the equal-error leg")
    ap.add_argument("--equal-error-q", type=lambda t: [float(v) for v in t.split(",")], default=[1.0, 3.0, 10.0],
                    help="thresholds q of the preconditioned legs")
    ap.add_argument("--equal-error-q-plain", type=lambda t: [float(v) for v in t.split(",")],
                    default=[0.5, 1.0, 3.0], help="thresholds q of the plain leg")
    ap.add_argument("--equal-error-ref-batches", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="skip the compact batched leg of the main line")
    ap.add_argument("--profile-kmv", action="store_true")
    ap.add_argument("--pipes", action="store_true",
                    help="issue-rate probe of the VALU, exp and MFMA pipes, alone and together")
    ap.add_argument("--kmv-report", action="store_true",
                    help="K.V throughput per precision mode on each workload shape (separate report)")
    ap.add_argument("--cpu-report", action="store_true",
                    help="the oracle's CPU timings on one and on all threads (no GPU; separate report)")
    ap.add_argument("--profile-util", action="store_true",
                    help="a few launches of each hot kernel (and of the n = 16384, m = 17 product), "
                         "for rocprofv3 counter passes")
    ap.add_argument("--error-sweep", action="store_true",
                    help="gradient error vs estimates/s, plain FP32 vs learned + BF16 (separate report)")
    ap.add_argument("--sweep-reps", type=int, default=100)
    ap.add_argument("--workload", choices=["rff", "mixture"], default="rff",
                    help="rff: n = 65536, d = 8 (default); mixture: n = 131072, d = 16 (error sweep only)")
    ap.add_argument("--sweep-q", type=lambda t: [float(v) for v in t.split(",")], default=[0.3, 1.0, 3.0])
    ap.add_argument("--sweep-methods", type=lambda t: t.split(","), default=["plain_fp32", "learned_bf16"],
                    help="any of plain_fp32, plain_bf16, learned_fp32, learned_bf16")
    ap.add_argument("--ref-probes", type=int, default=1024)
    ap.add_argument("--batched", action="store_true",
                    help="64 chains over 64 GPs: batched graphs vs unbatched calls (separate report)")
    ap.add_argument("--batch-chains", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=20)
    ap.add_argument("--batch-only-graphs", action="store_true",
                    help="with --batched: time only the batched FP32 form (captured graphs, no autotuning)")
    ap.add_argument("--batch-bf16", choices=("kv", "v"), default="kv",
                    help="batched BF16 forms: K and V split (kv, no residual replacement) or V split "
                         "with residual replacement every 2^refresh (v; K rounded whole is indefinite "
                         "for many of these GPs, whose chains are then redone in FP32 step by step)")
    ap.add_argument("--chains", action="store_true",
                    help="the paper's multi-chain protocol with PSRF and ESS (separate report)")
    ap.add_argument("--chain-count", type=int, default=10)
    ap.add_argument("--chain-steps", type=int, default=6000)
    ap.add_argument("--chain-probes", type=int, default=4, help="probes per estimate (the paper: 4)")
    ap.add_argument("--chain-q", type=float, default=1.0, help="alpha = q sqrt(n) (the paper: 1)")
    ap.add_argument("--solver-study", action="store_true",
                    help="CG/ULISSE iterations, spread and gradient error against kappa (separate report)")
    ap.add_argument("--study-lambdas", type=lambda t: [float(v) for v in t.split(",")],
                    default=[1.0, 0.1, 0.01, 1e-3, 1e-4])
    ap.add_argument("--study-reps", type=int, default=30)
    ap.add_argument("--study-probes", type=int, default=1, help="probes per gradient estimate (Fig. 4: 1)")
    ap.add_argument("--study-ref-batches", type=int, default=8)
    ap.add_argument("--study-max-iter", type=int, default=20000)
    args = ap.parse_args()
    if args.learned_steps is None:
        args.learned_steps = args.steps
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(its kernels run one GPU's share of the work; the rows would shard across GPUs)", file=sys.stderr)
        sys.exit(2)

    if args.cpu_report:
        cpu_baseline_report()
        return

    import numpy as np
    import torch

    import workloads
    from paper_1501_05427_amd import binding as pb

    if not os.path.exists(pb.LIB_PATH):
        from paper_1501_05427_amd import build as _b
        _b.build()
    torch.cuda.init()
    global N, D, WORKLOAD
    if args.workload == "mixture":
        # the learned-part configuration: 8-Gaussian mixture inputs, n = 131072, d = 16
        if not args.error_sweep:
            print("--workload mixture is measured by --error-sweep only", file=sys.stderr)
            sys.exit(2)
        N, D, WORKLOAD = 131072, 16, "mixture_n131072_d16_m32"
        w = workloads.mixture(n=N, d=D, seed=4)
    else:
        w = workloads.rff_gp(n=N, d=D, seed=2)
    X = torch.from_numpy(w["X"]).cuda()
    psi0 = torch.from_numpy(w["psi"]).cuda()
    y = torch.from_numpy(w["y"]).cuda()
    h = pb.Handle(0, seed=2015)

    if args.kmv_report:
        kmv_report(pb, h)
        return
    if args.pipes:
        pipes_report(pb, h)
        return
    if args.error_sweep:
        error_sweep(args, pb, h, X, y, w, psi0)
        return
    if args.solver_study:
        solver_study(args, pb, h)
        return
    if args.batched:
        batched_bench(args, pb)
        return
    if args.chains:
        chains_bench(args, pb)
        return

    if args.profile_util:
        # the hot kernels of both paths, a few launches each, for counter passes
        V = pb.colmajor(N, M)
        V.copy_(torch.from_numpy(workloads.gaussian_matrix(N, M, seed=11)).cuda())
        out = pb.colmajor(N, M)
        for prec in (pb.GP_FP32, pb.GP_BF16_SPLIT_KV, pb.GP_BF16_SPLIT_V):
            for _ in range(3):
                pb.gp_kmv(h, X, psi0, V, out=out, prec=prec)
        # the n = 16384, d = 8 shape with y + 16 probes (one MFMA block, one VALU column)
        w2 = workloads.rff_gp(n=16384, d=8, seed=1)
        X2, psi2 = torch.from_numpy(w2["X"]).cuda(), torch.from_numpy(w2["psi"]).cuda()
        V2 = pb.colmajor(16384, 17)
        V2.copy_(torch.from_numpy(workloads.gaussian_matrix(16384, 17, seed=12)).cuda())
        for _ in range(3):
            pb.gp_kmv(h, X2, psi2, V2)
        R = pb.colmajor(N, NPROBES)
        R.copy_(V[:, 1:])
        S_warm = torch.zeros((M, N), dtype=torch.float64, device="cuda").t()
        for prec in (pb.GP_FP32, pb.GP_BF16_SPLIT_KV):
            params = pb.make_params(q=1.0, rate=1.0, eps=1e-6, eps_relative=1, max_iter=1000)
            params.prec = prec
            for _ in range(2):
                pb.gp_stoch_grad(h, X, psi0, y, params, R=R, S_warm=S_warm)
        torch.cuda.synchronize()
        print(json.dumps({"profile_util": "done"}), flush=True)
        return

    if args.profile_kmv:
        V = pb.colmajor(N, M)
        V.copy_(torch.from_numpy(workloads.gaussian_matrix(N, M, seed=11)).cuda())
        out = pb.colmajor(N, M)
        for _ in range(5):
            pb.gp_kmv(h, X, psi0, V, out=out)
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"profile_kmv": "done", "copy_bytes": a.numel() * 4,
                          "kmv_source_sha256_16": kmv_source_hash()}), flush=True)
        return

    rec = main_line(args, pb, h, X, y, w, psi0)
    if not args.no_batched:
        # the batched forms on 64 GPs (n 2048 to 32768, d 2 to 16; inputs with 256 random
        # features to keep their generation short); 3 + 20 steps span one probe redraw
        try:
            sv = (args.batch_steps, args.warmup)
            args.batch_steps, args.warmup = 20, 3
            bt = batched_bench(args, pb, n_features=256, learn_pairs=128, learn_epochs=1000, emit=False)
            args.batch_steps, args.warmup = sv
            rec["batched_64_gps"] = {
                "workload": bt["workload"], "steps": bt["steps"],
                "grad_estimates_per_s": {k: bt[k]["grad_estimates_per_s"] for k in
                                         ("unbatched", "batched_graphs", "batched_graphs_autotuned",
                                          f"batched_graphs_autotuned_bf16_split_{args.batch_bf16}",
                                          f"batched_graphs_autotuned_learned_bf16_split_{args.batch_bf16}")},
                "speedup_vs_unbatched": bt["speedup_vs_unbatched"]}
        except Exception as e:  # the main line must still be printed
            rec["batched_64_gps"] = {"error": repr(e)}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w["X"], w["psi"], rec["kmv_passes_per_estimate"])
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
