/*
 * ulisse_gp.h -- C ABI of the MI355X (gfx950) library for the hot path of SGLD with the
 * ULISSE solver for Gaussian-process covariance parameters (Filippone & Engler, ICML 2015).
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers unless stated otherwise.  The caller owns them;
 *     the library never returns memory it allocated.  The handle owns only its workspace
 *     (grown on demand with hipMalloc), a pinned host word used to follow the solver,
 *     and the RNG seed.
 *   - Work is ordered on `stream` (a hipStream_t passed as void*; NULL = default stream).
 *     gp_kmv, gp_dkmv, sgld_step, gp_draw_probes and gp_philox only enqueue work.
 *     ulisse_solve and gp_stoch_grad enqueue work and also wait on the host for the
 *     solver's per-iteration "systems still running" count, because the length of the
 *     randomly truncated series is only known on the device; their outputs are still
 *     delivered in stream order.
 *   - Inputs X (n x d) are row-major FP32 with leading dimension ldx >= d.  Vectors and
 *     multi-right-hand-side blocks are column-major: column c of V starts at V + c*ldv.
 *   - Log-parameters psi are FP64 on the device, in the fixed order
 *       psi = (log sigma^2, log ell_1, ..., log ell_d, log lambda),  P = d + 2.
 *   - Validation is synchronous: bad sizes, null or misaligned pointers return GP_EINVAL;
 *     a failed HIP call or launch returns GP_EDEVICE; in both cases gp_last_error() gives
 *     a message.  Numerical outcomes of the solver (no convergence within max_iter,
 *     breakdown) are reported per system in ulisse_sysstat.flags, never as return codes.
 *   - One handle per host thread.  Limits: 1 <= n <= 2^26, 1 <= d <= 16, 1 <= m <= 64.
 */
#ifndef ULISSE_GP_H
#define ULISSE_GP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_handle gp_handle;

typedef enum {
    GP_OK = 0,
    GP_EINVAL = -1,
    GP_ENOMEM = -2,
    GP_EDEVICE = -3,
    GP_EUNSUPPORTED = -4
} gp_status;

/* Arithmetic of the K-tile x V contraction on the MFMA path (m >= 16 right-hand sides).
 * GP_FP32: K entries and products in FP32 (v_mfma_f32_16x16x4f32).
 * GP_BF16_SPLIT_V: K rounded to BF16, V split as V_hi + V_lo (both BF16), FP32
 * accumulation (v_mfma_f32_16x16x32_bf16): relative error per product term <= 2^-9.
 * GP_BF16_SPLIT_KV: K and V both split, K_hi V_hi + K_hi V_lo + K_lo V_hi: relative error
 * per product term about 3 * 2^-18.
 * Distances and exponentials are FP32 in every mode; with fewer than 16 right-hand sides
 * the contraction is FP32 whatever the mode (on the VALU, or in GP_FP32 as one zero-padded
 * MFMA block of the symmetric product).  Where the products run in a BF16 mode, the G tiles
 * of gp_stoch_grad's gradient reduction come from split BF16 operands too; its sums are
 * FP32 within a tile and FP64 across tiles. */
typedef enum { GP_FP32 = 0, GP_BF16_SPLIT_V = 1, GP_BF16_SPLIT_KV = 2 } gp_precision;

/* Inputs x_1..x_n, row-major FP32, device memory. */
typedef struct {
    const float* X;
    int64_t n;
    int32_t d;
    int64_t ldx;
} gp_data;

/* Create a handle on HIP device `device`.  `seed` is the first Philox key word of every
 * draw the library makes (probes, ULISSE uniforms, SGLD noise). */
gp_status gp_create(gp_handle** h, int device, uint64_t seed);
void gp_destroy(gp_handle* h);
/* Message of the last failure on this host thread ("" if none).  Owned by the library. */
const char* gp_last_error(void);

/*
 * Covariance matrix-vector products (Sec. 3: the CMVP, O(n^2) time and O(n) memory, K is
 * never stored).  out = K(psi) V, in the arithmetic chosen by prec, with
 *   K_ij = sigma^2 exp(-1/2 sum_k (x_ik - x_jk)^2 / ell_k^2) + lambda delta_ij
 * (the covariance function of Sec. 2 in its ARD form).  V is n x m (ldv >= n), out is
 * n x m (ldo >= n); out must not overlap V.  Tiles of K are rebuilt from X on the fly.
 */
gp_status gp_kmv(gp_handle* h, gp_data X, const double* psi, const float* V, int32_t m,
                 int64_t ldv, float* out, int64_t ldo, gp_precision prec, void* stream);

/*
 * gp_kmv for callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  Same arguments, results and
 * conventions as gp_kmv, but every intermediate buffer (scaled inputs, packed V, split-K
 * partials, BF16 halves) lives in one fixed device array of the library, 32 MiB per
 * device, held from the first call on a device until the process ends; the call makes no
 * allocation and uses none of the handle's workspace (the handle only names the device).
 * A shape whose buffers do not fit even with a single split-K chunk is rejected with
 * GP_EINVAL (at n = 65536, d = 8: up to m = 51 fits in FP32, m = 32 in the BF16 modes).
 * Calls that overlap on one device
 * share that array and race: order them on one stream.
 */
gp_status gp_kmv_noalloc(gp_handle* h, gp_data X, const double* psi, const float* V, int32_t m,
                         int64_t ldv, float* out, int64_t ldo, gp_precision prec, void* stream);

/*
 * Products with every derivative of K (used by the exact gradient of Sec. 2.1):
 *   block j of out (j = 0..d+1) = dK/dpsi_j V, at out + j*block_stride, n x m, ldo >= n,
 *   dK/dpsi_0 = K_f (signal part), dK/dpsi_k = K_f o (x_.k - x_.k)^2 / ell_k^2,
 *   dK/dpsi_{d+1} = lambda I.  block_stride >= ldo*m.  FP32 only (prec must be GP_FP32).
 */
gp_status gp_dkmv(gp_handle* h, gp_data X, const double* psi, const float* V, int32_t m,
                  int64_t ldv, float* out, int64_t ldo, int64_t block_stride,
                  gp_precision prec, void* stream);

/* Parameters of one ULISSE solve (Sec. 3.1 Alg. 1 and Sec. 4). */
typedef struct {
    double q;               /* early-stop threshold alpha = q sqrt(n)                      */
    double rate;            /* weights w_r = exp(rate r); the paper's experiments: 1      */
    double eps;             /* CG convergence: ||e||_2 < eps (or eps ||b||_2, see below)   */
    int32_t eps_relative;   /* 1: threshold eps ||b||_2 per system; 0: absolute eps        */
    int32_t max_iter;       /* T of Alg. 1: at most this many products K d per system     */
    int32_t two_track_first;/* 1: system 0 keeps two estimates drawn independently        */
    int32_t refresh;        /* residual replacement, k in [1, 30]: after an iteration whose
                               residual norm has fallen below 2^-k of its value at the last
                               replacement (or the start) and is above the convergence
                               threshold, the recursive residual is replaced by b - K s
                               computed with an FP32 product and the iteration restarts
                               from it (next direction = residual); a replacement that gains
                               less than 2x ends the replacements of that system.  Removes
                               the bias that BF16 products leave in the limit of the
                               iterates (Sec. 3.2 on reduced precision).  0: never         */
    uint64_t rng_stream;    /* second Philox key word                                       */
    uint64_t rng_counter;   /* step word of the Philox counter                              */
    gp_precision prec;      /* arithmetic of the products K d; in the BF16 modes the G tiles
                               of the gradient reduction (gp_stoch_grad*) also come from
                               split BF16 (hi + lo) operands                               */
} ulisse_params;

/* Preconditioner for the CG iterations under ULISSE (the preconditioned variant of
 * Sec. 3.3 with a fixed preconditioner; the series of Sec. 4 stays unbiased for any CG
 * variant):  P^-1 v = tau_inv v + U (h o (U^T v)), i.e. P = U diag(d) U^T + tau (I - U U^T)
 * with h_kappa = 1/d_kappa - tau_inv for orthonormal U.  U: n x k FP32 device, column-major
 * with ld ldu >= n, k in {16, 32, 64}.  coef: k + 1 FP64 device values, h_0..h_{k-1}
 * then tau_inv.  P must be SPD (d_kappa > 0, tau_inv > 0).  The residual norms that set l
 * and the convergence test stay unpreconditioned (||b - K s||_2).
 * Fallback: a negative tau_inv (precond_from_mlp writes -1 when the network output is
 * unusable) makes every solve over this descriptor the plain CG of Alg. 1 (P = I, the
 * warm start below unused) and sets ULISSE_FALLBACK in the statistics of every system.
 * Warm start: with warm_start = 1, system 0 (y in gp_stoch_grad_pc) starts from s0 = U c,
 * c = k FP64 device values (the network's warm-start coefficients), instead of its column
 * of S0 / S_warm. */
typedef struct {
    const float* U;
    int64_t ldu;
    int32_t k;
    int32_t warm_start;
    const double* coef;
    const double* c;
} gp_precond;

/* Per-system outcome, written by the device.  J_b = -1 for a single-track system. */
typedef struct {
    int32_t l;       /* first iteration with ||e|| below alpha (0: never reached)           */
    int32_t J_a;     /* last kept tail index of track a                                     */
    int32_t J_b;     /* last kept tail index of track b                                     */
    int32_t iters;   /* products K d taken (excluding the warm-start residual)              */
    double final_res;/* ||e|| of Alg. 1's recursive residual at the last iteration         */
    uint32_t flags;  /* ULISSE_NOTCONV | ULISSE_BREAKDOWN | ULISSE_FALLBACK | ULISSE_FP32_RERUN */
    uint32_t pad;
} ulisse_sysstat;

#define ULISSE_NOTCONV 1u    /* max_iter reached before the series ended (biased estimate) */
#define ULISSE_BREAKDOWN 2u  /* d^T K d <= 0 or a non-finite scalar; the system stopped    */
#define ULISSE_FALLBACK 4u   /* the preconditioner was unusable: the plain solver ran       */
/* A solve in a BF16 mode in which some system broke down was run again in FP32, every
 * system of it, from the same warm starts with the same draws (ulisse_solve*,
 * gp_stoch_grad*, and a batch's chains): rounded to BF16, K can lose its positive
 * definiteness where its smallest eigenvalue is below the rounding error
 * (GP_BF16_SPLIT_V: 2^-9 of each entry).  The outcome, flags aside, is that of the same
 * call in GP_FP32 with refresh = 0.  Deciding it reads a count back: these calls then
 * return with their stream synchronised.                                               */
#define ULISSE_FP32_RERUN 8u

/*
 * Unbiased solves K s = b_c for the m columns of B (n x m FP32, ldb >= n) by the ULISSE
 * series over one CG run per system (Sec. 4).  S0 (n x m FP64, ld n) is the warm start,
 * NULL for zero.  Output S_tilde is n x (m + two_track_first) FP64 with ld n: with
 * two_track_first, columns 0 and 1 are the two estimates for system 0 and column c+1
 * holds system c >= 1; otherwise column c holds system c.  S_cg (nullable, n x m FP64,
 * ld n) receives each system's last CG iterate, the vector to warm-start a later solve
 * with.  stats: m entries, device memory (nullable).
 * The u_j of system c, track t are Philox words j of key (seed, rng_stream) and counter
 * (j/4, 2c+t, 2, rng_counter).
 */
gp_status ulisse_solve(gp_handle* h, gp_data X, const double* psi, const float* B,
                       int32_t m, int64_t ldb, const double* S0, const ulisse_params* params,
                       double* S_tilde, double* S_cg, ulisse_sysstat* stats, void* stream);

/* ulisse_solve over preconditioned CG (pc non-null; same conventions otherwise). */
gp_status ulisse_solve_pc(gp_handle* h, gp_data X, const double* psi, const float* B,
                          int32_t m, int64_t ldb, const double* S0, const ulisse_params* params,
                          const gp_precond* pc, double* S_tilde, double* S_cg,
                          ulisse_sysstat* stats, void* stream);

/* The PCG variant of Sec. 3.3 whose preconditioner is J = K + delta I (delta > 0), applied
 * to each residual by an inner run of Alg. 1 on (K + delta I) z = e from z = 0.  The inner
 * run stops at ||r|| < eps_inner ||e|| (relative; eps_inner = 0 never stops early) or after
 * max_inner products, whichever comes first; it takes no ULISSE truncation, its products use
 * prec_inner, and its right-hand side is e rounded to FP32.  Since CG is not linear in its
 * right-hand side, an inner run that stops early applies a slightly different operator at
 * every outer iteration; the outer series stays unbiased either way (it only needs the
 * iterates to converge).  Each outer iteration waits on the host for the inner run.  The
 * outer iteration count (stats.iters) excludes the inner products. */
typedef struct {
    double delta;         /* shift of J = K + delta I, > 0                                 */
    double eps_inner;     /* inner relative tolerance, >= 0                                 */
    int32_t max_inner;    /* inner products per application, >= 1                           */
    gp_precision prec_inner;
} gp_shift_precond;

/* ulisse_solve over PCG with J = K + delta I (sp non-null; same conventions otherwise). */
gp_status ulisse_solve_shift_pc(gp_handle* h, gp_data X, const double* psi, const float* B,
                                int32_t m, int64_t ldb, const double* S0,
                                const ulisse_params* params, const gp_shift_precond* sp,
                                double* S_tilde, double* S_cg, ulisse_sysstat* stats,
                                void* stream);

/*
 * One unbiased estimate of the gradient of log p(y | psi, X) with respect to psi
 * (eq. gradient:unbiased with the two-estimate quadratic term of Sec. 4.1):
 *   g_j = 1/2 s_a^T dK_j s_b - 1/(2 N_r) sum_c r_c^T dK_j s_c.
 * y: n FP32.  R: n x n_probes FP32 (ld n), or NULL to draw the probes with key
 * (seed, rng_stream) and counter (i/4, c, 1, rng_counter) -- probe_kind 0 Gaussian
 * (Box-Muller), 1 Rademacher.  S_warm (nullable, n x (1 + n_probes) FP64, ld n): warm
 * starts in, last CG iterates out; when R is NULL only its column 0 (y) is used as a warm
 * start, because freshly drawn probes make the old probe solutions useless.
 * g: d + 2 FP64 (device).  stats: 1 + n_probes entries (nullable).
 */
gp_status gp_stoch_grad(gp_handle* h, gp_data X, const double* psi, const float* y,
                        const float* R, int32_t n_probes, int32_t probe_kind,
                        const ulisse_params* params, double* S_warm, double* g,
                        ulisse_sysstat* stats, void* stream);

/* gp_stoch_grad with its solves over preconditioned CG (pc non-null). */
gp_status gp_stoch_grad_pc(gp_handle* h, gp_data X, const double* psi, const float* y,
                           const float* R, int32_t n_probes, int32_t probe_kind,
                           const ulisse_params* params, const gp_precond* pc, double* S_warm,
                           double* g, ulisse_sysstat* stats, void* stream);

/* gp_stoch_grad with its solves over PCG with J = K + delta I (sp non-null). */
gp_status gp_stoch_grad_shift_pc(gp_handle* h, gp_data X, const double* psi, const float* y,
                                 const float* R, int32_t n_probes, int32_t probe_kind,
                                 const ulisse_params* params, const gp_shift_precond* sp,
                                 double* S_warm, double* g, ulisse_sysstat* stats,
                                 void* stream);

/* Prior on psi: kind 0 flat; kind 1 psi_j ~ N(a_j, b_j^2); kind 2 exp(psi_j) ~ Gamma(shape
 * a_j, rate b_j) with the Jacobian of the log transform.  a, b: P FP64 device (NULL for
 * kind 0). */
typedef struct {
    int32_t kind;
    int32_t reserved;
    const double* a;
    const double* b;
} gp_prior;

/*
 * SGLD update of Sec. 2.1, in place on psi (P = d + 2 FP64 device):
 *   psi += eps_t/2 M (g + grad log p(psi)) + sqrt(eps_t) L xi,   M = L L^T,
 * with L = M_chol (P x P lower-triangular, column-major FP64 device; NULL = identity) and
 * xi standard normals from key (seed, rng_stream), counter (i/4, 0, 3, rng_counter).
 */
gp_status sgld_step(gp_handle* h, int32_t P, double* psi, const double* g,
                    const gp_prior* prior, const double* M_chol, double eps_t,
                    uint64_t rng_stream, uint64_t rng_counter, void* stream);

/* Probe matrix R (n x n_probes FP32, ld ldr >= n) as drawn by gp_stoch_grad. */
gp_status gp_draw_probes(gp_handle* h, int64_t n, int32_t n_probes, int32_t probe_kind,
                         uint64_t rng_stream, uint64_t rng_counter, float* R, int64_t ldr,
                         void* stream);

/* Raw Philox4x64-10 blocks (Salmon et al., SC 2011): out[4b + w] = word w of the block at
 * counter (first_block + b, w1, w2, w3) with key (k0, k1).  out: 4 * nblocks uint64 device. */
gp_status gp_philox(uint64_t k0, uint64_t k1, uint64_t first_block, uint64_t w1, uint64_t w2,
                    uint64_t w3, int64_t nblocks, uint64_t* out, void* stream);

/*
 * The paper's SGLD protocol (Sec. 2.1 and Sec. 5.1) run on the device for steps
 * t = state->t, ..., state->t + T - 1 of one chain:
 *   - probes redrawn every `probe_period` steps (key (seed, params->rng_stream), counter
 *     (i/4, c, 1, t / probe_period)); each system is warm started from its last CG iterate
 *     and the probe columns restart from zero when the probes change;
 *   - g_t = gp_stoch_grad with the ULISSE draws of step t (params->rng_counter = t);
 *   - step size eps_t = a (b + t)^(-gamma) until frozen (the decreasing schedule of
 *     Sec. 2.1 and Sec. 5.1);
 *   - psi += eps_t/2 M (g_t + grad log p) + sqrt(eps_t) L xi_t (SGLD noise counter t);
 *   - after every `batch` steps, V = sample covariance of the batch's gradients and the
 *     Langevin-phase ratio (eps_t / 4) lambda_max(L^T V L) (= the ratio of Sec. 2.1 with
 *     M = L L^T); the first ratio below `freeze_ratio` freezes eps at its current value.
 * Outputs (device, caller-owned): trace T x P (psi after each step, row t), eps_trace T,
 * ratio_trace floor(T / batch) (nullable each).  Work arrays (device, caller-owned, kept
 * between calls of one chain): S_warm n x (1 + n_probes) FP64 and R n x n_probes FP32,
 * both ld n.  state (host memory) carries t and the freeze across calls, so a chain can be
 * resumed; with counter-based draws a resumed chain is bit-identical to an uninterrupted
 * one.  probe_period >= 1, batch >= 2, T >= 0.
 */
typedef struct {
    double a, b, gamma;      /* eps_t = a (b + t)^(-gamma)                             */
    double freeze_ratio;     /* 0.002 in the paper's experiments                        */
    int32_t batch;           /* gradients per covariance estimate (100 in the paper)    */
    int32_t probe_period;    /* 20 in the paper                                         */
    int32_t n_probes;
    int32_t probe_kind;      /* 0 Gaussian, 1 Rademacher                               */
} sgld_schedule;

typedef struct {
    int64_t t;               /* next step index                                        */
    int32_t frozen;          /* eps frozen                                             */
    int32_t frozen_at;       /* step at which it froze (-1 if not)                      */
    double eps_frozen;
} sgld_state;

gp_status sgld_run(gp_handle* h, gp_data X, double* psi, const float* y,
                   const ulisse_params* params, const gp_prior* prior, const double* M_chol,
                   const sgld_schedule* sched, sgld_state* state, int32_t T, double* S_warm,
                   float* R, double* trace, double* eps_trace, double* ratio_trace,
                   void* stream);

/*
 * Learned warm start and preconditioner.  A fixed orthonormal basis U (n x k) and a small
 * network psi -> (c, log d, log tau) give, for every psi of the chain,
 *   s0 = U c  (warm start of the y system) and  P^-1 = tau^-1 I + U diag(1/d - 1/tau) U^T
 * (the preconditioned variant of Sec. 3.3 with a fixed P; the series of Sec. 4 stays
 * unbiased for any SPD P, so the network changes only the cost of the solves).
 *
 * precond_build_basis: randomized range finder of K(psi_ref) with one power step
 *   (Omega from Philox purpose 4), CholeskyQR2 in FP64, Rayleigh-Ritz rotation; writes U
 *   (n x k FP32, ld ldu >= n) and the Ritz values (k FP64, decreasing).  k in {16, 32, 64}.
 * precond_targets: for N log-parameter vectors psis (N x P FP64 row-major, device) the
 *   Galerkin targets (N x (2k + 1) FP32 row-major): c = T^-1 U^T y, log diag T and
 *   log tau, tau = (tr K - tr T) / (n - k), with T = U^T K(psi) U.
 * MLP in -> hidden (tanh) -> hidden (tanh) -> out, FP32 parameters in one buffer of
 *   precond_mlp_size(in, hidden, out) floats (weights, biases, then input/target
 *   standardisation constants); hidden <= 1024.
 * precond_mlp_init: standardisation constants from (psis, targets), Xavier-normal weights
 *   (Philox purpose 5, key (seed, 0)), zero biases.
 * precond_mlp_train: `steps` full-batch Adam steps (beta 0.9 / 0.999, eps 1e-8, learning
 *   rate lr) on the mean squared error of the standardised targets; adam: 2 x trainable
 *   floats (moments, zero at the first step); first_step = number of steps already taken;
 *   loss_trace (nullable) receives the loss before each step.
 * precond_mlp_forward: outputs (B x out, standardised) for B inputs, FP32 or, with bf16,
 *   BF16 operands and FP32 accumulation.
 * precond_mlp_grad: loss and gradient of the trainable parameters (for checks).
 * precond_from_mlp: BF16 forward at one psi (device, P) -> coef (k + 1 FP64: h, tau_inv;
 *   d is floored at tau so P stays SPD) and, if non-null, c (k FP64).  If any output is
 *   not finite, or a log d or log tau lies outside [-60, 60], the output is rejected: coef
 *   becomes h = 0, tau_inv = -1 (the fallback marker of gp_precond: the plain solver runs)
 *   and c = 0.  Everything happens on the device, so the call never waits.
 * precond_from_targets: the same coefficients (and rejection rule) from one row of
 *   precond_targets (2k + 1 FP32: c, log d, log tau) instead of the network: the Galerkin
 *   preconditioner computed directly at a psi, without learning.
 * precond_warm_start: s0 = U c (n FP64).
 */
gp_status precond_build_basis(gp_handle* h, gp_data X, const double* psi_ref, int32_t k,
                              float* U, int64_t ldu, double* ritz, void* stream);
gp_status precond_targets(gp_handle* h, gp_data X, const float* y, const float* U, int64_t ldu,
                          int32_t k, const double* psis, int32_t N, float* targets, void* stream);
int64_t precond_mlp_size(int32_t in, int32_t hidden, int32_t out);
gp_status precond_mlp_init(gp_handle* h, float* params, int32_t in, int32_t hidden, int32_t out,
                           const double* psis, const float* targets, int32_t N, uint64_t seed,
                           void* stream);
gp_status precond_mlp_train(gp_handle* h, float* params, float* adam, int32_t in, int32_t hidden,
                            int32_t out, const double* psis, const float* targets, int32_t N,
                            int32_t steps, int32_t first_step, float lr, float* loss_trace,
                            void* stream);
gp_status precond_mlp_forward(gp_handle* h, const float* params, int32_t in, int32_t hidden,
                              int32_t out, const double* psis, int32_t B, float* Y, int32_t bf16,
                              void* stream);
gp_status precond_mlp_grad(gp_handle* h, const float* params, int32_t in, int32_t hidden,
                           int32_t out, const double* psis, const float* targets, int32_t N,
                           float* grad, float* loss, void* stream);
gp_status precond_from_mlp(gp_handle* h, const float* params, int32_t in, int32_t hidden,
                           int32_t out, const double* psi, int32_t k, double* coef, double* c,
                           void* stream);
gp_status precond_from_targets(gp_handle* h, const float* targets, int32_t k, double* coef,
                               double* c, void* stream);
gp_status precond_warm_start(gp_handle* h, const float* U, int64_t ldu, int32_t k, int64_t n,
                             const double* c, double* s0, void* stream);

/*
 * Batched SGLD: B independent chains, each over its own GP (own X, n, d, y), advanced one
 * SGLD step per gp_batch_step call with the protocol of sgld_run (probes redrawn every
 * probe_period steps with warm starts from the last CG iterates; Sec. 5).  Chain b draws
 * with Philox key (seed + b, rng_stream): its probes, uniforms and SGLD noise are those of
 * gp_draw_probes (counter t / probe_period), gp_stoch_grad (counter t) and sgld_step
 * (counter t) on a handle created with seed + b, so a batched step reproduces the unbatched
 * calls exactly.
 *
 * The first step runs eagerly (sizing every workspace and, with autotune, timing the
 * product shapes); later steps replay graphs captured once: set-up (probes, right-hand
 * sides, initial residuals), a chunk of iters_per_graph solver iterations for every chain
 * (replayed until no system of any chain is running: as many replays as the last step of
 * the same kind needed are queued at once, each followed by a device count of the running
 * systems, so the host usually waits once per step), then the gradient reduction and the
 * SGLD update of every chain.  In the BF16 modes a chain whose solve broke down is then
 * taken back to where its step began and its step redone outside the graphs in FP32 with
 * the same draws, as gp_stoch_grad does (ULISSE_FP32_RERUN), so a batch still reproduces
 * the unbatched calls; each chain's psi and warm starts are copied at the start of every
 * step for that (in the BF16 modes the batch holds d + 2 + n (1 + n_probes) FP64 values of
 * device memory per chain for these copies, and a second handle for the reruns).  The chains
 * are spread over `streams` side streams, so the small ones run alongside the large ones.
 * The step index and step size are read by the kernels from device memory, so the graphs
 * never change.
 *
 * Every pointer of every problem is device memory owned by the caller and must stay valid,
 * at the same address, for the batch's lifetime: X (n x d, ld ldx), y (n), psi (d + 2,
 * in/out), S_warm (n x (1 + n_probes) FP64, ld n, zero at the start), R (n x n_probes FP32,
 * ld n; the batch writes it), g (d + 2, out), stats (1 + n_probes entries, nullable),
 * M_chol (nullable = I), prior as for sgld_step.  iters_per_graph: even, >= 2.  With mlp
 * set, the chain's solves run over the learned preconditioner (gp_stoch_grad_pc); the
 * shifted preconditioner is not available in a batch.
 */
typedef struct {
    gp_data X;
    const float* y;
    double* psi;
    double* S_warm;
    float* R;
    double* g;
    ulisse_sysstat* stats;
    const double* M_chol;
    gp_prior prior;
    /* Learned preconditioner (optional, mlp = NULL for none): a network trained by
     * precond_mlp_train for this GP (in = d + 2, hidden, out = 2k + 1), the basis U of
     * precond_build_basis (n x k, ld ldu) and coef (k + 1 FP64, written by the batch every
     * step from the network at the chain's psi, as precond_from_mlp does). */
    const float* mlp;
    int32_t mlp_hidden;
    int32_t k;
    const float* U;
    int64_t ldu;
    double* coef;
} gp_batch_problem;

typedef struct gp_batch gp_batch;

typedef struct {
    int64_t eager_steps;       /* steps run without graphs                              */
    int64_t graph_steps;       /* steps run by graph replays                            */
    int64_t iteration_graphs;  /* replays of the solver-iteration graph (queued ones    */
                               /* that found every system stopped included)             */
    int64_t captures;          /* graphs captured                                       */
    int64_t fp32_reruns;       /* chain steps redone in FP32 after a BF16 breakdown     */
} gp_batch_stats;

gp_status gp_batch_create(gp_batch** b, int device, uint64_t seed, int32_t B,
                          const gp_batch_problem* problems, int32_t n_probes, int32_t probe_kind,
                          int32_t probe_period, const ulisse_params* params,
                          int32_t iters_per_graph, int32_t autotune, int32_t streams);
/* One SGLD step (step index t, step size eps_t) of every chain, ordered after prior work on
 * `stream`; returns when the step is complete. */
gp_status gp_batch_step(gp_batch* b, uint64_t t, double eps_t, void* stream);
gp_status gp_batch_read_stats(const gp_batch* b, gp_batch_stats* out);
void gp_batch_destroy(gp_batch* b);

/*
 * Shape of the covariance products.  A shape code names how a product of K by V is split
 * into work: 0 = the symmetric product (row tiles of 256 rows against column chunks; each
 * entry of K off the diagonal tiles is built once and used for its row and, through a
 * transposed product, for its column; n >= 1793; FP32 with at most 17 or with 21 to 33
 * right-hand sides (under 16 as one zero-padded block of 16), BF16 modes with 17 to 32; its
 * partials, (1 + n/cs + n/256) mp n floats, within 24 GiB: n up to about 213000 at 32
 * right-hand sides); c > 0 = the split-K product
 * whose number of column chunks gives about c
 * workgroups (chunk partials reduced in FP64 in a fixed order).  Both give the same values
 * to FP32 rounding, not bit for bit.
 *
 * The code a product takes is, per shape key (n rounded up to 256, d, padded column count,
 * precision) on this handle: the pin set by gp_tune_set, else, with gp_autotune(h, 1), the
 * autotuner's entry, else the default (symmetric where it applies and was measured faster:
 * from 16 right-hand sides on, for d >= 12 always; for d <= 11 FP32 with one MFMA block of
 * right-hand sides or n >= 32768, BF16 with 17 to 32 right-hand sides and n >= 32768; below
 * 16, FP32 with m + d >= 12 and n >= 16129; else split-K for 2048 workgroups, or below 16
 * right-hand sides for 8192 with at most 32 chunks per row tile).  With the autotuner on,
 * the first product of a key without an entry times the candidates (the symmetric product
 * where it applies; split-K for 256 to 8192 workgroups, at most 64 chunks) on the stream and
 * keeps the fastest; that first call synchronises the stream.
 *
 *   gp_tune_set     pins code (>= 0) for the key of (n, d, m, prec), or removes the pin
 *                   (code -1).  GP_EINVAL for code 0 where the symmetric product does not
 *                   apply, or a code above 2^20.
 *   gp_tune_get     the code (-1: not tuned yet, the next product times it) and the number
 *                   of split-K chunks (1 for the symmetric product, 0 for -1) used now.
 *   gp_tune_save    writes the autotuner's entries (not the pins) as text: a header line,
 *                   then one "n_pad d mp prec code" line per key.
 *   gp_tune_load    reads such a file into the autotuner's entries (used while the
 *                   autotuner is on, which then times none of those keys).  All or nothing:
 *                   GP_EINVAL names the first malformed line and leaves the handle as it was.
 *   gp_autotune_split  the chunk count only (kept for older callers).
 * Host-only calls: none of them touches the device.
 */
gp_status gp_autotune(gp_handle* h, int32_t enable);
gp_status gp_autotune_split(gp_handle* h, int64_t n, int32_t d, int32_t m, gp_precision prec,
                            int32_t* split);
gp_status gp_tune_set(gp_handle* h, int64_t n, int32_t d, int32_t m, gp_precision prec, int32_t code);
gp_status gp_tune_get(gp_handle* h, int64_t n, int32_t d, int32_t m, gp_precision prec,
                      int32_t* code, int32_t* split);
gp_status gp_tune_save(const gp_handle* h, const char* path);
/*
 * The shape a product of (n, d, m, prec) takes by default, or the shape of `code` (>= 0; -1 =
 * the default), without a handle or a device: *code_out the shape code, *split_out the split-K
 * chunks (1 for the symmetric product), *mp_out the padded column count of V, *partial_floats
 * the floats of the partial sums the product needs (the workspace that grows with n).
 * GP_EINVAL for a bad shape, code or null output, and for code 0 where the symmetric product
 * does not apply.
 */
gp_status gp_shape_query(int64_t n, int32_t d, int32_t m, gp_precision prec, int32_t code,
                         int32_t* code_out, int32_t* split_out, int32_t* mp_out,
                         int64_t* partial_floats);
gp_status gp_tune_load(gp_handle* h, const char* path);

/*
 * Pipe probe, for measurement: times six synthetic kernels on the stream (eight waves per
 * SIMD, `iters` loop iterations each, the second of two runs) and returns, per kernel, the
 * time in ms and the clock cycles of one loop iteration of one wave at the device's peak
 * clock.  Kernels: 0 = 128 FP32 VALU FMAs; 1 = 4 FP32 MFMAs (v_mfma_f32_16x16x4f32);
 * 2 = both in one loop, independent of each other; 3 = 4 BF16 MFMAs (16x16x32); 4 = 3 with
 * the 128 FMAs; 5 = 128 v_exp_f32.  cycles[2] against cycles[0] + cycles[1] shows how much
 * of the FP32 MFMA time independent VALU work can hide (none when they add up), likewise 4
 * against 0 + 3 for BF16.  ms and cycles: 6 doubles each, host memory.  Synchronises the
 * stream.
 */
gp_status gp_pipe_probe(gp_handle* h, int32_t iters, double* ms, double* cycles, void* stream);

/*
 * Kernel timing for measurement.  While enabled, the handle records a pair of hipEvents on
 * the launch stream around every covariance-product launch that does work (kmv, in the
 * solver and in gp_kmv) and around every fused gradient reduction (dquad).
 * gp_profile(h, 1) clears the totals and starts recording, gp_profile(h, 0) stops.
 * gp_profile_read waits for the recorded events, returns the totals since the last
 * gp_profile(h, 1) and keeps recording if enabled.  kmv_passes counts the products taken
 * by ULISSE solves (warm-start residual products included).  kmv_ms covers each product
 * whole; kmv_main_ms the same launches up to the end of the main product kernel, leaving
 * out the symmetric shape's reduce of its partials (equal to kmv_ms for the other shapes).
 */
typedef struct {
    int64_t kmv_launches;
    double kmv_ms;
    int64_t dquad_launches;
    double dquad_ms;
    int64_t solves;
    int64_t kmv_passes;
    int64_t kmv_main_launches;
    double kmv_main_ms;
} gp_profile_stats;

gp_status gp_profile(gp_handle* h, int32_t enable);
gp_status gp_profile_read(gp_handle* h, gp_profile_stats* out);

#ifdef __cplusplus
}
#endif

#endif /* ULISSE_GP_H */
