// Solver state shared by solver.hip and the host orchestration in api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gp_common.h"
#include "ulisse_gp.h"

namespace gpk {

constexpr int kMaxSys = 64;
enum { kPre = 0, kTail = 1, kDone = 2 };

// Per-system state of one ULISSE solve (device memory, one entry per system).
struct SysState {
    double rho;        // e^T e of the current iterate
    double alpha;      // step of the current iteration
    double beta;
    double thr_alpha;  // early-stop threshold q sqrt(n)
    double thr_eps;    // convergence threshold
    double res;        // ||e|| after the last iteration
    double W[2];       // weight of the increment of the current iteration, per track (0: done)
    int32_t phase[2];  // kPre, kTail, kDone
    int32_t j[2];      // tail index of the increment of the current iteration
    int32_t ntracks;
    int32_t l, iters, flags;
    int32_t active;    // the CG run of this system continues
    int32_t rf_on;     // residual replacement still enabled for this run
    double res_ref;    // residual norm at the last replacement (or at the start)
};

// Column of the series estimate of track t of system c in the output block.
__host__ __device__ inline int sys_col(int two_track, int c, int t) {
    return two_track ? (c == 0 ? t : c + 1) : c;
}

struct SolverArgs {
    int64_t n, n_pad;
    int32_t m;       // systems
    int32_t mp;      // padded columns of the product partials
    int32_t split;   // chunks of the product partials
    int32_t nb;      // row blocks of the vector kernels (solver_blocks(n))
    int64_t ldb;
    const float* B;
    const double* S0;
    double* Q;       // K d (FP64), ld n_pad
    double* S;       // CG iterate, ld n_pad
    double* E;       // residual, ld n_pad
    float* D;        // direction (FP32), ld n_pad, zero rows past n
    double* St;      // series estimates, ld n
    const float* kpart;
    const KParams* kp;
    double* part;
    double* part2;
    int* n_active;
    SysState* state;  // state read by the kernels of the current iteration
    ulisse_sysstat* stats;
    double q, rate, eps;
    int32_t eps_relative, max_iter, two_track, pad_;
    uint64_t seed, rng_stream, rng_counter;
    const uint64_t* counter_dev;  // non-null: the step word of the counter is read here
    // pcm: 0 plain CG; 1 P^-1 v = tau_inv v + U (h o U^T v); 2 z from an inner CG on
    // (K + delta I) z = e.  For 1 and 2 the step lengths use rho = e^T z (partials in part3).
    int32_t pcm, pad2_;
    const float* U;        // n x pk, ld ldu (FP32)
    int64_t ldu;
    int32_t pk;            // 16, 32 or 64
    int32_t nb256;         // workgroups of the preconditioner kernels (pc_chunks(n))
    const double* coef;    // h[0..pk-1], tau_inv at [pk]
    double* Zp;            // z = P^-1 e, ld n_pad
    double* utv_part;      // nb256 x pk x m
    double* HW;            // pk x m
    double* part3;         // nb256 x m partial sums of e^T z
    // residual replacement (refresh = k > 0): rflag[c] = 1 when system c replaces its
    // residual in the current iteration; rcount = number of such systems (0 skips the
    // replacement product)
    int32_t refresh, pad3_;
    int* rflag;
    int* rcount;
};

int solver_blocks(int64_t n);
hipError_t solver_init(const SolverArgs& a, int warm, hipStream_t s);
hipError_t solver_reduce(const SolverArgs& a, hipStream_t s);
hipError_t solver_update(const SolverArgs& a, hipStream_t s);
// Residual replacement: decides per system whether the residual is replaced in this
// iteration (its norm has fallen by 2^refresh since the last replacement and is above the
// convergence threshold, and replacements are still on), sets rflag / rcount, and packs
// fp32(s) of those systems into Dr (ld n_pad); once an FP32 product of Dr (skipped when
// rcount is 0) has left its chunk partials in kpr (split x mpr x n_pad), e = b - K s with
// the partials of e^T e for the flagged systems.  The direction kernel then restarts
// them (beta = 0).
hipError_t solver_refresh_pack(const SolverArgs& a, float* Dr, hipStream_t s);
hipError_t solver_refresh(const SolverArgs& a, const float* kpr, int split, int mpr, hipStream_t s);
// Reads the state at a.state and writes the advanced state to `next`.
hipError_t solver_direction(const SolverArgs& a, SysState* next, hipStream_t s);
hipError_t solver_copy_s(const SolverArgs& a, double* out, hipStream_t s);
hipError_t launch_pack_f64(const double* S0, int64_t n, int m, float* D, int64_t n_pad,
                           hipStream_t s);
// step_dev / eps_dev (nullable): read the step word (and the step size) from device memory,
// so that a captured graph can be replayed for a new step.
hipError_t launch_probes(int64_t n, int nprobes, int kind, uint64_t k0, uint64_t k1,
                         uint64_t step, float* R, int64_t ldr, hipStream_t s,
                         const uint64_t* step_dev = nullptr);
hipError_t launch_philox(uint64_t k0, uint64_t k1, uint64_t first, uint64_t w1, uint64_t w2,
                         uint64_t w3, int64_t nblocks, uint64_t* out, hipStream_t s);
hipError_t launch_build_ab(const double* St, const float* R, int64_t ldr, int64_t n,
                           int nprobes, float* A, float* Bm, int64_t n_pad, int mq4,
                           hipStream_t s);
// The same operands split into BF16 halves (hi + lo), row-major with row stride mqb (a
// multiple of 32), for the BF16 form of the gradient reduction.
hipError_t launch_build_ab_bf16(const double* St, const float* R, int64_t ldr, int64_t n,
                                int nprobes, uint16_t* AH, uint16_t* AL, uint16_t* BH,
                                uint16_t* BL, int64_t n_pad, int mqb, hipStream_t s);
// dpart: solver_blocks(n) doubles of scratch.
hipError_t launch_grad_finish(const double* St, const float* R, int64_t ldr, int64_t n,
                              int nprobes, const double* gpart, int nwg, int d,
                              const KParams* kp, double* dpart, double* g, hipStream_t s);
hipError_t launch_sgld(int P, double* psi, const double* g, int prior_kind, const double* pa,
                       const double* pb, const double* L, double eps, uint64_t k0,
                       uint64_t k1, uint64_t step, hipStream_t s,
                       const uint64_t* step_dev = nullptr, const double* eps_dev = nullptr);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// out = sum of *counts[b], b < B (counts: device array of B device pointers).
hipError_t launch_sum_active(const int* const* counts, int B, int* out, hipStream_t s);
// *out = number of the m systems whose statistics carry `flag`; or `flag` into all of them.
hipError_t launch_count_flag(const ulisse_sysstat* st, int m, uint32_t flag, int* out, hipStream_t s);
hipError_t launch_or_flag(ulisse_sysstat* st, int m, uint32_t flag, hipStream_t s);
// dst[e] = src[e], e < count (a kernel, so that graphs record no copy node).
hipError_t launch_copy_f64(const double* src, double* dst, int64_t count, hipStream_t s);

// z = P^-1 e for every active system and the partials of e^T z; `first` also sets d = z.
int pc_chunks(int64_t n);
hipError_t launch_pc_step(const SolverArgs& a, int first, hipStream_t s);
// Inner-CG preconditioner (pcm 2): the outer residuals rounded to FP32 as the inner
// right-hand sides (n_pad x m, ld n_pad), and, once the inner run has left z in Zin
// (n x m FP64, ld n), Zp = z, the partials of e^T z and, with `first`, d = z.
hipError_t launch_icg_rhs(const SolverArgs& a, float* Bin, int first, hipStream_t s);
hipError_t launch_icg_finish(const SolverArgs& a, const double* Zin, int first, hipStream_t s);
// out = in with lambda replaced by lambda + delta (the covariance of J = K + delta I).
hipError_t launch_shift_kp(const KParams* in, double delta, KParams* out, hipStream_t s);
// Initial state once the initial residual (and z for PCG) are in place.
hipError_t solver_init_state(const SolverArgs& a, hipStream_t s);

// ratio = eps / 4 * lambda_max(L^T cov(G) L) for a batch x P row-major G.
hipError_t launch_langevin_ratio(const double* G, int batch, int P, const double* L, double eps,
                                 double* ratio, hipStream_t s);

}  // namespace gpk
