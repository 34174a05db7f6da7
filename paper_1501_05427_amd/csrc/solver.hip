// ULISSE on the GPU: the per-iteration vector work of Alg. 1 (CG) with the randomly
// truncated series of Sec. 4, plus the draws (probes, u_j, SGLD noise), the assembly of
// the stochastic gradient from the solutions and the SGLD update.
//
// Every system (column) keeps FP64 iterate s, FP64 residual e (Alg. 1's recursive one),
// an FP32 direction d (the vector the covariance product consumes) and one FP64 series
// estimate per track.  Dot products are FP64 per workgroup; the last workgroup to finish
// combines the partials in a fixed order and runs the per-system decisions (threshold l,
// tail draws, convergence, iteration cap), so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gp_common.h"
#include "internal.h"
#include "solver.h"

namespace gpk {

__device__ inline void write_stat(const SysState& st, ulisse_sysstat* out) {
    ulisse_sysstat r;
    r.l = st.l;
    r.J_a = st.j[0];
    r.J_b = st.ntracks > 1 ? st.j[1] : -1;
    r.iters = st.iters;
    r.final_res = st.res;
    r.flags = (uint32_t)st.flags;
    r.pad = 0;
    *out = r;
}

// The vector kernels run on a (row block, system) grid: blockIdx.x covers kRowsPerBlock
// rows (kRowsPerThread per thread, strided by the workgroup size), blockIdx.y is the
// system.  Each workgroup leaves one FP64 partial per reduction in part[bx * m + c].
// A later kernel combines the partials of a column in every workgroup that needs the
// total, with the same fixed order everywhere (wave 0: lane-strided sums, then an xor
// butterfly), so all workgroups see bit-identical scalars and take the same decisions
// without any grid-wide synchronisation.  The per-system state is double buffered: the
// direction kernel reads `cur` and its row-block-0 workgroup writes `next`.
constexpr int kRowsPerThread = 4;
constexpr int kRowsPerBlock = kWG * kRowsPerThread;

__device__ inline double column_total(const double* __restrict__ part, int nb, int m, int c,
                                      double* bcast) {
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += 64) s += part[(int64_t)b * m + c];
        s = wave_sum(s);
        if (threadIdx.x == 0) *bcast = s;
    }
    __syncthreads();
    const double v = *bcast;
    __syncthreads();
    return v;
}

// ---------------------------------------------------------------------------------------
// Initialisation: e = b - K s0, d = e, s~ = s0; partials of e^T e and b^T b.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void ulisse_init_kernel(SolverArgs a, int warm) {
    __shared__ double scratch[4];
    const int c = blockIdx.y;
    const int nt = (a.two_track && c == 0) ? 2 : 1;
    double ee = 0.0, bb = 0.0;
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + r * kWG + threadIdx.x;
        if (i >= a.n) break;
        const double b = (double)a.B[c * a.ldb + i];
        const double s0 = warm ? a.S0[c * a.n + i] : 0.0;
        double e = b;
        if (warm) {  // K s0 from the chunk partials of the product with fp32(s0) held in D
            double kq = 0.0;
            for (int k = 0; k < a.split; ++k) kq += (double)a.kpart[((int64_t)k * a.mp + c) * a.n_pad + i];
            kq += a.kp->lam64 * (double)a.D[c * a.n_pad + i];
            e = b - kq;
        }
        a.S[c * a.n_pad + i] = s0;
        a.E[c * a.n_pad + i] = e;
        a.D[c * a.n_pad + i] = (float)e;
        for (int t = 0; t < nt; ++t) a.St[(int64_t)sys_col(a.two_track, c, t) * a.n + i] = s0;
        ee += e * e;
        bb += b * b;
    }
    ee = block_sum256(ee, scratch);
    bb = block_sum256(bb, scratch);
    if (threadIdx.x == 0) {
        a.part[(int64_t)blockIdx.x * a.m + c] = ee;
        a.part2[(int64_t)blockIdx.x * a.m + c] = bb;
    }
}

// One workgroup per system: thresholds, rho_0 and the initial state.
__global__ __launch_bounds__(kWG) void ulisse_init_state_kernel(SolverArgs a) {
    __shared__ double bcast;
    const int c = blockIdx.x;
    const double ee = column_total(a.part, a.nb, a.m, c, &bcast);
    const double b2 = column_total(a.part2, a.nb, a.m, c, &bcast);
    const double rho = a.pcm != 0 ? column_total(a.part3, a.nb256, a.m, c, &bcast) : ee;
    if (threadIdx.x != 0) return;
    SysState st;
    st.rho = rho;
    st.alpha = 0.0;
    st.beta = 0.0;
    st.thr_alpha = a.q * sqrt((double)a.n);
    st.thr_eps = a.eps_relative ? a.eps * sqrt(b2) : a.eps;
    st.res = sqrt(ee);
    st.ntracks = (a.two_track && c == 0) ? 2 : 1;
    for (int t = 0; t < 2; ++t) {
        st.W[t] = t < st.ntracks ? 1.0 : 0.0;
        st.phase[t] = t < st.ntracks ? kPre : kDone;
        st.j[t] = 0;
    }
    st.l = 0;
    st.iters = 0;
    // a negative tau_inv in the rank-k preconditioner marks the fallback to plain CG
    st.flags = (a.pcm == 1 && a.coef[a.pk] < 0.0) ? (int)ULISSE_FALLBACK : 0;
    st.active = 1;
    st.rf_on = a.refresh > 0 ? 1 : 0;
    st.res_ref = st.res;
    a.state[c] = st;
    if (a.refresh > 0) a.rflag[c] = 0;
    if (c == 0) {
        *a.n_active = a.m;
        if (a.refresh > 0) *a.rcount = 0;
    }
}

// ---------------------------------------------------------------------------------------
// After the covariance product: Q = sum of chunk partials + lambda d (FP64); partials of
// gamma = d^T Q.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void ulisse_reduce_kernel(SolverArgs a) {
    if (*a.n_active == 0) return;
    __shared__ double scratch[4];
    const int c = blockIdx.y;
    if (!a.state[c].active) return;  // uniform over the workgroup
    const double lam = a.kp->lam64;
    double dq = 0.0;
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + r * kWG + threadIdx.x;
        if (i >= a.n) break;
        double s = 0.0;
        for (int k = 0; k < a.split; ++k) s += (double)a.kpart[((int64_t)k * a.mp + c) * a.n_pad + i];
        const double dv = (double)a.D[c * a.n_pad + i];
        s += lam * dv;
        a.Q[c * a.n_pad + i] = s;
        dq += dv * s;
    }
    dq = block_sum256(dq, scratch);
    if (threadIdx.x == 0) a.part[(int64_t)blockIdx.x * a.m + c] = dq;
}

__device__ inline bool alpha_ok(double gamma, double alpha) { return gamma > 0.0 && isfinite(alpha); }

// ---------------------------------------------------------------------------------------
// alpha = rho / gamma; delta = alpha d;  s += delta;  e -= alpha Q;  s~_t += W_t delta;
// partials of rho' = e^T e.  A breakdown (gamma <= 0 or alpha not finite) skips the update;
// the direction kernel records it.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void ulisse_update_kernel(SolverArgs a) {
    if (*a.n_active == 0) return;
    __shared__ double scratch[4];
    __shared__ double bcast;
    const int c = blockIdx.y;
    const SysState& st0 = a.state[c];
    if (!st0.active) return;  // uniform over the workgroup
    const double gamma = column_total(a.part, a.nb, a.m, c, &bcast);
    const double al = st0.rho / gamma;
    if (!alpha_ok(gamma, al)) return;
    const int nt = st0.ntracks;
    const double W0 = st0.W[0], W1 = st0.W[1];
    double* st_a = a.St + (int64_t)sys_col(a.two_track, c, 0) * a.n;
    double* st_b = a.St + (int64_t)sys_col(a.two_track, c, 1) * a.n;
    double ee = 0.0;
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + r * kWG + threadIdx.x;
        if (i >= a.n) break;
        const double delta = al * (double)a.D[c * a.n_pad + i];
        a.S[c * a.n_pad + i] += delta;
        const double e = a.E[c * a.n_pad + i] - al * a.Q[c * a.n_pad + i];
        a.E[c * a.n_pad + i] = e;
        ee += e * e;
        if (W0 != 0.0) st_a[i] += W0 * delta;
        if (nt > 1 && W1 != 0.0) st_b[i] += W1 * delta;
    }
    ee = block_sum256(ee, scratch);
    if (threadIdx.x == 0) a.part2[(int64_t)blockIdx.x * a.m + c] = ee;
}

// ---------------------------------------------------------------------------------------
// Residual replacement: fp32(s) of the running systems into Dr (n_pad x mpr, ld n_pad; rows
// past n zero) for an FP32 product, then e = b - (K_f fp32(s) + lambda s) in FP64 with new
// partials of e^T e in place of the update kernel's.
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void ulisse_refresh_pack_kernel(SolverArgs a, float* __restrict__ Dr) {
    if (*a.n_active == 0) return;
    __shared__ double bcast;
    const int c = blockIdx.y;
    const SysState& st = a.state[c];
    // every workgroup of the system derives the same decision from the same partials
    const double ee = column_total(a.part2, a.nb, a.m, c, &bcast);
    const double r = sqrt(ee);
    const bool go = st.active && st.rf_on && r < st.res_ref * exp2(-(double)a.refresh) && r > st.thr_eps;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        a.rflag[c] = go ? 1 : 0;
        if (go) atomicAdd(a.rcount, 1);
    }
    if (!go) return;
#pragma unroll
    for (int rr = 0; rr < kRowsPerThread; ++rr) {
        const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + rr * kWG + threadIdx.x;
        if (i >= a.n_pad) break;
        Dr[c * a.n_pad + i] = i < a.n ? (float)a.S[c * a.n_pad + i] : 0.f;
    }
}

__global__ __launch_bounds__(kWG) void ulisse_refresh_kernel(SolverArgs a, const float* __restrict__ kpr,
                                                             int split, int mpr) {
    if (*a.n_active == 0 || *a.rcount == 0) return;
    __shared__ double scratch[4];
    const int c = blockIdx.y;
    if (!a.rflag[c]) return;  // uniform over the workgroup
    const double lam = a.kp->lam64;
    double ee = 0.0;
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + r * kWG + threadIdx.x;
        if (i >= a.n) break;
        double kq = 0.0;
        for (int k = 0; k < split; ++k) kq += (double)kpr[((int64_t)k * mpr + c) * a.n_pad + i];
        kq += lam * a.S[c * a.n_pad + i];
        const double e = (double)a.B[c * a.ldb + i] - kq;
        a.E[c * a.n_pad + i] = e;
        ee += e * e;
    }
    ee = block_sum256(ee, scratch);
    if (threadIdx.x == 0) a.part2[(int64_t)blockIdx.x * a.m + c] = ee;
}

// u_j of track t of system c: word j of Philox stream (key (seed, stream), counter
// (j/4, 2c + t, 2, step)), mapped to [0, 1).
__device__ inline double ulisse_u(const SolverArgs& a, int c, int t, int j) {
    const uint64_t step = a.counter_dev != nullptr ? *a.counter_dev : a.rng_counter;
    const u64x4 w = philox4x64_10((uint64_t)(j >> 2), (uint64_t)(2 * c + t), kPurposeUlisse,
                                  step, a.seed, a.rng_stream);
    return u01_co(w.v[j & 3]);
}

// The increment with tail index j[t] has just been added: continue or stop the track.
__device__ inline void tail_decide(const SolverArgs& a, SysState& st, int c, int t) {
    if (st.res < st.thr_eps) {
        st.phase[t] = kDone;
    } else if (st.iters >= a.max_iter) {
        st.phase[t] = kDone;
        st.flags |= (int)ULISSE_NOTCONV;
    } else {
        const int jn = st.j[t] + 1;
        if (ulisse_u(a, c, t, jn) < exp(-a.rate * (double)jn)) {
            st.phase[t] = kTail;
            st.j[t] = jn;
            st.W[t] = exp(a.rate * (double)jn * (double)(jn + 1) * 0.5);
        } else {
            st.phase[t] = kDone;
        }
    }
    if (st.phase[t] == kDone) st.W[t] = 0.0;
}

// The per-system decisions after one CG iteration (threshold l, tail draws, convergence,
// iteration cap, breakdown), applied to a copy of the state.
__device__ inline void advance(const SolverArgs& a, SysState& st, int c, double gamma,
                               double rho_new, double ee, bool replaced) {
    const double al = st.rho / gamma;
    if (!alpha_ok(gamma, al)) {
        st.flags |= (int)ULISSE_BREAKDOWN;
        for (int t = 0; t < 2; ++t) {
            st.phase[t] = kDone;
            st.W[t] = 0.0;
        }
        st.active = 0;
        return;
    }
    st.alpha = al;
    st.res = sqrt(ee);
    st.iters += 1;
    for (int t = 0; t < st.ntracks; ++t) {
        if (st.phase[t] == kDone) continue;
        if (st.phase[t] == kPre) {
            if (st.res < st.thr_alpha || st.res < st.thr_eps) {
                st.l = st.iters;  // this increment was delta_l, kept with W_0 = 1
                st.j[t] = 0;
                tail_decide(a, st, c, t);
            } else if (st.iters >= a.max_iter) {
                st.phase[t] = kDone;
                st.W[t] = 0.0;
                st.flags |= (int)ULISSE_NOTCONV;
            }
        } else {
            tail_decide(a, st, c, t);
        }
    }
    bool done = true;
    for (int t = 0; t < st.ntracks; ++t) done = done && st.phase[t] == kDone;
    if (!isfinite(rho_new) || !isfinite(ee)) {
        done = true;
        st.flags |= (int)ULISSE_BREAKDOWN;
    }
    // a replaced residual restarts the recurrences: the next direction is the residual
    // (preconditioned) itself; replacements stop once one of them gains less than 2x
    st.beta = replaced ? 0.0 : rho_new / st.rho;
    st.rho = rho_new;
    if (replaced) {
        if (!(st.res < 0.5 * st.res_ref)) st.rf_on = 0;
        st.res_ref = st.res;
    }
    if (done) st.active = 0;
}

// ---------------------------------------------------------------------------------------
// Decisions and d = e + beta d (rounded to FP32 for the next covariance product).  Every
// workgroup of a system derives the same new state; the one with blockIdx.x == 0 stores it
// (and the statistics when the system stops).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void ulisse_direction_kernel(SolverArgs a, const SysState* cur,
                                                               SysState* next) {
    if (*a.n_active == 0) return;
    // the replacement product and kernel of this iteration have consumed the count
    if (a.refresh > 0 && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *a.rcount = 0;
    __shared__ double bcast;
    const int c = blockIdx.y;
    SysState st = cur[c];
    if (!st.active) {
        if (blockIdx.x == 0 && threadIdx.x == 0) next[c] = st;
        return;
    }
    const double gamma = column_total(a.part, a.nb, a.m, c, &bcast);
    const double ee = column_total(a.part2, a.nb, a.m, c, &bcast);
    const double rho_new = a.pcm != 0 ? column_total(a.part3, a.nb256, a.m, c, &bcast) : ee;
    const bool replaced = a.refresh > 0 && a.rflag[c] != 0;
    advance(a, st, c, gamma, rho_new, ee, replaced);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        next[c] = st;
        if (!st.active) {
            write_stat(st, a.stats + c);
            atomicSub(a.n_active, 1);
        }
    }
    if (!st.active) return;
    const double beta = st.beta;
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + r * kWG + threadIdx.x;
        if (i >= a.n) break;
        const int64_t o = c * a.n_pad + i;
        const double zv = a.pcm != 0 ? a.Zp[o] : a.E[o];
        a.D[o] = (float)(zv + beta * (double)a.D[o]);
    }
}

// S_cg = last CG iterate (ld n).
__global__ void ulisse_copy_s_kernel(SolverArgs a, double* __restrict__ out) {
    const int64_t total = a.n * a.m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / a.n);
        const int64_t i = e % a.n;
        out[c * a.n + i] = a.S[c * a.n_pad + i];
    }
}

// FP32 copy of the warm start, zero padded, as the input of K s0.
__global__ void pack_f64_kernel(const double* __restrict__ S0, int64_t n, int m,
                                float* __restrict__ D, int64_t n_pad) {
    const int64_t total = n_pad * m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / n_pad);
        const int64_t i = e % n_pad;
        D[e] = i < n ? (float)S0[c * n + i] : 0.f;
    }
}

// ---------------------------------------------------------------------------------------
// Draws
// ---------------------------------------------------------------------------------------
__global__ void probes_kernel(int64_t n, int nprobes, int kind, uint64_t k0, uint64_t k1,
                              uint64_t step_arg, const uint64_t* __restrict__ step_dev,
                              float* __restrict__ R, int64_t ldr) {
    const uint64_t step = step_dev != nullptr ? *step_dev : step_arg;
    const int64_t nblk = (n + 3) / 4;
    const int64_t total = nblk * nprobes;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / nblk);
        const int64_t b = e % nblk;
        const u64x4 w = philox4x64_10((uint64_t)b, (uint64_t)c, kPurposeProbe, step, k0, k1);
        double z[4];
        if (kind == 0) {
            box_muller(w.v[0], w.v[1], &z[0], &z[1]);
            box_muller(w.v[2], w.v[3], &z[2], &z[3]);
        } else {
            for (int u = 0; u < 4; ++u) z[u] = (w.v[u] >> 63) ? -1.0 : 1.0;
        }
        for (int u = 0; u < 4; ++u) {
            const int64_t i = 4 * b + u;
            if (i < n) R[c * ldr + i] = (float)z[u];
        }
    }
}

__global__ void philox_kernel(uint64_t k0, uint64_t k1, uint64_t first, uint64_t w1,
                              uint64_t w2, uint64_t w3, int64_t nblocks, uint64_t* __restrict__ out) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < nblocks;
         b += (int64_t)gridDim.x * blockDim.x) {
        const u64x4 w = philox4x64_10(first + (uint64_t)b, w1, w2, w3, k0, k1);
        for (int u = 0; u < 4; ++u) out[4 * b + u] = w.v[u];
    }
}

// ---------------------------------------------------------------------------------------
// Gradient assembly
// ---------------------------------------------------------------------------------------
// A = [1/2 s_a, -r_1/(2 N_r), ...],  B = [s_b, s_1, ...]  as zero-padded FP32 (ld n_pad).
__global__ void build_ab_kernel(const double* __restrict__ St, const float* __restrict__ R,
                                int64_t ldr, int64_t n, int nprobes, float* __restrict__ A,
                                float* __restrict__ Bm, int64_t n_pad, int mq4) {
    const int64_t total = n_pad * mq4;
    const double w = -1.0 / (2.0 * nprobes);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / n_pad);
        const int64_t i = e % n_pad;
        float av = 0.f, bv = 0.f;
        if (i < n && c <= nprobes) {
            if (c == 0) {
                av = (float)(0.5 * St[i]);
                bv = (float)St[n + i];
            } else {
                av = (float)(w * (double)R[(c - 1) * ldr + i]);
                bv = (float)St[(int64_t)(c + 1) * n + i];
            }
        }
        A[e] = av;
        Bm[e] = bv;
    }
}

// Per-workgroup partials of the diagonal (noise) term sum_i G_ii in FP64 from the FP64
// solutions: G_ii = 1/2 s_a,i s_b,i - 1/(2 N_r) sum_c r_c,i s_c,i.
__global__ __launch_bounds__(kWG) void grad_diag_kernel(const double* __restrict__ St,
                                                        const float* __restrict__ R, int64_t ldr,
                                                        int64_t n, int nprobes,
                                                        double* __restrict__ dpart) {
    __shared__ double scratch[4];
    const double w = 1.0 / (2.0 * nprobes);
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < kRowsPerThread; ++r) {
        const int64_t i = (int64_t)blockIdx.x * kRowsPerBlock + r * kWG + threadIdx.x;
        if (i >= n) break;
        double v = 0.5 * St[i] * St[n + i];
        double t = 0.0;
        for (int c = 0; c < nprobes; ++c) t += (double)R[c * ldr + i] * St[(int64_t)(c + 2) * n + i];
        acc += v - w * t;
    }
    acc = block_sum256(acc, scratch);
    if (threadIdx.x == 0) dpart[blockIdx.x] = acc;
}

// Final fixed-order sums, one workgroup per component: g_0 and 2 ln 2 * (g_1..g_d) from the
// tile partials (gpart[j * nwg + w]); g_{d+1} = lambda * (diagonal term) from its partials.
__global__ __launch_bounds__(kWG) void grad_finish_kernel(const double* __restrict__ gpart,
                                                          int nwg, int d,
                                                          const double* __restrict__ dpart,
                                                          int ndb, const KParams* __restrict__ kp,
                                                          double* __restrict__ g) {
    __shared__ double scratch[4];
    const int p = blockIdx.x;
    const double* src = p <= d ? gpart + (int64_t)p * nwg : dpart;
    const int cnt = p <= d ? nwg : ndb;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * kWG < cnt; b += 4 * kWG) {
        s0 += src[b];
        s1 += src[b + kWG];
        s2 += src[b + 2 * kWG];
        s3 += src[b + 3 * kWG];
    }
    for (; b < cnt; b += kWG) s0 += src[b];
    const double s = block_sum256((s0 + s1) + (s2 + s3), scratch);
    if (threadIdx.x == 0) g[p] = p == 0 ? s : (p <= d ? 2.0 * M_LN2 * s : kp->lam64 * s);
}

// ---------------------------------------------------------------------------------------
// SGLD update in FP64, one wave: lane i < P owns component i of psi.  Each lane sums its
// own row or column in the natural index order, so the result does not depend on the wave
// size.  The P normal draws come from ceil(P / 4) Philox blocks, one per lane.
// ---------------------------------------------------------------------------------------
__global__ void sgld_kernel(int P, double* __restrict__ psi, const double* __restrict__ g,
                            int prior_kind, const double* __restrict__ pa,
                            const double* __restrict__ pb, const double* __restrict__ L,
                            double eps_arg, uint64_t k0, uint64_t k1, uint64_t step_arg,
                            const uint64_t* __restrict__ step_dev, const double* __restrict__ eps_dev) {
    __shared__ double v[kMaxP], xi[kMaxP + 4], t[kMaxP];
    if (blockIdx.x != 0) return;
    const int i = threadIdx.x;
    const uint64_t step = step_dev != nullptr ? *step_dev : step_arg;
    const double eps = eps_dev != nullptr ? *eps_dev : eps_arg;
    double psi_i = 0.0;
    if (i < P) {
        psi_i = psi[i];
        double pg = 0.0;
        if (prior_kind == 1) pg = -(psi_i - pa[i]) / (pb[i] * pb[i]);
        if (prior_kind == 2) pg = pa[i] - pb[i] * exp(psi_i);
        v[i] = g[i] + pg;
    }
    if (i < (P + 3) / 4) {
        const u64x4 w = philox4x64_10((uint64_t)i, 0, kPurposeSgld, step, k0, k1);
        box_muller(w.v[0], w.v[1], &xi[4 * i], &xi[4 * i + 1]);
        box_muller(w.v[2], w.v[3], &xi[4 * i + 2], &xi[4 * i + 3]);
    }
    __syncthreads();
    // t = L^T v (lane j: column j of L), then M v = L t and L xi (lane i: row i of L)
    if (i < P) {
        double s = 0.0;
        for (int k = 0; k < P; ++k) s += (L ? L[k + i * P] : (k == i ? 1.0 : 0.0)) * v[k];
        t[i] = s;
    }
    __syncthreads();
    if (i < P) {
        double mv = 0.0, lx = 0.0;
        for (int j = 0; j < P; ++j) {
            const double lij = L ? L[i + j * P] : (i == j ? 1.0 : 0.0);
            mv += lij * t[j];
            lx += lij * xi[j];
        }
        psi[i] = psi_i + 0.5 * eps * mv + sqrt(eps) * lx;
    }
}

// ---------------------------------------------------------------------------------------
// Langevin-phase monitor: ratio = eps / 4 * lambda_max(L^T V L), V the sample covariance
// (divisor batch - 1) of the batch x P gradients G (row-major); L^T V L has the
// eigenvalues of M^(1/2) V M^(1/2) for M = L L^T.  Cyclic Jacobi rotations on the P x P
// symmetric matrix (one thread; P <= 18).
// ---------------------------------------------------------------------------------------
__global__ void langevin_ratio_kernel(const double* __restrict__ G, int batch, int P,
                                      const double* __restrict__ L, double eps,
                                      double* __restrict__ ratio) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double mu[kMaxP], V[kMaxP][kMaxP], B[kMaxP][kMaxP];
    for (int i = 0; i < P; ++i) {
        double s = 0.0;
        for (int t = 0; t < batch; ++t) s += G[t * P + i];
        mu[i] = s / batch;
    }
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            double s = 0.0;
            for (int t = 0; t < batch; ++t) s += (G[t * P + i] - mu[i]) * (G[t * P + j] - mu[j]);
            V[i][j] = s / (batch - 1);
        }
    // B = L^T V L (L lower triangular, column-major; identity when null)
    for (int i = 0; i < P; ++i)
        for (int j = 0; j < P; ++j) {
            double s = 0.0;
            for (int a = 0; a < P; ++a)
                for (int b = 0; b < P; ++b) {
                    const double lai = L ? L[a + i * P] : (a == i ? 1.0 : 0.0);
                    const double lbj = L ? L[b + j * P] : (b == j ? 1.0 : 0.0);
                    s += lai * V[a][b] * lbj;
                }
            B[i][j] = s;
        }
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < P; ++i)
            for (int j = 0; j < P; ++j) (i == j ? diag : off) += B[i][j] * B[i][j];
        if (off <= 1e-30 * diag) break;
        for (int p = 0; p < P - 1; ++p)
            for (int q = p + 1; q < P; ++q) {
                if (B[p][q] == 0.0) continue;
                const double theta = (B[q][q] - B[p][p]) / (2.0 * B[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < P; ++k) {  // rotate columns p, q
                    const double bkp = B[k][p], bkq = B[k][q];
                    B[k][p] = c * bkp - sn * bkq;
                    B[k][q] = sn * bkp + c * bkq;
                }
                for (int k = 0; k < P; ++k) {  // rotate rows p, q
                    const double bpk = B[p][k], bqk = B[q][k];
                    B[p][k] = c * bpk - sn * bqk;
                    B[q][k] = sn * bpk + c * bqk;
                }
            }
    }
    double lmax = B[0][0];
    for (int i = 1; i < P; ++i) lmax = fmax(lmax, B[i][i]);
    *ratio = 0.25 * eps * lmax;
}

// ---------------------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------------------
static int grid_of(int64_t total) {
    return (int)std::max<int64_t>(1, std::min<int64_t>((total + kWG - 1) / kWG, 65536));
}

static dim3 vec_grid(const SolverArgs& a) { return dim3((unsigned)a.nb, (unsigned)a.m); }

int solver_blocks(int64_t n) { return (int)((n + kRowsPerBlock - 1) / kRowsPerBlock); }

hipError_t solver_init(const SolverArgs& a, int warm, hipStream_t s) {
    ulisse_init_kernel<<<vec_grid(a), kWG, 0, s>>>(a, warm);
    return hipGetLastError();
}
hipError_t solver_init_state(const SolverArgs& a, hipStream_t s) {
    ulisse_init_state_kernel<<<(unsigned)a.m, kWG, 0, s>>>(a);
    return hipGetLastError();
}
hipError_t solver_reduce(const SolverArgs& a, hipStream_t s) {
    ulisse_reduce_kernel<<<vec_grid(a), kWG, 0, s>>>(a);
    return hipGetLastError();
}
hipError_t solver_update(const SolverArgs& a, hipStream_t s) {
    ulisse_update_kernel<<<vec_grid(a), kWG, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t solver_refresh_pack(const SolverArgs& a, float* Dr, hipStream_t s) {
    ulisse_refresh_pack_kernel<<<vec_grid(a), kWG, 0, s>>>(a, Dr);
    return hipGetLastError();
}

hipError_t solver_refresh(const SolverArgs& a, const float* kpr, int split, int mpr, hipStream_t s) {
    ulisse_refresh_kernel<<<vec_grid(a), kWG, 0, s>>>(a, kpr, split, mpr);
    return hipGetLastError();
}
hipError_t solver_direction(const SolverArgs& a, SysState* next, hipStream_t s) {
    ulisse_direction_kernel<<<vec_grid(a), kWG, 0, s>>>(a, a.state, next);
    return hipGetLastError();
}
hipError_t solver_copy_s(const SolverArgs& a, double* out, hipStream_t s) {
    ulisse_copy_s_kernel<<<grid_of(a.n * a.m), kWG, 0, s>>>(a, out);
    return hipGetLastError();
}
hipError_t launch_pack_f64(const double* S0, int64_t n, int m, float* D, int64_t n_pad,
                           hipStream_t s) {
    pack_f64_kernel<<<grid_of(n_pad * m), kWG, 0, s>>>(S0, n, m, D, n_pad);
    return hipGetLastError();
}
hipError_t launch_probes(int64_t n, int nprobes, int kind, uint64_t k0, uint64_t k1,
                         uint64_t step, float* R, int64_t ldr, hipStream_t s,
                         const uint64_t* step_dev) {
    probes_kernel<<<grid_of((n + 3) / 4 * nprobes), kWG, 0, s>>>(n, nprobes, kind, k0, k1, step, step_dev,
                                                                   R, ldr);
    return hipGetLastError();
}
hipError_t launch_philox(uint64_t k0, uint64_t k1, uint64_t first, uint64_t w1, uint64_t w2,
                         uint64_t w3, int64_t nblocks, uint64_t* out, hipStream_t s) {
    philox_kernel<<<grid_of(nblocks), kWG, 0, s>>>(k0, k1, first, w1, w2, w3, nblocks, out);
    return hipGetLastError();
}
hipError_t launch_build_ab(const double* St, const float* R, int64_t ldr, int64_t n,
                           int nprobes, float* A, float* Bm, int64_t n_pad, int mq4,
                           hipStream_t s) {
    build_ab_kernel<<<grid_of(n_pad * mq4), kWG, 0, s>>>(St, R, ldr, n, nprobes, A, Bm, n_pad, mq4);
    return hipGetLastError();
}
hipError_t launch_grad_finish(const double* St, const float* R, int64_t ldr, int64_t n,
                              int nprobes, const double* gpart, int nwg, int d,
                              const KParams* kp, double* dpart, double* g, hipStream_t s) {
    const int ndb = solver_blocks(n);
    grad_diag_kernel<<<ndb, kWG, 0, s>>>(St, R, ldr, n, nprobes, dpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    grad_finish_kernel<<<d + 2, kWG, 0, s>>>(gpart, nwg, d, dpart, ndb, kp, g);
    return hipGetLastError();
}
hipError_t launch_sgld(int P, double* psi, const double* g, int prior_kind, const double* pa,
                       const double* pb, const double* L, double eps, uint64_t k0,
                       uint64_t k1, uint64_t step, hipStream_t s, const uint64_t* step_dev,
                       const double* eps_dev) {
    sgld_kernel<<<1, 64, 0, s>>>(P, psi, g, prior_kind, pa, pb, L, eps, k0, k1, step, step_dev, eps_dev);
    return hipGetLastError();
}

}  // namespace gpk

namespace gpk {
hipError_t launch_langevin_ratio(const double* G, int batch, int P, const double* L, double eps,
                                 double* ratio, hipStream_t s) {
    langevin_ratio_kernel<<<1, 64, 0, s>>>(G, batch, P, L, eps, ratio);
    return hipGetLastError();
}
}  // namespace gpk

namespace gpk {

__global__ void copy_f64_kernel(const double* __restrict__ src, double* __restrict__ dst, int64_t count) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        dst[e] = src[e];
}

hipError_t launch_copy_f64(const double* src, double* dst, int64_t count, hipStream_t s) {
    if (count == 0) return hipSuccess;
    copy_f64_kernel<<<grid_of(count), kWG, 0, s>>>(src, dst, count);
    return hipGetLastError();
}

// Systems whose statistics carry `flag` (one wave), and the flag ORed into every system's.
__global__ void count_flag_kernel(const ulisse_sysstat* __restrict__ st, int m, uint32_t flag,
                                  int* __restrict__ out) {
    int t = 0;
    for (int c = threadIdx.x; c < m; c += 64) t += (st[c].flags & flag) != 0u;
    for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
    if (threadIdx.x == 0) *out = t;
}

__global__ void or_flag_kernel(ulisse_sysstat* __restrict__ st, int m, uint32_t flag) {
    for (int c = threadIdx.x; c < m; c += 64) st[c].flags |= flag;
}

hipError_t launch_count_flag(const ulisse_sysstat* st, int m, uint32_t flag, int* out, hipStream_t s) {
    count_flag_kernel<<<1, 64, 0, s>>>(st, m, flag, out);
    return hipGetLastError();
}

hipError_t launch_or_flag(ulisse_sysstat* st, int m, uint32_t flag, hipStream_t s) {
    or_flag_kernel<<<1, 64, 0, s>>>(st, m, flag);
    return hipGetLastError();
}

// Zero fill by a kernel (a memset node recorded into a captured graph is avoided).
__global__ void zero_kernel(uint32_t* __restrict__ p, int64_t words) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < words;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0u;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t words = (int64_t)(bytes / 4);
    if (words == 0) return hipSuccess;
    zero_kernel<<<grid_of(words), kWG, 0, s>>>(static_cast<uint32_t*>(p), words);
    return hipGetLastError();
}

// out = sum over b of *counts[b] (one wave).
__global__ void sum_active_kernel(const int* const* __restrict__ counts, int B, int* __restrict__ out) {
    int t = 0;
    for (int b = threadIdx.x; b < B; b += 64) t += *counts[b];
    for (int o = 32; o >= 1; o >>= 1) t += __shfl_xor(t, o);
    if (threadIdx.x == 0) *out = t;
}

hipError_t launch_sum_active(const int* const* counts, int B, int* out, hipStream_t s) {
    sum_active_kernel<<<1, 64, 0, s>>>(counts, B, out);
    return hipGetLastError();
}

}  // namespace gpk

namespace gpk {

// The operands of the gradient reduction split into BF16 halves (v = hi + lo, both BF16),
// row-major with row stride mqb (a multiple of 32): AH[i * mqb + c] etc.  Column c of A / B
// as in build_ab_kernel.
__device__ inline uint32_t pack2_bf16(float a, float b) {
    typedef float f2 __attribute__((ext_vector_type(2)));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    const f2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, b2));
}

__global__ void build_ab_bf16_kernel(const double* __restrict__ St, const float* __restrict__ R,
                                     int64_t ldr, int64_t n, int nprobes,
                                     uint32_t* __restrict__ AH, uint32_t* __restrict__ AL,
                                     uint32_t* __restrict__ BH, uint32_t* __restrict__ BL,
                                     int64_t n_pad, int mqb) {
    const int half = mqb / 2;  // column pairs per row
    const int64_t total = n_pad * half;
    const double w = -1.0 / (2.0 * nprobes);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / half;
        const int c0 = (int)(e % half) * 2;
        float av[2] = {0.f, 0.f}, bv[2] = {0.f, 0.f};
        for (int u = 0; u < 2; ++u) {
            const int c = c0 + u;
            if (i < n && c <= nprobes) {
                if (c == 0) {
                    av[u] = (float)(0.5 * St[i]);
                    bv[u] = (float)St[n + i];
                } else {
                    av[u] = (float)(w * (double)R[(c - 1) * ldr + i]);
                    bv[u] = (float)St[(int64_t)(c + 1) * n + i];
                }
            }
        }
        const uint32_t ah = pack2_bf16(av[0], av[1]);
        const uint32_t bh = pack2_bf16(bv[0], bv[1]);
        AH[e] = ah;
        BH[e] = bh;
        AL[e] = pack2_bf16(av[0] - __uint_as_float(ah << 16), av[1] - __uint_as_float(ah & 0xffff0000u));
        BL[e] = pack2_bf16(bv[0] - __uint_as_float(bh << 16), bv[1] - __uint_as_float(bh & 0xffff0000u));
    }
}

hipError_t launch_build_ab_bf16(const double* St, const float* R, int64_t ldr, int64_t n,
                                int nprobes, uint16_t* AH, uint16_t* AL, uint16_t* BH,
                                uint16_t* BL, int64_t n_pad, int mqb, hipStream_t s) {
    build_ab_bf16_kernel<<<grid_of(n_pad * (mqb / 2)), kWG, 0, s>>>(
        St, R, ldr, n, nprobes, reinterpret_cast<uint32_t*>(AH), reinterpret_cast<uint32_t*>(AL),
        reinterpret_cast<uint32_t*>(BH), reinterpret_cast<uint32_t*>(BL), n_pad, mqb);
    return hipGetLastError();
}

}  // namespace gpk
