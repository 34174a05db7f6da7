// Rank-k plus scaled-identity preconditioner inside the ULISSE/CG iterations.
//
//   P^-1 v = tau_inv v + U (h o (U^T v)),   U: n x k orthonormal columns (FP32),
//   h_kappa = 1/d_kappa - tau_inv, the inverse of P = U diag(d) U^T + tau (I - U U^T).
// Preconditioned CG (the variant of Sec. 3.3 with a fixed preconditioner) keeps the
// estimator of Sec. 4 unbiased: the series is still a telescoping sum of CG increments
// that converges to K^-1 b.
//
// Per iteration: U^T E for all systems (a k x n by n x m product, split over 256-row chunks
// with FP32 partials), a fixed-order FP64 sum of the chunks scaled by h, then z for every
// row and system with the partial sums of e^T z.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gp_common.h"
#include "internal.h"
#include "solver.h"

namespace gpk {

constexpr int kChunk = 256;  // rows per workgroup of the U^T E partials and of the apply
constexpr int kSub = 64;     // rows staged in LDS at a time

// part[chunk][kappa][c] = sum over the chunk's rows of U[kappa][i] * E[c][i], in FP64: once
// the residual lies mostly in span(U), e^T z = tau_inv ||e||^2 + sum h (u^T e)^2 cancels
// (h ~ -tau_inv), and FP32 partial sums can make it negative.
// With `first` (the initial residual, before the per-system state exists) every system is
// processed and the "no system running" early exit is off.
template <int KB>
__global__ __launch_bounds__(kWG) void pc_utv_partial_kernel(SolverArgs a, int first) {
    if (!first && *a.n_active == 0) return;
    __shared__ float us[KB][kSub + 1];
    __shared__ double es[kMaxSys][kSub + 1];
    const int m = a.m;
    const int nout = KB * m;
    // each thread owns blocks of 2 basis vectors x 4 systems, so that one pass over the
    // staged rows reads 6 LDS operands per 8 FMAs; every output still sums its rows in
    // order.  Block b: kappa = 2 (b / nq) + {0, 1}, c = 4 (b % nq) + {0..3}.
    constexpr int NJ = (KB / 2 * (kMaxSys / 4) + kWG - 1) / kWG;
    const int nq = (m + 3) / 4;
    const int nblk = KB / 2 * nq;
    double acc[NJ][2][4];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[j][u][t] = 0.0;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    for (int sub = 0; sub < kChunk / kSub; ++sub) {
        const int64_t r0 = base + sub * kSub;
        for (int e = threadIdx.x; e < KB * kSub; e += kWG) {
            const int kappa = e / kSub, rr = e % kSub;
            const int64_t i = r0 + rr;
            us[kappa][rr] = i < a.n ? a.U[kappa * a.ldu + i] : 0.f;
        }
        // systems m .. 4 nq - 1 of the last quad are staged as zeros
        for (int e = threadIdx.x; e < 4 * nq * kSub; e += kWG) {
            const int c = e / kSub, rr = e % kSub;
            const int64_t i = r0 + rr;
            es[c][rr] = (c < m && i < a.n) ? a.E[c * a.n_pad + i] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            const int b = threadIdx.x + j * kWG;
            if (b < nblk) {
                const int k0 = 2 * (b / nq), c0 = 4 * (b % nq);
                for (int rr = 0; rr < kSub; ++rr) {
                    const double u0 = (double)us[k0][rr], u1 = (double)us[k0 + 1][rr];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const double ev = es[c0 + t][rr];
                        acc[j][0][t] = fma(u0, ev, acc[j][0][t]);
                        acc[j][1][t] = fma(u1, ev, acc[j][1][t]);
                    }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int b = threadIdx.x + j * kWG;
        if (b < nblk) {
            const int k0 = 2 * (b / nq), c0 = 4 * (b % nq);
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    if (c0 + t < m) a.utv_part[(int64_t)blockIdx.x * nout + (k0 + u) * m + c0 + t] = acc[j][u][t];
        }
    }
}

// HW[kappa][c] = h_kappa * sum over chunks (fixed order, FP64)
__global__ void pc_reduce_kernel(SolverArgs a, int nchunk, int first) {
    if (!first && *a.n_active == 0) return;
    const int nout = a.pk * a.m;
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nout) return;
    // chunks summed in order; eight loads in flight at a time (the adds stay sequential)
    double s = 0.0;
    int b = 0;
    for (; b + 8 <= nchunk; b += 8) {
        double v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = a.utv_part[(int64_t)(b + t) * nout + o];
#pragma unroll
        for (int t = 0; t < 8; ++t) s += v[t];
    }
    for (; b < nchunk; ++b) s += a.utv_part[(int64_t)b * nout + o];
    // a negative tau_inv marks the fallback: P = I, so the U terms vanish
    a.HW[o] = a.coef[a.pk] < 0.0 ? 0.0 : a.coef[o / a.m] * s;
}

// z = tau_inv e + U HW[:, c] for every active system; partial sums of e^T z per workgroup;
// with `first`, also the initial direction d = fp32(z).
template <int KB>
__global__ __launch_bounds__(kWG) void pc_apply_kernel(SolverArgs a, int first) {
    if (!first && *a.n_active == 0) return;
    __shared__ double hw[KB][kMaxSys];
    __shared__ double red[4][kMaxSys];
    const int m = a.m;
    for (int e = threadIdx.x; e < KB * m; e += kWG) hw[e / m][e % m] = a.HW[e];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kChunk + threadIdx.x;
    const bool in = i < a.n;
    float u[KB];
#pragma unroll
    for (int kappa = 0; kappa < KB; ++kappa) u[kappa] = in ? a.U[kappa * a.ldu + i] : 0.f;
    // fallback (negative tau_inv): z = e exactly, the plain CG of Alg. 1
    const double tau_inv = a.coef[a.pk] < 0.0 ? 1.0 : a.coef[a.pk];
    for (int c = 0; c < m; ++c) {
        if (!first && !a.state[c].active) continue;  // uniform over the workgroup
        double ez = 0.0;
        if (in) {
            double z = 0.0;
#pragma unroll
            for (int kappa = 0; kappa < KB; ++kappa) z += (double)u[kappa] * hw[kappa][c];
            const double e = a.E[c * a.n_pad + i];
            z += tau_inv * e;
            a.Zp[c * a.n_pad + i] = z;
            if (first) a.D[c * a.n_pad + i] = (float)z;
            ez = e * z;
        }
        const double w = wave_sum(ez);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = w;
    }
    __syncthreads();
    if ((int)threadIdx.x < m && (first || a.state[threadIdx.x].active)) {
        const int c = threadIdx.x;
        a.part3[(int64_t)blockIdx.x * m + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    }
}

int pc_chunks(int64_t n) { return (int)((n + kChunk - 1) / kChunk); }

template <int KB>
static hipError_t pc_step_k(const SolverArgs& a, int first, hipStream_t s) {
    const int nchunk = pc_chunks(a.n);
    pc_utv_partial_kernel<KB><<<nchunk, kWG, 0, s>>>(a, first);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    pc_reduce_kernel<<<(KB * a.m + kWG - 1) / kWG, kWG, 0, s>>>(a, nchunk, first);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    pc_apply_kernel<KB><<<nchunk, kWG, 0, s>>>(a, first);
    return hipGetLastError();
}

hipError_t launch_pc_step(const SolverArgs& a, int first, hipStream_t s) {
    switch (a.pk) {
        case 16: return pc_step_k<16>(a, first, s);
        case 32: return pc_step_k<32>(a, first, s);
        case 64: return pc_step_k<64>(a, first, s);
        default: return hipErrorInvalidValue;
    }
}

// ---------------------------------------------------------------------------------------
// J = K + delta I applied by an inner CG (the PCG variant of Sec. 3.3).  The inner run is
// an ordinary solve on the shifted covariance; these kernels hand the outer residuals to
// it and take its result back into the outer iteration.
// ---------------------------------------------------------------------------------------
__global__ void icg_rhs_kernel(SolverArgs a, float* __restrict__ Bin, int first) {
    if (!first && *a.n_active == 0) return;
    const int64_t total = a.n_pad * a.m;
    for (int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < total;
         o += (int64_t)gridDim.x * blockDim.x)
        Bin[o] = (float)a.E[o];
}

__global__ __launch_bounds__(kWG) void icg_finish_kernel(SolverArgs a, const double* __restrict__ Zin,
                                                         int first) {
    if (!first && *a.n_active == 0) return;
    __shared__ double red[4][kMaxSys];
    const int m = a.m;
    const int64_t i = (int64_t)blockIdx.x * kChunk + threadIdx.x;
    const bool in = i < a.n;
    for (int c = 0; c < m; ++c) {
        if (!first && !a.state[c].active) continue;  // uniform over the workgroup
        double ez = 0.0;
        if (in) {
            const double z = Zin[c * a.n + i];
            a.Zp[c * a.n_pad + i] = z;
            if (first) a.D[c * a.n_pad + i] = (float)z;
            ez = a.E[c * a.n_pad + i] * z;
        }
        const double w = wave_sum(ez);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][c] = w;
    }
    __syncthreads();
    if ((int)threadIdx.x < m && (first || a.state[threadIdx.x].active)) {
        const int c = threadIdx.x;
        a.part3[(int64_t)blockIdx.x * m + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    }
}

__global__ void shift_kp_kernel(const KParams* in, double delta, KParams* out) {
    if (threadIdx.x != 0) return;
    // word copy (a struct copy would go through private memory)
    static_assert(sizeof(KParams) % 4 == 0, "KParams is a whole number of words");
    const uint32_t* src = reinterpret_cast<const uint32_t*>(in);
    uint32_t* dst = reinterpret_cast<uint32_t*>(out);
    for (size_t w = 0; w < sizeof(KParams) / 4; ++w) dst[w] = src[w];
    const double lam = in->lam64 + delta;
    out->lam64 = lam;
    out->lam = (float)lam;
}

hipError_t launch_icg_rhs(const SolverArgs& a, float* Bin, int first, hipStream_t s) {
    const int64_t total = a.n_pad * a.m;
    const int blocks = (int)std::min<int64_t>((total + kWG - 1) / kWG, 4096);
    icg_rhs_kernel<<<blocks, kWG, 0, s>>>(a, Bin, first);
    return hipGetLastError();
}

hipError_t launch_icg_finish(const SolverArgs& a, const double* Zin, int first, hipStream_t s) {
    icg_finish_kernel<<<pc_chunks(a.n), kWG, 0, s>>>(a, Zin, first);
    return hipGetLastError();
}

hipError_t launch_shift_kp(const KParams* in, double delta, KParams* out, hipStream_t s) {
    shift_kp_kernel<<<1, 64, 0, s>>>(in, delta, out);
    return hipGetLastError();
}

}  // namespace gpk
