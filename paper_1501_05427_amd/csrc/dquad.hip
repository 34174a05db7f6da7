// Fused bilinear reduction for the stochastic gradient.
//
// For every log-parameter j the gradient estimate is a sum over all pairs (i, k) of
// dK_j(i, k) G(i, k) with G = A B^T, where the columns of A and B are the weighted
// solutions and probes of the estimator (1/2 s_a with s_b, and -r_c / (2 N_r) with s_c).
// A 16 x 16 tile of G comes out of a chain of v_mfma_f32_16x16x4f32 over the columns of
// A and B; the matching tile of K_f and the squared scaled differences are formed on the
// VALU from explicit FP32 differences, so no derivative matrix and no n x n tile is ever
// written.  Partials go to FP64 per lane, then per workgroup in a fixed order.
//   j = 0      : sum K_f G
//   j = 1..d   : 2 ln 2 * sum K_f dz_k^2 G     (dz_k^2 = (x_ik - x_jk)^2 log2(e) / (2 ell_k^2))
// The noise derivative (lambda I) is a plain FP64 dot product done elsewhere.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gp_common.h"
#include "internal.h"

namespace gpk {

constexpr int kJSq = 64;  // columns per LDS stage

template <int D>
__device__ inline void load_row_q(const float* __restrict__ p, float (&z)[D]) {
    constexpr int DP = (D + 3) & ~3;
    float tmp[DP];
#pragma unroll
    for (int k = 0; k < DP; k += 4) {
        const float4 v = *reinterpret_cast<const float4*>(p + k);
        tmp[k] = v.x;
        tmp[k + 1] = v.y;
        tmp[k + 2] = v.z;
        tmp[k + 3] = v.w;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) z[k] = tmp[k];
}

// MQ = (padded columns of A and B) / 4: k-slot q of MFMA step t is column q*MQ + t, so a
// lane's operand for all MQ steps is MQ consecutive floats of one row.
template <int D, int MQ, int R>
__global__ __launch_bounds__(kWG) void dquad_kernel(
    const float* __restrict__ Z, const float* __restrict__ A, const float* __restrict__ B,
    double* __restrict__ gpart, int64_t n_pad, int chunk, int split,
    const KParams* __restrict__ kp) {
    constexpr int DP = (D + 3) & ~3;
    constexpr int MC = 4 * MQ;
    constexpr int BST = MC + 4;  // LDS row stride of B (floats)
    constexpr int NZ4 = kJSq * DP / 4;
    constexpr int NB4 = MC * kJSq / 4;
    constexpr int NL = (NZ4 + NB4 + kWG - 1) / kWG;
    __shared__ float4 zs[2][NZ4];
    __shared__ float bs[2][kJSq * BST];
    __shared__ double red[4][D + 1];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int cidx = blockIdx.x % split;
    const int64_t rt = blockIdx.x / split;
    const int64_t row0 = rt * (64 * R) + wave * (16 * R);
    const int64_t jb = (int64_t)cidx * chunk;
    const int64_t je = min(jb + (int64_t)chunk, n_pad);
    const float negc0 = -kp->c0;

    // A operand (row row0 + 16r + col, columns q*MQ .. q*MQ + MQ - 1) and the four rows
    // 4q .. 4q + 3 of each block whose G entries this lane receives.
    float aop[R][MQ];
    float zi[R][4][D];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int64_t ia = row0 + r * 16 + col;
#pragma unroll
        for (int t = 0; t < MQ; ++t) aop[r][t] = A[(int64_t)(q * MQ + t) * n_pad + ia];
#pragma unroll
        for (int u = 0; u < 4; ++u) load_row_q<D>(Z + (row0 + r * 16 + 4 * q + u) * DP, zi[r][u]);
    }

    float gacc[D + 1];
    double gsum[D + 1];
#pragma unroll
    for (int p = 0; p <= D; ++p) {
        gacc[p] = 0.f;
        gsum[p] = 0.0;
    }

    auto load = [&](int64_t j0, float4(&buf)[NL]) {
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NZ4) {
                buf[t] = reinterpret_cast<const float4*>(Z + j0 * DP)[idx];
            } else if (idx < NZ4 + NB4) {
                const int v = idx - NZ4;
                const int c = v / (kJSq / 4);
                const int jj = (v % (kJSq / 4)) * 4;
                buf[t] = *reinterpret_cast<const float4*>(B + c * n_pad + j0 + jj);
            }
        }
    };
    auto store = [&](int b, const float4(&buf)[NL]) {
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NZ4) {
                zs[b][idx] = buf[t];
            } else if (idx < NZ4 + NB4) {
                const int v = idx - NZ4;
                const int c = v / (kJSq / 4);
                const int jj = (v % (kJSq / 4)) * 4;
                bs[b][(jj + 0) * BST + c] = buf[t].x;
                bs[b][(jj + 1) * BST + c] = buf[t].y;
                bs[b][(jj + 2) * BST + c] = buf[t].z;
                bs[b][(jj + 3) * BST + c] = buf[t].w;
            }
        }
    };

    float4 pre[NL];
    if (jb < je) {
        load(jb, pre);
        store(0, pre);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kJSq) {
        const bool more = j0 + kJSq < je;
        if (more) load(j0 + kJSq, pre);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
        const float* bsb = bs[buf];
#pragma unroll 1
        for (int jt = 0; jt < kJSq / 16; ++jt) {
            const int jr = jt * 16 + col;  // this lane's column of the G tile
            float bop[MQ];
#pragma unroll
            for (int t = 0; t < MQ; t += 4) {
                const float4 v = *reinterpret_cast<const float4*>(bsb + jr * BST + q * MQ + t);
                bop[t] = v.x;
                if (t + 1 < MQ) bop[t + 1] = v.y;
                if (t + 2 < MQ) bop[t + 2] = v.z;
                if (t + 3 < MQ) bop[t + 3] = v.w;
            }
            float zj[D];
            load_row_q<D>(zsb + jr * DP, zj);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                floatx4 G = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < MQ; ++t)
                    G = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[r][t], bop[t], G, 0, 0, 0);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    float sq[D];
                    float a = negc0;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const float t = zi[r][u][k] - zj[k];
                        sq[k] = t * t;
                        a += sq[k];
                    }
                    const float w = __builtin_amdgcn_exp2f(-a) * G[u];
                    gacc[0] += w;
#pragma unroll
                    for (int k = 0; k < D; ++k) gacc[k + 1] = __builtin_fmaf(w, sq[k], gacc[k + 1]);
                }
            }
        }
        // flush the FP32 partials of this stage (at most 16 R terms each) to FP64
#pragma unroll
        for (int p = 0; p <= D; ++p) {
            gsum[p] += (double)gacc[p];
            gacc[p] = 0.f;
        }
        if (more) store(buf ^ 1, pre);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int p = 0; p <= D; ++p) {
        const double v = wave_sum(gsum[p]);
        if (lane == 0) red[wave][p] = v;
    }
    __syncthreads();
    if (threadIdx.x <= D) {
        const int p = threadIdx.x;
        gpart[(int64_t)blockIdx.x * (D + 1) + p] = (red[0][p] + red[1][p]) + (red[2][p] + red[3][p]);
    }
}

DquadShape dquad_shape(int64_t n, int d, int mcols) {
    DquadShape sh;
    sh.n_pad = round_up(std::max<int64_t>(n, 1), kRowPad);
    sh.mq4 = (int)round_up(std::max(mcols, 1), 16);
    const int R = d <= 8 ? 2 : 1;
    sh.rows_per_wg = 64 * R;
    const int64_t row_tiles = sh.n_pad / sh.rows_per_wg;
    int64_t split = std::max<int64_t>(1, 2048 / row_tiles);
    split = std::min<int64_t>(split, sh.n_pad / kJSq);
    if (split >= 8) split = split / 8 * 8;
    sh.chunk = (int)round_up((sh.n_pad + split - 1) / split, kJSq);
    sh.split = (int)((sh.n_pad + sh.chunk - 1) / sh.chunk);
    sh.nwg = (int)(row_tiles * sh.split);
    return sh;
}

template <int D>
static hipError_t dquad_d(const DquadShape& sh, const float* Z, const float* A, const float* B,
                          const KParams* kp, double* gpart, hipStream_t s) {
    constexpr int R = D <= 8 ? 2 : 1;
    const dim3 grid((unsigned)sh.nwg);
    switch (sh.mq4) {
        case 16: dquad_kernel<D, 4, R><<<grid, kWG, 0, s>>>(Z, A, B, gpart, sh.n_pad, sh.chunk, sh.split, kp); break;
        case 32: dquad_kernel<D, 8, R><<<grid, kWG, 0, s>>>(Z, A, B, gpart, sh.n_pad, sh.chunk, sh.split, kp); break;
        case 48: dquad_kernel<D, 12, R><<<grid, kWG, 0, s>>>(Z, A, B, gpart, sh.n_pad, sh.chunk, sh.split, kp); break;
        case 64: dquad_kernel<D, 16, R><<<grid, kWG, 0, s>>>(Z, A, B, gpart, sh.n_pad, sh.chunk, sh.split, kp); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dquad(const DquadShape& sh, int d, const float* Z, const float* A,
                        const float* B, const KParams* kp, double* gpart, hipStream_t s) {
    switch (d) {
        case 1: return dquad_d<1>(sh, Z, A, B, kp, gpart, s);
        case 2: return dquad_d<2>(sh, Z, A, B, kp, gpart, s);
        case 3: return dquad_d<3>(sh, Z, A, B, kp, gpart, s);
        case 4: return dquad_d<4>(sh, Z, A, B, kp, gpart, s);
        case 5: return dquad_d<5>(sh, Z, A, B, kp, gpart, s);
        case 6: return dquad_d<6>(sh, Z, A, B, kp, gpart, s);
        case 7: return dquad_d<7>(sh, Z, A, B, kp, gpart, s);
        case 8: return dquad_d<8>(sh, Z, A, B, kp, gpart, s);
        case 9: return dquad_d<9>(sh, Z, A, B, kp, gpart, s);
        case 10: return dquad_d<10>(sh, Z, A, B, kp, gpart, s);
        case 11: return dquad_d<11>(sh, Z, A, B, kp, gpart, s);
        case 12: return dquad_d<12>(sh, Z, A, B, kp, gpart, s);
        case 13: return dquad_d<13>(sh, Z, A, B, kp, gpart, s);
        case 14: return dquad_d<14>(sh, Z, A, B, kp, gpart, s);
        case 15: return dquad_d<15>(sh, Z, A, B, kp, gpart, s);
        case 16: return dquad_d<16>(sh, Z, A, B, kp, gpart, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gpk
