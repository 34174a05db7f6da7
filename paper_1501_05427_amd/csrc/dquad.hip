// Fused bilinear reduction for the stochastic gradient.
//
// For every log-parameter j the gradient estimate is a sum over all pairs (i, k) of
// dK_j(i, k) G(i, k) with G = A B^T, where the columns of A and B are the weighted
// solutions and probes of the estimator (1/2 s_a with s_b, and -r_c / (2 N_r) with s_c).
// Every dK_j is symmetric, so the sum runs over the upper triangle of 16 x 16 tiles only:
// a diagonal tile contributes G_II, an off-diagonal tile (I < J) contributes
// G_IJ + G_JI^T = A_I B_J^T + B_I A_J^T.  Both products come out of chains of
// v_mfma_f32_16x16x4f32 over the columns of A and B; the matching tile of K_f and the
// squared scaled differences are formed on the VALU from explicit FP32 differences, so no
// derivative matrix and no n x n tile is ever written.  Per-lane FP32 partials are flushed
// to FP64 every stage, then summed per workgroup and finally over workgroups in a fixed
// order.
//   j = 0      : sum K_f G
//   j = 1..d   : 2 ln 2 * sum K_f dz_k^2 G     (dz_k^2 = (x_ik - x_jk)^2 log2(e) / (2 ell_k^2))
// The noise derivative (lambda I) is a plain FP64 dot product done elsewhere.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "gp_common.h"
#include "internal.h"

namespace gpk {

constexpr int kTile = 64;  // rows of a workgroup's row tile = columns of one LDS stage

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

// MQ consecutive floats from LDS: 16-byte reads when MQ is a multiple of 4, else 8-byte
// reads (MQ even; the row stride and q * MQ keep the address 8-byte aligned).
template <int MQ>
__device__ inline void load_op(const float* __restrict__ p, float (&o)[MQ]) {
    static_assert(MQ % 2 == 0, "even operand length");
    if constexpr (MQ % 4 == 0) {
#pragma unroll
        for (int t = 0; t < MQ; t += 4) {
            const float4 v = *reinterpret_cast<const float4*>(p + t);
            o[t] = v.x;
            o[t + 1] = v.y;
            o[t + 2] = v.z;
            o[t + 3] = v.w;
        }
    } else {
#pragma unroll
        for (int t = 0; t < MQ; t += 2) {
            const float2 v = *reinterpret_cast<const float2*>(p + t);
            o[t] = v.x;
            o[t + 1] = v.y;
        }
    }
}

// MQ = (padded columns of A and B) / 4: k-slot q of MFMA step t is column q*MQ + t, so a
// lane's operand for all MQ steps is MQ consecutive floats of one row.
// work[blockIdx.x] = (row tile a, first column tile b0); columns tiles b0 .. b0 + L - 1
// (clipped to the matrix), with b0 >= a.
// (register budget for two workgroups per CU where it fits without spilling: the MFMA
// results feed long VALU chains, so the extra waves hide latency; measured 17% faster than
// the unconstrained allocation at d = 8)
template <int D, int MQ>
__global__ __launch_bounds__(kWG, (D <= 8 && MQ <= 8) ? 2 : 1) void dquad_sym_kernel(
    const float* __restrict__ Z, const float* __restrict__ A, const float* __restrict__ B,
    double* __restrict__ gpart, int64_t n_pad, const int2* __restrict__ work, int L,
    const KParams* __restrict__ kp) {
    constexpr int DP = (D + 3) & ~3;
    constexpr int MC = 4 * MQ;
    constexpr int ST = MC + 4;  // LDS row stride of A and B (floats)
    constexpr int NZ4 = kTile * DP / 4;
    constexpr int NA4 = MC * kTile / 4;
    constexpr int NL = (NZ4 + 2 * NA4 + kWG - 1) / kWG;
    __shared__ float4 zs[2][NZ4];
    __shared__ float as[2][kTile * ST];
    __shared__ float bs[2][kTile * ST];
    __shared__ double red[4][D + 1];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int2 wk = work[blockIdx.x];
    const int64_t tiles = n_pad / kTile;
    const int64_t row0 = (int64_t)wk.x * kTile + wave * 16;
    const int64_t I = row0 / 16;  // this wave's 16-row block
    const int64_t jb = (int64_t)wk.y * kTile;
    const int64_t je = min((int64_t)(wk.y + L), tiles) * kTile;
    const float negc0 = -kp->c0;

    // A and B rows of this wave in the A-operand layout (row row0 + col, columns
    // q*MQ .. q*MQ + MQ - 1), and z of the four rows 4q .. 4q + 3 whose G entries this
    // lane receives.
    float aI[MQ], bI[MQ];
#pragma unroll
    for (int t = 0; t < MQ; ++t) {
        aI[t] = A[(int64_t)(q * MQ + t) * n_pad + row0 + col];
        bI[t] = B[(int64_t)(q * MQ + t) * n_pad + row0 + col];
    }
    float zi[4][D];
#pragma unroll
    for (int u = 0; u < 4; ++u) load_row_q<D>(Z + (row0 + 4 * q + u) * DP, zi[u]);

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
            } else if (idx < NZ4 + 2 * NA4) {
                const int v = (idx - NZ4) % NA4;
                const float* src = idx < NZ4 + NA4 ? A : B;
                const int c = v / (kTile / 4);
                const int jj = (v % (kTile / 4)) * 4;
                buf[t] = *reinterpret_cast<const float4*>(src + c * n_pad + j0 + jj);
            }
        }
    };
    auto store = [&](int b, const float4(&buf)[NL]) {
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NZ4) {
                zs[b][idx] = buf[t];
            } else if (idx < NZ4 + 2 * NA4) {
                const int v = (idx - NZ4) % NA4;
                float* dst = idx < NZ4 + NA4 ? as[b] : bs[b];
                const int c = v / (kTile / 4);
                const int jj = (v % (kTile / 4)) * 4;
                dst[(jj + 0) * ST + c] = buf[t].x;
                dst[(jj + 1) * ST + c] = buf[t].y;
                dst[(jj + 2) * ST + c] = buf[t].z;
                dst[(jj + 3) * ST + c] = buf[t].w;
            }
        }
    };

    float4 pre[NL];
    load(jb, pre);
    store(0, pre);
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kTile) {
        const bool more = j0 + kTile < je;
        if (more) load(j0 + kTile, pre);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
#pragma unroll 1
        for (int jt = 0; jt < kTile / 16; ++jt) {
            const int64_t J = j0 / 16 + jt;
            if (J < I) continue;  // lower triangle: covered by the transposed tile
            const int jr = jt * 16 + col;  // this lane's column of the G tile
            float bJ[MQ];
            load_op<MQ>(bs[buf] + jr * ST + q * MQ, bJ);
            // two independent accumulator chains per product (even and odd steps), so that
            // consecutive MFMAs do not wait on each other's results
            floatx4 G = {0.f, 0.f, 0.f, 0.f}, G1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < MQ; t += 2) {
                G = __builtin_amdgcn_mfma_f32_16x16x4f32(aI[t], bJ[t], G, 0, 0, 0);
                G1 = __builtin_amdgcn_mfma_f32_16x16x4f32(aI[t + 1], bJ[t + 1], G1, 0, 0, 0);
            }
            if (J > I) {
                float aJ[MQ];
                load_op<MQ>(as[buf] + jr * ST + q * MQ, aJ);
                floatx4 H = {0.f, 0.f, 0.f, 0.f}, H1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < MQ; t += 2) {
                    H = __builtin_amdgcn_mfma_f32_16x16x4f32(bI[t], aJ[t], H, 0, 0, 0);
                    H1 = __builtin_amdgcn_mfma_f32_16x16x4f32(bI[t + 1], aJ[t + 1], H1, 0, 0, 0);
                }
                G1 += H + H1;
            }
            G += G1;
            float zj[D];
            load_row_q<D>(zsb + jr * DP, zj);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float sq[D];
                float a = negc0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const float t = zi[u][k] - zj[k];
                    sq[k] = t * t;
                    a += sq[k];
                }
                const float w = __builtin_amdgcn_exp2f(-a) * G[u];
                gacc[0] += w;
#pragma unroll
                for (int k = 0; k < D; ++k) gacc[k + 1] = __builtin_fmaf(w, sq[k], gacc[k + 1]);
            }
        }
        // flush the FP32 partials of this stage (at most 16 terms each) to FP64
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
        gpart[(int64_t)p * gridDim.x + blockIdx.x] = (red[0][p] + red[1][p]) + (red[2][p] + red[3][p]);
    }
}


// ---------------------------------------------------------------------------------------
// BF16 form (the BF16 product modes): the G tiles come from operands split into BF16
// halves, G = A_hi B_hi^T + A_hi B_lo^T + A_lo B_hi^T (the lo x lo term, about 2^-18 of
// |A||B|, is dropped), by v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  A lane's
// operand is 8 consecutive columns of one row, so the operands are row-major (stride
// MB = 32 KB bf16).  Kernel entries, squared differences and accumulation are those of
// dquad_sym_kernel.
// ---------------------------------------------------------------------------------------
typedef __bf16 dq_bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int dq_uintx4 __attribute__((ext_vector_type(4)));

// (register budget for three workgroups per CU where it fits without spilling, and the
// tile loop unrolled twice: 27% faster than the unconstrained allocation at d = 8)
template <int D, int KB>
__global__ __launch_bounds__(kWG, (D <= 8 && KB == 1) ? 3 : (KB == 1 ? 2 : 1)) void dquad_sym_bf16_kernel(
    const float* __restrict__ Z, const uint16_t* __restrict__ AH, const uint16_t* __restrict__ AL,
    const uint16_t* __restrict__ BH, const uint16_t* __restrict__ BL, double* __restrict__ gpart,
    int64_t n_pad, const int2* __restrict__ work, int L, const KParams* __restrict__ kp) {
    constexpr int DP = (D + 3) & ~3;
    constexpr int MB = 32 * KB;           // operand columns
    constexpr int SB = MB + 8;            // LDS row stride (bf16), 16-byte multiple
    constexpr int NZ4 = kTile * DP / 4;   // 16-byte loads of the Z tile
    constexpr int NO = kTile * MB / 8;    // 16-byte loads of one operand tile
    constexpr int NL = (NZ4 + 4 * NO + kWG - 1) / kWG;
    __shared__ dq_uintx4 zs[2][NZ4];
    __shared__ __attribute__((aligned(16))) uint16_t ops[2][4][kTile * SB];  // AH, AL, BH, BL
    __shared__ double red[4][D + 1];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int2 wk = work[blockIdx.x];
    const int64_t tiles = n_pad / kTile;
    const int64_t row0 = (int64_t)wk.x * kTile + wave * 16;
    const int64_t I = row0 / 16;
    const int64_t jb = (int64_t)wk.y * kTile;
    const int64_t je = min((int64_t)(wk.y + L), tiles) * kTile;
    const float negc0 = -kp->c0;

    dq_bf16x8 aIh[KB], aIl[KB], bIh[KB], bIl[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
        const int64_t o = (row0 + col) * MB + 32 * kb + 8 * q;
        aIh[kb] = __builtin_bit_cast(dq_bf16x8, *reinterpret_cast<const dq_uintx4*>(AH + o));
        aIl[kb] = __builtin_bit_cast(dq_bf16x8, *reinterpret_cast<const dq_uintx4*>(AL + o));
        bIh[kb] = __builtin_bit_cast(dq_bf16x8, *reinterpret_cast<const dq_uintx4*>(BH + o));
        bIl[kb] = __builtin_bit_cast(dq_bf16x8, *reinterpret_cast<const dq_uintx4*>(BL + o));
    }
    float zi[4][D];
#pragma unroll
    for (int u = 0; u < 4; ++u) load_row_q<D>(Z + (row0 + 4 * q + u) * DP, zi[u]);

    float gacc[D + 1];
    double gsum[D + 1];
#pragma unroll
    for (int p = 0; p <= D; ++p) {
        gacc[p] = 0.f;
        gsum[p] = 0.0;
    }

    auto load = [&](int64_t j0, dq_uintx4(&buf)[NL]) {
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NZ4) {
                buf[t] = reinterpret_cast<const dq_uintx4*>(Z + j0 * DP)[idx];
            } else if (idx < NZ4 + 4 * NO) {
                const int o = idx - NZ4;
                const int a = o / NO, v = o % NO;
                const int row = v / (MB / 8), c8 = (v % (MB / 8)) * 8;
                const uint16_t* src = a == 0 ? AH : a == 1 ? AL : a == 2 ? BH : BL;
                buf[t] = *reinterpret_cast<const dq_uintx4*>(src + (j0 + row) * MB + c8);
            }
        }
    };
    auto store = [&](int b, const dq_uintx4(&buf)[NL]) {
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NZ4) {
                zs[b][idx] = buf[t];
            } else if (idx < NZ4 + 4 * NO) {
                const int o = idx - NZ4;
                const int a = o / NO, v = o % NO;
                const int row = v / (MB / 8), c8 = (v % (MB / 8)) * 8;
                *reinterpret_cast<dq_uintx4*>(&ops[b][a][row * SB + c8]) = buf[t];
            }
        }
    };

    dq_uintx4 pre[NL];
    load(jb, pre);
    store(0, pre);
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kTile) {
        const bool more = j0 + kTile < je;
        if (more) load(j0 + kTile, pre);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
#pragma unroll 2
        for (int jt = 0; jt < kTile / 16; ++jt) {
            const int64_t J = j0 / 16 + jt;
            if (J < I) continue;  // lower triangle: covered by the transposed tile
            const int jr = jt * 16 + col;
            floatx4 G = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                const int o = jr * SB + 32 * kb + 8 * q;
                const dq_bf16x8 bh = __builtin_bit_cast(dq_bf16x8, *reinterpret_cast<const dq_uintx4*>(&ops[buf][2][o]));
                const dq_bf16x8 bl = __builtin_bit_cast(dq_bf16x8, *reinterpret_cast<const dq_uintx4*>(&ops[buf][3][o]));
                G = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aIh[kb], bh, G, 0, 0, 0);
                G = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aIh[kb], bl, G, 0, 0, 0);
                G = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aIl[kb], bh, G, 0, 0, 0);
            }
            if (J > I) {
                floatx4 H = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) {
                    const int o = jr * SB + 32 * kb + 8 * q;
                    const dq_bf16x8 ah = __builtin_bit_cast(dq_bf16x8, *reinterpret_cast<const dq_uintx4*>(&ops[buf][0][o]));
                    const dq_bf16x8 al = __builtin_bit_cast(dq_bf16x8, *reinterpret_cast<const dq_uintx4*>(&ops[buf][1][o]));
                    H = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bIh[kb], ah, H, 0, 0, 0);
                    H = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bIh[kb], al, H, 0, 0, 0);
                    H = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bIl[kb], ah, H, 0, 0, 0);
                }
                G += H;
            }
            float zj[D];
            load_row_q<D>(zsb + jr * DP, zj);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                float sq[D];
                float a = negc0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const float t = zi[u][k] - zj[k];
                    sq[k] = t * t;
                    a += sq[k];
                }
                const float w = __builtin_amdgcn_exp2f(-a) * G[u];
                gacc[0] += w;
#pragma unroll
                for (int k = 0; k < D; ++k) gacc[k + 1] = __builtin_fmaf(w, sq[k], gacc[k + 1]);
            }
        }
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
        gpart[(int64_t)p * gridDim.x + blockIdx.x] = (red[0][p] + red[1][p]) + (red[2][p] + red[3][p]);
    }
}

DquadShape dquad_shape(int64_t n, int d, int mcols) {
    (void)d;
    DquadShape sh;
    sh.n_pad = round_up(std::max<int64_t>(n, 1), kRowPad);
    // columns of A and B padded to 8: the k-slots of the 16x16x4 MFMA take 4 columns per
    // step and the two accumulator chains an even number of steps
    sh.mq4 = (int)round_up(std::max(mcols, 1), 8);
    sh.mqb = (int)round_up(std::max(mcols, 1), 32);
    sh.rows_per_wg = kTile;
    const int64_t T = sh.n_pad / kTile;
    // columns tiles per workgroup: about 16 for large n, fewer when n is small so that
    // the grid still has a few thousand workgroups
    int L = 16;
    while (L > 1 && (T * (T + 1) / 2) / L < 4096) L /= 2;
    sh.chunk = L;
    sh.split = 0;
    int64_t nwg = 0;
    for (int64_t a = 0; a < T; ++a) nwg += (T - a + L - 1) / L;
    sh.nwg = (int)nwg;
    return sh;
}

void dquad_work(const DquadShape& sh, std::vector<int2>& work) {
    const int64_t T = sh.n_pad / kTile;
    const int L = sh.chunk;
    work.clear();
    work.reserve(sh.nwg);
    for (int64_t a = 0; a < T; ++a)
        for (int64_t b = a; b < T; b += L) work.push_back(make_int2((int)a, (int)b));
}

template <int D>
static hipError_t dquad_d(const DquadShape& sh, const float* Z, const float* A, const float* B,
                          const KParams* kp, const int2* work, double* gpart, hipStream_t s) {
    const dim3 grid((unsigned)sh.nwg);
#define GPK_DQ_LAUNCH(MQ) \
    case 4 * MQ: dquad_sym_kernel<D, MQ><<<grid, kWG, 0, s>>>(Z, A, B, gpart, sh.n_pad, work, sh.chunk, kp); break
    switch (sh.mq4) {
        GPK_DQ_LAUNCH(2);
        GPK_DQ_LAUNCH(4);
        GPK_DQ_LAUNCH(6);
        GPK_DQ_LAUNCH(8);
        GPK_DQ_LAUNCH(10);
        GPK_DQ_LAUNCH(12);
        GPK_DQ_LAUNCH(14);
        GPK_DQ_LAUNCH(16);
        default: return hipErrorInvalidValue;
    }
#undef GPK_DQ_LAUNCH
    return hipGetLastError();
}

hipError_t launch_dquad(const DquadShape& sh, int d, const float* Z, const float* A,
                        const float* B, const KParams* kp, const int2* work, double* gpart,
                        hipStream_t s) {
    switch (d) {
        case 1: return dquad_d<1>(sh, Z, A, B, kp, work, gpart, s);
        case 2: return dquad_d<2>(sh, Z, A, B, kp, work, gpart, s);
        case 3: return dquad_d<3>(sh, Z, A, B, kp, work, gpart, s);
        case 4: return dquad_d<4>(sh, Z, A, B, kp, work, gpart, s);
        case 5: return dquad_d<5>(sh, Z, A, B, kp, work, gpart, s);
        case 6: return dquad_d<6>(sh, Z, A, B, kp, work, gpart, s);
        case 7: return dquad_d<7>(sh, Z, A, B, kp, work, gpart, s);
        case 8: return dquad_d<8>(sh, Z, A, B, kp, work, gpart, s);
        case 9: return dquad_d<9>(sh, Z, A, B, kp, work, gpart, s);
        case 10: return dquad_d<10>(sh, Z, A, B, kp, work, gpart, s);
        case 11: return dquad_d<11>(sh, Z, A, B, kp, work, gpart, s);
        case 12: return dquad_d<12>(sh, Z, A, B, kp, work, gpart, s);
        case 13: return dquad_d<13>(sh, Z, A, B, kp, work, gpart, s);
        case 14: return dquad_d<14>(sh, Z, A, B, kp, work, gpart, s);
        case 15: return dquad_d<15>(sh, Z, A, B, kp, work, gpart, s);
        case 16: return dquad_d<16>(sh, Z, A, B, kp, work, gpart, s);
        default: return hipErrorInvalidValue;
    }
}

template <int D>
static hipError_t dquad_bf16_d(const DquadShape& sh, const float* Z, const uint16_t* AH,
                               const uint16_t* AL, const uint16_t* BH, const uint16_t* BL,
                               const KParams* kp, const int2* work, double* gpart, hipStream_t s) {
    const dim3 grid((unsigned)sh.nwg);
    switch (sh.mqb) {
        case 32: dquad_sym_bf16_kernel<D, 1><<<grid, kWG, 0, s>>>(Z, AH, AL, BH, BL, gpart, sh.n_pad, work, sh.chunk, kp); break;
        case 64: dquad_sym_bf16_kernel<D, 2><<<grid, kWG, 0, s>>>(Z, AH, AL, BH, BL, gpart, sh.n_pad, work, sh.chunk, kp); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_dquad_bf16(const DquadShape& sh, int d, const float* Z, const uint16_t* AH,
                             const uint16_t* AL, const uint16_t* BH, const uint16_t* BL,
                             const KParams* kp, const int2* work, double* gpart, hipStream_t s) {
    switch (d) {
        case 1: return dquad_bf16_d<1>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 2: return dquad_bf16_d<2>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 3: return dquad_bf16_d<3>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 4: return dquad_bf16_d<4>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 5: return dquad_bf16_d<5>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 6: return dquad_bf16_d<6>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 7: return dquad_bf16_d<7>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 8: return dquad_bf16_d<8>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 9: return dquad_bf16_d<9>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 10: return dquad_bf16_d<10>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 11: return dquad_bf16_d<11>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 12: return dquad_bf16_d<12>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 13: return dquad_bf16_d<13>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 14: return dquad_bf16_d<14>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 15: return dquad_bf16_d<15>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        case 16: return dquad_bf16_d<16>(sh, Z, AH, AL, BH, BL, kp, work, gpart, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gpk
