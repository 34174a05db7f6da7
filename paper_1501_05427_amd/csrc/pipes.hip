// Issue-rate probe of the compute pipes that the covariance products use: FP32 VALU FMAs,
// v_exp_f32, FP32 MFMA (v_mfma_f32_16x16x4f32) and BF16 MFMA (v_mfma_f32_16x16x32_bf16),
// alone and with independent VALU work in the same loop.  With eight waves per SIMD the
// scheduler is free to issue one wave's VALU work while another wave's MFMA runs, so the
// time of "MFMA + VALU" against the sum of the two alone shows how much of the MFMA time
// the VALU work can hide.  Every kernel writes one float per thread so that nothing is
// optimised away.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace gpk {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// MODE: 0 VALU, 1 FP32 MFMA, 2 FP32 MFMA + VALU, 3 BF16 MFMA, 4 BF16 MFMA + VALU, 5 exp.
// Per iteration: 128 VALU FMAs in eight independent chains, 4 MFMAs on four independent
// accumulators, or 128 exp2 in eight chains.
template <int MODE>
__global__ __launch_bounds__(256) void pipe_probe_kernel(float* __restrict__ out, int iters, float s) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    float a0 = threadIdx.x * 1e-3f, a1 = a0 + 1, a2 = a0 + 2, a3 = a0 + 3, a4 = a0 + 4,
          a5 = a0 + 5, a6 = a0 + 6, a7 = a0 + 7;
    floatx4 c0 = {0.f, 0.f, 0.f, 0.f}, c1 = c0, c2 = c0, c3 = c0;
    const float av = s * threadIdx.x, bv = s + threadIdx.x;
    bf16x8 ab, bb;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        ab[t] = (__bf16)(av + t);
        bb[t] = (__bf16)(bv - t);
    }
    for (int it = 0; it < iters; ++it) {
        if constexpr (MODE == 1 || MODE == 2) {
            c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, c1, 0, 0, 0);
            c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, c2, 0, 0, 0);
            c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, c3, 0, 0, 0);
        }
        if constexpr (MODE == 3 || MODE == 4) {
            c0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, c0, 0, 0, 0);
            c1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, c1, 0, 0, 0);
            c2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, c2, 0, 0, 0);
            c3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ab, bb, c3, 0, 0, 0);
        }
        if constexpr (MODE == 0 || MODE == 2 || MODE == 4) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                a0 = __builtin_fmaf(a0, s, a1); a1 = __builtin_fmaf(a1, s, a2);
                a2 = __builtin_fmaf(a2, s, a3); a3 = __builtin_fmaf(a3, s, a4);
                a4 = __builtin_fmaf(a4, s, a5); a5 = __builtin_fmaf(a5, s, a6);
                a6 = __builtin_fmaf(a6, s, a7); a7 = __builtin_fmaf(a7, s, a0);
            }
        }
        if constexpr (MODE == 5) {
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                a0 = __builtin_amdgcn_exp2f(a0); a1 = __builtin_amdgcn_exp2f(a1);
                a2 = __builtin_amdgcn_exp2f(a2); a3 = __builtin_amdgcn_exp2f(a3);
                a4 = __builtin_amdgcn_exp2f(a4); a5 = __builtin_amdgcn_exp2f(a5);
                a6 = __builtin_amdgcn_exp2f(a6); a7 = __builtin_amdgcn_exp2f(a7);
            }
        }
    }
    out[gid] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7 + c0[0] + c1[1] + c2[2] + c3[3];
}

}  // namespace

hipError_t launch_pipe_probe(int mode, int blocks, int iters, float* out, hipStream_t s) {
    const float sc = 0.999f;
    switch (mode) {
        case 0: pipe_probe_kernel<0><<<blocks, 256, 0, s>>>(out, iters, sc); break;
        case 1: pipe_probe_kernel<1><<<blocks, 256, 0, s>>>(out, iters, sc); break;
        case 2: pipe_probe_kernel<2><<<blocks, 256, 0, s>>>(out, iters, sc); break;
        case 3: pipe_probe_kernel<3><<<blocks, 256, 0, s>>>(out, iters, sc); break;
        case 4: pipe_probe_kernel<4><<<blocks, 256, 0, s>>>(out, iters, sc); break;
        case 5: pipe_probe_kernel<5><<<blocks, 256, 0, s>>>(out, iters, sc); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace gpk
