// Shared device-side definitions of the HIP library: the covariance parameter block,
// Philox4x64-10, draw mappings and FP64 reductions.  gfx950 only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpk {

constexpr int kMaxD = 16;
constexpr int kMaxP = kMaxD + 2;
constexpr int kWG = 256;          // threads per workgroup of the streaming kernels
constexpr int kRowPad = 256;      // row padding of every internal n-length buffer

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Covariance parameters derived on the device from psi (never read back by the host).
//   K_f(i, j) = exp2(c0 - sum_k (z_ik - z_jk)^2),  z_ik = x_ik * sc[k]
//   sc[k] = sqrt(log2(e) / 2) / ell_k,  c0 = log2(sigma^2)
struct KParams {
    float c0;
    float lam;
    float sc[kMaxD];
    double sigma2;
    double lam64;
    double psi[kMaxP];
};

// Counter words of the three draw purposes.
constexpr uint64_t kPurposeProbe = 1, kPurposeUlisse = 2, kPurposeSgld = 3;

// ---------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC 2011): 10 rounds of two 64x64->128
// multiplications per round with a Weyl-sequence key schedule.
// ---------------------------------------------------------------------------------------
struct u64x4 {
    uint64_t v[4];
};

__host__ __device__ inline uint64_t mulhi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul64hi(a, b);
#else
    return (uint64_t)(((unsigned __int128)a * b) >> 64);
#endif
}

__host__ __device__ inline u64x4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                uint64_t c3, uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t lo0 = M0 * c0, hi0 = mulhi64(M0, c0);
        const uint64_t lo1 = M1 * c2, hi1 = mulhi64(M1, c2);
        const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    u64x4 o;
    o.v[0] = c0;
    o.v[1] = c1;
    o.v[2] = c2;
    o.v[3] = c3;
    return o;
}

// [0, 1) and (0, 1] from the top 53 bits of a word.
__host__ __device__ inline double u01_co(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }
__host__ __device__ inline double u01_oc(uint64_t x) {
    return ((double)(x >> 11) + 1.0) * 0x1.0p-53;
}

// Box-Muller on a pair of words: radius from the (0, 1] uniform, angle from the [0, 1) one.
__device__ inline void box_muller(uint64_t xa, uint64_t xb, double* za, double* zb) {
    const double r = sqrt(-2.0 * log(u01_oc(xa)));
    const double t = 2.0 * M_PI * u01_co(xb);
    double s, c;
    sincos(t, &s, &c);
    *za = r * c;
    *zb = r * s;
}

// ---------------------------------------------------------------------------------------
// Reductions (64-wide wavefronts).
// ---------------------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a 256-thread workgroup in a fixed order; result valid in every thread.
// `scratch` holds at least 4 doubles; calls must be separated by the caller's own barrier
// when scratch is reused.
__device__ inline double block_sum256(double v, double* scratch) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) scratch[w] = v;
    __syncthreads();
    const double s = (scratch[0] + scratch[1]) + (scratch[2] + scratch[3]);
    __syncthreads();
    return s;
}

}  // namespace gpk
