// Matrix-free covariance products for the squared-exponential ARD kernel plus noise.
//
// K(i, j) = sigma^2 exp(-1/2 sum_k (x_ik - x_jk)^2 / ell_k^2) + lambda delta_ij is never
// stored: every workgroup rebuilds its tiles of K from the pre-scaled inputs
// z_ik = x_ik sqrt(log2(e)/2) / ell_k, so that K_f(i, j) = exp2(log2 sigma^2 - |z_i - z_j|^2)
// with the distance formed from explicit FP32 differences.  The product with V is a
// VALU contraction for fewer than 16 right-hand sides and an MFMA contraction otherwise,
// with K generated directly in the MFMA A-operand layout: FP32 MFMA
// (v_mfma_f32_16x16x4f32) in GP_FP32 mode, BF16 MFMA (v_mfma_f32_16x16x32_bf16) with a
// hi+lo split of V (and optionally of K) in the BF16 modes.  Work is split over (row tile, column chunk); chunk partials are summed in a
// fixed order by a second kernel in FP64, which also adds lambda V.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "gp_common.h"
#include "internal.h"

namespace gpk {

constexpr int kJS = 64;  // columns of K per LDS stage

// ---------------------------------------------------------------------------------------
// psi -> parameters and scaled inputs
// ---------------------------------------------------------------------------------------
__global__ void prep_kernel(const float* __restrict__ X, int64_t n, int d, int64_t ldx,
                            const double* __restrict__ psi, float* __restrict__ Z, int64_t n_pad,
                            KParams* __restrict__ kp) {
    const int dp = (d + 3) & ~3;
    const double base = sqrt(0.5 / M_LN2);  // sqrt(log2(e) / 2)
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        KParams p;
        p.c0 = (float)(psi[0] / M_LN2);
        p.sigma2 = exp(psi[0]);
        p.lam64 = exp(psi[d + 1]);
        p.lam = (float)p.lam64;
        for (int k = 0; k < kMaxD; ++k) p.sc[k] = k < d ? (float)(base * exp(-psi[1 + k])) : 0.f;
        for (int k = 0; k < kMaxP; ++k) p.psi[k] = k < d + 2 ? psi[k] : 0.0;
        *kp = p;
    }
    const int64_t total = n_pad * dp;
    for (int64_t e = t; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / dp;
        const int k = (int)(e % dp);
        float z = 0.f;
        if (i < n && k < d) z = (float)((double)X[i * ldx + k] * (base * exp(-psi[1 + k])));
        Z[e] = z;
    }
}

__global__ void pack_kernel(const float* __restrict__ V, int64_t n, int m, int64_t ldv,
                            float* __restrict__ Vp, int64_t n_pad, int mp) {
    const int64_t total = n_pad * mp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / n_pad);
        const int64_t i = e % n_pad;
        Vp[e] = (i < n && c < m) ? V[c * ldv + i] : 0.f;
    }
}

// ---------------------------------------------------------------------------------------
// Stage loader: kJS rows of Z (row-major, DP floats each) and kJS entries of MP columns of
// V (column-major, ld n_pad) through registers into LDS.  V is stored in LDS either
// column-major with a padded stride (MFMA B-operand reads) or row-major (VALU broadcast).
// Every load count is a multiple of 64, so the bounds tests below are uniform per wave.
// The staged values are native vector types: copies of HIP's float4/uint4 structs lower
// to memcpy, which keeps the stage in private (scratch) memory instead of registers.
// ---------------------------------------------------------------------------------------
typedef unsigned int uintx4 __attribute__((ext_vector_type(4)));

template <int DP, int MP, bool VROWMAJOR>
struct Stage {
    static constexpr int NZ4 = kJS * DP / 4;
    static constexpr int NV4 = MP * kJS / 4;
    static constexpr int LZ = (NZ4 + kWG - 1) / kWG;
    static constexpr int LV = (NV4 + kWG - 1) / kWG;
    static constexpr int VST = VROWMAJOR ? MP : (kJS + 4);
    static constexpr int VSIZE = VROWMAJOR ? kJS * MP : MP * (kJS + 4);
    static_assert(NZ4 % 64 == 0 && NV4 % 64 == 0, "wave-uniform stage loads");

    floatx4 z[LZ];
    floatx4 v[LV];

    __device__ __attribute__((always_inline)) void load(const float* __restrict__ Z, const float* __restrict__ V, int64_t ldv,
                         int64_t j0) {
#pragma unroll
        for (int t = 0; t < LZ; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NZ4) z[t] = reinterpret_cast<const floatx4*>(Z + j0 * DP)[idx];
        }
#pragma unroll
        for (int t = 0; t < LV; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NV4) {
                const int c = idx / (kJS / 4);
                const int jj = (idx % (kJS / 4)) * 4;
                v[t] = *reinterpret_cast<const floatx4*>(V + c * ldv + j0 + jj);
            }
        }
    }
    __device__ __attribute__((always_inline)) void store(float4* __restrict__ zs, float* __restrict__ vs) const {
#pragma unroll
        for (int t = 0; t < LZ; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NZ4) reinterpret_cast<floatx4*>(zs)[idx] = z[t];
        }
#pragma unroll
        for (int t = 0; t < LV; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NV4) {
                const int c = idx / (kJS / 4);
                const int jj = (idx % (kJS / 4)) * 4;
                if (VROWMAJOR) {
                    vs[(jj + 0) * MP + c] = v[t].x;
                    vs[(jj + 1) * MP + c] = v[t].y;
                    vs[(jj + 2) * MP + c] = v[t].z;
                    vs[(jj + 3) * MP + c] = v[t].w;
                } else {
                    *reinterpret_cast<floatx4*>(vs + c * VST + jj) = v[t];
                }
            }
        }
    }
};

// The same for the BF16 halves of a split V (column-major bf16, ld n_pad): MP columns of
// kJS entries per part, kept column-major in LDS with a padded stride of VST bf16.
template <int DP, int MP>
struct StageB16 {
    static constexpr int NZ4 = kJS * DP / 4;
    static constexpr int NV = MP * kJS * 2 / 16;  // 16-byte loads per part
    static constexpr int LZ = (NZ4 + kWG - 1) / kWG;
    static constexpr int LV = (NV + kWG - 1) / kWG;
    static constexpr int VST = kJS + 8;
    static constexpr int VSIZE = MP * VST;
    static_assert(NZ4 % 64 == 0 && NV % 64 == 0, "wave-uniform stage loads");

    floatx4 z[LZ];
    uintx4 h[LV], l[LV];

    __device__ __attribute__((always_inline)) void load(const float* __restrict__ Z, const uint16_t* __restrict__ VH,
                         const uint16_t* __restrict__ VL, int64_t ldv, int64_t j0) {
#pragma unroll
        for (int t = 0; t < LZ; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NZ4) z[t] = reinterpret_cast<const floatx4*>(Z + j0 * DP)[idx];
        }
#pragma unroll
        for (int t = 0; t < LV; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NV) {
                const int c = idx / (kJS / 8);
                const int jj = (idx % (kJS / 8)) * 8;
                h[t] = *reinterpret_cast<const uintx4*>(VH + c * ldv + j0 + jj);
                if (VL != nullptr) l[t] = *reinterpret_cast<const uintx4*>(VL + c * ldv + j0 + jj);
            }
        }
    }
    __device__ __attribute__((always_inline)) void store(float4* __restrict__ zs, uint16_t* __restrict__ hs,
                          uint16_t* __restrict__ ls, bool with_lo) const {
#pragma unroll
        for (int t = 0; t < LZ; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NZ4) reinterpret_cast<floatx4*>(zs)[idx] = z[t];
        }
#pragma unroll
        for (int t = 0; t < LV; ++t) {
            const int idx = threadIdx.x + t * kWG;
            if (idx < NV) {
                const int c = idx / (kJS / 8);
                const int jj = (idx % (kJS / 8)) * 8;
                *reinterpret_cast<uintx4*>(hs + c * VST + jj) = h[t];
                if (with_lo) *reinterpret_cast<uintx4*>(ls + c * VST + jj) = l[t];
            }
        }
    }
};

template <int D>
__device__ inline void load_row(const float* __restrict__ p, float (&z)[D]) {
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

// exp2(c0 - |zi - zj|^2): acc starts at -c0, the FMA chain adds the squared differences.
template <int D>
__device__ inline float kf_entry(const float (&zi)[D], const float (&zj)[D], float negc0) {
    float a = negc0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        const float t = zi[k] - zj[k];
        a = __builtin_fmaf(t, t, a);
    }
    return __builtin_amdgcn_exp2f(-a);
}

// ---------------------------------------------------------------------------------------
// MFMA FP32 product: each wave owns R blocks of 16 rows; each lane keeps z_i of its row
// (lane % 16) for every block.  Inside a 16-column group, lane l takes columns
// j = 4 (l / 16) + s for s = 0..3 -- the k-slot of v_mfma_f32_16x16x4f32 is l / 16 -- so
// the B operand of four consecutive MFMA steps is one 16-byte LDS read.
// TC > 0 right-hand sides past the NB MFMA blocks (m = 16 NB + TC, TC <= 4) go through
// the VALU instead of a mostly empty extra MFMA block: each lane accumulates
// K_ij V_jc over its own k-slots, and the four k-slot lanes of a row (l % 16 equal) are
// summed by cross-lane shuffles once at the end.  V is staged with 16 NB + 4 columns.
// ---------------------------------------------------------------------------------------
template <int D, int NB, int TC, int R>
__global__ __launch_bounds__(kWG) void kmv_mfma_f32_kernel(
    const float* __restrict__ Z, const float* __restrict__ V, int64_t ldv,
    float* __restrict__ part, int64_t n_pad, int chunk, int split,
    const KParams* __restrict__ kp, const int* __restrict__ n_active) {
    if (n_active != nullptr && *n_active == 0) return;
    constexpr int DP = (D + 3) & ~3;
    static_assert(TC >= 0 && TC <= 4, "at most four VALU columns");
    constexpr int MP = NB * 16 + (TC > 0 ? 4 : 0);
    constexpr int TCA = TC > 0 ? TC : 1;  // array extent (unused when TC == 0)
    using S = Stage<DP, MP, false>;
    __shared__ float4 zs[2][S::NZ4];
    __shared__ float vs[2][S::VSIZE];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int cidx = blockIdx.x % split;
    const int64_t rt = blockIdx.x / split;
    const int64_t row0 = rt * (64 * R) + wave * (16 * R);
    const int64_t jb = (int64_t)cidx * chunk;
    const int64_t je = min(jb + (int64_t)chunk, n_pad);
    const float negc0 = -kp->c0;

    float zi[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r) load_row<D>(Z + (row0 + r * 16 + col) * DP, zi[r]);

    floatx4 acc[R][NB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[r][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    float tacc[R][TCA];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < TCA; ++t) tacc[r][t] = 0.f;

    S st;
    if (jb < je) {
        st.load(Z, V, ldv, jb);
        st.store(zs[0], vs[0]);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kJS) {
        const bool more = j0 + kJS < je;
        if (more) st.load(Z, V, ldv, j0 + kJS);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
        const float* vsb = vs[buf];
#pragma unroll 1
        for (int g = 0; g < kJS / 16; ++g) {
            float4 vv[NB];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb)
                vv[cb] = *reinterpret_cast<const float4*>(vsb + (cb * 16 + col) * S::VST + g * 16 + 4 * q);
            float4 vt[TCA];
#pragma unroll
            for (int t = 0; t < TC; ++t)
                vt[t] = *reinterpret_cast<const float4*>(vsb + (NB * 16 + t) * S::VST + g * 16 + 4 * q);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                float zj[D];
                load_row<D>(zsb + (g * 16 + 4 * q + s) * DP, zj);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const float kv = kf_entry<D>(zi[r], zj, negc0);
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb) {
                        const float b = s == 0 ? vv[cb].x : s == 1 ? vv[cb].y : s == 2 ? vv[cb].z : vv[cb].w;
                        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv, b, acc[r][cb], 0, 0, 0);
                    }
#pragma unroll
                    for (int t = 0; t < TC; ++t) {
                        const float b = s == 0 ? vt[t].x : s == 1 ? vt[t].y : s == 2 ? vt[t].z : vt[t].w;
                        tacc[r][t] = __builtin_fmaf(kv, b, tacc[r][t]);
                    }
                }
            }
        }
        if (more) st.store(zs[buf ^ 1], vs[buf ^ 1]);
        __syncthreads();
        buf ^= 1;
    }
    // lane holds rows 4q..4q+3 of column cb*16 + col: one 16-byte store per block
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            const int64_t i = row0 + r * 16 + 4 * q;
            const int c = cb * 16 + col;
            float4 o;
            o.x = acc[r][cb][0];
            o.y = acc[r][cb][1];
            o.z = acc[r][cb][2];
            o.w = acc[r][cb][3];
            *reinterpret_cast<float4*>(part + ((int64_t)cidx * MP + c) * n_pad + i) = o;
        }
    // VALU columns: sum the four k-slot lanes of each row (lanes col, col + 16, col + 32,
    // col + 48); the lanes of k-slot 0 store rows row0 + 16 r + col
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < TC; ++t) {
            float v = tacc[r][t];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (q == 0) part[((int64_t)cidx * MP + NB * 16 + t) * n_pad + row0 + r * 16 + col] = v;
        }
}

// ---------------------------------------------------------------------------------------
// Symmetric FP32 product.  K is symmetric, so an entry K_ij off the diagonal blocks serves
// both out_i += K_ij v_j and out_j += K_ij v_i: computed once, it halves the VALU work of
// forming K, which with the FP32 matrix unit (whose instructions do not overlap with VALU
// instructions on this chip) sets the time of the product.
//
// Work item (k, I): row tile I (256 rows: 4 waves x 4 blocks of 16) against the columns of
// column chunk k (cs columns), from column 256 I on when the chunk holds the tile's diagonal
// block.  Stages of 64 columns inside the diagonal block are forward only (all their
// entries); the others are symmetric: the forward product is the MFMA chain of
// kmv_mfma_f32_kernel, and the transposed one takes each 16 x 16 block of K through a
// per-wave LDS tile into the A-operand layout of (K^T)(16 j x 4 i), against the wave's own
// rows of V held in registers.  The four waves' transposed partials of a stage are summed
// in LDS in a fixed order and stored per row tile.  A right-hand-side column past the MFMA
// blocks (tc = 1) is taken on the VALU in both directions.
//
// Outputs (float, ld n_pad): F[k][c][i], the forward sums of chunk k for the rows of tiles
// whose diagonal chunk is at or before k; Tt[I][c][j], the transposed sums of tile I for
// columns j past its diagonal block.  kmv_sym_reduce_kernel adds them up in a fixed order.
// ---------------------------------------------------------------------------------------
constexpr int kSymTile = 256;  // rows of a row tile (4 waves x 4 blocks of 16)

__device__ inline void sym_item(int bid, int NT, int cs, int* k_out, int* I_out) {
    // Full items first, chunk-major: chunk k pairs with the tiles I wholly before it
    // (256 I < k cs, cs columns each).  Then the items that hold a diagonal tile, heaviest
    // first: offset s = I mod (cs / 256) ascending (cs - 256 s columns), chunk-major inside
    // an offset.  The hardware hands out workgroups in about this order, so the last round
    // of the grid is filled by the lightest items.
    const int per = cs / kSymTile;
    const int nch = (NT + per - 1) / per;
    for (int k = 1; k < nch; ++k) {
        const int cnt = k * per;
        if (bid < cnt) {
            *k_out = k;
            *I_out = bid;
            return;
        }
        bid -= cnt;
    }
    for (int o = 0;; ++o) {
        const int cnt = (NT - o + per - 1) / per;  // chunks with a tile at offset o
        if (bid < cnt) {
            *k_out = bid;
            *I_out = bid * per + o;
            return;
        }
        bid -= cnt;
    }
}

template <int D, int NB, int TC>
__global__ __launch_bounds__(kWG) void kmv_sym_f32_kernel(
    const float* __restrict__ Z, const float* __restrict__ V, float* __restrict__ F,
    float* __restrict__ Tt, int64_t n_pad, int NT, int cs, const KParams* __restrict__ kp,
    const int* __restrict__ n_active) {
    if (n_active != nullptr && *n_active == 0) return;
    constexpr int R = 4;
    constexpr int DP = (D + 3) & ~3;
    static_assert(TC == 0 || TC == 1, "at most one VALU column");
    constexpr int MP = NB * 16 + (TC > 0 ? 4 : 0);
    constexpr int MU = NB * 16 + TC;    // columns with results
    constexpr int TCA = TC > 0 ? TC : 1;
    constexpr int RS = 20;              // row stride of a wave's 16 x 16 transpose tile
    constexpr int RED = MU + 1;         // row stride of a wave's transposed partial
    using S = Stage<DP, MP, false>;
    __shared__ float4 zs[2][S::NZ4];
    __shared__ float vs[2][S::VSIZE];
    __shared__ __align__(16) float tb[4][16 * RS];
    __shared__ float red[4][64 * RED];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    int k, I;
    sym_item(blockIdx.x, NT, cs, &k, &I);
    const int64_t tile0 = (int64_t)I * kSymTile;
    const int64_t row0 = tile0 + wave * (16 * R);
    const int64_t diag_end = tile0 + kSymTile;
    const int64_t jb = max((int64_t)k * cs, tile0);
    const int64_t je = min((int64_t)(k + 1) * cs, n_pad);
    const float negc0 = -kp->c0;

    float zi[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r) load_row<D>(Z + (row0 + r * 16 + col) * DP, zi[r]);
    // the wave's own rows of V, B operand of the transposed product: lane (q, col) holds
    // V[row0 + 16 r + 4 q + t][16 cb + col] for t = 0..3
    float vI[R][4][NB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) vI[r][t][cb] = V[(cb * 16 + col) * n_pad + row0 + r * 16 + 4 * q + t];
    float vIt[R][TCA];  // the VALU column at the lane's own rows
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < TCA; ++t) vIt[r][t] = TC > 0 ? V[(NB * 16 + t) * n_pad + row0 + r * 16 + col] : 0.f;
    // complete these loads here: used inside the stage loop, they would otherwise make the
    // compiler wait for every outstanding load there, the next stage's prefetch included
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) asm volatile("" : "+v"(vI[r][t][cb]));
#pragma unroll
        for (int t = 0; t < TCA; ++t) asm volatile("" : "+v"(vIt[r][t]));
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) asm volatile("" : "+v"(zi[r][k2]));
    }

    floatx4 acc[R][NB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[r][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    float tacc[R][TCA];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < TCA; ++t) tacc[r][t] = 0.f;

    float* tbw = tb[wave];
    float* redw = red[wave];
    S st;
    st.load(Z, V, n_pad, jb);
    st.store(zs[0], vs[0]);
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kJS) {
        const bool more = j0 + kJS < je;
        const bool sym = j0 >= diag_end;  // uniform over the workgroup
        if (more) st.load(Z, V, n_pad, j0 + kJS);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
        const float* vsb = vs[buf];
#pragma unroll 1
        for (int g = 0; g < kJS / 16; ++g) {
            float4 vv[NB];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb)
                vv[cb] = *reinterpret_cast<const float4*>(vsb + (cb * 16 + col) * S::VST + g * 16 + 4 * q);
            float4 vt[TCA];
#pragma unroll
            for (int t = 0; t < TC; ++t)
                vt[t] = *reinterpret_cast<const float4*>(vsb + (NB * 16 + t) * S::VST + g * 16 + 4 * q);
            float kv[R][4];
#pragma unroll
            for (int s_ = 0; s_ < 4; ++s_) {
                float zj[D];
                load_row<D>(zsb + (g * 16 + 4 * q + s_) * DP, zj);
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    kv[r][s_] = kf_entry<D>(zi[r], zj, negc0);
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb) {
                        const float b = s_ == 0 ? vv[cb].x : s_ == 1 ? vv[cb].y : s_ == 2 ? vv[cb].z : vv[cb].w;
                        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[r][s_], b, acc[r][cb], 0, 0, 0);
                    }
#pragma unroll
                    for (int t = 0; t < TC; ++t) {
                        const float b = s_ == 0 ? vt[t].x : s_ == 1 ? vt[t].y : s_ == 2 ? vt[t].z : vt[t].w;
                        tacc[r][t] = __builtin_fmaf(kv[r][s_], b, tacc[r][t]);
                    }
                }
            }
            if (sym) {
                // transposed: out_j += sum_i K_ij V_i for the 16 columns j of this group
                floatx4 tr[NB];
#pragma unroll
                for (int cb = 0; cb < NB; ++cb) tr[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    // tb[j][i] = K(16 r + i, 16 g + j): lane (q, col) holds i = col, j = 4 q + s
#pragma unroll
                    for (int s_ = 0; s_ < 4; ++s_) tbw[(4 * q + s_) * RS + col] = kv[r][s_];
                    // the other lanes' writes before the reads, the reads before the next writes
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    // A operand of K^T: lane (q, col) takes j = col, i = 4 q + t
                    const float4 a = *reinterpret_cast<const float4*>(tbw + col * RS + 4 * q);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        const float at = t == 0 ? a.x : t == 1 ? a.y : t == 2 ? a.z : a.w;
#pragma unroll
                        for (int cb = 0; cb < NB; ++cb)
                            tr[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(at, vI[r][t][cb], tr[cb], 0, 0, 0);
                    }
                }
                // lane (q, col) holds columns j = 16 g + 4 q + v of output column 16 cb + col
#pragma unroll
                for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                    for (int v = 0; v < 4; ++v) redw[(g * 16 + 4 * q + v) * RED + cb * 16 + col] = tr[cb][v];
#pragma unroll
                for (int t = 0; t < TC; ++t) {
#pragma unroll
                    for (int s_ = 0; s_ < 4; ++s_) {
                        float p = 0.f;
#pragma unroll
                        for (int r = 0; r < R; ++r) p = __builtin_fmaf(kv[r][s_], vIt[r][t], p);
                        // sum over the 16 rows of each block: lanes with equal q
                        p += __shfl_xor(p, 1);
                        p += __shfl_xor(p, 2);
                        p += __shfl_xor(p, 4);
                        p += __shfl_xor(p, 8);
                        if (col == 0) redw[(g * 16 + 4 * q + s_) * RED + NB * 16 + t] = p;
                    }
                }
            }
        }
        if (more) st.store(zs[buf ^ 1], vs[buf ^ 1]);
        __syncthreads();
        if (sym) {
            // the four waves' partials in a fixed order -> Tt[I][c][j0 + j]
            for (int e = threadIdx.x; e < MU * kJS; e += kWG) {
                const int c = e / kJS, j = e % kJS;
                const float v = ((red[0][j * RED + c] + red[1][j * RED + c]) + red[2][j * RED + c]) + red[3][j * RED + c];
                Tt[((int64_t)I * MP + c) * n_pad + j0 + j] = v;
            }
            __syncthreads();
        }
        buf ^= 1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            const int64_t i = row0 + r * 16 + 4 * q;
            const int c = cb * 16 + col;
            float4 o;
            o.x = acc[r][cb][0];
            o.y = acc[r][cb][1];
            o.z = acc[r][cb][2];
            o.w = acc[r][cb][3];
            *reinterpret_cast<float4*>(F + ((int64_t)k * MP + c) * n_pad + i) = o;
        }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int t = 0; t < TC; ++t) {
            float v = tacc[r][t];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (q == 0) F[((int64_t)k * MP + NB * 16 + t) * n_pad + row0 + r * 16 + col] = v;
        }
}

// out[c][i] = sum over the chunks at or after row i's diagonal chunk of F[k][c][i] + sum over
// the row tiles before row i's of Tt[I][c][i], in that fixed order, in FP64.
__global__ void kmv_sym_reduce_kernel(const float* __restrict__ F, const float* __restrict__ Tt,
                                      float* __restrict__ out, int64_t n_pad, int mp, int mu,
                                      int cs, int nch, const int* __restrict__ n_active) {
    if (n_active != nullptr && *n_active == 0) return;
    const int64_t total = (int64_t)mu * n_pad;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / n_pad);
        const int64_t i = e % n_pad;
        const int tile = (int)(i / kSymTile);
        const int kd = (int)((int64_t)tile * kSymTile / cs);
        // loads in batches of eight so that many are in flight; the sum keeps its order
        const int64_t pl = (int64_t)mp * n_pad;
        double s = 0.0;
        const float* f = F + (int64_t)kd * pl + (int64_t)c * n_pad + i;
        int k = kd;
        for (; k + 8 <= nch; k += 8, f += 8 * pl) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = f[u * pl];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += (double)v[u];
        }
        for (; k < nch; ++k, f += pl) s += (double)*f;
        const float* t = Tt + (int64_t)c * n_pad + i;
        int I = 0;
        for (; I + 8 <= tile; I += 8, t += 8 * pl) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = t[u * pl];
#pragma unroll
            for (int u = 0; u < 8; ++u) s += (double)v[u];
        }
        for (; I < tile; ++I, t += pl) s += (double)*t;
        out[(int64_t)c * n_pad + i] = (float)s;
    }
}

// ---------------------------------------------------------------------------------------
// BF16 MFMA product (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  Inside a 32-column
// group, lane l takes columns j = 8 (l / 16) + s for s = 0..7: its 8 K values for row
// lane % 16 form the A operand, and the B operand is the matching 8 consecutive entries of
// one V column, a single 16-byte LDS read.  V arrives split as V = V_hi + V_lo (both BF16).
//   SPLITK = false: K_hi (V_hi + V_lo)                       (two products)
//   SPLITK = true : K_hi V_hi + K_hi V_lo + K_lo V_hi         (three products)
// with K_hi = bf16(K), K_lo = bf16(K - K_hi).  Distances and exp2 stay in FP32.
// ---------------------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

__device__ inline uint32_t pack_bf16(float a, float b) {
    const floatx2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ inline float bf16_lo_as_f32(uint32_t p) { return __uint_as_float(p << 16); }
__device__ inline float bf16_hi_as_f32(uint32_t p) { return __uint_as_float(p & 0xffff0000u); }

template <int D, int NB, int R, bool SPLITK>
__global__ __launch_bounds__(kWG) void kmv_mfma_bf16_kernel(
    const float* __restrict__ Z, const uint16_t* __restrict__ VH, const uint16_t* __restrict__ VL,
    int64_t ldv, float* __restrict__ part, int64_t n_pad, int chunk, int split,
    const KParams* __restrict__ kp, const int* __restrict__ n_active) {
    if (n_active != nullptr && *n_active == 0) return;
    constexpr int DP = (D + 3) & ~3;
    constexpr int MP = NB * 16;
    using S = StageB16<DP, MP>;
    __shared__ float4 zs[2][S::NZ4];
    __shared__ uint16_t hs[2][S::VSIZE];
    __shared__ uint16_t ls[2][S::VSIZE];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int cidx = blockIdx.x % split;
    const int64_t rt = blockIdx.x / split;
    const int64_t row0 = rt * (64 * R) + wave * (16 * R);
    const int64_t jb = (int64_t)cidx * chunk;
    const int64_t je = min(jb + (int64_t)chunk, n_pad);
    const float negc0 = -kp->c0;

    float zi[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r) load_row<D>(Z + (row0 + r * 16 + col) * DP, zi[r]);
    floatx4 acc[R][NB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[r][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    S st;
    if (jb < je) {
        st.load(Z, VH, VL, ldv, jb);
        st.store(zs[0], hs[0], ls[0], true);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kJS) {
        const bool more = j0 + kJS < je;
        if (more) st.load(Z, VH, VL, ldv, j0 + kJS);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
#pragma unroll 1
        for (int g = 0; g < kJS / 32; ++g) {
            bf16x8 bh[NB], bl[NB];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                const int o = (cb * 16 + col) * S::VST + g * 32 + 8 * q;
                bh[cb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(hs[buf] + o));
                bl[cb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(ls[buf] + o));
            }
            float kv[R][8];
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                float zj[D];
                load_row<D>(zsb + (g * 32 + 8 * q + s) * DP, zj);
#pragma unroll
                for (int r = 0; r < R; ++r) kv[r][s] = kf_entry<D>(zi[r], zj, negc0);
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                uint32_t hi[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) hi[u] = pack_bf16(kv[r][2 * u], kv[r][2 * u + 1]);
                const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(hi));
#pragma unroll
                for (int cb = 0; cb < NB; ++cb) {
                    acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cb], acc[r][cb], 0, 0, 0);
                    acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cb], acc[r][cb], 0, 0, 0);
                }
                if (SPLITK) {
                    uint32_t lo[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        lo[u] = pack_bf16(kv[r][2 * u] - bf16_lo_as_f32(hi[u]),
                                          kv[r][2 * u + 1] - bf16_hi_as_f32(hi[u]));
                    const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(lo));
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb)
                        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cb], acc[r][cb], 0, 0, 0);
                }
            }
        }
        if (more) st.store(zs[buf ^ 1], hs[buf ^ 1], ls[buf ^ 1], true);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            const int64_t i = row0 + r * 16 + 4 * q;
            const int c = cb * 16 + col;
            float4 o;
            o.x = acc[r][cb][0];
            o.y = acc[r][cb][1];
            o.z = acc[r][cb][2];
            o.w = acc[r][cb][3];
            *reinterpret_cast<float4*>(part + ((int64_t)cidx * MP + c) * n_pad + i) = o;
        }
}

// ---------------------------------------------------------------------------------------
// Symmetric BF16 product: the work items, partials and reduce of the symmetric FP32 product,
// with the BF16 contraction above, for two MFMA blocks of right-hand sides (17 to 32).
// Forward: as kmv_mfma_bf16_kernel, R = 4 blocks of 16 rows per wave, four waves per 256-row
// tile.  Transposed: each wave contracts its own 64 rows, 32 at a time.  It stores the packed
// K values of two row blocks (hi, and lo with SPLITK) transposed into a 32 x 32 BF16 tile of
// its own in LDS: two lanes of neighbouring rows i, i + 1 swap their packed pairs (one DPP
// move) and each stores one 32-bit word (K[i][j], K[i+1][j]); the 16-byte chunks of a tile
// row are XOR-swizzled by tw_swz(j), which puts a wave's stores two lanes per bank and its
// 16-byte reads on distinct banks.  A operand = 8 consecutive i of one tile row, B operand =
// the wave's own V rows, held in registers for the whole item.  The four waves' partials of
// a 64-column stage are summed in LDS in a fixed order and written to Tt, as in the FP32
// kernel.  The product terms are those of the forward direction: K_hi (V_hi + V_lo), plus
// K_lo V_hi with SPLITK.
// ---------------------------------------------------------------------------------------
__device__ inline int tw_swz(int j) { return ((j & 3) ^ ((j >> 2) & 3)) & 3; }

template <int D, bool SPLITK>
__global__ __launch_bounds__(kWG, 2) void kmv_sym_bf16_kernel(
    const float* __restrict__ Z, const uint16_t* __restrict__ VH, const uint16_t* __restrict__ VL,
    float* __restrict__ F, float* __restrict__ Tt, int64_t n_pad, int NT, int cs,
    const KParams* __restrict__ kp, const int* __restrict__ n_active) {
    if (n_active != nullptr && *n_active == 0) return;
    constexpr int R = 4;
    constexpr int NB = 2;
    constexpr int DP = (D + 3) & ~3;
    constexpr int MP = NB * 16;
    constexpr int RED = MP + 1;  // row stride of a wave's transposed partial
    using S = StageB16<DP, MP>;
    __shared__ float4 zs[2][S::NZ4];
    __shared__ uint16_t hs[2][S::VSIZE];
    __shared__ uint16_t ls[2][S::VSIZE];
    __shared__ __align__(16) uint16_t tw[4][SPLITK ? 2 : 1][32 * 32];
    __shared__ float red[4][kJS * RED];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    int k, I;
    sym_item(blockIdx.x, NT, cs, &k, &I);
    const int64_t tile0 = (int64_t)I * kSymTile;
    const int64_t row0 = tile0 + wave * (16 * R);
    const int64_t diag_end = tile0 + kSymTile;
    const int64_t jb = max((int64_t)k * cs, tile0);
    const int64_t je = min((int64_t)(k + 1) * cs, n_pad);
    const float negc0 = -kp->c0;
    // the word a lane stores: even lane (row i) (K[i][j], K[i+1][j]) for j = 8 q + 2 u, odd
    // lane (row i + 1) the same for j + 1; v_perm selectors over (partner's pair, own pair)
    const int odd = col & 1;
    const uint32_t psel = odd ? 0x03020706u : 0x05040100u;

    float zi[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r) load_row<D>(Z + (row0 + r * 16 + col) * DP, zi[r]);
    // B operand of the transposed products: lane (q, col) holds
    // V[row0 + 32 p + 8 q + s][16 cb + col], s = 0..7, for the wave's two 32-row halves p
    uintx4 vh[2][NB], vl[2][NB];
#pragma unroll
    for (int p2 = 0; p2 < 2; ++p2)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            const int64_t o = (int64_t)(16 * cb + col) * n_pad + row0 + 32 * p2 + 8 * q;
            vh[p2][cb] = *reinterpret_cast<const uintx4*>(VH + o);
            vl[p2][cb] = *reinterpret_cast<const uintx4*>(VL + o);
        }
    // complete these loads here (see kmv_sym_f32_kernel)
#pragma unroll
    for (int p2 = 0; p2 < 2; ++p2)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) asm volatile("" : "+v"(vh[p2][cb]), "+v"(vl[p2][cb]));
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int k2 = 0; k2 < D; ++k2) asm volatile("" : "+v"(zi[r][k2]));

    floatx4 acc[R][NB];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[r][cb] = floatx4{0.f, 0.f, 0.f, 0.f};

    uint32_t* twh = reinterpret_cast<uint32_t*>(tw[wave][0]);
    uint32_t* twl = reinterpret_cast<uint32_t*>(tw[wave][SPLITK ? 1 : 0]);
    float* redw = red[wave];
    S st;
    st.load(Z, VH, VL, n_pad, jb);
    st.store(zs[0], hs[0], ls[0], true);
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kJS) {
        const bool more = j0 + kJS < je;
        const bool sym = j0 >= diag_end;  // uniform over the workgroup
        if (more) st.load(Z, VH, VL, n_pad, j0 + kJS);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
#pragma unroll 1
        for (int g = 0; g < kJS / 32; ++g) {
            bf16x8 bh[NB], bl[NB];
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) {
                const int o = (cb * 16 + col) * S::VST + g * 32 + 8 * q;
                bh[cb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(hs[buf] + o));
                bl[cb] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(ls[buf] + o));
            }
            float kv[R][8];
#pragma unroll
            for (int s_ = 0; s_ < 8; ++s_) {
                float zj[D];
                load_row<D>(zsb + (g * 32 + 8 * q + s_) * DP, zj);
#pragma unroll
                for (int r = 0; r < R; ++r) kv[r][s_] = kf_entry<D>(zi[r], zj, negc0);
            }
            uint32_t hi[R][4], lo[R][4];
#pragma unroll
            for (int r = 0; r < R; ++r) {
#pragma unroll
                for (int u = 0; u < 4; ++u) hi[r][u] = pack_bf16(kv[r][2 * u], kv[r][2 * u + 1]);
                const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(hi[r]));
#pragma unroll
                for (int cb = 0; cb < NB; ++cb) {
                    acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[cb], acc[r][cb], 0, 0, 0);
                    acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[cb], acc[r][cb], 0, 0, 0);
                }
                if (SPLITK) {
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        lo[r][u] = pack_bf16(kv[r][2 * u] - bf16_lo_as_f32(hi[r][u]),
                                             kv[r][2 * u + 1] - bf16_hi_as_f32(hi[r][u]));
                    const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(lo[r]));
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb)
                        acc[r][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[cb], acc[r][cb], 0, 0, 0);
                }
            }
            if (sym) {
                // transposed: T[j][c] = sum over the wave's 64 rows i of K(i, j) V(i, c) for the
                // 32 columns j of this group; lane (q, col) accumulates T[16 jb + 4 q + t][16 cb + col]
                floatx4 tr[2][NB];
#pragma unroll
                for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb) tr[a2][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int p2 = 0; p2 < 2; ++p2) {
                    // tile[j][i] = K(row0 + 32 p2 + i, j0 + 32 g + j): row blocks r = 2 p2, 2 p2 + 1
#pragma unroll
                    for (int rr = 0; rr < 2; ++rr) {
                        const int r = 2 * p2 + rr;
                        const int ie = 16 * rr + (col & ~1);  // even row of the lane pair
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const int j = 8 * q + 2 * u + odd;
                            const int w = (j * 32 + (((ie >> 3) ^ tw_swz(j)) << 3) + (ie & 7)) >> 1;
                            const uint32_t xh = (uint32_t)__builtin_amdgcn_mov_dpp((int)hi[r][u], 0xB1, 0xF, 0xF, false);
                            twh[w] = __builtin_amdgcn_perm(xh, hi[r][u], psel);
                            if (SPLITK) {
                                const uint32_t xl = (uint32_t)__builtin_amdgcn_mov_dpp((int)lo[r][u], 0xB1, 0xF, 0xF, false);
                                twl[w] = __builtin_amdgcn_perm(xl, lo[r][u], psel);
                            }
                        }
                    }
                    // the other lanes' stores before the reads, the reads before the next stores
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
                    for (int a2 = 0; a2 < 2; ++a2) {
                        const int jr = 16 * a2 + col;
                        const int e = (jr * 32 + ((q ^ tw_swz(jr)) << 3)) >> 1;  // 8 i = 8 q .. 8 q + 7
                        const bf16x8 ah = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uintx4*>(twh + e));
#pragma unroll
                        for (int cb = 0; cb < NB; ++cb) {
                            tr[a2][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                ah, __builtin_bit_cast(bf16x8, vh[p2][cb]), tr[a2][cb], 0, 0, 0);
                            tr[a2][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                ah, __builtin_bit_cast(bf16x8, vl[p2][cb]), tr[a2][cb], 0, 0, 0);
                        }
                        if (SPLITK) {
                            const bf16x8 al = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uintx4*>(twl + e));
#pragma unroll
                            for (int cb = 0; cb < NB; ++cb)
                                tr[a2][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                    al, __builtin_bit_cast(bf16x8, vh[p2][cb]), tr[a2][cb], 0, 0, 0);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
                // the wave's partial: columns j = 32 g + 16 a2 + 4 q + t of the stage
#pragma unroll
                for (int a2 = 0; a2 < 2; ++a2)
#pragma unroll
                    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
                        for (int t = 0; t < 4; ++t)
                            redw[(g * 32 + 16 * a2 + 4 * q + t) * RED + cb * 16 + col] = tr[a2][cb][t];
            }
        }
        if (more) st.store(zs[buf ^ 1], hs[buf ^ 1], ls[buf ^ 1], true);
        __syncthreads();
        if (sym) {
            // the four waves' partials in a fixed order -> Tt[I][c][j0 + j]
            for (int e = threadIdx.x; e < MP * kJS; e += kWG) {
                const int c = e / kJS, j = e % kJS;
                const float v = ((red[0][j * RED + c] + red[1][j * RED + c]) + red[2][j * RED + c]) + red[3][j * RED + c];
                Tt[((int64_t)I * MP + c) * n_pad + j0 + j] = v;
            }
            __syncthreads();
        }
        buf ^= 1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
            const int64_t i = row0 + r * 16 + 4 * q;
            const int c = cb * 16 + col;
            float4 o;
            o.x = acc[r][cb][0];
            o.y = acc[r][cb][1];
            o.z = acc[r][cb][2];
            o.w = acc[r][cb][3];
            *reinterpret_cast<float4*>(F + ((int64_t)k * MP + c) * n_pad + i) = o;
        }
}

// V (FP32, n_pad x mp, ld n_pad) -> V_hi = bf16(V), V_lo = bf16(V - V_hi).
__global__ void split_bf16_kernel(const float* __restrict__ V, int64_t total,
                                  uint16_t* __restrict__ VH, uint16_t* __restrict__ VL) {
    for (int64_t e = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 2; e < total;
         e += (int64_t)gridDim.x * blockDim.x * 2) {
        const float a = V[e], b = V[e + 1];
        const uint32_t hi = pack_bf16(a, b);
        const uint32_t lo = pack_bf16(a - bf16_lo_as_f32(hi), b - bf16_hi_as_f32(hi));
        *reinterpret_cast<uint32_t*>(VH + e) = hi;
        *reinterpret_cast<uint32_t*>(VL + e) = lo;
    }
}

// ---------------------------------------------------------------------------------------
// VALU product for MC (= 4, 8, 12) columns: one row per lane and per R; every column j of
// the stage is read by all lanes at once (LDS broadcast).
// ---------------------------------------------------------------------------------------
// MC staged columns (m rounded up to 4), of which the first MU are contracted: the padding
// columns cost LDS space but no FMAs.
template <int D, int MC, int MU, int R>
__global__ __launch_bounds__(kWG) void kmv_valu_kernel(
    const float* __restrict__ Z, const float* __restrict__ V, int64_t ldv,
    float* __restrict__ part, int64_t n_pad, int chunk, int split,
    const KParams* __restrict__ kp, const int* __restrict__ n_active) {
    if (n_active != nullptr && *n_active == 0) return;
    constexpr int DP = (D + 3) & ~3;
    static_assert(MU >= 1 && MU <= MC && MC - MU < 4, "MU columns of MC staged");
    using S = Stage<DP, MC, true>;
    __shared__ float4 zs[2][S::NZ4];
    __shared__ float vs[2][S::VSIZE];

    const int cidx = blockIdx.x % split;
    const int64_t rt = blockIdx.x / split;
    const int64_t row0 = rt * (kWG * R);
    const int64_t jb = (int64_t)cidx * chunk;
    const int64_t je = min(jb + (int64_t)chunk, n_pad);
    const float negc0 = -kp->c0;

    float zi[R][D];
#pragma unroll
    for (int r = 0; r < R; ++r) load_row<D>(Z + (row0 + r * kWG + threadIdx.x) * DP, zi[r]);
    float acc[R][MU];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < MU; ++c) acc[r][c] = 0.f;

    S st;
    if (jb < je) {
        st.load(Z, V, ldv, jb);
        st.store(zs[0], vs[0]);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kJS) {
        const bool more = j0 + kJS < je;
        if (more) st.load(Z, V, ldv, j0 + kJS);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
        const float* vsb = vs[buf];
#pragma unroll 4
        for (int j = 0; j < kJS; ++j) {
            float zj[D];
            load_row<D>(zsb + j * DP, zj);
            float vj[MC];
#pragma unroll
            for (int c = 0; c < MC; c += 4) {
                const float4 v4 = *reinterpret_cast<const float4*>(vsb + j * MC + c);
                vj[c] = v4.x;
                vj[c + 1] = v4.y;
                vj[c + 2] = v4.z;
                vj[c + 3] = v4.w;
            }
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float kv = kf_entry<D>(zi[r], zj, negc0);
#pragma unroll
                for (int c = 0; c < MU; ++c) acc[r][c] = __builtin_fmaf(kv, vj[c], acc[r][c]);
            }
        }
        if (more) st.store(zs[buf ^ 1], vs[buf ^ 1]);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int c = 0; c < MU; ++c)
            part[((int64_t)cidx * MC + c) * n_pad + row0 + r * kWG + threadIdx.x] = acc[r][c];
}

// ---------------------------------------------------------------------------------------
// Derivative products.  MFMA form for 16 columns per pass (one accumulator set per
// derivative), VALU form for 4 columns per pass.  part layout: [split][D+1][MP][n_pad];
// block 0 is K_f V, block k is (K_f o dz_k^2) V, still to be scaled by 2 ln 2.
// ---------------------------------------------------------------------------------------
template <int D>
__global__ __launch_bounds__(kWG) void dkmv_mfma_kernel(
    const float* __restrict__ Z, const float* __restrict__ V, int64_t ldv,
    float* __restrict__ part, int64_t n_pad, int chunk, int split,
    const KParams* __restrict__ kp) {
    constexpr int DP = (D + 3) & ~3;
    constexpr int MP = 16;
    using S = Stage<DP, MP, false>;
    __shared__ float4 zs[2][S::NZ4];
    __shared__ float vs[2][S::VSIZE];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, col = lane & 15;
    const int cidx = blockIdx.x % split;
    const int64_t rt = blockIdx.x / split;
    const int64_t row0 = rt * 64 + wave * 16;
    const int64_t jb = (int64_t)cidx * chunk;
    const int64_t je = min(jb + (int64_t)chunk, n_pad);
    const float negc0 = -kp->c0;

    float zi[D];
    load_row<D>(Z + (row0 + col) * DP, zi);
    floatx4 acc[D + 1];
#pragma unroll
    for (int p = 0; p <= D; ++p) acc[p] = floatx4{0.f, 0.f, 0.f, 0.f};

    S st;
    if (jb < je) {
        st.load(Z, V, ldv, jb);
        st.store(zs[0], vs[0]);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kJS) {
        const bool more = j0 + kJS < je;
        if (more) st.load(Z, V, ldv, j0 + kJS);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
        const float* vsb = vs[buf];
#pragma unroll 1
        for (int g = 0; g < kJS / 16; ++g) {
            const float4 vv = *reinterpret_cast<const float4*>(vsb + col * S::VST + g * 16 + 4 * q);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                float zj[D];
                load_row<D>(zsb + (g * 16 + 4 * q + s) * DP, zj);
                float sq[D];
                float a = negc0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const float t = zi[k] - zj[k];
                    sq[k] = t * t;
                    a += sq[k];
                }
                const float kv = __builtin_amdgcn_exp2f(-a);
                const float b = s == 0 ? vv.x : s == 1 ? vv.y : s == 2 ? vv.z : vv.w;
                acc[0] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv, b, acc[0], 0, 0, 0);
#pragma unroll
                for (int k = 0; k < D; ++k)
                    acc[k + 1] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv * sq[k], b, acc[k + 1], 0, 0, 0);
            }
        }
        if (more) st.store(zs[buf ^ 1], vs[buf ^ 1]);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int p = 0; p <= D; ++p) {
        float4 o;
        o.x = acc[p][0];
        o.y = acc[p][1];
        o.z = acc[p][2];
        o.w = acc[p][3];
        *reinterpret_cast<float4*>(part + (((int64_t)cidx * (D + 1) + p) * MP + col) * n_pad + row0 + 4 * q) = o;
    }
}

template <int D>
__global__ __launch_bounds__(kWG) void dkmv_valu_kernel(
    const float* __restrict__ Z, const float* __restrict__ V, int64_t ldv,
    float* __restrict__ part, int64_t n_pad, int chunk, int split,
    const KParams* __restrict__ kp) {
    constexpr int DP = (D + 3) & ~3;
    constexpr int MC = 4;
    using S = Stage<DP, MC, true>;
    __shared__ float4 zs[2][S::NZ4];
    __shared__ float vs[2][S::VSIZE];

    const int cidx = blockIdx.x % split;
    const int64_t rt = blockIdx.x / split;
    const int64_t i = rt * kWG + threadIdx.x;
    const int64_t jb = (int64_t)cidx * chunk;
    const int64_t je = min(jb + (int64_t)chunk, n_pad);
    const float negc0 = -kp->c0;

    float zi[D];
    load_row<D>(Z + i * DP, zi);
    float acc[D + 1][MC];
#pragma unroll
    for (int p = 0; p <= D; ++p)
#pragma unroll
        for (int c = 0; c < MC; ++c) acc[p][c] = 0.f;

    S st;
    if (jb < je) {
        st.load(Z, V, ldv, jb);
        st.store(zs[0], vs[0]);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = jb; j0 < je; j0 += kJS) {
        const bool more = j0 + kJS < je;
        if (more) st.load(Z, V, ldv, j0 + kJS);
        const float* zsb = reinterpret_cast<const float*>(zs[buf]);
        const float* vsb = vs[buf];
#pragma unroll 2
        for (int j = 0; j < kJS; ++j) {
            float zj[D];
            load_row<D>(zsb + j * DP, zj);
            const float4 v4 = *reinterpret_cast<const float4*>(vsb + j * MC);
            const float vj[4] = {v4.x, v4.y, v4.z, v4.w};
            float sq[D];
            float a = negc0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const float t = zi[k] - zj[k];
                sq[k] = t * t;
                a += sq[k];
            }
            const float kv = __builtin_amdgcn_exp2f(-a);
#pragma unroll
            for (int c = 0; c < MC; ++c) acc[0][c] = __builtin_fmaf(kv, vj[c], acc[0][c]);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const float w = kv * sq[k];
#pragma unroll
                for (int c = 0; c < MC; ++c) acc[k + 1][c] = __builtin_fmaf(w, vj[c], acc[k + 1][c]);
            }
        }
        if (more) st.store(zs[buf ^ 1], vs[buf ^ 1]);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int p = 0; p <= D; ++p)
#pragma unroll
        for (int c = 0; c < MC; ++c)
            part[(((int64_t)cidx * (D + 1) + p) * MC + c) * n_pad + i] = acc[p][c];
}

// ---------------------------------------------------------------------------------------
// Fixed-order combination of the chunk partials.
// ---------------------------------------------------------------------------------------
__global__ void kmv_reduce_kernel(const float* __restrict__ part, int split, int mp,
                                  int64_t n_pad, const float* __restrict__ Vp,
                                  const KParams* __restrict__ kp, int64_t n, int m,
                                  float* __restrict__ out, int64_t ldo) {
    const double lam = kp->lam64;
    const int64_t total = n * m;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / n);
        const int64_t i = e % n;
        double s = 0.0;
        for (int k = 0; k < split; ++k) s += (double)part[((int64_t)k * mp + c) * n_pad + i];
        s += lam * (double)Vp[c * n_pad + i];
        out[c * ldo + i] = (float)s;
    }
}

__global__ void dkmv_reduce_kernel(const float* __restrict__ part, int split, int d, int mp,
                                   int64_t n_pad, const float* __restrict__ Vp,
                                   const KParams* __restrict__ kp, int64_t n, int mcols,
                                   float* __restrict__ out, int64_t ldo, int64_t bstride) {
    const double lam = kp->lam64;
    const double two_ln2 = 2.0 * M_LN2;
    const int64_t total = n * mcols * (int64_t)(d + 2);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e % n;
        const int c = (int)((e / n) % mcols);
        const int p = (int)(e / (n * mcols));
        double s = 0.0;
        if (p <= d) {
            for (int k = 0; k < split; ++k)
                s += (double)part[(((int64_t)k * (d + 1) + p) * mp + c) * n_pad + i];
            if (p > 0) s *= two_ln2;
        } else {
            s = lam * (double)Vp[c * n_pad + i];
        }
        out[p * bstride + c * ldo + i] = (float)s;
    }
}

// ---------------------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------------------
static int grid_for(int64_t total, int per = kWG) {
    int64_t g = (total + per - 1) / per;
    return (int)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

static void pick_split(KmvShape& sh, int target_wg) {
    const int64_t row_tiles = sh.n_pad / sh.rows_per_wg;
    const int64_t max_split = sh.n_pad / kJS;
    int64_t split = std::max<int64_t>(1, target_wg / std::max<int64_t>(1, row_tiles));
    split = std::min<int64_t>(split, max_split);
    if (split >= 8) split = split / 8 * 8;  // chunk index = blockIdx % split: XCD-aligned
    sh.chunk = (int)round_up((sh.n_pad + split - 1) / split, kJS);
    sh.split = (int)((sh.n_pad + sh.chunk - 1) / sh.chunk);
}

int kmv_default_code(int64_t n, int d, int m, gp_precision prec) {
    // the symmetric product by default where it was measured faster than split-K.  d >= 12:
    // wherever it applies (at d = 16 each entry costs twice the VALU work of d = 8, and the
    // shape was 4-46% faster from n = 16384 to 131072 in every mode).  d <= 8, FP32: one MFMA
    // block of columns, or n of 32768 and more (two blocks at n = 16384 are 9% slower: the
    // transposed partials cost more than the halved entry work saves); BF16: two MFMA blocks
    // and n of 32768 and more.  9 <= d <= 11 keeps the d <= 8 rule (not measured).
    const KmvShape sy = kmv_shape_sym(n, d, m, prec);
    const bool wide = m >= 16;
    // FP32 under 16 right-hand sides: the symmetric product with one zero-padded MFMA block
    // costs about the same at every m, the VALU contraction 2d + 3 + m instructions per entry;
    // the former is taken where m + d >= 12 from n = 16384 on (d = 8: 1.04-1.86x for m = 4 to
    // 15, 0.88-0.94x at m = 1; d = 16, m = 5: 1.41x; d = 2, m = 5: 0.91x)
    if (sy.sym && !wide && prec == GP_FP32 && m + d >= 12 && sy.n_pad >= 16384) return 0;
    if (sy.sym && wide && d >= 12) return 0;
    if (sy.sym && wide && prec == GP_FP32 && (sy.mp <= 20 || sy.n_pad >= 32768)) return 0;
    if (sy.sym && wide && prec != GP_FP32 && sy.mp == 32 && sy.n_pad >= 32768) return 0;
    const KmvShape sk = kmv_shape_target(n, d, m, prec, 2048);
    if (sk.mfma) return 2048;
    // the VALU contraction (under 16 columns): finer column chunks, up to 32 per row tile
    // (at n = 65536, m = 4 the autotuner's split of 32 was 17% faster than 8)
    const int64_t tiles = sk.n_pad / sk.rows_per_wg;
    return (int)std::min<int64_t>(8192, 32 * tiles);
}

KmvShape kmv_shape(int64_t n, int d, int m, gp_precision prec) {
    const int code = kmv_default_code(n, d, m, prec);
    return code == 0 ? kmv_shape_sym(n, d, m, prec) : kmv_shape_target(n, d, m, prec, code);
}

static int64_t sym_items(int nt, int nch, int cs) {
    int64_t t = 0;
    for (int k = 0; k < nch; ++k) t += std::min<int64_t>(nt, (int64_t)(k + 1) * (cs / kSymTile));
    return t;
}

KmvShape kmv_shape_sym(int64_t n, int d, int m, gp_precision prec) {
    const KmvShape base = kmv_shape_target(n, d, m, prec, 2048);
    // MFMA products with at least 8 row tiles: FP32 with one or two MFMA blocks and at most
    // one VALU column (under 16 right-hand sides: one block, zero-padded), BF16 with two
    // blocks; four row blocks of 16 per wave at every d (the d = 16 kernels still fit two
    // waves per SIMD)
    KmvShape sh = prec == GP_FP32 && m < 16 ? kmv_shape_target(n, d, 16, prec, 2048) : base;
    const int nb = sh.mp / 16;
    const bool f32 = prec == GP_FP32 && sh.tail <= 1 && (nb == 1 || nb == 2);
    const bool b16 = prec != GP_FP32 && sh.tail == 0 && nb == 2;
    if (!sh.mfma || d > kMaxD || sh.n_pad < 8 * kSymTile || !(f32 || b16)) return base;
    sh.sym = true;
    sh.nt = (int)(sh.n_pad / kSymTile);
    sh.rows_per_wg = kSymTile;
    // the widest column chunk that still gives 2048 work items
    sh.cs = kSymTile;
    for (int cs = 2 * kSymTile; cs <= 8 * kSymTile && cs <= sh.n_pad; cs *= 2) {
        const int nch = (int)((sh.n_pad + cs - 1) / cs);
        if (sym_items(sh.nt, nch, cs) >= 2048) sh.cs = cs;
    }
    sh.nch = (int)((sh.n_pad + sh.cs - 1) / sh.cs);
    sh.split = 1;
    sh.chunk = (int)sh.n_pad;
    if (kmv_part_floats(sh) * sizeof(float) > kSymPartialBytesMax) return base;
    return sh;
}

size_t kmv_part_floats(const KmvShape& sh) {
    const size_t plane = (size_t)sh.mp * (size_t)sh.n_pad;
    return sh.sym ? (size_t)(1 + sh.nch + sh.nt) * plane : (size_t)sh.split * plane;
}

KmvShape kmv_shape_target(int64_t n, int d, int m, gp_precision prec, int target_wg) {
    KmvShape sh;
    sh.n_pad = round_up(std::max<int64_t>(n, 1), kRowPad);
    sh.mfma = m >= 16;
    sh.tail = 0;
    if (sh.mfma) {
        sh.mp = (int)round_up(m, 16);
        // FP32: up to three columns past a multiple of 16 (four when m < 32) go through
        // the VALU instead of another MFMA block (m < 64)
        const int t = m % 16;
        if (prec == GP_FP32 && m < 64 && t != 0 && (t <= 3 || (t == 4 && m < 32))) {
            sh.tail = t;
            sh.mp = m / 16 * 16 + 4;
        }
        const int R = d <= 8 ? 4 : 2;
        sh.rows_per_wg = 64 * R;
    } else {
        sh.mp = (int)round_up(m, 4);
        // contract only the m real columns when that saves two or three FMAs per entry
        // (m mod 4 = 1 or 2: 3-14% faster); one padding column is cheaper to keep
        sh.mu = (m % 4 == 1 || m % 4 == 2) ? m : sh.mp;
        sh.rows_per_wg = kWG;
    }
    pick_split(sh, target_wg);
    return sh;
}

KmvShape dkmv_shape(int64_t n, int d, int m) {
    KmvShape sh;
    sh.n_pad = round_up(std::max<int64_t>(n, 1), kRowPad);
    sh.mfma = m >= 16;
    sh.mp = sh.mfma ? 16 : 4;  // columns per pass
    sh.rows_per_wg = sh.mfma ? 64 : kWG;
    (void)d;
    pick_split(sh, 2048);
    return sh;
}

size_t dkmv_part_floats(const KmvShape& sh, int d) {
    return (size_t)sh.split * (d + 1) * sh.mp * sh.n_pad;
}

hipError_t launch_prep(const float* X, int64_t n, int d, int64_t ldx, const double* psi,
                       float* Z, int64_t n_pad, KParams* kp, hipStream_t s) {
    prep_kernel<<<grid_for(n_pad * dpad(d)), kWG, 0, s>>>(X, n, d, ldx, psi, Z, n_pad, kp);
    return hipGetLastError();
}

hipError_t launch_pack(const float* V, int64_t n, int m, int64_t ldv, float* Vp, int64_t n_pad,
                       int mp, hipStream_t s) {
    pack_kernel<<<grid_for(n_pad * mp), kWG, 0, s>>>(V, n, m, ldv, Vp, n_pad, mp);
    return hipGetLastError();
}

template <int D, bool SPLITK>
static hipError_t kmv_bf16_d(const KmvShape& sh, const float* Z, const uint16_t* VH,
                             const uint16_t* VL, const KParams* kp, float* part,
                             const int* n_active, hipStream_t s) {
    const int64_t tiles = sh.n_pad / sh.rows_per_wg;
    const dim3 grid((unsigned)(tiles * sh.split));
    constexpr int R = D <= 8 ? 4 : 2;
    switch (sh.mp) {
        case 16: kmv_mfma_bf16_kernel<D, 1, R, SPLITK><<<grid, kWG, 0, s>>>(Z, VH, VL, sh.n_pad, part, sh.n_pad, sh.chunk, sh.split, kp, n_active); break;
        case 32: kmv_mfma_bf16_kernel<D, 2, R, SPLITK><<<grid, kWG, 0, s>>>(Z, VH, VL, sh.n_pad, part, sh.n_pad, sh.chunk, sh.split, kp, n_active); break;
        case 48: kmv_mfma_bf16_kernel<D, 3, R, SPLITK><<<grid, kWG, 0, s>>>(Z, VH, VL, sh.n_pad, part, sh.n_pad, sh.chunk, sh.split, kp, n_active); break;
        case 64: kmv_mfma_bf16_kernel<D, 4, R, SPLITK><<<grid, kWG, 0, s>>>(Z, VH, VL, sh.n_pad, part, sh.n_pad, sh.chunk, sh.split, kp, n_active); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define GPK_F32_LAUNCH(NB, TC)                                                              \
    kmv_mfma_f32_kernel<D, NB, TC, R><<<grid, kWG, 0, s>>>(Z, Vp, sh.n_pad, part, sh.n_pad, \
                                                             sh.chunk, sh.split, kp, n_active)

// (NB, TC) pairs that kmv_shape_target produces: TC <= 3, or TC = 4 with one MFMA block;
// other tails would lower the occupancy below that of the padded kernel.
template <int D, int R>
static hipError_t kmv_f32_nb(int nb, int tc, dim3 grid, const float* Z, const float* Vp, float* part,
                             const KmvShape& sh, const KParams* kp, const int* n_active, hipStream_t s) {
    switch (nb * 8 + tc) {
        case 8: GPK_F32_LAUNCH(1, 0); break;
        case 9: GPK_F32_LAUNCH(1, 1); break;
        case 10: GPK_F32_LAUNCH(1, 2); break;
        case 11: GPK_F32_LAUNCH(1, 3); break;
        case 12: GPK_F32_LAUNCH(1, 4); break;
        case 16: GPK_F32_LAUNCH(2, 0); break;
        case 17: GPK_F32_LAUNCH(2, 1); break;
        case 18: GPK_F32_LAUNCH(2, 2); break;
        case 19: GPK_F32_LAUNCH(2, 3); break;
        case 24: GPK_F32_LAUNCH(3, 0); break;
        case 25: GPK_F32_LAUNCH(3, 1); break;
        case 26: GPK_F32_LAUNCH(3, 2); break;
        case 27: GPK_F32_LAUNCH(3, 3); break;
        case 32: GPK_F32_LAUNCH(4, 0); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
#undef GPK_F32_LAUNCH

template <int D>
static hipError_t kmv_sym_d(const KmvShape& sh, const float* Z, const float* Vp, const uint16_t* VH,
                            const uint16_t* VL, const KParams* kp, float* part, const int* n_active,
                            gp_precision prec, hipStream_t s, hipEvent_t after_main) {
    if constexpr (D > 16) {
        return hipErrorInvalidValue;
    } else {
        const size_t plane = (size_t)sh.mp * (size_t)sh.n_pad;
        float* F = part + plane;
        float* Tt = F + (size_t)sh.nch * plane;
        const dim3 grid((unsigned)sym_items(sh.nt, sh.nch, sh.cs));
        const int nb = sh.mp / 16;
        if (prec != GP_FP32) {
            if (sh.tail != 0 || nb != 2 || VH == nullptr || VL == nullptr) return hipErrorInvalidValue;
            if (prec == GP_BF16_SPLIT_KV)
                kmv_sym_bf16_kernel<D, true><<<grid, kWG, 0, s>>>(Z, VH, VL, F, Tt, sh.n_pad, sh.nt, sh.cs, kp, n_active);
            else
                kmv_sym_bf16_kernel<D, false><<<grid, kWG, 0, s>>>(Z, VH, VL, F, Tt, sh.n_pad, sh.nt, sh.cs, kp, n_active);
        } else if (nb == 1 && sh.tail == 0)
            kmv_sym_f32_kernel<D, 1, 0><<<grid, kWG, 0, s>>>(Z, Vp, F, Tt, sh.n_pad, sh.nt, sh.cs, kp, n_active);
        else if (nb == 1 && sh.tail == 1)
            kmv_sym_f32_kernel<D, 1, 1><<<grid, kWG, 0, s>>>(Z, Vp, F, Tt, sh.n_pad, sh.nt, sh.cs, kp, n_active);
        else if (nb == 2 && sh.tail == 0)
            kmv_sym_f32_kernel<D, 2, 0><<<grid, kWG, 0, s>>>(Z, Vp, F, Tt, sh.n_pad, sh.nt, sh.cs, kp, n_active);
        else if (nb == 2 && sh.tail == 1)
            kmv_sym_f32_kernel<D, 2, 1><<<grid, kWG, 0, s>>>(Z, Vp, F, Tt, sh.n_pad, sh.nt, sh.cs, kp, n_active);
        else
            return hipErrorInvalidValue;
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (after_main != nullptr) {
            e = hipEventRecord(after_main, s);
            if (e != hipSuccess) return e;
        }
        const int mu = nb * 16 + sh.tail;  // BF16: tail 0
        kmv_sym_reduce_kernel<<<grid_for((int64_t)mu * sh.n_pad), kWG, 0, s>>>(F, Tt, part, sh.n_pad, sh.mp, mu,
                                                                                 sh.cs, sh.nch, n_active);
        return hipGetLastError();
    }
}

template <int D>
static hipError_t kmv_d(const KmvShape& sh, const float* Z, const float* Vp,
                        const uint16_t* VH, const uint16_t* VL, const KParams* kp,
                        float* part, const int* n_active, gp_precision prec, hipStream_t s,
                        hipEvent_t after_main) {
    if (sh.sym) return kmv_sym_d<D>(sh, Z, Vp, VH, VL, kp, part, n_active, prec, s, after_main);
    if (sh.mfma && prec == GP_BF16_SPLIT_V) return kmv_bf16_d<D, false>(sh, Z, VH, VL, kp, part, n_active, s);
    if (sh.mfma && prec == GP_BF16_SPLIT_KV) return kmv_bf16_d<D, true>(sh, Z, VH, VL, kp, part, n_active, s);
    const int64_t tiles = sh.n_pad / sh.rows_per_wg;
    const dim3 grid((unsigned)(tiles * sh.split));
    if (sh.mfma) {
        constexpr int R = D <= 8 ? 4 : 2;
        const int nb = sh.mp / 16;
        if (sh.tail == 0 ? sh.mp % 16 != 0 : sh.mp != nb * 16 + 4) return hipErrorInvalidValue;
        return kmv_f32_nb<D, R>(nb, sh.tail, grid, Z, Vp, part, sh, kp, n_active, s);
    } else {
        const int mu = sh.mu > 0 ? sh.mu : sh.mp;
        if (mu > sh.mp || sh.mp - mu >= 4) return hipErrorInvalidValue;
#define GPK_VALU_LAUNCH(MC, MU)                                                                   \
    case MU: kmv_valu_kernel<D, MC, MU, 1><<<grid, kWG, 0, s>>>(Z, Vp, sh.n_pad, part, sh.n_pad, \
                                                                  sh.chunk, sh.split, kp, n_active); break
        switch (sh.mp) {
            case 4: switch (mu) { GPK_VALU_LAUNCH(4, 1); GPK_VALU_LAUNCH(4, 2); GPK_VALU_LAUNCH(4, 4); default: return hipErrorInvalidValue; } break;
            case 8: switch (mu) { GPK_VALU_LAUNCH(8, 5); GPK_VALU_LAUNCH(8, 6); GPK_VALU_LAUNCH(8, 8); default: return hipErrorInvalidValue; } break;
            case 12: switch (mu) { GPK_VALU_LAUNCH(12, 9); GPK_VALU_LAUNCH(12, 10); GPK_VALU_LAUNCH(12, 12); default: return hipErrorInvalidValue; } break;
            case 16: switch (mu) { GPK_VALU_LAUNCH(16, 13); GPK_VALU_LAUNCH(16, 14); GPK_VALU_LAUNCH(16, 16); default: return hipErrorInvalidValue; } break;
            default: return hipErrorInvalidValue;
        }
#undef GPK_VALU_LAUNCH
    }
    return hipGetLastError();
}

#define GPK_DISPATCH_D(d, FN, ...)                    \
    switch (d) {                                      \
        case 1: return FN<1>(__VA_ARGS__);            \
        case 2: return FN<2>(__VA_ARGS__);            \
        case 3: return FN<3>(__VA_ARGS__);            \
        case 4: return FN<4>(__VA_ARGS__);            \
        case 5: return FN<5>(__VA_ARGS__);            \
        case 6: return FN<6>(__VA_ARGS__);            \
        case 7: return FN<7>(__VA_ARGS__);            \
        case 8: return FN<8>(__VA_ARGS__);            \
        case 9: return FN<9>(__VA_ARGS__);            \
        case 10: return FN<10>(__VA_ARGS__);          \
        case 11: return FN<11>(__VA_ARGS__);          \
        case 12: return FN<12>(__VA_ARGS__);          \
        case 13: return FN<13>(__VA_ARGS__);          \
        case 14: return FN<14>(__VA_ARGS__);          \
        case 15: return FN<15>(__VA_ARGS__);          \
        case 16: return FN<16>(__VA_ARGS__);          \
        default: return hipErrorInvalidValue;         \
    }

static hipError_t kmv_any_d(const KmvShape& sh, int d, const float* Z, const float* Vp,
                            const uint16_t* VH, const uint16_t* VL, const KParams* kp, float* part,
                            const int* n_active, gp_precision prec, hipStream_t s, hipEvent_t after_main) {
    GPK_DISPATCH_D(d, kmv_d, sh, Z, Vp, VH, VL, kp, part, n_active, prec, s, after_main);
}

hipError_t launch_kmv_partials(const KmvShape& sh, int d, const float* Z, const float* Vp,
                               const uint16_t* VH, const uint16_t* VL, const KParams* kp,
                               float* part, const int* n_active, gp_precision prec,
                               hipStream_t s, hipEvent_t after_main) {
    hipError_t e = kmv_any_d(sh, d, Z, Vp, VH, VL, kp, part, n_active, prec, s, after_main);
    // shapes without a separate reduce: the main kernel ends with the launch
    if (e == hipSuccess && after_main != nullptr && !sh.sym) e = hipEventRecord(after_main, s);
    return e;
}

hipError_t launch_split_bf16(const float* Vp, int64_t total, uint16_t* VH, uint16_t* VL,
                             hipStream_t s) {
    split_bf16_kernel<<<grid_for(total / 2), kWG, 0, s>>>(Vp, total, VH, VL);
    return hipGetLastError();
}

hipError_t launch_kmv_reduce(const KmvShape& sh, const float* part, const float* Vp,
                             const KParams* kp, int64_t n, int m, float* out, int64_t ldo,
                             hipStream_t s) {
    kmv_reduce_kernel<<<grid_for(n * m), kWG, 0, s>>>(part, sh.split, sh.mp, sh.n_pad, Vp, kp,
                                                       n, m, out, ldo);
    return hipGetLastError();
}

template <int D>
static hipError_t dkmv_d(const KmvShape& sh, const float* Z, const float* Vp, const KParams* kp,
                         float* part, int64_t n, int m, float* out, int64_t ldo,
                         int64_t bstride, hipStream_t s) {
    const int64_t tiles = sh.n_pad / sh.rows_per_wg;
    const dim3 grid((unsigned)(tiles * sh.split));
    for (int c0 = 0; c0 < m; c0 += sh.mp) {
        const int mc = std::min(sh.mp, m - c0);
        const float* Vc = Vp + (int64_t)c0 * sh.n_pad;
        if (sh.mfma)
            dkmv_mfma_kernel<D><<<grid, kWG, 0, s>>>(Z, Vc, sh.n_pad, part, sh.n_pad, sh.chunk, sh.split, kp);
        else
            dkmv_valu_kernel<D><<<grid, kWG, 0, s>>>(Z, Vc, sh.n_pad, part, sh.n_pad, sh.chunk, sh.split, kp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        dkmv_reduce_kernel<<<grid_for(n * mc * (int64_t)(D + 2)), kWG, 0, s>>>(
            part, sh.split, D, sh.mp, sh.n_pad, Vc, kp, n, mc, out + c0 * ldo, ldo, bstride);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_dkmv(const KmvShape& sh, int d, const float* Z, const float* Vp,
                       const KParams* kp, float* part, int64_t n, int m, float* out,
                       int64_t ldo, int64_t block_stride, hipStream_t s) {
    GPK_DISPATCH_D(d, dkmv_d, sh, Z, Vp, kp, part, n, m, out, ldo, block_stride, s);
}

}  // namespace gpk
