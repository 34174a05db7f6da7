// Host-side declarations shared by the translation units of the HIP library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "gp_common.h"
#include "ulisse_gp.h"

namespace gpk {

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int dpad(int d) { return (d + 3) & ~3; }

// Launch shape of one covariance product, chosen on the host.
struct KmvShape {
    bool mfma;        // MFMA contraction (m >= 16; the FP32 symmetric product also under
                      // 16 columns, one zero-padded block) or VALU contraction (m < 16)
    int mp;           // padded column count of V seen by the kernel
    int tail = 0;     // FP32 MFMA path: columns past the last multiple of 16 taken on the
                      // VALU (1..4; mp is then 16 floor(m / 16) + 4), else 0
    int mu = 0;       // VALU path: columns contracted (m or mp; mp - mu < 4), 0 = all mp
    int rows_per_wg;  // rows of K handled by one workgroup
    int split;        // column chunks (split-K), chunk index = blockIdx % split
    int chunk;        // columns of K per chunk (multiple of 64)
    int64_t n_pad;
    // symmetric FP32 product (each off-diagonal entry of K used twice): row tiles of 256
    // rows against column chunks of cs columns; the partials buffer then holds the result
    // (split = 1 layout) followed by the forward (nch chunks) and transposed (nt tiles)
    // partials, kmv_part_floats(sh) floats in all
    bool sym = false;
    int cs = 0, nch = 0, nt = 0;
};

// The default shape of a product: the symmetric product where it applies and was measured
// faster (16 columns and more: d >= 12 always; d <= 11, FP32: one MFMA block of columns, or
// n_pad >= 32768; BF16: two blocks and n_pad >= 32768; under 16 columns, FP32 only, one
// zero-padded block: m + d >= 12 and n_pad >= 16384), else the split-K product for about
// 2048 workgroups (the VALU contraction below 16 columns: 8192, at most 32 chunks per row
// tile).
KmvShape kmv_shape(int64_t n, int d, int m, gp_precision prec);
// The shape code of that default: 0 symmetric, else the split-K workgroup target.
int kmv_default_code(int64_t n, int d, int m, gp_precision prec);
// The split-K product with the factor chosen for about target_wg workgroups (the
// autotuner times several targets per shape); never symmetric.
KmvShape kmv_shape_target(int64_t n, int d, int m, gp_precision prec, int target_wg);
// The symmetric shape of (n, d, m, prec), or a shape with sym = false if it does not apply.
KmvShape kmv_shape_sym(int64_t n, int d, int m, gp_precision prec);
// Floats of the partials buffer that launch_kmv_partials needs for shape sh.
size_t kmv_part_floats(const KmvShape& sh);
KmvShape dkmv_shape(int64_t n, int d, int m);

// Size of the fixed device scratch of the no-allocation entry points, and its device
// address on `device` (which must be current), looked up once per device.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
// The symmetric product keeps one partial vector per (row tile, column) and per (column
// chunk, row): (1 + n/cs + n/256) m n floats, which grows as n^2.  Above this many bytes the
// shape does not apply (n beyond about 200000 at 32 right-hand sides) and split-K is used.
constexpr size_t kSymPartialBytesMax = size_t(24) << 30;
hipError_t noalloc_scratch(int device, void** out);

// psi -> KParams and the scaled, padded inputs Z (n_pad x dpad(d), zero rows past n).
hipError_t launch_prep(const float* X, int64_t n, int d, int64_t ldx, const double* psi,
                       float* Z, int64_t n_pad, KParams* kp, hipStream_t s);
// Copy V (n x m, ldv) into a zero-padded n_pad x mp buffer (ld n_pad).
hipError_t launch_pack(const float* V, int64_t n, int m, int64_t ldv, float* Vp, int64_t n_pad,
                       int mp, hipStream_t s);
// Split-K partial products K V into part[split][mp][n_pad].  Vp is n_pad x mp, ld n_pad
// (GP_FP32, or any mode on the VALU path); the BF16 modes on the MFMA path read the split
// halves VH, VL (bf16, same layout) made by launch_split_bf16 instead.
// If n_active is non-null and *n_active == 0 on the device, the launch does nothing.
// after_main (nullable) is recorded on s once the main product kernel is queued: before the
// symmetric shape's reduce, at the end for the other shapes.
hipError_t launch_kmv_partials(const KmvShape& sh, int d, const float* Z, const float* Vp,
                               const uint16_t* VH, const uint16_t* VL, const KParams* kp,
                               float* part, const int* n_active, gp_precision prec,
                               hipStream_t s, hipEvent_t after_main = nullptr);
// V_hi = bf16(V), V_lo = bf16(V - V_hi) elementwise over `total` (even) floats.
hipError_t launch_split_bf16(const float* Vp, int64_t total, uint16_t* VH, uint16_t* VL,
                             hipStream_t s);
inline bool uses_bf16(const KmvShape& sh, gp_precision prec) { return sh.mfma && prec != GP_FP32; }
// out[c*ldo + i] = sum_s part + lambda V  for i < n, c < m.
hipError_t launch_kmv_reduce(const KmvShape& sh, const float* part, const float* Vp,
                             const KParams* kp, int64_t n, int m, float* out, int64_t ldo,
                             hipStream_t s);
// Derivative products; see gp_dkmv.
hipError_t launch_dkmv(const KmvShape& sh, int d, const float* Z, const float* Vp,
                       const KParams* kp, float* part, int64_t n, int m, float* out,
                       int64_t ldo, int64_t block_stride, hipStream_t s);
size_t dkmv_part_floats(const KmvShape& sh, int d);

// Fused gradient reduction g_j = sum_ik dK_j(i,k) G(i,k), G = A B^T (A, B: n_pad x mq4,
// ld n_pad, zero padded), over the upper triangle of tiles.  Writes per-workgroup FP64
// partials for j = 0..d at gpart[j * nwg + workgroup].  The work table lists (row tile, first column tile) per
// workgroup; dquad_work builds it on the host.
struct DquadShape {
    int mq4;          // padded column count of A and B (multiple of 8)
    int mqb;          // padded column count of the BF16 operands (multiple of 32)
    int rows_per_wg;  // rows of a row tile (64)
    int split;        // unused
    int chunk;        // column tiles per workgroup (L)
    int64_t n_pad;
    int nwg;
};
DquadShape dquad_shape(int64_t n, int d, int mcols);
void dquad_work(const DquadShape& sh, std::vector<int2>& work);
// BF16 form: operands split into hi + lo halves, row-major with row stride sh.mqb.
hipError_t launch_dquad_bf16(const DquadShape& sh, int d, const float* Z, const uint16_t* AH,
                             const uint16_t* AL, const uint16_t* BH, const uint16_t* BL,
                             const KParams* kp, const int2* work, double* gpart, hipStream_t s);
hipError_t launch_dquad(const DquadShape& sh, int d, const float* Z, const float* A,
                        const float* B, const KParams* kp, const int2* work, double* gpart,
                        hipStream_t s);

// Pipe probe (pipes.hip): mode 0..5, `blocks` workgroups of 256 threads, one float of out
// per thread.
hipError_t launch_pipe_probe(int mode, int blocks, int iters, float* out, hipStream_t s);

}  // namespace gpk
