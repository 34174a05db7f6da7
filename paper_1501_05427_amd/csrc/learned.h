// Host-side declarations of the learned preconditioner kernels (learned.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gp_common.h"

namespace gpk {

// Offsets (in floats) of the MLP parameter buffer: in -> H (tanh) -> H (tanh) -> O.
struct MlpLayout {
    int in, H, O;
    int64_t w1, b1, w2, b2, w3, b3, trainable;
    int64_t in_mu, in_sd, out_mu, out_sd, total;
};
MlpLayout mlp_layout(int in, int H, int O);

int ts_blocks(int64_t n);
// out (ka x kb, row-major, FP64) = A^T B over n rows; part: ts_blocks(n) * ka * kb doubles.
hipError_t launch_gram(const float* A, int64_t lda, int ka, const float* B, int64_t ldb, int kb,
                       int64_t n, double* part, double* out, hipStream_t s);
// Yout = Yin M (M k x k row-major FP64), n rows; Yin and Yout must not overlap.
hipError_t launch_right_mul(const float* Yin, int64_t ldi, float* Yout, int64_t ldo, int k,
                            int64_t n, const double* M, hipStream_t s);
// M = L^-T for G + shift_rel (tr G / k) I = L L^T (k x k, row-major); *status = 1 if the
// matrix is not positive definite.
hipError_t launch_chol_inv(const double* G, int k, double shift_rel, double* M, int* status,
                           hipStream_t s);
// Eigenvectors (columns of Q, row-major) and eigenvalues (decreasing) of symmetric T.
hipError_t launch_jacobi_eig(const double* T, int k, double* Q, double* evals, hipStream_t s);
hipError_t launch_omega(int64_t n, int k, int64_t ld, uint64_t k0, uint64_t k1, float* Om,
                        hipStream_t s);
// out (2k + 1 floats) = (T^-1 w, log diag T, log tau) from T = U^T K U and w = U^T y.
hipError_t launch_targets(const double* Tm, const double* w, int k, int64_t n, const KParams* kp,
                          float* out, hipStream_t s);
hipError_t launch_mlp_init(float* prm, const MlpLayout& L, const double* psis, const float* T, int N,
                           uint64_t k0, uint64_t k1, hipStream_t s);
hipError_t launch_mlp_forward(const float* prm, const MlpLayout& L, const double* psis, int B,
                              float* xs, float* a1, float* a2, float* y, int bf16, hipStream_t s);
hipError_t launch_mlp_backward(const float* prm, const MlpLayout& L, const float* T, int B,
                               const float* xs, const float* a1, const float* a2, const float* y,
                               float* dy, float* d2, float* d1, float* grad, double* lpart,
                               float* loss, hipStream_t s);
hipError_t launch_adam(float* prm, const float* grad, float* m, float* v, int64_t count, float lr,
                       int t, hipStream_t s);
hipError_t launch_mlp_to_precond(const float* y, const MlpLayout& L, int k, const float* prm,
                                 double* coef, double* cvec, hipStream_t s);
hipError_t launch_warm_from_c(const float* U, int64_t ldu, int k, int64_t n, const double* c,
                              double* s0, hipStream_t s);
// Galerkin targets (2k + 1 FP32: c, log d, log tau) -> coef and c, as from the network.
hipError_t launch_targets_to_precond(const float* T, int k, double* coef, double* cvec, hipStream_t s);
// s0 = U c if coef[k] > 0 (the preconditioner is in use), else alt (zero if null).
hipError_t launch_pc_warm(const float* U, int64_t ldu, int k, int64_t n, const double* c,
                          const double* coef, const double* alt, double* s0, hipStream_t s);

}  // namespace gpk
