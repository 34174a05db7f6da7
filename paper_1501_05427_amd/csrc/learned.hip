// Learned warm start and preconditioner for the ULISSE solves.
//
// A fixed basis U (n x k, orthonormal) is built once at a reference psi by a randomized
// range finder of K (two steps of subspace iteration, each orthonormalised by shifted
// CholeskyQR2 in FP64) and a Rayleigh-Ritz rotation, so that U^T K(psi_ref) U is diagonal.  For any psi the Galerkin quantities
//   T(psi) = U^T K(psi) U,  w(psi) = U^T y
// give the training targets: c = T^-1 w (warm start s0 = U c), log diag T (the rank-k part
// of the preconditioner) and log tau with tau = (tr K - tr T) / (n - k) (its scaled
// identity part; tr K = n (sigma^2 + lambda)).  A small MLP psi -> (c, log d, log tau) is
// trained on those pairs with FP32 weights and Adam, and evaluated with BF16 operands at
// sampling time; its output becomes
//   P^-1 = tau^-1 I + U diag(1/d - 1/tau) U^T
// for gp_stoch_grad_pc.  Any SPD P keeps the estimator unbiased, so the network only
// changes the cost of the solves, never their expectation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "gp_common.h"
#include "internal.h"
#include "learned.h"

namespace gpk {

// ---------------------------------------------------------------------------------------
// Tall-skinny products
// ---------------------------------------------------------------------------------------
constexpr int kTS = 256;  // rows per workgroup

// part[blk][a][b] = sum over the block's rows of A[a][i] * B[b][i] (A: ka columns, B: kb
// columns, both column-major FP32 with their own leading dimensions), FP64.
__global__ __launch_bounds__(kWG) void gram_partial_kernel(const float* __restrict__ A, int64_t lda,
                                                           int ka, const float* __restrict__ B,
                                                           int64_t ldb, int kb, int64_t n,
                                                           double* __restrict__ part) {
    __shared__ float as[64][65];
    __shared__ float bs[64][65];
    const int64_t base = (int64_t)blockIdx.x * kTS;
    const int nout = ka * kb;
    double acc[16];
    for (int r = 0; r < 16; ++r) acc[r] = 0.0;
    for (int sub = 0; sub < kTS / 64; ++sub) {
        const int64_t r0 = base + sub * 64;
        for (int e = threadIdx.x; e < ka * 64; e += kWG) {
            const int a = e / 64, rr = e % 64;
            as[a][rr] = r0 + rr < n ? A[a * lda + r0 + rr] : 0.f;
        }
        for (int e = threadIdx.x; e < kb * 64; e += kWG) {
            const int b = e / 64, rr = e % 64;
            bs[b][rr] = r0 + rr < n ? B[b * ldb + r0 + rr] : 0.f;
        }
        __syncthreads();
        for (int r = 0; r < 16; ++r) {
            const int o = threadIdx.x + r * kWG;
            if (o < nout) {
                const int a = o / kb, b = o % kb;
                double s = acc[r];
                for (int rr = 0; rr < 64; ++rr) s = fma((double)as[a][rr], (double)bs[b][rr], s);
                acc[r] = s;
            }
        }
        __syncthreads();
    }
    for (int r = 0; r < 16; ++r) {
        const int o = threadIdx.x + r * kWG;
        if (o < nout) part[(int64_t)blockIdx.x * nout + o] = acc[r];
    }
}

__global__ void sum_partials_kernel(const double* __restrict__ part, int nblk, int nout,
                                    double* __restrict__ out) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nout) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * nout + o];
    out[o] = s;
}

// Y[:, b] <- sum_a Y[:, a] * M[a][b] (M: k x k FP64 row-major), in place through a copy.
__global__ __launch_bounds__(kWG) void right_mul_kernel(const float* __restrict__ Yin, int64_t ldi,
                                                        float* __restrict__ Yout, int64_t ldo, int k,
                                                        int64_t n, const double* __restrict__ M) {
    __shared__ double ms[64 * 64];
    for (int e = threadIdx.x; e < k * k; e += kWG) ms[e] = M[e];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kWG + threadIdx.x;
    if (i >= n) return;
    double y[64];
    for (int a = 0; a < k; ++a) y[a] = (double)Yin[a * ldi + i];
    for (int b = 0; b < k; ++b) {
        double s = 0.0;
        for (int a = 0; a < k; ++a) s += y[a] * ms[a * k + b];
        Yout[b * ldo + i] = (float)s;
    }
}

// Lower Cholesky factor of the k x k SPD matrix G (row-major) and M = L^-T (so that
// Y M has orthonormal columns when G = Y^T Y).  One workgroup; column-oriented updates.
// With shift_rel > 0 the factorised matrix is G + shift_rel * (tr G / k) I (shifted
// CholeskyQR: the factor exists even when the FP32 block is numerically rank deficient, and
// a following unshifted pass restores orthonormality).
__global__ __launch_bounds__(kWG) void chol_inv_kernel(const double* __restrict__ G, int k,
                                                       double shift_rel, double* __restrict__ M,
                                                       int* __restrict__ status) {
    __shared__ double L[64 * 64];
    __shared__ double Li[64 * 64];
    __shared__ double shift;
    if (threadIdx.x == 0) {
        double tr = 0.0;
        for (int i = 0; i < k; ++i) tr += G[i * k + i];
        shift = shift_rel * tr / k;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += kWG) L[e] = G[e] + ((e / k == e % k) ? shift : 0.0);
    __syncthreads();
    for (int j = 0; j < k; ++j) {
        if (threadIdx.x == 0) {
            const double djj = L[j * k + j];
            L[j * k + j] = djj > 0.0 ? sqrt(djj) : 0.0;
            if (!(djj > 0.0)) *status = 1;
        }
        __syncthreads();
        const double ljj = L[j * k + j];
        for (int i = j + 1 + threadIdx.x; i < k; i += kWG) L[i * k + j] = ljj > 0.0 ? L[i * k + j] / ljj : 0.0;
        __syncthreads();
        // trailing update of the lower triangle
        for (int e = threadIdx.x; e < k * k; e += kWG) {
            const int i = e / k, c = e % k;
            if (i > j && c > j && c <= i) L[i * k + c] -= L[i * k + j] * L[c * k + j];
        }
        __syncthreads();
    }
    // Li = L^-1 by forward substitution, one column per thread
    for (int c = threadIdx.x; c < k; c += kWG) {
        for (int i = 0; i < k; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int t = c; t < i; ++t) s -= L[i * k + t] * Li[t * k + c];
            Li[i * k + c] = (i >= c && L[i * k + i] > 0.0) ? s / L[i * k + i] : 0.0;
        }
    }
    __syncthreads();
    // M = L^-T (row-major): M[a][b] = Li[b][a]
    for (int e = threadIdx.x; e < k * k; e += kWG) M[e] = Li[(e % k) * k + e / k];
}

// Eigen-decomposition of a symmetric k x k matrix (row-major) by cyclic Jacobi rotations;
// Q (row-major, columns = eigenvectors) and the eigenvalues, in decreasing order.
__global__ __launch_bounds__(kWG) void jacobi_eig_kernel(const double* __restrict__ T, int k,
                                                         double* __restrict__ Qout,
                                                         double* __restrict__ evals) {
    __shared__ double A[64 * 64];
    __shared__ double Q[64 * 64];
    __shared__ double cs[2];
    for (int e = threadIdx.x; e < k * k; e += kWG) {
        A[e] = 0.5 * (T[e] + T[(e % k) * k + e / k]);
        Q[e] = (e / k == e % k) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 30; ++sweep) {
        for (int p = 0; p < k - 1; ++p)
            for (int q = p + 1; q < k; ++q) {
                if (threadIdx.x == 0) {
                    const double apq = A[p * k + q];
                    double c = 1.0, sn = 0.0;
                    if (fabs(apq) > 1e-300) {
                        const double theta = (A[q * k + q] - A[p * k + p]) / (2.0 * apq);
                        const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        sn = t * c;
                    }
                    cs[0] = c;
                    cs[1] = sn;
                }
                __syncthreads();
                const double c = cs[0], sn = cs[1];
                if (sn != 0.0) {
                    for (int r = threadIdx.x; r < k; r += kWG) {  // columns p, q of A and Q
                        const double arp = A[r * k + p], arq = A[r * k + q];
                        A[r * k + p] = c * arp - sn * arq;
                        A[r * k + q] = sn * arp + c * arq;
                        const double qrp = Q[r * k + p], qrq = Q[r * k + q];
                        Q[r * k + p] = c * qrp - sn * qrq;
                        Q[r * k + q] = sn * qrp + c * qrq;
                    }
                    __syncthreads();
                    for (int r = threadIdx.x; r < k; r += kWG) {  // rows p, q of A
                        const double apr = A[p * k + r], aqr = A[q * k + r];
                        A[p * k + r] = c * apr - sn * aqr;
                        A[q * k + r] = sn * apr + c * aqr;
                    }
                }
                __syncthreads();
            }
        // convergence check
        __shared__ double off;
        if (threadIdx.x == 0) {
            double o = 0.0, dg = 0.0;
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < k; ++j) (i == j ? dg : o) += A[i * k + j] * A[i * k + j];
            off = o / fmax(dg, 1e-300);
        }
        __syncthreads();
        if (off < 1e-28) break;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // order by decreasing eigenvalue (selection on indices)
        int idx[64];
        for (int i = 0; i < k; ++i) idx[i] = i;
        for (int i = 0; i < k; ++i)
            for (int j = i + 1; j < k; ++j)
                if (A[idx[j] * k + idx[j]] > A[idx[i] * k + idx[i]]) {
                    const int t = idx[i];
                    idx[i] = idx[j];
                    idx[j] = t;
                }
        for (int j = 0; j < k; ++j) {
            evals[j] = A[idx[j] * k + idx[j]];
            for (int r = 0; r < k; ++r) Qout[r * k + j] = Q[r * k + idx[j]];
        }
    }
}

// Omega: n x k standard normals (Philox purpose 4, column c, block i/4), FP32 column-major.
__global__ void omega_kernel(int64_t n, int k, int64_t ld, uint64_t k0, uint64_t k1,
                             float* __restrict__ Om) {
    const int64_t nblk = (n + 3) / 4;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nblk * k;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(e / nblk);
        const int64_t b = e % nblk;
        const u64x4 w = philox4x64_10((uint64_t)b, (uint64_t)c, 4, 0, k0, k1);
        double z[4];
        box_muller(w.v[0], w.v[1], &z[0], &z[1]);
        box_muller(w.v[2], w.v[3], &z[2], &z[3]);
        for (int u = 0; u < 4; ++u)
            if (4 * b + u < n) Om[c * ld + 4 * b + u] = (float)z[u];
    }
}

// Targets from T = U^T K U (k x k row-major), w = U^T y and the trace of K:
// out = (c = T^-1 w (k), log diag T (k), log tau (1)) with tau = (tr K - tr T) / (n - k).
__global__ __launch_bounds__(kWG) void targets_kernel(const double* __restrict__ Tm, const double* __restrict__ w,
                                                      int k, int64_t n, const KParams* __restrict__ kp,
                                                      float* __restrict__ out) {
    __shared__ double L[64 * 64];
    __shared__ double x[64];
    for (int e = threadIdx.x; e < k * k; e += kWG) L[e] = 0.5 * (Tm[e] + Tm[(e % k) * k + e / k]);
    __syncthreads();
    if (threadIdx.x == 0) {
        double trT = 0.0;
        for (int i = 0; i < k; ++i) trT += L[i * k + i];
        for (int i = 0; i < k; ++i) out[k + i] = (float)log(fmax(L[i * k + i], 1e-300));
        const double trK = (double)n * (kp->sigma2 + kp->lam64);
        out[2 * k] = (float)log(fmax((trK - trT) / (double)(n - k), 1e-300));
    }
    __syncthreads();
    // Cholesky factor of T, column by column: the diagonal on one thread, the column below it
    // one row per thread (every entry summed in the same order as a sequential factorization)
    for (int j = 0; j < k; ++j) {
        if (threadIdx.x == 0) {
            double s = L[j * k + j];
            for (int t = 0; t < j; ++t) s -= L[j * k + t] * L[j * k + t];
            L[j * k + j] = sqrt(fmax(s, 1e-300));
        }
        __syncthreads();
        const double ljj = L[j * k + j];
        for (int i = j + 1 + (int)threadIdx.x; i < k; i += kWG) {
            double v = L[i * k + j];
            for (int t = 0; t < j; ++t) v -= L[i * k + t] * L[j * k + t];
            L[i * k + j] = v / ljj;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        // T c = w: forward and back substitution with the factor
        for (int i = 0; i < k; ++i) {
            double s = w[i];
            for (int t = 0; t < i; ++t) s -= L[i * k + t] * x[t];
            x[i] = s / L[i * k + i];
        }
        for (int i = k - 1; i >= 0; --i) {
            double s = x[i];
            for (int t = i + 1; t < k; ++t) s -= L[t * k + i] * x[t];
            x[i] = s / L[i * k + i];
        }
        for (int i = 0; i < k; ++i) out[i] = (float)x[i];
    }
}

// ---------------------------------------------------------------------------------------
// MLP: in -> H (tanh) -> H (tanh) -> O, FP32 parameters.  Layout of the parameter buffer:
//   W1 [in][H], b1 [H], W2 [H][H], b2 [H], W3 [H][O], b3 [O],
//   then (not trained) in_mu [in], in_sd [in], out_mu [O], out_sd [O].
// Inputs are standardised with (in_mu, in_sd); the network predicts standardised targets.
// ---------------------------------------------------------------------------------------
MlpLayout mlp_layout(int in, int H, int O) {
    MlpLayout L;
    L.in = in;
    L.H = H;
    L.O = O;
    L.w1 = 0;
    L.b1 = L.w1 + (int64_t)in * H;
    L.w2 = L.b1 + H;
    L.b2 = L.w2 + (int64_t)H * H;
    L.w3 = L.b2 + H;
    L.b3 = L.w3 + (int64_t)H * O;
    L.trainable = L.b3 + O;
    L.in_mu = L.trainable;
    L.in_sd = L.in_mu + in;
    L.out_mu = L.in_sd + in;
    L.out_sd = L.out_mu + O;
    L.total = L.out_sd + O;
    return L;
}

__device__ inline float bf16_round(float x) { return (float)(__bf16)x; }

// Y[b][o] = act(bias[o] + sum_i X[b][i] W[i][o]); X rows of length I (row-major).  With
// bf16, X and W enter the products rounded to BF16 (FP32 accumulation).
__global__ void dense_fwd_kernel(const float* __restrict__ X, int B, int I, const float* __restrict__ W,
                                 const float* __restrict__ bias, int O, float* __restrict__ Y, int act,
                                 int bf16) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * O) return;
    const int b = (int)(e / O), o = (int)(e % O);
    float s = bias[o];
    // the dot products below load eight terms at a time and add them in order: at batch 1
    // (one evaluation per SGLD step) a thread otherwise waits on one load per term
    int i = 0;
    for (; i + 8 <= I; i += 8) {
        float xv[8], wv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            xv[t] = X[(int64_t)b * I + i + t];
            wv[t] = W[(int64_t)(i + t) * O + o];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const float x = bf16 ? bf16_round(xv[t]) : xv[t], w = bf16 ? bf16_round(wv[t]) : wv[t];
            s = __builtin_fmaf(x, w, s);
        }
    }
    for (; i < I; ++i) {
        float x = X[(int64_t)b * I + i], w = W[(int64_t)i * O + o];
        if (bf16) {
            x = bf16_round(x);
            w = bf16_round(w);
        }
        s = __builtin_fmaf(x, w, s);
    }
    Y[e] = act ? tanhf(s) : s;
}

// dX[b][i] = sum_o dY[b][o] W[i][o]  (then times (1 - X^2) when X is a tanh output)
__global__ void dense_bwd_in_kernel(const float* __restrict__ dY, int B, int O, const float* __restrict__ W,
                                    int I, const float* __restrict__ Xact, float* __restrict__ dX) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * I) return;
    const int b = (int)(e / I), i = (int)(e % I);
    float s = 0.f;
    int o = 0;
    for (; o + 8 <= O; o += 8) {
        float dv[8], wv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            dv[t] = dY[(int64_t)b * O + o + t];
            wv[t] = W[(int64_t)i * O + o + t];
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) s = __builtin_fmaf(dv[t], wv[t], s);
    }
    for (; o < O; ++o) s = __builtin_fmaf(dY[(int64_t)b * O + o], W[(int64_t)i * O + o], s);
    if (Xact) {
        const float x = Xact[e];
        s *= 1.f - x * x;
    }
    dX[e] = s;
}

// dW[i][o] = sum_b X[b][i] dY[b][o];  db[o] = sum_b dY[b][o]  (one thread per (i, o) / o)
__global__ void dense_bwd_w_kernel(const float* __restrict__ X, const float* __restrict__ dY, int B, int I,
                                   int O, float* __restrict__ dW, float* __restrict__ db) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (int64_t)I * O) {
        const int i = (int)(e / O), o = (int)(e % O);
        float s = 0.f;
        int b = 0;
        for (; b + 8 <= B; b += 8) {
            float xv[8], dv[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                xv[t] = X[(int64_t)(b + t) * I + i];
                dv[t] = dY[(int64_t)(b + t) * O + o];
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) s = __builtin_fmaf(xv[t], dv[t], s);
        }
        for (; b < B; ++b) s = __builtin_fmaf(X[(int64_t)b * I + i], dY[(int64_t)b * O + o], s);
        dW[e] = s;
    } else if (e < (int64_t)I * O + O) {
        const int o = (int)(e - (int64_t)I * O);
        float s = 0.f;
        for (int b = 0; b < B; ++b) s += dY[(int64_t)b * O + o];
        db[o] = s;
    }
}

// standardised inputs: Xs[b][i] = (psi[b][i] - mu[i]) / sd[i]
__global__ void standardise_kernel(const double* __restrict__ psi, int B, int I,
                                   const float* __restrict__ mu, const float* __restrict__ sd,
                                   float* __restrict__ Xs) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)B * I) return;
    const int i = (int)(e % I);
    Xs[e] = (float)((psi[e] - (double)mu[i]) / (double)sd[i]);
}

// loss = mean over (b, o) of (Y - (T - mu)/sd)^2 ; dY = 2 (Y - t~) / (B O).
// One workgroup per 256 outputs writes a partial loss.
__global__ __launch_bounds__(kWG) void mse_kernel(const float* __restrict__ Y, const float* __restrict__ T,
                                                  int B, int O, const float* __restrict__ mu,
                                                  const float* __restrict__ sd, float* __restrict__ dY,
                                                  double* __restrict__ lpart) {
    __shared__ double scratch[4];
    const int64_t e = (int64_t)blockIdx.x * kWG + threadIdx.x;
    double l = 0.0;
    if (e < (int64_t)B * O) {
        const int o = (int)(e % O);
        const float t = (T[e] - mu[o]) / sd[o];
        const float r = Y[e] - t;
        dY[e] = 2.f * r / (float)((int64_t)B * O);
        l = (double)r * r;
    }
    l = block_sum256(l, scratch);
    if (threadIdx.x == 0) lpart[blockIdx.x] = l;
}

__global__ void loss_finish_kernel(const double* __restrict__ lpart, int nb, int64_t count,
                                   float* __restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += lpart[b];
    *loss = (float)(s / (double)count);
}

// Adam (Kingma & Ba) on the trainable prefix of the parameter buffer; step t >= 1.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t count, float lr, float b1, float b2,
                            float eps, int t) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gi;
    const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float mh = mi / (1.f - powf(b1, (float)t));
    const float vh = vi / (1.f - powf(b2, (float)t));
    p[e] -= lr * mh / (sqrtf(vh) + eps);
}

// Normalisation constants from the training set (column means and standard deviations,
// floored) and Xavier-normal initial weights from Philox (purpose 5), zero biases.
__global__ __launch_bounds__(kWG) void mlp_init_kernel(float* __restrict__ prm, MlpLayout L,
                                                       const double* __restrict__ psis,
                                                       const float* __restrict__ T, int N,
                                                       uint64_t k0, uint64_t k1) {
    const int tid = threadIdx.x;
    for (int i = tid; i < L.in; i += kWG) {
        double s = 0.0, s2 = 0.0;
        for (int b = 0; b < N; ++b) {
            const double v = psis[(int64_t)b * L.in + i];
            s += v;
            s2 += v * v;
        }
        const double mu = s / N, var = fmax(s2 / N - mu * mu, 0.0);
        prm[L.in_mu + i] = (float)mu;
        prm[L.in_sd + i] = (float)fmax(sqrt(var), 1e-6);
    }
    for (int o = tid; o < L.O; o += kWG) {
        double s = 0.0, s2 = 0.0;
        for (int b = 0; b < N; ++b) {
            const double v = T[(int64_t)b * L.O + o];
            s += v;
            s2 += v * v;
        }
        const double mu = s / N, var = fmax(s2 / N - mu * mu, 0.0);
        prm[L.out_mu + o] = (float)mu;
        prm[L.out_sd + o] = (float)fmax(sqrt(var), 1e-6);
    }
    const int64_t segs[3][3] = {{L.w1, L.in, L.H}, {L.w2, L.H, L.H}, {L.w3, L.H, L.O}};
    for (int sgi = 0; sgi < 3; ++sgi) {
        const int64_t off = segs[sgi][0], fin = segs[sgi][1], fout = segs[sgi][2];
        const double scale = sqrt(2.0 / (double)(fin + fout));
        for (int64_t e = tid; e < fin * fout; e += kWG) {
            const u64x4 w = philox4x64_10((uint64_t)e, (uint64_t)sgi, 5, 0, k0, k1);
            double z0, z1;
            box_muller(w.v[0], w.v[1], &z0, &z1);
            prm[off + e] = (float)(scale * z0);
        }
    }
    for (int e = tid; e < L.H; e += kWG) {
        prm[L.b1 + e] = 0.f;
        prm[L.b2 + e] = 0.f;
    }
    for (int e = tid; e < L.O; e += kWG) prm[L.b3 + e] = 0.f;
}

// MLP output (standardised) -> preconditioner coefficients and warm-start coefficients:
// u = out_mu + out_sd * y holds c, log d and log tau; h = 1/d - 1/tau, coef[k] = 1/tau, with
// d floored at tau so that P stays SPD.  An output with a non-finite value, or a log d or
// log tau outside [-60, 60], is rejected: h = 0, coef[k] = -1 (the marker that makes the
// solvers run plain CG) and c = 0.
__global__ void mlp_to_precond_kernel(const float* __restrict__ Y, MlpLayout L, int k,
                                      const float* __restrict__ prm, double* __restrict__ coef,
                                      double* __restrict__ cvec) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    auto un = [&](int o) { return (double)prm[L.out_mu + o] + (double)prm[L.out_sd + o] * (double)Y[o]; };
    bool ok = true;
    for (int o = 0; o <= 2 * k; ++o) {
        const double u = un(o);
        if (!isfinite(u) || (o >= k && fabs(u) > 60.0)) ok = false;
    }
    if (!ok) {
        for (int j = 0; j < k; ++j) {
            coef[j] = 0.0;
            if (cvec) cvec[j] = 0.0;
        }
        coef[k] = -1.0;
        return;
    }
    const double tau = exp(un(2 * k));
    for (int j = 0; j < k; ++j) {
        const double d = fmax(exp(un(k + j)), tau);
        coef[j] = 1.0 / d - 1.0 / tau;
        if (cvec) cvec[j] = un(j);
    }
    coef[k] = 1.0 / tau;
}

// Galerkin targets (c, log d, log tau; FP32, as precond_targets writes them) -> the same
// coefficients as mlp_to_precond_kernel, with the same rejection rule.
__global__ void targets_to_precond_kernel(const float* __restrict__ T, int k, double* __restrict__ coef,
                                          double* __restrict__ cvec) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    bool ok = true;
    for (int o = 0; o <= 2 * k; ++o) {
        const double u = (double)T[o];
        if (!isfinite(u) || (o >= k && fabs(u) > 60.0)) ok = false;
    }
    if (!ok) {
        for (int j = 0; j < k; ++j) {
            coef[j] = 0.0;
            if (cvec) cvec[j] = 0.0;
        }
        coef[k] = -1.0;
        return;
    }
    const double tau = exp((double)T[2 * k]);
    for (int j = 0; j < k; ++j) {
        const double d = fmax(exp((double)T[k + j]), tau);
        coef[j] = 1.0 / d - 1.0 / tau;
        if (cvec) cvec[j] = (double)T[j];
    }
    coef[k] = 1.0 / tau;
}

// s0[:, 0] = U c (FP64), the learned warm start of the y system.
__global__ void warm_from_c_kernel(const float* __restrict__ U, int64_t ldu, int k, int64_t n,
                                   const double* __restrict__ c, double* __restrict__ s0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += (double)U[j * ldu + i] * c[j];
    s0[i] = s;
}

// The warm start of system 0 inside a preconditioned solve: U c while the preconditioner is
// in use (coef[k] > 0), otherwise the caller's start `alt` (zero when alt is null).
__global__ void pc_warm_kernel(const float* __restrict__ U, int64_t ldu, int k, int64_t n,
                               const double* __restrict__ c, const double* __restrict__ coef,
                               const double* __restrict__ alt, double* __restrict__ s0) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!(coef[k] > 0.0)) {
        s0[i] = alt != nullptr ? alt[i] : 0.0;
        return;
    }
    double s = 0.0;
    for (int j = 0; j < k; ++j) s += (double)U[j * ldu + i] * c[j];
    s0[i] = s;
}

// ---------------------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------------------
static unsigned g1(int64_t total, int per = kWG) {
    return (unsigned)std::max<int64_t>(1, (total + per - 1) / per);
}

int ts_blocks(int64_t n) { return (int)((n + kTS - 1) / kTS); }

hipError_t launch_gram(const float* A, int64_t lda, int ka, const float* B, int64_t ldb, int kb,
                       int64_t n, double* part, double* out, hipStream_t s) {
    const int nb = ts_blocks(n);
    gram_partial_kernel<<<nb, kWG, 0, s>>>(A, lda, ka, B, ldb, kb, n, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    sum_partials_kernel<<<g1(ka * kb), kWG, 0, s>>>(part, nb, ka * kb, out);
    return hipGetLastError();
}

hipError_t launch_right_mul(const float* Yin, int64_t ldi, float* Yout, int64_t ldo, int k,
                            int64_t n, const double* M, hipStream_t s) {
    right_mul_kernel<<<g1(n), kWG, 0, s>>>(Yin, ldi, Yout, ldo, k, n, M);
    return hipGetLastError();
}

hipError_t launch_chol_inv(const double* G, int k, double shift_rel, double* M, int* status,
                           hipStream_t s) {
    chol_inv_kernel<<<1, kWG, 0, s>>>(G, k, shift_rel, M, status);
    return hipGetLastError();
}

hipError_t launch_jacobi_eig(const double* T, int k, double* Q, double* evals, hipStream_t s) {
    jacobi_eig_kernel<<<1, kWG, 0, s>>>(T, k, Q, evals);
    return hipGetLastError();
}

hipError_t launch_omega(int64_t n, int k, int64_t ld, uint64_t k0, uint64_t k1, float* Om,
                        hipStream_t s) {
    omega_kernel<<<g1((n + 3) / 4 * k), kWG, 0, s>>>(n, k, ld, k0, k1, Om);
    return hipGetLastError();
}

hipError_t launch_targets(const double* Tm, const double* w, int k, int64_t n, const KParams* kp,
                          float* out, hipStream_t s) {
    targets_kernel<<<1, kWG, 0, s>>>(Tm, w, k, n, kp, out);
    return hipGetLastError();
}

hipError_t launch_mlp_init(float* prm, const MlpLayout& L, const double* psis, const float* T, int N,
                           uint64_t k0, uint64_t k1, hipStream_t s) {
    mlp_init_kernel<<<1, kWG, 0, s>>>(prm, L, psis, T, N, k0, k1);
    return hipGetLastError();
}

// Forward pass for B inputs: activations a1, a2 (B x H) and output y (B x O) in `act`.
hipError_t launch_mlp_forward(const float* prm, const MlpLayout& L, const double* psis, int B,
                              float* xs, float* a1, float* a2, float* y, int bf16, hipStream_t s) {
    standardise_kernel<<<g1((int64_t)B * L.in), kWG, 0, s>>>(psis, B, L.in, prm + L.in_mu, prm + L.in_sd, xs);
    dense_fwd_kernel<<<g1((int64_t)B * L.H), kWG, 0, s>>>(xs, B, L.in, prm + L.w1, prm + L.b1, L.H, a1, 1, bf16);
    dense_fwd_kernel<<<g1((int64_t)B * L.H), kWG, 0, s>>>(a1, B, L.H, prm + L.w2, prm + L.b2, L.H, a2, 1, bf16);
    dense_fwd_kernel<<<g1((int64_t)B * L.O), kWG, 0, s>>>(a2, B, L.H, prm + L.w3, prm + L.b3, L.O, y, 0, bf16);
    return hipGetLastError();
}

// Loss and gradient of the trainable parameters (grad: L.trainable floats).
hipError_t launch_mlp_backward(const float* prm, const MlpLayout& L, const float* T, int B,
                               const float* xs, const float* a1, const float* a2, const float* y,
                               float* dy, float* d2, float* d1, float* grad, double* lpart,
                               float* loss, hipStream_t s) {
    const int nb = (int)g1((int64_t)B * L.O);
    mse_kernel<<<nb, kWG, 0, s>>>(y, T, B, L.O, prm + L.out_mu, prm + L.out_sd, dy, lpart);
    loss_finish_kernel<<<1, 64, 0, s>>>(lpart, nb, (int64_t)B * L.O, loss);
    dense_bwd_w_kernel<<<g1((int64_t)L.H * L.O + L.O), kWG, 0, s>>>(a2, dy, B, L.H, L.O, grad + L.w3, grad + L.b3);
    dense_bwd_in_kernel<<<g1((int64_t)B * L.H), kWG, 0, s>>>(dy, B, L.O, prm + L.w3, L.H, a2, d2);
    dense_bwd_w_kernel<<<g1((int64_t)L.H * L.H + L.H), kWG, 0, s>>>(a1, d2, B, L.H, L.H, grad + L.w2, grad + L.b2);
    dense_bwd_in_kernel<<<g1((int64_t)B * L.H), kWG, 0, s>>>(d2, B, L.H, prm + L.w2, L.H, a1, d1);
    dense_bwd_w_kernel<<<g1((int64_t)L.in * L.H + L.H), kWG, 0, s>>>(xs, d1, B, L.in, L.H, grad + L.w1, grad + L.b1);
    return hipGetLastError();
}

hipError_t launch_adam(float* prm, const float* grad, float* m, float* v, int64_t count, float lr,
                       int t, hipStream_t s) {
    adam_kernel<<<g1(count), kWG, 0, s>>>(prm, grad, m, v, count, lr, 0.9f, 0.999f, 1e-8f, t);
    return hipGetLastError();
}

hipError_t launch_mlp_to_precond(const float* y, const MlpLayout& L, int k, const float* prm,
                                 double* coef, double* cvec, hipStream_t s) {
    mlp_to_precond_kernel<<<1, 64, 0, s>>>(y, L, k, prm, coef, cvec);
    return hipGetLastError();
}

hipError_t launch_targets_to_precond(const float* T, int k, double* coef, double* cvec, hipStream_t s) {
    targets_to_precond_kernel<<<1, 64, 0, s>>>(T, k, coef, cvec);
    return hipGetLastError();
}

hipError_t launch_warm_from_c(const float* U, int64_t ldu, int k, int64_t n, const double* c,
                              double* s0, hipStream_t s) {
    warm_from_c_kernel<<<g1(n), kWG, 0, s>>>(U, ldu, k, n, c, s0);
    return hipGetLastError();
}

hipError_t launch_pc_warm(const float* U, int64_t ldu, int k, int64_t n, const double* c,
                          const double* coef, const double* alt, double* s0, hipStream_t s) {
    pc_warm_kernel<<<g1(n), kWG, 0, s>>>(U, ldu, k, n, c, coef, alt, s0);
    return hipGetLastError();
}

}  // namespace gpk
