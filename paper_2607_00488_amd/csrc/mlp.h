// Internal declarations of the learned surrogate (MLP on BF16 matrix cores).
#pragma once
#include "common.h"

namespace nr {

typedef __bf16 bf16;

// Epilogues of the generic BF16 GEMM.
enum MlpMode {
    kMlpStore32 = 0,   // C32 = acc                       (weight gradients)
    kMlpSilu = 1,      // C32 = z = acc; C16 = SiLU(z)     (hidden forward)
    kMlpMse = 2,       // r = acc - T; C16 = scale * 2r    (output, training)
    kMlpDSilu = 3,     // C16 = acc * SiLU'(Z)             (hidden backward)
    kMlpNll = 4,       // mu = exp(mean + std * acc); per point partial
                       // sums of mu - n ln mu (its own kernel, k_mlp_nll)
    kMlpLogMu = 5,     // C32 = mean + std * acc           (log mu output)
};

// C[M][N] = A[M][K] B[K][N] with A(m,k) = A[m*sam + k*sak] and
// B(k,n) = B[k*sbk + n*sbn]; one of (sam, sak) and one of (sbk, sbn) is 1,
// M, N, K are multiples of 8 and the operands 16-byte aligned.
struct MlpGemm {
    const bf16* A;
    long sam, sak;
    const bf16* B;
    long sbk, sbn;
    int M, N, K;
    float* C32;
    long ldc;
    bf16* C16;
    long ldc16;
    const float* aux;   // Z (DSilu) or targets T (Mse)
    long ldaux;
    float scale;
    double* tile_loss;  // [gridDim.y][gridDim.x] (Mse)
    const float* mean;  // [N] (Nll, LogMu)
    const float* stdv;  // [N]
    const double* nobs; // [N] data (Nll)
    double* part;       // [M][n_nt] partial sums of mu - n ln mu (Nll)
    int n_nt;
    // K split (Store32 only): work-group z sums k in [z k_chunk, (z+1)
    // k_chunk) into the slab C32 + z c_split; 0 = one pass over all of K
    int k_chunk;
    long c_split;
};

// v[m][n] = sum_s part[s][m][n] over n_split slabs of stride c_split
// (rows of ldc floats), in slab order; then out[m][n] = v (FP32), or with
// dsilu C16[m][n] = v SiLU'(aux[m][n]) as the GEMM's kMlpDSilu epilogue.
struct KSumArgs {
    const float* part;
    long c_split, ldc;
    int n_split, M, N;
    float* out;
    long ldo;
    int dsilu;
    const float* aux;
    long ldaux;
    bf16* C16;
    long ldc16;
};

struct MlpInput {
    const double* theta;  // [B][7]
    int B;
    double lo[kNTheta], hi[kNTheta];
    bf16* x;              // [B][32]: normalised theta, 1 (bias), zeros
    int* outside;         // [B] 1 if theta lies outside the box
};

struct AdamArgs {
    float* w;             // fp32 master parameters [n]
    bf16* w16;            // bf16 copy [n]
    const float* g;       // gradient [n]
    float* m;
    float* v;
    long n;
    float lr, b1, b2, eps, bc1, bc2;  // bc = 1 - beta^t
};

struct TargetArgs {
    const double* mu;     // [P][N]
    int P, N;
    const float* mean;
    const float* stdv;
    float* t;             // [P][N] standardised log mu
};

// The hidden layers for the fused inference kernel: input x [M][32]
// (normalised theta, 1, zeros) and three layers of kFusedHidden outputs
// with weights W_l [kFusedHidden][k_l], k_0 = 32 and k_1 = k_2 =
// kFusedHidden + 8 (the inputs, the bias column, zeros).
constexpr int kFusedHidden = 256;
struct MlpHidden {
    const bf16* x;
    const bf16* w[3];
    int k[3];
};

hipError_t launch_mlp_gemm(int mode, const MlpGemm& g, hipStream_t s);
// The whole network and the likelihood partials in one launch (kMlpNll's
// output with the hidden layers formed in LDS); g as for kMlpNll except
// that g.A is not read.
hipError_t launch_mlp_nll_fused(const MlpGemm& g, const MlpHidden& h, hipStream_t s);
hipError_t launch_mlp_ksum(const KSumArgs& a, hipStream_t s);
hipError_t launch_mlp_input(const MlpInput& a, hipStream_t s);
// dst[c][r] = src[r][c] for a rows x cols row-major BF16 matrix
hipError_t launch_transpose_bf16(const bf16* src, bf16* dst, int rows, int cols,
                                 hipStream_t s);
hipError_t launch_adam(const AdamArgs& a, hipStream_t s);
hipError_t launch_targets(const TargetArgs& a, hipStream_t s);
hipError_t launch_fill_ones_col(bf16* h, int B, int ld, int col, hipStream_t s);

}  // namespace nr
