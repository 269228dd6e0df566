// Internal declarations of the batched (GEMM) path.
#pragma once
#include "common.h"

namespace nr {

constexpr int kModeNll = 0;  // forward: fused Poisson epilogue
constexpr int kModeAdj = 1;  // adjoint: C = A R^T written as FP32

struct WgenArgs {
    const double* theta;  // [n_pts][7]
    int n_pts, ldw, n_t;
    const double* basis;  // [kNBasis][n_t]
    const double* ssm;    // [n_t]
    const double* mrow;   // [n_t]
    Phys ph;
    double* wt;           // [n_t][ldw]
};

// One GEMM problem of the grouped launch (one dataset / analysis).
// Forward: C[M=n_pts][N=n_reco] = A[M][K=n_t] B[K][N] with A given as its
// transpose At[K][lda] (M contiguous) and B = R[K][ldb].
// Adjoint: C[M][N=n_t] = A[M][K=n_reco] R^T with At[K][lda] and R[N][ldb].
// A is FP64, R FP32 (widened on the way into LDS), products/sums FP64.
struct GemmProb {
    const double* At;
    const float* B;
    int lda, ldb, M, N, K;
    // forward epilogue
    const double* n;
    const double* b;
    const double* theta;  // [M][7]
    double* part;         // [M][n_nt] deviance partials
    double* part_gb;      // [M][n_nt] sum_j a_j b_j partials (with aout)
    int n_nt;
    double* aout;         // [N][lda_out] d(-2lnL)/d mu, or null
    int lda_out;
    double* mu;           // [M][N] or null
    // adjoint output
    double* C;
    int ldc;
    int pad;
};

// One output tile of a problem: its reduction runs over k in [k0, k1)
// (the whole K, or with band skipping the K-steps of 16 whose response
// entries for this tile are not all zero).
constexpr int kGemmBK = 16;  // K step of the GEMM kernels

struct GemmTile {
    int prob, mt, nt, cost;
    int k0, k1;
};

struct FinalArgs {
    const double* part;
    const double* theta;
    int n_pts, n_nt;
    double cdata;
    double pull_mean[kNTheta];
    double pull_sigma[kNTheta];
    double* nll;
};

struct ContractArgs {
    double* U;       // [n_pts][ldu]; its chunks' first columns take the partial sums
    int ldu, n_t, n_pts, n_nt;
    const double* ssm;
    const double* mrow;
    const double* basis;
    const double* theta;
    const double* part_gb;
    double pull_mean[kNTheta];
    double pull_sigma[kNTheta];
    Phys ph;
    double* grad;    // [n_pts][7]
};


// Template form.  S_theta = sum_b c_b(theta) I_b with theta-independent
// basis spectra I_b, so the fold separates into templates folded once:
//   mu_j = f_bkg b_j + G0_j + sum_b c_b(theta) G_bj,
//   G_bj = sum_{l: S_SM(T_l) > 0} F_bl R_lj,  F_bl = m_l I_b(T_l) / S_SM(T_l),
//   G0_j = sum_{l: S_SM(T_l) = 0} m_l R_lj   (rows with w := 1).
constexpr int kTmplCols = kNBasis + 1;     // G_0..G_19, G0
constexpr int kTmplRec = 24;               // per reco bin: G_0..G_19, G0, b, n, pad
constexpr int kTmplSlabRows = 256;         // response rows per template-fold work-group
constexpr int kTmplWave = 64;              // points per evaluation work-group

struct TmplFoldArgs {
    const float* R;
    int ldr, n_t, n_reco;
    const double* F;   // [n_t][kTmplCols] row factors
    double* part;      // [n_slab][kTmplCols][n_reco]
};

struct TmplRecArgs {
    const double* part;
    int n_slab, n_reco;
    double* rec;       // [n_reco][rl]
    int rl;            // record length (doubles)
    int dst[kTmplCols];  // record column of each folded column, -1: not kept
};

struct TmplDataArgs {
    const double* n;   // [n_reco] data
    const double* b;   // [n_reco] background
    int n_reco;
    double* rec;       // [n_reco][kTmplRec]
};

struct TmplEvalArgs {
    const double* rec;    // [n_reco][kTmplRec]
    const double* theta;  // [n_pts][7]
    int n_reco, n_pts, cols_per;
    Phys ph;
    double* dpart;        // [n_split][n_pts] deviance partials
    double* hpart;        // [n_split][kTmplCols][n_pts] or null (gradient)
    double* mu;           // [n_pts][n_reco] or null
};

// Slice sums in slice order: red[0][p] = deviance, red[1 + v][p] = the
// gradient contraction v (n_acc of them).
struct TmplReduceArgs {
    const double* dpart;
    const double* hpart;  // [n_split][n_acc][n_pts] or null
    int n_pts, n_split, n_acc;
    double* red;          // [1 + n_acc][n_pts] (first row only without hpart)
};

struct TmplFinalArgs {
    const double* red;    // [1 + kTmplCols][n_pts] (first row only without grad)
    const double* theta;
    int n_pts;
    double cdata;
    double pull_mean[kNTheta];
    double pull_sigma[kNTheta];
    Phys ph;
    double* nll;
    double* grad;         // [n_pts][7] or null
};

// Multi-component template form (Eqs. (Rij), (fNp_reweight), (mu_total)):
// component k's sources give 10 basis spectra (no group scaling: the rate
// parameter r_k scales the component), so per reco bin the record holds
// G^(k)_0..9 and G0^(k) for each component, the background templates
// MT Rate_q pdf_q(j), the common mask M_j and the data n_j:
//   mu_j = M_j [ sum_k r_k (G0^(k)_j + sum_b c_b G^(k)_bj) + sum_q r_q B_qj ].
constexpr int kTmplMaxComp = 8;
constexpr int kTmplMaxBkg = 8;
constexpr int kTmplSmallComp = 5;  // a smaller register class of the kernel
constexpr int kTmplSmallBkg = 4;
constexpr int kTmplCompCols = 11;

struct TmplMultiDataArgs {
    const double* n;     // [n_reco]
    const double* bkg;   // [B][n_reco]
    const double* mask;  // [n_reco] or null (1)
    int n_reco, K, B, rl;
    double* rec;
};

struct TmplMultiEvalArgs {
    const double* rec;    // [n_reco][rl]
    const double* theta;  // [n_pts][n_theta], n_theta = 5 + K + B
    int rl, K, B, n_theta, n_reco, n_pts, cols_per;
    Phys ph;
    double* dpart;        // [n_split][n_pts]
    double* hpart;        // [n_split][10 + K + B][n_pts] or null (gradient)
    double* mu;           // [n_pts][n_reco] or null
};

struct TmplMultiFinalArgs {
    const double* red;    // [1 + 10 + K + B][n_pts]
    const double* theta;
    int n_theta, K, B, n_pts;
    double cdata;
    double pull_mean[kMaxTheta];
    double pull_sigma[kMaxTheta];
    Phys ph;
    double* nll;
    double* grad;         // [n_pts][n_theta] or null
};

hipError_t launch_tmpl_fold(const TmplFoldArgs& a, int n_slab, hipStream_t s);
hipError_t launch_tmpl_mdata(const TmplMultiDataArgs& a, hipStream_t s);
hipError_t launch_tmpl_meval(const TmplMultiEvalArgs& a, int n_split, hipStream_t s);
hipError_t launch_tmpl_mfinal(const TmplMultiFinalArgs& a, hipStream_t s);
hipError_t launch_tmpl_records(const TmplRecArgs& a, hipStream_t s);
hipError_t launch_tmpl_data(const TmplDataArgs& a, hipStream_t s);
hipError_t launch_tmpl_eval(const TmplEvalArgs& a, int n_split, hipStream_t s);
hipError_t launch_tmpl_reduce(const TmplReduceArgs& a, hipStream_t s);
hipError_t launch_tmpl_final(const TmplFinalArgs& a, hipStream_t s);

hipError_t launch_wgen(const WgenArgs& a, hipStream_t s);
// Tile configurations of the GEMM: 0: 128x128, 1: 64x128, 2: 128x64,
// 3: 64x64 (M x N per work-group).
constexpr int kGemmConfigs = 4;
hipError_t launch_gemm(int mode, int cfg, const GemmProb* probs, const GemmTile* tiles,
                       int n_tiles, unsigned* ctr, int grid, hipStream_t s);
int gemm_tile_m(int cfg);
int gemm_tile_n(int cfg);
hipError_t launch_finalize(const FinalArgs& a, hipStream_t s);
hipError_t launch_adj_contract(const ContractArgs& a, hipStream_t s);
int gemm_grid(int mode, int cfg, int n_tiles);

}  // namespace nr
