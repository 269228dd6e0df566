// Internal declarations shared by the HIP translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace nr {

constexpr int kNTheta = 7;
constexpr int kMaxTheta = 32;       // parameters of the multi-component form
constexpr int kStepRows = 512;      // recoil rows per weights work-group
constexpr int kNBasis = 20;         // theta-independent recoil basis spectra

// Physical constants in the units the device works in: the weak prefactor
// 2 G_F^2 m_e / pi of Eq. (sm_cross_section) is set to one, so the
// magnetic-moment term carries cmm = (pi alpha^2/m_e^2) / (2 G_F^2 m_e/pi)
// per unit m2 = (mu_nu / 1e-11 mu_B)^2.
struct Phys {
    double me;        // MeV
    double sw2;
    double tau_frac;  // nu_tau share of 1 - P_ee
    double cmm;       // MeV per unit m2
    double gLe, gLm, gR;  // tree-level chiral couplings (e, mu/tau, R)
};

// Node table of one point: one work-group per source k builds the suffix
// sums C_k(j) = sum_{i >= j} c_i of the per-node Laurent coefficients
// (a0, a1, a2, am) into table[j + k]; table[srcOff[k+1] + k] is zero.
struct ScanArgs {
    const double* nodeIE;  // [n_nodes] 1 / E_j, E-sorted within a source
    const double* nodeW;   // [n_nodes] quadrature weight times flux
    const double* nodePe;  // [n_nodes] P_ee(E_j)
    const int* srcOff;     // [n_src+1] first node of each source
    const int* srcGroup;   // [n_src] 1: scaled by f_8B
    const double* theta;   // device, 7 doubles
    Phys ph;
    double4* table;        // [n_nodes + n_src]
    const int* blocks;     // [nb_scan][2]: source, chunk (0 = highest 512 nodes)
    double4* ctot;         // [n_src][max_chunks] chunk totals
    int max_chunks;
};

// Weights of one point from its node table, one thread per row of the
// (stacked) response: row r = k * n_t + l is recoil bin l of signal
// component k, whose spectrum sums the sources compSrc[compOff[k] ..
// compOff[k+1]).  The single-component form has one component holding every
// source.
struct RowArgs {
    const double4* table;
    const int* srcOff;     // [n_src+1]
    const double4* ctot;   // [n_src][max_chunks] chunk totals of the node scan
    int max_chunks;
    const int* jmin;      // [n_src][n_t] first reachable global node index
    const double* tc;     // [n_t] recoil-bin centres
    int n_t, n_comp;
    const int* compOff;   // [n_comp+1]
    const int* compSrc;   // [n_src] source indices grouped by component
    const double* ssm;    // [n_comp*n_t] S_SM per component (this code at theta_SM)
    const double* mrow;   // [n_comp*n_t] row factors
    const double* theta;  // device, the point (for the component rates)
    int rate_index;       // theta index of component 0's rate; -1: none
    double* v;            // [n_comp*n_t] row factor x weight (x rate)
    double* out_w;        // [n_comp*n_t] or null: weights w
    double* out_s;        // [n_comp*n_t] or null: write S_theta itself and stop
};

struct FoldArgs {
    const float* R;       // [n_t][ldr]
    int ldr;              // leading dimension (floats), multiple of 4
    int n_t, n_reco;
    const double* v;      // [n_t] m_l w_l
    const double* n;      // [n_reco]
    const double* b;      // [n_reco]
    const double* theta;  // device, 7 doubles
    double* colpart;      // [n_rb][ldr] partial rows of the fold tiles
    double* chunk_dev;    // [n_cc] group sums of the deviance
    double* chunk_gb;     // [n_cc] group sums of a_j b_j
    double* out_nll;      // [1]
    double* out_mu;       // [n_reco] or null
    double* out_a;        // [ldr] or null: d(-2lnL)/d mu_j
    double* out_gb;       // [1] or null: sum_j a_j b_j
    double cdata;
    double pull_mean[kMaxTheta];
    double pull_sigma[kMaxTheta];
    int n_theta;          // parameters per point
    int bkg_index;        // theta index of the first background rate
    int n_bkg;            // background templates: mu_j += theta[bkg_index+b] b[b][j]
    const double* mask;   // [n_reco] or null: mu_j = mask_j (fold_j + backgrounds)
    int rows_per_wg;      // recoil rows per fold tile
    int n_rb;             // fold row tiles = partial rows
    int n_fc;             // fold column tiles (2048 columns each)
    int n_cc;             // reduction groups (64 columns each)
    int reverse;          // fold: walk the tile's rows last to first
    int stream_nt;        // fold: read R without cache allocation
    // fold: per tile (index cc * n_rb + rb) the float4 columns [lo, hi) that
    // hold its rows' non-zero responses, or null (read every column)
    const int* band;
};

// One launch of the single-point step kernel: nb_fold = n_rb * n_fc
// work-groups fold the point `fold` describes, nb_rows form the weights of
// the point `rows` describes (512 rows each), nb_scan = n_src build the
// node table of the point `scan` describes, nb_fin = n_cc reduce the fold of
// the point `fin` describes into group sums, and nb_final (0 or 1) adds the
// group sums of the point `fnl` describes.  Any of the counts may be zero.
struct StepArgs {
    FoldArgs fold;
    FoldArgs fin;
    FoldArgs fnl;
    RowArgs rows;
    ScanArgs scan;
    int nb_fold, nb_rows, nb_scan, nb_fin, nb_final;
};

struct AdjArgs {
    const float* R;
    int ldr, n_t, n_reco;
    const double* a;      // [ldr]
    const double* ssm;
    const double* mrow;
    const double* basis;  // [kNBasis][n_t]
    const double* theta;
    const double* gb;     // [1]
    double* jpart;        // [grid][kNBasis]
    // per row the float4 columns [lo, hi) holding its non-zero responses,
    // or null (read every column)
    const int* rowband;
    double* out_grad;     // [7]
    double pull_mean[kNTheta];
    double pull_sigma[kNTheta];
    Phys ph;
};

// Launchers (plain.hip)
hipError_t launch_step(const StepArgs& a, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs& a, int grid, hipStream_t s);
int adjoint_grid(int n_t);

}  // namespace nr
