// Internal declarations shared by the HIP translation units of the library.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace nr {

constexpr int kNTheta = 7;
constexpr int kRowsPerBlock = 64;   // recoil rows per E-integral block (lanes)
constexpr int kUnitNodes = 64;      // energy nodes per E-integral work unit
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

// One E-integral work unit: a block of 64 consecutive recoil rows and up to
// 64 consecutive energy nodes of one source.  Nodes with global index
// >= jfull are reachable from every row of the block.
struct EUnit {
    int block;
    int src;
    int j0;
    int cnt;
    int jfull;
    int pad[3];
};

struct EintArgs {
    const EUnit* units;
    int n_units;
    const double* nodeIE;  // 1 / E_j
    const double* nodeW;
    const double* nodePe;
    const int* srcGroup;
    const int* jmin;      // [n_src][n_t] first reachable global node index
    const double* tc;     // [n_t] recoil-bin centres
    int n_t;
    const double* theta;  // device, 7 doubles
    Phys ph;
    double* part;         // [n_units][64]
};

struct WeightArgs {
    const double* part;   // E-integral partials
    const int* ustart;    // [n_blocks+1] first unit of each row block
    const double* ssm;    // [n_t] S_SM (device E-integral at theta_SM)
    const double* mrow;   // [n_t] row factors m_l
    int n_t;
    double* v;            // [n_t] m_l w_l
    double* out_w;        // [n_t] or null: weights w_l
};

struct FoldArgs {
    const float* R;       // [n_t][ldr]
    int ldr;              // leading dimension (floats), multiple of 4
    int n_t, n_reco;
    const double* v;      // [n_t] m_l w_l
    const double* n;      // [n_reco]
    const double* b;      // [n_reco]
    const double* theta;  // device, 7 doubles
    double* colpart;      // [n_rb][ldr]
    unsigned* ctr;        // [n_cc + 1], zero between launches
    double* chunk_dev;    // [n_cc]
    double* chunk_gb;     // [n_cc]
    double* out_nll;      // [1]
    double* out_mu;       // [n_reco] or null
    double* out_a;        // [ldr] or null: d(-2lnL)/d mu_j
    double* out_gb;       // [1] or null: sum_j a_j b_j
    double cdata;
    double pull_mean[kNTheta];
    double pull_sigma[kNTheta];
    int rows_per_wg, n_rb, n_cc;
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
    unsigned* ctr;        // [1]
    double* out_grad;     // [7]
    double pull_mean[kNTheta];
    double pull_sigma[kNTheta];
    Phys ph;
};

// Launchers (plain.hip)
hipError_t launch_eint(const EintArgs& a, hipStream_t s);
hipError_t launch_spectrum_reduce(const double* part, const int* ustart,
                                  int n_t, double* out, hipStream_t s);
hipError_t launch_weights(const WeightArgs& a, hipStream_t s);
hipError_t launch_fold(const FoldArgs& a, hipStream_t s);
hipError_t launch_fold_stream(const FoldArgs& a, hipStream_t s);
hipError_t launch_fold_finish(const FoldArgs& a, hipStream_t s);
hipError_t launch_adjoint(const AdjArgs& a, int grid, hipStream_t s);
int adjoint_grid(int n_t);

}  // namespace nr
