// Effective-sample-size diagnostic (ess.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace nr {

struct EssArgs {
    const float* R;       // [n_t][ldr]
    int ldr, n_t, n_reco;
    const double* w;      // [n_t] weights of the point
    const double* nev;    // [n_t] MC events generated per true recoil row
    double* colpart;      // [2][n_rb][ldr]
    int rows_per_wg, n_rb, n_cc;
    double* out;          // [n_reco] ESS_j
};

// Column tiles of the ESS fold for a response row of ldr floats (n_cc).
int ess_col_tiles(int ldr);

hipError_t launch_ess(const EssArgs& a, hipStream_t s);

}  // namespace nr
