// Effective sample size of the reweighted Monte Carlo per observed bin,
// ESS_j = (sum_l N_lj w_l)^2 / sum_l N_lj w_l^2 with N_lj = R_lj n_l the MC
// events of true recoil bin l seen in bin j (n_l events generated in row l).
// A diagnostic of where reweighting runs short of MC support (Sec. VI.A:
// large weights where the SM spectrum is small, at low recoil energy for a
// magnetic moment).  One streaming pass over R accumulates both sums.
#include "common.h"
#include "ess.h"

namespace nr {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline float4 ld_stream4(const float4* p) {
    const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

constexpr int kEssThreads = 512;
constexpr int kEssWaves = kEssThreads / 64;
constexpr int kEssCols = kEssWaves * 256;  // columns per tile: 256 per wave
constexpr int kEssUnroll = 8;              // rows in flight per wave
constexpr int kEssMaxRows = 2048;

// Tile (rb, cc): rows [rb*rows, +rows), columns [cc*2048, +2048) of R.  Each
// wave takes 256 columns of every row, so the work-group reads each row as
// one 8 KB run, kEssUnroll rows in flight per wave; u_l = n_l w_l and
// u2_l = n_l w_l^2 in LDS; FP64 products and sums.  A lane's four columns'
// two partial sums go to colpart[0] and colpart[1] directly (no other wave
// touches its columns).
__global__ __launch_bounds__(kEssThreads) void k_ess_fold(EssArgs a) {
    __shared__ double u1[kEssMaxRows], u2[kEssMaxRows];
    const int rb = blockIdx.x % a.n_rb, cc = blockIdx.x / a.n_rb;
    const int row0 = rb * a.rows_per_wg;
    int nrows = a.n_t - row0;
    if (nrows > a.rows_per_wg) nrows = a.rows_per_wg;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int q = tid; q < nrows; q += kEssThreads) {
        const double w = a.w[row0 + q], n = a.nev[row0 + q];
        u1[q] = n * w;
        u2[q] = n * w * w;
    }
    __syncthreads();
    const int ld4 = a.ldr >> 2;
    const int c4 = cc * (kEssCols / 4) + wave * 64 + lane;
    if (c4 >= ld4) return;
    double s[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    const float4* __restrict__ Rp =
        reinterpret_cast<const float4*>(a.R) + (size_t)row0 * ld4 + c4;
    auto acc = [&](const float4 x, int r) {
        const double v = u1[r], v2 = u2[r];
        s[0][0] = fma((double)x.x, v, s[0][0]);
        s[0][1] = fma((double)x.y, v, s[0][1]);
        s[0][2] = fma((double)x.z, v, s[0][2]);
        s[0][3] = fma((double)x.w, v, s[0][3]);
        s[1][0] = fma((double)x.x, v2, s[1][0]);
        s[1][1] = fma((double)x.y, v2, s[1][1]);
        s[1][2] = fma((double)x.z, v2, s[1][2]);
        s[1][3] = fma((double)x.w, v2, s[1][3]);
    };
    int r = 0;
    for (; r + kEssUnroll <= nrows; r += kEssUnroll) {
        float4 x[kEssUnroll];
#pragma unroll
        for (int q = 0; q < kEssUnroll; ++q) x[q] = ld_stream4(Rp + (size_t)(r + q) * ld4);
#pragma unroll
        for (int q = 0; q < kEssUnroll; ++q) acc(x[q], r + q);
    }
    for (; r < nrows; ++r) acc(ld_stream4(Rp + (size_t)r * ld4), r);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a.colpart[((size_t)k * a.n_rb + rb) * a.ldr + 4 * c4 + i] = s[k][i];
}

// ESS_j from the row-tile partials; 0 for a bin that no weighted event
// reaches.  64 columns per work-group, 8 waves each adding every 8th
// row-tile partial of its columns (all its loads in flight together), the
// eight sums then combined in wave order: a fixed order, so the result is
// reproducible.
constexpr int kEssFinCols = 64;
constexpr int kEssFinParts = 8;

__global__ __launch_bounds__(kEssFinCols * kEssFinParts) void k_ess_finish(EssArgs a) {
    __shared__ double part[2][kEssFinParts][kEssFinCols];
    const int ci = threadIdx.x % kEssFinCols, q = threadIdx.x / kEssFinCols;
    const int col = blockIdx.x * kEssFinCols + ci;
    double s1 = 0.0, s2 = 0.0;
    if (col < a.n_reco) {
        for (int rb = q; rb < a.n_rb; rb += kEssFinParts) {
            s1 += a.colpart[(size_t)rb * a.ldr + col];
            s2 += a.colpart[((size_t)a.n_rb + rb) * a.ldr + col];
        }
    }
    part[0][q][ci] = s1;
    part[1][q][ci] = s2;
    __syncthreads();
    if (q == 0 && col < a.n_reco) {
        double t1 = 0.0, t2 = 0.0;
#pragma unroll
        for (int k = 0; k < kEssFinParts; ++k) {
            t1 += part[0][k][ci];
            t2 += part[1][k][ci];
        }
        a.out[col] = t2 > 0.0 ? t1 * t1 / t2 : 0.0;
    }
}

}  // namespace

int ess_col_tiles(int ldr) { return (ldr / 4 + kEssCols / 4 - 1) / (kEssCols / 4); }

hipError_t launch_ess(const EssArgs& a, hipStream_t s) {
    if (a.rows_per_wg <= 0 || a.rows_per_wg > kEssMaxRows || a.n_rb <= 0 ||
        a.n_cc != ess_col_tiles(a.ldr) ||
        (size_t)a.n_rb * a.rows_per_wg < (size_t)a.n_t)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ess_fold, dim3(a.n_rb * a.n_cc), dim3(kEssThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ess_finish, dim3((a.n_reco + kEssFinCols - 1) / kEssFinCols),
                       dim3(kEssFinCols * kEssFinParts), 0, s, a);
    return hipGetLastError();
}

}  // namespace nr
