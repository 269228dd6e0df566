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
constexpr int kEssCols = 256;
constexpr int kEssUnroll = 4;
constexpr int kEssMaxRows = 2048;

// Tile (rb, cc): rows [rb*rows, +rows), columns [cc*256, +256) of R, four
// rows in flight per wave; u_l = n_l w_l and u2_l = n_l w_l^2 in LDS; FP64
// products and sums; the two column partial sums of the tile go to
// colpart[0] and colpart[1].
__global__ __launch_bounds__(kEssThreads) void k_ess_fold(EssArgs a) {
    __shared__ double u1[kEssMaxRows], u2[kEssMaxRows];
    __shared__ double red[2][kEssWaves][kEssCols + 1];
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
    const int c4 = cc * 64 + lane;
    double s[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    if (c4 < ld4) {
        const float4* __restrict__ Rp =
            reinterpret_cast<const float4*>(a.R) + (size_t)row0 * ld4 + c4;
        int r = wave;
        for (; r + kEssWaves * (kEssUnroll - 1) < nrows; r += kEssWaves * kEssUnroll) {
            float4 x[kEssUnroll];
#pragma unroll
            for (int q = 0; q < kEssUnroll; ++q)
                x[q] = ld_stream4(Rp + (size_t)(r + q * kEssWaves) * ld4);
#pragma unroll
            for (int q = 0; q < kEssUnroll; ++q) {
                const double v = u1[r + q * kEssWaves], v2 = u2[r + q * kEssWaves];
                s[0][0] = fma((double)x[q].x, v, s[0][0]);
                s[0][1] = fma((double)x[q].y, v, s[0][1]);
                s[0][2] = fma((double)x[q].z, v, s[0][2]);
                s[0][3] = fma((double)x[q].w, v, s[0][3]);
                s[1][0] = fma((double)x[q].x, v2, s[1][0]);
                s[1][1] = fma((double)x[q].y, v2, s[1][1]);
                s[1][2] = fma((double)x[q].z, v2, s[1][2]);
                s[1][3] = fma((double)x[q].w, v2, s[1][3]);
            }
        }
        for (; r < nrows; r += kEssWaves) {
            const float4 z = ld_stream4(Rp + (size_t)r * ld4);
            const double v = u1[r], v2 = u2[r];
            s[0][0] = fma((double)z.x, v, s[0][0]);
            s[0][1] = fma((double)z.y, v, s[0][1]);
            s[0][2] = fma((double)z.z, v, s[0][2]);
            s[0][3] = fma((double)z.w, v, s[0][3]);
            s[1][0] = fma((double)z.x, v2, s[1][0]);
            s[1][1] = fma((double)z.y, v2, s[1][1]);
            s[1][2] = fma((double)z.z, v2, s[1][2]);
            s[1][3] = fma((double)z.w, v2, s[1][3]);
        }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[k][wave][4 * lane + i] = s[k][i];
    __syncthreads();
    if (tid < 2 * kEssCols) {
        const int k = tid / kEssCols, ci = tid % kEssCols;
        const int col = cc * kEssCols + ci;
        if (col < a.ldr) {
            double t = 0.0;
            for (int w = 0; w < kEssWaves; ++w) t += red[k][w][ci];
            a.colpart[((size_t)k * a.n_rb + rb) * a.ldr + col] = t;
        }
    }
}

// ESS_j from the row-tile partials (added in row-tile order); 0 for a bin
// that no weighted event reaches.
__global__ __launch_bounds__(256) void k_ess_finish(EssArgs a) {
    const int col = blockIdx.x * 256 + threadIdx.x;
    if (col >= a.n_reco) return;
    double s1 = 0.0, s2 = 0.0;
    for (int rb = 0; rb < a.n_rb; ++rb) {
        s1 += a.colpart[(size_t)rb * a.ldr + col];
        s2 += a.colpart[((size_t)a.n_rb + rb) * a.ldr + col];
    }
    a.out[col] = s2 > 0.0 ? s1 * s1 / s2 : 0.0;
}

}  // namespace

hipError_t launch_ess(const EssArgs& a, hipStream_t s) {
    if (a.rows_per_wg <= 0 || a.rows_per_wg > kEssMaxRows || a.n_rb <= 0 ||
        a.n_cc != (a.ldr / 4 + 63) / 64 ||
        (size_t)a.n_rb * a.rows_per_wg < (size_t)a.n_t)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ess_fold, dim3(a.n_rb * a.n_cc), dim3(kEssThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ess_finish, dim3((a.n_reco + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace nr
