// Single-point path on gfx950: E-integral, weights, HBM-streaming fold,
// Poisson likelihood reduction, and the adjoint of the fold.
#include "common.h"

#include <cmath>

namespace nr {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// 16-byte streaming load (R is read once per evaluation).
__device__ inline float4 ld_stream(const float4* p) {
    const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Flavour-weighted couplings for one node (Sec. II.B, Eq. (g_tilde)):
// A = sum_a P_a gL_a^2, B = sum_a P_a gR_a^2, C = sum_a P_a gL_a gR_a.
struct NodeCoef {
    double a0, a1, a2, am;
};

// nu-weighted recoil polynomial of one energy node.  The flavour sum of
// Eq. (sm_cross_section) with the couplings of Eq. (xs_nsi) plus the
// magnetic term of Eq. (xs_mm), Eq. (xs_total), written as a Laurent
// polynomial in T:  a0 + a1 T + a2 T^2 + am / T  (weak prefactor = 1).
__device__ inline NodeCoef node_coef(double iE, double nu, double pe,
                                     const double* th, const Phys& ph) {
    const double Pe = pe;
    const double Pm = (1.0 - pe) * (1.0 - ph.tau_frac);
    const double Pt = (1.0 - pe) * ph.tau_frac;
    const double gle = ph.gLe + th[0], gre = ph.gR + th[1];
    const double glm = ph.gLm, grm = ph.gR;
    const double glt = ph.gLm + th[2], grt = ph.gR + th[3];
    const double A = Pe * gle * gle + Pm * glm * glm + Pt * glt * glt;
    const double B = Pe * gre * gre + Pm * grm * grm + Pt * grt * grt;
    const double C = Pe * gle * gre + Pm * glm * grm + Pt * glt * grt;
    const double mm = ph.cmm * th[4] * (Pe + Pm + Pt);
    NodeCoef c;
    c.a0 = nu * (A + B - mm * iE);
    c.a1 = nu * (-2.0 * B * iE - C * ph.me * iE * iE);
    c.a2 = nu * (B * iE * iE);
    c.am = nu * mm;
    return c;
}

// ---------------------------------------------------------------- a1
// Eq. (fT): every wave takes one work unit (64 recoil rows x <= 64 energy
// nodes of one source).  Lane i first builds node i's coefficients; the
// coefficients are then broadcast from LDS while each lane, owning one
// recoil row, evaluates nu_j dsigma/dT(E_j, T_l) for every node of the unit
// and accumulates in FP64.  Pairs beyond the kinematic limit are masked
// with the host-computed first reachable node jmin(k, l).
__global__ __launch_bounds__(256) void k_eint(EintArgs a) {
    __shared__ double4 cs[4][kUnitNodes];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int u = blockIdx.x * 4 + wave;
    if (u >= a.n_units) return;
    const EUnit un = a.units[u];
    double th[kNTheta];
#pragma unroll
    for (int i = 0; i < kNTheta; ++i) th[i] = a.theta[i];
    const double f = a.srcGroup[un.src] ? th[5] : 1.0;
    if (lane < un.cnt) {
        const int j = un.j0 + lane;
        NodeCoef c = node_coef(a.nodeIE[j], a.nodeW[j] * f, a.nodePe[j], th,
                               a.ph);
        cs[wave][lane] = make_double4(c.a0, c.a1, c.a2, c.am);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int l = un.block * kRowsPerBlock + lane;
    const bool rowok = l < a.n_t;
    const double T = rowok ? a.tc[l] : 1.0;
    const double iT = 1.0 / T;
    const int jm = rowok ? a.jmin[(size_t)un.src * a.n_t + l] : 0x7fffffff;
    int nmask = un.jfull - un.j0;
    nmask = nmask < 0 ? 0 : (nmask > un.cnt ? un.cnt : nmask);
    double acc = 0.0;
    int i = 0;
    for (; i < nmask; ++i) {
        const double4 c = cs[wave][i];
        double t = fma(T, fma(T, c.z, c.y), c.x);
        t = fma(iT, c.w, t);
        acc += (un.j0 + i >= jm) ? t : 0.0;
    }
    if (rowok) {
        for (; i < un.cnt; ++i) {
            const double4 c = cs[wave][i];
            acc = fma(T, fma(T, c.z, c.y), acc + c.x);
            acc = fma(iT, c.w, acc);
        }
    }
    a.part[(size_t)u * kRowsPerBlock + lane] = rowok ? acc : 0.0;
}

// Sum of the unit partials of every recoil row of a 64-row block,
// S_theta(T_l) = sum_u part[u][l].  Sixteen waves take every sixteenth unit
// (four loads in flight each) and the per-wave sums are added in a fixed
// order, so the result is bitwise reproducible and identical in both uses
// below.
constexpr int kRowSumThreads = 1024;
constexpr int kRowSumWaves = kRowSumThreads / 64;

__device__ inline double block_row_sum(const double* __restrict__ part,
                                       const int* __restrict__ ustart,
                                       int blk, double* sh) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int u0 = ustart[blk], u1 = ustart[blk + 1];
    double s = 0.0;
    int u = u0 + wave;
    for (; u + 3 * kRowSumWaves < u1; u += 4 * kRowSumWaves) {
        const double p0 = part[(size_t)u * kRowsPerBlock + lane];
        const double p1 = part[(size_t)(u + kRowSumWaves) * kRowsPerBlock + lane];
        const double p2 = part[(size_t)(u + 2 * kRowSumWaves) * kRowsPerBlock + lane];
        const double p3 = part[(size_t)(u + 3 * kRowSumWaves) * kRowsPerBlock + lane];
        s += p0;
        s += p1;
        s += p2;
        s += p3;
    }
    for (; u < u1; u += kRowSumWaves) s += part[(size_t)u * kRowsPerBlock + lane];
    sh[wave * kRowsPerBlock + lane] = s;
    __syncthreads();
    double t = 0.0;
    if (wave == 0)
        for (int w = 0; w < kRowSumWaves; ++w) t += sh[w * kRowsPerBlock + lane];
    return t;  // valid in wave 0
}

__global__ __launch_bounds__(kRowSumThreads) void k_spectrum_reduce(
    const double* __restrict__ part, const int* __restrict__ ustart, int n_t,
    double* __restrict__ out) {
    __shared__ double sh[kRowSumWaves * kRowsPerBlock];
    const int blk = blockIdx.x;
    const double s = block_row_sum(part, ustart, blk, sh);
    const int l = blk * kRowsPerBlock + (threadIdx.x & 63);
    if (threadIdx.x < 64 && l < n_t) out[l] = s;
}

// a2: weights w_l = S_theta(T_l) / S_SM(T_l) (Eqs. (fT_norm),
// (reweight_factor)), w_l := 1 where S_SM = 0, and the fold vector
// v_l = m_l w_l.  S_theta is summed exactly as the SM reference was, so
// w = 1 exactly at theta_SM.
__global__ __launch_bounds__(kRowSumThreads) void k_weights(WeightArgs a) {
    __shared__ double sh[kRowSumWaves * kRowsPerBlock];
    const int blk = blockIdx.x;
    const double s = block_row_sum(a.part, a.ustart, blk, sh);
    const int l = blk * kRowsPerBlock + (threadIdx.x & 63);
    if (threadIdx.x < 64 && l < a.n_t) {
        const double ssm = a.ssm[l];
        const double w = ssm > 0.0 ? s / ssm : 1.0;
        if (a.out_w) a.out_w[l] = w;
        a.v[l] = a.mrow[l] * w;
    }
}

// ------------------------------------------------------------- a3 - a5
constexpr int kFoldThreads = 512;          // 8 waves
constexpr int kFoldWaves = kFoldThreads / 64;
constexpr int kFoldCols = 256;             // 64 lanes x float4
constexpr int kFoldUnroll = 8;
constexpr int kFoldMaxRows = 2048;


// Fold through the response (Eqs. (Rij), (fNp_reweight), (mu_total)).
// Work-group (rb, cc) streams rows [rb*rows, +rows) and columns
// [cc*256, +256) of R with 16-byte streaming loads, eight rows in flight per
// wave (the first eight are issued before the weights are staged); the
// per-row weights v_l = m_l w_l sit in LDS.  R is FP32 in HBM; products and
// sums are FP64, which the full-rate FP64 vector units of gfx950 absorb at
// no cost to this bandwidth-bound loop.  The work-group writes its column
// partial sums; no cross-work-group synchronisation happens here (the
// partial sums are read by the next kernel).
__global__ __launch_bounds__(kFoldThreads) void k_fold(FoldArgs a) {
    __shared__ double vs[kFoldMaxRows];
    __shared__ double red[kFoldWaves][kFoldCols + 1];
    const int rb = blockIdx.x, cc = blockIdx.y;
    const int row0 = rb * a.rows_per_wg;
    int nrows = a.n_t - row0;
    if (nrows > a.rows_per_wg) nrows = a.rows_per_wg;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;

    const int ld4 = a.ldr >> 2;
    const int c4 = cc * 64 + lane;
    const bool colok = c4 < ld4;
    const float4* __restrict__ Rp =
        reinterpret_cast<const float4*>(a.R) + (size_t)row0 * ld4 + c4;
    constexpr int U = kFoldUnroll;
    float4 x[U];
    int r = wave;
    bool full = colok && r + kFoldWaves * (U - 1) < nrows;
    if (full) {
#pragma unroll
        for (int q = 0; q < U; ++q)
            x[q] = ld_stream(Rp + (size_t)(r + q * kFoldWaves) * ld4);
    }
    for (int q = tid; q < nrows; q += kFoldThreads) vs[q] = a.v[row0 + q];
    __syncthreads();
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    while (full) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const double v = vs[r + q * kFoldWaves];
            acc0 = fma((double)x[q].x, v, acc0);
            acc1 = fma((double)x[q].y, v, acc1);
            acc2 = fma((double)x[q].z, v, acc2);
            acc3 = fma((double)x[q].w, v, acc3);
        }
        r += kFoldWaves * U;
        full = r + kFoldWaves * (U - 1) < nrows;
        if (full) {
#pragma unroll
            for (int q = 0; q < U; ++q)
                x[q] = ld_stream(Rp + (size_t)(r + q * kFoldWaves) * ld4);
        }
    }
    if (colok) {
        for (; r < nrows; r += kFoldWaves) {
            const float4 z = ld_stream(Rp + (size_t)r * ld4);
            const double v = vs[r];
            acc0 = fma((double)z.x, v, acc0);
            acc1 = fma((double)z.y, v, acc1);
            acc2 = fma((double)z.z, v, acc2);
            acc3 = fma((double)z.w, v, acc3);
        }
    }
    red[wave][4 * lane + 0] = acc0;
    red[wave][4 * lane + 1] = acc1;
    red[wave][4 * lane + 2] = acc2;
    red[wave][4 * lane + 3] = acc3;
    __syncthreads();
    if (tid < kFoldCols) {
        const int col = cc * kFoldCols + tid;
        if (col < a.ldr) {
            double s = 0.0;
            for (int w = 0; w < kFoldWaves; ++w) s += red[w][tid];
            a.colpart[(size_t)rb * a.ldr + col] = s;
        }
    }
}

// Poisson likelihood (Eq. (logL)) from the fold partials.  Work-group cc
// owns 256 columns; four threads per column add the row-block partials in a
// fixed order, then mu_j, the deviance mu - n + n ln(n/mu) and
// a_j = d(-2lnL)/d mu_j.  The chunk sums meet in the last work-group
// (arrival counter; only the writing wave fences), which adds the data
// constant and the pulls.  Deterministic: no float atomics.
constexpr int kFinThreads = 1024;

__global__ __launch_bounds__(kFinThreads) void k_fold_finish(FoldArgs a) {
    __shared__ double ps[4][kFoldCols];
    __shared__ double dred[kFinThreads / 64];
    __shared__ double gred[kFinThreads / 64];
    __shared__ int s_last;
    const int cc = blockIdx.x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ci = tid & (kFoldCols - 1), qd = tid >> 8;
    const int col = cc * kFoldCols + ci;
    double s = 0.0;
    if (col < a.n_reco) {
        int q = qd;
        for (; q + 12 < a.n_rb; q += 16) {
            const double v0 = a.colpart[(size_t)q * a.ldr + col];
            const double v1 = a.colpart[(size_t)(q + 4) * a.ldr + col];
            const double v2 = a.colpart[(size_t)(q + 8) * a.ldr + col];
            const double v3 = a.colpart[(size_t)(q + 12) * a.ldr + col];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; q < a.n_rb; q += 4) s += a.colpart[(size_t)q * a.ldr + col];
    }
    ps[qd][ci] = s;
    __syncthreads();
    double dev = 0.0, gb = 0.0;
    if (qd == 0 && col < a.n_reco) {
        const double fold = ps[0][ci] + ps[1][ci] + ps[2][ci] + ps[3][ci];
        const double bj = a.b[col];
        const double mu = fold + a.theta[6] * bj;
        const double nj = a.n[col];
        if (a.out_mu) a.out_mu[col] = mu;
        if (nj > 0.0)
            dev = mu > 0.0 ? (mu - nj + nj * log(nj / mu)) : INFINITY;
        else
            dev = mu;
        const double aj = 2.0 * (1.0 - nj / mu);
        if (a.out_a) a.out_a[col] = aj;
        gb = aj * bj;
    } else if (qd == 0 && col < a.ldr && a.out_a) {
        a.out_a[col] = 0.0;
    }
    dev = wave_sum(dev);
    gb = wave_sum(gb);
    if (lane == 0) {
        dred[wave] = dev;
        gred[wave] = gb;
    }
    __syncthreads();
    if (wave == 0) {
        double d = 0.0, g = 0.0;
        if (lane == 0) {
            for (int w = 0; w < kFinThreads / 64; ++w) {
                d += dred[w];
                g += gred[w];
            }
            a.chunk_dev[cc] = d;
            a.chunk_gb[cc] = g;
        }
        __threadfence();
        if (lane == 0) {
            const unsigned prev = atomicAdd(&a.ctr[0], 1u);
            s_last = prev == (unsigned)(a.n_cc - 1);
        }
    }
    __syncthreads();
    if (!s_last || wave != 0) return;
    __threadfence();
    if (lane == 0) {
        double d = 0.0, g = 0.0;
        for (int q = 0; q < a.n_cc; ++q) {
            d += a.chunk_dev[q];
            g += a.chunk_gb[q];
        }
        double pulls = 0.0;
        for (int i = 0; i < kNTheta; ++i)
            if (a.pull_sigma[i] > 0.0) {
                const double z = (a.theta[i] - a.pull_mean[i]) / a.pull_sigma[i];
                pulls += z * z;
            }
        a.out_nll[0] = 2.0 * d + 2.0 * a.cdata + pulls;
        if (a.out_gb) a.out_gb[0] = g;
        a.ctr[0] = 0u;
    }
}

// ------------------------------------------------------------- adjoint
constexpr int kAdjThreads = 256;
constexpr int kAdjMaxLd = 4096;

// Coefficients of the 20 basis spectra and their theta-derivatives.  The
// basis (per group g = non-8B / 8B, per flavour e, mu, tau) is
// I_{g,a,LL} = sum nu P_a, I_{g,a,RR} = sum nu P_a y^2, I_{g,a,LR} =
// sum nu P_a x, I_{g,D} = sum nu (sum_a P_a)(1/T - 1/E), so that
// S_theta = sum_b c_b(theta) I_b  exactly (Eqs. (fT), (xs_total)).
__device__ inline void basis_dcoef(const double* th, const Phys& ph,
                                   double dc[kNTheta][kNBasis]) {
    for (int i = 0; i < kNTheta; ++i)
        for (int b = 0; b < kNBasis; ++b) dc[i][b] = 0.0;
    const double gle = ph.gLe + th[0], gre = ph.gR + th[1];
    const double glm = ph.gLm, grm = ph.gR;
    const double glt = ph.gLm + th[2], grt = ph.gR + th[3];
    for (int g = 0; g < 2; ++g) {
        const double f = g ? th[5] : 1.0;
        const int o = g * 10;
        dc[0][o + 0] = f * 2.0 * gle;
        dc[0][o + 2] = -f * gre;
        dc[1][o + 1] = f * 2.0 * gre;
        dc[1][o + 2] = -f * gle;
        dc[2][o + 6] = f * 2.0 * glt;
        dc[2][o + 8] = -f * grt;
        dc[3][o + 7] = f * 2.0 * grt;
        dc[3][o + 8] = -f * glt;
        dc[4][o + 9] = f * ph.cmm;
        if (g == 1) {
            dc[5][o + 0] = gle * gle;
            dc[5][o + 1] = gre * gre;
            dc[5][o + 2] = -gle * gre;
            dc[5][o + 3] = glm * glm;
            dc[5][o + 4] = grm * grm;
            dc[5][o + 5] = -glm * grm;
            dc[5][o + 6] = glt * glt;
            dc[5][o + 7] = grt * grt;
            dc[5][o + 8] = -glt * grt;
            dc[5][o + 9] = ph.cmm * th[4];
        }
    }
}

// Adjoint of the fold: u_l = sum_j R_lj a_j with a_j = d(-2lnL)/d mu_j
// (one wave per row, 16-byte loads, wave-shuffle reduction), then the
// contraction with the weight derivatives
// d v_l / d theta_i = m_l / S_SM(T_l) * sum_b dc_ib I_b(T_l).
__global__ __launch_bounds__(kAdjThreads) void k_adjoint(AdjArgs a) {
    __shared__ double as[kAdjMaxLd];
    __shared__ double jsh[kAdjThreads / 64][kNBasis];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ld4 = a.ldr >> 2;
    const bool lds = a.ldr <= kAdjMaxLd;
    if (lds)
        for (int c = tid; c < a.ldr; c += kAdjThreads) as[c] = a.a[c];
    __syncthreads();
    const double* av = lds ? as : a.a;
    double J = 0.0;  // lane b < kNBasis holds J_b of this wave
    const int nwaves = gridDim.x * (kAdjThreads / 64);
    for (int l = blockIdx.x * (kAdjThreads / 64) + wave; l < a.n_t;
         l += nwaves) {
        const float4* Rp = reinterpret_cast<const float4*>(a.R) + (size_t)l * ld4;
        double s = 0.0;
        for (int c = lane; c < ld4; c += 64) {
            const float4 x = ld_stream(Rp + c);
            s = fma((double)x.x, av[4 * c + 0], s);
            s = fma((double)x.y, av[4 * c + 1], s);
            s = fma((double)x.z, av[4 * c + 2], s);
            s = fma((double)x.w, av[4 * c + 3], s);
        }
        const double u = wave_sum(s);
        const double ssm = a.ssm[l];
        if (ssm > 0.0 && lane < kNBasis)
            J += u * (a.mrow[l] / ssm) * a.basis[(size_t)lane * a.n_t + l];
    }
    if (lane < kNBasis) jsh[wave][lane] = J;
    __syncthreads();
    if (tid < kNBasis) {
        double s = 0.0;
        for (int w = 0; w < kAdjThreads / 64; ++w) s += jsh[w][tid];
        a.jpart[(size_t)blockIdx.x * kNBasis + tid] = s;
    }
}

// Sum of the per-work-group basis contractions (fixed order) and the
// gradient: grad_i = sum_b dc_ib(theta) J_b + [i = f_bkg] sum_j a_j b_j +
// the pull term.
constexpr int kAdjGroups = 12;

__global__ __launch_bounds__(256) void k_adjoint_finish(AdjArgs a, int grid) {
    __shared__ double jsh[kAdjGroups][kNBasis];
    __shared__ double jt[kNBasis];
    const int tid = threadIdx.x;
    if (tid < kAdjGroups * kNBasis) {
        const int b = tid % kNBasis, g = tid / kNBasis;
        double s = 0.0;
        for (int q = g; q < grid; q += kAdjGroups) s += a.jpart[(size_t)q * kNBasis + b];
        jsh[g][b] = s;
    }
    __syncthreads();
    if (tid < kNBasis) {
        double s = 0.0;
        for (int g = 0; g < kAdjGroups; ++g) s += jsh[g][tid];
        jt[tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
        double th[kNTheta];
        for (int i = 0; i < kNTheta; ++i) th[i] = a.theta[i];
        double dc[kNTheta][kNBasis];
        basis_dcoef(th, a.ph, dc);
        for (int i = 0; i < kNTheta; ++i) {
            double g = 0.0;
            for (int b = 0; b < kNBasis; ++b) g += dc[i][b] * jt[b];
            if (i == 6) g += a.gb[0];
            if (a.pull_sigma[i] > 0.0)
                g += 2.0 * (th[i] - a.pull_mean[i]) /
                     (a.pull_sigma[i] * a.pull_sigma[i]);
            a.out_grad[i] = g;
        }
    }
}

}  // namespace

hipError_t launch_eint(const EintArgs& a, hipStream_t s) {
    const int grid = (a.n_units + 3) / 4;
    hipLaunchKernelGGL(k_eint, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_spectrum_reduce(const double* part, const int* ustart,
                                  int n_t, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_spectrum_reduce, dim3((n_t + kRowsPerBlock - 1) / kRowsPerBlock),
                       dim3(kRowSumThreads), 0, s, part, ustart, n_t, out);
    return hipGetLastError();
}

hipError_t launch_weights(const WeightArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_weights, dim3((a.n_t + kRowsPerBlock - 1) / kRowsPerBlock),
                       dim3(kRowSumThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fold_stream(const FoldArgs& a, hipStream_t s) {
    if (a.rows_per_wg > kFoldMaxRows || a.rows_per_wg <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fold, dim3(a.n_rb, a.n_cc), dim3(kFoldThreads), 0, s,
                       a);
    return hipGetLastError();
}

hipError_t launch_fold_finish(const FoldArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_fold_finish, dim3(a.n_cc), dim3(kFinThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fold(const FoldArgs& a, hipStream_t s) {
    if (a.rows_per_wg > kFoldMaxRows || a.rows_per_wg <= 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fold, dim3(a.n_rb, a.n_cc), dim3(kFoldThreads), 0, s,
                       a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fold_finish, dim3(a.n_cc), dim3(kFinThreads), 0, s, a);
    return hipGetLastError();
}

int adjoint_grid(int n_t) {
    int g = (n_t + 15) / 16;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return g;
}

hipError_t launch_adjoint(const AdjArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(k_adjoint, dim3(grid), dim3(kAdjThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adjoint_finish, dim3(1), dim3(256), 0, s, a, grid);
    return hipGetLastError();
}

}  // namespace nr
