// Learned surrogate on gfx950: an MLP theta -> log mu_j whose forward,
// backward and optimiser steps run on BF16 matrix cores
// (v_mfma_f32_32x32x16_bf16) with FP32 accumulation.  Biases ride along as
// an extra input column fixed to one, so every layer is one GEMM.
#include "mlp.h"

#include <cmath>
#include <type_traits>

namespace nr {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TM = 128, TN = 128, TK = 32;
constexpr int kMlpThreads = 256;
constexpr int LDK = TK + 8;  // LDS row stride (bf16): rows stay 16-byte aligned

// SiLU(z) = z sigma(z) with the hardware reciprocal (one rounding of
// ~1 ulp) in place of an IEEE division: the result is rounded to BF16
// (2^-8 relative) right after, and the division's ten instructions per
// value were a third of the fused network kernel's hidden-layer time.
// z -> -inf gives z * rcp(inf) = -0, as the division would.
__device__ inline float silu(float z) {
    return z * __builtin_amdgcn_rcpf(1.f + __expf(-z));
}

// Loads one 128 x 32 operand tile (rows = m or n, k contiguous in LDS).
// kc: the operand is k-contiguous in memory (16-byte chunks along k);
// otherwise it is row-contiguous and each 16-byte chunk scatters along k.
__device__ inline void load_tile(const bf16* __restrict__ P, long s_row,
                                 long s_k, int rows, int K, int r0, int k0,
                                 uint4 reg[2]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int c = tid + i * kMlpThreads;  // 0..511 chunks of 8
        int r, k;
        if (s_k == 1) {
            r = c >> 2;
            k = (c & 3) * 8;
        } else {
            k = c >> 4;
            r = (c & 15) * 8;
        }
        const int gr = r0 + r, gk = k0 + k;
        const bool ok = gr < rows && gk < K;
        reg[i] = ok ? *reinterpret_cast<const uint4*>(P + (long)gr * s_row + (long)gk * s_k)
                    : make_uint4(0u, 0u, 0u, 0u);
    }
}

__device__ inline void store_tile(bf16 (*S)[LDK], long s_k, const uint4 reg[2]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const int c = tid + i * kMlpThreads;
        if (s_k == 1) {
            const int r = c >> 2, k = (c & 3) * 8;
            *reinterpret_cast<uint4*>(&S[r][k]) = reg[i];
        } else {
            const int k = c >> 4, r = (c & 15) * 8;
            const bf16* v = reinterpret_cast<const bf16*>(&reg[i]);
#pragma unroll
            for (int e = 0; e < 8; ++e) S[r + e][k] = v[e];
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(kMlpThreads) void k_mlp_gemm(MlpGemm g) {
    __shared__ bf16 As[TM][LDK];
    __shared__ bf16 Bs[TN][LDK];
    __shared__ double red[4];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int li = lane & 31, lh = lane >> 5;
    const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
    // A tile rows are m (stride sam along m, sak along k); B tile rows are n
    const long a_row = g.sam, a_k = g.sak;
    const long b_row = g.sbn, b_k = g.sbk;

    f32x16 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    // this work-group's range of k (all of it unless K is split)
    const int kb = g.k_chunk ? (int)blockIdx.z * g.k_chunk : 0;
    const int ke = g.k_chunk ? min(g.K, kb + g.k_chunk) : g.K;
    uint4 ra[2], rb[2];
    load_tile(g.A, a_row, a_k, g.M, ke, m0, kb, ra);
    load_tile(g.B, b_row, b_k, g.N, ke, n0, kb, rb);
    for (int k0 = kb; k0 < ke; k0 += TK) {
        __syncthreads();
        store_tile(As, a_k, ra);
        store_tile(Bs, b_k, rb);
        __syncthreads();
        if (k0 + TK < ke) {
            load_tile(g.A, a_row, a_k, g.M, ke, m0, k0 + TK, ra);
            load_tile(g.B, b_row, b_k, g.N, ke, n0, k0 + TK, rb);
        }
#pragma unroll
        for (int ks = 0; ks < TK; ks += 16) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[x] = *reinterpret_cast<const bf16x8*>(&As[wm * 64 + x * 32 + li][ks + 8 * lh]);
                b[x] = *reinterpret_cast<const bf16x8*>(&Bs[wn * 64 + x * 32 + li][ks + 8 * lh]);
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[x], b[y], acc[x][y], 0, 0, 0);
        }
    }

    // Output (i, j) of a 32x32 block: lane j + 32 * ((i / 4) % 2),
    // register (i / 8) * 4 + i % 4.
    double lsum = 0.0;
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int i = wm * 64 + bi * 32 + (r >> 2) * 8 + lh * 4 + (r & 3);
            const int m = m0 + i;
#pragma unroll
            for (int bj = 0; bj < 2; ++bj) {
                const int n = n0 + wn * 64 + bj * 32 + li;
                if (m >= g.M || n >= g.N) continue;
                const float v = acc[bi][bj][r];
                if (MODE == kMlpStore32) {
                    g.C32[(long)blockIdx.z * g.c_split + (long)m * g.ldc + n] = v;
                } else if (MODE == kMlpSilu) {
                    g.C32[(long)m * g.ldc + n] = v;
                    g.C16[(long)m * g.ldc16 + n] = (bf16)silu(v);
                } else if (MODE == kMlpMse) {
                    const float rr = v - g.aux[(long)m * g.ldaux + n];
                    g.C16[(long)m * g.ldc16 + n] = (bf16)(g.scale * 2.f * rr);
                    lsum += (double)rr * rr;
                } else if (MODE == kMlpDSilu) {
                    const float z = g.aux[(long)m * g.ldaux + n];
                    const float sg = 1.f / (1.f + __expf(-z));
                    g.C16[(long)m * g.ldc16 + n] = (bf16)(v * sg * (1.f + z * (1.f - sg)));
                } else if (MODE == kMlpLogMu) {
                    g.C32[(long)m * g.ldc + n] = fmaf(g.stdv[n], v, g.mean[n]);
                }
            }
        }
    }
    if (MODE == kMlpMse) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
        if (lane == 0) red[wave] = lsum;
        __syncthreads();
        if (tid == 0)
            g.tile_loss[blockIdx.y * gridDim.x + blockIdx.x] =
                red[0] + red[1] + red[2] + red[3];
    }
}

// Inference output layer fused with the Poisson likelihood: per point m and
// bin n, ln mu = mean_n + std_n (W h_m)_n (FP32, as the log-mu output forms
// it), mu = exp(ln mu), and the point's sum over all bins of mu - n_n ln mu
// (FP64; the data terms lnGamma(n + 1) are added by the finishing kernel).
// One work-group per 128 points and group of bins (gridDim.y groups, so
// that small batches still fill the chip), persistent over its bins: the
// points' hidden activations (all of K <= 272) stay in LDS for the launch,
// and each wave takes 64 bins of every 256-bin step, with the weights of
// those bins loaded straight from memory (L2-resident) into the registers
// that feed the matrix instruction, four K-steps ahead in a ring that runs
// on into the next step (its first loads are in flight while the wave forms
// this step's exponentials).  Each activation fragment read from LDS feeds
// two matrix instructions (136 per step, no barrier).  The bins are the
// instruction's row operand and the points its column operand, so a lane
// holds 16 bins of one point in each 32 x 32 block (lane = point + 32 *
// half, register r = bin (r / 4) * 8 + half * 4 + r % 4) and the sum over
// bins stays in registers until the end.
constexpr int kNllKS = 17;                  // K steps of 16: K <= 272
constexpr int kNllLda = kNllKS * 16 + 8;    // A row stride in LDS (bf16)
constexpr int kOutBins = 64;                // bins per wave and step
constexpr int kOutStep = 4 * kOutBins;      // bins per work-group and step
constexpr int kOutRing = 4;                 // weight K-steps in flight

// One hidden layer of the fused inference kernel, in place on the LDS
// activation tile: wave w forms outputs [64 w, 64 w + 64) of all 128 points
// (weights of its outputs as the row operand, straight from L2 into
// registers four K-steps ahead; activations as the column operand from
// LDS), then, once every wave has read the layer's input, writes SiLU of
// them back as BF16.  A lane holds four consecutive outputs of one point
// per register quad, stored as one 8-byte write.  The products and their
// K order are those of the unfused layer GEMM.
template <int NKS>
__device__ __forceinline__ void hidden_layer(bf16 (*As)[kNllLda], const bf16* __restrict__ W, int K,
                                    int wave, int li, int lh) {
    f32x16 acc[4][2];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[x][y][r] = 0.f;
    constexpr int D = NKS < 4 ? NKS : 4;  // weight loads in flight (K-steps)
    uint4 ring[D][2];
    // k clamped into the row: columns past K meet the tile's zero columns
    auto wload = [&](int ks, uint4 out[2]) {
        const int k = min(ks * 16 + lh * 8, K - 8);
#pragma unroll
        for (int y = 0; y < 2; ++y) {
            const int o = wave * 64 + y * 32 + li;
            out[y] = *reinterpret_cast<const uint4*>(W + (long)o * K + k);
        }
    };
#pragma unroll
    for (int ks = 0; ks < D; ++ks) wload(ks, ring[ks]);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
        const uint4 w0 = ring[ks % D][0], w1 = ring[ks % D][1];
        if (ks + D < NKS) wload(ks + D, ring[ks % D]);
        const bf16x8 b0 = *reinterpret_cast<const bf16x8*>(&w0);
        const bf16x8 b1 = *reinterpret_cast<const bf16x8*>(&w1);
#pragma unroll
        for (int x = 0; x < 4; ++x) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[x * 32 + li][ks * 16 + lh * 8]);
            acc[x][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b0, a, acc[x][0], 0, 0, 0);
            acc[x][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b1, a, acc[x][1], 0, 0, 0);
        }
    }
    __syncthreads();  // every wave has read this layer's input
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                // outputs 8 q + 4 lh + e of block y, point x * 32 + li
                bf16 v[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = (bf16)silu(acc[x][y][4 * q + e]);
                *reinterpret_cast<uint2*>(&As[x * 32 + li][wave * 64 + y * 32 + 8 * q + 4 * lh]) =
                    *reinterpret_cast<const uint2*>(v);
            }
    __syncthreads();
}

// FUSED: the kernel first forms the points' activations itself from the
// network input through the three hidden layers (the whole network in one
// launch, nothing but theta's encoding read and the partial sums written);
// otherwise it loads the last hidden layer's activations from g.A.
template <bool FUSED>
__global__ __launch_bounds__(kMlpThreads, 2) void k_mlp_nll(MlpGemm g, MlpHidden hd) {
    __shared__ bf16 As[TM][kNllLda];        // points x k
    __shared__ float2 cms[4][kOutBins];     // per wave: its bins' (mean, std)
    __shared__ double cnb[4][kOutBins];     // per wave: its bins' counts
    __shared__ double red[4][TM];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 31, lh = lane >> 5;
    const int m0 = blockIdx.x * TM;
    constexpr int CH = kNllKS * 2;          // 16-byte chunks per row
    if constexpr (FUSED) {
        // the tile: inputs in columns 0..31, the bias input (1) at column
        // kFusedHidden, zeros elsewhere
        for (int q = tid; q < TM * (kNllLda / 8); q += kMlpThreads) {
            const int row = q / (kNllLda / 8), k = (q % (kNllLda / 8)) * 8, m = m0 + row;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (k < 32 && m < g.M) v = *reinterpret_cast<const uint4*>(hd.x + (long)m * 32 + k);
            *reinterpret_cast<uint4*>(&As[row][k]) = v;
        }
        __syncthreads();
        if (tid < TM) As[tid][kFusedHidden] = (bf16)1.f;
        __syncthreads();
        hidden_layer<2>(As, hd.w[0], hd.k[0], wave, li, lh);
        hidden_layer<kNllKS>(As, hd.w[1], hd.k[1], wave, li, lh);
        hidden_layer<kNllKS>(As, hd.w[2], hd.k[2], wave, li, lh);
    } else {
        for (int q = tid; q < TM * CH; q += kMlpThreads) {
            const int row = q / CH, k = (q % CH) * 8, m = m0 + row;
            const uint4 v = (m < g.M && k < g.K)
                                ? *reinterpret_cast<const uint4*>(g.A + (long)m * g.sam + k)
                                : make_uint4(0u, 0u, 0u, 0u);
            *reinterpret_cast<uint4*>(&As[row][k]) = v;
        }
        __syncthreads();
    }
    double pp[4] = {0.0, 0.0, 0.0, 0.0};
    const int nbt = (g.N + kOutStep - 1) / kOutStep;
    const int bt0 = (int)((long)nbt * blockIdx.y / gridDim.y);
    const int bt1 = (int)((long)nbt * (blockIdx.y + 1) / gridDim.y);
    // weight fragment of K-step ks of block x of step bt: bin bt kOutStep +
    // 64 wave + 32 x + li, k = 16 ks + 8 lh, both clamped into the matrix
    // (no predicated loads): columns past K meet the tile's zero columns,
    // and a row past the bins (or past the last step, never used) feeds
    // only terms whose constants below make them zero
    auto wload = [&](int bt, int x, int ks) {
        const int k = min(ks * 16 + lh * 8, g.K - 8);
        const int n = min(bt * kOutStep + wave * kOutBins + x * 32 + li, g.N - 1);
        return *reinterpret_cast<const uint4*>(g.B + (long)n * g.sbn + k);
    };
    // lane l's bin of step bt: its constants, neutral past the bins (ln mu
    // = -200 gives mu = 0 in FP32, with n = 0: a zero term)
    float cm, cs;
    double cn;
    auto cload = [&](int bt) {
        const int nl = bt * kOutStep + wave * kOutBins + lane;
        const bool okn = nl < g.N;
        cm = okn ? g.mean[nl] : -200.f;
        cs = okn ? g.stdv[nl] : 0.f;
        cn = okn ? g.nobs[nl] : 0.0;
    };
    // the wave's 64 bins' constants, shared through its own LDS slots
    // (every lane has read the previous step's)
    auto cstore = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        cms[wave][lane] = make_float2(cm, cs);
        cnb[wave][lane] = cn;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    f32x16 acc[2][4];
    // the four points' terms of register r of block x: -n ln mu exactly in
    // FP64 (an integer count times an FP32 value), mu summed in FP32 over
    // four registers (three roundings of at most 2^-24 of the partial sum,
    // below the exponential's own error) before it joins the FP64 sum
    float ms[4] = {0.f, 0.f, 0.f, 0.f};
    auto epi_row = [&](int x, int r) {
        const int i = x * 32 + (r >> 2) * 8 + lh * 4 + (r & 3);
        const float2 c = cms[wave][i];
        const double nob = cnb[wave][i];
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const float lm = fmaf(c.y, acc[x][y][r], c.x);
            ms[y] = (r & 3) ? ms[y] + __expf(lm) : __expf(lm);
            pp[y] = fma(-nob, (double)lm, pp[y]);
            if ((r & 3) == 3) pp[y] += (double)ms[y];
        }
    };
    // Half a step: the 68 matrix instructions of block X of step bt, with
    // the exponentials of the other block (finished by the previous half
    // step) interleaved, one register row per K-step, so that the wave's
    // own vector instructions run while its matrix instructions execute.
    // Weight fragments stream through a ring kOutRing K-steps deep whose
    // stages run (bt, 0, 0..16), (bt, 1, 0..16), (bt + 1, 0, 0..16), ...
    uint4 wr[kOutRing];
    const f32x16 zero = {};
    auto half = [&](int bt, auto xc, auto ec) {
        constexpr int X = decltype(xc)::value;
        constexpr bool EPI = decltype(ec)::value;
#pragma unroll
        for (int ks = 0; ks < kNllKS; ++ks) {
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&wr[0]);
#pragma unroll
            for (int q = 0; q + 1 < kOutRing; ++q) wr[q] = wr[q + 1];
            const int ahead = ks + kOutRing;
            if (ahead < kNllKS)
                wr[kOutRing - 1] = wload(bt, X, ahead);
            else
                wr[kOutRing - 1] = X == 0 ? wload(bt, 1, ahead - kNllKS)
                                          : wload(bt + 1, 0, ahead - kNllKS);
#pragma unroll
            for (int y = 0; y < 4; ++y) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[y * 32 + li][ks * 16 + lh * 8]);
                acc[X][y] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(b, a, ks == 0 ? zero : acc[X][y],
                                                                   0, 0, 0);
            }
            if (EPI && ks < 16) epi_row(1 - X, ks);
        }
    };
    using X0 = std::integral_constant<int, 0>;
    using X1 = std::integral_constant<int, 1>;
    using Epi = std::true_type;
    using NoEpi = std::false_type;
    if (bt0 < bt1) {
#pragma unroll
        for (int q = 0; q < kOutRing; ++q) wr[q] = wload(bt0, 0, q);
        cload(bt0);
        half(bt0, X0{}, NoEpi{});
        cstore();
        half(bt0, X1{}, Epi{});              // block 0 of step bt0
        for (int bt = bt0 + 1; bt < bt1; ++bt) {
            cload(bt);
            half(bt, X0{}, Epi{});           // block 1 of step bt - 1
            cstore();
            half(bt, X1{}, Epi{});           // block 0 of step bt
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) epi_row(1, r);  // block 1 of the last step
    }
#pragma unroll
    for (int y = 0; y < 4; ++y) {
        pp[y] += __shfl_xor(pp[y], 32, 64);
        if (lh == 0) red[wave][y * 32 + li] = pp[y];
    }
    __syncthreads();
    if (tid < TM && m0 + tid < g.M)
        g.part[(long)(m0 + tid) * g.n_nt + blockIdx.y] =
            red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

__global__ void k_mlp_input(MlpInput a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.B) return;
    bool out = false;
    bf16* x = a.x + (long)p * 32;
    for (int i = 0; i < kNTheta; ++i) {
        const double t = a.theta[(long)p * kNTheta + i];
        out = out || !(t >= a.lo[i] && t <= a.hi[i]);
        x[i] = (bf16)(float)(2.0 * (t - a.lo[i]) / (a.hi[i] - a.lo[i]) - 1.0);
    }
    x[kNTheta] = (bf16)1.f;
    for (int i = kNTheta + 1; i < 32; ++i) x[i] = (bf16)0.f;
    if (a.outside) a.outside[p] = out ? 1 : 0;
}

__global__ void k_adam(AdamArgs a) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n) return;
    const float g = a.g[i];
    const float m = a.b1 * a.m[i] + (1.f - a.b1) * g;
    const float v = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
    a.m[i] = m;
    a.v[i] = v;
    const float w = a.w[i] - a.lr * (m / a.bc1) / (sqrtf(v / a.bc2) + a.eps);
    a.w[i] = w;
    a.w16[i] = (bf16)w;
}

__global__ void k_targets(TargetArgs a) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (long)a.P * a.N) return;
    const int n = (int)(i % a.N);
    const double mu = a.mu[i];
    const float lm = (float)log(mu > 1e-300 ? mu : 1e-300);
    a.t[i] = (lm - a.mean[n]) / a.stdv[n];
}

__global__ void k_ones_col(bf16* h, int B, int ld, int col) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= B) return;
    h[(long)p * ld + col] = (bf16)1.f;
    for (int c = col + 1; c < ld; ++c) h[(long)p * ld + c] = (bf16)0.f;
}

__global__ void k_transpose_bf16(const bf16* __restrict__ src, bf16* __restrict__ dst,
                                 int rows, int cols) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)rows * cols) return;
    const long r = e / cols, c = e % cols;
    dst[c * rows + r] = src[e];
}

// Sum of the K-split slabs of a GEMM, one element per thread, with the
// epilogue of the split GEMM (plain FP32 store, or SiLU').
__global__ __launch_bounds__(256) void k_mlp_ksum(KSumArgs a) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)a.M * a.N) return;
    const long m = e / a.N, n = e % a.N;
    const long o = m * a.ldc + n;
    float v = 0.f;
    for (int q = 0; q < a.n_split; ++q) v += a.part[(long)q * a.c_split + o];
    if (a.dsilu) {
        const float z = a.aux[m * a.ldaux + n];
        const float sg = 1.f / (1.f + __expf(-z));
        a.C16[m * a.ldc16 + n] = (bf16)(v * sg * (1.f + z * (1.f - sg)));
    } else {
        a.out[m * a.ldo + n] = v;
    }
}

}  // namespace

hipError_t launch_mlp_ksum(const KSumArgs& a, hipStream_t s) {
    const long n = (long)a.M * a.N;
    hipLaunchKernelGGL(k_mlp_ksum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_mlp_gemm(int mode, const MlpGemm& g, hipStream_t s) {
    if (g.M % 8 || g.N % 8 || g.K % 8 || (g.sak != 1 && g.sam != 1) ||
        (g.sbk != 1 && g.sbn != 1))
        return hipErrorInvalidValue;
    if (g.k_chunk && (mode != kMlpStore32 || g.k_chunk % TK || g.k_chunk <= 0))
        return hipErrorInvalidValue;
    const int n_split = g.k_chunk ? (g.K + g.k_chunk - 1) / g.k_chunk : 1;
    dim3 grid((g.N + TN - 1) / TN, (g.M + TM - 1) / TM, n_split);
    switch (mode) {
        case kMlpStore32: hipLaunchKernelGGL(k_mlp_gemm<kMlpStore32>, grid, dim3(kMlpThreads), 0, s, g); break;
        case kMlpSilu: hipLaunchKernelGGL(k_mlp_gemm<kMlpSilu>, grid, dim3(kMlpThreads), 0, s, g); break;
        case kMlpMse: hipLaunchKernelGGL(k_mlp_gemm<kMlpMse>, grid, dim3(kMlpThreads), 0, s, g); break;
        case kMlpDSilu: hipLaunchKernelGGL(k_mlp_gemm<kMlpDSilu>, grid, dim3(kMlpThreads), 0, s, g); break;
        case kMlpNll:
            // the whole reduction in LDS, k contiguous in both operands
            // (n_nt bin groups, at most one per 128 bins)
            if (g.K > kNllKS * 16 || g.K < 8 || g.sak != 1 || g.sbk != 1 || g.n_nt < 1 ||
                g.n_nt > (g.N + TN - 1) / TN)
                return hipErrorInvalidValue;
            hipLaunchKernelGGL(k_mlp_nll<false>, dim3((g.M + TM - 1) / TM, g.n_nt),
                               dim3(kMlpThreads), 0, s, g, MlpHidden{});
            break;
        case kMlpLogMu: hipLaunchKernelGGL(k_mlp_gemm<kMlpLogMu>, grid, dim3(kMlpThreads), 0, s, g); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mlp_nll_fused(const MlpGemm& g, const MlpHidden& h, hipStream_t s) {
    if (g.K > kNllKS * 16 || g.sak != 1 || g.sbk != 1 || g.n_nt < 1 || g.N % 8 ||
        g.n_nt > (g.N + TN - 1) / TN || g.M % 8 || h.k[0] != 32 ||
        h.k[1] != kFusedHidden + 8 || h.k[2] != kFusedHidden + 8 || g.K != kFusedHidden + 8)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_nll<true>, dim3((g.M + TM - 1) / TM, g.n_nt), dim3(kMlpThreads),
                       0, s, g, h);
    return hipGetLastError();
}

hipError_t launch_transpose_bf16(const bf16* src, bf16* dst, int rows, int cols,
                                 hipStream_t s) {
    const long n = (long)rows * cols;
    hipLaunchKernelGGL(k_transpose_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       src, dst, rows, cols);
    return hipGetLastError();
}

hipError_t launch_mlp_input(const MlpInput& a, hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_input, dim3((a.B + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((a.n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_targets(const TargetArgs& a, hipStream_t s) {
    const long n = (long)a.P * a.N;
    hipLaunchKernelGGL(k_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_ones_col(bf16* h, int B, int ld, int col, hipStream_t s) {
    hipLaunchKernelGGL(k_ones_col, dim3((B + 255) / 256), dim3(256), 0, s, h, B, ld, col);
    return hipGetLastError();
}

}  // namespace nr
