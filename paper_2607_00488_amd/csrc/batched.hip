// Batched path on gfx950: many parameter points (and many datasets of
// uneven binning) at once.  The per-point weights turn the fold into a dense
// GEMM  mu[p][j] = f_bkg b_j + sum_l W[p][l] R[l][j]  (Eq. (matrix_reweight)
// applied to a batch), run on the matrix cores in one
// persistent grouped launch with a fused Poisson epilogue (Eq. (logL)).
// The products and sums are FP64 (v_mfma_f64_16x16x4_f64): with FP32
// matrix cores the -2lnL of prior-box corner points drifts by ~1.3e-3 from
// the FP64 reference, above the 1e-3 budget.
#include "batched.h"
#include "lnpos.h"

#include <cmath>

namespace nr {

namespace {


// The GEMM takes its operand pointers from a problem table in memory, so
// the compiler cannot tell that they point to global memory and emits flat
// loads and stores, which also count against the LDS wait counter: every
// wait for the staged tile would then wait for the next tile's global
// loads as well.  These views make the accesses global ones.
template <class T>
__device__ inline const __attribute__((address_space(1))) T* gmem(const T* p) {
    return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ inline __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
typedef double gd2 __attribute__((ext_vector_type(2)));
typedef float gf4 __attribute__((ext_vector_type(4)));
__device__ inline double2 ld_global(const double2* p) {
    const gd2 v = *(const __attribute__((address_space(1))) gd2*)p;
    return make_double2(v.x, v.y);
}
__device__ inline float4 ld_global(const float4* p) {
    const gf4 v = *(const __attribute__((address_space(1))) gf4*)p;
    return make_float4(v.x, v.y, v.z, v.w);
}

__device__ inline double wave_sum64(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Basis coefficients c_b(theta) of S_theta = sum_b c_b I_b (the flavour sum
// of Eq. (sm_cross_section) with Eq. (xs_nsi) couplings and the magnetic
// term of Eq. (xs_mm), split by source group and by the coupling products).
__device__ inline void basis_coef(const double* th, const Phys& ph,
                                  double c[kNBasis]) {
    const double gle = ph.gLe + th[0], gre = ph.gR + th[1];
    const double glm = ph.gLm, grm = ph.gR;
    const double glt = ph.gLm + th[2], grt = ph.gR + th[3];
    for (int g = 0; g < 2; ++g) {
        const double f = g ? th[5] : 1.0;
        const int o = g * 10;
        c[o + 0] = f * gle * gle;
        c[o + 1] = f * gre * gre;
        c[o + 2] = -f * gle * gre;
        c[o + 3] = f * glm * glm;
        c[o + 4] = f * grm * grm;
        c[o + 5] = -f * glm * grm;
        c[o + 6] = f * glt * glt;
        c[o + 7] = f * grt * grt;
        c[o + 8] = -f * glt * grt;
        c[o + 9] = f * ph.cmm * th[4];
    }
}

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
    }
    dc[5][10] = gle * gle;
    dc[5][11] = gre * gre;
    dc[5][12] = -gle * gre;
    dc[5][13] = glm * glm;
    dc[5][14] = grm * grm;
    dc[5][15] = -glm * grm;
    dc[5][16] = glt * glt;
    dc[5][17] = grt * grt;
    dc[5][18] = -glt * grt;
    dc[5][19] = ph.cmm * th[4];
}

// ------------------------------------------------------------ weights
// W^T[l][p] = m_l * w_l(theta_p) with w_l = S_theta(T_l) / S_SM(T_l) and
// S_theta(T_l) = sum_b c_b(theta_p) I_b(T_l) (FP64), stored in the
// K-major layout the GEMM streams.  One thread per point, a strip of rows
// per work-group row; the basis row is wave-uniform.
constexpr int kWgenRows = 32;
constexpr int kWgenCols = kNBasis + 2;  // the basis, S_SM and m of a row

__global__ __launch_bounds__(256) void k_wgen(WgenArgs a) {
    // The work-group's strip of rows (basis values, S_SM, m) is staged in
    // LDS once; every lane then reads the same entries (broadcast).  Read
    // from memory inside the per-row loop they were a chain of dependent
    // round trips per row.
    __shared__ double strip[kWgenRows][kWgenCols];
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int l0 = blockIdx.y * kWgenRows;
    const int nrow = min(kWgenRows, a.n_t - l0);
    for (int q = threadIdx.x; q < kWgenRows * kWgenCols; q += 256) {
        const int col = q / kWgenRows, r = q % kWgenRows, l = l0 + r;
        double v = 0.0;
        if (r < nrow)
            v = col < kNBasis ? a.basis[(size_t)col * a.n_t + l]
                              : (col == kNBasis ? a.ssm[l] : a.mrow[l]);
        strip[r][col] = v;
    }
    __syncthreads();
    if (p >= a.ldw) return;
    double c[kNBasis];
    const bool ok = p < a.n_pts;
    if (ok) {
        double th[kNTheta];
        for (int i = 0; i < kNTheta; ++i) th[i] = a.theta[(size_t)p * kNTheta + i];
        basis_coef(th, a.ph, c);
    } else {
        for (int b = 0; b < kNBasis; ++b) c[b] = 0.0;
    }
    for (int r = 0; r < nrow; ++r) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < kNBasis; ++b) s = fma(c[b], strip[r][b], s);
        const double ssm = strip[r][kNBasis];
        const double w = ssm > 0.0 ? s / ssm : 1.0;
        a.wt[(size_t)(l0 + r) * a.ldw + p] = ok ? strip[r][kNBasis + 1] * w : 0.0;
    }
}

// --------------------------------------------------------------- GEMM
// Tiles of BM x BN outputs, K-steps of 16; four waves in 2 x 2, each
// (BM/2) x (BN/2) = blocks of v_mfma_f64_16x16x4_f64.  The tile shape is a
// template parameter; the host picks one per shape class by timing.
//
// Operands reach LDS by gfx950's global-to-LDS copies: one instruction moves
// 16 bytes per lane from any global address and writes them, in lane order,
// as 1 KiB at a wave-uniform LDS base, without passing through registers.
// The K-steps rotate through a ring of three stages (four for the adjoint
// where LDS allows), so each step waits only for its own stage (copied two
// or three steps earlier) and has one barrier, which also frees the stage
// read one step before for the next copy.  R
// stays FP32 in LDS (half the bytes of FP64) and is widened when a wave
// takes its fragment.  Lanes past an operand's edge copy a zero chunk.
//
// Within a K-step, MFMA sub-step s gives lane row (k) 4 * (lane / 16) + s,
// and the wave's 16 x 16 blocks interleave their rows and columns so that
// each lane's operands of one sub-step sit side by side in LDS: one 16-byte
// read gives two A values (or four R values) instead of one each.
constexpr int BK = kGemmBK;
constexpr int kGemmThreads = 256;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) void glb_void;

// Source of the chunks that lie past an operand's edge (never written).
__device__ __align__(16) double g_zero_chunk[2];

// Written as assembly so that the compiler does not track these copies:
// with them in view it waited for every copy in flight before any LDS read
// of the loop, which undoes the ring.  The waits are explicit instead.
// (m0 is named as clobbered; the compiler keeps nothing in it here.)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
// `lds` is the wave's LDS byte address (the same in every lane).
__device__ inline void copy16_to_lds(const void* src, unsigned lds) {
    asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off"
                 :
                 : "v"(src), "s"(lds)
                 : "memory", "m0");
}
#pragma clang diagnostic pop

// 16-byte slot of (row n, k-chunk) in the adjoint's [n][16 k] stage of R:
// rotated with n so that the 16 rows one read touches fall on distinct
// banks (for 32 and for 64 four-byte banks alike).
__device__ inline int adj_swz(int n) {
    return 2 * ((n >> 2) & 1) + (((n >> 1) & 1) ^ ((n >> 3) & 1));
}

// s_waitcnt with vmcnt = N and lgkmcnt = 0 (expcnt left alone).
template <int N>
__device__ inline void wait_vm_lgkm0() {
    static_assert(N >= 0 && N < 16, "vmcnt immediate");
    __builtin_amdgcn_s_waitcnt(N | (7 << 4));
}

// The tiles of 8192 outputs ask the compiler for register use that lets
// three work-groups share a compute unit, the 128 x 128 tile two.
template <int MODE, int BM, int BN>
__global__ __launch_bounds__(kGemmThreads, BM * BN <= 8192 ? 3 : 2)
void k_gemm(const GemmProb* probs, const GemmTile* tiles, int n_tiles, unsigned* ctr) {
    constexpr bool ADJ = MODE == kModeAdj;
    constexpr int WTM = BM / 2, WTN = BN / 2;   // wave tile
    constexpr int BI = WTM / 16, BJ = WTN / 16;  // 16x16 blocks per wave
    constexpr int NIA = BM / 32, NIB = BN / 64;  // copies per wave and stage
    constexpr int NI = NIA + NIB;
    // forward R stage: [16][BN] floats in 1 KiB blocks of 256 / BN rows; with
    // BN = 64 a 128-byte gap after each block puts rows 4 apart on other banks
    constexpr int RPB = 256 / BN;
    constexpr int PADB = (!ADJ && BN == 64) ? 32 : 0;  // floats
    constexpr int A_DBL = BK * BM;
    constexpr int B_FLT = (BN / 16) * (256 + PADB);
    constexpr int SLOT = A_DBL * 8 + B_FLT * 4;
    constexpr int EPI = WTN + 1;  // epilogue staging stride (doubles)
    // ring slots: stage s + RING - 1 is copied during step s.  The adjoint's
    // R chunks (64 bytes of each of 16 rows per copy) arrive later than the
    // forward's contiguous rows; it prefetches one step deeper where LDS
    // still leaves room for two work-groups per compute unit.
    constexpr int RING = (ADJ && 4 * SLOT <= 65536) ? 4 : 3;
    static_assert(BI % 2 == 0 && (ADJ || BJ == 2 || BJ == 4), "tile shape");
    static_assert(4 * 16 * EPI * 8 <= RING * SLOT, "epilogue staging fits the ring");
    static_assert(RING == 3 || RING == 4, "ring length");
    __shared__ __align__(16) unsigned char ring[RING * SLOT];
    __shared__ double rowred[BM][2];
    __shared__ double rowred2[BM][2];
    __shared__ int s_tile;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave >> 1, wn = wave & 1;
    const int li = lane & 15, lk = lane >> 4;
    // held in scalar registers (not re-derived inside the loop)
    const double* zp = g_zero_chunk;
    asm volatile("" : "+s"(zp));
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    const unsigned ring_lds =
        __builtin_amdgcn_readfirstlane((unsigned)(uintptr_t)(lds_void*)ring);

    for (;;) {
        if (tid == 0) s_tile = (int)atomicAdd(&ctr[0], 1u);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (t >= n_tiles) break;
        const GemmTile tl = tiles[t];
        const GemmProb pr = probs[tl.prob];
        const int m0 = tl.mt * BM, n0 = tl.nt * BN;
        const int K = pr.K;

        v4d acc[BI][BJ];
#pragma unroll
        for (int i = 0; i < BI; ++i)
#pragma unroll
            for (int j = 0; j < BJ; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

        const int kb = tl.k0;
        const int nst = (tl.k1 - tl.k0 + BK - 1) / BK;
        // Each copy instruction of a wave moves one 16-byte chunk per lane.
        // Its source is lane-constant within the tile up to an advance of
        // one stage per K-step, so the pointers are set up once here and
        // stepped; a chunk past the operand's edge (a column beyond the
        // stored width, a row beyond K) is taken from the zero chunk.
        const char* src[NI];
        long adv[NI];   // bytes per K-step (0 for a chunk that stays zero)
        int c0[NI];     // chunk's K coordinate at the tile's first step
        int lim[NI];    // its K coordinate must stay below this
#pragma unroll
        for (int q = 0; q < NIA; ++q) {  // A^T: [16][BM] doubles, M contiguous
            const int e = 2 * ((wave + 4 * q) * 64 + lane);
            const int kk = e / BM, m = m0 + e % BM;
            const bool ok = m < pr.lda;
            src[q] = ok ? (const char*)(pr.At + (size_t)(kb + kk) * pr.lda + m) : (const char*)zp;
            adv[q] = ok ? (long)BK * pr.lda * 8 : 0;
            c0[q] = kb + kk;
            lim[q] = K;
        }
#pragma unroll
        for (int q = 0; q < NIB; ++q) {
            const int I = wave + 4 * q;
            if constexpr (!ADJ) {  // R[k][n], N contiguous: [16][BN]
                const int e = 4 * (I * 64 + lane);
                const int kk = e / BN, n = n0 + e % BN;
                const bool ok = n < pr.ldb;
                src[NIA + q] = ok ? (const char*)(pr.B + (size_t)(kb + kk) * pr.ldb + n)
                                  : (const char*)zp;
                adv[NIA + q] = ok ? (long)BK * pr.ldb * 4 : 0;
                c0[NIA + q] = kb + kk;
                lim[NIA + q] = K;
            } else {  // R[n][k], K contiguous: [BN][16] in rotated chunks
                const int c = I * 64 + lane;
                const int nl = c >> 2, k4 = (c & 3) ^ adj_swz(c >> 2);
                const int n = n0 + nl;
                const bool ok = n < pr.N;
                src[NIA + q] = ok ? (const char*)(pr.B + (size_t)n * pr.ldb + kb + 4 * k4)
                                  : (const char*)zp;
                adv[NIA + q] = ok ? (long)BK * 4 : 0;
                c0[NIA + q] = kb + 4 * k4;
                lim[NIA + q] = pr.ldb;
            }
        }
        // LDS byte address of each copy's 1 KiB in slot 0 (wave-uniform)
        auto lds_of = [&](int q) -> unsigned {
            return q < NIA ? ring_lds + (unsigned)((wave_u + 4 * q) * 1024)
                           : ring_lds + (unsigned)(A_DBL * 8 +
                                                   (wave_u + 4 * (q - NIA)) * (1024 + 4 * PADB));
        };
        // copy q of stage st (K-steps from the tile's first) into ring slot `slot`
        auto issue_one = [&](int slot, int st, int q) {
            const char* p = c0[q] + st * BK < lim[q] ? src[q] : (const char*)zp;
            copy16_to_lds(p, lds_of(q) + (unsigned)(slot * SLOT));
            src[q] += adv[q];
        };
        auto issue = [&](int slot, int st) {
#pragma unroll
            for (int q = 0; q < NI; ++q) issue_one(slot, st, q);
        };

        // nothing of this tile's set-up left in flight: the loop's explicit
        // waits then count only the ring's copies
        __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
        for (int st = 0; st < RING - 1; ++st)
            if (st < nst) issue(st, st);
        // one K-step on the stage in slot `cur`; stage s + 2 goes into the
        // slot stage s - 1 used
        auto step = [&](int cur, int s) {
            // this stage is in; the later ones already issued may still fly
            if (RING == 4 && s + 2 < nst)
                wait_vm_lgkm0<(RING == 4 ? 2 * NI : NI)>();
            else if (s + 1 < nst)
                wait_vm_lgkm0<NI>();
            else
                wait_vm_lgkm0<0>();
            asm volatile("s_barrier" ::: "memory");
            const double* SA = reinterpret_cast<const double*>(ring + cur * SLOT);
            const float* SB = reinterpret_cast<const float*>(ring + cur * SLOT + A_DBL * 8);
            double2 fa[4][BI / 2];
            float fb[4][BJ];
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
                const int row = 4 * lk + s4;
#pragma unroll
                for (int h = 0; h < BI / 2; ++h)
                    fa[s4][h] = *reinterpret_cast<const double2*>(
                        SA + row * BM + wm * WTM + 32 * h + 2 * li);
                if constexpr (!ADJ) {
                    const float* rp = SB + (row / RPB) * (256 + PADB) + (row % RPB) * BN +
                                      wn * WTN + BJ * li;
                    if constexpr (BJ == 4) {
                        const float4 v = *reinterpret_cast<const float4*>(rp);
                        fb[s4][0] = v.x; fb[s4][1] = v.y; fb[s4][2] = v.z; fb[s4][3] = v.w;
                    } else {
                        const float2 v = *reinterpret_cast<const float2*>(rp);
                        fb[s4][0] = v.x; fb[s4][1] = v.y;
                    }
                }
            }
            if constexpr (ADJ) {
#pragma unroll
                for (int y = 0; y < BJ; ++y) {
                    const int nl = wn * WTN + 16 * y + li;
                    const float4 v = *reinterpret_cast<const float4*>(
                        SB + 4 * (4 * nl + (lk ^ adj_swz(nl))));
                    fb[0][y] = v.x; fb[1][y] = v.y; fb[2][y] = v.z; fb[3][y] = v.w;
                }
            }
            // the next stage's copies go out between the sub-steps' matrix
            // instructions rather than in one burst ahead of them
            const bool more = s + RING - 1 < nst;
            const int nslot = cur == 0 ? RING - 1 : cur - 1;
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4) {
#pragma unroll
                for (int x = 0; x < BI; ++x) {
                    const double a = (x & 1) ? fa[s4][x >> 1].y : fa[s4][x >> 1].x;
#pragma unroll
                    for (int y = 0; y < BJ; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                            a, (double)fb[s4][y], acc[x][y], 0, 0, 0);
                }
                if (more) {
#pragma unroll
                    for (int q = s4; q < NI; q += 4) issue_one(nslot, s + RING - 1, q);
                }
            }
        };
        // unrolled by the ring's length so that every slot offset is a constant
        for (int s = 0; s < nst; s += RING) {
            step(0, s);
            if (s + 1 < nst) step(1, s + 1);
            if (s + 2 < nst) step(2, s + 2);
            if (RING == 4 && s + 3 < nst) step(3, s + 3);
        }

        // ---- epilogue.  Output (i, j) of a 16x16 block sits in lane
        // j + 16 * (i % 4), register i / 4; block x's row i is tile row
        // wm * WTM + 32 * (x / 2) + 2 * i + x % 2.
        if constexpr (ADJ) {
#pragma unroll
            for (int bi = 0; bi < BI; ++bi)
#pragma unroll
                for (int bj = 0; bj < BJ; ++bj)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int p = m0 + wm * WTM + 32 * (bi >> 1) + 2 * (lk + 4 * r) + (bi & 1);
                        const int col = n0 + wn * WTN + bj * 16 + li;
                        if (p < pr.M && col < pr.N)
                            *gmem(pr.C + (size_t)p * pr.ldc + col) = acc[bi][bj][r];
                    }
        } else {
            // one 16-row strip of each wave at a time through the (now idle)
            // ring; four lanes share a row and take a quarter of the wave's
            // columns each, in column order
            double* stage = reinterpret_cast<double*>(ring) + wave * 16 * EPI;
            constexpr int CQ = WTN / 4;
#pragma unroll
            for (int bi = 0; bi < BI; ++bi) {
                __syncthreads();
#pragma unroll
                for (int y = 0; y < BJ; ++y)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        stage[(lk + 4 * r) * EPI + BJ * li + y] = acc[bi][y][r];
                __syncthreads();
                const int r16 = lane >> 2, cs = lane & 3;
                const int i = wm * WTM + 32 * (bi >> 1) + 2 * r16 + (bi & 1);
                const int p = m0 + i;
                double dsum = 0.0, gsum = 0.0;
                if (p < pr.M) {
                    const double fbk = *gmem(pr.theta + (size_t)p * kNTheta + 6);
                    for (int q = 0; q < CQ; ++q) {
                        const int col = n0 + wn * WTN + cs * CQ + q;
                        if (col >= pr.N) break;
                        const double bj_ = *gmem(pr.b + col);
                        const double mu = fbk * bj_ + stage[r16 * EPI + cs * CQ + q];
                        const double nj = *gmem(pr.n + col);
                        double d;
                        if (nj > 0.0)
                            d = mu > 0.0 ? (mu - nj + nj * log(nj / mu)) : INFINITY;
                        else
                            d = mu;
                        dsum += d;
                        if (pr.mu) *gmem(pr.mu + (size_t)p * pr.N + col) = mu;
                        if (pr.aout) {
                            // an empty bin's term is 2 mu_j: derivative 2
                            const double aj = nj > 0.0 ? 2.0 * (1.0 - nj / mu) : 2.0;
                            *gmem(pr.aout + (size_t)col * pr.lda_out + p) = aj;
                            gsum += aj * bj_;
                        }
                    }
                }
                dsum += __shfl_xor(dsum, 1, 64);
                dsum += __shfl_xor(dsum, 2, 64);
                gsum += __shfl_xor(gsum, 1, 64);
                gsum += __shfl_xor(gsum, 2, 64);
                if (cs == 0) {
                    rowred[i][wn] = dsum;
                    rowred2[i][wn] = gsum;
                }
            }
            __syncthreads();
            if (tid < BM) {
                const int p = m0 + tid;
                if (p < pr.M) {
                    *gmem(pr.part + (size_t)p * pr.n_nt + tl.nt) = rowred[tid][0] + rowred[tid][1];
                    if (pr.aout)
                        *gmem(pr.part_gb + (size_t)p * pr.n_nt + tl.nt) = rowred2[tid][0] + rowred2[tid][1];
                }
            }
        }
    }
    // the last work-group out resets the tile counter for the next launch
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        const unsigned prev = atomicAdd(&ctr[1], 1u);
        if (prev == gridDim.x - 1) {
            ctr[0] = 0u;
            ctr[1] = 0u;
        }
    }
}

// -2lnL per point: sum of the column-tile deviance partials, data constant,
// pulls (Eq. (logL)).
// x[0] + x[1] + ... + x[n - 1] in index order; with n even (so that every
// row of a [P][n] array starts 16-byte aligned) eight values at a time as
// 16-byte pairs, all in flight before the additions.
__device__ inline double row_sum(const double* x, int n) {
    double s = 0.0;
    int q = 0;
    if ((n & 1) == 0) {
        for (; q + 8 <= n; q += 8) {
            double2 v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) v[i] = reinterpret_cast<const double2*>(x + q)[i];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                s += v[i].x;
                s += v[i].y;
            }
        }
    }
    for (; q < n; ++q) s += x[q];
    return s;
}

__global__ void k_finalize(FinalArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= a.n_pts) return;
    const double d = row_sum(a.part + (size_t)p * a.n_nt, a.n_nt);
    double pulls = 0.0;
    for (int i = 0; i < kNTheta; ++i)
        if (a.pull_sigma[i] > 0.0) {
            const double z = (a.theta[(size_t)p * kNTheta + i] - a.pull_mean[i]) / a.pull_sigma[i];
            pulls += z * z;
        }
    a.nll[p] = 2.0 * d + 2.0 * a.cdata + pulls;
}

// Gradient per point from the adjoint U[p][l] = sum_j a_pj R_lj:
// grad_i = sum_l U_pl (m_l / S_SM(T_l)) sum_b dc_ib I_b(T_l) + [i = f_bkg]
// sum_j a_pj b_j + pull term.
// The contraction J[p][b] = sum_l U[p][l] v_l I_b(T_l), v_l = m_l / S_SM(T_l)
// (0 where S_SM = 0), is itself a product of U (points x rows) with the
// weighted basis (rows x 20): FP64 matrix instructions over blocks of 16
// points and chunks of kCtrChunk rows, the four waves of a work-group on
// quarters of its chunk.  With several chunks, each work-group leaves its
// 16 x 20 partial sums in the first 20 columns of its own chunk of U (rows
// only it reads, already consumed) and k_adj_final adds them per point in
// chunk order; a single chunk finishes in place.
constexpr int kCtrChunk = 1024;

__host__ __device__ inline int ctr_chunks(int n_t) {
    return n_t >= 2 * kCtrChunk ? n_t / kCtrChunk : 1;
}

// d(-2lnL)/d theta of point p from its contracted basis sums J (Eqs.
// (logL), (reweight_factor): the chain through c_b(theta) and f_bkg) plus
// the pulls.
__device__ inline void contract_finish(const ContractArgs& a, int p, const double J[kNBasis]) {
    double th[kNTheta];
    for (int i = 0; i < kNTheta; ++i) th[i] = a.theta[(size_t)p * kNTheta + i];
    double dc[kNTheta][kNBasis];
    basis_dcoef(th, a.ph, dc);
    const double gb = row_sum(a.part_gb + (size_t)p * a.n_nt, a.n_nt);
    for (int i = 0; i < kNTheta; ++i) {
        double g = 0.0;
        for (int b = 0; b < kNBasis; ++b) g += dc[i][b] * J[b];
        if (i == 6) g += gb;
        if (a.pull_sigma[i] > 0.0)
            g += 2.0 * (th[i] - a.pull_mean[i]) / (a.pull_sigma[i] * a.pull_sigma[i]);
        a.grad[(size_t)p * kNTheta + i] = g;
    }
}

__global__ __launch_bounds__(256) void k_adj_contract(ContractArgs a) {
    __shared__ double red[4][16][kNBasis];
    const int pb = blockIdx.x, ch = blockIdx.y, nch = gridDim.y;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int c0 = ch * kCtrChunk;
    const int c1 = ch == nch - 1 ? a.n_t : c0 + kCtrChunk;
    const int len = c1 - c0;
    // quarters start on multiples of four rows (16-byte aligned pairs below)
    const int q0 = c0 + ((int)((long)len * wave / 4) & ~3);
    const int q1 = wave == 3 ? c1 : c0 + ((int)((long)len * (wave + 1) / 4) & ~3);
    const int p = pb * 16 + li;  // this lane's row of the point operand
    v4d acc[2] = {(v4d){0.0, 0.0, 0.0, 0.0}, (v4d){0.0, 0.0, 0.0, 0.0}};
    // MFMA sub-step e gives lane row l + 4 (lane / 16) + e of the 16-row
    // step; the next step's loads are issued before this step's arithmetic.
    // A lane's four rows are consecutive: with even row strides they are
    // read as 16-byte pairs (every row offset of a lane is even), else, and
    // for a group that runs past the quarter, one by one.
    const bool pairs = a.ldu % 2 == 0 && a.n_t % 2 == 0;
    struct Step { double u[4], b0[4], b1[4], sm[4], m[4]; };
    auto pair4 = [](const double* src, double out[4]) {
        const double2 x = *reinterpret_cast<const double2*>(src);
        const double2 y = *reinterpret_cast<const double2*>(src + 2);
        out[0] = x.x; out[1] = x.y; out[2] = y.x; out[3] = y.y;
    };
    auto load = [&](int l, Step& t) {
        const int r0 = l + 4 * lk;
        if (pairs && r0 + 3 < q1) {
            pair4(a.ssm + r0, t.sm);
            pair4(a.mrow + r0, t.m);
            if (p < a.n_pts) pair4(a.U + (size_t)p * a.ldu + r0, t.u);
            else t.u[0] = t.u[1] = t.u[2] = t.u[3] = 0.0;
            pair4(a.basis + (size_t)li * a.n_t + r0, t.b0);
            if (16 + li < kNBasis) pair4(a.basis + (size_t)(16 + li) * a.n_t + r0, t.b1);
            else t.b1[0] = t.b1[1] = t.b1[2] = t.b1[3] = 0.0;
            return;
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int r = r0 + e;
            const bool ok = r < q1;
            t.sm[e] = ok ? a.ssm[r] : 0.0;
            t.m[e] = ok ? a.mrow[r] : 0.0;
            t.u[e] = ok && p < a.n_pts ? a.U[(size_t)p * a.ldu + r] : 0.0;
            t.b0[e] = ok ? a.basis[(size_t)li * a.n_t + r] : 0.0;
            t.b1[e] = ok && 16 + li < kNBasis ? a.basis[(size_t)(16 + li) * a.n_t + r] : 0.0;
        }
    };
    Step cur, nxt;
    if (q0 < q1) load(q0, cur);
    for (int l = q0; l < q1; l += 16) {
        if (l + 16 < q1) load(l + 16, nxt);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const double v = cur.sm[e] > 0.0 ? cur.m[e] / cur.sm[e] : 0.0;
            acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur.u[e], cur.b0[e] * v, acc[0], 0, 0, 0);
            acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur.u[e], cur.b1[e] * v, acc[1], 0, 0, 0);
        }
        cur = nxt;
    }
    // output (i, j) of a block: lane j + 16 (i % 4), register i / 4; here
    // i is the point and j the basis index within block y
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int b = 16 * y + li;
            if (b < kNBasis) red[wave][4 * r + lk][b] = acc[y][r];
        }
    __syncthreads();
    // the four quarters in order; every wave has read its rows of U
    for (int q = tid; q < 16 * kNBasis; q += 256) {
        const int i = q / kNBasis, b = q % kNBasis, pp = pb * 16 + i;
        const double J = red[0][i][b] + red[1][i][b] + red[2][i][b] + red[3][i][b];
        if (nch > 1 && pp < a.n_pts) a.U[(size_t)pp * a.ldu + c0 + b] = J;
        red[0][i][b] = J;
    }
    if (nch > 1) return;
    __syncthreads();
    if (tid < 16 && pb * 16 + tid < a.n_pts) contract_finish(a, pb * 16 + tid, red[0][tid]);
}

// The chunk partials of each point, added in chunk order (one lane per
// point and basis index, so that a point's 20 partials of a chunk are one
// contiguous read), then the gradient.
constexpr int kFinPts = 256 / kNBasis;  // points per work-group

__global__ __launch_bounds__(256) void k_adj_final(ContractArgs a, int nch) {
    __shared__ double js[kFinPts][kNBasis];
    const int t = threadIdx.x, i = t / kNBasis, b = t % kNBasis;
    const int p = blockIdx.x * kFinPts + i;
    if (i < kFinPts && p < a.n_pts) {
        double J = 0.0;
        for (int ch = 0; ch < nch; ++ch) J += a.U[(size_t)p * a.ldu + ch * kCtrChunk + b];
        js[i][b] = J;
    }
    __syncthreads();
    const int pf = blockIdx.x * kFinPts + t;
    if (t < kFinPts && pf < a.n_pts) contract_finish(a, pf, js[t]);
}

// ------------------------------------------------------------ templates
// One thread per reco bin, one work-group row per slab of response rows:
// kTmplCols FP64 sums of F_bl R_lj.  The row factors are wave-uniform.
__global__ __launch_bounds__(256) void k_tmpl_fold(TmplFoldArgs a) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= a.n_reco) return;
    const int l0 = blockIdx.y * kTmplSlabRows;
    const int l1 = min(l0 + kTmplSlabRows, a.n_t);
    double acc[kTmplCols];
#pragma unroll
    for (int b = 0; b < kTmplCols; ++b) acc[b] = 0.0;
    for (int l = l0; l < l1; ++l) {
        const double r = a.R[(size_t)l * a.ldr + j];
        const double* f = a.F + (size_t)l * kTmplCols;
#pragma unroll
        for (int b = 0; b < kTmplCols; ++b) acc[b] = fma(f[b], r, acc[b]);
    }
#pragma unroll
    for (int b = 0; b < kTmplCols; ++b)
        a.part[((size_t)blockIdx.y * kTmplCols + b) * a.n_reco + j] = acc[b];
}

// Slab sums in slab order, one (bin, template) per thread, into the record
// column the caller maps each folded column to.
__global__ __launch_bounds__(256) void k_tmpl_records(TmplRecArgs a) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (j >= a.n_reco || a.dst[b] < 0) return;
    double s = 0.0;
    for (int q = 0; q < a.n_slab; ++q) s += a.part[((size_t)q * kTmplCols + b) * a.n_reco + j];
    a.rec[(size_t)j * a.rl + a.dst[b]] = s;
}

// The data of each bin beside its templates (rewritten alone by set_data).
__global__ __launch_bounds__(256) void k_tmpl_data(TmplDataArgs a) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= a.n_reco) return;
    double* r = a.rec + (size_t)j * kTmplRec;
    const double nj = a.n[j];
    r[kTmplCols] = a.b[j];
    r[kTmplCols + 1] = nj;
    r[kTmplCols + 2] = 0.0;  // pads the record to 24 doubles
}

// One thread per point, one work-group column per slice of reco bins.  The
// bin record is the same for every lane (scalar loads); each lane forms
// mu_j, the deviance term of Eq. (logL) and, for the gradient, the
// contractions h_b = sum_j a_j G_bj with a_j = 2 (1 - n_j / mu_j).  The
// logarithm is the plain-FP64 series of lnpos.h (the library one spends
// ~85 double-double operations per bin on accuracy the sum cannot use).
template <bool GRAD, bool MU>
__global__ __launch_bounds__(kTmplWave) void k_tmpl_eval(TmplEvalArgs a) {
    const int p = blockIdx.x * kTmplWave + threadIdx.x;
    const int sl = blockIdx.y;
    const bool ok = p < a.n_pts;
    const int pc = ok ? p : a.n_pts - 1;
    double th[kNTheta], c[kNBasis];
    for (int i = 0; i < kNTheta; ++i) th[i] = a.theta[(size_t)pc * kNTheta + i];
    basis_coef(th, a.ph, c);
    const double fb = th[6];
    const int j0 = sl * a.cols_per;
    const int j1 = min(j0 + a.cols_per, a.n_reco);
    double dsum = 0.0;
    double h[kTmplCols];
#pragma unroll
    for (int b = 0; b < kTmplCols; ++b) h[b] = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double* __restrict__ r = a.rec + (size_t)j * kTmplRec;
        double mu = fma(fb, r[kTmplCols], r[kNBasis]);
#pragma unroll
        for (int b = 0; b < kNBasis; ++b) mu = fma(c[b], r[b], mu);
        const double nj = r[kTmplCols + 1];
        // n ln(n / mu), not n (ln n - ln mu): near a fit's minimum the two
        // logarithms agree to many digits and their separate roundings
        // would leave ~1e-10 of noise in -2lnL, enough to stall a line
        // search; the logarithm of the ratio is accurate relative to its
        // own small size.
        const double q = nj > 0.0 ? nj / mu : 0.0;
        double d;
        if (nj > 0.0)
            d = mu > 0.0 ? (mu - nj) + nj * ln_pos(q) : INFINITY;
        else
            d = mu;
        dsum += d;
        if (MU && ok) a.mu[(size_t)p * a.n_reco + j] = mu;
        if (GRAD) {
            const double aj = 2.0 * (1.0 - q);
#pragma unroll
            for (int b = 0; b < kNBasis; ++b) h[b] = fma(aj, r[b], h[b]);
            h[kNBasis] = fma(aj, r[kTmplCols], h[kNBasis]);  // sum_j a_j b_j
        }
    }
    if (!ok) return;
    a.dpart[(size_t)sl * a.n_pts + p] = dsum;
    if (GRAD) {
#pragma unroll
        for (int b = 0; b < kTmplCols; ++b)
            a.hpart[((size_t)sl * kTmplCols + b) * a.n_pts + p] = h[b];
    }
}

// Sums over the column slices, one (point, quantity) per thread, in slice
// order (bitwise reproducible).
__global__ __launch_bounds__(kTmplWave) void k_tmpl_reduce(TmplReduceArgs a) {
    const int p = blockIdx.x * kTmplWave + threadIdx.x;
    if (p >= a.n_pts) return;
    const int v = blockIdx.y;
    double s = 0.0;
    if (v == 0) {
        for (int q = 0; q < a.n_split; ++q) s += a.dpart[(size_t)q * a.n_pts + p];
    } else {
        for (int q = 0; q < a.n_split; ++q)
            s += a.hpart[((size_t)q * a.n_acc + v - 1) * a.n_pts + p];
    }
    a.red[(size_t)v * a.n_pts + p] = s;
}

// -2lnL per point (Eq. (logL)) and, with the contractions, its gradient:
// d mu_j / d theta_i = sum_b dc_ib G_bj + [i = f_bkg] b_j.
__global__ __launch_bounds__(256) void k_tmpl_final(TmplFinalArgs a) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n_pts) return;
    const double d = a.red[p];
    double th[kNTheta];
    for (int i = 0; i < kNTheta; ++i) th[i] = a.theta[(size_t)p * kNTheta + i];
    double pulls = 0.0;
    for (int i = 0; i < kNTheta; ++i)
        if (a.pull_sigma[i] > 0.0) {
            const double z = (th[i] - a.pull_mean[i]) / a.pull_sigma[i];
            pulls += z * z;
        }
    a.nll[p] = 2.0 * d + 2.0 * a.cdata + pulls;
    if (!a.grad) return;
    double h[kTmplCols];
    for (int b = 0; b < kTmplCols; ++b) h[b] = a.red[(size_t)(1 + b) * a.n_pts + p];
    double dc[kNTheta][kNBasis];
    basis_dcoef(th, a.ph, dc);
    for (int i = 0; i < kNTheta; ++i) {
        double g = 0.0;
        for (int b = 0; b < kNBasis; ++b) g += dc[i][b] * h[b];
        if (i == 6) g += h[kNBasis];
        if (a.pull_sigma[i] > 0.0)
            g += 2.0 * (th[i] - a.pull_mean[i]) / (a.pull_sigma[i] * a.pull_sigma[i]);
        a.grad[(size_t)p * kNTheta + i] = g;
    }
}

// ------------------------------------------------ multi-component templates
// Backgrounds, mask and data of each bin after the component templates.
__global__ __launch_bounds__(256) void k_tmpl_mdata(TmplMultiDataArgs a) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= a.n_reco) return;
    double* r = a.rec + (size_t)j * a.rl;
    const int ob = kTmplCompCols * a.K;
    for (int q = 0; q < a.B; ++q) r[ob + q] = a.bkg[(size_t)q * a.n_reco + j];
    r[ob + a.B] = a.mask ? a.mask[j] : 1.0;
    r[ob + a.B + 1] = a.n[j];
}

// As k_tmpl_eval, for the multi-component record: per (point, bin) the
// component sums t_k = G0^(k) + sum_b c_b G^(k)_b (11 K products), mu from
// the rates, and for the gradient the 10 + K + B contractions
//   H_b = sum_j a'_j sum_k r_k G^(k)_bj,  R_k = sum_j a'_j t_kj,
//   Q_q = sum_j a'_j B_qj,  a'_j = M_j d(-2lnL)/d mu_j.
// Loops run to compile-time maxima KM, BM with uniform predicates, so every
// accumulator stays in registers; the smaller size class (five components,
// four backgrounds: the solar species) needs fewer registers and keeps more
// waves resident.
template <bool GRAD, bool MU, int KM, int BM>
__global__ __launch_bounds__(kTmplWave) void k_tmpl_meval(TmplMultiEvalArgs a) {
    const int p = blockIdx.x * kTmplWave + threadIdx.x;
    const int sl = blockIdx.y;
    const bool ok = p < a.n_pts;
    const int pc = ok ? p : a.n_pts - 1;
    const double* th = a.theta + (size_t)pc * a.n_theta;
    double t7[kNTheta] = {th[0], th[1], th[2], th[3], th[4], 1.0, 1.0};
    double c[kNBasis];
    basis_coef(t7, a.ph, c);  // c[0..9]: the coefficients without group scaling
    double rk[KM], rb[BM];
#pragma unroll
    for (int k = 0; k < KM; ++k) rk[k] = k < a.K ? th[5 + k] : 0.0;
#pragma unroll
    for (int q = 0; q < BM; ++q) rb[q] = q < a.B ? th[5 + a.K + q] : 0.0;
    const int ob = kTmplCompCols * a.K;
    const int j0 = sl * a.cols_per;
    const int j1 = min(j0 + a.cols_per, a.n_reco);
    double dsum = 0.0;
    double H[10], Rk[KM], Qb[BM];
#pragma unroll
    for (int b = 0; b < 10; ++b) H[b] = 0.0;
#pragma unroll
    for (int k = 0; k < KM; ++k) Rk[k] = 0.0;
#pragma unroll
    for (int q = 0; q < BM; ++q) Qb[q] = 0.0;
    for (int j = j0; j < j1; ++j) {
        const double* __restrict__ r = a.rec + (size_t)j * a.rl;
        double s = 0.0, tk[KM], T[10];
#pragma unroll
        for (int b = 0; b < 10; ++b) T[b] = 0.0;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
            tk[k] = 0.0;
            if (k < a.K) {
                const double* g = r + kTmplCompCols * k;
                double t = g[10];
#pragma unroll
                for (int b = 0; b < 10; ++b) t = fma(c[b], g[b], t);
                if (GRAD) {  // T_b = sum_k r_k G^(k)_bj, for H_b
#pragma unroll
                    for (int b = 0; b < 10; ++b) T[b] = fma(rk[k], g[b], T[b]);
                }
                tk[k] = t;
                s = fma(rk[k], t, s);
            }
        }
#pragma unroll
        for (int q = 0; q < BM; ++q)
            if (q < a.B) s = fma(rb[q], r[ob + q], s);
        const double mask = r[ob + a.B], nj = r[ob + a.B + 1];
        const double mu = s * mask;
        const double qn = nj > 0.0 ? nj / mu : 0.0;
        double d;
        if (nj > 0.0)
            d = mu > 0.0 ? (mu - nj) + nj * ln_pos(qn) : INFINITY;
        else
            d = mu;
        dsum += d;
        if (MU && ok) a.mu[(size_t)p * a.n_reco + j] = mu;
        if (GRAD) {
            const double ap = 2.0 * (1.0 - qn) * mask;
#pragma unroll
            for (int k = 0; k < KM; ++k)
                if (k < a.K) Rk[k] = fma(ap, tk[k], Rk[k]);
#pragma unroll
            for (int b = 0; b < 10; ++b) H[b] = fma(ap, T[b], H[b]);
#pragma unroll
            for (int q = 0; q < BM; ++q)
                if (q < a.B) Qb[q] = fma(ap, r[ob + q], Qb[q]);
        }
    }
    if (!ok) return;
    a.dpart[(size_t)sl * a.n_pts + p] = dsum;
    if (GRAD) {
        const int na = 10 + a.K + a.B;
        double* hp = a.hpart + (size_t)sl * na * a.n_pts + p;
#pragma unroll
        for (int b = 0; b < 10; ++b) hp[(size_t)b * a.n_pts] = H[b];
#pragma unroll
        for (int k = 0; k < KM; ++k)
            if (k < a.K) hp[(size_t)(10 + k) * a.n_pts] = Rk[k];
#pragma unroll
        for (int q = 0; q < BM; ++q)
            if (q < a.B) hp[(size_t)(10 + a.K + q) * a.n_pts] = Qb[q];
    }
}

// -2lnL and gradient of the multi-component form: d/d theta_i (i < 5) =
// sum_b dc_ib H_b, d/d r_k = R_k, d/d r_q = Q_q, plus the pulls.
__global__ __launch_bounds__(256) void k_tmpl_mfinal(TmplMultiFinalArgs a) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= a.n_pts) return;
    const double* th = a.theta + (size_t)p * a.n_theta;
    double pulls = 0.0;
    for (int i = 0; i < a.n_theta; ++i)
        if (a.pull_sigma[i] > 0.0) {
            const double z = (th[i] - a.pull_mean[i]) / a.pull_sigma[i];
            pulls += z * z;
        }
    a.nll[p] = 2.0 * a.red[p] + 2.0 * a.cdata + pulls;
    if (!a.grad) return;
    const double* h = a.red + a.n_pts + p;  // contraction v at h[v * n_pts]
    double t7[kNTheta] = {th[0], th[1], th[2], th[3], th[4], 1.0, 1.0};
    double dc[kNTheta][kNBasis];
    basis_dcoef(t7, a.ph, dc);
    double* g = a.grad + (size_t)p * a.n_theta;
    double hb[10];
#pragma unroll
    for (int b = 0; b < 10; ++b) hb[b] = h[(size_t)b * a.n_pts];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < 10; ++b) v += dc[i][b] * hb[b];
        g[i] = v;
    }
    for (int i = 5; i < a.n_theta; ++i) g[i] = h[(size_t)(10 + i - 5) * a.n_pts];  // R_k, Q_q
    for (int i = 0; i < a.n_theta; ++i)
        if (a.pull_sigma[i] > 0.0)
            g[i] += 2.0 * (th[i] - a.pull_mean[i]) / (a.pull_sigma[i] * a.pull_sigma[i]);
}

}  // namespace

hipError_t launch_tmpl_mdata(const TmplMultiDataArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_tmpl_mdata, dim3((a.n_reco + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tmpl_meval(const TmplMultiEvalArgs& a, int n_split, hipStream_t s) {
    if (a.K < 1 || a.K > kTmplMaxComp || a.B < 0 || a.B > kTmplMaxBkg || (a.hpart && a.mu))
        return hipErrorInvalidValue;
    const dim3 grid((a.n_pts + kTmplWave - 1) / kTmplWave, n_split);
    const bool small = a.K <= kTmplSmallComp && a.B <= kTmplSmallBkg;
    constexpr int KS = kTmplSmallComp, BS = kTmplSmallBkg, KL = kTmplMaxComp, BL = kTmplMaxBkg;
    if (a.hpart) {
        if (small) hipLaunchKernelGGL((k_tmpl_meval<true, false, KS, BS>), grid, dim3(kTmplWave), 0, s, a);
        else hipLaunchKernelGGL((k_tmpl_meval<true, false, KL, BL>), grid, dim3(kTmplWave), 0, s, a);
    } else if (a.mu) {
        hipLaunchKernelGGL((k_tmpl_meval<false, true, KL, BL>), grid, dim3(kTmplWave), 0, s, a);
    } else {
        if (small) hipLaunchKernelGGL((k_tmpl_meval<false, false, KS, BS>), grid, dim3(kTmplWave), 0, s, a);
        else hipLaunchKernelGGL((k_tmpl_meval<false, false, KL, BL>), grid, dim3(kTmplWave), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_tmpl_mfinal(const TmplMultiFinalArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_tmpl_mfinal, dim3((a.n_pts + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tmpl_fold(const TmplFoldArgs& a, int n_slab, hipStream_t s) {
    hipLaunchKernelGGL(k_tmpl_fold, dim3((a.n_reco + 255) / 256, n_slab), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tmpl_records(const TmplRecArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_tmpl_records, dim3((a.n_reco + 255) / 256, kTmplCols), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tmpl_data(const TmplDataArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_tmpl_data, dim3((a.n_reco + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tmpl_eval(const TmplEvalArgs& a, int n_split, hipStream_t s) {
    const dim3 grid((a.n_pts + kTmplWave - 1) / kTmplWave, n_split);
    if (a.hpart && a.mu) return hipErrorInvalidValue;
    if (a.hpart)
        hipLaunchKernelGGL((k_tmpl_eval<true, false>), grid, dim3(kTmplWave), 0, s, a);
    else if (a.mu)
        hipLaunchKernelGGL((k_tmpl_eval<false, true>), grid, dim3(kTmplWave), 0, s, a);
    else
        hipLaunchKernelGGL((k_tmpl_eval<false, false>), grid, dim3(kTmplWave), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tmpl_reduce(const TmplReduceArgs& a, hipStream_t s) {
    const dim3 grid((a.n_pts + kTmplWave - 1) / kTmplWave, a.hpart ? 1 + a.n_acc : 1);
    hipLaunchKernelGGL(k_tmpl_reduce, grid, dim3(kTmplWave), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tmpl_final(const TmplFinalArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_tmpl_final, dim3((a.n_pts + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_wgen(const WgenArgs& a, hipStream_t s) {
    dim3 grid((a.ldw + 255) / 256, (a.n_t + kWgenRows - 1) / kWgenRows);
    hipLaunchKernelGGL(k_wgen, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int MODE, int BM, int BN>
static hipError_t launch_one(const GemmProb* probs, const GemmTile* tiles,
                             int n_tiles, unsigned* ctr, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_gemm<MODE, BM, BN>), dim3(grid), dim3(kGemmThreads), 0, s,
                       probs, tiles, n_tiles, ctr);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_mode(int cfg, const GemmProb* probs, const GemmTile* tiles,
                              int n_tiles, unsigned* ctr, int grid, hipStream_t s) {
    switch (cfg) {
        case 0: return launch_one<MODE, 128, 128>(probs, tiles, n_tiles, ctr, grid, s);
        case 1: return launch_one<MODE, 64, 128>(probs, tiles, n_tiles, ctr, grid, s);
        case 2: return launch_one<MODE, 128, 64>(probs, tiles, n_tiles, ctr, grid, s);
        case 3: return launch_one<MODE, 64, 64>(probs, tiles, n_tiles, ctr, grid, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gemm(int mode, int cfg, const GemmProb* probs, const GemmTile* tiles,
                       int n_tiles, unsigned* ctr, int grid, hipStream_t s) {
    if (mode == kModeAdj) return launch_mode<kModeAdj>(cfg, probs, tiles, n_tiles, ctr, grid, s);
    return launch_mode<kModeNll>(cfg, probs, tiles, n_tiles, ctr, grid, s);
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((a.n_pts + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adj_contract(const ContractArgs& a, hipStream_t s) {
    const int nch = ctr_chunks(a.n_t);
    hipLaunchKernelGGL(k_adj_contract, dim3((a.n_pts + 15) / 16, nch), dim3(256), 0, s, a);
    if (nch > 1)
        hipLaunchKernelGGL(k_adj_final, dim3((a.n_pts + kFinPts - 1) / kFinPts), dim3(256), 0, s,
                           a, nch);
    return hipGetLastError();
}

}  // namespace nr

namespace nr {

// Persistent grid: as many work-groups as can be resident at once.
template <int MODE, int BM, int BN>
static int per_cu() {
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_gemm<MODE, BM, BN>,
                                                       kGemmThreads, 0);
    return n;
}

int gemm_grid(int mode, int cfg, int n_tiles) {
    int dev = 0, cus = 0, pc = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const bool adj = mode == kModeAdj;
    switch (cfg) {
        case 0: pc = adj ? per_cu<kModeAdj, 128, 128>() : per_cu<kModeNll, 128, 128>(); break;
        case 1: pc = adj ? per_cu<kModeAdj, 64, 128>() : per_cu<kModeNll, 64, 128>(); break;
        case 2: pc = adj ? per_cu<kModeAdj, 128, 64>() : per_cu<kModeNll, 128, 64>(); break;
        default: pc = adj ? per_cu<kModeAdj, 64, 64>() : per_cu<kModeNll, 64, 64>(); break;
    }
    if (cus <= 0) cus = 256;
    if (pc <= 0) pc = 1;
    int g = cus * pc;
    if (g > n_tiles) g = n_tiles;
    return g < 1 ? 1 : g;
}

int gemm_tile_m(int cfg) { return (cfg == 1 || cfg == 3) ? 64 : 128; }
int gemm_tile_n(int cfg) { return (cfg == 2 || cfg == 3) ? 64 : 128; }

}  // namespace nr
