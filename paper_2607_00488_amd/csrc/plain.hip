// Single-point path on gfx950: E-integral, weights, HBM-streaming fold,
// Poisson likelihood reduction, and the adjoint of the fold.
#include "common.h"

#include <cmath>

namespace nr {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// 16-byte streaming load without cache allocation (the adjoint pass).
__device__ inline float4 ld_stream(const float4* p) {
    const v4f v = __builtin_nontemporal_load(reinterpret_cast<const v4f*>(p));
    return make_float4(v.x, v.y, v.z, v.w);
}

// 16-byte load of R in the fold.  A response that the 256 MB Infinity Cache
// can partly hold is read with ordinary (allocating) loads, so the rows read
// last stay cached for the next point, which walks its tile in the opposite
// direction; a much larger one (the stacked multi-component responses) is
// streamed without allocating.  Measured on MI355X: 16384 x 4096 (268 MB),
// 41.1 us per point with ordinary loads against 43.3 us non-temporal, 38.5
// us with the alternating direction; five stacked responses (1.34 GB),
// 6.68 TB/s non-temporal against 6.45 TB/s ordinary.
__device__ inline float4 ld_row(const float4* p, bool nt) {
    return nt ? ld_stream(p) : *p;
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

// The roles of the single-point path run in one kernel, k_step, as separate
// ranges of work-groups of the same launch: the node table of one point,
// the weights of another, the R-streaming fold of a third and the
// likelihood reduction of a fourth.  Consecutive launches on one stream
// form a software pipeline with no cross-stream waits: launch k builds the
// table of point k, the weights of point k - 1, folds point k - 2 and
// reduces point k - 3; stream order is the only synchronisation.
constexpr int kStepThreads = 512;          // 8 waves in every role
constexpr int kStepWaves = kStepThreads / 64;
constexpr int kFoldTile4 = kStepThreads;   // float4 columns per fold tile
constexpr int kFoldUnroll = 8;
constexpr int kFoldMaxRows = 2048;
constexpr int kFinCols = 64;               // columns per reduction group
constexpr int kFinSplit = kStepThreads / kFinCols;  // threads per column
constexpr int kSmemFold = kFoldMaxRows;
constexpr int kSmemScan = 4 * kStepWaves;
constexpr int kSmemFin = kFinSplit * kFinCols;
constexpr int kSmemDoubles = kSmemFold > kSmemFin ? kSmemFold : kSmemFin;
static_assert(kSmemScan <= kSmemDoubles, "scan scratch");
static_assert(kStepRows == kStepThreads, "one recoil row per thread");

// ---------------------------------------------------------------- a1
// Eq. (fT) as a sum over the nodes a recoil bin can reach.  For node j the
// flux-weighted cross section is a Laurent polynomial in T with
// coefficients c_j = (a0, a1, a2, am) (node_coef), and the nodes of a source
// that reach T_l are those with index >= jmin(k, l), a suffix of the
// E-ordered nodes.  So S_theta(T_l) = sum_k C_k(jmin(k, l)) . (1, T, T^2, 1/T)
// with the suffix sums C_k(j) = sum_{i >= j} c_i: the same quadrature sum,
// summed in another order.  A source's nodes are split into chunks of 512
// counted from the high-energy end, one work-group per chunk: each wave
// scans its 64 nodes with shuffles and the wave totals of the chunk meet in
// LDS.  Table entry j + k holds the suffix sum of node j within its chunk,
// and the chunk's total goes to ctot[k][chunk]; the weights role adds the
// totals of the chunks above (higher energies) when it reads an entry.  The
// entry after the source's last node is zero (no reachable node).
__device__ inline void suffix_scan_wave(double& x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const double y = __shfl_down(x, o, 64);
        if (lane + o < 64) x += y;
    }
}

__device__ void scan_role(const ScanArgs& a, int blk, double* smem) {
    double4* wt = reinterpret_cast<double4*>(smem);          // [8]
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int k = a.blocks[2 * blk], ch = a.blocks[2 * blk + 1];
    double th[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) th[i] = a.theta[i];
    const double f = a.srcGroup[k] ? a.theta[5] : 1.0;
    const int off = a.srcOff[k], end = a.srcOff[k + 1];
    double4* tab = a.table + k;  // entry j + k for global node j
    if (ch == 0 && threadIdx.x == 0) tab[end] = make_double4(0.0, 0.0, 0.0, 0.0);
    // this chunk: nodes [hi - 512, hi) of the source; wave 7 holds the
    // highest 64
    const int hi = end - ch * kStepThreads;
    const int j = hi - kStepThreads + (int)threadIdx.x;
    const bool have = j >= off;
    double4 c = make_double4(0.0, 0.0, 0.0, 0.0);
    if (have) {
        const NodeCoef q = node_coef(a.nodeIE[j], a.nodeW[j] * f, a.nodePe[j], th, a.ph);
        c = make_double4(q.a0, q.a1, q.a2, q.am);
    }
    suffix_scan_wave(c.x, lane);
    suffix_scan_wave(c.y, lane);
    suffix_scan_wave(c.z, lane);
    suffix_scan_wave(c.w, lane);
    if (lane == 0) wt[wave] = c;  // lane 0 holds the wave's total
    __syncthreads();
    double4 add = make_double4(0.0, 0.0, 0.0, 0.0);
    for (int w = kStepWaves - 1; w > wave; --w) {
        const double4 t = wt[w];
        add.x += t.x;
        add.y += t.y;
        add.z += t.z;
        add.w += t.w;
    }
    if (have)
        tab[j] = make_double4(c.x + add.x, c.y + add.y, c.z + add.z, c.w + add.w);
    if (threadIdx.x == 0) {
        double4 tot = make_double4(0.0, 0.0, 0.0, 0.0);
        for (int w = kStepWaves - 1; w >= 0; --w) {
            const double4 t = wt[w];
            tot.x += t.x;
            tot.y += t.y;
            tot.z += t.z;
            tot.w += t.w;
        }
        a.ctot[(size_t)k * a.max_chunks + ch] = tot;
    }
}

// ---------------------------------------------------------------- a2
// S_theta(T_l) from the table (sources added in order, then one Laurent
// evaluation), then Eqs. (fT_norm), (reweight_factor): w_l = S_theta /
// S_SM, w_l := 1 where S_SM = 0, and the fold vector v_l = m_l w_l.  The SM
// reference is formed by this same code, so w = 1 exactly at theta_SM.
__device__ void rows_role(const RowArgs& a, int blk) {
    const int r = blk * kStepThreads + (int)threadIdx.x;
    if (r >= a.n_comp * a.n_t) return;
    const int c = r / a.n_t, l = r - c * a.n_t;
    double4 s = make_double4(0.0, 0.0, 0.0, 0.0);
    // Sources in groups of G: the node indices of a group, then its table
    // entries, are loaded together rather than one source after another
    // (each step is a dependent load; in sequence they set this role's
    // time).  The sums keep their order.
    constexpr int G = 8;
    const int q0 = a.compOff[c], q1 = a.compOff[c + 1];
    for (int g0 = q0; g0 < q1; g0 += G) {
        int kk[G], jj[G];
#pragma unroll
        for (int u = 0; u < G; ++u) kk[u] = g0 + u < q1 ? a.compSrc[g0 + u] : -1;
#pragma unroll
        for (int u = 0; u < G; ++u)
            jj[u] = kk[u] >= 0 ? a.jmin[(size_t)kk[u] * a.n_t + l] : 0;
        double4 t[G];
#pragma unroll
        for (int u = 0; u < G; ++u)
            t[u] = kk[u] >= 0 ? a.table[jj[u] + kk[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
        for (int u = 0; u < G; ++u) {
            if (kk[u] < 0) continue;
            // totals of the chunks above node jj's chunk (none for the empty
            // entry at the source's end)
            const int end = a.srcOff[kk[u] + 1];
            const int nch = jj[u] < end ? (end - 1 - jj[u]) / kStepThreads : 0;
            for (int h = 0; h < nch; ++h) {
                const double4 v = a.ctot[(size_t)kk[u] * a.max_chunks + h];
                t[u].x += v.x;
                t[u].y += v.y;
                t[u].z += v.z;
                t[u].w += v.w;
            }
            s.x += t[u].x;
            s.y += t[u].y;
            s.z += t[u].z;
            s.w += t[u].w;
        }
    }
    const double T = a.tc[l];
    const double S = fma(T, fma(T, s.z, s.y), s.x) + s.w / T;
    if (a.out_s) {
        a.out_s[r] = S;
        return;
    }
    const double ssm = a.ssm[r];
    const double w = ssm > 0.0 ? S / ssm : 1.0;
    if (a.out_w) a.out_w[r] = w;
    // multi-component form: the component's rate nuisance scales its rows
    const double mr = a.rate_index >= 0 ? a.mrow[r] * a.theta[a.rate_index + c]
                                        : a.mrow[r];
    a.v[r] = mr * w;
}

// ------------------------------------------------------------------ a3
// Fold through the response (Eqs. (Rij), (fNp_reweight), (mu_total)).
// Tile (rb, cc) covers rows [rb*rows, +rows) and 2048 columns: wave w owns
// the 64 float4 columns cc*512 + w*64 + lane and walks every row of the
// tile, eight rows in flight (the first eight issued before the weights are
// staged), so each row of the tile is read as one contiguous 8 KB run by
// the work-group.  Consecutive points walk the rows in opposite directions
// (the sums then add the rows in opposite orders: results of a point differ
// between the two by rounding only, ~1e-16 relative).  The per-row weights v_l = m_l w_l sit in LDS.  R is FP32
// in HBM; products and sums are FP64, which the full-rate FP64 vector units
// of gfx950 absorb at no cost to this bandwidth-bound loop.  Every lane
// writes its four column sums as the tile's partial row; no cross-work-group
// synchronisation happens here (the reduction role of the next launch adds
// the partial rows).
__device__ void fold_role(const FoldArgs& a, int rb, int cc, double* smem) {
    // walk position r reads row rr(r) of the tile: first to last, or last to
    // first when a.reverse (every other point of a scan)
    double* vs = smem;                                         // [2048]
    const int row0 = rb * a.rows_per_wg;
    int nrows = a.n_t - row0;
    if (nrows > a.rows_per_wg) nrows = a.rows_per_wg;
    const int tid = threadIdx.x;
    const int ld4 = a.ldr >> 2;
    const int c4 = cc * kFoldTile4 + tid;
    const bool incol = c4 < ld4;
    // with band skipping, columns outside the tile's non-zero band hold
    // exact zeros: their sums are zero without reading them
    const int* bd = a.band ? a.band + 2 * ((size_t)cc * a.n_rb + rb) : nullptr;
    const bool colok = incol && (!bd || (c4 >= bd[0] && c4 < bd[1]));
    const float4* __restrict__ Rp =
        reinterpret_cast<const float4*>(a.R) + (size_t)row0 * ld4 + c4;
    constexpr int U = kFoldUnroll;
    const bool rev = a.reverse != 0;
    const bool nt = a.stream_nt != 0;
    auto rr = [&](int r) { return rev ? nrows - 1 - r : r; };
    float4 x[U];
    int r = 0;
    bool full = colok && U <= nrows;
    if (full) {
#pragma unroll
        for (int q = 0; q < U; ++q) x[q] = ld_row(Rp + (size_t)rr(q) * ld4, nt);
    }
    for (int q = tid; q < nrows; q += kStepThreads) vs[q] = a.v[row0 + q];
    __syncthreads();
    if (!incol) return;
    if (!colok) {
        double* z = a.colpart + (size_t)rb * a.ldr + 4 * c4;
        z[0] = z[1] = z[2] = z[3] = 0.0;
        return;
    }
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
    while (full) {
#pragma unroll
        for (int q = 0; q < U; ++q) {
            const double v = vs[rr(r + q)];
            acc0 = fma((double)x[q].x, v, acc0);
            acc1 = fma((double)x[q].y, v, acc1);
            acc2 = fma((double)x[q].z, v, acc2);
            acc3 = fma((double)x[q].w, v, acc3);
        }
        r += U;
        full = r + U <= nrows;
        if (full) {
#pragma unroll
            for (int q = 0; q < U; ++q) x[q] = ld_row(Rp + (size_t)rr(r + q) * ld4, nt);
        }
    }
    for (; r < nrows; ++r) {
        const float4 z = ld_row(Rp + (size_t)rr(r) * ld4, nt);
        const double v = vs[rr(r)];
        acc0 = fma((double)z.x, v, acc0);
        acc1 = fma((double)z.y, v, acc1);
        acc2 = fma((double)z.z, v, acc2);
        acc3 = fma((double)z.w, v, acc3);
    }
    double* o = a.colpart + (size_t)rb * a.ldr + 4 * c4;
    o[0] = acc0;
    o[1] = acc1;
    o[2] = acc2;
    o[3] = acc3;
}

// ------------------------------------------------------------- a4, a5
// Poisson likelihood (Eq. (logL)) from the fold partials.  Group cc owns 64
// columns; eight threads per column add every eighth partial row, the eight
// sums meet in LDS in a fixed order, and wave 0 forms mu_j (backgrounds and
// mask of the multi-component form included), the deviance
// mu - n + n ln(n/mu) and a_j = d(-2lnL)/d mu_j, and writes the group's
// sums.  No fence and no counter: the final role of the next launch adds
// the group sums.  Deterministic: no float atomics.
__device__ void finish_role(const FoldArgs& a, int cc, double* smem) {
    double (*ps)[kFinCols] = reinterpret_cast<double (*)[kFinCols]>(smem);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int ci = tid % kFinCols, qd = tid / kFinCols;
    const int col = cc * kFinCols + ci;
    // up to 16 partial rows per thread are loaded before any is added
    double s = 0.0;
    if (col < a.n_reco) {
        constexpr int G = 16;
        for (int q0 = qd; q0 < a.n_rb; q0 += G * kFinSplit) {
            double v[G];
#pragma unroll
            for (int k = 0; k < G; ++k) {
                const int q = q0 + k * kFinSplit;
                v[k] = q < a.n_rb ? a.colpart[(size_t)q * a.ldr + col] : 0.0;
            }
#pragma unroll
            for (int k = 0; k < G; ++k) s += v[k];
        }
    }
    ps[qd][ci] = s;
    __syncthreads();
    if (wave != 0) return;
    double dev = 0.0, gb = 0.0;
    if (col < a.n_reco) {
        double fold = 0.0;
#pragma unroll
        for (int k = 0; k < kFinSplit; ++k) fold += ps[k][ci];
        double mu = fold, bj = 0.0;
        for (int q = 0; q < a.n_bkg; ++q) {
            const double t = a.b[(size_t)q * a.n_reco + col];
            mu += a.theta[a.bkg_index + q] * t;
            bj = t;  // the single-template form's b_j (gradient of f_bkg)
        }
        if (a.mask) mu *= a.mask[col];
        const double nj = a.n[col];
        if (a.out_mu) a.out_mu[col] = mu;
        if (nj > 0.0)
            dev = mu > 0.0 ? (mu - nj + nj * log(nj / mu)) : INFINITY;
        else
            dev = mu;
        // an empty bin's term is 2 mu_j: its derivative is 2 at any mu_j
        const double aj = nj > 0.0 ? 2.0 * (1.0 - nj / mu) : 2.0;
        if (a.out_a) a.out_a[col] = aj;
        gb = aj * bj;
    } else if (col < a.ldr && a.out_a) {
        a.out_a[col] = 0.0;
    }
    dev = wave_sum(dev);
    gb = wave_sum(gb);
    if (lane == 0) {
        a.chunk_dev[cc] = dev;
        a.chunk_gb[cc] = gb;
    }
}

// a5: -2lnL = 2 (sum of the group deviances + C_data) + pulls, and
// sum_j a_j b_j for the gradient.  Lane q adds the group sums q, q + 64, ...;
// the butterfly then adds the lanes in a fixed order.
__device__ void final_role(const FoldArgs& a) {
    if (threadIdx.x >= 64) return;
    const int lane = threadIdx.x;
    double d = 0.0, g = 0.0;
    for (int q = lane; q < a.n_cc; q += 64) {
        d += a.chunk_dev[q];
        g += a.chunk_gb[q];
    }
    d = wave_sum(d);
    g = wave_sum(g);
    if (lane == 0) {
        double pulls = 0.0;
        for (int i = 0; i < a.n_theta; ++i)
            if (a.pull_sigma[i] > 0.0) {
                const double z = (a.theta[i] - a.pull_mean[i]) / a.pull_sigma[i];
                pulls += z * z;
            }
        a.out_nll[0] = 2.0 * d + 2.0 * a.cdata + pulls;
        if (a.out_gb) a.out_gb[0] = g;
    }
}

// Work-group 0 (when nb_final = 1) completes the likelihood of one point,
// the next nb_fin reduce the fold of another, the next nb_scan (one per
// source) build the node table of a third, the next nb_rows form the
// weights of a fourth and the rest fold a fifth.  The short roles come
// first: their few dependent loads go out before the fold tiles saturate
// HBM, and every work-group of a launch is resident at once, so they finish
// well inside the fold.  No role of a launch waits for another: nothing in
// the kernel fences.  The role branch is uniform over the work-group.
__device__ __forceinline__ void step_body(const StepArgs& a) {
    __shared__ __attribute__((aligned(16))) double smem[kSmemDoubles];
    int b = blockIdx.x;
    if (b < a.nb_final) {
        final_role(a.fnl);
        return;
    }
    b -= a.nb_final;
    if (b < a.nb_fin) {
        finish_role(a.fin, b, smem);
        return;
    }
    b -= a.nb_fin;
    if (b < a.nb_scan) {
        scan_role(a.scan, b, smem);
        return;
    }
    b -= a.nb_scan;
    if (b < a.nb_rows) {
        rows_role(a.rows, b);
        return;
    }
    b -= a.nb_rows;
    fold_role(a.fold, b % a.fold.n_rb, b / a.fold.n_rb, smem);
}

// The steady-state launch of the pipeline (all four roles) and every other
// launch (pipeline fill and drain, single stages) are separate symbols so
// that profiles report the steady state on its own.
__global__ __launch_bounds__(kStepThreads) void k_step(StepArgs a) {
    step_body(a);
}

__global__ __launch_bounds__(kStepThreads) void k_step_part(StepArgs a) {
    step_body(a);
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
        // with band skipping only the 64-column groups that meet the row's
        // non-zero band are read; each lane keeps its columns, and the
        // skipped terms are exact zeros, so the sums are unchanged
        int c0 = lane, c1 = ld4;
        if (a.rowband) {
            c0 = a.rowband[2 * (size_t)l] / 64 * 64 + lane;
            c1 = a.rowband[2 * (size_t)l + 1];
        }
        for (int c = c0; c < c1; c += 64) {
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

hipError_t launch_step(const StepArgs& a, hipStream_t s) {
    if (a.nb_fold > 0 &&
        (a.fold.rows_per_wg > kFoldMaxRows || a.fold.rows_per_wg <= 0 ||
         a.fold.n_fc != (a.fold.ldr / 4 + kFoldTile4 - 1) / kFoldTile4 ||
         a.nb_fold != a.fold.n_rb * a.fold.n_fc ||
         (size_t)a.fold.n_rb * a.fold.rows_per_wg < (size_t)a.fold.n_t))
        return hipErrorInvalidValue;
    if (a.nb_fin > 0 && (a.nb_fin != a.fin.n_cc ||
                         a.fin.n_cc != (a.fin.n_reco + kFinCols - 1) / kFinCols))
        return hipErrorInvalidValue;
    if (a.nb_rows > 0 &&
        a.nb_rows != (a.rows.n_comp * a.rows.n_t + kStepThreads - 1) / kStepThreads)
        return hipErrorInvalidValue;
    if (a.nb_final < 0 || a.nb_final > 1) return hipErrorInvalidValue;
    const int grid = a.nb_fold + a.nb_rows + a.nb_scan + a.nb_fin + a.nb_final;
    if (grid <= 0) return hipSuccess;
    const bool full = a.nb_fold > 0 && a.nb_rows > 0 && a.nb_scan > 0 && a.nb_fin > 0 &&
                      a.nb_final > 0;
    if (full)
        hipLaunchKernelGGL(k_step, dim3(grid), dim3(kStepThreads), 0, s, a);
    else
        hipLaunchKernelGGL(k_step_part, dim3(grid), dim3(kStepThreads), 0, s, a);
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
