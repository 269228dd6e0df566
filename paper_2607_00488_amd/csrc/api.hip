// C-ABI context: validation, theta-independent setup (Sec. III.A last
// paragraph and Sec. III.B: the SM reference and the response are built once
// and kept resident), stream-ordered launches, HIP-graph replay, errors.
#include "batched.h"
#include "ess.h"
#include "mlp.h"
#include "../../include/nureweight.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>
#include <sys/stat.h>

// Workspace of the allocation-free entry point nr_eval_nll_dev_noalloc: the
// single-point pipeline's node tables, fold vectors, partial sums and
// adjoint buffers for any context on the device, in place of the context's
// own.  One copy per device, resident until the process ends.  Host code
// never passes this name to a kernel or a copy: it uses the device address
// hipGetSymbolAddress returns on each device (g_scratch_dev).
static __device__ __align__(256) double scratch[NR_NOALLOC_WORKSPACE_BYTES / sizeof(double)];

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                        \
    do {                                                                    \
        hipError_t e_ = (expr);                                             \
        if (e_ != hipSuccess)                                               \
            return fail(NR_EHIP, "%s: %s (%s:%d)", #expr,                   \
                        hipGetErrorString(e_), __FILE__, __LINE__);         \
    } while (0)

template <class T>
int dalloc(T** p, size_t n) {
    if (*p) {  // the old buffer may still be read by in-flight work
        (void)hipDeviceSynchronize();
        (void)hipFree(*p);
        *p = nullptr;
    }
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(NR_ENOMEM, "hipMalloc(%zu bytes): %s", n * sizeof(T),
                    hipGetErrorString(e));
    }
    return 0;
}

template <class T>
void dfree(T** p) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
}

// A NULL stream argument of the _dev entry points means the HIP default
// stream.  Work cannot be captured on it, so it runs on an internal stream
// ordered after everything already on the default stream, and the default
// stream waits for its end.
struct Bridge {
    hipStream_t work = nullptr;
    hipEvent_t out = nullptr;
    bool on = false;
};

int bridge_begin(Bridge& b, void* user, hipStream_t internal, hipEvent_t in,
                 hipEvent_t out) {
    if (user) {
        b.work = (hipStream_t)user;
        b.on = false;
        return 0;
    }
    b.work = internal;
    b.out = out;
    b.on = true;
    HIPCHK(hipEventRecord(in, nullptr));
    HIPCHK(hipStreamWaitEvent(internal, in, 0));
    return 0;
}

int bridge_end(Bridge& b) {
    if (!b.on) return 0;
    HIPCHK(hipEventRecord(b.out, b.work));
    HIPCHK(hipStreamWaitEvent(nullptr, b.out, 0));
    return 0;
}

bool finite_all(const double* p, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

using GraphKey = std::tuple<const void*, int, void*, void*, void*, void*>;

}  // namespace

// One process-wide lock around the host side of every entry point (taken
// again, recursively, when an entry point calls another).  Calls from
// different threads then run their host work one at a time: a call may open
// a graph capture on its stream, and the HIP runtime fails a capture when
// another thread issues a default-stream operation (a synchronous copy, a
// set) while it is open.  Device work of different calls still overlaps.
namespace nr {
std::recursive_mutex& api_mutex() {
    static std::recursive_mutex m;
    return m;
}
}  // namespace nr

namespace {

struct ApiLock {
    std::lock_guard<std::recursive_mutex> g{nr::api_mutex()};
};

// Incremented whenever a context's device buffers may have moved; cached
// grouped-launch plans built under an older epoch are rebuilt.
std::atomic<unsigned long> g_epoch{1};

// Device address of the static workspace on each device, looked up once per
// device by the first nr_create on it (under the API lock).
std::vector<double*> g_scratch_dev;

int lookup_scratch(int device, int ndev) {
    if ((int)g_scratch_dev.size() < ndev) g_scratch_dev.resize(ndev, nullptr);
    if (g_scratch_dev[device]) return 0;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(NR_EHIP, "hipGetSymbolAddress(static workspace) on device %d: %s",
                    device, hipGetErrorString(e));
    g_scratch_dev[device] = static_cast<double*>(p);
    return 0;
}

// One grouped launch over several analyses: GEMM problem tables, tile lists
// and the captured graph of the whole batched evaluation.
struct BatchPlan {
    nr::GemmProb* d_probs_f = nullptr;
    nr::GemmTile* d_tiles_f = nullptr;
    nr::GemmProb* d_probs_a = nullptr;
    nr::GemmTile* d_tiles_a = nullptr;
    int n_tiles_f = 0, n_tiles_a = 0, grid_f = 1, grid_a = 1;
    int cfg = 0;  // GEMM tile configuration (see batched.h)
    hipGraphExec_t graph = nullptr;
    unsigned long epoch = 0;
};

}  // namespace

struct nr_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;  // default-stream bridge
    double* d_v[2] = {nullptr, nullptr};  // [n_t] fold vectors, by parity
    nr::Phys ph{};
    // sources and grid
    bool have_src = false, have_rsp = false, have_data = false;
    int n_src = 0, n_t = 0, n_nodes = 0, n_blocks = 0;
    double t_lo = 0, t_hi = 0;
    std::vector<int> src_off, src_n, src_group;
    std::vector<double> hE, hW, hPe, tc;
    std::vector<int> jmin;
    std::vector<double> ssm, basis;
    double *d_E = nullptr /* 1/E per node */, *d_W = nullptr, *d_Pe = nullptr, *d_tc = nullptr;
    double *d_ssm = nullptr, *d_basis = nullptr;
    int *d_group = nullptr, *d_jmin = nullptr, *d_srcoff = nullptr;
    double* d_table[2] = {nullptr, nullptr};  // [n_nodes + n_src] double4, by parity
    // node-scan work-groups: (source, 512-node chunk) pairs, and the chunk
    // totals [n_src][max_chunks] double4, by parity
    int nb_scan = 0, max_chunks = 1;
    int* d_scanblk = nullptr;
    double* d_ctot[2] = {nullptr, nullptr};
    // response
    int n_reco = 0, ldr = 0;
    float* d_R = nullptr;
    // per response row the float4 columns [lo, hi) holding its non-zero
    // entries (host and device), and per fold tile the same for its rows;
    // read by the fold and the adjoint only when band skipping is on
    std::vector<int> rowband;
    int *d_rowband = nullptr, *d_tileband = nullptr;
    bool skip_zero = false;
    bool m_user = false;
    double n_sig = 0;
    std::vector<double> mrow;
    double* d_mrow = nullptr;
    // data
    double *d_n = nullptr, *d_b = nullptr;
    double cdata = 0;
    double lgsum = 0;  // sum_j lnGamma(n_j + 1)
    double pull_mean[nr::kMaxTheta] = {0}, pull_sigma[nr::kMaxTheta] = {0};
    // multi-component form (Eqs. (Rij), (fNp_reweight), (mu_total)): the
    // component responses are stacked row-wise in d_R, n_rows = n_comp * n_t
    bool multi = false;
    int n_theta = NR_NTHETA, n_comp = 1, n_bkg = 1, n_rows = 0;
    std::vector<int> comp_off, comp_src;
    int *d_compoff = nullptr, *d_compsrc = nullptr, *d_group0 = nullptr;
    double *d_ssmc = nullptr, *d_bkg = nullptr, *d_mask = nullptr;
    // fold / adjoint scratch
    int rows_per_wg = 0, n_rb = 0, n_fc = 0, n_cc = 0, adj_grid = 0;
    double *d_colpart = nullptr;  // [2][n_rb][ldr]
    double *d_chunk_dev = nullptr, *d_chunk_gb = nullptr;
    double* d_a = nullptr;
    double *d_gb = nullptr, *d_jpart = nullptr;
    // staging for the synchronous entry points
    double *d_th = nullptr, *d_out = nullptr, *d_grad = nullptr;
    double *d_mu = nullptr, *d_w = nullptr;
    size_t cap_pts = 0, cap_mu = 0, cap_w = 0;
    // pinned host staging of the synchronous likelihood entry points: the
    // kernels read theta from it and write -2lnL and the gradient into it
    // directly, so a call needs no copy between host and device
    double *h_th = nullptr, *h_out = nullptr, *h_grad = nullptr;
    double *hd_th = nullptr, *hd_out = nullptr, *hd_grad = nullptr;  // device views
    size_t h_cap = 0;
    double* d_thsm = nullptr;
    double* d_tnll = nullptr;  // [1] output of timing-only launches
    double* d_nev = nullptr;   // [n_t] MC events per true recoil row
    bool have_nev = false;
    // graphs
    bool use_graph = true;
    std::map<GraphKey, hipGraphExec_t> graphs;
    // batched (GEMM) path workspace
    int b_cap = 0, b_ldw = 0, b_nnt = 0;
    bool b_grad = false;
    double* d_wt = nullptr;     // [n_t][ldw]   weights, K-major
    double* d_bpart = nullptr;  // [cap][n_nt]  deviance partials
    double* d_bpgb = nullptr;   // [cap][n_nt]  sum a b partials
    double* d_bat = nullptr;    // [ldr][ldw]   d(-2lnL)/d mu, j-major
    double* d_bu = nullptr;     // [cap][n_t]   adjoint rows
    double *d_bth = nullptr, *d_bnll = nullptr, *d_bgrad = nullptr, *d_bmu = nullptr;
    size_t b_cap_mu = 0;
    unsigned* d_gctr = nullptr;  // [4] tile counters (forward, adjoint)
    std::map<std::vector<const void*>, BatchPlan*> plans;
    // template form: folded basis templates and the data, per reco bin
    bool tmpl_ok = false, tmpl_data_ok = false;
    double* d_trec = nullptr;  // [n_reco][kTmplRec]
    double *d_tdp = nullptr, *d_thp = nullptr;  // evaluation partials
    double* d_tred = nullptr;                   // [1 + kTmplCols][points] slice sums
    size_t t_cap_d = 0, t_cap_h = 0, t_cap_r = 0;
};

namespace {

// Graph executables and the tile tables their kernels read may still be in
// flight (the _dev entry points return without waiting): wait for the device
// before destroying or freeing them.
void free_plan(BatchPlan* p) {
    if (!p) return;
    (void)hipDeviceSynchronize();
    if (p->graph) (void)hipGraphExecDestroy(p->graph);
    if (p->d_probs_f) (void)hipFree(p->d_probs_f);
    if (p->d_tiles_f) (void)hipFree(p->d_tiles_f);
    if (p->d_probs_a) (void)hipFree(p->d_probs_a);
    if (p->d_tiles_a) (void)hipFree(p->d_tiles_a);
    delete p;
}

void clear_graphs(nr_ctx* c) {
    if (!c->graphs.empty() || !c->plans.empty()) (void)hipDeviceSynchronize();
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    for (auto& kv : c->plans) free_plan(kv.second);
    c->plans.clear();
    ++g_epoch;
}

int set_device(nr_ctx* c) {
    HIPCHK(hipSetDevice(c->device));
    return 0;
}

nr::Phys make_phys(const nr_physics* p) {
    nr_physics d{0.51099895, 1.1663788e-11, 0.23122, 1.0 / 137.035999084, 0.5};
    if (p) d = *p;
    const double pi = 3.14159265358979323846;
    nr::Phys ph;
    ph.me = d.me;
    ph.sw2 = d.sw2;
    ph.tau_frac = d.tau_frac;
    // ratio of the magnetic prefactor pi alpha^2/m_e^2 (Eq. (xs_mm)) with
    // (mu_nu/mu_B)^2 = 1e-22 m2 to the weak prefactor 2 G_F^2 m_e / pi
    ph.cmm = pi * pi * d.alpha_em * d.alpha_em * 1e-22 /
             (2.0 * d.gf * d.gf * d.me * d.me * d.me);
    ph.gLe = 0.5 + d.sw2;   // Sec. II.A tree-level couplings
    ph.gLm = -0.5 + d.sw2;
    ph.gR = d.sw2;
    return ph;
}

// Two-body kinematics: recoil T is reachable from neutrino energy E iff
// T <= 2E^2 / (m_e + 2E).
inline bool reach(double me, double E, double T) {
    return T <= 2.0 * E * E / (me + 2.0 * E);
}

// The ten theta-independent pieces of source k's recoil spectrum at bin l:
// per flavour the sums of nu P_a, nu P_a y^2 and nu P_a x over the reachable
// nodes (the coefficients of g_L^2, g_R^2 and -g_L g_R in Eq.
// (sm_cross_section)), and nu (1/T - 1/E) for the magnetic term (Eq.
// (xs_mm)); S_theta(T_l) is sum_b c_b(theta) times these.
void source_basis(const nr_ctx* c, int k, int l, double acc[10]) {
    const int n_t = c->n_t;
    const double T = c->tc[l];
    const int hi = c->src_off[k] + c->src_n[k];
    for (int q = 0; q < 10; ++q) acc[q] = 0.0;
    for (int j = c->jmin[(size_t)k * n_t + l]; j < hi; ++j) {
        const double E = c->hE[j], nu = c->hW[j], pe = c->hPe[j];
        const double P[3] = {pe, (1 - pe) * (1 - c->ph.tau_frac),
                             (1 - pe) * c->ph.tau_frac};
        const double y = 1.0 - T / E, x = c->ph.me * T / (E * E);
        for (int a = 0; a < 3; ++a) {
            acc[3 * a + 0] += nu * P[a];
            acc[3 * a + 1] += nu * P[a] * y * y;
            acc[3 * a + 2] += nu * P[a] * x;
        }
        acc[9] += nu * (P[0] + P[1] + P[2]) * (1.0 / T - 1.0 / E);
    }
}

void recompute_mrow(nr_ctx* c) {
    if (c->m_user || !c->have_src || c->multi) return;
    double tot = 0;
    for (int l = 0; l < c->n_t; ++l) tot += c->ssm[l];
    c->mrow.assign(c->n_t, 0.0);
    for (int l = 0; l < c->n_t; ++l)
        c->mrow[l] = tot > 0 ? c->n_sig * c->ssm[l] / tot : 0.0;
}

int upload_mrow(nr_ctx* c) {
    if (!c->have_rsp || c->multi) return 0;
    HIPCHK(hipMemcpy(c->d_mrow, c->mrow.data(), sizeof(double) * c->n_t,
                     hipMemcpyHostToDevice));
    return 0;
}

// Non-zero column band of every response row (float4 units, [lo, hi); an
// all-zero row gets lo = hi = 0), from the host copy of the stacked rows.
int set_row_bands(nr_ctx* c, const float* R, int n_rows, int n_cols, size_t ld) {
    c->rowband.assign((size_t)2 * n_rows, 0);
    for (int l = 0; l < n_rows; ++l) {
        const float* r = R + (size_t)l * ld;
        int lo = 0, hi = n_cols;
        while (lo < n_cols && r[lo] == 0.0f) ++lo;
        while (hi > lo && r[hi - 1] == 0.0f) --hi;
        if (lo < hi) {
            c->rowband[2 * (size_t)l] = lo / 4;
            c->rowband[2 * (size_t)l + 1] = (hi + 3) / 4;
        }
    }
    int rc;
    if ((rc = dalloc(&c->d_rowband, c->rowband.size()))) return rc;
    HIPCHK(hipMemcpy(c->d_rowband, c->rowband.data(), sizeof(int) * c->rowband.size(),
                     hipMemcpyHostToDevice));
    return 0;
}

// Band of every fold tile (the union of its rows' bands, clipped to the
// tile's columns), in the fold's tile order cc * n_rb + rb.
int set_tile_bands(nr_ctx* c) {
    constexpr int kTile4 = 512;  // float4 columns per fold tile
    std::vector<int> tb((size_t)2 * c->n_rb * c->n_fc);
    for (int cc = 0; cc < c->n_fc; ++cc)
        for (int rb = 0; rb < c->n_rb; ++rb) {
            const int c0 = cc * kTile4, c1 = c0 + kTile4;
            int lo = c1, hi = c0;
            const int l1 = std::min(c->n_rows, (rb + 1) * c->rows_per_wg);
            for (int l = rb * c->rows_per_wg; l < l1; ++l) {
                const int a = c->rowband[2 * (size_t)l], b = c->rowband[2 * (size_t)l + 1];
                if (a >= b) continue;
                lo = std::min(lo, std::max(a, c0));
                hi = std::max(hi, std::min(b, c1));
            }
            const size_t t = (size_t)cc * c->n_rb + rb;
            tb[2 * t] = lo < hi ? lo : c0;
            tb[2 * t + 1] = lo < hi ? hi : c0;
        }
    int rc;
    if ((rc = dalloc(&c->d_tileband, tb.size()))) return rc;
    HIPCHK(hipMemcpy(c->d_tileband, tb.data(), sizeof(int) * tb.size(), hipMemcpyHostToDevice));
    return 0;
}

int choose_tiling(nr_ctx* c, int rows_req) {
    c->n_fc = (c->ldr / 4 + 511) / 512;   // fold tiles are 2048 columns wide
    c->n_cc = (c->n_reco + 63) / 64;      // reduction groups of 64 columns
    int rows;
    if (rows_req > 0) {
        rows = rows_req;
    } else {
        // one fold tile per compute unit: measured on MI355X at 16384 x 4096,
        // 128-row x 2048-column tiles (128 x 2 work-groups) stream fastest
        const int target_rb = std::max(1, 256 / c->n_fc);
        rows = (c->n_rows + target_rb - 1) / target_rb;
        rows = (rows + 7) / 8 * 8;
    }
    rows = std::max(8, std::min(rows, 2048));
    c->rows_per_wg = rows;
    c->n_rb = (c->n_rows + rows - 1) / rows;
    int rc;
    if ((rc = dalloc(&c->d_colpart, (size_t)2 * c->n_rb * c->ldr))) return rc;
    if ((rc = dalloc(&c->d_chunk_dev, (size_t)2 * c->n_cc))) return rc;
    if ((rc = dalloc(&c->d_chunk_gb, (size_t)2 * c->n_cc))) return rc;
    c->adj_grid = nr::adjoint_grid(c->n_t);
    if ((rc = dalloc(&c->d_jpart, (size_t)c->adj_grid * nr::kNBasis))) return rc;
    if ((rc = set_tile_bands(c))) return rc;
    clear_graphs(c);
    return 0;
}

void free_pinned(nr_ctx* c) {
    if (c->h_cap) (void)hipDeviceSynchronize();  // no launch still reads them
    for (double** p : {&c->h_th, &c->h_out, &c->h_grad}) {
        if (*p) (void)hipHostFree(*p);
        *p = nullptr;
    }
    c->hd_th = c->hd_out = c->hd_grad = nullptr;
    c->h_cap = 0;
}

// Pinned, device-accessible host buffers for pts points (theta, -2lnL and
// gradient of any form).
int ensure_pinned(nr_ctx* c, size_t pts) {
    if (pts <= c->h_cap) return 0;
    free_pinned(c);
    clear_graphs(c);  // cached graphs hold the old addresses
    const size_t n = std::max(pts, (size_t)64);
    struct Buf { double** h; double** d; size_t len; };
    for (const Buf& b : {Buf{&c->h_th, &c->hd_th, n * nr::kMaxTheta},
                         Buf{&c->h_out, &c->hd_out, n},
                         Buf{&c->h_grad, &c->hd_grad, n * nr::kMaxTheta}}) {
        hipError_t e = hipHostMalloc((void**)b.h, b.len * sizeof(double), hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void**)b.d, *b.h, 0);
        if (e != hipSuccess) {
            c->h_cap = n;  // free what exists
            free_pinned(c);
            return fail(NR_ENOMEM, "pinned staging of %zu bytes: %s", b.len * sizeof(double),
                        hipGetErrorString(e));
        }
    }
    c->h_cap = n;
    return 0;
}

int ensure_stage(nr_ctx* c, size_t pts, size_t mu_elems, size_t w_elems) {
    int rc;
    if (pts > c->cap_pts) {
        size_t n = std::max(pts, (size_t)64);
        if ((rc = dalloc(&c->d_th, n * nr::kMaxTheta))) return rc;  // any form's theta
        if ((rc = dalloc(&c->d_out, n))) return rc;
        if ((rc = dalloc(&c->d_grad, n * nr::kMaxTheta))) return rc;  // any form's gradient
        c->cap_pts = n;
        clear_graphs(c);
    }
    if (mu_elems > c->cap_mu) {
        if ((rc = dalloc(&c->d_mu, mu_elems))) return rc;
        c->cap_mu = mu_elems;
        clear_graphs(c);
    }
    if (w_elems > c->cap_w) {
        if ((rc = dalloc(&c->d_w, w_elems))) return rc;
        c->cap_w = w_elems;
    }
    return 0;
}

// Device buffers of the single-point pipeline: node tables, fold vectors,
// fold partial rows and likelihood group sums (each by point parity), and
// the adjoint's a_j, sum_j a_j b_j and basis contractions.  A context owns
// one set; the allocation-free entry point carves another out of the
// library's static workspace (NULL = the context's).
struct Work {
    double* table[2];   // [4 (n_nodes + n_src)] each
    double* ctot[2];    // [4 n_src max_chunks] each
    double* v[2];       // [n_rows] each
    double* colpart;    // [2][n_rb][ldr]
    double* chunk_dev;  // [2][n_cc]
    double* chunk_gb;   // [2][n_cc]
    double* a;          // [ldr]
    double* gb;         // [1]
    double* jpart;      // [adj_grid][kNBasis]
};

// Lays the buffers of Work out from base (256-byte pieces) and returns the
// bytes they take; with base NULL only the size is formed.
size_t carve_work(const nr_ctx* c, double* base, Work* w) {
    size_t off = 0;
    auto take = [&](size_t n) {
        double* p = base ? base + off : nullptr;
        off += (n + 31) / 32 * 32;
        return p;
    };
    const size_t nt = (size_t)4 * (c->n_nodes + c->n_src);
    w->table[0] = take(nt);
    w->table[1] = take(nt);
    w->ctot[0] = take((size_t)4 * c->n_src * c->max_chunks);
    w->ctot[1] = take((size_t)4 * c->n_src * c->max_chunks);
    w->v[0] = take(c->n_rows);
    w->v[1] = take(c->n_rows);
    w->colpart = take((size_t)2 * c->n_rb * c->ldr);
    w->chunk_dev = take((size_t)2 * c->n_cc);
    w->chunk_gb = take((size_t)2 * c->n_cc);
    w->a = take(c->ldr);
    w->gb = take(1);
    w->jpart = take((size_t)c->adj_grid * nr::kNBasis);
    return off * sizeof(double);
}

nr::ScanArgs scan_args(nr_ctx* c, const double* d_theta, int par,
                       const Work* wk = nullptr) {
    nr::ScanArgs a{};
    a.nodeIE = c->d_E;
    a.nodeW = c->d_W;
    a.nodePe = c->d_Pe;
    a.srcOff = c->d_srcoff;
    // the multi-component form scales components by their rates instead
    a.srcGroup = c->multi ? c->d_group0 : c->d_group;
    a.theta = d_theta;
    a.ph = c->ph;
    a.table = reinterpret_cast<double4*>(wk ? wk->table[par] : c->d_table[par]);
    a.blocks = c->d_scanblk;
    a.ctot = reinterpret_cast<double4*>(wk ? wk->ctot[par] : c->d_ctot[par]);
    a.max_chunks = c->max_chunks;
    return a;
}

nr::RowArgs row_args(nr_ctx* c, int par, double* v, double* out_w,
                     double* out_s, const double* d_theta,
                     const Work* wk = nullptr) {
    nr::RowArgs a{};
    a.table = reinterpret_cast<const double4*>(wk ? wk->table[par] : c->d_table[par]);
    a.srcOff = c->d_srcoff;
    a.ctot = reinterpret_cast<const double4*>(wk ? wk->ctot[par] : c->d_ctot[par]);
    a.max_chunks = c->max_chunks;
    a.jmin = c->d_jmin;
    a.tc = c->d_tc;
    a.n_t = c->n_t;
    a.n_comp = c->multi ? c->n_comp : 1;
    a.compOff = c->d_compoff;
    a.compSrc = c->d_compsrc;
    a.ssm = c->multi ? c->d_ssmc : c->d_ssm;
    a.mrow = c->d_mrow;
    a.theta = nullptr;
    a.rate_index = c->multi ? 5 : -1;
    a.theta = d_theta;
    a.v = v;
    a.out_w = out_w;
    a.out_s = out_s;
    return a;
}

nr::FoldArgs fold_args(nr_ctx* c, const double* thp, const double* v,
                       double* colpart, double* nll, double* mu, bool grad,
                       int cpar = 0, const Work* wk = nullptr) {
    nr::FoldArgs fa{};
    fa.R = c->d_R;
    fa.ldr = c->ldr;
    fa.n_t = c->n_rows;
    fa.n_reco = c->n_reco;
    fa.v = v;
    fa.n = c->d_n;
    fa.b = c->multi ? c->d_bkg : c->d_b;
    fa.n_bkg = c->multi ? c->n_bkg : 1;
    fa.bkg_index = c->multi ? 5 + c->n_comp : 6;
    fa.mask = c->multi ? c->d_mask : nullptr;
    fa.n_theta = c->n_theta;
    fa.theta = thp;
    fa.colpart = colpart;
    // group sums, by parity
    fa.chunk_dev = (wk ? wk->chunk_dev : c->d_chunk_dev) + (size_t)cpar * c->n_cc;
    fa.chunk_gb = (wk ? wk->chunk_gb : c->d_chunk_gb) + (size_t)cpar * c->n_cc;
    fa.out_nll = nll;
    fa.out_mu = mu;
    fa.out_a = grad ? (wk ? wk->a : c->d_a) : nullptr;
    fa.out_gb = grad ? (wk ? wk->gb : c->d_gb) : nullptr;
    fa.cdata = c->cdata;
    for (int i = 0; i < c->n_theta; ++i) {
        fa.pull_mean[i] = c->pull_mean[i];
        fa.pull_sigma[i] = c->pull_sigma[i];
    }
    fa.rows_per_wg = c->rows_per_wg;
    fa.n_rb = c->n_rb;
    fa.n_fc = c->n_fc;
    fa.n_cc = c->n_cc;
    fa.reverse = 0;
    fa.band = c->skip_zero ? c->d_tileband : nullptr;
    // responses beyond twice the 256 MB Infinity Cache stream past it
    fa.stream_nt = (double)c->n_rows * c->ldr * sizeof(float) > 512.0e6;
    return fa;
}

int step(nr_ctx* c, const nr::FoldArgs* fold, const nr::RowArgs* rows,
         const nr::ScanArgs* scan, const nr::FoldArgs* fin, hipStream_t s,
         const nr::FoldArgs* fnl = nullptr) {
    nr::StepArgs a{};
    if (fold) {
        a.fold = *fold;
        a.nb_fold = c->n_rb * c->n_fc;
    }
    if (rows) {
        a.rows = *rows;
        a.nb_rows = (rows->n_comp * c->n_t + nr::kStepRows - 1) / nr::kStepRows;
    }
    if (scan) {
        a.scan = *scan;
        a.nb_scan = c->nb_scan;
    }
    if (fin) {
        a.fin = *fin;
        a.nb_fin = c->n_cc;
    }
    if (fnl) {
        a.fnl = *fnl;
        a.nb_final = 1;
    }
    HIPCHK(nr::launch_step(a, s));
    return 0;
}

// Single-point evaluations of a list of points on one stream.  Launch k of
// the step kernel builds the node table of point k (a1), forms the weights
// of point k - 1 (a2), folds point k - 2 (a3) and reduces the likelihood of
// point k - 3 (a4, a5), so all but the fold run beside the R stream
// instead of after it.  Node tables, weight vectors and fold partial sums
// alternate between two buffers by point parity, and stream order is the
// only synchronisation.  With a gradient each point runs its stages in
// turn, the adjoint pass (which needs the finished a_j) last.
int enqueue_points(nr_ctx* c, const double* th, int n_pts, double* nll,
                   double* grad, double* mu, double* w, hipStream_t s,
                   const Work* wk = nullptr) {
    const Work own{{c->d_table[0], c->d_table[1]}, {c->d_ctot[0], c->d_ctot[1]},
                   {c->d_v[0], c->d_v[1]},
                   c->d_colpart, c->d_chunk_dev, c->d_chunk_gb, c->d_a, c->d_gb,
                   c->d_jpart};
    if (!wk) wk = &own;
    const size_t cp = (size_t)c->n_rb * c->ldr;
    auto thp = [&](int p) { return th + (size_t)p * c->n_theta; };
    auto sa = [&](int p) { return scan_args(c, thp(p), p & 1, wk); };
    auto ra = [&](int p) {
        return row_args(c, p & 1, wk->v[p & 1],
                        w ? w + (size_t)p * c->n_rows : nullptr, nullptr, thp(p), wk);
    };
    auto fa = [&](int p) {
        nr::FoldArgs f = fold_args(c, thp(p), wk->v[p & 1],
                                   wk->colpart + (p & 1) * cp, nll + p,
                                   mu ? mu + (size_t)p * c->n_reco : nullptr,
                                   grad != nullptr, p & 1, wk);
        // a scan walks R forwards and backwards in turn, so each point starts
        // on the rows the previous one left in the Infinity Cache
        f.reverse = (grad || f.stream_nt) ? 0 : (p & 1);
        return f;
    };
    auto in = [&](int p) { return p >= 0 && p < n_pts; };
    int rc;
    if (!grad) {
        for (int k = 0; k <= n_pts + 3; ++k) {
            nr::ScanArgs a1;
            nr::RowArgs a2;
            nr::FoldArgs a3, a4, a5;
            if (in(k)) a1 = sa(k);
            if (in(k - 1)) a2 = ra(k - 1);
            if (in(k - 2)) a3 = fa(k - 2);
            if (in(k - 3)) a4 = fa(k - 3);
            if (in(k - 4)) a5 = fa(k - 4);
            if ((rc = step(c, in(k - 2) ? &a3 : nullptr, in(k - 1) ? &a2 : nullptr,
                           in(k) ? &a1 : nullptr, in(k - 3) ? &a4 : nullptr, s,
                           in(k - 4) ? &a5 : nullptr)))
                return rc;
        }
        return 0;
    }
    for (int p = 0; p < n_pts; ++p) {
        const nr::ScanArgs a1 = sa(p);
        const nr::RowArgs a2 = ra(p);
        const nr::FoldArgs f = fa(p);
        if ((rc = step(c, nullptr, nullptr, &a1, nullptr, s))) return rc;
        if ((rc = step(c, nullptr, &a2, nullptr, nullptr, s))) return rc;
        if ((rc = step(c, &f, nullptr, nullptr, nullptr, s))) return rc;
        if ((rc = step(c, nullptr, nullptr, nullptr, &f, s))) return rc;
        if ((rc = step(c, nullptr, nullptr, nullptr, nullptr, s, &f))) return rc;
        nr::AdjArgs aa{};
        aa.R = c->d_R;
        aa.ldr = c->ldr;
        aa.n_t = c->n_t;
        aa.n_reco = c->n_reco;
        aa.a = wk->a;
        aa.ssm = c->d_ssm;
        aa.mrow = c->d_mrow;
        aa.basis = c->d_basis;
        aa.theta = thp(p);
        aa.gb = wk->gb;
        aa.jpart = wk->jpart;
        aa.rowband = c->skip_zero ? c->d_rowband : nullptr;
        aa.out_grad = grad + (size_t)p * NR_NTHETA;
        for (int i = 0; i < NR_NTHETA; ++i) {
            aa.pull_mean[i] = c->pull_mean[i];
            aa.pull_sigma[i] = c->pull_sigma[i];
        }
        aa.ph = c->ph;
        HIPCHK(nr::launch_adjoint(aa, c->adj_grid, s));
    }
    return 0;
}

// Replays a cached graph of the per-point launches when the same buffers and
// point count come back (the common case in fits and scans).  One or two
// points launch their five or six kernels directly: a graph replay starts
// its first kernel later than a direct launch does, which at 16384 x 4096
// cost ~8 us of a ~88 us isolated call.
constexpr int kDirectMaxPts = 2;

int run_points(nr_ctx* c, const double* th, int n_pts, double* nll,
               double* grad, double* mu, double* w, hipStream_t s) {
    if (!c->use_graph || n_pts > 4096 || w || n_pts <= kDirectMaxPts)
        return enqueue_points(c, th, n_pts, nll, grad, mu, w, s);
    GraphKey key{th, n_pts, nll, grad, mu, (void*)s};
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        if (c->graphs.size() >= 16) clear_graphs(c);
        hipGraph_t g = nullptr;
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        int rc = enqueue_points(c, th, n_pts, nll, grad, mu, w, s);
        hipError_t e = hipStreamEndCapture(s, &g);
        if (rc) {
            if (e == hipSuccess && g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess)
            return fail(NR_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        hipGraphExec_t ex;
        e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess)
            return fail(NR_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
        it = c->graphs.emplace(key, ex).first;
    }
    HIPCHK(hipGraphLaunch(it->second, s));
    return 0;
}

int check_ready(nr_ctx* c) {
    if (!c) return fail(NR_EINVAL, "null context");
    if (!c->have_src || !c->have_rsp || !c->have_data)
        return fail(NR_ESTATE,
                    "evaluation before set_sources, set_response and set_data");
    return 0;
}

int check_theta(const double* th, int n_pts, int n_theta = NR_NTHETA) {
    if (!th || n_pts <= 0) return fail(NR_EINVAL, "theta null or n_pts <= 0");
    if (!finite_all(th, (size_t)n_pts * n_theta))
        return fail(NR_EINVAL, "non-finite theta");
    return 0;
}

// Entry points of the single-component form only (gradient, batched,
// diagnostics, surrogate) refuse a multi-component context.
int check_single(nr_ctx* c) {
    if (c && c->multi)
        return fail(NR_ESTATE, "not available for a multi-component context");
    return 0;
}

}  // namespace

namespace {

// ------------------------------------------------------------ batched path
int ensure_batch(nr_ctx* c, int n_pts, bool grad, size_t mu_elems) {
    const int ldw = (n_pts + 3) / 4 * 4;
    const int nnt = (c->n_reco + 63) / 64;  // column tiles of the narrowest config
    int rc;
    bool moved = false;
    if (n_pts > c->b_cap || ldw > c->b_ldw || nnt != c->b_nnt) {
        const int cap = std::max(n_pts, 64);
        const int ldc = (cap + 3) / 4 * 4;
        if ((rc = dalloc(&c->d_wt, (size_t)c->n_t * ldc))) return rc;
        HIPCHK(hipMemset(c->d_wt, 0, sizeof(double) * (size_t)c->n_t * ldc));
        if ((rc = dalloc(&c->d_bpart, (size_t)cap * nnt))) return rc;
        if ((rc = dalloc(&c->d_bpgb, (size_t)cap * nnt))) return rc;
        if ((rc = dalloc(&c->d_bth, (size_t)cap * NR_NTHETA))) return rc;
        if ((rc = dalloc(&c->d_bnll, (size_t)cap))) return rc;
        if ((rc = dalloc(&c->d_bgrad, (size_t)cap * NR_NTHETA))) return rc;
        c->b_cap = cap;
        c->b_ldw = ldc;
        c->b_nnt = nnt;
        c->b_grad = false;
        moved = true;
    }
    if (grad && !c->b_grad) {
        if ((rc = dalloc(&c->d_bat, (size_t)c->ldr * c->b_ldw))) return rc;
        HIPCHK(hipMemset(c->d_bat, 0, sizeof(double) * (size_t)c->ldr * c->b_ldw));
        if ((rc = dalloc(&c->d_bu, (size_t)c->b_cap * c->n_t))) return rc;
        c->b_grad = true;
        moved = true;
    }
    if (mu_elems > c->b_cap_mu) {
        if ((rc = dalloc(&c->d_bmu, mu_elems))) return rc;
        c->b_cap_mu = mu_elems;
        moved = true;
    }
    if (moved) ++g_epoch;
    return 0;
}

struct MultiCall {
    nr_ctx* const* ctx;
    int n;
    const double* const* theta;  // device
    const int* n_pts;
    double* const* nll;          // device
    double* const* grad;         // device or null (array may be null)
    double* const* mu;           // device or null (array may be null)
};

nr::WgenArgs wgen_args(nr_ctx* c, const double* th, int P) {
    nr::WgenArgs w{};
    w.theta = th;
    w.n_pts = P;
    w.ldw = c->b_ldw;
    w.n_t = c->n_t;
    w.basis = c->d_basis;
    w.ssm = c->d_ssm;
    w.mrow = c->d_mrow;
    w.ph = c->ph;
    w.wt = c->d_wt;
    return w;
}

// K range of a GEMM tile: the whole reduction, or with band skipping the
// K-steps whose response entries for the tile are not all zero.  Forward
// tiles cover response columns [c0, c1) and reduce over its rows; adjoint
// tiles cover rows [c0, c1) and reduce over its columns.  An empty range
// leaves the tile's sums at zero, as the skipped products are.
void tile_k_range(const nr_ctx* c, bool adjoint, int c0, int c1, int K, int* k0, int* k1) {
    constexpr int BK = nr::kGemmBK;
    if (!c->skip_zero) {
        *k0 = 0;
        *k1 = K;
        return;
    }
    int lo = K, hi = 0;
    if (!adjoint) {
        for (int l = 0; l < c->n_t; ++l) {
            const int a = 4 * c->rowband[2 * (size_t)l], b = 4 * c->rowband[2 * (size_t)l + 1];
            if (a < b && a < c1 && b > c0) {
                lo = std::min(lo, l);
                hi = std::max(hi, l + 1);
            }
        }
    } else {
        for (int l = c0; l < std::min(c1, c->n_t); ++l) {
            const int a = 4 * c->rowband[2 * (size_t)l], b = 4 * c->rowband[2 * (size_t)l + 1];
            if (a < b) {
                lo = std::min(lo, a);
                hi = std::max(hi, b);
            }
        }
    }
    if (lo >= hi) {
        *k0 = *k1 = 0;
        return;
    }
    *k0 = lo / BK * BK;
    *k1 = std::min(K, (hi + BK - 1) / BK * BK);
}

int build_plan(const MultiCall& mc, bool grad, int cfg, BatchPlan* pl) {
    const int TMt = nr::gemm_tile_m(cfg), TNt = nr::gemm_tile_n(cfg);
    std::vector<nr::GemmProb> pf(mc.n), pa(mc.n);
    std::vector<nr::GemmTile> tf, ta;
    for (int d = 0; d < mc.n; ++d) {
        nr_ctx* c = mc.ctx[d];
        const int P = mc.n_pts[d];
        nr::GemmProb f{};
        f.At = c->d_wt;
        f.lda = c->b_ldw;
        f.B = c->d_R;
        f.ldb = c->ldr;
        f.M = P;
        f.N = c->n_reco;
        f.K = c->n_t;
        f.n = c->d_n;
        f.b = c->d_b;
        f.theta = mc.theta[d];
        f.part = c->d_bpart;
        f.part_gb = c->d_bpgb;
        f.n_nt = (c->n_reco + TNt - 1) / TNt;
        f.aout = grad ? c->d_bat : nullptr;
        f.lda_out = c->b_ldw;
        f.mu = mc.mu ? mc.mu[d] : nullptr;
        pf[d] = f;
        const int mt = (P + TMt - 1) / TMt;
        std::vector<int> kr(2 * (size_t)f.n_nt);
        for (int j = 0; j < f.n_nt; ++j)
            tile_k_range(c, false, j * TNt, (j + 1) * TNt, c->n_t, &kr[2 * j], &kr[2 * j + 1]);
        for (int i = 0; i < mt; ++i)
            for (int j = 0; j < f.n_nt; ++j)
                tf.push_back({d, i, j, kr[2 * j + 1] - kr[2 * j], kr[2 * j], kr[2 * j + 1]});
        if (grad) {
            nr::GemmProb a{};
            a.At = c->d_bat;
            a.lda = c->b_ldw;
            a.B = c->d_R;
            a.ldb = c->ldr;
            a.M = P;
            a.N = c->n_t;
            a.K = c->n_reco;
            a.C = c->d_bu;
            a.ldc = c->n_t;
            pa[d] = a;
            const int nt = (c->n_t + TNt - 1) / TNt;
            std::vector<int> ka(2 * (size_t)nt);
            for (int j = 0; j < nt; ++j)
                tile_k_range(c, true, j * TNt, (j + 1) * TNt, c->n_reco, &ka[2 * j],
                             &ka[2 * j + 1]);
            for (int i = 0; i < mt; ++i)
                for (int j = 0; j < nt; ++j)
                    ta.push_back({d, i, j, ka[2 * j + 1] - ka[2 * j], ka[2 * j], ka[2 * j + 1]});
        }
    }
    // longest tiles first: the persistent work-groups pull from this list
    auto by_cost = [](const nr::GemmTile& x, const nr::GemmTile& y) { return x.cost > y.cost; };
    std::stable_sort(tf.begin(), tf.end(), by_cost);
    std::stable_sort(ta.begin(), ta.end(), by_cost);
    int rc;
    if ((rc = dalloc(&pl->d_probs_f, pf.size())) || (rc = dalloc(&pl->d_tiles_f, tf.size())))
        return rc;
    HIPCHK(hipMemcpy(pl->d_probs_f, pf.data(), sizeof(nr::GemmProb) * pf.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(pl->d_tiles_f, tf.data(), sizeof(nr::GemmTile) * tf.size(), hipMemcpyHostToDevice));
    pl->n_tiles_f = (int)tf.size();
    pl->cfg = cfg;
    pl->grid_f = nr::gemm_grid(nr::kModeNll, cfg, pl->n_tiles_f);
    if (grad) {
        if ((rc = dalloc(&pl->d_probs_a, pa.size())) || (rc = dalloc(&pl->d_tiles_a, ta.size())))
            return rc;
        HIPCHK(hipMemcpy(pl->d_probs_a, pa.data(), sizeof(nr::GemmProb) * pa.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(pl->d_tiles_a, ta.data(), sizeof(nr::GemmTile) * ta.size(), hipMemcpyHostToDevice));
        pl->n_tiles_a = (int)ta.size();
        pl->grid_a = nr::gemm_grid(nr::kModeAdj, cfg, pl->n_tiles_a);
    }
    pl->epoch = g_epoch.load();
    return 0;
}

int enqueue_plan(const MultiCall& mc, bool grad, BatchPlan* pl, unsigned* ctr,
                 hipStream_t s) {
    for (int d = 0; d < mc.n; ++d)
        HIPCHK(nr::launch_wgen(wgen_args(mc.ctx[d], mc.theta[d], mc.n_pts[d]), s));
    HIPCHK(nr::launch_gemm(nr::kModeNll, pl->cfg, pl->d_probs_f, pl->d_tiles_f,
                           pl->n_tiles_f, ctr, pl->grid_f, s));
    for (int d = 0; d < mc.n; ++d) {
        nr_ctx* c = mc.ctx[d];
        nr::FinalArgs f{};
        f.part = c->d_bpart;
        f.theta = mc.theta[d];
        f.n_pts = mc.n_pts[d];
        f.n_nt = (c->n_reco + nr::gemm_tile_n(pl->cfg) - 1) / nr::gemm_tile_n(pl->cfg);
        f.cdata = c->cdata;
        for (int i = 0; i < NR_NTHETA; ++i) {
            f.pull_mean[i] = c->pull_mean[i];
            f.pull_sigma[i] = c->pull_sigma[i];
        }
        f.nll = mc.nll[d];
        HIPCHK(nr::launch_finalize(f, s));
    }
    if (grad) {
        HIPCHK(nr::launch_gemm(nr::kModeAdj, pl->cfg, pl->d_probs_a, pl->d_tiles_a,
                               pl->n_tiles_a, ctr + 2, pl->grid_a, s));
        for (int d = 0; d < mc.n; ++d) {
            nr_ctx* c = mc.ctx[d];
            nr::ContractArgs a{};
            a.U = c->d_bu;
            a.ldu = c->n_t;
            a.n_t = c->n_t;
            a.n_pts = mc.n_pts[d];
            a.n_nt = (c->n_reco + nr::gemm_tile_n(pl->cfg) - 1) / nr::gemm_tile_n(pl->cfg);
            a.ssm = c->d_ssm;
            a.mrow = c->d_mrow;
            a.basis = c->d_basis;
            a.theta = mc.theta[d];
            a.part_gb = c->d_bpgb;
            for (int i = 0; i < NR_NTHETA; ++i) {
                a.pull_mean[i] = c->pull_mean[i];
                a.pull_sigma[i] = c->pull_sigma[i];
            }
            a.ph = c->ph;
            a.grad = mc.grad[d];
            HIPCHK(nr::launch_adj_contract(a, s));
        }
    }
    return 0;
}

// ---- project autotuner for the grouped GEMM.  A shape class is the sorted
// list of (points rounded up to 64, N_reco, N_T) of the call plus the mode;
// the first call of a class times every tile configuration on the real
// problem (one warm-up and two timed runs each) and keeps the fastest, in
// memory and in a small JSON file (NR_AUTOTUNE_CACHE, default
// $HOME/.cache/nureweight/autotune.json).  NR_AUTOTUNE=0 skips tuning; a
// missing, unreadable or corrupt cache file only means tuning again.  The
// table is shared by every context of the process: g_tune_mu guards it and
// the file (held for lookups and updates, not while a class is timed, so
// two threads may time the same class once each).
struct TuneCache {
    bool loaded = false;
    std::map<std::string, int> best;
    std::string path;
};
TuneCache g_tune;
std::mutex g_tune_mu;

std::string tune_path() {
    const char* p = getenv("NR_AUTOTUNE_CACHE");
    if (p && *p) return p;
    const char* h = getenv("HOME");
    return std::string(h && *h ? h : "/tmp") + "/.cache/nureweight/autotune.json";
}

void tune_load() {
    const std::string path = tune_path();
    if (g_tune.loaded && path == g_tune.path) return;
    g_tune.loaded = true;
    g_tune.best.clear();
    g_tune.path = path;
    FILE* f = fopen(g_tune.path.c_str(), "r");
    if (!f) return;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, n);
    fclose(f);
    // entries are "key": value with keys free of quotes
    size_t i = 0;
    while ((i = txt.find('"', i)) != std::string::npos) {
        const size_t j = txt.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = txt.substr(i + 1, j - i - 1);
        const size_t c = txt.find(':', j);
        if (c == std::string::npos) break;
        char* end = nullptr;
        const long v = strtol(txt.c_str() + c + 1, &end, 10);
        if (end != txt.c_str() + c + 1 && v >= 0 && v < nr::kGemmConfigs)
            g_tune.best[key] = (int)v;
        i = (end && end > txt.c_str() + c) ? (size_t)(end - txt.c_str()) : j + 1;
    }
}

void tune_save() {
    std::string dir = g_tune.path.substr(0, g_tune.path.rfind('/'));
    std::string cmd;
    for (size_t k = 1; k <= dir.size(); ++k)  // mkdir -p without a shell
        if (k == dir.size() || dir[k] == '/') (void)mkdir(dir.substr(0, k).c_str(), 0755);
    FILE* f = fopen((g_tune.path + ".tmp").c_str(), "w");
    if (!f) return;
    fprintf(f, "{\n");
    size_t k = 0;
    for (auto& kv : g_tune.best)
        fprintf(f, "  \"%s\": %d%s\n", kv.first.c_str(), kv.second,
                ++k < g_tune.best.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    (void)rename((g_tune.path + ".tmp").c_str(), g_tune.path.c_str());
}

std::string shape_class(const MultiCall& mc, bool grad) {
    std::vector<std::string> parts;
    for (int d = 0; d < mc.n; ++d) {
        char b[96];
        snprintf(b, sizeof(b), "%dx%dx%d%s", (mc.n_pts[d] + 63) / 64 * 64,
                 mc.ctx[d]->n_reco, mc.ctx[d]->n_t, mc.ctx[d]->skip_zero ? "b" : "");
        parts.push_back(b);
    }
    std::sort(parts.begin(), parts.end());
    std::string key = grad ? "grad" : "nll";
    for (auto& p : parts) key += "|" + p;
    if (key.size() > 200) {  // long groups: a stable hash keeps the file small
        unsigned long h = 1469598103934665603ul;
        for (char ch : key) h = (h ^ (unsigned char)ch) * 1099511628211ul;
        char b[64];
        snprintf(b, sizeof(b), "%s|n%d|h%016lx", grad ? "grad" : "nll", mc.n, h);
        key = b;
    }
    return key;
}

int tuned_config(const MultiCall& mc, bool grad, hipStream_t s, int* cfg_out) {
    const char* force = getenv("NR_GEMM_CONFIG");  // pins a configuration
    if (force && force[0] >= '0' && force[0] < '0' + nr::kGemmConfigs && !force[1]) {
        *cfg_out = force[0] - '0';
        return 0;
    }
    const char* e = getenv("NR_AUTOTUNE");
    if (e && e[0] == '0') { *cfg_out = 0; return 0; }
    const std::string key = shape_class(mc, grad);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load();
        auto it = g_tune.best.find(key);
        if (it != g_tune.best.end()) { *cfg_out = it->second; return 0; }
    }
    nr_ctx* owner = mc.ctx[0];
    // events and the trial plan's tables are released on every return
    struct Trial {
        hipStream_t st;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        BatchPlan pl;
        void drop_plan() {
            if (pl.d_probs_f) (void)hipFree(pl.d_probs_f);
            if (pl.d_tiles_f) (void)hipFree(pl.d_tiles_f);
            if (pl.d_probs_a) (void)hipFree(pl.d_probs_a);
            if (pl.d_tiles_a) (void)hipFree(pl.d_tiles_a);
            pl = BatchPlan{};
        }
        ~Trial() {
            (void)hipStreamSynchronize(st);  // nothing in flight reads the tables
            drop_plan();
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    } t{s};
    HIPCHK(hipEventCreate(&t.e0));
    HIPCHK(hipEventCreate(&t.e1));
    float best_ms = 1e30f;
    int best = 0;
    for (int cfg = 0; cfg < nr::kGemmConfigs; ++cfg) {
        int rc = build_plan(mc, grad, cfg, &t.pl);
        if (rc) return rc;
        rc = enqueue_plan(mc, grad, &t.pl, owner->d_gctr, s);  // warm-up
        if (rc) return rc;
        HIPCHK(hipEventRecord(t.e0, s));
        for (int r = 0; r < 2 && !rc; ++r) rc = enqueue_plan(mc, grad, &t.pl, owner->d_gctr, s);
        HIPCHK(hipEventRecord(t.e1, s));
        HIPCHK(hipEventSynchronize(t.e1));
        if (rc) return rc;
        float ms = 0;
        HIPCHK(hipEventElapsedTime(&ms, t.e0, t.e1));
        t.drop_plan();
        if (ms < best_ms) { best_ms = ms; best = cfg; }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_load();  // the cache path may have changed meanwhile
        g_tune.best[key] = best;
        tune_save();
    }
    *cfg_out = best;
    return 0;
}

int run_multi(const MultiCall& mc, hipStream_t s) {
    nr_ctx* owner = mc.ctx[0];
    const bool grad = mc.grad != nullptr;
    std::vector<const void*> key;
    key.push_back((const void*)s);
    key.push_back((const void*)(size_t)grad);
    key.push_back((const void*)(size_t)(mc.mu != nullptr));
    for (int d = 0; d < mc.n; ++d) {
        key.push_back(mc.ctx[d]);
        key.push_back(mc.theta[d]);
        key.push_back((const void*)(size_t)mc.n_pts[d]);
        key.push_back(mc.nll[d]);
        if (grad) key.push_back(mc.grad[d]);
        if (mc.mu) key.push_back(mc.mu[d]);
    }
    BatchPlan*& pl = owner->plans[key];
    if (pl && pl->epoch != g_epoch) {
        free_plan(pl);
        pl = nullptr;
    }
    if (!pl) {
        if (owner->plans.size() > 16) {
            for (auto& kv : owner->plans)
                if (kv.second && kv.first != key) free_plan(kv.second);
            owner->plans.clear();
        }
        int cfg = 0;
        int rc = tuned_config(mc, grad, s, &cfg);
        if (rc) return rc;
        BatchPlan*& np = owner->plans[key];
        np = new BatchPlan();
        rc = build_plan(mc, grad, cfg, np);
        if (rc) { free_plan(np); owner->plans.erase(key); return rc; }
        if (owner->use_graph) {
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                rc = enqueue_plan(mc, grad, np, owner->d_gctr, s);
                e = hipStreamEndCapture(s, &g);
            }
            if (!rc && e == hipSuccess) {
                e = hipGraphInstantiate(&np->graph, g, nullptr, nullptr, 0);
                if (e != hipSuccess) np->graph = nullptr;
            }
            if (g) (void)hipGraphDestroy(g);
            if (rc || e != hipSuccess) {  // no half-built plan stays cached
                free_plan(np);
                owner->plans.erase(key);
                return rc ? rc : fail(NR_EHIP, "graph capture: %s", hipGetErrorString(e));
            }
        }
        np->epoch = g_epoch;
        BatchPlan* use = np;
        if (use->graph) HIPCHK(hipGraphLaunch(use->graph, s));
        else return enqueue_plan(mc, grad, use, owner->d_gctr, s);
        return 0;
    }
    if (pl->graph) HIPCHK(hipGraphLaunch(pl->graph, s));
    else return enqueue_plan(mc, grad, pl, owner->d_gctr, s);
    return 0;
}

int check_multi(nr_ctx* const* ctx, int n_ctx, const int* n_pts) {
    if (!ctx || n_ctx <= 0 || !n_pts) return fail(NR_EINVAL, "null argument or n_ctx <= 0");
    for (int d = 0; d < n_ctx; ++d) {
        int rc;
        if ((rc = check_ready(ctx[d]))) return rc;
        if ((rc = check_single(ctx[d]))) return rc;
        if (n_pts[d] <= 0) return fail(NR_EINVAL, "n_pts[%d] <= 0", d);
        if (ctx[d]->device != ctx[0]->device)
            return fail(NR_EINVAL, "all contexts of a grouped call share one device");
    }
    return 0;
}

int batched_sync(nr_ctx* c, const double* theta, int n_pts, double* nll,
                 double* grad, double* mu) {
    int rc;
    if ((rc = check_ready(c))) return rc;
    if ((rc = check_single(c))) return rc;
    if ((rc = check_theta(theta, n_pts))) return rc;
    if ((rc = set_device(c))) return rc;
    if ((rc = ensure_batch(c, n_pts, grad != nullptr, mu ? (size_t)n_pts * c->n_reco : 0)))
        return rc;
    HIPCHK(hipMemcpyAsync(c->d_bth, theta, sizeof(double) * n_pts * NR_NTHETA,
                          hipMemcpyHostToDevice, c->stream));
    nr_ctx* cs[1] = {c};
    const double* ths[1] = {c->d_bth};
    double* nls[1] = {c->d_bnll};
    double* grs[1] = {c->d_bgrad};
    double* mus[1] = {c->d_bmu};
    MultiCall mc{cs, 1, ths, &n_pts, nls, grad ? grs : nullptr, mu ? mus : nullptr};
    if ((rc = run_multi(mc, c->stream))) return rc;
    if (nll)
        HIPCHK(hipMemcpyAsync(nll, c->d_bnll, sizeof(double) * n_pts, hipMemcpyDeviceToHost, c->stream));
    if (grad)
        HIPCHK(hipMemcpyAsync(grad, c->d_bgrad, sizeof(double) * n_pts * NR_NTHETA,
                              hipMemcpyDeviceToHost, c->stream));
    if (mu)
        HIPCHK(hipMemcpyAsync(mu, c->d_bmu, sizeof(double) * n_pts * c->n_reco,
                              hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

}  // namespace

extern "C" {

const char* nr_last_error(void) { return g_err.c_str(); }

int nr_create(int device, nr_ctx** out) {
    const ApiLock api_lock;
    if (!out) return fail(NR_EINVAL, "out is null");
    *out = nullptr;
    int ndev = 0;
    HIPCHK(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(NR_EINVAL, "device %d out of range (%d devices)", device, ndev);
    nr_ctx* c = new (std::nothrow) nr_ctx();
    if (!c) return fail(NR_ENOMEM, "context allocation");
    c->device = device;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete c;
        return fail(NR_EHIP, "stream creation: %s", hipGetErrorString(e));
    }
    if (int rc = lookup_scratch(device, ndev)) {
        nr_destroy(c);
        return rc;
    }
    if (dalloc(&c->d_a, 1) || dalloc(&c->d_gb, 1) || dalloc(&c->d_thsm, nr::kMaxTheta) ||
        dalloc(&c->d_gctr, 4) || dalloc(&c->d_tnll, 1 + NR_NTHETA)) {
        delete c;
        return NR_ENOMEM;
    }
    (void)hipMemset(c->d_gctr, 0, 4 * sizeof(unsigned));
    // the SM point of either form: NSI and m2 zero, every rate one
    double sm[nr::kMaxTheta];
    for (int i = 0; i < nr::kMaxTheta; ++i) sm[i] = i < 5 ? 0.0 : 1.0;
    (void)hipMemcpy(c->d_thsm, sm, sizeof(sm), hipMemcpyHostToDevice);
    *out = c;
    return 0;
}

void nr_destroy(nr_ctx* c) {
    const ApiLock api_lock;
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    clear_graphs(c);
    dfree(&c->d_E); dfree(&c->d_W); dfree(&c->d_Pe); dfree(&c->d_tc);
    dfree(&c->d_ssm); dfree(&c->d_basis); dfree(&c->d_tnll); dfree(&c->d_nev);
    dfree(&c->d_compoff); dfree(&c->d_compsrc); dfree(&c->d_group0);
    dfree(&c->d_ssmc); dfree(&c->d_bkg); dfree(&c->d_mask);
    dfree(&c->d_group); dfree(&c->d_jmin); dfree(&c->d_srcoff);
    dfree(&c->d_table[0]); dfree(&c->d_table[1]); dfree(&c->d_R); dfree(&c->d_mrow);
    dfree(&c->d_n); dfree(&c->d_b); dfree(&c->d_colpart);
    dfree(&c->d_chunk_dev); dfree(&c->d_chunk_gb);
    dfree(&c->d_a); dfree(&c->d_gb); dfree(&c->d_jpart);
    dfree(&c->d_th); dfree(&c->d_out); dfree(&c->d_grad);
    dfree(&c->d_mu); dfree(&c->d_w); dfree(&c->d_thsm);
    dfree(&c->d_wt); dfree(&c->d_bpart); dfree(&c->d_bpgb); dfree(&c->d_bat);
    dfree(&c->d_bu); dfree(&c->d_bth); dfree(&c->d_bnll); dfree(&c->d_bgrad);
    dfree(&c->d_bmu); dfree(&c->d_gctr);
    dfree(&c->d_trec); dfree(&c->d_tdp); dfree(&c->d_thp); dfree(&c->d_tred);
    dfree(&c->d_v[0]); dfree(&c->d_v[1]);
    dfree(&c->d_rowband); dfree(&c->d_tileband);
    dfree(&c->d_scanblk); dfree(&c->d_ctot[0]); dfree(&c->d_ctot[1]);
    free_pinned(c);
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    (void)hipStreamDestroy(c->stream);
    delete c;
}

void* nr_stream(nr_ctx* c) { return c ? (void*)c->stream : nullptr; }

int nr_set_sources(nr_ctx* c, const nr_source* src, int n_src, int n_t,
                   double t_lo, double t_hi, const nr_physics* phys) {
    const ApiLock api_lock;
    if (!c || !src || n_src <= 0 || n_t <= 0)
        return fail(NR_EINVAL, "null argument or non-positive size");
    if (!(std::isfinite(t_lo) && std::isfinite(t_hi) && t_hi > t_lo && t_lo >= 0))
        return fail(NR_EINVAL, "recoil range must satisfy 0 <= t_lo < t_hi");
    if (c->have_rsp && n_t != c->n_t)
        return fail(NR_EINVAL, "n_t %d differs from the response (%d)", n_t, c->n_t);
    if (phys && !(phys->me > 0 && phys->gf > 0 && phys->alpha_em > 0 &&
                  phys->tau_frac >= 0 && phys->tau_frac <= 1))
        return fail(NR_EINVAL, "invalid physical constants");
    int rc;
    if ((rc = set_device(c))) return rc;
    c->ph = make_phys(phys);
    // copy, validate and sort the node tables (summation order is free)
    c->src_off.assign(n_src + 1, 0);
    c->src_n.assign(n_src, 0);
    c->src_group.assign(n_src, 0);
    c->hE.clear(); c->hW.clear(); c->hPe.clear();
    double wmax = 0;
    for (int k = 0; k < n_src; ++k) {
        const nr_source& s = src[k];
        if (s.n <= 0 || !s.E || !s.weight || !s.p_ee)
            return fail(NR_EINVAL, "source %d: empty or null arrays", k);
        if (s.kind == 0 && s.n != 1)
            return fail(NR_EINVAL, "source %d: a line has exactly one node", k);
        if (s.group != 0 && s.group != 1)
            return fail(NR_EINVAL, "source %d: group must be 0 or 1", k);
        std::vector<int> idx(s.n);
        for (int j = 0; j < s.n; ++j) {
            idx[j] = j;
            if (!(std::isfinite(s.E[j]) && s.E[j] > 0 && std::isfinite(s.weight[j])
                  && s.weight[j] >= 0 && s.p_ee[j] >= 0 && s.p_ee[j] <= 1))
                return fail(NR_EINVAL, "source %d node %d: invalid E/weight/p_ee", k, j);
            wmax = std::max(wmax, s.weight[j]);
        }
        std::stable_sort(idx.begin(), idx.end(),
                         [&](int a, int b) { return s.E[a] < s.E[b]; });
        c->src_off[k] = (int)c->hE.size();
        c->src_n[k] = s.n;
        c->src_group[k] = s.group;
        for (int j : idx) {
            c->hE.push_back(s.E[j]);
            c->hW.push_back(s.weight[j]);
            c->hPe.push_back(s.p_ee[j]);
        }
    }
    if (!(wmax > 0)) return fail(NR_EINVAL, "all source weights are zero");
    // S is linear in the weights and only ratios enter w; scale to O(1).
    for (double& w : c->hW) w /= wmax;
    if (c->multi) {  // new sources drop the components built on the old ones
        c->multi = false;
        c->have_rsp = c->have_data = false;
        c->n_theta = NR_NTHETA;
        c->n_comp = c->n_bkg = 1;
    }
    c->n_src = n_src;
    c->n_nodes = (int)c->hE.size();
    c->src_off[n_src] = c->n_nodes;
    c->n_t = n_t;
    c->n_rows = n_t;
    c->t_lo = t_lo;
    c->t_hi = t_hi;
    c->tc.resize(n_t);
    const double dt = (t_hi - t_lo) / n_t;
    for (int l = 0; l < n_t; ++l) c->tc[l] = t_lo + (l + 0.5) * dt;
    // first reachable node of every (source, row); rows are increasing in T
    // and T_max(E) is increasing in E, so the reachable nodes are a suffix.
    c->jmin.assign((size_t)n_src * n_t, 0);
    for (int k = 0; k < n_src; ++k) {
        const int off = c->src_off[k], n = c->src_n[k];
        for (int l = 0; l < n_t; ++l) {
            int lo = 0, hi = n;
            while (lo < hi) {
                int mid = (lo + hi) / 2;
                if (reach(c->ph.me, c->hE[off + mid], c->tc[l])) hi = mid;
                else lo = mid + 1;
            }
            c->jmin[(size_t)k * n_t + l] = off + lo;
        }
    }
    c->n_blocks = (n_t + nr::kStepRows - 1) / nr::kStepRows;
    // theta-independent basis spectra (FP64), used by the adjoint
    c->basis.assign((size_t)nr::kNBasis * n_t, 0.0);
    for (int l = 0; l < n_t; ++l)
        for (int k = 0; k < n_src; ++k) {
            double acc[10];
            source_basis(c, k, l, acc);
            const int g = c->src_group[k] ? 10 : 0;
            for (int q = 0; q < 10; ++q)
                c->basis[(size_t)(g + q) * n_t + l] += acc[q];
        }
    // upload
    if ((rc = dalloc(&c->d_E, c->n_nodes)) || (rc = dalloc(&c->d_W, c->n_nodes)) ||
        (rc = dalloc(&c->d_Pe, c->n_nodes)) || (rc = dalloc(&c->d_tc, n_t)) ||
        (rc = dalloc(&c->d_ssm, n_t)) || (rc = dalloc(&c->d_group, n_src)) ||
        (rc = dalloc(&c->d_jmin, (size_t)n_src * n_t)) ||
        (rc = dalloc(&c->d_srcoff, n_src + 1)) ||
        (rc = dalloc(&c->d_compoff, n_src + 1)) || (rc = dalloc(&c->d_compsrc, n_src)) ||
        (rc = dalloc(&c->d_group0, n_src)) ||
        (rc = dalloc(&c->d_table[0], (size_t)4 * (c->n_nodes + n_src))) ||
        (rc = dalloc(&c->d_table[1], (size_t)4 * (c->n_nodes + n_src))) ||
        (rc = dalloc(&c->d_basis, (size_t)nr::kNBasis * n_t)) ||
        (rc = dalloc(&c->d_v[0], n_t)) || (rc = dalloc(&c->d_v[1], n_t)))
        return rc;
    {
        // one node-scan work-group per 512 nodes of each source
        std::vector<int> blk;
        c->max_chunks = 1;
        for (int k = 0; k < n_src; ++k) {
            const int nch = std::max(1, (c->src_n[k] + nr::kStepRows - 1) / nr::kStepRows);
            c->max_chunks = std::max(c->max_chunks, nch);
            for (int h = 0; h < nch; ++h) {
                blk.push_back(k);
                blk.push_back(h);
            }
        }
        c->nb_scan = (int)blk.size() / 2;
        if ((rc = dalloc(&c->d_scanblk, blk.size())) ||
            (rc = dalloc(&c->d_ctot[0], (size_t)4 * n_src * c->max_chunks)) ||
            (rc = dalloc(&c->d_ctot[1], (size_t)4 * n_src * c->max_chunks)))
            return rc;
        HIPCHK(hipMemcpy(c->d_scanblk, blk.data(), sizeof(int) * blk.size(),
                         hipMemcpyHostToDevice));
    }
    {
        std::vector<double> ie(c->n_nodes);
        for (int j = 0; j < c->n_nodes; ++j) ie[j] = 1.0 / c->hE[j];
        HIPCHK(hipMemcpy(c->d_E, ie.data(), sizeof(double) * c->n_nodes, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(c->d_W, c->hW.data(), sizeof(double) * c->n_nodes, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_Pe, c->hPe.data(), sizeof(double) * c->n_nodes, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_tc, c->tc.data(), sizeof(double) * n_t, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_group, c->src_group.data(), sizeof(int) * n_src, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_jmin, c->jmin.data(), sizeof(int) * c->jmin.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_srcoff, c->src_off.data(), sizeof(int) * (n_src + 1), hipMemcpyHostToDevice));
    // the single-component form: one component holding every source
    c->comp_off = {0, n_src};
    c->comp_src.resize(n_src);
    for (int k = 0; k < n_src; ++k) c->comp_src[k] = k;
    HIPCHK(hipMemcpy(c->d_compoff, c->comp_off.data(), sizeof(int) * 2, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_compsrc, c->comp_src.data(), sizeof(int) * n_src, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(c->d_group0, 0, sizeof(int) * n_src));
    HIPCHK(hipMemcpy(c->d_basis, c->basis.data(), sizeof(double) * c->basis.size(), hipMemcpyHostToDevice));
    // SM reference on the device with the same E-integral code the
    // evaluations use, so that w = S_theta / S_SM is exactly 1 at theta_SM.
    {
        const nr::ScanArgs sa = scan_args(c, c->d_thsm, 0);
        const nr::RowArgs ra = row_args(c, 0, nullptr, nullptr, c->d_ssm, c->d_thsm);
        if ((rc = step(c, nullptr, nullptr, &sa, nullptr, c->stream))) return rc;
        if ((rc = step(c, nullptr, &ra, nullptr, nullptr, c->stream))) return rc;
    }
    c->ssm.resize(n_t);
    HIPCHK(hipMemcpyAsync(c->ssm.data(), c->d_ssm, sizeof(double) * n_t,
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->have_src = true;
    c->tmpl_ok = false;
    clear_graphs(c);
    recompute_mrow(c);
    if ((rc = upload_mrow(c))) return rc;
    return 0;
}

int nr_set_response(nr_ctx* c, const float* R, int n_t, int n_reco,
                    const double* m, double n_sig) {
    const ApiLock api_lock;
    if (!c || !R || n_t <= 0 || n_reco <= 0)
        return fail(NR_EINVAL, "null argument or non-positive size");
    if (c->have_src && n_t != c->n_t)
        return fail(NR_EINVAL, "n_t %d differs from the sources (%d)", n_t, c->n_t);
    if (c->have_data && n_reco != c->n_reco)
        return fail(NR_EINVAL, "n_reco %d differs from the data (%d)", n_reco, c->n_reco);
    if (!m && !c->have_src)
        return fail(NR_ESTATE, "m == NULL needs set_sources first");
    if (!m && !(std::isfinite(n_sig) && n_sig >= 0))
        return fail(NR_EINVAL, "n_sig must be finite and >= 0");
    if (m && !finite_all(m, n_t)) return fail(NR_EINVAL, "non-finite m");
    const size_t nel = (size_t)n_t * n_reco;
    for (size_t i = 0; i < nel; ++i)
        if (!std::isfinite(R[i])) return fail(NR_EINVAL, "non-finite R at %zu", i);
    int rc;
    if ((rc = set_device(c))) return rc;
    if (c->multi) {  // back to the single-component form
        c->multi = false;
        c->have_data = false;
        c->n_theta = NR_NTHETA;
        c->n_comp = c->n_bkg = 1;
        if (c->have_src) {
            if ((rc = dalloc(&c->d_v[0], n_t)) || (rc = dalloc(&c->d_v[1], n_t))) return rc;
            c->comp_off = {0, c->n_src};
            c->comp_src.resize(c->n_src);
            for (int q = 0; q < c->n_src; ++q) c->comp_src[q] = q;
            HIPCHK(hipMemcpy(c->d_compoff, c->comp_off.data(), sizeof(int) * 2,
                             hipMemcpyHostToDevice));
            HIPCHK(hipMemcpy(c->d_compsrc, c->comp_src.data(), sizeof(int) * c->n_src,
                             hipMemcpyHostToDevice));
        }
    }
    c->n_t = n_t;
    c->n_rows = n_t;
    c->n_reco = n_reco;
    c->ldr = (n_reco + 3) / 4 * 4;
    if ((rc = dalloc(&c->d_R, (size_t)n_t * c->ldr))) return rc;
    if (c->ldr != n_reco)
        HIPCHK(hipMemset(c->d_R, 0, sizeof(float) * (size_t)n_t * c->ldr));
    HIPCHK(hipMemcpy2D(c->d_R, sizeof(float) * c->ldr, R, sizeof(float) * n_reco,
                       sizeof(float) * n_reco, n_t, hipMemcpyHostToDevice));
    if ((rc = set_row_bands(c, R, n_t, n_reco, n_reco))) return rc;
    if ((rc = dalloc(&c->d_mrow, n_t))) return rc;
    if ((rc = dalloc(&c->d_a, c->ldr))) return rc;
    c->m_user = m != nullptr;
    c->n_sig = n_sig;
    if (m) c->mrow.assign(m, m + n_t);
    c->have_rsp = true;
    c->tmpl_ok = false;
    recompute_mrow(c);
    if ((rc = upload_mrow(c))) return rc;
    if ((rc = choose_tiling(c, 0))) return rc;
    return 0;
}

int nr_set_data(nr_ctx* c, const double* n, const double* b, int n_reco,
                const double* pull_mean, const double* pull_sigma) {
    const ApiLock api_lock;
    if (!c || !n || n_reco <= 0) return fail(NR_EINVAL, "null argument or n_reco <= 0");
    if (!b && !c->multi) return fail(NR_EINVAL, "b is null");
    if (c->have_rsp && n_reco != c->n_reco)
        return fail(NR_EINVAL, "n_reco %d differs from the response (%d)", n_reco, c->n_reco);
    if ((pull_mean == nullptr) != (pull_sigma == nullptr))
        return fail(NR_EINVAL, "pull_mean and pull_sigma must both be given or both NULL");
    for (int j = 0; j < n_reco; ++j) {
        if (!(std::isfinite(n[j]) && n[j] >= 0)) return fail(NR_EINVAL, "n[%d] must be finite and >= 0", j);
        if (b && !(std::isfinite(b[j]) && b[j] >= 0)) return fail(NR_EINVAL, "b[%d] must be finite and >= 0", j);
    }
    if (pull_mean && (!finite_all(pull_mean, c->n_theta) || !finite_all(pull_sigma, c->n_theta)))
        return fail(NR_EINVAL, "non-finite pulls");
    int rc;
    if ((rc = set_device(c))) return rc;
    if ((rc = dalloc(&c->d_n, n_reco)) || (rc = dalloc(&c->d_b, n_reco))) return rc;
    HIPCHK(hipMemcpy(c->d_n, n, sizeof(double) * n_reco, hipMemcpyHostToDevice));
    if (b) HIPCHK(hipMemcpy(c->d_b, b, sizeof(double) * n_reco, hipMemcpyHostToDevice));
    else HIPCHK(hipMemset(c->d_b, 0, sizeof(double) * n_reco));
    // data-only constant of Eq. (logL): the device reduces the deviance
    // mu - n + n ln(n/mu); -2lnL = 2 (deviance + C_data) + pulls.
    double cd = 0, lg = 0;
    for (int j = 0; j < n_reco; ++j) {
        const double l = std::lgamma(n[j] + 1.0);
        cd += n[j] - (n[j] > 0 ? n[j] * std::log(n[j]) : 0.0) + l;
        lg += l;
    }
    c->cdata = cd;
    c->lgsum = lg;
    for (int i = 0; i < nr::kMaxTheta; ++i) {
        c->pull_mean[i] = pull_mean && i < c->n_theta ? pull_mean[i] : 0.0;
        c->pull_sigma[i] = pull_sigma && i < c->n_theta ? pull_sigma[i] : 0.0;
    }
    c->n_reco = n_reco;
    c->have_data = true;
    c->tmpl_data_ok = false;  // the templates themselves stay valid
    clear_graphs(c);
    return 0;
}

int nr_eval_nll_dev(nr_ctx* c, const double* d_theta, int n_pts, double* d_nll,
                    double* d_grad, void* stream) {
    const ApiLock api_lock;
    int rc;
    if ((rc = check_ready(c))) return rc;
    if (!d_theta || !d_nll || n_pts <= 0)
        return fail(NR_EINVAL, "null device pointer or n_pts <= 0");
    if (d_grad && (rc = check_single(c))) return rc;
    if ((rc = set_device(c))) return rc;
    Bridge br;
    if ((rc = bridge_begin(br, stream, c->stream, c->ev_in, c->ev_out))) return rc;
    if ((rc = run_points(c, d_theta, n_pts, d_nll, d_grad, nullptr, nullptr, br.work)))
        return rc;
    return bridge_end(br);
}

int nr_eval_nll_dev_noalloc(nr_ctx* c, const double* d_theta, int n_pts,
                            double* d_nll, double* d_grad, void* stream) {
    const ApiLock api_lock;
    int rc;
    if ((rc = check_ready(c))) return rc;
    if (!d_theta || !d_nll || n_pts <= 0)
        return fail(NR_EINVAL, "null device pointer or n_pts <= 0");
    if (d_grad && (rc = check_single(c))) return rc;
    if ((rc = set_device(c))) return rc;
    double* base = c->device < (int)g_scratch_dev.size() ? g_scratch_dev[c->device] : nullptr;
    if (!base) return fail(NR_ESTATE, "no static workspace on device %d", c->device);
    Work w;
    const size_t need = carve_work(c, nullptr, &w);
    if (need > (size_t)NR_NOALLOC_WORKSPACE_BYTES)
        return fail(NR_EINVAL, "this context's shapes need %zu bytes of workspace; "
                    "the static workspace holds %zu", need,
                    (size_t)NR_NOALLOC_WORKSPACE_BYTES);
    carve_work(c, base, &w);
    // launched directly on the caller's stream (no graph of our own), so
    // that a caller may capture them in its own graph
    Bridge br;
    if ((rc = bridge_begin(br, stream, c->stream, c->ev_in, c->ev_out))) return rc;
    if ((rc = enqueue_points(c, d_theta, n_pts, d_nll, d_grad, nullptr, nullptr,
                             br.work, &w)))
        return rc;
    return bridge_end(br);
}

static int eval_sync(nr_ctx* c, const double* theta, int n_pts, double* nll,
                     double* grad, double* mu, double* w) {
    int rc;
    if ((rc = check_ready(c))) return rc;
    if ((grad || w) && (rc = check_single(c))) return rc;
    if ((rc = check_theta(theta, n_pts, c->n_theta))) return rc;
    if ((rc = set_device(c))) return rc;
    if (!mu && !w) {
        // likelihood (and gradient): theta in and -2lnL out through pinned
        // host memory the kernels read and write directly, no copies
        if ((rc = ensure_pinned(c, n_pts))) return rc;
        std::memcpy(c->h_th, theta, sizeof(double) * n_pts * c->n_theta);
        rc = run_points(c, c->hd_th, n_pts, c->hd_out, grad ? c->hd_grad : nullptr,
                        nullptr, nullptr, c->stream);
        if (rc) return rc;
        HIPCHK(hipStreamSynchronize(c->stream));
        std::memcpy(nll, c->h_out, sizeof(double) * n_pts);
        if (grad) std::memcpy(grad, c->h_grad, sizeof(double) * n_pts * NR_NTHETA);
        return 0;
    }
    const size_t mu_elems = mu ? (size_t)n_pts * c->n_reco : 0;
    const size_t w_elems = w ? (size_t)n_pts * c->n_rows : 0;
    if ((rc = ensure_stage(c, n_pts, mu_elems, w_elems))) return rc;
    // every staged copy and every per-point offset the launches form
    // (theta, -2lnL, gradient, spectra, weights) lies inside the buffer
    // ensure_stage sized for it
    if ((size_t)n_pts > c->cap_pts || c->n_theta > nr::kMaxTheta ||
        mu_elems > c->cap_mu || w_elems > c->cap_w ||
        (mu && !c->d_mu) || (w && !c->d_w))
        return fail(NR_EHIP, "staging buffers too small for %d points "
                    "(capacity %zu points, %zu spectrum and %zu weight values)",
                    n_pts, c->cap_pts, c->cap_mu, c->cap_w);
    HIPCHK(hipMemcpyAsync(c->d_th, theta, sizeof(double) * n_pts * c->n_theta,
                          hipMemcpyHostToDevice, c->stream));
    rc = run_points(c, c->d_th, n_pts, c->d_out, grad ? c->d_grad : nullptr,
                    mu ? c->d_mu : nullptr, w ? c->d_w : nullptr, c->stream);
    if (rc) return rc;
    if (nll)
        HIPCHK(hipMemcpyAsync(nll, c->d_out, sizeof(double) * n_pts,
                              hipMemcpyDeviceToHost, c->stream));
    if (grad)
        HIPCHK(hipMemcpyAsync(grad, c->d_grad, sizeof(double) * n_pts * NR_NTHETA,
                              hipMemcpyDeviceToHost, c->stream));
    if (mu)
        HIPCHK(hipMemcpyAsync(mu, c->d_mu, sizeof(double) * n_pts * c->n_reco,
                              hipMemcpyDeviceToHost, c->stream));
    if (w)
        HIPCHK(hipMemcpyAsync(w, c->d_w, sizeof(double) * n_pts * c->n_t,
                              hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int nr_eval_nll(nr_ctx* c, const double* theta, int n_pts, double* nll) {
    const ApiLock api_lock;
    if (!nll) return fail(NR_EINVAL, "nll is null");
    return eval_sync(c, theta, n_pts, nll, nullptr, nullptr, nullptr);
}

int nr_eval_nll_grad(nr_ctx* c, const double* theta, int n_pts, double* nll,
                     double* grad) {
    const ApiLock api_lock;
    if (!nll || !grad) return fail(NR_EINVAL, "nll or grad is null");
    return eval_sync(c, theta, n_pts, nll, grad, nullptr, nullptr);
}

int nr_eval_mu(nr_ctx* c, const double* theta, int n_pts, double* mu) {
    const ApiLock api_lock;
    if (!mu) return fail(NR_EINVAL, "mu is null");
    return eval_sync(c, theta, n_pts, nullptr, nullptr, mu, nullptr);
}

int nr_set_mc_events(nr_ctx* c, const double* n_events, int n_t) {
    const ApiLock api_lock;
    if (!c || !n_events || n_t <= 0) return fail(NR_EINVAL, "null argument or n_t <= 0");
    if (int rc = check_single(c)) return rc;
    if (!c->have_rsp) return fail(NR_ESTATE, "nr_set_mc_events needs nr_set_response first");
    if (n_t != c->n_t) return fail(NR_EINVAL, "n_t %d differs from the response (%d)", n_t, c->n_t);
    for (int l = 0; l < n_t; ++l)
        if (!(std::isfinite(n_events[l]) && n_events[l] >= 0))
            return fail(NR_EINVAL, "n_events[%d] must be finite and >= 0", l);
    int rc;
    if ((rc = set_device(c))) return rc;
    if ((rc = dalloc(&c->d_nev, n_t))) return rc;
    HIPCHK(hipMemcpy(c->d_nev, n_events, sizeof(double) * n_t, hipMemcpyHostToDevice));
    c->have_nev = true;
    return 0;
}

int nr_eval_ess(nr_ctx* c, const double* theta, int n_pts, double* ess) {
    const ApiLock api_lock;
    int rc;
    if (!ess) return fail(NR_EINVAL, "ess is null");
    if ((rc = check_ready(c))) return rc;
    if ((rc = check_single(c))) return rc;
    if (!c->have_nev) return fail(NR_ESTATE, "nr_eval_ess needs nr_set_mc_events first");
    if ((rc = check_theta(theta, n_pts))) return rc;
    if ((rc = set_device(c))) return rc;
    if ((rc = ensure_stage(c, n_pts, (size_t)n_pts * c->n_reco, c->n_t))) return rc;
    HIPCHK(hipMemcpyAsync(c->d_th, theta, sizeof(double) * n_pts * NR_NTHETA,
                          hipMemcpyHostToDevice, c->stream));
    for (int p = 0; p < n_pts; ++p) {
        const nr::ScanArgs a1 = scan_args(c, c->d_th + (size_t)p * NR_NTHETA, 0);
        const nr::RowArgs a2 = row_args(c, 0, c->d_v[0], c->d_w, nullptr,
                                        c->d_th + (size_t)p * NR_NTHETA);
        if ((rc = step(c, nullptr, nullptr, &a1, nullptr, c->stream))) return rc;
        if ((rc = step(c, nullptr, &a2, nullptr, nullptr, c->stream))) return rc;
        nr::EssArgs ea{};
        ea.R = c->d_R;
        ea.ldr = c->ldr;
        ea.n_t = c->n_t;
        ea.n_reco = c->n_reco;
        ea.w = c->d_w;
        ea.nev = c->d_nev;
        ea.colpart = c->d_colpart;
        ea.rows_per_wg = c->rows_per_wg;
        ea.n_rb = c->n_rb;
        ea.n_cc = nr::ess_col_tiles(c->ldr);  // the ESS fold's own column tiles
        ea.out = c->d_mu + (size_t)p * c->n_reco;
        HIPCHK(nr::launch_ess(ea, c->stream));
    }
    HIPCHK(hipMemcpyAsync(ess, c->d_mu, sizeof(double) * n_pts * c->n_reco,
                          hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int nr_num_theta(nr_ctx* c) { return c ? c->n_theta : NR_EINVAL; }

int nr_set_components(nr_ctx* c, const nr_components* k, int n_reco) {
    const ApiLock api_lock;
    if (!c || !k || n_reco <= 0) return fail(NR_EINVAL, "null argument or n_reco <= 0");
    if (!c->have_src) return fail(NR_ESTATE, "nr_set_components needs nr_set_sources first");
    const int K = k->n_comp, B = k->n_bkg, n_t = c->n_t, n_src = c->n_src;
    if (K <= 0 || B < 0 || 5 + K + B > nr::kMaxTheta)
        return fail(NR_EINVAL, "need n_comp >= 1, n_bkg >= 0 and 5 + n_comp + n_bkg <= %d",
                    nr::kMaxTheta);
    if (!k->comp_of_source || !k->hist || !k->scale || !k->rate_sm ||
        (B > 0 && (!k->bkg_pdf || !k->bkg_rate)))
        return fail(NR_EINVAL, "null component or background array");
    if (!(std::isfinite(k->exposure) && k->exposure > 0))
        return fail(NR_EINVAL, "exposure must be finite and > 0");
    // sources grouped by component, in source order within a component
    std::vector<int> off(K + 1, 0), src(n_src);
    for (int s = 0; s < n_src; ++s) {
        const int q = k->comp_of_source[s];
        if (q < 0 || q >= K) return fail(NR_EINVAL, "source %d: component %d out of range", s, q);
        ++off[q + 1];
    }
    for (int q = 0; q < K; ++q) {
        if (off[q + 1] == 0) return fail(NR_EINVAL, "component %d has no source", q);
        off[q + 1] += off[q];
    }
    {
        std::vector<int> fill(off.begin(), off.end() - 1);
        for (int s = 0; s < n_src; ++s) src[fill[k->comp_of_source[s]]++] = s;
    }
    for (int q = 0; q < K; ++q) {
        if (!(std::isfinite(k->scale[q]) && k->scale[q] > 0))
            return fail(NR_EINVAL, "scale[%d] must be finite and > 0", q);
        if (!(std::isfinite(k->rate_sm[q]) && k->rate_sm[q] >= 0))
            return fail(NR_EINVAL, "rate_sm[%d] must be finite and >= 0", q);
    }
    for (int b = 0; b < B; ++b) {
        if (!(std::isfinite(k->bkg_rate[b]) && k->bkg_rate[b] >= 0))
            return fail(NR_EINVAL, "bkg_rate[%d] must be finite and >= 0", b);
        for (int j = 0; j < n_reco; ++j) {
            const double v = k->bkg_pdf[(size_t)b * n_reco + j];
            if (!(std::isfinite(v) && v >= 0))
                return fail(NR_EINVAL, "bkg_pdf[%d][%d] must be finite and >= 0", b, j);
        }
    }
    if (k->mask)
        for (int j = 0; j < n_reco; ++j)
            if (!(std::isfinite(k->mask[j]) && k->mask[j] >= 0))
                return fail(NR_EINVAL, "mask[%d] must be finite and >= 0", j);
    // Eq. (Rij): R^(k)_ij = (N^(k)_ij / M^(k)_j) / sum_{i'j'} (N^(k)_i'j' / M^(k)_j')
    // x s^(k), formed in FP64 and stored in FP32, the components stacked
    // row-wise
    const int ldr = (n_reco + 3) / 4 * 4;
    const size_t n_rows = (size_t)K * n_t;
    std::vector<float> Rs(n_rows * ldr, 0.0f);
    for (int q = 0; q < K; ++q) {
        const float* N = k->hist + (size_t)q * n_t * n_reco;
        const double* M = k->comp_mask ? k->comp_mask + (size_t)q * n_reco : nullptr;
        double tot = 0.0;
        for (int i = 0; i < n_t; ++i)
            for (int j = 0; j < n_reco; ++j) {
                const double v = N[(size_t)i * n_reco + j];
                if (!(std::isfinite(v) && v >= 0))
                    return fail(NR_EINVAL, "hist[%d][%d][%d] must be finite and >= 0", q, i, j);
                if (v == 0.0) continue;
                if (M && !(std::isfinite(M[j]) && M[j] > 0))
                    return fail(NR_EINVAL, "comp_mask[%d][%d] must be > 0 where the histogram is not", q, j);
                tot += M ? v / M[j] : v;
            }
        if (!(tot > 0)) return fail(NR_EINVAL, "component %d: empty histogram", q);
        const double f = k->scale[q] / tot;
        for (int i = 0; i < n_t; ++i)
            for (int j = 0; j < n_reco; ++j) {
                const double v = N[(size_t)i * n_reco + j];
                if (v != 0.0)
                    Rs[((size_t)q * n_t + i) * ldr + j] = (float)((M ? v / M[j] : v) * f);
            }
    }
    // Eq. (mu_total): MT x rate; the signal rows carry MT Rate_SM,k (the
    // theta-dependent share of the rate comes with the unnormalised weights
    // and the component's rate parameter), the templates MT Rate_b f_b,j.
    std::vector<double> mrow(n_rows), bkg((size_t)std::max(B, 1) * n_reco, 0.0);
    for (int q = 0; q < K; ++q)
        for (int i = 0; i < n_t; ++i) mrow[(size_t)q * n_t + i] = k->exposure * k->rate_sm[q];
    for (int b = 0; b < B; ++b)
        for (int j = 0; j < n_reco; ++j)
            bkg[(size_t)b * n_reco + j] =
                k->exposure * k->bkg_rate[b] * k->bkg_pdf[(size_t)b * n_reco + j];
    int rc;
    if ((rc = set_device(c))) return rc;
    clear_graphs(c);
    if ((rc = dalloc(&c->d_R, n_rows * ldr)) || (rc = dalloc(&c->d_mrow, n_rows)) ||
        (rc = dalloc(&c->d_bkg, bkg.size())) || (rc = dalloc(&c->d_ssmc, n_rows)) ||
        (rc = dalloc(&c->d_v[0], n_rows)) || (rc = dalloc(&c->d_v[1], n_rows)) ||
        (rc = dalloc(&c->d_compoff, K + 1)) || (rc = dalloc(&c->d_compsrc, n_src)) ||
        (rc = dalloc(&c->d_a, ldr)))
        return rc;
    dfree(&c->d_mask);
    if (k->mask) {
        if ((rc = dalloc(&c->d_mask, n_reco))) return rc;
        HIPCHK(hipMemcpy(c->d_mask, k->mask, sizeof(double) * n_reco, hipMemcpyHostToDevice));
    }
    HIPCHK(hipMemcpy(c->d_R, Rs.data(), sizeof(float) * Rs.size(), hipMemcpyHostToDevice));
    if ((rc = set_row_bands(c, Rs.data(), (int)n_rows, n_reco, ldr))) return rc;
    HIPCHK(hipMemcpy(c->d_mrow, mrow.data(), sizeof(double) * n_rows, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_bkg, bkg.data(), sizeof(double) * bkg.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_compoff, off.data(), sizeof(int) * (K + 1), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->d_compsrc, src.data(), sizeof(int) * n_src, hipMemcpyHostToDevice));
    c->comp_off = off;
    c->comp_src = src;
    c->multi = true;
    c->tmpl_ok = false;
    c->n_comp = K;
    c->n_bkg = B;
    c->n_theta = 5 + K + B;
    c->n_rows = (int)n_rows;
    c->n_reco = n_reco;
    c->ldr = ldr;
    c->m_user = true;
    c->have_rsp = true;
    c->have_data = false;  // data and pulls follow the new parameter layout
    // per-component SM spectra with the code the evaluations use (w = 1
    // exactly at the SM point)
    {
        const nr::ScanArgs sa = scan_args(c, c->d_thsm, 0);
        const nr::RowArgs ra = row_args(c, 0, nullptr, nullptr, c->d_ssmc, c->d_thsm);
        if ((rc = step(c, nullptr, nullptr, &sa, nullptr, c->stream))) return rc;
        if ((rc = step(c, nullptr, &ra, nullptr, nullptr, c->stream))) return rc;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    if ((rc = choose_tiling(c, 0))) return rc;
    return 0;
}

int nr_eval_weights(nr_ctx* c, const double* theta, int n_pts, double* w) {
    const ApiLock api_lock;
    if (!w) return fail(NR_EINVAL, "w is null");
    return eval_sync(c, theta, n_pts, nullptr, nullptr, nullptr, w);
}

int nr_get_reference(nr_ctx* c, double* s_sm, double* m) {
    const ApiLock api_lock;
    if (!c) return fail(NR_EINVAL, "null context");
    if (int rc = check_single(c)) return rc;
    if (s_sm) {
        if (!c->have_src) return fail(NR_ESTATE, "no sources set");
        std::memcpy(s_sm, c->ssm.data(), sizeof(double) * c->n_t);
    }
    if (m) {
        if (!c->have_rsp) return fail(NR_ESTATE, "no response set");
        std::memcpy(m, c->mrow.data(), sizeof(double) * c->n_t);
    }
    return 0;
}

int nr_set_fold_tiling(nr_ctx* c, int rows_per_wg, int use_graph) {
    const ApiLock api_lock;
    if (!c) return fail(NR_EINVAL, "null context");
    if (use_graph >= 0) c->use_graph = use_graph != 0;
    clear_graphs(c);
    if (rows_per_wg > 0) {
        if (!c->have_rsp) return fail(NR_ESTATE, "no response set");
        if (rows_per_wg > 2048 || rows_per_wg % 8)
            return fail(NR_EINVAL, "rows_per_wg must be a multiple of 8 and <= 2048");
        int rc;
        if ((rc = set_device(c))) return rc;
        HIPCHK(hipStreamSynchronize(c->stream));
        return choose_tiling(c, rows_per_wg);
    }
    return 0;
}

int nr_set_band_skipping(nr_ctx* c, int on) {
    const ApiLock api_lock;
    if (!c) return fail(NR_EINVAL, "null context");
    if (!c->have_rsp) return fail(NR_ESTATE, "band skipping needs a response first");
    if ((on != 0) != c->skip_zero) {
        c->skip_zero = on != 0;
        clear_graphs(c);  // cached graphs hold the other setting
    }
    return 0;
}

int nr_time_stage(nr_ctx* c, int stage, int iters, double* avg_ms) {
    const ApiLock api_lock;
    if (!c || !avg_ms || iters <= 0) return fail(NR_EINVAL, "bad argument");
    if (stage < 1 || stage > 5) return fail(NR_EINVAL, "stage must be 1 to 5");
    int rc;
    if ((rc = check_ready(c))) return rc;
    if (stage == 3 && (rc = check_single(c))) return rc;
    if ((rc = set_device(c))) return rc;
    // Timing launches read the context's own inputs at the SM point (the
    // work of every stage does not depend on theta) and write only internal
    // buffers: the fold reads fold vector 0 and writes partial sums 0, the
    // table and weights of the same launch go to copy 1, the reduction reads
    // partial sums 1 into group sums 1, the final role adds group sums 0
    // into a scratch word.
    const size_t cp = (size_t)c->n_rb * c->ldr;
    const double* th = c->d_thsm;
    const nr::FoldArgs f = fold_args(c, th, c->d_v[0], c->d_colpart, c->d_tnll,
                                     nullptr, false, 0);
    const nr::ScanArgs sa = scan_args(c, th, 1);
    const nr::RowArgs ra = row_args(c, 0, c->d_v[1], nullptr, nullptr, th);
    const nr::FoldArgs g = fold_args(c, th, c->d_v[1], c->d_colpart + cp, c->d_tnll,
                                     nullptr, false, 1);
    const nr::FoldArgs fo = g;
    nr::AdjArgs aa{};
    if (stage == 3) {
        aa.R = c->d_R;
        aa.ldr = c->ldr;
        aa.n_t = c->n_t;
        aa.n_reco = c->n_reco;
        aa.a = c->d_a;
        aa.ssm = c->d_ssm;
        aa.mrow = c->d_mrow;
        aa.basis = c->d_basis;
        aa.theta = th;
        aa.gb = c->d_gb;
        aa.jpart = c->d_jpart;
        aa.out_grad = c->d_tnll + 1;
        aa.ph = c->ph;
    }
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    HIPCHK(hipEventRecord(e0, c->stream));
    for (int i = 0; i < iters; ++i) {
        if (stage == 1) {
            rc = step(c, nullptr, nullptr, &sa, nullptr, c->stream);
            if (!rc) rc = step(c, nullptr, &ra, nullptr, nullptr, c->stream);
        }
        if (stage == 2) {
            rc = step(c, &fo, nullptr, nullptr, nullptr, c->stream);
            if (!rc) rc = step(c, nullptr, nullptr, nullptr, &g, c->stream);
            if (!rc) rc = step(c, nullptr, nullptr, nullptr, nullptr, c->stream, &g);
        }
        if (stage == 3) HIPCHK(nr::launch_adjoint(aa, c->adj_grid, c->stream));
        if (stage == 4) rc = step(c, &fo, nullptr, nullptr, nullptr, c->stream);
        if (stage == 5) rc = step(c, &f, &ra, &sa, &g, c->stream, &f);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(e1, c->stream));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *avg_ms = ms / iters;
    return 0;
}

int nr_eval_nll_batched(nr_ctx* c, const double* theta, int n_pts, double* nll) {
    const ApiLock api_lock;
    if (!nll) return fail(NR_EINVAL, "nll is null");
    return batched_sync(c, theta, n_pts, nll, nullptr, nullptr);
}

int nr_eval_nll_grad_batched(nr_ctx* c, const double* theta, int n_pts,
                             double* nll, double* grad) {
    const ApiLock api_lock;
    if (!nll || !grad) return fail(NR_EINVAL, "nll or grad is null");
    return batched_sync(c, theta, n_pts, nll, grad, nullptr);
}

int nr_eval_mu_batched(nr_ctx* c, const double* theta, int n_pts, double* mu) {
    const ApiLock api_lock;
    if (!mu) return fail(NR_EINVAL, "mu is null");
    return batched_sync(c, theta, n_pts, nullptr, nullptr, mu);
}

int nr_eval_nll_multi_dev(nr_ctx* const* ctx, int n_ctx,
                          const double* const* d_theta, const int* n_pts,
                          double* const* d_nll, double* const* d_grad,
                          void* stream) {
    const ApiLock api_lock;
    int rc;
    if ((rc = check_multi(ctx, n_ctx, n_pts))) return rc;
    if (!d_theta || !d_nll) return fail(NR_EINVAL, "null theta or nll array");
    for (int d = 0; d < n_ctx; ++d) {
        if (!d_theta[d] || !d_nll[d] || (d_grad && !d_grad[d]))
            return fail(NR_EINVAL, "null device pointer for dataset %d", d);
    }
    if ((rc = set_device(ctx[0]))) return rc;
    for (int d = 0; d < n_ctx; ++d)
        if ((rc = ensure_batch(ctx[d], n_pts[d], d_grad != nullptr, 0))) return rc;
    Bridge br;
    if ((rc = bridge_begin(br, stream, ctx[0]->stream, ctx[0]->ev_in, ctx[0]->ev_out)))
        return rc;
    MultiCall mc{ctx, n_ctx, d_theta, n_pts, d_nll, d_grad, nullptr};
    if ((rc = run_multi(mc, br.work))) return rc;
    return bridge_end(br);
}

int nr_eval_nll_multi(nr_ctx* const* ctx, int n_ctx, const double* const* theta,
                      const int* n_pts, double* const* nll) {
    const ApiLock api_lock;
    int rc;
    if ((rc = check_multi(ctx, n_ctx, n_pts))) return rc;
    if (!theta || !nll) return fail(NR_EINVAL, "null theta or nll array");
    for (int d = 0; d < n_ctx; ++d) {
        if (!nll[d]) return fail(NR_EINVAL, "nll[%d] is null", d);
        if ((rc = check_theta(theta[d], n_pts[d]))) return rc;
    }
    if ((rc = set_device(ctx[0]))) return rc;
    std::vector<const double*> ths(n_ctx);
    std::vector<double*> nls(n_ctx);
    hipStream_t s = ctx[0]->stream;
    for (int d = 0; d < n_ctx; ++d) {
        nr_ctx* c = ctx[d];
        if ((rc = ensure_batch(c, n_pts[d], false, 0))) return rc;
    }
    for (int d = 0; d < n_ctx; ++d) {
        nr_ctx* c = ctx[d];
        HIPCHK(hipMemcpyAsync(c->d_bth, theta[d], sizeof(double) * n_pts[d] * NR_NTHETA,
                              hipMemcpyHostToDevice, s));
        ths[d] = c->d_bth;
        nls[d] = c->d_bnll;
    }
    MultiCall mc{ctx, n_ctx, ths.data(), n_pts, nls.data(), nullptr, nullptr};
    if ((rc = run_multi(mc, s))) return rc;
    for (int d = 0; d < n_ctx; ++d)
        HIPCHK(hipMemcpyAsync(nll[d], ctx[d]->d_bnll, sizeof(double) * n_pts[d],
                              hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return 0;
}

}  // extern "C"

// ------------------------------------------------------------- surrogate
struct nr_mlp {
    int device = 0;
    int H = 256, n_out = 0, cap = 0, n_layers = 4;
    int kp[4] = {32, 0, 0, 0};  // padded input width of each layer
    int nn[4] = {0, 0, 0, 0};   // outputs of each layer
    long off[5] = {0, 0, 0, 0, 0};
    long n_params = 0;
    float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    nr::bf16* w16 = nullptr;
    // per layer the BF16 weights transposed, [kp_l][nn_l] (input-major): the
    // operand of the backward product dY W, read along its reduction index
    nr::bf16* w16t = nullptr;
    nr::bf16 *x = nullptr, *h[3] = {nullptr, nullptr, nullptr};
    float* z[3] = {nullptr, nullptr, nullptr};
    nr::bf16 *dy = nullptr, *dz[2] = {nullptr, nullptr};
    double* tile_loss = nullptr;
    double* part = nullptr;
    float* gpart = nullptr;     // K-split weight-gradient slabs
    size_t gpart_cap = 0;
    int* outside = nullptr;
    float *mean = nullptr, *stdv = nullptr;
    double lo[NR_NTHETA] = {-0.5, -0.5, -0.5, -0.5, 0.0, 0.8, 0.8};
    double hi[NR_NTHETA] = {0.5, 0.5, 0.5, 0.5, 25.0, 1.2, 1.2};
    long step = 0;
    int train_cap = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
};

namespace {

int mlp_alloc_batch(nr_mlp* q, int B, bool train) {
    int rc;
    if (B > q->cap) {
        const int cap = (B + 127) / 128 * 128;
        if ((rc = dalloc(&q->x, (size_t)cap * 32))) return rc;
        for (int l = 0; l < 3; ++l) {
            if ((rc = dalloc(&q->h[l], (size_t)cap * (q->H + 8)))) return rc;
            if ((rc = dalloc(&q->z[l], (size_t)cap * q->H))) return rc;
            HIPCHK(nr::launch_fill_ones_col(q->h[l], cap, q->H + 8, q->H, q->stream));
        }
        const int nnt = (q->n_out + 127) / 128;
        if ((rc = dalloc(&q->part, (size_t)cap * nnt))) return rc;
        if ((rc = dalloc(&q->outside, (size_t)cap))) return rc;
        q->cap = cap;
        q->train_cap = 0;
    }
    if (train && B > q->train_cap) {
        const int cap = q->cap;
        if ((rc = dalloc(&q->dy, (size_t)cap * q->n_out))) return rc;
        if ((rc = dalloc(&q->dz[0], (size_t)cap * q->H))) return rc;
        if ((rc = dalloc(&q->dz[1], (size_t)cap * q->H))) return rc;
        const int tiles = (cap / 128) * ((q->n_out + 127) / 128);
        if ((rc = dalloc(&q->tile_loss, (size_t)tiles))) return rc;
        q->train_cap = cap;
    }
    return 0;
}

// Refreshes the transposed BF16 copies of the weights of layers 1 to 3.
int mlp_transpose(nr_mlp* q, hipStream_t s) {
    for (int l = 1; l < 4; ++l)
        HIPCHK(nr::launch_transpose_bf16(q->w16 + q->off[l], q->w16t + q->off[l],
                                         q->nn[l], q->kp[l], s));
    return 0;
}

nr::MlpGemm mg(const nr::bf16* A, long sam, long sak, const nr::bf16* B,
               long sbk, long sbn, int M, int N, int K) {
    nr::MlpGemm g{};
    g.A = A; g.sam = sam; g.sak = sak;
    g.B = B; g.sbk = sbk; g.sbn = sbn;
    g.M = M; g.N = N; g.K = K;
    return g;
}

// A GEMM with a long reduction and few output tiles — the weight gradients
// G^T = dZ^T H (K = batch; 256 x 264 for a hidden layer: 6 tiles) and the
// first backward product dY W (K = the 4096 outputs) — is split along K
// over enough work-groups to fill the chip (about two per compute unit,
// chunks of at least 64), each split writing its own FP32 slab; the slabs
// are then summed in order and the GEMM's epilogue applied (FP32 store into
// C32, or SiLU' into g.C16).  No float atomics: a training step stays
// bitwise reproducible.
int mlp_split_gemm(nr_mlp* q, nr::MlpGemm g, int mode, float* C32, long ldc, hipStream_t s) {
    constexpr int kTK = 32, kTile = 128, kMinChunk = 64;
    const int tiles = ((g.M + kTile - 1) / kTile) * ((g.N + kTile - 1) / kTile);
    int n_split = std::max(1, std::min((512 + tiles - 1) / tiles, g.K / kMinChunk));
    if (n_split <= 1) {
        g.C32 = C32;
        g.ldc = ldc;
        HIPCHK(nr::launch_mlp_gemm(mode, g, s));
        return 0;
    }
    const int chunk = ((g.K + n_split - 1) / n_split + kTK - 1) / kTK * kTK;
    n_split = (g.K + chunk - 1) / chunk;
    const long ldp = g.N;                 // slab rows
    const long slab = (long)g.M * ldp;
    const size_t need = (size_t)n_split * slab;
    if (need > q->gpart_cap) {
        int rc;
        if ((rc = dalloc(&q->gpart, need))) return rc;
        q->gpart_cap = need;
    }
    nr::MlpGemm gp = g;
    gp.C32 = q->gpart;
    gp.ldc = ldp;
    gp.k_chunk = chunk;
    gp.c_split = slab;
    HIPCHK(nr::launch_mlp_gemm(nr::kMlpStore32, gp, s));
    nr::KSumArgs ks{};
    ks.part = q->gpart;
    ks.c_split = slab;
    ks.ldc = ldp;
    ks.n_split = n_split;
    ks.M = g.M;
    ks.N = g.N;
    ks.out = C32;
    ks.ldo = ldc;
    ks.dsilu = mode == nr::kMlpDSilu;
    ks.aux = g.aux;
    ks.ldaux = g.ldaux;
    ks.C16 = g.C16;
    ks.ldc16 = g.ldc16;
    HIPCHK(nr::launch_mlp_ksum(ks, s));
    return 0;
}

// Forward through the three hidden layers: Z_l = H_{l-1} W_l (bias in the
// ones column), H_l = SiLU(Z_l).
int mlp_hidden_forward(nr_mlp* q, int B, hipStream_t s) {
    const int H = q->H, ldh = H + 8;
    for (int l = 0; l < 3; ++l) {
        const nr::bf16* in = l == 0 ? q->x : q->h[l - 1];
        const int kin = l == 0 ? 32 : ldh;
        nr::MlpGemm g = mg(in, kin, 1, q->w16 + q->off[l], 1, q->kp[l], B, H, q->kp[l]);
        g.C32 = q->z[l];
        g.ldc = H;
        g.C16 = q->h[l];
        g.ldc16 = ldh;
        HIPCHK(nr::launch_mlp_gemm(nr::kMlpSilu, g, s));
    }
    return 0;
}

int mlp_input(nr_mlp* q, const double* th, int B, hipStream_t s,
              int* outside = nullptr) {
    nr::MlpInput in{};
    in.theta = th;
    in.B = B;
    for (int i = 0; i < NR_NTHETA; ++i) {
        in.lo[i] = q->lo[i];
        in.hi[i] = q->hi[i];
    }
    in.x = q->x;
    in.outside = outside ? outside : q->outside;
    HIPCHK(nr::launch_mlp_input(in, s));
    return 0;
}

}  // namespace

extern "C" {

int nr_mlp_create(int device, int hidden, int n_out, nr_mlp** out) {
    const ApiLock api_lock;
    if (!out || hidden <= 0 || hidden % 8 || n_out <= 0 || n_out % 8)
        return fail(NR_EINVAL, "hidden and n_out must be positive multiples of 8");
    *out = nullptr;
    nr_mlp* q = new (std::nothrow) nr_mlp();
    if (!q) return fail(NR_ENOMEM, "mlp allocation");
    q->device = device;
    q->H = hidden;
    q->n_out = n_out;
    q->kp[0] = 32;
    q->kp[1] = q->kp[2] = q->kp[3] = hidden + 8;
    q->nn[0] = q->nn[1] = q->nn[2] = hidden;
    q->nn[3] = n_out;
    q->off[0] = 0;
    for (int l = 0; l < 4; ++l) q->off[l + 1] = q->off[l] + (long)q->nn[l] * q->kp[l];
    q->n_params = q->off[4];
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&q->stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev_in, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&q->ev_out, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete q;
        return fail(NR_EHIP, "mlp stream: %s", hipGetErrorString(e));
    }
    int rc;
    if ((rc = dalloc(&q->w, q->n_params)) || (rc = dalloc(&q->g, q->n_params)) ||
        (rc = dalloc(&q->m, q->n_params)) || (rc = dalloc(&q->v, q->n_params)) ||
        (rc = dalloc(&q->w16, q->n_params)) || (rc = dalloc(&q->w16t, q->n_params)) ||
        (rc = dalloc(&q->mean, n_out)) ||
        (rc = dalloc(&q->stdv, n_out))) {
        delete q;
        return rc;
    }
    (void)hipMemset(q->w, 0, sizeof(float) * q->n_params);
    (void)hipMemset(q->w16, 0, sizeof(nr::bf16) * q->n_params);
    (void)hipMemset(q->w16t, 0, sizeof(nr::bf16) * q->n_params);
    (void)hipMemset(q->m, 0, sizeof(float) * q->n_params);
    (void)hipMemset(q->v, 0, sizeof(float) * q->n_params);
    *out = q;
    return 0;
}

void nr_mlp_destroy(nr_mlp* q) {
    const ApiLock api_lock;
    if (!q) return;
    (void)hipSetDevice(q->device);
    (void)hipStreamSynchronize(q->stream);
    dfree(&q->w); dfree(&q->g); dfree(&q->m); dfree(&q->v); dfree(&q->w16);
    dfree(&q->w16t);
    dfree(&q->x); dfree(&q->dy); dfree(&q->dz[0]); dfree(&q->dz[1]);
    for (int l = 0; l < 3; ++l) { dfree(&q->h[l]); dfree(&q->z[l]); }
    dfree(&q->tile_loss); dfree(&q->part); dfree(&q->outside);
    dfree(&q->mean); dfree(&q->stdv); dfree(&q->gpart);
    if (q->ev_in) (void)hipEventDestroy(q->ev_in);
    if (q->ev_out) (void)hipEventDestroy(q->ev_out);
    (void)hipStreamDestroy(q->stream);
    delete q;
}

long nr_mlp_num_params(nr_mlp* q) { return q ? q->n_params : -1; }

int nr_mlp_set_params(nr_mlp* q, const float* params, long n) {
    const ApiLock api_lock;
    if (!q || !params || n != q->n_params) return fail(NR_EINVAL, "expected %ld parameters", q ? q->n_params : -1L);
    int rc;
    if ((rc = dalloc(&q->g, q->n_params))) return rc;
    HIPCHK(hipSetDevice(q->device));
    std::vector<nr::bf16> h16(n);
    for (long i = 0; i < n; ++i) h16[i] = (nr::bf16)params[i];
    HIPCHK(hipMemcpy(q->w, params, sizeof(float) * n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(q->w16, h16.data(), sizeof(nr::bf16) * n, hipMemcpyHostToDevice));
    int rt;
    if ((rt = mlp_transpose(q, q->stream))) return rt;
    HIPCHK(hipStreamSynchronize(q->stream));
    HIPCHK(hipMemset(q->m, 0, sizeof(float) * n));
    HIPCHK(hipMemset(q->v, 0, sizeof(float) * n));
    q->step = 0;
    return 0;
}

int nr_mlp_get_params(nr_mlp* q, float* params, long n) {
    const ApiLock api_lock;
    if (!q || !params || n != q->n_params) return fail(NR_EINVAL, "expected %ld parameters", q ? q->n_params : -1L);
    HIPCHK(hipSetDevice(q->device));
    HIPCHK(hipStreamSynchronize(q->stream));
    HIPCHK(hipMemcpy(params, q->w, sizeof(float) * n, hipMemcpyDeviceToHost));
    return 0;
}

int nr_mlp_get_grads(nr_mlp* q, float* grads, long n) {
    const ApiLock api_lock;
    if (!q || !grads || n != q->n_params) return fail(NR_EINVAL, "expected %ld values", q ? q->n_params : -1L);
    HIPCHK(hipSetDevice(q->device));
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(grads, q->g, sizeof(float) * n, hipMemcpyDeviceToHost));
    return 0;
}

int nr_mlp_set_box(nr_mlp* q, const double* lo, const double* hi) {
    const ApiLock api_lock;
    if (!q || !lo || !hi) return fail(NR_EINVAL, "null argument");
    for (int i = 0; i < NR_NTHETA; ++i)
        if (!(std::isfinite(lo[i]) && std::isfinite(hi[i]) && hi[i] > lo[i]))
            return fail(NR_EINVAL, "box component %d must satisfy lo < hi", i);
    for (int i = 0; i < NR_NTHETA; ++i) {
        q->lo[i] = lo[i];
        q->hi[i] = hi[i];
    }
    return 0;
}

int nr_mlp_set_output_norm(nr_mlp* q, const float* mean, const float* stdv) {
    const ApiLock api_lock;
    if (!q || !mean || !stdv) return fail(NR_EINVAL, "null argument");
    for (int j = 0; j < q->n_out; ++j)
        if (!(std::isfinite(mean[j]) && stdv[j] > 0)) return fail(NR_EINVAL, "bad output norm at %d", j);
    HIPCHK(hipSetDevice(q->device));
    HIPCHK(hipMemcpy(q->mean, mean, sizeof(float) * q->n_out, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(q->stdv, stdv, sizeof(float) * q->n_out, hipMemcpyHostToDevice));
    return 0;
}

int nr_mlp_targets_dev(nr_mlp* q, const double* d_mu, int P, float* d_t, void* stream) {
    const ApiLock api_lock;
    if (!q || !d_mu || !d_t || P <= 0) return fail(NR_EINVAL, "bad argument");
    HIPCHK(hipSetDevice(q->device));
    nr::TargetArgs a{d_mu, P, q->n_out, q->mean, q->stdv, d_t};
    Bridge br;
    int rc;
    if ((rc = bridge_begin(br, stream, q->stream, q->ev_in, q->ev_out))) return rc;
    HIPCHK(nr::launch_targets(a, br.work));
    return bridge_end(br);
}

int nr_mlp_train_step_dev(nr_mlp* q, const double* d_theta, const float* d_t,
                          int B, float lr, double* loss, void* stream) {
    const ApiLock api_lock;
    if (!q || !d_theta || !d_t || B <= 0 || B % 8)
        return fail(NR_EINVAL, "batch must be a positive multiple of 8");
    HIPCHK(hipSetDevice(q->device));
    int rc;
    if ((rc = mlp_alloc_batch(q, B, true))) return rc;
    Bridge br;
    if ((rc = bridge_begin(br, stream, q->stream, q->ev_in, q->ev_out))) return rc;
    hipStream_t s = br.work;
    const int H = q->H, ldh = H + 8, N = q->n_out;
    if ((rc = mlp_input(q, d_theta, B, s))) return rc;
    if ((rc = mlp_hidden_forward(q, B, s))) return rc;
    // output layer with the MSE gradient in the epilogue
    nr::MlpGemm go = mg(q->h[2], ldh, 1, q->w16 + q->off[3], 1, ldh, B, N, ldh);
    go.aux = d_t;
    go.ldaux = N;
    go.C16 = q->dy;
    go.ldc16 = N;
    go.scale = 1.0f / ((float)B * (float)N);
    go.tile_loss = q->tile_loss;
    HIPCHK(nr::launch_mlp_gemm(nr::kMlpMse, go, s));
    // output layer weight gradient: G3^T = dY^T H2
    if ((rc = mlp_split_gemm(q, mg(q->dy, 1, N, q->h[2], ldh, 1, N, ldh, B),
                             nr::kMlpStore32, q->g + q->off[3], ldh, s)))
        return rc;
    // back through the hidden layers
    const nr::bf16* up = q->dy;   // gradient w.r.t. the next layer's output
    int upw = N;                  // its width
    for (int l = 2; l >= 0; --l) {
        nr::bf16* dzl = q->dz[l & 1];
        // dZ_l = (up W_{l+1}) * SiLU'(Z_l): W_{l+1}(k, n) from the transposed
        // copy [kp][nn], contiguous along the reduction index k
        nr::MlpGemm gd = mg(up, upw, 1, q->w16t + q->off[l + 1], 1, q->nn[l + 1],
                            B, H, upw);
        gd.aux = q->z[l];
        gd.ldaux = H;
        gd.C16 = dzl;
        gd.ldc16 = H;
        if ((rc = mlp_split_gemm(q, gd, nr::kMlpDSilu, nullptr, 0, s))) return rc;
        // G_l^T = dZ_l^T H_{l-1}  (H_{-1} = x)
        const nr::bf16* in = l == 0 ? q->x : q->h[l - 1];
        const int kin = l == 0 ? 32 : ldh;
        if ((rc = mlp_split_gemm(q, mg(dzl, 1, H, in, kin, 1, H, q->kp[l], B),
                                 nr::kMlpStore32, q->g + q->off[l], q->kp[l], s)))
            return rc;
        up = dzl;
        upw = H;
    }
    q->step += 1;
    nr::AdamArgs ad{};
    ad.w = q->w;
    ad.w16 = q->w16;
    ad.g = q->g;
    ad.m = q->m;
    ad.v = q->v;
    ad.n = q->n_params;
    ad.lr = lr;
    ad.b1 = 0.9f;
    ad.b2 = 0.999f;
    ad.eps = 1e-8f;
    ad.bc1 = 1.0f - powf(0.9f, (float)q->step);
    ad.bc2 = 1.0f - powf(0.999f, (float)q->step);
    HIPCHK(nr::launch_adam(ad, s));
    if ((rc = mlp_transpose(q, s))) return rc;
    if ((rc = bridge_end(br))) return rc;
    if (loss) {
        const int tiles = ((B + 127) / 128) * ((N + 127) / 128);
        std::vector<double> tl(tiles);
        HIPCHK(hipMemcpyAsync(tl.data(), q->tile_loss, sizeof(double) * tiles,
                              hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        double t = 0;
        for (double x : tl) t += x;
        *loss = t / ((double)B * N);
    }
    return 0;
}

int nr_mlp_logmu_dev(nr_mlp* q, const double* d_theta, int B, float* d_logmu,
                     void* stream) {
    const ApiLock api_lock;
    if (!q || !d_theta || !d_logmu || B <= 0 || B % 8)
        return fail(NR_EINVAL, "batch must be a positive multiple of 8");
    HIPCHK(hipSetDevice(q->device));
    int rc;
    if ((rc = mlp_alloc_batch(q, B, false))) return rc;
    Bridge br;
    if ((rc = bridge_begin(br, stream, q->stream, q->ev_in, q->ev_out))) return rc;
    hipStream_t s = br.work;
    const int ldh = q->H + 8;
    if ((rc = mlp_input(q, d_theta, B, s))) return rc;
    if ((rc = mlp_hidden_forward(q, B, s))) return rc;
    nr::MlpGemm go = mg(q->h[2], ldh, 1, q->w16 + q->off[3], 1, ldh, B, q->n_out, ldh);
    go.mean = q->mean;
    go.stdv = q->stdv;
    go.C32 = d_logmu;
    go.ldc = q->n_out;
    HIPCHK(nr::launch_mlp_gemm(nr::kMlpLogMu, go, s));
    return bridge_end(br);
}

int nr_mlp_nll_dev(nr_mlp* q, nr_ctx* c, const double* d_theta, int B,
                   double* d_nll, int* d_outside, void* stream) {
    const ApiLock api_lock;
    int rc;
    if (!q || !d_theta || !d_nll || B <= 0 || B % 8)
        return fail(NR_EINVAL, "batch must be a positive multiple of 8");
    if ((rc = check_ready(c))) return rc;
    if ((rc = check_single(c))) return rc;
    if (c->n_reco != q->n_out) return fail(NR_EINVAL, "surrogate outputs %d bins, data has %d", q->n_out, c->n_reco);
    HIPCHK(hipSetDevice(q->device));
    if ((rc = mlp_alloc_batch(q, B, false))) return rc;
    Bridge br;
    if ((rc = bridge_begin(br, stream, q->stream, q->ev_in, q->ev_out))) return rc;
    hipStream_t s = br.work;
    const int ldh = q->H + 8;
    // bin groups per point tile: about two work-groups per compute unit
    const int n_pt = (B + 127) / 128;
    const int nnt = std::max(1, std::min((q->n_out + 127) / 128, (512 + n_pt - 1) / n_pt));
    if ((rc = mlp_input(q, d_theta, B, s, d_outside))) return rc;
    nr::MlpGemm go = mg(q->h[2], ldh, 1, q->w16 + q->off[3], 1, ldh, B, q->n_out, ldh);
    go.mean = q->mean;
    go.stdv = q->stdv;
    go.nobs = c->d_n;
    go.part = q->part;
    go.n_nt = nnt;
    if (q->H == nr::kFusedHidden) {
        // the whole network in one launch, activations kept in LDS
        nr::MlpHidden hd{};
        hd.x = q->x;
        for (int l = 0; l < 3; ++l) {
            hd.w[l] = q->w16 + q->off[l];
            hd.k[l] = q->kp[l];
        }
        HIPCHK(nr::launch_mlp_nll_fused(go, hd, s));
    } else {
        if ((rc = mlp_hidden_forward(q, B, s))) return rc;
        HIPCHK(nr::launch_mlp_gemm(nr::kMlpNll, go, s));
    }
    nr::FinalArgs f{};
    f.part = q->part;
    f.theta = d_theta;
    f.n_pts = B;
    f.n_nt = nnt;
    // the partial sums are of mu - n ln mu: -2lnL = 2 (sum + sum lnGamma(n + 1))
    f.cdata = c->lgsum;
    for (int i = 0; i < NR_NTHETA; ++i) {
        f.pull_mean[i] = c->pull_mean[i];
        f.pull_sigma[i] = c->pull_sigma[i];
    }
    f.nll = d_nll;
    HIPCHK(nr::launch_finalize(f, s));
    return bridge_end(br);
}

int nr_eval_mu_batched_dev(nr_ctx* c, const double* d_theta, int n_pts,
                           double* d_mu, void* stream) {
    const ApiLock api_lock;
    int rc;
    if ((rc = check_ready(c))) return rc;
    if ((rc = check_single(c))) return rc;
    if (!d_theta || !d_mu || n_pts <= 0) return fail(NR_EINVAL, "bad argument");
    if ((rc = set_device(c))) return rc;
    if ((rc = ensure_batch(c, n_pts, false, 0))) return rc;
    Bridge br;
    if ((rc = bridge_begin(br, stream, c->stream, c->ev_in, c->ev_out))) return rc;
    nr_ctx* cs[1] = {c};
    const double* ths[1] = {d_theta};
    double* nls[1] = {c->d_bnll};
    double* mus[1] = {d_mu};
    MultiCall mc{cs, 1, ths, &n_pts, nls, nullptr, mus};
    if ((rc = run_multi(mc, br.work))) return rc;
    return bridge_end(br);
}

// ------------------------------------------------------------ templates
// Row factors F_bl = m_l I_b(T_l) / S_SM(T_l) (and m_l alone for the rows
// with S_SM = 0, whose weight is 1) in FP64 on the host, one streaming pass
// over R on the device, then the data of each bin beside its templates.
// New data alone rewrite only the data slots.  In the multi-component form
// each component's row block is folded with that component's basis and
// SM spectrum.

// Record length and gradient contractions per point of the context's form.
static int tmpl_rl(const nr_ctx* c) {
    return c->multi ? (nr::kTmplCompCols * c->n_comp + c->n_bkg + 2 + 1) / 2 * 2
                    : nr::kTmplRec;
}
static int tmpl_nacc(const nr_ctx* c) {
    return c->multi ? 10 + c->n_comp + c->n_bkg : nr::kTmplCols;
}

// Fold the row block [row0, row0 + n_t) of R with factors F [n_t][kTmplCols]
// into the record columns dst (of records rl doubles long).
static hipError_t fold_block(nr_ctx* c, const std::vector<double>& F, size_t row0,
                             const int dst[nr::kTmplCols], int rl, double* d_F,
                             double* d_part, int n_slab) {
    hipError_t e = hipMemcpy(d_F, F.data(), sizeof(double) * F.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    nr::TmplFoldArgs fa{c->d_R + row0 * c->ldr, c->ldr, c->n_t, c->n_reco, d_F, d_part};
    if ((e = nr::launch_tmpl_fold(fa, n_slab, c->stream)) != hipSuccess) return e;
    nr::TmplRecArgs ra{};
    ra.part = d_part;
    ra.n_slab = n_slab;
    ra.n_reco = c->n_reco;
    ra.rec = c->d_trec;
    ra.rl = rl;
    for (int b = 0; b < nr::kTmplCols; ++b) ra.dst[b] = dst[b];
    if ((e = nr::launch_tmpl_records(ra, c->stream)) != hipSuccess) return e;
    return hipStreamSynchronize(c->stream);  // F and part are reused
}

static int build_templates(nr_ctx* c) {
    const int n_t = c->n_t, n_reco = c->n_reco, rl = tmpl_rl(c);
    constexpr int NC = nr::kTmplCols;
    int rc;
    hipError_t e = hipSuccess;
    if (!c->tmpl_ok) {
        const int n_slab = (n_t + nr::kTmplSlabRows - 1) / nr::kTmplSlabRows;
        double *d_F = nullptr, *d_part = nullptr;
        c->tmpl_data_ok = false;
        if ((rc = dalloc(&d_F, (size_t)n_t * NC)) ||
            (rc = dalloc(&d_part, (size_t)n_slab * NC * n_reco)) ||
            (rc = dalloc(&c->d_trec, (size_t)n_reco * rl))) {
            dfree(&d_F);
            dfree(&d_part);
            return rc;
        }
        std::vector<double> F((size_t)n_t * NC);
        int dst[NC];
        if (!c->multi) {
            for (int l = 0; l < n_t; ++l) {
                const double ssm = c->ssm[l], m = c->mrow[l];
                for (int b = 0; b < NC; ++b) F[(size_t)l * NC + b] = 0.0;
                if (ssm > 0.0) {
                    for (int b = 0; b < nr::kNBasis; ++b)
                        F[(size_t)l * NC + b] = m * c->basis[(size_t)b * n_t + l] / ssm;
                } else {
                    F[(size_t)l * NC + nr::kNBasis] = m;
                }
            }
            for (int b = 0; b < NC; ++b) dst[b] = b;
            e = fold_block(c, F, 0, dst, rl, d_F, d_part, n_slab);
        } else {
            // per component: its sources' basis, its SM spectrum, its rows
            const int K = c->n_comp;
            std::vector<double> ssmc((size_t)K * n_t), mrow((size_t)K * n_t);
            e = hipMemcpy(ssmc.data(), c->d_ssmc, sizeof(double) * ssmc.size(), hipMemcpyDeviceToHost);
            if (e == hipSuccess)
                e = hipMemcpy(mrow.data(), c->d_mrow, sizeof(double) * mrow.size(), hipMemcpyDeviceToHost);
            for (int k = 0; k < K && e == hipSuccess; ++k) {
                for (int l = 0; l < n_t; ++l) {
                    double I[10] = {0}, acc[10];
                    for (int q = c->comp_off[k]; q < c->comp_off[k + 1]; ++q) {
                        source_basis(c, c->comp_src[q], l, acc);
                        for (int b = 0; b < 10; ++b) I[b] += acc[b];
                    }
                    const size_t row = (size_t)k * n_t + l;
                    double* f = &F[(size_t)l * NC];
                    for (int b = 0; b < NC; ++b) f[b] = 0.0;
                    if (ssmc[row] > 0.0) {
                        for (int b = 0; b < 10; ++b) f[b] = mrow[row] * I[b] / ssmc[row];
                    } else {
                        f[nr::kNBasis] = mrow[row];
                    }
                }
                for (int b = 0; b < NC; ++b) dst[b] = -1;
                for (int b = 0; b < 10; ++b) dst[b] = nr::kTmplCompCols * k + b;
                dst[nr::kNBasis] = nr::kTmplCompCols * k + 10;
                e = fold_block(c, F, (size_t)k * n_t, dst, rl, d_F, d_part, n_slab);
            }
        }
        dfree(&d_F);
        dfree(&d_part);
        if (e != hipSuccess) return fail(NR_EHIP, "template fold: %s", hipGetErrorString(e));
        c->tmpl_ok = true;
    }
    if (!c->tmpl_data_ok) {
        if (!c->multi) {
            nr::TmplDataArgs da{c->d_n, c->d_b, n_reco, c->d_trec};
            e = nr::launch_tmpl_data(da, c->stream);
        } else {
            nr::TmplMultiDataArgs da{c->d_n, c->d_bkg, c->d_mask, n_reco, c->n_comp,
                                     c->n_bkg, rl, c->d_trec};
            e = nr::launch_tmpl_mdata(da, c->stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return fail(NR_EHIP, "template data: %s", hipGetErrorString(e));
        c->tmpl_data_ok = true;
    }
    return 0;
}

// Reco bins per column slice: enough (point block x slice) work-groups for
// 16 waves per SIMD (8 with the gradient, whose partial sums are 22 times
// larger), at least 16 bins and at most 64 slices.  Measured on MI355X at
// 65536 points x 4096 bins: 4, 8, 16 waves per SIMD run 1.10, 1.02, 0.99 ms.
static int tmpl_split(const nr_ctx* c, int n_pts, bool grad, int* cols_per) {
    const int n_pb = (n_pts + nr::kTmplWave - 1) / nr::kTmplWave;
    const int target = grad ? 8192 : 16384;
    int ns = (target + n_pb - 1) / n_pb;
    ns = std::max(1, std::min(ns, std::min(64, (c->n_reco + 15) / 16)));
    const int cp = (c->n_reco + ns - 1) / ns;
    *cols_per = cp;
    return (c->n_reco + cp - 1) / cp;
}

static int check_tmpl_form(const nr_ctx* c) {
    if (c->multi && (c->n_comp > nr::kTmplMaxComp || c->n_bkg > nr::kTmplMaxBkg))
        return fail(NR_EINVAL, "the template form takes up to %d components and %d "
                    "background templates (have %d and %d)", nr::kTmplMaxComp,
                    nr::kTmplMaxBkg, c->n_comp, c->n_bkg);
    return 0;
}

static int ensure_tmpl(nr_ctx* c, int n_pts, bool grad) {
    int rc;
    if ((rc = check_tmpl_form(c))) return rc;
    if ((!c->tmpl_ok || !c->tmpl_data_ok) && (rc = build_templates(c))) return rc;
    int cp;
    const size_t ns = (size_t)tmpl_split(c, n_pts, grad, &cp);
    const size_t na = (size_t)tmpl_nacc(c);
    if (ns * n_pts > c->t_cap_d) {
        if ((rc = dalloc(&c->d_tdp, ns * n_pts))) return rc;
        c->t_cap_d = ns * n_pts;
    }
    if (grad && ns * na * n_pts > c->t_cap_h) {
        if ((rc = dalloc(&c->d_thp, ns * na * n_pts))) return rc;
        c->t_cap_h = ns * na * n_pts;
    }
    const size_t nred = (1 + na) * n_pts;
    if (nred > c->t_cap_r) {
        if ((rc = dalloc(&c->d_tred, nred))) return rc;
        c->t_cap_r = nred;
    }
    return 0;
}

static int enqueue_tmpl(nr_ctx* c, const double* d_th, int n_pts, double* d_nll,
                        double* d_grad, double* d_mu, hipStream_t s) {
    int cp;
    const int ns = tmpl_split(c, n_pts, d_grad != nullptr, &cp);
    double* hpart = d_grad ? c->d_thp : nullptr;
    if (!c->multi) {
        nr::TmplEvalArgs e{};
        e.rec = c->d_trec;
        e.theta = d_th;
        e.n_reco = c->n_reco;
        e.n_pts = n_pts;
        e.cols_per = cp;
        e.ph = c->ph;
        e.dpart = c->d_tdp;
        e.hpart = hpart;
        e.mu = d_mu;
        HIPCHK(nr::launch_tmpl_eval(e, ns, s));
    } else {
        nr::TmplMultiEvalArgs e{};
        e.rec = c->d_trec;
        e.theta = d_th;
        e.rl = tmpl_rl(c);
        e.K = c->n_comp;
        e.B = c->n_bkg;
        e.n_theta = c->n_theta;
        e.n_reco = c->n_reco;
        e.n_pts = n_pts;
        e.cols_per = cp;
        e.ph = c->ph;
        e.dpart = c->d_tdp;
        e.hpart = hpart;
        e.mu = d_mu;
        HIPCHK(nr::launch_tmpl_meval(e, ns, s));
    }
    nr::TmplReduceArgs r{c->d_tdp, hpart, n_pts, ns, tmpl_nacc(c), c->d_tred};
    HIPCHK(nr::launch_tmpl_reduce(r, s));
    if (!c->multi) {
        nr::TmplFinalArgs f{};
        f.red = c->d_tred;
        f.theta = d_th;
        f.n_pts = n_pts;
        f.cdata = c->cdata;
        for (int i = 0; i < NR_NTHETA; ++i) {
            f.pull_mean[i] = c->pull_mean[i];
            f.pull_sigma[i] = c->pull_sigma[i];
        }
        f.ph = c->ph;
        f.nll = d_nll;
        f.grad = d_grad;
        HIPCHK(nr::launch_tmpl_final(f, s));
    } else {
        nr::TmplMultiFinalArgs f{};
        f.red = c->d_tred;
        f.theta = d_th;
        f.n_theta = c->n_theta;
        f.K = c->n_comp;
        f.B = c->n_bkg;
        f.n_pts = n_pts;
        f.cdata = c->cdata;
        for (int i = 0; i < nr::kMaxTheta; ++i) {
            f.pull_mean[i] = c->pull_mean[i];
            f.pull_sigma[i] = c->pull_sigma[i];
        }
        f.ph = c->ph;
        f.nll = d_nll;
        f.grad = d_grad;
        HIPCHK(nr::launch_tmpl_mfinal(f, s));
    }
    return 0;
}

int nr_build_templates(nr_ctx* c) {
    const ApiLock api_lock;
    int rc;
    if ((rc = check_ready(c))) return rc;
    if ((rc = check_tmpl_form(c))) return rc;
    if ((rc = set_device(c))) return rc;
    return build_templates(c);
}

int nr_eval_nll_templates_dev(nr_ctx* c, const double* d_theta, int n_pts,
                              double* d_nll, double* d_grad, void* stream) {
    const ApiLock api_lock;
    int rc;
    if ((rc = check_ready(c))) return rc;
    if (!d_theta || !d_nll || n_pts <= 0)
        return fail(NR_EINVAL, "null device pointer or n_pts <= 0");
    if ((rc = set_device(c))) return rc;
    if ((rc = ensure_tmpl(c, n_pts, d_grad != nullptr))) return rc;
    Bridge br;
    if ((rc = bridge_begin(br, stream, c->stream, c->ev_in, c->ev_out))) return rc;
    if ((rc = enqueue_tmpl(c, d_theta, n_pts, d_nll, d_grad, nullptr, br.work))) return rc;
    return bridge_end(br);
}

static int tmpl_sync(nr_ctx* c, const double* theta, int n_pts, double* nll,
                     double* grad, double* mu) {
    int rc;
    if ((rc = check_ready(c))) return rc;
    if ((rc = check_theta(theta, n_pts, c->n_theta))) return rc;
    if ((rc = set_device(c))) return rc;
    if (!mu) {
        // theta in and -2lnL out through pinned host memory, no copies
        if ((rc = ensure_pinned(c, n_pts))) return rc;
        if ((rc = ensure_tmpl(c, n_pts, grad != nullptr))) return rc;
        std::memcpy(c->h_th, theta, sizeof(double) * n_pts * c->n_theta);
        if ((rc = enqueue_tmpl(c, c->hd_th, n_pts, c->hd_out, grad ? c->hd_grad : nullptr,
                               nullptr, c->stream)))
            return rc;
        HIPCHK(hipStreamSynchronize(c->stream));
        std::memcpy(nll, c->h_out, sizeof(double) * n_pts);
        if (grad) std::memcpy(grad, c->h_grad, sizeof(double) * n_pts * c->n_theta);
        return 0;
    }
    if ((rc = ensure_stage(c, n_pts, mu ? (size_t)n_pts * c->n_reco : 0, 0))) return rc;
    if ((rc = ensure_tmpl(c, n_pts, grad != nullptr))) return rc;
    HIPCHK(hipMemcpyAsync(c->d_th, theta, sizeof(double) * n_pts * c->n_theta,
                          hipMemcpyHostToDevice, c->stream));
    if ((rc = enqueue_tmpl(c, c->d_th, n_pts, c->d_out, grad ? c->d_grad : nullptr,
                           mu ? c->d_mu : nullptr, c->stream)))
        return rc;
    if (nll)
        HIPCHK(hipMemcpyAsync(nll, c->d_out, sizeof(double) * n_pts,
                              hipMemcpyDeviceToHost, c->stream));
    if (grad)
        HIPCHK(hipMemcpyAsync(grad, c->d_grad, sizeof(double) * n_pts * c->n_theta,
                              hipMemcpyDeviceToHost, c->stream));
    if (mu)
        HIPCHK(hipMemcpyAsync(mu, c->d_mu, sizeof(double) * n_pts * c->n_reco,
                              hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return 0;
}

int nr_eval_nll_templates(nr_ctx* c, const double* theta, int n_pts, double* nll,
                          double* grad) {
    const ApiLock api_lock;
    if (!nll) return fail(NR_EINVAL, "nll is null");
    return tmpl_sync(c, theta, n_pts, nll, grad, nullptr);
}

int nr_eval_mu_templates(nr_ctx* c, const double* theta, int n_pts, double* mu) {
    const ApiLock api_lock;
    if (!mu) return fail(NR_EINVAL, "mu is null");
    return tmpl_sync(c, theta, n_pts, nullptr, nullptr, mu);
}

}  // extern "C"
