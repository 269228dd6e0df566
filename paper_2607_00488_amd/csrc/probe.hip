// Diagnostics: what this device sustains, measured rather than taken from
// the data sheet.  The FP64 matrix-core rate from a stream of independent
// v_mfma_f64_16x16x4_f64 on register operands (no memory traffic inside the
// timed loop), which the batched GEMM's TFLOP/s are read against; and the
// read rate of a plain streaming sum, over a buffer much larger than the
// caches (HBM) or, with ordinary loads and alternating directions, over a
// buffer the size of the response the single-point fold walks the same way
// (HBM plus what the caches keep between passes); the fold's bytes per
// second are read against both.
#include "../../include/nureweight.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace nr {
std::recursive_mutex& api_mutex();  // the library's entry-point lock
}

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kChains = 8;   // independent accumulators per wave
constexpr int kRounds = 16;  // rounds over the chains per loop trip

__global__ __launch_bounds__(256) void k_probe_mfma_f64(double* out, int iters) {
    v4d acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = (v4d){0.0, 0.0, 0.0, 0.0};
    const double a = threadIdx.x * 1e-3, b = 1.0 + blockIdx.x * 1e-6;
    // kRounds rounds per trip: the compiler moves the loop-carried
    // accumulators between register files once per trip, which a short
    // body would make the bottleneck instead of the matrix cores
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < kRounds; ++r)
#pragma unroll
            for (int c = 0; c < kChains; ++c)
                acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;  // keeps the chains live
}

// Grid-stride sum of a buffer with 16-byte loads, eight in flight per lane,
// 32 work-groups per compute unit.  Non-temporal loads are the fastest way
// to stream a buffer much larger than the caches (non-temporal / ordinary
// loads, 4 / 8 in flight and 4..32 work-groups per CU measured on MI355X:
// 6.3 TB/s over 2 GiB); ordinary loads allocate in L2 and the Infinity
// Cache, which serve part of a buffer near their size on the next pass.
// With `rev` the pass walks the buffer last to first.  The sum decides a
// store that never happens for the zero-filled buffer, which keeps every
// load live.
constexpr int kReadUnroll = 8;
typedef float f4v __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ inline f4v ld4(const f4v* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

template <bool NT>
__global__ __launch_bounds__(256) void k_probe_read(const f4v* __restrict__ p, size_t n4,
                                                    int rev, float* out) {
    const size_t stride = (size_t)gridDim.x * 256;
    size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    float s = 0.0f;
    for (; i + (kReadUnroll - 1) * stride < n4; i += kReadUnroll * stride) {
        f4v v[kReadUnroll];
#pragma unroll
        for (int q = 0; q < kReadUnroll; ++q) {
            const size_t k = i + q * stride;
            v[q] = ld4<NT>(p + (rev ? n4 - 1 - k : k));
        }
#pragma unroll
        for (int q = 0; q < kReadUnroll; ++q) s += v[q].x + v[q].y + v[q].z + v[q].w;
    }
    for (; i < n4; i += stride) {
        const f4v v = ld4<NT>(p + (rev ? n4 - 1 - i : i));
        s += v.x + v.y + v.z + v.w;
    }
    if (s == 1234.5f) out[0] = s;
}

void launch_read(bool nt, int grid, const f4v* p, size_t n4, int rev, float* out) {
    if (nt) hipLaunchKernelGGL(k_probe_read<true>, dim3(grid), dim3(256), 0, nullptr, p, n4, rev, out);
    else hipLaunchKernelGGL(k_probe_read<false>, dim3(grid), dim3(256), 0, nullptr, p, n4, rev, out);
}

// Read rate over `reps` passes after two untimed ones; pass r walks
// backwards when `alternate` and r is odd.
int read_rate(int device, long long bytes, int reps, bool nt, bool alternate, double* gbs) {
    if (hipSetDevice(device) != hipSuccess) return NR_EHIP;
    float* d = nullptr;
    float* o = nullptr;
    if (hipMalloc((void**)&d, (size_t)bytes) != hipSuccess) return NR_ENOMEM;
    if (hipMalloc((void**)&o, sizeof(float)) != hipSuccess) {
        (void)hipFree(d);
        return NR_ENOMEM;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = NR_EHIP;
    float ms = 0.0f;
    const size_t n4 = (size_t)bytes / 16;
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    const int grid = (cus > 0 ? cus : 256) * 32;
    const f4v* p = reinterpret_cast<const f4v*>(d);
    if (hipMemset(d, 0, (size_t)bytes) == hipSuccess && hipEventCreate(&e0) == hipSuccess &&
        hipEventCreate(&e1) == hipSuccess) {
        for (int r = 0; r < 2; ++r) launch_read(nt, grid, p, n4, alternate ? r & 1 : 0, o);
        (void)hipEventRecord(e0, nullptr);
        for (int r = 0; r < reps; ++r) launch_read(nt, grid, p, n4, alternate ? r & 1 : 0, o);
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) == hipSuccess && hipGetLastError() == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f) {
            *gbs = (double)bytes * reps / (ms * 1e-3) / 1e9;
            rc = NR_OK;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(o);
    (void)hipFree(d);
    return rc;
}

}  // namespace

extern "C" int nr_probe_hbm_read(int device, long long bytes, int reps, double* gbs) {
    const std::lock_guard<std::recursive_mutex> lk(nr::api_mutex());
    if (!gbs || bytes < (1 << 20) || bytes > (1LL << 36) || (bytes & 15) || reps <= 0)
        return NR_EINVAL;
    return read_rate(device, bytes, reps, true, false, gbs);
}

extern "C" int nr_probe_read(int device, long long bytes, int reps, int flags, double* gbs) {
    const std::lock_guard<std::recursive_mutex> lk(nr::api_mutex());
    if (!gbs || bytes < (1 << 20) || bytes > (1LL << 36) || (bytes & 15) || reps <= 0 ||
        (flags & ~(NR_PROBE_CACHED | NR_PROBE_ALTERNATE)))
        return NR_EINVAL;
    return read_rate(device, bytes, reps, !(flags & NR_PROBE_CACHED),
                     (flags & NR_PROBE_ALTERNATE) != 0, gbs);
}

extern "C" int nr_probe_mfma_f64(int device, int blocks, int iters, double* tflops) {
    const std::lock_guard<std::recursive_mutex> lk(nr::api_mutex());
    if (!tflops || blocks <= 0 || blocks > (1 << 16) || iters <= 0) return NR_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return NR_EHIP;
    double* d = nullptr;
    if (hipMalloc((void**)&d, sizeof(double) * 256 * (size_t)blocks) != hipSuccess) return NR_ENOMEM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = NR_EHIP;
    float ms = 0.0f;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
        hipLaunchKernelGGL(k_probe_mfma_f64, dim3(blocks), dim3(256), 0, nullptr, d, 16);
        (void)hipEventRecord(e0, nullptr);
        hipLaunchKernelGGL(k_probe_mfma_f64, dim3(blocks), dim3(256), 0, nullptr, d, iters);
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) == hipSuccess && hipGetLastError() == hipSuccess &&
            hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f) {
            // 4 waves per work-group, 16 x 16 x 4 multiply-adds per instruction
            *tflops = (double)blocks * 4 * iters * kRounds * kChains * 2048.0 / (ms * 1e-3) / 1e12;
            rc = NR_OK;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(d);
    return rc;
}
