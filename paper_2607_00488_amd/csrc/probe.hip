// Diagnostic: the FP64 matrix-core rate this device sustains, measured by a
// stream of independent v_mfma_f64_16x16x4_f64 on register operands (no
// memory traffic inside the timed loop).  The batched GEMM's TFLOP/s are
// read against it beside the data-sheet peak.
#include "../../include/nureweight.h"

#include <hip/hip_runtime.h>

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kChains = 8;  // independent accumulators per wave

__global__ __launch_bounds__(256) void k_probe_mfma_f64(double* out, int iters) {
    v4d acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = (v4d){0.0, 0.0, 0.0, 0.0};
    const double a = threadIdx.x * 1e-3, b = 1.0 + blockIdx.x * 1e-6;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c)
            acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[(size_t)blockIdx.x * 256 + threadIdx.x] = s;  // keeps the chains live
}

}  // namespace

extern "C" int nr_probe_mfma_f64(int device, int blocks, int iters, double* tflops) {
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
            *tflops = (double)blocks * 4 * iters * kChains * 2048.0 / (ms * 1e-3) / 1e12;
            rc = NR_OK;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(d);
    return rc;
}
