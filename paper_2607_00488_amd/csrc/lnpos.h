// Natural logarithm of a positive double in plain FP64 arithmetic, for the
// per-bin Poisson terms of the template form.
//
// x = m 2^e with m brought into [sqrt(1/2), sqrt(2)); then
//   ln m = 2 atanh(s) = 2 (s + s^3/3 + s^5/5 + ...),  s = (m - 1) / (m + 1),
// the classical series for the logarithm (|s| <= 0.1716, so nine terms past
// the first leave a relative truncation of 2e-17), and
//   ln x = e ln 2 + ln m
// with ln 2 split into a 24-bit head (e * head is exact) and a tail.  The
// absolute error stays within a few 1e-16 times max(1, |ln x|), checked on
// the host against the C library over log-uniform arguments; that is far
// inside what a -2lnL budget of 1e-3 over thousands of bins needs, at about
// a third of the operations of a correctly rounded logarithm.
//
// Every multiply-add is fused.  The quotient s = (m - 1) / (m + 1) has a
// denominator in [1.70, 2.42], so it needs none of the scaling steps of a
// general IEEE division: a reciprocal estimate (the hardware one on the
// device, 1 / d on the host), two Newton steps and one residual correction
// give s to within an ulp or so.  Two Newton steps take an estimate
// with relative error up to 2^-13 to full precision; the host test
// also runs with an estimate that far off.
#pragma once

#include <cmath>

#ifndef NR_LNPOS_SEED
#if defined(__HIP_DEVICE_COMPILE__)
#define NR_LNPOS_SEED(d) __builtin_amdgcn_rcp(d)
#else
#define NR_LNPOS_SEED(d) (1.0 / (d))
#endif
#endif

namespace nr {

// a * b + c as one three-operand FP64 FMA on the device: the compiler's
// two-operand form (the addend tied to the destination) copies a constant
// addend into the destination before every step of a polynomial.
__host__ __device__ inline double fma3(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
#else
    return fma(a, b, c);
#endif
}

__host__ __device__ inline double ln_pos(double x) {
    if (!(x < INFINITY)) return x;
    int e;
    double m = frexp(x, &e);  // x = m 2^e, m in [0.5, 1); exact
    if (m < 0.70710678118654752) {
        m *= 2.0;
        --e;
    }
    const double u = m - 1.0;  // exact here
    const double d = m + 1.0;
    double y = NR_LNPOS_SEED(d);
    y = fma(y, fma(-d, y, 1.0), y);
    y = fma(y, fma(-d, y, 1.0), y);
    const double s0 = u * y;
    const double s = fma(fma(-d, s0, u), y, s0);
    const double z = s * s;
    double p = 1.0 / 19.0;
    p = fma3(p, z, 1.0 / 17.0);
    p = fma3(p, z, 1.0 / 15.0);
    p = fma3(p, z, 1.0 / 13.0);
    p = fma3(p, z, 1.0 / 11.0);
    p = fma3(p, z, 1.0 / 9.0);
    p = fma3(p, z, 1.0 / 7.0);
    p = fma3(p, z, 1.0 / 5.0);
    p = fma3(p, z, 1.0 / 3.0);
    const double t = 2.0 * s;
    const double lnm = fma(t * z, p, t);
    const double ln2_head = 0.6931471824645996;     // ln 2 rounded to 24 bits
    const double ln2_tail = -1.904654299957768e-09; // ln 2 - head
    const double de = (double)e;
    return fma(de, ln2_head, fma(de, ln2_tail, lnm));
}

}  // namespace nr
