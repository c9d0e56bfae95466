// sin and cos of a phase angle without table-driven argument reduction
// (which would put a private array in scratch memory).
//
// Reduction (binary64 in both variants): x = k pi/2 + r with
// k = rint(2x/pi) and pi/2 split into two doubles (Cody-Waite), each
// product folded with one fma; for the phase magnitudes met here
// (|x| < 1e9) r is accurate to a few units in the last place.
//
// sincos_phase:    Taylor series on |r| <= pi/4 in binary64, sin through
//                  r^17/17!, cos through r^18/18! (truncation < 1e-19).
//                  The coefficients are read from a device array (a
//                  writable global with external linkage, so the compiler
//                  cannot fold them into literals and hoist those into
//                  vector registers for the whole step loop); they arrive
//                  by scalar loads where they are used.
// sincos_phase32:  the same reduction, then binary32 Taylor series (sin
//                  through r^11/11!, cos through r^12/12!, truncation
//                  below 2e-9) for the binary32 path, whose walker weights
//                  carry binary32 phase factors.
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#endif

namespace qcl {

// 1/3!, 1/5!, ..., 1/17! with alternating signs, then 1/2!, 1/4!, ..., 1/18!
// Defined in every translation unit that includes this header: each unit's
// device code object holds its own copy (device code is not relocatable
// across units), and the host-side shadows are local symbols.
__device__ double kTaylorSinCos[18] = {
    -1.0 / 6.0, 1.0 / 120.0, -1.0 / 5040.0, 1.0 / 362880.0, -1.0 / 39916800.0, 1.0 / 6227020800.0,
    -1.0 / 1307674368000.0, 1.0 / 355687428096000.0, 0.0,
    0.5, -1.0 / 24.0, 1.0 / 720.0, -1.0 / 40320.0, 1.0 / 3628800.0, -1.0 / 479001600.0,
    1.0 / 87178291200.0, -1.0 / 20922789888000.0, 1.0 / 6402373705728000.0};

__device__ __forceinline__ double reduce_half_pi(double x, int &quadrant)
{
    constexpr double two_over_pi = 0.6366197723675814;
    constexpr double half_pi_hi = 0x1.921fb54442d18p+0;   // pi/2 rounded to binary64
    constexpr double half_pi_lo = 0x1.1a62633145c07p-54;  // pi/2 - half_pi_hi, rounded
    const double k = rint(x * two_over_pi);
    double r = fma(-k, half_pi_hi, x);
    r = fma(-k, half_pi_lo, r);
    // k mod 4 from the low word of k + 1.5 * 2^52 (exact for |k| < 2^51,
    // whose integer bits then fill the low mantissa bits)
    const double kb = k + 0x1.8p52;
    quadrant = (int)((uint32_t)__double_as_longlong(kb) & 3u);
    return r;
}

template <typename T>
__device__ __forceinline__ void apply_quadrant(int q, T sr, T cr, T &s, T &c)
{
    const T s0 = (q & 1) ? cr : sr;
    const T c0 = (q & 1) ? sr : cr;
    s = (q & 2) ? -s0 : s0;
    c = ((q + 1) & 2) ? -c0 : c0;
}

__device__ __forceinline__ void sincos_phase(double x, double &s, double &c)
{
    const double *__restrict__ t = kTaylorSinCos;
    int q;
    const double r = reduce_half_pi(x, q);
    const double r2 = r * r;
    double ps = t[7];
#pragma unroll
    for (int i = 6; i >= 0; --i)
        ps = fma(ps, r2, t[i]);
    const double sr = fma(ps * r2, r, r);  // r + r^3 (-1/3! + ...)
    double pc = t[17];
#pragma unroll
    for (int i = 16; i >= 9; --i)
        pc = fma(pc, r2, t[i]);
    const double cr = fma(-pc, r2, 1.0);  // 1 - r^2 (1/2! - ...)
    apply_quadrant<double>(q, sr, cr, s, c);
}

__device__ __forceinline__ void sincos_phase32(double x, float &s, float &c)
{
    int q;
    const float r = (float)reduce_half_pi(x, q);
    const float r2 = r * r;
    float ps = -1.0f / 39916800.0f;       // -1/11!
    ps = fmaf(ps, r2, 1.0f / 362880.0f);  // 1/9!
    ps = fmaf(ps, r2, -1.0f / 5040.0f);   // -1/7!
    ps = fmaf(ps, r2, 1.0f / 120.0f);     // 1/5!
    ps = fmaf(ps, r2, -1.0f / 6.0f);      // -1/3!
    const float sr = fmaf(ps * r2, r, r);
    float pc = 1.0f / 479001600.0f;       // 1/12!
    pc = fmaf(pc, r2, -1.0f / 3628800.0f);  // -1/10!
    pc = fmaf(pc, r2, 1.0f / 40320.0f);   // 1/8!
    pc = fmaf(pc, r2, -1.0f / 720.0f);    // -1/6!
    pc = fmaf(pc, r2, 1.0f / 24.0f);      // 1/4!
    pc = fmaf(pc, r2, -0.5f);             // -1/2!
    const float cr = fmaf(pc, r2, 1.0f);
    apply_quadrant<float>(q, sr, cr, s, c);
}

}  // namespace qcl
