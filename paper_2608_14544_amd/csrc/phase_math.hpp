// sin and cos of a phase angle in binary64 without table-driven argument
// reduction (which would put a private array in scratch memory).
//
// Reduction: x = k pi/2 + r with k = rint(2x/pi) and pi/2 split into two
// doubles (Cody-Waite), each product folded with one fma; for the phase
// magnitudes met here (|x| < 1e9) the reduced argument is accurate to a
// few units in the last place.  On |r| <= pi/4 the Taylor series of sin
// (through r^17/17!) and cos (through r^18/18!) truncate below 1e-19.
#pragma once

#include <hip/hip_runtime.h>

namespace qcl {

__device__ __forceinline__ void sincos_phase(double x, double &s, double &c)
{
    constexpr double two_over_pi = 0.6366197723675814;
    constexpr double half_pi_hi = 0x1.921fb54442d18p+0;   // pi/2 rounded to binary64
    constexpr double half_pi_lo = 0x1.1a62633145c07p-54;  // pi/2 - half_pi_hi, rounded
    const double k = rint(x * two_over_pi);
    double r = fma(-k, half_pi_hi, x);
    r = fma(-k, half_pi_lo, r);
    const double r2 = r * r;
    // sin r = r (1 - r^2/3! + r^4/5! - ... + r^16/17!)
    double ps = 1.0 / 355687428096000.0;       // 1/17!
    ps = fma(ps, r2, -1.0 / 1307674368000.0);  // 1/15!
    ps = fma(ps, r2, 1.0 / 6227020800.0);      // 1/13!
    ps = fma(ps, r2, -1.0 / 39916800.0);       // 1/11!
    ps = fma(ps, r2, 1.0 / 362880.0);          // 1/9!
    ps = fma(ps, r2, -1.0 / 5040.0);           // 1/7!
    ps = fma(ps, r2, 1.0 / 120.0);             // 1/5!
    ps = fma(ps, r2, -1.0 / 6.0);              // 1/3!
    const double sr = fma(ps * r2, r, r);
    // cos r = 1 - r^2/2! + r^4/4! - ... + r^18/18!
    double pc = 1.0 / 6402373705728000.0;      // 1/18!
    pc = fma(pc, r2, -1.0 / 20922789888000.0); // 1/16!
    pc = fma(pc, r2, 1.0 / 87178291200.0);     // 1/14!
    pc = fma(pc, r2, -1.0 / 479001600.0);      // 1/12!
    pc = fma(pc, r2, 1.0 / 3628800.0);         // 1/10!
    pc = fma(pc, r2, -1.0 / 40320.0);          // 1/8!
    pc = fma(pc, r2, 1.0 / 720.0);             // 1/6!
    pc = fma(pc, r2, -1.0 / 24.0);             // 1/4!
    pc = fma(pc, r2, 0.5);                     // sign folded below
    const double cr = fma(-pc, r2, 1.0);
    // quadrant: x = k pi/2 + r
    const long long q = (long long)k & 3;
    const double s0 = (q & 1) ? cr : sr;
    const double c0 = (q & 1) ? sr : cr;
    s = (q & 2) ? -s0 : s0;
    c = ((q + 1) & 2) ? -c0 : c0;
}

}  // namespace qcl
