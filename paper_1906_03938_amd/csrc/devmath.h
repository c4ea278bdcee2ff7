// Branch-free FP64 exp and sincos for the bounded arguments of the sweep.
//
// Method (Cody and Waite, "Software Manual for the Elementary Functions", 1980):
// additive argument reduction x = k C + y with the constant C (pi/2, resp. ln 2) split
// into parts whose leading parts carry 33 (resp. 32) significant bits, so that k times
// a leading part is exact for |k| < 2^20 (resp. 2^21); then the Taylor series of the
// reduced function, truncated below 2^-60 relative on the reduced range and evaluated
// by Horner's rule.  The split constants were derived from 80-digit values of pi/2 and
// ln 2.  No branches: quadrant and exponent handling use selects, so the whole
// generation step stays one basic block and can be interleaved with MFMA work.
//
// Valid ranges (checked by the host before launch): |x| <= 1e6 for sincos_cw,
// |x| <= 708 for exp_cw.
#pragma once

#include <hip/hip_runtime.h>

namespace bemrat {

// sin(x), cos(x): reduce by pi/2 to |y| <= pi/4, quadrant q = k mod 4.
__device__ __forceinline__ void sincos_cw(double x, double &s, double &c) {
    constexpr double two_over_pi = 0.6366197723675814;
    constexpr double pio2_1 = 1.5707963267341256;      // 33 significant bits
    constexpr double pio2_2 = 6.077100506303966e-11;   // 33 significant bits
    constexpr double pio2_3 = 2.0222662487959506e-21;  // remainder
    const double kd = rint(x * two_over_pi);
    double y = fma(-kd, pio2_1, x);
    y = fma(-kd, pio2_2, y);
    y = fma(-kd, pio2_3, y);
    const double y2 = y * y;
    // sin y = y sum_{j<=8} (-1)^j y^{2j}/(2j+1)!   (remainder (pi/4)^19/19! < 1e-19)
    double ps = -1.0 / 355687428096000.0;       // -1/17!
    ps = fma(ps, y2, 1.0 / 1307674368000.0);    //  1/15!
    ps = fma(ps, y2, -1.0 / 6227020800.0);      // -1/13!
    ps = fma(ps, y2, 1.0 / 39916800.0);         //  1/11!
    ps = fma(ps, y2, -1.0 / 362880.0);          // -1/9!
    ps = fma(ps, y2, 1.0 / 5040.0);             //  1/7!
    ps = fma(ps, y2, -1.0 / 120.0);             // -1/5!
    ps = fma(ps, y2, 1.0 / 6.0);                //  1/3!  (sign applied below)
    const double sy = fma(-y * y2, ps, y);
    // cos y = sum_{j<=9} (-1)^j y^{2j}/(2j)!   (remainder (pi/4)^20/20! < 1e-20)
    double pc = 1.0 / 6402373705728000.0;       //  1/18!
    pc = fma(pc, y2, -1.0 / 20922789888000.0);  // -1/16!
    pc = fma(pc, y2, 1.0 / 87178291200.0);      //  1/14!
    pc = fma(pc, y2, -1.0 / 479001600.0);       // -1/12!
    pc = fma(pc, y2, 1.0 / 3628800.0);          //  1/10!
    pc = fma(pc, y2, -1.0 / 40320.0);           // -1/8!
    pc = fma(pc, y2, 1.0 / 720.0);              //  1/6!
    pc = fma(pc, y2, -1.0 / 24.0);              // -1/4!
    pc = fma(pc, y2, 0.5);                      //  1/2!  (sign applied below)
    const double cy = fma(-y2, pc, 1.0);
    const int q = (int)kd;
    const double a = (q & 1) ? cy : sy;
    const double b = (q & 1) ? sy : cy;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

// exp(x): reduce by ln 2 to |y| <= ln2/2, exp(x) = 2^k exp(y).
__device__ __forceinline__ double exp_cw(double x) {
    constexpr double log2e = 1.4426950408889634;
    constexpr double ln2_hi = 0.6931471803691238;      // 32 significant bits
    constexpr double ln2_lo = 1.9082149292705877e-10;  // remainder
    const double kd = rint(x * log2e);
    double y = fma(-kd, ln2_hi, x);
    y = fma(-kd, ln2_lo, y);
    // sum_{j<=13} y^j/j!   (remainder (ln2/2)^14/14! < 5e-18)
    double p = 1.0 / 6227020800.0;  // 1/13!
    p = fma(p, y, 1.0 / 479001600.0);
    p = fma(p, y, 1.0 / 39916800.0);
    p = fma(p, y, 1.0 / 3628800.0);
    p = fma(p, y, 1.0 / 362880.0);
    p = fma(p, y, 1.0 / 40320.0);
    p = fma(p, y, 1.0 / 5040.0);
    p = fma(p, y, 1.0 / 720.0);
    p = fma(p, y, 1.0 / 120.0);
    p = fma(p, y, 1.0 / 24.0);
    p = fma(p, y, 1.0 / 6.0);
    p = fma(p, y, 0.5);
    p = fma(p, y, 1.0);
    p = fma(p, y, 1.0);
    return ldexp(p, (int)kd);
}

}  // namespace bemrat
