// Branch-free FP64 exp and sincos for the bounded arguments of the sweep.
//
// Method (Cody and Waite, "Software Manual for the Elementary Functions", 1980):
// additive argument reduction x = k C + y with the constant C (pi, resp. ln 2) split
// into parts whose leading parts carry 33 (resp. 32) significant bits, so that k times
// a leading part is exact for |k| < 2^20 (resp. 2^21); then the Taylor series of the
// reduced function, truncated below the unit roundoff on the reduced range and evaluated
// by Horner's rule.  The split constants were derived from 80-digit values of pi/2 and
// ln 2 (the parts of pi are exactly twice those of pi/2).  No branches: the sign of the
// reduced sine and cosine is set with a bit operation and the exponent with ldexp, so the
// whole generation step stays one basic block and can be interleaved with MFMA work.
//
// Valid ranges (checked by the host before launch): |x| <= 1e6 for sincos_cw,
// |x| <= 708 for exp_cw.  Both are also callable on the host, where a test measures their
// errors against long-double sin, cos and exp.
#pragma once

#include <hip/hip_runtime.h>

namespace bemrat {

// sin(x), cos(x): reduce by pi to |y| <= pi/2, k = round(x / pi); then
// sin x = (-1)^k sin y and cos x = (-1)^k cos y, so the quadrant costs one sign flip of
// both results instead of a swap and two sign selections.  Absolute error 1.0-1.8 ulp of 1
// (checked on the host against long-double sin/cos for |x| <= 1e6; 0.6 ulp with a reduction
// by pi/2 and its quadrant selects), which is what the kernel sums need: every use
// multiplies them by a weight and adds them to other terms.
__host__ __device__ __forceinline__ void sincos_cw(double x, double &s, double &c) {
    constexpr double one_over_pi = 0.3183098861837907;
    constexpr double pi_1 = 3.1415926534682512;      // 33 significant bits (2 x the pi/2 parts)
    constexpr double pi_2 = 1.2154201012607932e-10;  // 33 significant bits
    constexpr double pi_3 = 4.044532497591901e-21;   // remainder
    const double kd = rint(x * one_over_pi);
    double y = fma(-kd, pi_1, x);
    y = fma(-kd, pi_2, y);
    y = fma(-kd, pi_3, y);
    const double y2 = y * y;
    // sin y = y + y^3 P(y^2), cos y = 1 + y^2 Q(y^2): the Taylor series (to degree 31 and 32)
    // economised on |y| <= pi/2 by Chebyshev polynomials down to degree 17 and 16 (Lanczos'
    // economisation; coefficients computed in exact rational arithmetic, error bounds
    // 2e-19 and 4e-18, leading coefficients 1 - 2e-18 and 1 - 4e-18 rounded to 1)
    double ps = 2.7166581648246254e-15;
    ps = fma(ps, y2, -7.642510917660842e-13);
    ps = fma(ps, y2, 1.6058918611181144e-10);
    ps = fma(ps, y2, -2.505210638033204e-08);
    ps = fma(ps, y2, 2.7557319204570754e-06);
    ps = fma(ps, y2, -0.00019841269841159377);
    ps = fma(ps, y2, 0.008333333333332993);
    ps = fma(ps, y2, -0.16666666666666663);
    const double sy = fma(y * y2, ps, y);
    double pc = 4.608992189914223e-14;
    pc = fma(pc, y2, -1.1462903400770852e-11);
    pc = fma(pc, y2, 2.087656190004232e-09);
    pc = fma(pc, y2, -2.755731639228085e-07);
    pc = fma(pc, y2, 2.4801587277429444e-05);
    pc = fma(pc, y2, -0.0013888888888773081);
    pc = fma(pc, y2, 0.04166666666666388);
    pc = fma(pc, y2, -0.4999999999999997);
    const double cy = fma(y2, pc, 1.0);
    // (-1)^k: flip the sign bits when k is odd
    const unsigned long long flip = (unsigned long long)((int)kd & 1) << 63;
    s = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, sy) ^ flip);
    c = __builtin_bit_cast(double, __builtin_bit_cast(unsigned long long, cy) ^ flip);
}

// Sine and cosine for entries that are rounded to BF16 or FP16 afterwards: the argument is
// reduced in FP64 to t = x/(2 pi) - rint(x/(2 pi)) in [-1/2, 1/2] revolutions (the product's
// rounding, |x| 2^-53/(2 pi), is below 2^-33 revolutions for the admissible |x| <= 1e6) and
// evaluated by the FP32 hardware sine and cosine, which take revolutions.  Absolute error
// 1.2e-7 (measured on the device over [-1/2, 1/2] against FP64), against relative roundings
// of 2^-9 (BF16) and 2^-12 (FP16) of the entries.
__device__ __forceinline__ void sincos_lowp(double x, double &s, double &c) {
    const double t = x * 0.15915494309189535;
    const float f = (float)(t - rint(t));
    s = (double)__builtin_amdgcn_sinf(f);
    c = (double)__builtin_amdgcn_cosf(f);
}

// sincos_cw, or sincos_lowp for entries bound to a 16-bit type.
template <bool LOWP>
__device__ __forceinline__ void sincos_gen(double x, double &s, double &c) {
    if constexpr (LOWP)
        sincos_lowp(x, s, c);
    else
        sincos_cw(x, s, c);
}

// exp(x): reduce by ln 2 to |y| <= ln2/2, exp(x) = 2^k exp(y).
__host__ __device__ __forceinline__ double exp_cw(double x) {
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

// E(w) = (e^w - 1)/w for complex w (self and near-field integrals): Taylor series for
// |w| < 1/4, otherwise through expm1 so that no cancellation occurs at small |w|.
__device__ inline double2 exprel(double wr, double wi) {
    if (wr * wr + wi * wi < 0.0625) {
        // Taylor series sum_k w^k/(k+1)!, k <= 11: remainder < 0.25^12/13! / (1 - 0.25/14)
        // = 9.8e-18, below a tenth of the unit roundoff relative to |E(w)| >= 0.88
        const double c[12] = {1.0,
                              1.0 / 2.0,
                              1.0 / 6.0,
                              1.0 / 24.0,
                              1.0 / 120.0,
                              1.0 / 720.0,
                              1.0 / 5040.0,
                              1.0 / 40320.0,
                              1.0 / 362880.0,
                              1.0 / 3628800.0,
                              1.0 / 39916800.0,
                              1.0 / 479001600.0};
        double sr = c[11], si = 0.0;
        for (int k = 10; k >= 0; --k) {
            const double tr = sr * wr - si * wi + c[k];
            si = sr * wi + si * wr;
            sr = tr;
        }
        return make_double2(sr, si);
    }
    // e^w - 1 = (expm1(wr) cos wi - 2 sin^2(wi/2)) + i e^wr sin wi
    double s, co;
    sincos(wi, &s, &co);
    const double sh = sin(0.5 * wi);
    const double nr = expm1(wr) * co - 2.0 * sh * sh;
    const double ni = exp(wr) * s;
    const double den = wr * wr + wi * wi;
    return make_double2((nr * wr + ni * wi) / den, (ni * wr - nr * wi) / den);
}

}  // namespace bemrat
