// lm_math.h -- device math for the pair kernels (gfx950).
//
// The pair kernels need exp of a non-positive argument and 1/sqrt of a positive one, in
// double and in single precision.  There is no double-precision exp instruction; the one
// here follows Cody & Waite's argument reduction (W. J. Cody and W. Waite, "Software
// Manual for the Elementary Functions", 1980): x = k ln2 + r with integer k and
// |r| <= ln2/2, then exp(x) = 2^k P(r) with P a degree-11 polynomial.  The constants were
// derived for this library by gen_exp_coeffs.py (Chebyshev interpolation of exp on
// [-ln2/2, ln2/2] at 60 digits, rounded to double): the rounded polynomial is within
// 1.7e-17 of exp on that interval, so the result is within a few units in the last place.
//
// The reciprocal square root starts from the hardware estimate v_rsq_f64 (relative error
// 5.2e-8 = 2^-24.2, measured on gfx950 over 2^20 arguments in [2^-20, 2^20]) and applies one
// third-order correction y <- y (1 + t/2 + 3t^2/8), t = 1 - s y^2 (the Taylor series of
// (1 - t)^(-1/2)), which leaves about 2.5 (5.2e-8)^3 ~ 4e-22 before rounding.
#pragma once

#include <hip/hip_runtime.h>

namespace lm {

constexpr double kLog2e = 1.4426950408889634;       // 1/ln 2
constexpr double kLn2Hi = 0.6931471805599453;       // ln 2 rounded to double
constexpr double kLn2Lo = 2.3190468138462996e-17;   // ln 2 - kLn2Hi

// exp(x) for x <= 0.  Arguments below -1000 return 0 (exp underflows far earlier); the
// clamp also keeps the reduction finite for huge |x|.
__device__ __forceinline__ double exp_nonpos(double x)
{
    x = __builtin_fmax(x, -1000.0);
    const double k = __builtin_rint(x * kLog2e);
    double r = __builtin_fma(k, -kLn2Hi, x);
    r = __builtin_fma(k, -kLn2Lo, r);
    double p = 0x1.af631d0059becp-26;
    p = __builtin_fma(p, r, 0x1.28b4057f44145p-22);
    p = __builtin_fma(p, r, 0x1.71ddf5749d126p-19);
    p = __builtin_fma(p, r, 0x1.a01991ac8730ap-16);
    p = __builtin_fma(p, r, 0x1.a01a01b14378fp-13);
    p = __builtin_fma(p, r, 0x1.6c16c187fbe02p-10);
    p = __builtin_fma(p, r, 0x1.111111110f225p-7);
    p = __builtin_fma(p, r, 0x1.555555554f0cfp-5);
    p = __builtin_fma(p, r, 0x1.555555555555ap-3);
    p = __builtin_fma(p, r, 0x1.0000000000011p-1);
    p = __builtin_fma(p, r, 1.0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_ldexp(p, (int)k);
}

// 1/sqrt(s) for s > 0 (callers clamp s away from zero).
__device__ __forceinline__ double rsqrt_pos(double s)
{
    const double y = __builtin_amdgcn_rsq(s);
    const double e = s * y;
    const double t = __builtin_fma(-e, y, 1.0);
    const double c = __builtin_fma(t, 0.375, 0.5);
    return __builtin_fma(y * t, c, y);
}

// Single precision: the hardware 2^x and 1/sqrt(x) (about one ulp each).
__device__ __forceinline__ float exp2_f32(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rsqrt_f32(float s) { return __builtin_amdgcn_rsqf(s); }

}  // namespace lm
