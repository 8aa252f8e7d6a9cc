// lm_math.h -- device math for the pair kernels (gfx950).
//
// The pair kernels need exp of a non-positive argument and 1/sqrt of a positive one, in
// double and in single precision.  There is no double-precision exp instruction; the one
// here follows Cody & Waite's argument reduction (W. J. Cody and W. Waite, "Software
// Manual for the Elementary Functions", 1980): x = k ln2 + r with integer k and
// |r| <= ln2/2, then exp(x) = 2^k P(r) with P a degree-10 polynomial.  The constants were
// derived for this library by gen_exp_coeffs.py (Chebyshev interpolation of exp on
// [-ln2/2, ln2/2] at 60 digits, rounded to double): the rounded polynomial is within
// 3.3e-16 of exp on that interval (degree 11 would give 1.7e-17 for one more FMA per pair;
// the difference is far below the parity bar and the sums' own rounding).
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
// clamp also keeps the reduction finite for huge |x|.  k = round(x / ln2) comes from adding
// and subtracting 1.5 * 2^52 (one FMA and one subtraction): the low word of kd then holds k
// as a 32-bit integer for the final scaling, so no separate rounding or conversion is needed.
__device__ __forceinline__ double exp_nonpos(double x)
{
    x = __builtin_fmax(x, -1000.0);
    const double kd = __builtin_fma(x, kLog2e, 0x1.8p52);
    const double k = kd - 0x1.8p52;
    const int ki = (int)(unsigned)__builtin_bit_cast(unsigned long long, kd);
    double r = __builtin_fma(k, -kLn2Hi, x);
    r = __builtin_fma(k, -kLn2Lo, r);
    double p = 0x1.28a2c0a7209fbp-22;
    p = __builtin_fma(p, r, 0x1.72faf024b693bp-19);
    p = __builtin_fma(p, r, 0x1.a019a66a75dd4p-16);
    p = __builtin_fma(p, r, 0x1.a01978c6baf81p-13);
    p = __builtin_fma(p, r, 0x1.6c16c17f43a58p-10);
    p = __builtin_fma(p, r, 0x1.1111112dd67c5p-7);
    p = __builtin_fma(p, r, 0x1.55555555520afp-5);
    p = __builtin_fma(p, r, 0x1.555555554b757p-3);
    p = __builtin_fma(p, r, 0x1.0000000000005p-1);
    p = __builtin_fma(p, r, 0x1.000000000001ep+0);
    p = __builtin_fma(p, r, 1.0);
    return __builtin_ldexp(p, ki);
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
