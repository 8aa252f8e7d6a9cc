// lm_math.h -- device math for the pair kernels (gfx950).
//
// The pair kernels need exp of a non-positive argument and 1/sqrt of a positive one, in
// double and in single precision.  Both precisions take the exponential in base 2: the
// caller folds log2(e) into the kernel's scale constant, so the argument x = y log2(e) of
// 2^x arrives with the one rounding of the product that forms it.  There is no
// double-precision exp instruction; the one here reduces the argument after Cody & Waite
// (W. J. Cody and W. Waite, "Software Manual for the Elementary Functions", 1980), in base 2
// so that the reduction is exact: k = rint(x), f = x - k in [-1/2, 1/2], 2^x = 2^k P(f) with
// P a degree-10 polynomial.  The constants were derived for this library by
// gen_exp_coeffs.py (Chebyshev interpolation of 2^f on [-1/2, 1/2] at 60 digits, rounded to
// double): the rounded polynomial is within 3.1e-16 of 2^f on that interval (degree 11 would
// give 2.0e-17 for one more FMA per pair; the difference is far below the parity bar and the
// sums' own rounding).  Against the natural-base reduction it saves the second half of the
// split ln 2 (one FMA per pair) at the same accuracy: either way the argument carries the
// relative rounding error of the products that form it.
//
// The reciprocal square root starts from the hardware estimate v_rsq_f64 (relative error
// 5.2e-8 = 2^-24.2, measured on gfx950 over 2^20 arguments in [2^-20, 2^20]) and applies one
// third-order correction y <- y (1 + t/2 + 3t^2/8), t = 1 - s y^2 (the Taylor series of
// (1 - t)^(-1/2)), which leaves about 2.5 (5.2e-8)^3 ~ 4e-22 before rounding.
#pragma once

#include <hip/hip_runtime.h>

namespace lm {

// 2^x for x <= 0.  Arguments below -1500 return 0 (2^x underflows below -1075); the clamp
// also keeps the reduction finite for huge |x|.  k = rint(x) comes from adding and
// subtracting 1.5 * 2^52: the low word of kd then holds k as a 32-bit integer for the final
// scaling, so no separate rounding or conversion is needed, and f = x - k is exact.
__device__ __forceinline__ double exp2_nonpos(double x)
{
    x = __builtin_fmax(x, -1500.0);
    const double kd = x + 0x1.8p52;
    const double k = kd - 0x1.8p52;
    const int ki = (int)(unsigned)__builtin_bit_cast(unsigned long long, kd);
    const double f = x - k;
    double p = 0x1.e6063f7217bc6p-28;
    p = __builtin_fma(p, f, 0x1.b675bca4eeebbp-24);
    p = __builtin_fma(p, f, 0x1.62bfd47773353p-20);
    p = __builtin_fma(p, f, 0x1.ffcb54062e698p-17);
    p = __builtin_fma(p, f, 0x1.430913096fd9fp-13);
    p = __builtin_fma(p, f, 0x1.5d87fe9d7a584p-10);
    p = __builtin_fma(p, f, 0x1.3b2ab6fba1ddap-7);
    p = __builtin_fma(p, f, 0x1.c6b08d703ce49p-5);
    p = __builtin_fma(p, f, 0x1.ebfbdff82c598p-3);
    p = __builtin_fma(p, f, 0x1.62e42fefa3a19p-1);
    p = __builtin_fma(p, f, 1.0);
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
