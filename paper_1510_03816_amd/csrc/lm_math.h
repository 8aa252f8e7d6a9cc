// lm_math.h -- device math for the pair kernels (gfx950).
//
// The pair kernels need exp of a non-positive argument and 1/sqrt of a positive one, in
// double and in single precision.  Both precisions take the exponential in base 2: the
// caller folds log2(e) into the kernel's scale constant, so the argument x = y log2(e) of
// 2^x arrives with the one rounding of the product that forms it.  There is no
// double-precision exp instruction; the one here reduces the argument after Cody & Waite
// (W. J. Cody and W. Waite, "Software Manual for the Elementary Functions", 1980), in base 2
// so that the reduction is exact: k = rint(x), f = x - k in [-1/2, 1/2], 2^x = 2^k P(f) with
// P(f) = 1 + f Q(f) a degree-9 polynomial (P(0) = 1 exactly, so the kernel is exactly 1 at
// distance 0).  The constants were derived for this library by gen_exp_coeffs.py (Chebyshev
// interpolation of (2^f - 1)/f on [-1/2, 1/2] at 60 digits, rounded to double): the rounded
// polynomial is within 3.7e-14 of 2^f on that interval.  Degree 10 (5.7e-16) costs one more
// FMA per pair, measured as 1.6% of the N = 65536 stage, for an error that stays orders of
// magnitude below the 1e-10 parity bar.  Against the
// natural-base reduction the base-2 one saves the second half of the split ln 2 (one FMA per
// pair) at the same accuracy: either way the argument carries the relative rounding error of
// the products that form it.
//
// The reciprocal square root starts from the hardware estimate v_rsq_f64 (relative error
// 5.2e-8 = 2^-24.2, measured on gfx950 over 2^20 arguments in [2^-20, 2^20]) and applies one
// Newton step y <- y + (y/2) t, t = 1 - s y^2, which leaves 1.5 (5.2e-8)^2 ~ 4e-15 before
// rounding.  A third-order step (y (1 + t/2 + 3t^2/8), ~4e-22) costs one instruction more per
// pair: 2% of the N = 65536 stage.
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
    double p = 0x1.b63880a30e9ffp-24;
    p = __builtin_fma(p, f, 0x1.63d136366db24p-20);
    p = __builtin_fma(p, f, 0x1.ffcb9515a8016p-17);
    p = __builtin_fma(p, f, 0x1.4308ac85aa947p-13);
    p = __builtin_fma(p, f, 0x1.5d87fe86fe88ep-10);
    p = __builtin_fma(p, f, 0x1.3b2ab7181b755p-7);
    p = __builtin_fma(p, f, 0x1.c6b08d7047e52p-5);
    p = __builtin_fma(p, f, 0x1.ebfbdff823cedp-3);
    p = __builtin_fma(p, f, 0x1.62e42fefa39efp-1);
    p = __builtin_fma(p, f, 1.0);
    return __builtin_ldexp(p, ki);
}

// 2^x for x <= 0 to 5.7e-16: the same reduction with the degree-10 polynomial (gen_exp_coeffs.py
// 10).  For the entries of the dense kernel matrix, built once per match, whose solves amplify
// entry errors by the condition number; the pair sums use exp2_nonpos.
__device__ __forceinline__ double exp2_nonpos_fine(double x)
{
    x = __builtin_fmax(x, -1500.0);
    const double kd = x + 0x1.8p52;
    const double k = kd - 0x1.8p52;
    const int ki = (int)(unsigned)__builtin_bit_cast(unsigned long long, kd);
    const double f = x - k;
    double p = 0x1.e5e9f548e5725p-28;
    p = __builtin_fma(p, f, 0x1.b6571de2f2351p-24);
    p = __builtin_fma(p, f, 0x1.62bfe46117445p-20);
    p = __builtin_fma(p, f, 0x1.ffcb76789860fp-17);
    p = __builtin_fma(p, f, 0x1.4309130378460p-13);
    p = __builtin_fma(p, f, 0x1.5d87fe908f88ap-10);
    p = __builtin_fma(p, f, 0x1.3b2ab6fba385fp-7);
    p = __builtin_fma(p, f, 0x1.c6b08d7044119p-5);
    p = __builtin_fma(p, f, 0x1.ebfbdff82c590p-3);
    p = __builtin_fma(p, f, 0x1.62e42fefa39f7p-1);
    p = __builtin_fma(p, f, 1.0);
    return __builtin_ldexp(p, ki);
}

// 1/sqrt(s) for s > 0 (callers clamp s away from zero).
__device__ __forceinline__ double rsqrt_pos(double s)
{
    const double y = __builtin_amdgcn_rsq(s);
    const double e = s * y;
    const double t = __builtin_fma(-e, y, 1.0);
    return __builtin_fma(y * 0.5, t, y);
}

// Single precision: the hardware 2^x and 1/sqrt(x) (about one ulp each).
__device__ __forceinline__ float exp2_f32(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rsqrt_f32(float s) { return __builtin_amdgcn_rsqf(s); }

}  // namespace lm
