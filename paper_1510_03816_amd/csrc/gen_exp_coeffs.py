"""Derive the constants of the device exponential in lm_math.h (run: python gen_exp_coeffs.py).

The pair kernels need exp(y) for y <= 0.  The caller folds log2(e) into the kernel's scale
constant and asks for 2^x with x = y log2(e).  Reduction (after Cody & Waite, with base 2 so
that it is exact): k = rint(x), f = x - k in [-1/2, 1/2] (exact in double), 2^x = 2^k P(f).
P is the Chebyshev interpolant of 2^f on [-1/2, 1/2] (near-minimax), computed at 60 digits
with mpmath and rounded to doubles; its monomial coefficients are printed in the order
Horner's rule consumes them (highest degree first).
"""
import mpmath as mp

mp.mp.dps = 60


def main(deg=10):
    a = mp.mpf(1) / 2
    two = lambda t: mp.power(2, t)
    poly, err = mp.chebyfit(two, [-a, a], deg + 1, error=True)
    coeffs = [float(c) for c in poly]            # highest degree first
    # error of the rounded-coefficient polynomial, relative, sampled densely
    worst = mp.mpf(0)
    for t in mp.linspace(-a, a, 4001):
        pv = mp.mpf(0)
        for c in coeffs:
            pv = pv * t + mp.mpf(c)
        worst = max(worst, abs(pv / two(t) - 1))
    print("// degree %d, relative error of the rounded polynomial on [-1/2, 1/2]: %.3e" % (deg, float(worst)))
    print("LOG2E  = %r" % float(1 / mp.log(2)))
    for i, c in enumerate(coeffs):
        print("C%-2d = %s" % (deg - i, float.hex(c)))


if __name__ == "__main__":
    import sys
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 10)
