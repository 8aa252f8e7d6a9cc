"""Derive the constants of the device exponential in lm_math.h (run: python gen_exp_coeffs.py).

The pair kernels need exp(y) for y <= 0.  The caller folds log2(e) into the kernel's scale
constant and asks for 2^x with x = y log2(e).  Reduction (after Cody & Waite, with base 2 so
that it is exact): k = rint(x), f = x - k in [-1/2, 1/2] (exact in double), 2^x = 2^k P(f).
P(f) = 1 + f Q(f) keeps P(0) = 1 exactly (the kernel's value at distance 0 is exactly 1), with
Q the Chebyshev interpolant of (2^f - 1)/f on [-1/2, 1/2] (near-minimax), computed at 60
digits with mpmath and rounded to doubles; the monomial coefficients of P are printed in the
order Horner's rule consumes them (highest degree first, the constant 1 last).
"""
import mpmath as mp

mp.mp.dps = 60


def main(deg=9):
    a = mp.mpf(1) / 2
    two = lambda t: mp.power(2, t)
    q = lambda t: (two(t) - 1) / t if t != 0 else mp.log(2)
    poly, err = mp.chebyfit(q, [-a, a], deg, error=True)      # Q of degree deg - 1
    coeffs = [float(c) for c in poly] + [1.0]                 # P = 1 + f Q, highest degree first
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
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 9)
