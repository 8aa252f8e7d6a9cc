"""Derive the constants of the device exponential in lm_math.h (run: python gen_exp_coeffs.py).

Method (Cody & Waite argument reduction followed by a polynomial): for x <= 0,
    k = rint(x / ln 2),  r = x - k ln 2  in [-ln2/2, ln2/2],  exp(x) = 2^k * P(r).
ln 2 is split into a double LN2_HI and a correction LN2_LO = ln 2 - LN2_HI.  P is the
Chebyshev interpolant of exp on [-ln2/2, ln2/2] (near-minimax), computed at 60 digits with
mpmath and rounded to doubles; its monomial coefficients are printed in the order Horner's
rule consumes them (highest degree first).
"""
import mpmath as mp

mp.mp.dps = 60


def main(deg=10):
    ln2 = mp.log(2)
    hi = float(ln2)
    lo = float(ln2 - mp.mpf(hi))
    a = ln2 / 2
    poly, err = mp.chebyfit(mp.exp, [-a, a], deg + 1, error=True)
    coeffs = [float(c) for c in poly]            # highest degree first
    # error of the rounded-coefficient polynomial, relative, sampled densely
    worst = mp.mpf(0)
    for t in mp.linspace(-a, a, 4001):
        pv = mp.mpf(0)
        for c in coeffs:
            pv = pv * t + mp.mpf(c)
        worst = max(worst, abs(pv / mp.exp(t) - 1))
    print("// degree %d, relative error of the rounded polynomial on [-ln2/2, ln2/2]: %.3e" % (deg, float(worst)))
    print("LN2_HI = %r" % hi)
    print("LN2_LO = %r" % lo)
    print("LOG2E  = %r" % float(1 / ln2))
    for i, c in enumerate(coeffs):
        print("C%-2d = %s" % (deg - i, float.hex(c)))


if __name__ == "__main__":
    import sys
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 10)
