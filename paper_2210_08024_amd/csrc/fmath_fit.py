"""Coefficients of the polynomial in fmath.h's fexp.

e^r = 1 + r + r^2 g(r) with g(r) = (e^r - 1 - r) / r^2; g is fitted on |r| <= 0.35 (the
reduced argument stays within ln 2 / 2 = 0.3466) by Chebyshev interpolation of degree 9
(mpmath.chebyfit, 50 digits), and the coefficients are rounded to double.  Prints them
highest degree first as C hex literals, and the largest relative error of 1 + r + r^2 g(r)
with the rounded coefficients over the interval (about 0.2 ulp).

    python paper_2210_08024_amd/csrc/fmath_fit.py
"""
import mpmath as mp

mp.mp.dps = 50
A = mp.mpf("0.35")
DEG = 9


def g(r):
    if abs(r) < mp.mpf("1e-20"):
        return mp.mpf(1) / 2 + r / 6
    return (mp.exp(r) - 1 - r) / (r * r)


def main():
    poly, _ = mp.chebyfit(g, [-A, A], DEG + 1, error=True)
    co = [float(c) for c in poly]
    worst = mp.mpf(0)
    for i in range(4001):
        r = -A + 2 * A * i / 4000
        p = mp.mpf(0)
        for c in co:
            p = p * r + mp.mpf(c)
        worst = max(worst, abs(1 + r + r * r * p - mp.exp(r)) / mp.exp(r))
    for c in co:
        print(float.hex(c))
    print("max relative error", mp.nstr(worst, 3), "=", mp.nstr(worst / mp.mpf(2) ** -53, 3), "ulp")


if __name__ == "__main__":
    main()
