"""Coefficients of the polynomials in fmath.h's fexp and flog.

exp: e^r = 1 + r + r^2 g(r) with g(r) = (e^r - 1 - r) / r^2; g is fitted on |r| <= 0.35 (the
reduced argument stays within ln 2 / 2 = 0.3466) by Chebyshev interpolation of degree 9.
log: ln m = 2 atanh s = 2 s + s z p(z), z = s^2, with p(z) = 2 (atanh s - s) / s^3 fitted on
0 <= z <= 0.0295 (|s| <= 3 - 2 sqrt 2 = 0.1716) by Chebyshev interpolation of degree 6.
Both by mpmath.chebyfit at 50 digits, coefficients rounded to double.  Prints them highest
degree first as C hex literals, and the largest relative error of each approximation with
the rounded coefficients over its interval (about 0.2 and 0.04 ulp).

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


def p_log(z):
    if z < mp.mpf("1e-30"):
        return mp.mpf(2) / 3
    s = mp.sqrt(z)
    return 2 * (mp.atanh(s) - s) / s ** 3


def fit_log():
    poly, _ = mp.chebyfit(p_log, [0, mp.mpf("0.0295")], 7, error=True)
    co = [float(c) for c in poly]
    worst = mp.mpf(0)
    for i in range(1, 4001):
        s = mp.mpf("0.1716") * (-1 + 2 * mp.mpf(i) / 4001)
        z = s * s
        p = mp.mpf(0)
        for c in co:
            p = p * z + mp.mpf(c)
        ref = 2 * mp.atanh(s)
        worst = max(worst, abs(2 * s + s * z * p - ref) / abs(ref))
    print("log")
    for c in co:
        print(float.hex(c))
    print("max relative error", mp.nstr(worst, 3), "=", mp.nstr(worst / mp.mpf(2) ** -53, 3), "ulp")


def main():
    print("exp")
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
    fit_log()


if __name__ == "__main__":
    main()
