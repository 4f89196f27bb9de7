"""Coefficients of the reduced-range sincos in tdse_device.hpp (sincos_rr).

On |r| <= pi/4, sin r = r + r^3 S(r^2) and cos r = 1 - r^2/2 + r^4 C(r^2),
with S and C polynomials of degree 5 in t = r^2 obtained by Chebyshev
interpolation on t in [0, (pi/4)^2] at 50 significant digits (mpmath).  The
script prints the coefficients (highest degree first, rounded to double) and
the largest error of the double-precision Horner evaluation against mpmath
on a uniform grid of |r| <= pi/4.

Run: python sincos_coefficients.py   (needs mpmath)
"""
import mpmath as mp

mp.mp.dps = 50
T = (mp.pi / 4) ** 2
DEGREE = 5


def s_rest(t):
    if t == 0:
        return mp.mpf(-1) / 6
    r = mp.sqrt(t)
    return (mp.sin(r) - r) / r ** 3


def c_rest(t):
    if t == 0:
        return mp.mpf(1) / 24
    r = mp.sqrt(t)
    return (mp.cos(r) - 1 + t / 2) / t ** 2


def horner(coefs, t):
    p = coefs[0]
    for c in coefs[1:]:
        p = p * t + c
    return p


def main():
    cs = [float(c) for c in mp.chebyfit(s_rest, [0, T], DEGREE + 1)]
    cc = [float(c) for c in mp.chebyfit(c_rest, [0, T], DEGREE + 1)]
    print("S:", ", ".join(repr(c) for c in cs))
    print("C:", ", ".join(repr(c) for c in cc))
    err_s = err_c = mp.mpf(0)
    n = 4001
    for i in range(n):
        x = float(-mp.pi / 4 + (mp.pi / 2) * i / (n - 1))
        t = x * x
        # evaluated in the kernel's order: ((S t) r) + r and ((C t) - 1/2) t + 1
        s = (horner(cs, t) * t) * x + x
        c = (horner(cc, t) * t - 0.5) * t + 1.0
        err_s = max(err_s, abs(mp.mpf(s) - mp.sin(mp.mpf(x))))
        err_c = max(err_c, abs(mp.mpf(c) - mp.cos(mp.mpf(x))))
    print("max |error| in double: sin", mp.nstr(err_s, 3), "cos", mp.nstr(err_c, 3))


if __name__ == "__main__":
    main()
