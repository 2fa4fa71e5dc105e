"""Prints the polynomial coefficients of gccd_fp64.h: near-minimax
(Chebyshev) fits in 40-digit arithmetic, rounded to double, highest degree
first, with the largest relative error of the rounded polynomial on its
interval.

  exp(r)                      r in [-ln2/2, ln2/2]            degree 11
  q(s) = (2 atanh f - 2 f)/(f s), s = f^2 in [0, (3 - 2 sqrt 2)^2]   degree 6
  sin(pi r)/r, cos(pi r)      z = r^2 in [0, 1/16]            degrees 6, 7

Run: python fp64_coefficients.py
"""
import mpmath as mp

mp.mp.dps = 40


def fit(f, a, b, n):
    c = mp.chebyfit(f, [a, b], n)
    cd = [mp.mpf(float(x)) for x in c]
    worst = mp.mpf(0)
    for i in range(4001):
        x = a + (b - a) * i / 4000
        p = mp.mpf(0)
        for cc in cd:
            p = p * x + cc
        fx = f(x)
        worst = max(worst, abs(p - fx) / abs(fx))
    return [float(x) for x in c], float(worst)


def q(s):
    if s == 0:
        return mp.mpf(2) / 3
    f = mp.sqrt(s)
    return (2 * mp.atanh(f) - 2 * f) / (f * s)


def sinc(z):
    if z == 0:
        return mp.pi
    r = mp.sqrt(z)
    return mp.sin(mp.pi * r) / r


def cosr(z):
    return mp.cos(mp.pi * mp.sqrt(z))


if __name__ == "__main__":
    half = mp.log(2) / 2 * (1 + mp.mpf("1e-6"))
    smax = ((mp.sqrt(2) - 1) / (mp.sqrt(2) + 1)) ** 2 * (1 + mp.mpf("1e-6"))
    for name, f, a, b, n in (("exp", mp.exp, -half, half, 12), ("log q", q, mp.mpf(0), smax, 7),
                             ("sin(pi r)/r", sinc, mp.mpf(0), mp.mpf(1) / 16, 7),
                             ("cos(pi r)", cosr, mp.mpf(0), mp.mpf(1) / 16, 8)):
        c, w = fit(f, a, b, n)
        print(f"{name}: max relative error {w:.2e}")
        for x in c:
            print(f"    {x!r},")
