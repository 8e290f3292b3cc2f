"""Polynomial coefficients of rc_fastmath.hpp (prints them as hex floats).

    python paper_2505_08855_amd/csrc/fastmath_coeffs.py

Each polynomial starts from a Taylor series taken far beyond double precision
and is shortened by Chebyshev economization (Lanczos): the highest term
a_j x^j is replaced by the lower-degree part of a_j h^j T_j(x / h) / 2^(j-1)
on [-h, h] (of the shifted T_j(2 s / S - 1) on [0, S]), which moves the
polynomial by at most a_j h^j / 2^(j-1) over the interval.  All arithmetic
is exact (rational numbers); only the final coefficients are rounded to
double.

  2^f   on |f| <= 1/2:            (ln 2)^j / j!, economized to degree 11
  e^r   on |r| <= ln 2 / 2 + 1e-3: 1 / j!, economized to degree 11
  atanh on s = f^2 <= 0.02947:     2 atanh(f) = 2 f (1 + s p(s)),
                                   p(s) = sum_k s^k / (2 k + 3), to degree 6

Each replaced term moves the result by less than 2^-57 relative.  Measured
against quad-precision references on 4e6 random arguments each (host, fused
multiply-adds): exp2 and exp within 0.9 ulp, log within 2 ulp, the same
maxima as the degree-13 / degree-9 Taylor forms they replace; one degree
lower reaches 3-5 ulp.
"""
import math
from fractions import Fraction as F

LN2 = F("0.693147180559945309417232121458176568075500134360255254120680")
SQRT2 = F("1.41421356237309504880168872420969807856967187537694807317668")


def chebyshev(n):
    """Coefficients of T_n(y) in powers of y."""
    t = [[F(1)], [F(0), F(1)]]
    for k in range(2, n + 1):
        a = [F(0)] + [2 * c for c in t[k - 1]]
        b = t[k - 2] + [F(0)] * (len(a) - len(t[k - 2]))
        t.append([x - y for x, y in zip(a, b)])
    return t[n]


def economize(a, n, lo, hi):
    """Degree-n polynomial from the coefficients a (powers of x) on [lo, hi]."""
    a = list(a)
    mid, half = (lo + hi) / 2, (hi - lo) / 2
    for j in range(len(a) - 1, n, -1):
        if a[j] == 0:
            continue
        # T_j((x - mid) / half) expanded in powers of x
        poly = [F(0)] * (j + 1)
        for k, c in enumerate(chebyshev(j)):
            for m in range(k + 1):
                poly[m] += c * math.comb(k, m) * (1 / half) ** m * (-mid / half) ** (k - m)
        scale = a[j] / poly[j]
        for m in range(j + 1):
            a[m] -= scale * poly[m]
    return a[:n + 1]


def tables():
    terms = 24
    exp2 = economize([LN2 ** j / math.factorial(j) for j in range(terms)], 11, F(-1, 2), F(1, 2))
    h = LN2 / 2 + F(1, 1000)
    exp = economize([F(1, math.factorial(j)) for j in range(terms)], 11, -h, h)
    fmax = (SQRT2 - 1) / (SQRT2 + 1)
    atanh = economize([F(1, 2 * k + 3) for k in range(20)], 6, F(0), fmax ** 2 * F(1001, 1000))
    return {"exp2": exp2, "exp": exp, "atanh p": atanh}


if __name__ == "__main__":
    for name, c in tables().items():
        print(name + ", highest degree first:")
        for j in range(len(c) - 1, -1, -1):
            print("  %2d  %s" % (j, float.hex(float(c[j]))))
