"""Writes fp64_series.hpp: the polynomial coefficients of the FP64 Box-Muller
transform (ln of the radius uniform, sine and cosine of the reduced angle).

Each polynomial is the Taylor series of the function, economised on its
interval by Chebyshev truncation: the series (to a degree whose remainder is
negligible) is rewritten in Chebyshev polynomials of the interval, the
highest ones are dropped while their coefficients sum to at most 2^-57, and
the rest is converted back to powers.  All of it runs in exact rational
arithmetic; each coefficient is rounded once to FP64 at the end.

    sin r = r S(r^2),  cos r = C(r^2)   for 0 <= r <= pi/4
    ln m = 2 artanh z = 2 z A(z^2)      for |z| <= (sqrt2 - 1)/(sqrt2 + 1)

    python paper_1204_6734_amd/csrc/gen_fp64_series.py   # rewrites fp64_series.hpp
"""
import os
from fractions import Fraction as Fr
from math import comb, factorial

HERE = os.path.dirname(os.path.abspath(__file__))
TARGET = Fr(1, 2 ** 57)


def chebyshev_of(coef, X):
    """Chebyshev coefficients (in t, x = X (t + 1) / 2) of sum_k coef[k] x^k."""
    n = len(coef)
    pt = [Fr(0)] * n
    for k, a in enumerate(coef):
        s = a * X ** k / 2 ** k
        for m in range(k + 1):
            pt[m] += s * comb(k, m)
    c = [Fr(0)] * n
    for m, a in enumerate(pt):
        for i in range(m // 2 + 1):
            j = m - 2 * i
            w = Fr(comb(m, i), 2 ** (m - 1)) if m > 0 else Fr(1)
            if j == 0 and m > 0:
                w /= 2
            c[j] += a * w
    return c


def powers_of(c, X):
    """Coefficients of the powers of x for sum_j c[j] T_j(2 x / X - 1)."""
    n = len(c)
    T = [[Fr(1)], [Fr(0), Fr(1)]]
    for j in range(2, n):
        a = [Fr(0)] + [2 * v for v in T[j - 1]]
        b = T[j - 2] + [Fr(0)] * (len(a) - len(T[j - 2]))
        T.append([u - v for u, v in zip(a, b)])
    pt = [Fr(0)] * n
    for j, cj in enumerate(c):
        for m, v in enumerate(T[j]):
            pt[m] += cj * v
    px = [Fr(0)] * n
    for m, a in enumerate(pt):
        for k in range(m + 1):
            px[k] += a * comb(m, k) * Fr(2) ** k / X ** k * (-1) ** (m - k)
    return px


def economise(taylor, X):
    c = chebyshev_of(taylor, X)
    for n in range(1, len(c) + 1):
        tail = sum(abs(v) for v in c[n:])
        if tail <= TARGET:
            return powers_of(c[:n], X), tail
    raise ValueError("series too short")


def header_text() -> str:
    R2 = Fr(7854, 10000) ** 2        # (pi/4)^2 < 0.7854^2
    Z2 = Fr(1716, 10000) ** 2        # ((sqrt2 - 1)/(sqrt2 + 1))^2 = 0.17157^2 < 0.1716^2
    polys = {
        "kSinSeries": (economise([Fr((-1) ** k, factorial(2 * k + 1)) for k in range(16)], R2),
                       "sin r = r S(r^2), 0 <= r <= pi/4"),
        "kCosSeries": (economise([Fr((-1) ** k, factorial(2 * k)) for k in range(16)], R2),
                       "cos r = C(r^2), 0 <= r <= pi/4"),
        "kAtanhSeries": (economise([Fr(1, 2 * k + 1) for k in range(18)], Z2),
                         "artanh z = z A(z^2), |z| <= 0.1716"),
    }
    lines = ["// fp64_series.hpp — written by gen_fp64_series.py (same folder); do not edit.",
             "//",
             "// Coefficients, in increasing powers of the argument squared, of the",
             "// polynomials of the FP64 Box-Muller transform: Taylor series economised by",
             "// Chebyshev truncation (dropped coefficients sum to at most 2^-57) in exact",
             "// rational arithmetic, rounded once to FP64.",
             "#pragma once", "", "namespace flb {", ""]
    for name, ((px, tail), what) in polys.items():
        lines.append(f"// {what}; truncation {float(tail):.2e}")
        body = ", ".join(repr(float(v)) for v in px)
        lines.append(f"constexpr int {name}Terms = {len(px)};")
        lines.append(f"constexpr double {name}[{len(px)}] = {{{body}}};")
        lines.append("")
    lines.append("}  // namespace flb")
    return "\n".join(lines) + "\n"


def main():
    with open(os.path.join(HERE, "fp64_series.hpp"), "w") as fh:
        fh.write(header_text())


if __name__ == "__main__":
    main()
