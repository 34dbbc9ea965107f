"""Coefficients of exp2_d's polynomial (csrc/lps_math64.hpp): e^t on
[-ln 2 / 2, ln 2 / 2] interpolated at the 12 Chebyshev nodes of that interval
(degree 11, near the minimax polynomial), computed in 50-digit decimal
arithmetic and rounded to double; prints them with the largest relative error
of the rounded polynomial on a fine grid.  Run: python3 gen_exp2_poly.py"""
from decimal import Decimal as D, getcontext

getcontext().prec = 50
DEG = 11


def cos(x):
    c, term, i = D(1), D(1), 0
    while True:
        i += 2
        term = -term * x * x / (D(i - 1) * D(i))
        if abs(term) < D(10) ** -45:
            return c
        c += term


def coefficients(n):
    pi = D("3.14159265358979323846264338327950288419716939937510")
    h = D(2).ln() / 2
    nodes = [h * cos(pi * D(2 * k + 1) / D(2 * (n + 1))) for k in range(n + 1)]
    a = [[t ** j for j in range(n + 1)] + [t.exp()] for t in nodes]
    m = n + 1
    for col in range(m):   # Gauss-Jordan elimination with partial pivoting
        piv = max(range(col, m), key=lambda r: abs(a[r][col]))
        a[col], a[piv] = a[piv], a[col]
        for r in range(m):
            if r != col:
                f = a[r][col] / a[col][col]
                for cc in range(col, m + 1):
                    a[r][cc] -= f * a[col][cc]
    return [float(a[i][m] / a[i][i]) for i in range(m)], h


if __name__ == "__main__":
    c, h = coefficients(DEG)
    worst = D(0)
    for i in range(4001):
        t = -h + 2 * h * D(i) / D(4000)
        p = D(0)
        for v in reversed(c):
            p = p * t + D(v)
        worst = max(worst, abs(p - t.exp()) / t.exp())
    for j, v in enumerate(c):
        print(f"c{j} = {v.hex()}  ({v!r})")
    print(f"max relative error {float(worst):.3g} ({float(worst) / 2 ** -53:.3f} ulp)")
