"""Exact-rational references for tiny inputs (test infrastructure).

These evaluate the definitions behind the Ozaki scheme (Sec. 2.4) with
Python integers and fractions, with no floating-point rounding at all, so
they can pin the vectorised FP64 oracle in ``ozaki.py``:

* the digits of one matrix entry, from the integer
  X = round-half-even(A_ij 2^(8 S - 2 - e_i)) and its base-256 expansion with
  signed-byte lower digits;
* the exact product A B and its correctly rounded FP64 value;
* the exact value of the truncated slice sum (pairs with i + j <= S + 1).
"""
from __future__ import annotations

from fractions import Fraction
import math


def frexp_exponent(x):
    """e with 2^(e-1) <= |x| < 2^e, and 0 for x == 0 (exact, from the float)."""
    if x == 0:
        return 0
    return math.frexp(x)[1]


def entry_digits(x, e, s):
    """Digits d_1..d_S of float x scaled by 2^-e (definition, exact integers)."""
    big = round(Fraction(x) * Fraction(2) ** (8 * s - 2 - e))   # half to even
    digits = []
    rest = big
    for _ in range(s - 1):
        low = rest % 256
        if low >= 128:
            low -= 256
        digits.append(low)
        rest = (rest - low) // 256
    digits.append(rest)
    return digits[::-1]


def digits_value(digits, e):
    """Exact value 2^e sum_s d_s 2^-(8 s - 2)."""
    return sum(Fraction(d) * Fraction(2) ** (e - (8 * (i + 1) - 2))
               for i, d in enumerate(digits))


def exact_product(a, b):
    """Exact A B (list of lists of Fractions)."""
    m, k, n = len(a), len(a[0]), len(b[0])
    fa = [[Fraction(v) for v in row] for row in a]
    fb = [[Fraction(v) for v in row] for row in b]
    return [[sum(fa[i][t] * fb[t][j] for t in range(k)) for j in range(n)]
            for i in range(m)]


def exact_truncated_product(a, b, s):
    """Exact value of the Ozaki slice sum over pairs i + j <= S + 1."""
    m, k, n = len(a), len(a[0]), len(b[0])
    e = [frexp_exponent(max(abs(v) for v in row)) for row in a]
    f = [frexp_exponent(max(abs(b[t][j]) for t in range(k))) for j in range(n)]
    da = [[entry_digits(a[i][t], e[i], s) for t in range(k)] for i in range(m)]
    db = [[entry_digits(b[t][j], f[j], s) for j in range(n)] for t in range(k)]
    out = []
    for i in range(m):
        row = []
        for j in range(n):
            tot = Fraction(0)
            for si in range(1, s + 1):
                for sj in range(1, s + 2 - si):
                    w = Fraction(2) ** (e[i] + f[j] - (8 * (si + sj) - 4))
                    tot += w * sum(da[i][t][si - 1] * db[t][j][sj - 1]
                                   for t in range(k))
            row.append(tot)
        out.append(row)
    return out


def to_float(mat):
    """Correctly rounded float of every Fraction entry."""
    return [[float(v) for v in row] for row in mat]
