"""The Ozaki scheme for C = A B, step by step in FP64 (test infrastructure).

Sec. 2.4: each input is split into S matrices of the same size that are
exactly representable in the low-precision format, by rounding and bit
shifts, after a power-of-two scaling per row of A and per column of B that
keeps every slice in range; the slice products A_i B_j with i + j <= S + 1 are
formed without rounding error and the results are summed in the original
precision.  Products needed: S (S + 1) / 2.

The concrete split used here (a reading of the paper's pointer to the
round-to-nearest extraction of Minamihata et al.; the design notes list it):

  scaling   e_i = frexp exponent of max_j |A_ij|, i.e.
            2^(e_i - 1) <= max_j |A_ij| < 2^e_i  (e_i = 0 for a zero row),
            so r_ij = A_ij 2^-e_i lies in (-1, 1);
  digits    X_ij = round-to-nearest-even(r_ij 2^(8 S - 2)), an integer with
            |X_ij| <= 2^(8 S - 2); its digits d_1 .. d_S satisfy
                X = sum_s d_s 2^(8 (S - s)),
            d_2 .. d_S in [-128, 127] (signed bytes) and d_1 in [-64, 65],
            so every digit is an exact INT8 and an exact FP16 value;
  value     A_ij ~= 2^e_i sum_s d_s 2^-(8 s - 2), with error at most
            2^(e_i - 8 S + 1).

Columns of B are split the same way with exponents f_j.  The slice product
of digit planes s and t carries weight 2^-(8 (s + t) - 4); products are
grouped by g = s + t (2 <= g <= S + 1), every group sum G_g is an exact
integer, and

  C_ij = 2^(e_i + f_j) * sum_{g = S+1 down to 2} G_g,ij 2^-(8 g - 4),

added from the smallest weight up, one FP64 rounding per addition.

The digits are computed here by the greedy top-down extraction (round the
scaled value to the nearest integer, keep the exact remainder, shift it up by
8 bits, repeat), followed by a carry pass that moves any digit equal to 128
into the digit above; ``exact.py`` pins this against the integer definition.
"""
from __future__ import annotations

import numpy as np

DIGIT_BITS = 8          # bits carried by every digit after the first
TOP_BITS = 6            # fractional bits of the first digit


def row_exponents(a):
    """frexp exponent of every row's largest magnitude (0 for a zero row)."""
    m = np.max(np.abs(a), axis=1) if a.shape[1] else np.zeros(a.shape[0])
    _, e = np.frexp(m)
    return e.astype(np.int64)


def split_rows(a, s):
    """(e, D): row exponents and digit planes D[s-1] of shape a.shape."""
    a = np.asarray(a, dtype=np.float64)
    e = row_exponents(a)
    x = np.ldexp(a, (TOP_BITS - e)[:, None])     # exact: |x| < 2^6
    d = np.zeros((s,) + a.shape, dtype=np.int64)
    for i in range(s):
        q = np.rint(x)                            # ties to even
        d[i] = np.nan_to_num(q).astype(np.int64)
        x = (x - q) * 2.0 ** DIGIT_BITS           # exact remainder, |x| <= 128
    for i in range(s - 1, 0, -1):                 # carry 128 -> -128 (+1 above)
        hi = d[i] >= 128
        d[i][hi] -= 256
        d[i - 1][hi] += 1
    return e, d


def split_cols(b, s):
    """(f, E): column exponents and digit planes of b (split by columns)."""
    f, dt = split_rows(np.asarray(b, dtype=np.float64).T, s)
    return f, np.transpose(dt, (0, 2, 1))


def group_products(d, dt):
    """G[g-2] = sum_{i+j=g} D_i E_j for g = 2..S+1, as exact float64 integers.

    D: (S, m, k) row digits of A; dt: (S, k, n) column digits of B.  Every
    partial sum is an integer below 2^53, so the float64 products are exact.
    """
    s = d.shape[0]
    out = np.zeros((s, d.shape[1], dt.shape[2]))
    df = d.astype(np.float64)
    ef = dt.astype(np.float64)
    for g in range(2, s + 2):
        for i in range(1, g):
            j = g - i
            if j <= s:
                out[g - 2] += df[i - 1] @ ef[j - 1]
    return out


def combine(groups, e, f):
    """FP64 sum of the scaled group products, smallest weight first."""
    s = groups.shape[0]
    acc = np.zeros(groups.shape[1:])
    for g in range(s + 1, 1, -1):
        acc = acc + np.ldexp(groups[g - 2], -(DIGIT_BITS * g - 4))
    return np.ldexp(acc, e[:, None] + f[None, :])


def ozaki_gemm(a, b, s):
    """Approximate A @ B with S slices (exact up to the split truncation)."""
    e, d = split_rows(a, s)
    f, dt = split_cols(b, s)
    return combine(group_products(d, dt), e, f)


def products_count(s):
    """Number of slice-pair products, S (S + 1) / 2 (Sec. 2.4)."""
    return s * (s + 1) // 2


def error_bound(a, b, s):
    """Elementwise bound on |ozaki_gemm(a, b, s) - a @ b|.

    Split truncation of both operands (each digit string rounds to within
    2^(e - 8S + 1)), the slice pairs beyond the anti-diagonal that are left
    out, and one rounding per FP64 addition of the group sums.
    """
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    k = a.shape[1]
    e = row_exponents(a).astype(np.float64)
    f = row_exponents(b.T).astype(np.float64)
    scale = np.exp2(e[:, None] + f[None, :])
    trunc = scale * k * 2.0 ** (-DIGIT_BITS * s + 1) * 2.5
    dropped = scale * k * (s + 1) * 2.0 ** (-DIGIT_BITS * s + 2)
    rounding = (s + 2) * 2.0 ** -53 * (np.abs(a) @ np.abs(b) + scale * k * 2.0 ** -10)
    return trunc + dropped + rounding
