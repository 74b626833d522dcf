"""The Markidis two-term FP16 product (Sec. 4.5), FP64 reference of the terms
(test infrastructure).

Each operand is split into a high and a low FP16 part,
    X0 = FP16[X],  X1 = FP16[X - X0],
after the power-of-two row (column) scaling of the Ozaki scheme that the
paper applied to the Markidis method as well (Sec. 4.5): rows of A are
scaled by 2^-e_i and columns of B by 2^-f_j with the frexp exponents of their
largest entries, so every scaled value lies in (-1, 1).  The product keeps
1 to 4 terms, in the order Table 2 defines them:
    1 term   A0 B0
    2 terms  + A0 B1
    3 terms  + A1 B0
    4 terms  + A1 B1
and the method accumulates them in FP32 on FP16 tensor units.  Reading: the
fourth term of Table 2's caption repeats A0 B0, which the four-term product
written in Sec. 4.5 shows to be A1 B1.

``markidis_gemm`` forms the kept terms in FP64 (each FP16 x FP16 product is
exact in FP64 and the sums round at the FP64 level), so it is the value an
exact accumulator would give; an FP32 accumulation of the same terms stays
within ``fp32_accumulation_bound`` of it.  FP16 conversions are numpy's
round-to-nearest-even casts.
"""
from __future__ import annotations

import numpy as np

from .ozaki import row_exponents

FP16_UNIT = 2.0 ** -11      # unit roundoff of FP16 (11 significant bits)
FP32_UNIT = 2.0 ** -24


def to_fp16(x):
    """Round to the nearest FP16 value (ties to even), returned as float64."""
    return np.asarray(x, dtype=np.float64).astype(np.float16).astype(np.float64)


def split16(x):
    """(X0, X1) = (FP16[x], FP16[x - X0])."""
    hi = to_fp16(x)
    lo = to_fp16(np.asarray(x, dtype=np.float64) - hi)
    return hi, lo


def scaled_split(a, b):
    """Row / column exponents and the FP16 parts of the scaled operands."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    e = row_exponents(a)
    f = row_exponents(b.T)
    a0, a1 = split16(np.ldexp(a, -e[:, None]))
    b0, b1 = split16(np.ldexp(b, -f[None, :]))
    return e, f, (a0, a1), (b0, b1)


TERMS = ((0, 0), (0, 1), (1, 0), (1, 1))     # (A part, B part) of terms 1..4


def markidis_gemm(a, b, terms):
    """Sum of the first ``terms`` term products, scaled back (FP64)."""
    if not 1 <= terms <= 4:
        raise ValueError("terms must be 1..4")
    e, f, ap, bp = scaled_split(a, b)
    c = np.zeros((ap[0].shape[0], bp[0].shape[1]))
    for s, t in TERMS[:terms]:
        c = c + ap[s] @ bp[t]
    return np.ldexp(c, e[:, None] + f[None, :])


def fp32_accumulation_bound(a, b, terms):
    """Bound on |FP32-accumulated terms - markidis_gemm(a, b, terms)|: at most
    k * terms + 1 FP32 roundings, each of at most 2^-24 times the running
    magnitude, which is bounded by sum over kept terms of |A_s| |B_t|."""
    e, f, ap, bp = scaled_split(a, b)
    k = ap[0].shape[1]
    mag = np.zeros((ap[0].shape[0], bp[0].shape[1]))
    for s, t in TERMS[:terms]:
        mag = mag + np.abs(ap[s]) @ np.abs(bp[t])
    return np.ldexp((k * terms + 1) * FP32_UNIT * mag, e[:, None] + f[None, :])
