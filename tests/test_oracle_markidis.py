"""Pins for the Markidis-scheme oracle (Sec. 4.5)."""
import numpy as np
import pytest

from oracle import markidis


def test_split_of_one_third_by_hand():
    """1/3 = 0.0101...b: the nearest FP16 is 1365/4096 (11 significant bits,
    rounded down); the remainder 1/12288 = (4/3) 2^-14 is a normal FP16
    number whose nearest value is 1365 2^-24."""
    hi, lo = markidis.split16(np.array([1.0 / 3.0]))
    assert hi[0] == 1365 / 4096
    assert lo[0] == 1365 * 2.0 ** -24
    # what is left is 1/12288 - 1365 2^-24 = 2^-24 / 3
    assert abs((1.0 / 3.0 - hi[0] - lo[0]) - 2.0 ** -24 / 3.0) < 1e-16   # FP64 1/3 is rounded


def test_split_exact_and_subnormal_cases():
    hi, lo = markidis.split16(np.array([0.75, -2.0 ** -5, 0.0]))
    assert np.array_equal(hi, [0.75, -2.0 ** -5, 0.0]) and np.all(lo == 0.0)
    # FP16 subnormals: quantum 2^-24, so 2^-30 is lost entirely
    hi, lo = markidis.split16(np.array([2.0 ** -20 + 2.0 ** -30]))
    assert hi[0] == 2.0 ** -20 and lo[0] == 0.0
    # ties to even at the 11th bit: 1 + 2^-11 -> 1, 1 + 3 2^-11 -> 1 + 2^-9
    hi, _ = markidis.split16(np.array([1.0 + 2.0 ** -11, 1.0 + 3 * 2.0 ** -11]))
    assert np.array_equal(hi, [1.0, 1.0 + 2.0 ** -9])


def test_two_parts_carry_22_bits():
    x = np.random.default_rng(0).uniform(0.125, 1.0, 4000) * np.sign(
        np.random.default_rng(1).standard_normal(4000))
    hi, lo = markidis.split16(x)
    assert np.all(np.abs(x - hi) <= 2.0 ** -11 * np.abs(x))
    assert np.all(np.abs(x - hi - lo) <= 2.0 ** -22 * np.abs(x))


def test_term_order_and_exact_cases():
    rng = np.random.default_rng(2)
    # entries exactly representable in FP16 after scaling: one term is exact
    a = rng.integers(-1024, 1024, (20, 30)).astype(np.float64)
    b = rng.integers(-1024, 1024, (30, 10)).astype(np.float64)
    assert np.array_equal(markidis.markidis_gemm(a, b, 1), a @ b)
    # the four terms reproduce (A0 + A1)(B0 + B1) exactly in this size range
    a = rng.standard_normal((12, 16))
    b = rng.standard_normal((16, 9))
    e, f, (a0, a1), (b0, b1) = markidis.scaled_split(a, b)
    full = np.ldexp((a0 + a1) @ (b0 + b1), e[:, None] + f[None, :])
    assert np.allclose(markidis.markidis_gemm(a, b, 4), full, rtol=0, atol=1e-14 * np.abs(full).max())
    t2 = np.ldexp(a0 @ b0 + a0 @ b1, e[:, None] + f[None, :])
    assert np.allclose(markidis.markidis_gemm(a, b, 2), t2, rtol=0, atol=1e-15 * np.abs(t2).max())
    with pytest.raises(ValueError):
        markidis.markidis_gemm(a, b, 5)


def test_error_against_terms():
    """1 and 2 terms keep A to 11 bits (error ~2^-11 of |A||B|); 3 and 4 terms
    carry both operands to ~22 bits (the A1 B1 term is below that level)."""
    rng = np.random.default_rng(3)
    a = rng.uniform(0.0, 1.0, (64, 64))
    b = rng.uniform(0.0, 1.0, (64, 64))
    ref = a @ b
    err = [np.max(np.abs(markidis.markidis_gemm(a, b, t) - ref) / ref) for t in (1, 2, 3, 4)]
    assert 2.0 ** -14 < err[0] < 2.0 ** -10
    assert err[1] < err[0] and 2.0 ** -14 < err[1] < 2.0 ** -10
    assert err[2] < 2.0 ** -20 and err[3] <= err[2] * 1.01


def test_fp32_accumulation_stays_within_bound():
    """Sequential FP32 accumulation of the term products (a model of a tensor
    unit with FP32 accumulators) lies within the stated bound."""
    rng = np.random.default_rng(4)
    a = rng.standard_normal((16, 48))
    b = rng.standard_normal((48, 12))
    for terms in (1, 2, 3, 4):
        e, f, ap, bp = markidis.scaled_split(a, b)
        acc = np.zeros((16, 12), dtype=np.float32)
        for kk in range(48):
            for s, t in markidis.TERMS[:terms]:
                acc = (acc + np.float32(1) * (np.outer(ap[s][:, kk], bp[t][kk, :])).astype(np.float32)).astype(np.float32)
        c32 = np.ldexp(acc.astype(np.float64), e[:, None] + f[None, :])
        ref = markidis.markidis_gemm(a, b, terms)
        bound = markidis.fp32_accumulation_bound(a, b, terms)
        assert np.all(np.abs(c32 - ref) <= bound)
