"""Pins for the Ozaki-scheme oracle: exact definitions, brute force, bounds."""
import math

import numpy as np
import pytest

from oracle import exact, ozaki


def edge_values():
    v = [0.0, 1.0, -1.0, 0.5, -0.5, 0.75, 1 - 2 ** -53, -(1 - 2 ** -53),
         127.5 / 128, 255 / 256, 2 ** -30, -3 * 2 ** -60, 5e-324, 1e300,
         0.1, -0.3, 1 / 3]
    # values whose scaled digits land exactly on ties at every position
    for s in range(1, 9):
        v.append(0.5 + 2.0 ** -(8 * s - 2) * 0.5)
        v.append(-(0.25 + 2.0 ** -(8 * s - 2) * 1.5))
    return v


@pytest.mark.parametrize("s", [1, 2, 3, 5, 7, 8, 10])
def test_digits_match_integer_definition(s):
    rng = np.random.default_rng(s)
    rows = [edge_values()]
    for scale in (1.0, 1e-7, 3e5):
        rows.append(list(rng.standard_normal(len(rows[0])) * scale))
    rows.append(list(rng.uniform(-1, 1, len(rows[0])) * 2.0 ** rng.integers(-40, 40, len(rows[0]))))
    a = np.array(rows)
    e, d = ozaki.split_rows(a, s)
    for i in range(a.shape[0]):
        assert e[i] == exact.frexp_exponent(float(np.max(np.abs(a[i]))))
        for j in range(a.shape[1]):
            want = exact.entry_digits(float(a[i, j]), int(e[i]), s)
            assert list(d[:, i, j]) == want, (i, j, a[i, j])


@pytest.mark.parametrize("s", [1, 4, 7])
def test_digit_ranges_and_representation_error(s):
    rng = np.random.default_rng(10 + s)
    a = rng.standard_normal((40, 64)) * np.exp(rng.uniform(-20, 20, (40, 1)))
    a[3] = 0.0
    e, d = ozaki.split_rows(a, s)
    assert d[0].min() >= -64 and d[0].max() <= 65
    if s > 1:
        assert d[1:].min() >= -128 and d[1:].max() <= 127
    assert np.all(d[:, 3] == 0) and e[3] == 0
    w = 2.0 ** -(8 * np.arange(1, s + 1) - 2)
    recon = np.ldexp(np.tensordot(w, d.astype(np.float64), axes=1), e[:, None])
    bound = np.ldexp(1.0, (e - 8 * s + 1))[:, None]
    assert np.all(np.abs(recon - a) <= bound)


def test_group_products_brute_force():
    rng = np.random.default_rng(3)
    s = 4
    a = rng.standard_normal((5, 7))
    b = rng.standard_normal((7, 6))
    e, d = ozaki.split_rows(a, s)
    f, dt = ozaki.split_cols(b, s)
    g = ozaki.group_products(d, dt)
    for gi in range(2, s + 2):
        for i in range(5):
            for j in range(6):
                ref = 0
                for si in range(1, gi):
                    sj = gi - si
                    if sj > s:
                        continue
                    ref += sum(int(d[si - 1, i, t]) * int(dt[sj - 1, t, j]) for t in range(7))
                assert g[gi - 2, i, j] == ref


@pytest.mark.parametrize("s", [2, 3, 6])
def test_combine_against_exact_truncated_sum(s):
    rng = np.random.default_rng(20 + s)
    a = rng.standard_normal((4, 9))
    b = rng.uniform(0, 1, (9, 5))
    c = ozaki.ozaki_gemm(a, b, s)
    ref = exact.exact_truncated_product(a.tolist(), b.tolist(), s)
    absab = np.abs(a) @ np.abs(b)
    for i in range(4):
        for j in range(5):
            # S-1 additions, each rounding by at most half an ulp of a partial
            # sum bounded by the magnitude sum
            assert abs(c[i, j] - float(ref[i][j])) <= s * 2.0 ** -53 * 2 * absab[i, j]


@pytest.mark.parametrize("s", [1, 2, 3, 5, 7, 8])
def test_ozaki_against_exact_product_bound(s):
    rng = np.random.default_rng(40 + s)
    a = rng.standard_normal((6, 11)) * np.exp(rng.uniform(-5, 5, (6, 1)))
    b = rng.standard_normal((11, 7))
    c = ozaki.ozaki_gemm(a, b, s)
    ref = np.array(exact.to_float(exact.exact_product(a.tolist(), b.tolist())))
    assert np.all(np.abs(c - ref) <= ozaki.error_bound(a, b, s))


def test_special_cases_exact():
    rng = np.random.default_rng(5)
    # diagonal power-of-two A: one slice already exact
    a = np.diag(2.0 ** rng.integers(-8, 8, 6))
    b = rng.standard_normal((6, 6))
    assert np.array_equal(ozaki.ozaki_gemm(a, np.eye(6), 1), a)
    # identity times integer B is exact once 8S - 2 bits cover B's columns
    bi = rng.integers(-1000, 1001, (6, 5)).astype(float)
    assert np.array_equal(ozaki.ozaki_gemm(np.eye(6), bi, 2), bi)
    # zero operands and empty inner dimension
    assert np.array_equal(ozaki.ozaki_gemm(np.zeros((3, 4)), np.ones((4, 2)), 3), np.zeros((3, 2)))
    assert np.array_equal(ozaki.ozaki_gemm(np.zeros((3, 0)), np.zeros((0, 2)), 3), np.zeros((3, 2)))
    # powers of two scale out exactly
    c1 = ozaki.ozaki_gemm(a @ b, b, 5)
    c2 = ozaki.ozaki_gemm(4.0 * (a @ b), 0.125 * b, 5)
    assert np.array_equal(c1 * 0.5, c2)


def test_geometric_error_decrease_and_full_slices():
    """Error falls by about 2^8 per slice (the accumulation precision sets the
    result's precision, Sec. 2.4); at S = 7 the error is below
    1e-13 (|A||B|)_ij for uniform [0, 1] and normal inputs."""
    n = 256
    rng = np.random.default_rng(11)
    for a, b in ((rng.uniform(0, 1, (n, n)), rng.uniform(0, 1, (n, n))),
                 (rng.standard_normal((n, n)), rng.standard_normal((n, n)))):
        ref = (a.astype(np.longdouble) @ b.astype(np.longdouble))
        absab = np.abs(a) @ np.abs(b)
        errs = []
        for s in range(2, 9):
            c = ozaki.ozaki_gemm(a, b, s)
            errs.append(float(np.max(np.abs(c - ref) / absab)))
        for lo, hi in zip(errs[1:5], errs[:4]):
            assert lo < hi / 50
        assert errs[5] < 1e-13           # S = 7
        assert ozaki.products_count(7) == 28


def test_products_count():
    assert [ozaki.products_count(s) for s in (3, 4, 5, 6)] == [6, 10, 15, 21]
    assert math.comb(7, 2) + 7 == ozaki.products_count(7)
