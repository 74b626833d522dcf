"""GPU parity of the Ozaki-scheme GEMM against the CPU oracle (C ABI)."""
import numpy as np
import pytest

from oracle import ozaki

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

dmp = pytest.importorskip("paper_2407_13299_amd")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def run(a, b, s, kind, ta=False, tb=False):
    c = dmp.ozaki_gemm(dev(a), dev(b), slices=s, kind=kind, trans_a=ta, trans_b=tb)
    torch.cuda.synchronize()
    return c.cpu().numpy()


SHAPES = [(1, 1, 1), (64, 64, 64), (100, 70, 130), (65, 129, 33), (200, 192, 257), (31, 300, 64)]


@pytest.mark.parametrize("kind", ["int8", "fp16"])
@pytest.mark.parametrize("s", [1, 2, 3, 5, 7, 8])
@pytest.mark.parametrize("shape", SHAPES)
def test_bitwise_against_oracle_model(kind, s, shape):
    m, n, k = shape
    rng = np.random.default_rng(hash((m, n, k, s)) % 2 ** 32)
    a = rng.standard_normal((m, k)) * np.exp(rng.uniform(-8, 8, (m, 1)))
    b = rng.uniform(-1, 1, (k, n)) * np.exp(rng.uniform(-8, 8, (1, n)))
    got = run(a, b, s, kind)
    want = ozaki.ozaki_gemm(a, b, s)
    assert np.array_equal(got, want), np.max(np.abs(got - want))


@pytest.mark.parametrize("kind", ["int8", "fp16"])
@pytest.mark.parametrize("s", [1, 2, 4, 7, 8, 9])
def test_ties_and_carries_of_the_split(kind, s):
    """Entries exactly halfway between two multiples of the last digit's
    unit (ties, rounded to even), entries whose lower digits round up to 128
    (carries into the digit above) and entries at the top of the range,
    multiplied by the identity: the product is the kept value of every entry,
    bit for bit as the oracle's digits give it, for the digit kernel's
    integer form (S <= 8) and its rounding steps (S >= 9)."""
    rng = np.random.default_rng(40 + s)
    m, k = 96, 160
    top = 0.75 * np.exp2(rng.integers(-20, 20, (m, 1)))      # row maxima, e = top's exponent + 1
    _, e = np.frexp(top)
    unit = np.ldexp(1.0, e - (8 * s - 2))                    # weight of the last digit
    lim = 2.0 ** (8 * s - 2) * 0.74                          # |X| below the row maximum's
    ties = (rng.integers(-2 ** 40, 2 ** 40, (m, k)) % int(min(lim, 2 ** 52)) + 0.5) * unit
    ties *= rng.choice([-1.0, 1.0], (m, k))
    carry = np.zeros((m, k))
    if s >= 2:                                               # lower digits 127.5: carries
        x = sum(127.5 * 256.0 ** i for i in range(s - 1))
        carry = np.where(rng.random((m, k)) < 0.5, x, -x) * unit
    pick = rng.integers(0, 3, (m, k))
    a = np.where(pick == 0, ties, np.where(pick == 1, carry, rng.uniform(-1, 1, (m, k)) * top))
    a[:, 0] = top[:, 0]
    a[5, :] = 0.0
    ident = np.eye(k)
    got = run(a, ident, s, kind)
    want = ozaki.ozaki_gemm(a, ident, s)
    assert np.array_equal(got, want)
    # the kept value is a rounded to the nearest multiple of the unit, ties to even
    assert np.array_equal(got, np.rint(a / unit) * unit)


@pytest.mark.parametrize("kind", ["int8", "fp16"])
@pytest.mark.parametrize("s", [9, 10, 12])
def test_bitwise_many_slices(kind, s):
    rng = np.random.default_rng(s)
    a = rng.standard_normal((96, 160))
    b = rng.standard_normal((160, 80))
    assert np.array_equal(run(a, b, s, kind), ozaki.ozaki_gemm(a, b, s))


@pytest.mark.parametrize("kind", ["int8", "fp16"])
def test_split_tail_general_gemm(kind, monkeypatch):
    """A 2200 x 2200 product has 630 tiles of 128 x 64, more than the chip
    holds at once; its last round runs in parts along the reduction.  The
    result equals whole tiles (DMP_TAIL_SPLIT=0) bit for bit, and the oracle
    on sampled rows, two of them in the split tiles (rows >= 2048)."""
    rng = np.random.default_rng(21)
    a = rng.standard_normal((2200, 1500)) * np.exp(rng.uniform(-4, 4, (2200, 1)))
    b = rng.standard_normal((1500, 2200))
    monkeypatch.setenv("DMP_TAIL_SPLIT", "1")
    c1 = run(a, b, 7, kind)
    monkeypatch.setenv("DMP_TAIL_SPLIT", "0")
    c0 = run(a, b, 7, kind)
    assert np.array_equal(c1, c0)
    rows = [0, 700, 2100, 2199]
    assert np.array_equal(c1[rows], ozaki.ozaki_gemm(a[rows], b, 7))


@pytest.mark.parametrize("ta,tb", [(False, True), (True, False), (True, True)])
def test_transposes_bitwise(ta, tb):
    rng = np.random.default_rng(7)
    m, n, k = 90, 70, 150
    a = rng.standard_normal((k, m) if ta else (m, k))
    b = rng.standard_normal((n, k) if tb else (k, n))
    got = run(a, b, 6, "int8", ta, tb)
    want = ozaki.ozaki_gemm(a.T if ta else a, b.T if tb else b, 6)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dist", ["uniform", "normal"])
def test_full_slices_bound_against_longdouble(dist):
    """At S = 7 the error is below 1e-13 (|A||B|)_ij elementwise."""
    n = 512
    rng = np.random.default_rng(3)
    if dist == "uniform":
        a, b = rng.uniform(0, 1, (n, n)), rng.uniform(0, 1, (n, n))
    else:
        a, b = rng.standard_normal((n, n)), rng.standard_normal((n, n))
    ref = a.astype(np.longdouble) @ b.astype(np.longdouble)
    absab = np.abs(a) @ np.abs(b)
    for kind in ("int8", "fp16"):
        c = run(a, b, 7, kind)
        rel = np.max(np.abs(c - ref) / absab)
        assert rel < 1e-13, (kind, rel)
        assert np.all(np.abs(c - ref) <= ozaki.error_bound(a, b, 7))


def test_error_falls_with_slices():
    rng = np.random.default_rng(4)
    a, b = rng.uniform(0, 1, (256, 256)), rng.uniform(0, 1, (256, 256))
    ref = a.astype(np.longdouble) @ b.astype(np.longdouble)
    errs = [float(np.max(np.abs(run(a, b, s, "int8") - ref))) for s in range(2, 8)]
    for lo, hi in zip(errs[1:], errs[:-1]):
        assert lo < hi / 50


def test_native_kind_is_dgemm():
    rng = np.random.default_rng(5)
    a, b = rng.standard_normal((130, 90)), rng.standard_normal((90, 70))
    c = run(a, b, 7, "native")
    assert np.max(np.abs(c - a @ b)) < 1e-12


def test_edge_cases():
    a = np.zeros((5, 0))
    b = np.zeros((0, 3))
    c = dmp.ozaki_gemm(dev(np.ones((5, 1)))[:, :0].contiguous(), dev(np.ones((1, 3)))[:0].contiguous(),
                       slices=3)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), np.zeros((5, 3)))
    del a, b
    # zero rows and columns stay exactly zero
    rng = np.random.default_rng(6)
    a = rng.standard_normal((70, 40))
    a[3] = 0.0
    b = rng.standard_normal((40, 66))
    b[:, 5] = 0.0
    c = run(a, b, 4, "int8")
    assert np.all(c[3] == 0.0) and np.all(c[:, 5] == 0.0)
    assert np.array_equal(c, ozaki.ozaki_gemm(a, b, 4))


def test_nonfinite_rows_give_nan():
    rng = np.random.default_rng(8)
    a = rng.standard_normal((70, 40))
    b = rng.standard_normal((40, 66))
    a[2, 7] = np.nan
    b[9, 4] = np.inf
    c = run(a, b, 5, "int8")
    assert np.all(np.isnan(c[2])) and np.all(np.isnan(c[:, 4]))
    mask = np.ones_like(c, dtype=bool)
    mask[2] = False
    mask[:, 4] = False
    assert np.all(np.isfinite(c[mask]))


def test_batched_matches_single():
    rng = np.random.default_rng(9)
    shapes = [(64, 64, 64), (130, 70, 90), (1, 5, 7), (200, 33, 150)]
    As = [rng.standard_normal((m, k)) for m, n, k in shapes]
    Bs = [rng.standard_normal((k, n)) for m, n, k in shapes]
    for kind in ("int8", "fp16"):
        Cs = dmp.ozaki_gemm_batched([dev(a) for a in As], [dev(b) for b in Bs], slices=6, kind=kind)
        torch.cuda.synchronize()
        for a, b, c in zip(As, Bs, Cs):
            assert np.array_equal(c.cpu().numpy(), ozaki.ozaki_gemm(a, b, 6))


def test_deterministic():
    rng = np.random.default_rng(10)
    a, b = rng.standard_normal((300, 300)), rng.standard_normal((300, 300))
    c1 = run(a, b, 7, "int8")
    c2 = run(a, b, 7, "int8")
    assert np.array_equal(c1, c2)


@pytest.mark.parametrize("kind", ["int8", "fp16"])
def test_int32_group_sums_at_the_reduction_limit(kind):
    """k at the largest value the host accepts for S = 5, every entry split
    into the digits (-63, -128, -128, -128, -128): all slice products share a
    sign and the top group sum reaches 80 % of the INT32 range; the result is
    still bit-identical to the oracle's integer model.  One more element is
    rejected."""
    s = 5
    k = (2 ** 31 - 1) // (s * 16384)
    v = -(63.5 + 0.5 / 256 + 0.5 / 256 ** 2 + 0.5 / 256 ** 3 + 0.5 / 256 ** 4)
    _, d = ozaki.split_rows(np.full((1, 1), v), s)
    assert list(d[:, 0, 0]) == [-63, -128, -128, -128, -128]
    a = np.full((40, k), v)
    b = np.full((k, 36), v)
    b[:, 3] *= 0.5          # a second column exponent
    assert np.array_equal(run(a, b, s, kind), ozaki.ozaki_gemm(a, b, s))
    with pytest.raises(dmp.DmpError):
        dmp.ozaki_gemm(dev(np.full((4, k + 1), v)), dev(np.full((k + 1, 4), v)), slices=s, kind=kind)
