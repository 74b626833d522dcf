"""The allocation-free GEMM entry point (dmp_ozaki_gemm_noalloc, its scratch
a fixed device array of the library) against dmp_ozaki_gemm with a caller
workspace: bit for bit, on consecutive calls whose second input is smaller
than the first (the scratch keeps the previous call's contents)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dmp = pytest.importorskip("paper_2407_13299_amd")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def operands(m, k, n, ta, tb, seed):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((k, m) if ta else (m, k)) * np.exp(rng.uniform(-8, 8, (k, m) if ta else (m, k)))
    b = rng.standard_normal((n, k) if tb else (k, n))
    return dev(a), dev(b)


@pytest.mark.parametrize("kind,s", [("int8", 7), ("fp16", 5), ("markidis", 3)])
def test_noalloc_equals_workspace_gemm_on_consecutive_calls(kind, s):
    cases = [(1500, 1300, 1700, False, False), (300, 200, 257, True, False),
             (65, 33, 130, False, True)]
    for c, (m, k, n, ta, tb) in enumerate(cases):
        A, B = operands(m, k, n, ta, tb, seed=40 + c)
        ref = dmp.ozaki_gemm(A, B, slices=s, kind=kind, trans_a=ta, trans_b=tb)
        got = dmp.ozaki_gemm_noalloc(A, B, slices=s, kind=kind, trans_a=ta, trans_b=tb)
        torch.cuda.synchronize()
        assert got.shape == (m, n)
        assert torch.equal(got, ref), (kind, s, m, k, n)


def test_noalloc_on_a_side_stream_and_repeated():
    A, B = operands(700, 640, 900, False, False, seed=50)
    ref = dmp.ozaki_gemm(A, B, slices=6)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    out = torch.empty_like(ref)
    with torch.cuda.stream(side):
        for _ in range(3):
            dmp.ozaki_gemm_noalloc(A, B, slices=6, out=out, stream=side)
    side.synchronize()
    assert torch.equal(out, ref)


def test_noalloc_edges_and_limits():
    A, B = operands(40, 0, 30, False, False, seed=51)
    z = dmp.ozaki_gemm_noalloc(A, B, slices=7)
    torch.cuda.synchronize()
    assert torch.equal(z, torch.zeros_like(z))
    big = torch.zeros((4096, 4096), dtype=torch.float64, device="cuda")
    with pytest.raises(dmp.DmpError, match="scratch"):
        dmp.ozaki_gemm_noalloc(big, big, slices=7)
    small = torch.ones((8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(dmp.DmpError, match="Ozaki and Markidis"):
        dmp.ozaki_gemm_noalloc(small, small, kind="native")
    # the scratch still serves a valid product after the rejected ones
    A, B = operands(100, 90, 80, False, False, seed=52)
    assert torch.equal(dmp.ozaki_gemm_noalloc(A, B, slices=7), dmp.ozaki_gemm(A, B, slices=7))
