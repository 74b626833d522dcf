"""Argument checks of the Python binding and asynchronous GEMMs on a side
stream (C ABI through the binding)."""
import numpy as np
import pytest

from oracle import ozaki

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

dmp = pytest.importorskip("paper_2407_13299_amd")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def test_gemm_rejects_a_wrong_output_shape():
    a, b = dev(np.ones((40, 30))), dev(np.ones((30, 20)))
    with pytest.raises(ValueError):
        dmp.ozaki_gemm(a, b, slices=3, out=torch.empty((20, 40), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        dmp.ozaki_gemm(a, b, slices=3, out=torch.empty((39, 20), dtype=torch.float64, device="cuda"))


def test_purify_rejects_bad_arguments():
    h = dev(np.eye(64))
    with pytest.raises(ValueError):
        dmp.purify(dev(np.ones((64, 32))), 16)
    with pytest.raises(ValueError):
        dmp.purify(h, 16, out=torch.empty((32, 64), dtype=torch.float64, device="cuda"))
    with pytest.raises(TypeError):
        dmp.purify(h, 16, workspace=torch.empty(1 << 20, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        dmp.purify_batched([h], [16, 16])
    assert dmp.purify_batched([], []) == ([], [], [])
    assert dmp.ozaki_gemm_batched([], []) == []


def test_purify_uses_a_caller_workspace():
    from paper_2407_13299_amd.workloads import spectrum_hamiltonian
    h, _, _ = spectrum_hamiltonian(130, 65, seed=5)
    hd = dev(h)
    p0, e0, _ = dmp.purify(hd, 65, tol=1e-10, slices=7)
    ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    p1, e1, _ = dmp.purify(hd, 65, tol=1e-10, slices=7, workspace=ws)
    torch.cuda.synchronize()
    assert torch.equal(p0, p1) and e0 == e1


def test_misaligned_workspace_is_rejected():
    """A workspace that does not start on a 256-byte boundary is an argument
    error (DMP_EINVAL) at the C ABI, before any work is queued."""
    import ctypes
    from paper_2407_13299_amd import _lib
    lib = _lib.load()
    a = dev(np.ones((70, 50)))
    b = dev(np.ones((50, 40)))
    c = torch.full((70, 40), 7.0, dtype=torch.float64, device="cuda")
    need = lib.dmp_gemm_workspace_bytes(70, 40, 50, 3, _lib.KINDS["int8"])
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    st = lib.dmp_ozaki_gemm(b"N", b"N", 70, 40, 50, a.data_ptr(), 50, b.data_ptr(), 40,
                            c.data_ptr(), 40, 3, _lib.KINDS["int8"], ws.data_ptr() + 8,
                            need + 248, None)
    assert st == -1 and b"aligned" in lib.dmp_last_error()
    h = dev(np.diag(np.arange(64.0)))
    p = torch.empty_like(h)
    e = ctypes.c_double(0.0)
    need = lib.dmp_purify_workspace_bytes(64, 7, _lib.KINDS["int8"])
    ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    st = lib.dmp_purify(h.data_ptr(), 64, 16, 1e-8, 7, _lib.KINDS["int8"], 50, p.data_ptr(),
                        ctypes.byref(e), None, ws.data_ptr() + 16, need + 240, None)
    assert st == -1 and b"aligned" in lib.dmp_last_error()
    torch.cuda.synchronize()
    assert torch.all(c == 7.0)     # nothing was written
    st = lib.dmp_purify(h.data_ptr(), 64, 16, 1e-8, 7, _lib.KINDS["int8"], 50, p.data_ptr(),
                        ctypes.byref(e), None, ws.data_ptr(), need + 256, None)
    assert st == 0


@pytest.mark.parametrize("batched", [False, True])
def test_gemm_on_a_side_stream(batched):
    """The product is queued on a non-current stream and its temporary
    workspace is held for that stream; the current stream allocates and
    overwrites memory meanwhile.  The result equals the oracle's bit for bit."""
    rng = np.random.default_rng(11)
    a, b = rng.standard_normal((300, 257)), rng.standard_normal((257, 190))
    ref = ozaki.ozaki_gemm(a, b, 6)
    ad, bd = dev(a), dev(b)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    if batched:
        c = dmp.ozaki_gemm_batched([ad], [bd], slices=6, stream=side)[0]
    else:
        c = dmp.ozaki_gemm(ad, bd, slices=6, stream=side)
    junk = [torch.full((1 << 22,), 7.0, dtype=torch.float64, device="cuda") for _ in range(8)]
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    del junk
    assert np.array_equal(c.cpu().numpy(), ref)


def test_timing_clock_is_measured_inside_the_gemm():
    """With kernel timing on, the GEMM workgroups report their shader clock:
    a plausible value (the MI355X runs at up to 2.4 GHz), and a reset clears it."""
    from paper_2407_13299_amd import _lib
    from paper_2407_13299_amd.workloads import spectrum_hamiltonian
    import ctypes
    lib = _lib.load()
    h, _, _ = spectrum_hamiltonian(700, 350, seed=2)
    hd = dev(h)
    lib.dmp_timing_enable(1)
    try:
        lib.dmp_timing_reset()
        dmp.purify(hd, 350, tol=1e-10, slices=7)
        torch.cuda.synchronize()
        ghz = ctypes.c_double(-1.0)
        assert lib.dmp_timing_clock(0, ctypes.byref(ghz)) == 0 and ghz.value == 0.0   # mode 1: events only
        lib.dmp_timing_enable(2)
        lib.dmp_timing_reset()
        dmp.purify(hd, 350, tol=1e-10, slices=7)
        torch.cuda.synchronize()
        for which in (0, 1):
            ghz = ctypes.c_double()
            assert lib.dmp_timing_clock(which, ctypes.byref(ghz)) == 0
            assert 0.3 < ghz.value < 3.0, ghz.value
        lib.dmp_timing_reset()
        ghz = ctypes.c_double(-1.0)
        assert lib.dmp_timing_clock(0, ctypes.byref(ghz)) == 0 and ghz.value == 0.0
    finally:
        lib.dmp_timing_enable(0)
        lib.dmp_timing_reset()
