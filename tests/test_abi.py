"""The C-ABI library loads and exports every symbol its header declares; the
argument checks that run before any device work behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2407_13299_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(dmp_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdmp.so is not built (python -m paper_2407_13299_amd.build)")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(_lib.EXPORTS) == names


def test_version_and_limits(lib):
    assert lib.dmp_version().decode().startswith("dmp")
    assert lib.dmp_max_slices(1) == lib.dmp_max_slices(2) >= 8
    assert lib.dmp_max_slices(0) == 0
    assert lib.dmp_max_slices(3) == 4      # Markidis: terms


def test_workspace_queries(lib):
    s8 = lib.dmp_gemm_workspace_bytes(100, 70, 130, 7, 1)
    s16 = lib.dmp_gemm_workspace_bytes(100, 70, 130, 7, 2)
    # two operands of S digit planes, padded to 64 (1 byte INT8, 2 bytes FP16)
    assert s8 >= 7 * 128 * 192 + 7 * 128 * 192 // 2
    assert s16 > s8
    assert lib.dmp_gemm_workspace_bytes(10, 10, 10, 0, 1) == 0
    p = lib.dmp_purify_workspace_bytes(8192, 7, 1)
    assert p >= 2 * 8192 * 8192 * 8 + 2 * 7 * 8192 * 8192
    # Markidis: two FP16 planes whatever the number of terms; at most 4 terms
    m1 = lib.dmp_gemm_workspace_bytes(100, 70, 130, 1, 3)
    assert m1 == lib.dmp_gemm_workspace_bytes(100, 70, 130, 4, 3)
    assert m1 == lib.dmp_gemm_workspace_bytes(100, 70, 130, 2, 2)
    assert lib.dmp_gemm_workspace_bytes(100, 70, 130, 5, 3) == 0
    assert lib.dmp_purify_workspace_bytes(512, 5, 3) == 0
    # Markidis purification: one workspace for any number of terms (two FP16
    # planes), no larger than FP16 S = 2, which also holds the part buffer of
    # the split tail
    w = lib.dmp_purify_workspace_bytes(512, 3, 3)
    assert w == lib.dmp_purify_workspace_bytes(512, 1, 3)
    assert 0 < w <= lib.dmp_purify_workspace_bytes(512, 2, 2)
    n = (ctypes.c_int * 3)(128, 300, 1536)
    assert lib.dmp_purify_batched_workspace_bytes(3, n, 7, 1) > lib.dmp_purify_workspace_bytes(1536, 7, 1)


def test_argument_errors_without_device_work(lib):
    ws = ctypes.c_void_p(0)
    # bad slice count
    st = lib.dmp_ozaki_gemm(b"N", b"N", 4, 4, 4, None, 4, None, 4, None, 4, 0, 1, ws, 0, None)
    assert st == -1 and b"slices" in lib.dmp_last_error()
    # bad transpose flag
    st = lib.dmp_ozaki_gemm(b"X", b"N", 4, 4, 4, None, 4, None, 4, None, 4, 3, 1, ws, 0, None)
    assert st == -1
    # leading dimension too small
    st = lib.dmp_ozaki_gemm(b"N", b"N", 4, 4, 4, None, 2, None, 4, None, 4, 3, 1, ws, 0, None)
    assert st == -1
    # reduction too long for exact INT32 group sums
    st = lib.dmp_ozaki_gemm(b"N", b"N", 4, 4, 1 << 20, ctypes.c_void_p(8), 1 << 20,
                            ctypes.c_void_p(8), 4, ctypes.c_void_p(8), 4, 12, 1, ws, 0, None)
    assert st == -1 and b"exceeds" in lib.dmp_last_error()
    # empty output: nothing to do
    assert lib.dmp_ozaki_gemm(b"N", b"N", 0, 4, 4, None, 4, None, 4, None, 4, 3, 1, ws, 0, None) == 0
    e = ctypes.c_double()
    info = _lib.DmpInfo()
    # n < 1, nocc out of range, tol <= 0, aliasing
    for args in ((0, 0, 1e-8), (8, 9, 1e-8), (8, -1, 1e-8), (8, 4, 0.0)):
        st = lib.dmp_purify(ctypes.c_void_p(8), args[0], args[1], args[2], 7, 1, 100,
                            ctypes.c_void_p(16), ctypes.byref(e), ctypes.byref(info), ws, 0, None)
        assert st == -1
    st = lib.dmp_purify(ctypes.c_void_p(8), 8, 4, 1e-8, 7, 1, 100, ctypes.c_void_p(8),
                        ctypes.byref(e), ctypes.byref(info), ws, 0, None)
    assert st == -1
    # missing workspace
    st = lib.dmp_purify(ctypes.c_void_p(8), 8, 4, 1e-8, 7, 1, 100, ctypes.c_void_p(16),
                        ctypes.byref(e), ctypes.byref(info), ws, 0, None)
    assert st == -4
    # unknown kind
    st = lib.dmp_purify(ctypes.c_void_p(8), 8, 4, 1e-8, 7, 9, 100, ctypes.c_void_p(16),
                        ctypes.byref(e), ctypes.byref(info), ws, 0, None)
    assert st == -1
    # too many Markidis terms
    st = lib.dmp_purify(ctypes.c_void_p(8), 8, 4, 1e-8, 5, 3, 100, ctypes.c_void_p(16),
                        ctypes.byref(e), ctypes.byref(info), ws, 0, None)
    assert st == -1 and b"terms" in lib.dmp_last_error()
    # unknown method or flag of the _ex entry points
    for method, flags in ((2, 0), (-1, 0), (1, 4), (0, 0x10)):
        st = lib.dmp_purify_ex(ctypes.c_void_p(8), 8, 4, 1e-8, 7, 1, 100, method, flags,
                               ctypes.c_void_p(16), ctypes.byref(e), ctypes.byref(info), ws, 0,
                               None)
        assert st == -1 and (b"method" in lib.dmp_last_error() or b"flags" in lib.dmp_last_error())
        H = (ctypes.c_void_p * 1)(8)
        P = (ctypes.c_void_p * 1)(16)
        n = (ctypes.c_int * 1)(8)
        no = (ctypes.c_int * 1)(4)
        E = (ctypes.c_double * 1)()
        st = lib.dmp_purify_batched_ex(1, H, n, no, 1e-8, 7, 1, 100, method, flags, P, E,
                                       ctypes.byref(info), ws, 0, None)
        assert st == -1
    # valid method and flag: only the missing workspace is reported
    st = lib.dmp_purify_ex(ctypes.c_void_p(8), 8, 4, 1e-8, 7, 1, 100, 1, 1, ctypes.c_void_p(16),
                           ctypes.byref(e), ctypes.byref(info), ws, 0, None)
    assert st == -4


def test_timing_clock_without_timed_launches(lib):
    ghz = ctypes.c_double(-1.0)
    assert lib.dmp_timing_clock(2, ctypes.byref(ghz)) == -1
    assert lib.dmp_timing_clock(0, None) == -1
    # nothing timed in this process yet: 0 GHz, no device call made
    assert lib.dmp_timing_clock(1, ctypes.byref(ghz)) == 0 and ghz.value == 0.0


def test_autotune_table_monotone(lib):
    prev = 0
    for n in (64, 256, 1024, 4096, 8192):
        s = lib.dmp_autotune_slices(n, 1e-10, 1)
        assert 1 <= s <= lib.dmp_max_slices(1) and s >= prev
        prev = s
    assert lib.dmp_autotune_slices(256, 1e-4, 1) < lib.dmp_autotune_slices(256, 1e-12, 1)
    assert lib.dmp_autotune_slices(256, 1e-10, 0) == 0


def test_product_path_fails_loudly_without_library(tmp_path):
    with pytest.raises(_lib.DmpError):
        saved = _lib._lib
        try:
            _lib._lib = None
            _lib.load(str(tmp_path / "missing.so"))
        finally:
            _lib._lib = saved
