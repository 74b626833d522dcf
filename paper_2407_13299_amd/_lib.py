"""ctypes loader for libdmp.so (the HIP library); argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdmp.so")

KINDS = {"native": 0, "fp64": 0, "int8": 1, "fp16": 2, "markidis": 3}
METHODS = {"canonical": 0, "trs4": 1}
REFINE_MCWEENY = 1
NATIVE_TRIANGLE = 2
STOP_REASONS = {0: "converged", 1: "stagnated", 2: "max_iter", 3: "nonfinite"}
DMP_OK, DMP_NOT_CONVERGED = 0, 1
ERRORS = {-1: "DMP_EINVAL", -2: "DMP_ENONFINITE", -3: "DMP_EHIP", -4: "DMP_ENOMEM",
          -5: "DMP_EUNSUPPORTED"}

# Every symbol the public header declares (tests check the export list).
EXPORTS = [
    "dmp_last_error", "dmp_version", "dmp_max_slices",
    "dmp_gemm_workspace_bytes", "dmp_ozaki_gemm", "dmp_ozaki_gemm_noalloc",
    "dmp_gemm_batched_workspace_bytes", "dmp_ozaki_gemm_batched",
    "dmp_purify_workspace_bytes", "dmp_purify", "dmp_purify_ex",
    "dmp_purify_batched_workspace_bytes", "dmp_purify_batched", "dmp_purify_batched_ex",
    "dmp_autotune_slices",
    "dmp_purify_fwd_tape", "dmp_purify_bwd_workspace_bytes", "dmp_purify_bwd",
    "dmp_tape_info", "dmp_tape_coefficients", "dmp_tape_free",
    "dmp_timing_enable", "dmp_timing_reset", "dmp_timing_read", "dmp_timing_clock",
]


class DmpInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("stop_reason", ctypes.c_int),
                ("slices", ctypes.c_int), ("kind", ctypes.c_int),
                ("E", ctypes.c_double), ("last_dE", ctypes.c_double),
                ("trace", ctypes.c_double), ("idem", ctypes.c_double),
                ("h_min", ctypes.c_double), ("h_max", ctypes.c_double),
                ("mu", ctypes.c_double), ("lambda_", ctypes.c_double),
                ("method", ctypes.c_int), ("refined", ctypes.c_int),
                ("E_unrefined", ctypes.c_double), ("products", ctypes.c_int)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["lambda"] = d.pop("lambda_")
        d["stop"] = STOP_REASONS.get(self.stop_reason, str(self.stop_reason))
        d["method"] = {v: k for k, v in METHODS.items()}.get(self.method, str(self.method))
        return d


class DmpError(RuntimeError):
    pass


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_SZ = ctypes.c_size_t
_IP = ctypes.POINTER(ctypes.c_int)
_PP = ctypes.POINTER(ctypes.c_void_p)

_SIGS = {
    "dmp_last_error": (ctypes.c_char_p, []),
    "dmp_version": (ctypes.c_char_p, []),
    "dmp_max_slices": (_I, [_I]),
    "dmp_gemm_workspace_bytes": (_SZ, [_I, _I, _I, _I, _I]),
    "dmp_ozaki_gemm": (_I, [ctypes.c_char, ctypes.c_char, _I, _I, _I, _P, _I, _P, _I, _P, _I,
                            _I, _I, _P, _SZ, _P]),
    "dmp_ozaki_gemm_noalloc": (_I, [ctypes.c_char, ctypes.c_char, _I, _I, _I, _P, _I, _P, _I,
                                    _P, _I, _I, _I, _P]),
    "dmp_gemm_batched_workspace_bytes": (_SZ, [_I, _IP, _IP, _IP, _I, _I]),
    "dmp_ozaki_gemm_batched": (_I, [_I, _IP, _IP, _IP, _PP, _PP, _PP, _I, _I, _P, _SZ, _P]),
    "dmp_purify_workspace_bytes": (_SZ, [_I, _I, _I]),
    "dmp_purify": (_I, [_P, _I, _I, _D, _I, _I, _I, _P, ctypes.POINTER(_D),
                        ctypes.POINTER(DmpInfo), _P, _SZ, _P]),
    "dmp_purify_ex": (_I, [_P, _I, _I, _D, _I, _I, _I, _I, _I, _P, ctypes.POINTER(_D),
                           ctypes.POINTER(DmpInfo), _P, _SZ, _P]),
    "dmp_purify_batched_ex": (_I, [_I, _PP, _IP, _IP, _D, _I, _I, _I, _I, _I, _PP,
                                   ctypes.POINTER(_D), ctypes.POINTER(DmpInfo), _P, _SZ, _P]),
    "dmp_purify_batched_workspace_bytes": (_SZ, [_I, _IP, _I, _I]),
    "dmp_purify_batched": (_I, [_I, _PP, _IP, _IP, _D, _I, _I, _I, _PP, ctypes.POINTER(_D),
                                ctypes.POINTER(DmpInfo), _P, _SZ, _P]),
    "dmp_autotune_slices": (_I, [_I, _D, _I]),
    "dmp_purify_fwd_tape": (_I, [_P, _I, _I, _D, _I, _I, _I, _I, _P, ctypes.POINTER(_D),
                                 ctypes.POINTER(DmpInfo), ctypes.POINTER(_P), _P]),
    "dmp_purify_bwd_workspace_bytes": (_SZ, [_P]),
    "dmp_purify_bwd": (_I, [_P, _P, _P, _P, _SZ, _P]),
    "dmp_tape_info": (_I, [_P, _IP, _IP]),
    "dmp_tape_free": (None, [_P]),
    "dmp_tape_coefficients": (_I, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "dmp_timing_enable": (None, [_I]),
    "dmp_timing_reset": (None, []),
    "dmp_timing_read": (_I, [_I, ctypes.POINTER(_D), ctypes.POINTER(ctypes.c_longlong),
                             ctypes.POINTER(_D)]),
    "dmp_timing_clock": (_I, [_I, ctypes.POINTER(_D)]),
}


def load(path: str | None = None):
    """Load libdmp.so once; raise loudly if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise DmpError(
            f"libdmp.so not found at {path}: build it with "
            "`python -m paper_2407_13299_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, what: str):
    if status < 0:
        msg = load().dmp_last_error().decode(errors="replace")
        raise DmpError(f"{what} failed with {ERRORS.get(status, status)}: {msg}")
    return status
