"""Python binding of libdmp: the C-ABI entry points with torch tensors for
device memory and streams.  Every step of the computation runs in the HIP
library; this module only allocates outputs/workspace and marshals pointers.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib

__all__ = ["ozaki_gemm", "ozaki_gemm_noalloc", "ozaki_gemm_batched", "purify", "purify_batched",
           "autotune_slices", "Purify", "PurifyTape", "max_slices", "version"]


def _kind(kind) -> int:
    if isinstance(kind, int):
        return kind
    try:
        return _lib.KINDS[kind]
    except KeyError as e:
        raise ValueError(f"kind must be one of {sorted(_lib.KINDS)}") from e


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _check_matrix(t, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA (HIP) tensor")
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 2-D tensor")


def _workspace(nbytes: int, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _keep_for(ws: torch.Tensor, stream):
    """A temporary workspace that asynchronous work on a caller-given stream
    still reads: tell the caching allocator not to reuse it before that
    stream has passed this point."""
    if stream is not None:
        ws.record_stream(stream)


def _check_out(out, shape, like, name="out"):
    _check_matrix(out, name)
    if tuple(out.shape) != tuple(shape) or out.device != like.device:
        raise ValueError(f"{name} must be a {shape[0]}x{shape[1]} tensor on {like.device}")


def _square(h, name="H"):
    _check_matrix(h, name)
    if h.shape[0] != h.shape[1]:
        raise ValueError(f"{name} must be square")
    return h.shape[0]


def version() -> str:
    return _lib.load().dmp_version().decode()


def max_slices(kind="int8") -> int:
    return _lib.load().dmp_max_slices(_kind(kind))


def ozaki_gemm(A, B, slices=7, kind="int8", trans_a=False, trans_b=False, out=None,
               stream=None):
    """C = op(A) op(B) by the Ozaki scheme (kind 'int8' / 'fp16', ``slices``
    slices), the Markidis scheme (kind 'markidis', ``slices`` = 1..4 terms) or
    rocBLAS DGEMM (kind 'native')."""
    lib = _lib.load()
    _check_matrix(A, "A")
    _check_matrix(B, "B")
    m = A.shape[1] if trans_a else A.shape[0]
    k = A.shape[0] if trans_a else A.shape[1]
    kb = B.shape[1] if trans_b else B.shape[0]
    n = B.shape[0] if trans_b else B.shape[1]
    if k != kb:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    if A.device != B.device:
        raise ValueError("A and B are on different devices")
    if out is None:
        out = torch.empty((m, n), dtype=torch.float64, device=A.device)
    else:
        _check_out(out, (m, n), A)
    kd = _kind(kind)
    ws = _workspace(lib.dmp_gemm_workspace_bytes(m, n, k, slices, kd), A.device)
    st = lib.dmp_ozaki_gemm(b"T" if trans_a else b"N", b"T" if trans_b else b"N", m, n, k,
                            _ptr(A), max(1, A.shape[1]), _ptr(B), max(1, B.shape[1]),
                            _ptr(out), max(1, out.shape[1]), slices, kd, _ptr(ws), ws.numel(),
                            _stream(stream))
    _lib.check(st, "dmp_ozaki_gemm")
    _keep_for(ws, stream)
    return out


def ozaki_gemm_noalloc(A, B, slices=7, kind="int8", trans_a=False, trans_b=False, out=None,
                       stream=None):
    """C = op(A) op(B) through the allocation-free entry point: the library
    uses its own fixed device scratch instead of a workspace (only the
    output is allocated here, when ``out`` is None)."""
    lib = _lib.load()
    _check_matrix(A, "A")
    _check_matrix(B, "B")
    m = A.shape[1] if trans_a else A.shape[0]
    k = A.shape[0] if trans_a else A.shape[1]
    kb = B.shape[1] if trans_b else B.shape[0]
    n = B.shape[0] if trans_b else B.shape[1]
    if k != kb:
        raise ValueError(f"inner dimensions differ: {k} vs {kb}")
    if A.device != B.device:
        raise ValueError("A and B are on different devices")
    if out is None:
        out = torch.empty((m, n), dtype=torch.float64, device=A.device)
    else:
        _check_out(out, (m, n), A)
    st = lib.dmp_ozaki_gemm_noalloc(b"T" if trans_a else b"N", b"T" if trans_b else b"N", m, n,
                                    k, _ptr(A), max(1, A.shape[1]), _ptr(B), max(1, B.shape[1]),
                                    _ptr(out), max(1, out.shape[1]), slices, _kind(kind),
                                    _stream(stream))
    _lib.check(st, "dmp_ozaki_gemm_noalloc")
    return out


def ozaki_gemm_batched(As, Bs, slices=7, kind="int8", stream=None):
    """C_b = A_b B_b for lists of matrices (grouped row split and slice GEMM)."""
    lib = _lib.load()
    cnt = len(As)
    if len(Bs) != cnt:
        raise ValueError("As and Bs differ in length")
    if cnt == 0:
        return []
    for a, b in zip(As, Bs):
        _check_matrix(a, "A")
        _check_matrix(b, "B")
        if a.shape[1] != b.shape[0]:
            raise ValueError("inner dimensions differ")
        if a.device != As[0].device or b.device != As[0].device:
            raise ValueError("all matrices must be on one device")
    Cs = [torch.empty((a.shape[0], b.shape[1]), dtype=torch.float64, device=a.device)
          for a, b in zip(As, Bs)]
    IA = ctypes.c_int * cnt
    PA = ctypes.c_void_p * cnt
    m = IA(*[a.shape[0] for a in As])
    n = IA(*[b.shape[1] for b in Bs])
    k = IA(*[a.shape[1] for a in As])
    kd = _kind(kind)
    ws = _workspace(lib.dmp_gemm_batched_workspace_bytes(cnt, m, n, k, slices, kd), As[0].device)
    st = lib.dmp_ozaki_gemm_batched(cnt, m, n, k, PA(*[a.data_ptr() for a in As]),
                                    PA(*[b.data_ptr() for b in Bs]),
                                    PA(*[c.data_ptr() for c in Cs]), slices, kd, _ptr(ws),
                                    ws.numel(), _stream(stream))
    _lib.check(st, "dmp_ozaki_gemm_batched")
    _keep_for(ws, stream)
    return Cs


def _method(method) -> int:
    if isinstance(method, int):
        return method
    try:
        return _lib.METHODS[method]
    except KeyError as e:
        raise ValueError(f"method must be one of {sorted(_lib.METHODS)}") from e


def purify(H, nocc, tol=1e-8, slices=7, kind="int8", max_iter=200, out=None, stream=None,
           workspace=None, method="canonical", refine=False, triangle=False):
    """Density-matrix purification (canonical or TRS4), optionally followed
    by one FP64 McWeeny refinement step; returns (P, E, info dict).
    ``triangle`` (kind 'native'): rocBLAS dsyrk / dsyrkx upper-triangle
    products instead of full DGEMMs."""
    lib = _lib.load()
    n = _square(H)
    if out is not None:
        _check_out(out, (n, n), H)
    P = out if out is not None else torch.empty_like(H)
    kd = _kind(kind)
    need = lib.dmp_purify_workspace_bytes(n, slices, kd)
    ws = workspace
    if ws is not None and (not isinstance(ws, torch.Tensor) or ws.dtype != torch.uint8
                           or ws.device != H.device or not ws.is_contiguous()):
        raise TypeError("workspace must be a contiguous uint8 tensor on the device of H")
    if ws is None or ws.numel() < need:
        ws = _workspace(need, H.device)
    e = ctypes.c_double(0.0)
    info = _lib.DmpInfo()
    flags = (_lib.REFINE_MCWEENY if refine else 0) | (_lib.NATIVE_TRIANGLE if triangle else 0)
    st = lib.dmp_purify_ex(_ptr(H), n, int(nocc), float(tol), int(slices), kd, int(max_iter),
                           _method(method), flags, _ptr(P), ctypes.byref(e), ctypes.byref(info),
                           _ptr(ws), ws.numel(), _stream(stream))
    _lib.check(st, "dmp_purify_ex")
    return P, e.value, info.as_dict()


def purify_batched(Hs, noccs, tol=1e-8, slices=0, kind="int8", max_iter=200, stream=None,
                   method="canonical", refine=False):
    """Purify a list of Hamiltonians together; slices <= 0 uses the tuned table.

    Returns (list of P, list of E, list of info dicts)."""
    lib = _lib.load()
    cnt = len(Hs)
    if len(noccs) != cnt:
        raise ValueError("Hs and noccs differ in length")
    if cnt == 0:
        return [], [], []
    for h in Hs:
        _square(h)
        if h.device != Hs[0].device:
            raise ValueError("all Hamiltonians must be on one device")
    Ps = [torch.empty_like(h) for h in Hs]
    IA = ctypes.c_int * cnt
    PA = ctypes.c_void_p * cnt
    n = IA(*[h.shape[0] for h in Hs])
    nocc = IA(*[int(x) for x in noccs])
    kd = _kind(kind)
    ws = _workspace(lib.dmp_purify_batched_workspace_bytes(cnt, n, int(slices), kd), Hs[0].device)
    E = (ctypes.c_double * cnt)()
    infos = (_lib.DmpInfo * cnt)()
    flags = _lib.REFINE_MCWEENY if refine else 0
    st = lib.dmp_purify_batched_ex(cnt, PA(*[h.data_ptr() for h in Hs]), n, nocc, float(tol),
                                   int(slices), kd, int(max_iter), _method(method), flags,
                                   PA(*[p.data_ptr() for p in Ps]), E, infos, _ptr(ws),
                                   ws.numel(), _stream(stream))
    _lib.check(st, "dmp_purify_batched_ex")
    return Ps, list(E), [i.as_dict() for i in infos]


def autotune_slices(n, target=1e-10, kind="int8") -> int:
    return _lib.load().dmp_autotune_slices(int(n), float(target), _kind(kind))


class PurifyTape:
    """Owner of a forward tape (iterates checkpointed every ``stride`` steps)."""

    def __init__(self, H, nocc, tol=1e-8, slices=7, kind="int8", max_iter=200, stride=0,
                 stream=None):
        lib = _lib.load()
        n = _square(H)
        self.n = n
        self.device = H.device
        self.H = H          # the library copies H, this only keeps the caller's alive
        self.P = torch.empty_like(H)
        e = ctypes.c_double(0.0)
        info = _lib.DmpInfo()
        tape = ctypes.c_void_p()
        st = lib.dmp_purify_fwd_tape(_ptr(H), n, int(nocc), float(tol), int(slices), _kind(kind),
                                     int(max_iter), int(stride), _ptr(self.P), ctypes.byref(e),
                                     ctypes.byref(info), ctypes.byref(tape), _stream(stream))
        _lib.check(st, "dmp_purify_fwd_tape")
        self._tape = tape
        self.E = e.value
        self.info = info.as_dict()

    def branches(self):
        lib = _lib.load()
        it = ctypes.c_int(0)
        lib.dmp_tape_info(self._tape, ctypes.byref(it), None)
        br = (ctypes.c_int * max(1, it.value))()
        lib.dmp_tape_info(self._tape, ctypes.byref(it), br)
        return list(br)[: it.value]

    def coefficients(self):
        """Recorded (c_k, t1_k, t2_k) of every iteration, as lists."""
        lib = _lib.load()
        k = self.info["iters"]
        arr = [(ctypes.c_double * max(1, k))() for _ in range(3)]
        lib.dmp_tape_coefficients(self._tape, arr[0], arr[1], arr[2])
        return [list(a)[:k] for a in arr]

    def backward(self, Pbar, stream=None):
        lib = _lib.load()
        if not isinstance(Pbar, torch.Tensor) or Pbar.dim() != 2:
            raise TypeError("Pbar must be a 2-D float64 CUDA (HIP) tensor")
        # dmp_purify_bwd symmetrises Pbar itself (the adjoint of a symmetric
        # P); only the layout is fixed here
        Pbar = Pbar.contiguous()
        _check_out(Pbar, (self.n, self.n), self.P, "Pbar")
        Hbar = torch.empty_like(Pbar)
        ws = _workspace(lib.dmp_purify_bwd_workspace_bytes(self._tape), self.device)
        if stream is not None:
            # Pbar, Hbar and the workspace were produced or allocated on the
            # current stream: the library's stream starts after them
            stream.wait_stream(torch.cuda.current_stream())
        st = lib.dmp_purify_bwd(self._tape, _ptr(Pbar), _ptr(Hbar), _ptr(ws), ws.numel(),
                                _stream(stream))
        _lib.check(st, "dmp_purify_bwd")
        _keep_for(ws, stream)
        return Hbar

    def __del__(self):
        t = getattr(self, "_tape", None)
        if t is not None and t.value:
            try:
                _lib.load().dmp_tape_free(t)
            except Exception:
                pass
            self._tape = None


class Purify(torch.autograd.Function):
    """P = purify(H) with a hand-written adjoint: backward returns dL/dH."""

    @staticmethod
    def forward(ctx, H, nocc, tol=1e-8, slices=7, kind="int8", max_iter=200, stride=0):
        tape = PurifyTape(H, nocc, tol, slices, kind, max_iter, stride)
        ctx.tape = tape
        return tape.P.clone()

    @staticmethod
    def backward(ctx, grad_p):
        hbar = ctx.tape.backward(grad_p.contiguous())
        return hbar, None, None, None, None, None, None
