"""GEMM error against slice count on the n = 2048 tight-binding matrix
(sampled rows against long-double products), INT8 and FP16.

The operand H^2 keeps rounding residues near 1e-18 where exact entries
cancel; row and column scaling drops entries far below the row maximum, so
on those elements the error is not small relative to (|A||B|)_ij.  The check
is the scheme's own bound, which is relative to the row and column maxima
(the elementwise relative bound is checked on random inputs elsewhere)."""
import numpy as np
import pytest

from oracle import ozaki

from paper_2407_13299_amd.workloads import workload

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
dmp = pytest.importorskip("paper_2407_13299_amd")


def test_gemm_error_vs_slices_tb2048():
    h = workload("tb_2048")["H"]
    a = h @ h            # a dense, exactly symmetric operand with wide in-row range
    a = 0.5 * (a + a.T)
    rng = np.random.default_rng(0)
    rows = rng.choice(a.shape[0], 48, replace=False)
    ref = a[rows].astype(np.longdouble) @ a.astype(np.longdouble)
    A = torch.from_numpy(a).cuda()
    out = {}
    for kind in ("int8", "fp16"):
        for s in range(2, 9):
            c = dmp.ozaki_gemm(A, A, slices=s, kind=kind)
            torch.cuda.synchronize()
            err = np.abs(c[torch.from_numpy(rows).cuda()].cpu().numpy() - ref)
            assert np.all(err <= ozaki.error_bound(a[rows], a, s))
            scale = np.max(np.abs(a[rows]), axis=1)[:, None] * np.max(np.abs(a), axis=0)[None, :]
            out[(kind, s)] = (float(np.max(err / scale)), float(np.max(err)))
        assert out[(kind, 7)][0] < 1e-14
        for s in range(3, 8):
            assert out[(kind, s + 1)][0] < out[(kind, s)][0]
    print("GEMM error vs slices (kind, S): max |C - AB| / (rowmax |A| colmax |B|), max |C - AB|")
    for k in sorted(out):
        print(f"  {k[0]:5s} S={k[1]}: {out[k][0]:.2e} {out[k][1]:.2e}")
    for s in range(2, 9):
        assert out[("int8", s)] == out[("fp16", s)]   # same digits, exact sums: same result
