"""Write tests/golden/tb8192_reference.npz from the oracle only.

The 16x16x8 tight-binding workload (n = 8192, nocc = 2048) is too large for
the oracle to run inside a test, so its eigendecomposition result is stored:
E = tr(P H), the HOMO-LUMO gap, four full rows of P and 4096 seeded sampled
entries.  Run from the repository root:
    python tests/golden/make_tb8192_reference.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import projector  # noqa: E402
from paper_2407_13299_amd.workloads import workload  # noqa: E402


def main():
    w = workload("tb_8192")
    h, nocc = w["H"], w["nocc"]
    p, e, eps, gap = projector.eigh_projector(h, nocc)
    rng = np.random.default_rng(8192)
    rows = np.array([0, 1, 4097, 8191])
    si = rng.integers(0, h.shape[0], 4096)
    sj = rng.integers(0, h.shape[0], 4096)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tb8192_reference.npz")
    np.savez_compressed(out, E=e, gap=gap, eps_homo=eps[nocc - 1], eps_lumo=eps[nocc],
                        rows=rows, P_rows=p[rows], si=si, sj=sj, P_samples=p[si, sj],
                        H_checksum=np.array([h.sum(), np.abs(h).sum(), h[0, 0], h[-1, -1]]))
    print("E", e, "gap", gap, "->", out)


if __name__ == "__main__":
    main()
