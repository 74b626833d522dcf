"""CPU oracle for Ozaki-scheme density-matrix purification.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls, links or executes anything here; only the
test suite, the smoke check and the CPU-baseline leg of the benchmark do.  The
oracle shares no code, tables or constants with the GPU path: it is a plain,
slow, float64 numpy restatement of the method, written from the paper.

Modules
  projector   the plain definition the purification reaches: occupied-space
              projector and energy from an FP64 eigendecomposition
              (Sec. 2.3, density matrix from eigenvectors), and the paper's
              error measures (Sec. 3.1).
  canonical   canonical (trace-conserving) purification in FP64, the method
              the paper proposes to run with Ozaki products (Sec. 1 and 2.3),
              plus the eigenvalue-space simulator of the same iteration.
  ozaki       the Ozaki scheme (Sec. 2.4): per-row/column power-of-two
              scaling, split into fixed-point slices by rounding, exact
              slice-pair products for i + j <= S + 1, FP64 summation.
  exact       brute-force exact-rational references for tiny inputs.
  adjoint     first-order perturbation formula for dP/dH and the reverse-mode
              derivative of the canonical iteration.
  trs4        the trace-resetting fourth-order purification the paper runs
              (Sec. 3) and the one-step McWeeny refinement (Sec. 4.1).
  markidis    the two-term FP16 split of Sec. 4.5.
"""
