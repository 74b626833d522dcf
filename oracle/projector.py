"""Occupied-space projector from an FP64 eigendecomposition (test infrastructure).

Purification converges to the density matrix built from the eigenvectors of
the (orthogonalised) Hamiltonian (Sec. 2.3: K_ij = sum_a f_a c_ia c_ja with
f = 2 for occupied and 0 for virtual orbitals, and K = 2P).  The plain
definition of the result is therefore

    H = U diag(eps) U^T  (eps ascending),
    P = U[:, :nocc] U[:, :nocc]^T,
    E = tr(P H) = sum_{a < nocc} eps_a.

The paper reports the electronic energy Tr(H K) = 2 E; everything here uses
E = tr(P H) (the same quantity per orbital pair).  The error measures follow
Sec. 3.1: RMSD of the density-matrix difference, absolute energy error and the
Frobenius norm of the commutator H P - P H.
"""
from __future__ import annotations

import numpy as np


def eigh_projector(h, nocc):
    """Return (P, E, eps, gap) for a real symmetric h and nocc occupied levels.

    gap = eps[nocc] - eps[nocc-1] (inf when nocc is 0 or n).
    """
    h = np.asarray(h, dtype=np.float64)
    n = h.shape[0]
    if not (0 <= nocc <= n):
        raise ValueError("nocc must lie in [0, n]")
    eps, u = np.linalg.eigh(h)
    uo = u[:, :nocc]
    p = uo @ uo.T
    e = float(np.sum(eps[:nocc]))
    gap = float(eps[nocc] - eps[nocc - 1]) if 0 < nocc < n else float("inf")
    return p, e, eps, gap


def rmsd(p, p_ref):
    """Root-mean-square deviation ||P - P_ref||_F / n (Sec. 3.1)."""
    n = p.shape[0]
    return float(np.linalg.norm(p - p_ref) / n)


def commutator_norm(h, p):
    """||H P - P H||_F (Sec. 3.1, the DIIS error vector)."""
    return float(np.linalg.norm(h @ p - p @ h))


def idempotency_error(p):
    """max |P^2 - P|."""
    return float(np.max(np.abs(p @ p - p)))


def measures(p, e, h, nocc, p_ref, e_ref):
    """Every error measure used by the tests, as a dict."""
    return dict(
        max_dP=float(np.max(np.abs(p - p_ref))),
        rmsd=rmsd(p, p_ref),
        dE=abs(e - e_ref),
        commutator=commutator_norm(h, p),
        idempotency=idempotency_error(p),
        trace_err=abs(float(np.trace(p)) - nocc),
    )
