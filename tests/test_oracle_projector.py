"""Pins for the eigendecomposition oracle (closed forms and invariants)."""
import numpy as np
import pytest

from oracle import projector
from paper_2407_13299_amd.workloads import (spectrum_hamiltonian,
                                            tight_binding_hamiltonian)


def bloch_energy(lx, ly, lz, e_s=-0.5, e_p=0.5, t=0.1):
    """Sum of the lowest band over the k-grid of the clean sp3 lattice.

    Independent of the real-space generator: Bloch Hamiltonian of one site,
      H_ss(k)   = e_s - 2t sum_d cos k_d
      H_sp_d(k) = 2 i t sin k_d        (from the odd parity of p_d)
      H_p_dp_d  = e_p + 2t cos k_d,   no p_d / p_d' coupling.
    At quarter filling exactly one band per k is occupied.
    """
    tot = 0.0
    for kx in 2 * np.pi * np.arange(lx) / lx:
        for ky in 2 * np.pi * np.arange(ly) / ly:
            for kz in 2 * np.pi * np.arange(lz) / lz:
                k = np.array([kx, ky, kz])
                hk = np.zeros((4, 4), dtype=complex)
                hk[0, 0] = e_s - 2 * t * np.sum(np.cos(k))
                for d in range(3):
                    hk[0, 1 + d] = 2j * t * np.sin(k[d])
                    hk[1 + d, 0] = -2j * t * np.sin(k[d])
                    hk[1 + d, 1 + d] = e_p + 2 * t * np.cos(k[d])
                tot += np.linalg.eigvalsh(hk)[0]
    return tot


def test_spectrum_closed_form():
    n, nocc = 96, 40
    h, q, lam = spectrum_hamiltonian(n, nocc, seed=7)
    p, e, eps, gap = projector.eigh_projector(h, nocc)
    occ = lam < 0
    assert occ.sum() == nocc
    p_exact = q[:, occ] @ q[:, occ].T
    assert np.max(np.abs(p - p_exact)) < 1e-12
    assert abs(e - lam[occ].sum()) < 1e-11
    assert gap >= 0.2 - 1e-12


@pytest.mark.parametrize("dims", [(3, 3, 3), (4, 4, 4), (6, 4, 3)])
def test_tight_binding_bloch_energy(dims):
    h = tight_binding_hamiltonian(*dims, seed=None)
    nocc = h.shape[0] // 4
    _, e, eps, gap = projector.eigh_projector(h, nocc)
    assert abs(e - bloch_energy(*dims)) < 1e-10
    assert gap > 0.1


@pytest.mark.slow
def test_tight_binding_bloch_energy_8cube():
    h = tight_binding_hamiltonian(8, 8, 8, seed=None)
    _, e, _, gap = projector.eigh_projector(h, 512)
    assert abs(e - bloch_energy(8, 8, 8)) < 1e-9
    assert abs(gap - 0.2) < 1e-9


def test_tight_binding_structure():
    h = tight_binding_hamiltonian(4, 3, 5, seed=3)
    assert np.array_equal(h, h.T)
    # every site couples to 6 neighbours: s row has 6 s-s and 6 s-p entries
    s_row = h[0]
    assert np.count_nonzero(np.isclose(np.abs(s_row), 0.1)) == 12
    # clean model has exact on-site energies
    hc = tight_binding_hamiltonian(4, 3, 5, seed=None)
    assert np.allclose(np.diag(hc)[0::4], -0.5) and np.allclose(np.diag(hc)[1::4], 0.5)


def test_projector_invariants_disordered():
    h = tight_binding_hamiltonian(4, 4, 4, seed=1)
    nocc = 64
    p, e, eps, gap = projector.eigh_projector(h, nocc)
    assert projector.idempotency_error(p) < 1e-13
    assert abs(np.trace(p) - nocc) < 1e-11
    assert projector.commutator_norm(h, p) < 1e-12
    assert abs(np.sum(p * h) - e) < 1e-11
    assert gap > 0.1


def test_measures_definitions():
    rng = np.random.default_rng(0)
    a = rng.standard_normal((5, 5))
    b = a + 1e-3
    assert abs(projector.rmsd(b, a) - 1e-3) < 1e-15
    m = projector.measures(b, 1.0, np.eye(5), 2, a, 1.5)
    assert abs(m["dE"] - 0.5) < 1e-15 and m["commutator"] == 0.0
