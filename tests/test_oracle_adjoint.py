"""Pins for the adjoint oracle: finite differences and perturbation theory."""
import numpy as np
import pytest

from oracle import adjoint, canonical, projector
from paper_2407_13299_amd.workloads import (spectrum_hamiltonian,
                                            symmetric_direction,
                                            symmetric_weight,
                                            tight_binding_hamiltonian)


def eigh_loss(h, nocc, w):
    p, _, _, _ = projector.eigh_projector(h, nocc)
    return float(np.sum(p * w))


def test_perturbation_formula_matches_finite_differences():
    h, _, _ = spectrum_hamiltonian(24, 10, seed=1)
    w = symmetric_weight(24, seed=2)
    g = adjoint.perturbation_gradient(h, 10, w)
    for seed in (3, 4):
        d = symmetric_direction(24, seed)
        hs = 1e-5
        fd = (eigh_loss(h + hs * d, 10, w) - eigh_loss(h - hs * d, 10, w)) / (2 * hs)
        assert abs(fd - np.sum(g * d)) < 1e-8 * max(1.0, abs(fd))


def test_perturbation_gradient_invariants():
    """P is unchanged by shifts and scalings of H and by perturbations that
    commute with it, so the gradient has tr G = 0, <G, H> = 0 and no
    occupied-occupied or virtual-virtual block."""
    h, _, _ = spectrum_hamiltonian(30, 12, seed=5)
    w = symmetric_weight(30, seed=6)
    g = adjoint.perturbation_gradient(h, 12, w)
    p, _, _, _ = projector.eigh_projector(h, 12)
    q = np.eye(30) - p
    assert abs(np.trace(g)) < 1e-12
    assert abs(np.sum(g * h)) < 1e-12
    assert np.max(np.abs(p @ g @ p)) < 1e-12
    assert np.max(np.abs(q @ g @ q)) < 1e-12


@pytest.mark.parametrize("kind", ["spectrum", "tb"])
def test_canonical_adjoint_matches_finite_differences(kind):
    if kind == "spectrum":
        h, _, _ = spectrum_hamiltonian(20, 8, seed=7)
        nocc = 8
    else:
        h = tight_binding_hamiltonian(3, 3, 3, seed=8)[:, :]
        nocc = 27
    n = h.shape[0]
    w = symmetric_weight(n, seed=9)
    run = canonical.purify(h, nocc, tol=0.0, max_iter=8)
    branches = [hh[1] for hh in run["history"]]
    g = adjoint.canonical_adjoint(h, nocc, w, branches)
    for seed in (10, 11):
        d = symmetric_direction(n, seed)
        hs = 1e-6
        fd = (adjoint.loss(h + hs * d, nocc, w, branches)
              - adjoint.loss(h - hs * d, nocc, w, branches)) / (2 * hs)
        an = float(np.sum(g * d))
        assert abs(fd - an) < 1e-6 * max(1.0, abs(fd)), (fd, an)


def test_canonical_adjoint_converged_matches_perturbation():
    h, _, _ = spectrum_hamiltonian(48, 20, seed=12)
    w = symmetric_weight(48, seed=13)
    run = canonical.purify(h, 20, tol=1e-13)
    branches = [hh[1] for hh in run["history"]]
    g = adjoint.canonical_adjoint(h, 20, w, branches)
    gp = adjoint.perturbation_gradient(h, 20, w)
    assert np.max(np.abs(g - gp)) < 1e-6 * np.max(np.abs(gp))
    assert abs(np.trace(g)) < 1e-8


def test_weight_derivatives_by_differences():
    for c, br in ((0.3, 0), (0.7, 1), (0.55, 1), (0.1, 0)):
        d = adjoint.weight_derivatives(c, br)
        hs = 1e-7
        up = adjoint.branch_weights(c + hs, br)
        dn = adjoint.branch_weights(c - hs, br)
        for k in range(3):
            assert abs((up[k] - dn[k]) / (2 * hs) - d[k]) < 1e-6 * max(1, abs(d[k]))
