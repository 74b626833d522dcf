"""Pins for the TRS4 oracle and the one-step McWeeny refinement."""
import numpy as np

from oracle import canonical, projector, trs4
from paper_2407_13299_amd.workloads import (spectrum_hamiltonian,
                                            tight_binding_hamiltonian)


def test_polynomials_on_exact_binary_values():
    """F = x^2 (4x - 3x^2) and G = x^2 (1 - x)^2 at points where every value
    is an exact binary fraction (computed by hand)."""
    x = np.diag([0.0, 1.0, 0.5, 0.25, 0.75])
    x2, f, g = trs4.polynomials(x)
    assert np.array_equal(np.diag(x2), [0.0, 1.0, 0.25, 0.0625, 0.5625])
    assert np.array_equal(np.diag(f), [0.0, 1.0, 0.3125, 0.05078125, 0.73828125])
    assert np.array_equal(np.diag(g), [0.0, 0.0, 0.0625, 0.03515625, 0.03515625])
    assert np.count_nonzero(f - np.diag(np.diag(f))) == 0


def test_branches_by_hand():
    # tr F = 1, tr G = 0.25: gamma = (nocc - 1) / 0.25
    assert trs4.reset_coefficient(2, 1.0, 0.25) == (4.0, trs4.BRANCH_RESET)
    assert trs4.reset_coefficient(3, 1.0, 0.25) == (8.0, trs4.BRANCH_RAISE)
    assert trs4.reset_coefficient(0.5, 1.0, 0.25) == (-2.0, trs4.BRANCH_SQUARE)
    assert trs4.reset_coefficient(1, 1.0, 0.0) == (0.0, trs4.BRANCH_RESET)
    # on a diagonal the three branches are the scalar maps
    x = np.diag([0.1, 0.5, 0.9])
    x_sq, _, br, _, _ = trs4.step(x, 0.0)        # gamma < 0 -> X^2
    assert br == trs4.BRANCH_SQUARE and np.allclose(np.diag(x_sq), [0.01, 0.25, 0.81])
    x_up, _, br, _, _ = trs4.step(x, 3.0)        # gamma > 6 -> 2X - X^2
    assert br == trs4.BRANCH_RAISE and np.allclose(np.diag(x_up), [0.19, 0.75, 0.99])


def test_trace_reset_every_in_range_step():
    """On the F + gamma G branch tr X_{k+1} = nocc (the trace reset)."""
    h = tight_binding_hamiltonian(3, 4, 3, seed=5)
    n = h.shape[0]
    nocc = n // 4
    x = trs4.initial_guess(h)
    ev = np.linalg.eigvalsh(x)
    assert ev.min() >= -1e-12 and ev.max() <= 1 + 1e-12
    seen = 0
    for _ in range(25):
        x, gamma, br, _, tr_g = trs4.step(x, nocc)
        if br == trs4.BRANCH_RESET and tr_g > 1e-12:
            seen += 1
            assert abs(np.trace(x) - nocc) < 1e-9
    assert seen >= 3


def test_projectors_are_fixed_points():
    rng = np.random.default_rng(3)
    q, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    p = q[:, :15] @ q[:, :15].T
    for nocc in (15, 5, 30):
        x, gamma, br, tr_f, tr_g = trs4.step(p, nocc)
        assert np.max(np.abs(x - p)) < 1e-13


def test_map_is_quadratic_at_both_ends():
    """Every branch polynomial fixes 0 and 1; the reset one with zero slope."""
    eps = 1e-4
    for gamma in (0.0, 2.0, 6.0):
        f = lambda t: t * t * (4 * t - 3 * t * t) + gamma * t * t * (1 - t) ** 2
        assert abs(f(eps)) < 10 * eps ** 2
        assert abs(1 - f(1 - eps)) < 10 * eps ** 2


def test_converges_to_projector_spectrum():
    h, q, lam = spectrum_hamiltonian(256, 128, seed=0)
    r = trs4.purify(h, 128, tol=1e-12)
    p_ref, e_ref, _, _ = projector.eigh_projector(h, 128)
    assert r["stop"] == canonical.STOP_CONVERGED
    assert np.max(np.abs(r["P"] - p_ref)) < 1e-10
    assert abs(r["E"] - lam[lam < 0].sum()) < 1e-10


def test_converges_to_projector_tight_binding_in_fewer_iterations():
    h = tight_binding_hamiltonian(4, 4, 4, seed=1)
    nocc = 64
    r = trs4.purify(h, nocc, tol=1e-10)
    p_ref, e_ref, _, _ = projector.eigh_projector(h, nocc)
    assert r["stop"] == canonical.STOP_CONVERGED
    assert np.max(np.abs(r["P"] - p_ref)) < 1e-10
    assert abs(r["E"] - e_ref) < 1e-9
    rc = canonical.purify(h, nocc, tol=1e-10)
    assert r["iters"] * 2 < rc["iters"]


def test_eigen_simulator_matches_matrix_iteration():
    h = tight_binding_hamiltonian(4, 4, 3, seed=7)
    nocc = h.shape[0] // 4
    r = trs4.purify(h, nocc, tol=1e-10)
    s = trs4.eigen_simulate(h, nocc, tol=1e-10)
    assert abs(r["iters"] - s["iters"]) <= 1
    k = 0
    for (g1, b1, _, tg1, e1), (g2, b2, _, tg2, e2) in zip(r["history"], s["history"]):
        if tg1 < 1e-8:
            break
        assert b1 == b2 and abs(g1 - g2) < 1e-8 * max(1, abs(g1))
        assert abs(e1 - e2) < 1e-9
        k += 1
    assert k >= 5


def test_special_occupations():
    h, _, _ = spectrum_hamiltonian(32, 16, seed=2)
    assert np.array_equal(trs4.purify(h, 0)["P"], np.zeros((32, 32)))
    assert np.array_equal(trs4.purify(h, 32)["P"], np.eye(32))


def test_mcweeny_refine_eigenvalue_map():
    x = np.diag([0.0, 1.0, 0.5, 0.25])
    p, e = trs4.mcweeny_refine(x, np.eye(4))
    assert np.array_equal(np.diag(p), [0.0, 1.0, 0.5, 0.15625])
    assert e == 1.65625


def test_mcweeny_refine_squares_the_energy_error():
    """A symmetric error inside the occupied and virtual blocks (it commutes
    with H) shifts E to first order; one refinement step leaves only the
    second-order part.  The occupied-virtual part does not move E to first
    order and is not removed (as observed for RMSD and commutator)."""
    h, q, lam = spectrum_hamiltonian(60, 25, seed=4)
    p_ref, e_ref, _, _ = projector.eigh_projector(h, 25)
    rng = np.random.default_rng(5)
    eps = 1e-5
    d = np.diag(rng.uniform(-1, 1, 60))
    delta = q @ d @ q.T
    p = p_ref + eps * delta
    e0 = float(np.sum(p * h))
    p1, e1 = trs4.mcweeny_refine(p, h)
    assert abs(e0 - e_ref) > 1e-7
    assert abs(e1 - e_ref) < 1e-8
    assert abs(e1 - e_ref) < 1e-2 * abs(e0 - e_ref)
    # occupied-virtual error: first order stays in P
    a = q[:, :25] @ rng.standard_normal((25, 35)) @ q[:, 25:].T
    p = p_ref + eps * (a + a.T)
    p1, _ = trs4.mcweeny_refine(p, h)
    assert np.max(np.abs(p1 - p_ref)) > 0.5 * np.max(np.abs(p - p_ref))
